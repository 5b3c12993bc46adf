"""Python binding of the MI355X parallel parser (libparparaw.so).

Argument marshalling only: every step of the parse runs in the HIP kernels
behind the C ABI declared in include/parparaw.h. PyTorch supplies device
memory and streams. There is no CPU fallback: if the library is not built,
loading fails with an error.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass
from typing import List, Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
LIB_PATH = os.path.join(_HERE, "libparparaw.so")
SOURCES = [os.path.join(_HERE, "csrc", f) for f in ("parse.hip", "batch.hip", "serve.hip", "tune.hip", "copy.hip",
                                                     "stream.hip", "materialize.hip", "infer.hip",
                                                     "rows.hip")]
BUILD_DIR = os.path.join(_ROOT, "_build")

PP_OK = 0
STATUS_TEXT = {0: "ok", -1: "invalid argument", -2: "invalid DFA", -3: "invalid schema",
               -4: "workspace too small", -5: "HIP launch failed", -6: "unsupported",
               -7: "larger than the device budget"}
PP_ERR_BUDGET = -7
INT64, FLOAT64, TIMESTAMP_S, DATE_DAYS, STRING, SKIP = 0, 1, 2, 3, 4, 5
RESULT_OK, RESULT_INVALID_INPUT, RESULT_NON_ACCEPTING_END, RESULT_CAPACITY = 0, 1, 2, 3
MAX_COLUMNS = 64

COMPILE_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
                 "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    """Compile the HIP sources for gfx950 (one hipcc per source, in
    parallel) and link them into libparparaw.so (in-tree)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(BUILD_DIR, exist_ok=True)
    inc = ["-I", os.path.join(_ROOT, "include"), "-I", os.path.join(_HERE, "csrc")]
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
        objs.append(obj)
        procs.append(subprocess.Popen([hipcc] + COMPILE_FLAGS + inc + ["-c", src, "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    errs = []
    for src, pr in zip(SOURCES, procs):
        out, err = pr.communicate()
        if pr.returncode != 0:
            errs.append(f"{src}:\n{out}{err}")
        elif verbose:
            print(err)
    if errs:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errs))
    r = subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", LIB_PATH + ".tmp"],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc link failed:\n" + r.stdout + r.stderr)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class PpDfa(ctypes.Structure):
    _fields_ = [("num_states", ctypes.c_int32), ("num_groups", ctypes.c_int32),
                ("start_state", ctypes.c_int32), ("invalid_state", ctypes.c_int32),
                ("accept_mask", ctypes.c_uint32), ("group_of", ctypes.c_uint8 * 256),
                ("next", (ctypes.c_uint8 * 16) * 16), ("tag", (ctypes.c_uint8 * 16) * 16)]


class PpOutputs(ctypes.Structure):
    _fields_ = [("cap_records", ctypes.c_int64), ("cap_fields", ctypes.c_int64),
                ("d_record_offsets", ctypes.c_void_p), ("d_field_offsets", ctypes.c_void_p),
                ("d_column_ids", ctypes.c_void_p), ("d_values", ctypes.c_void_p),
                ("d_valid", ctypes.c_void_p), ("d_str_end", ctypes.c_void_p),
                ("d_result", ctypes.c_void_p), ("d_control_bitmap", ctypes.c_void_p)]


class PpSchema(ctypes.Structure):
    _fields_ = [("ncols", ctypes.c_int32), ("flags", ctypes.c_int32), ("types", ctypes.c_void_p)]


SCHEMA_REJECT_RAGGED = 1


class PpOptions(ctypes.Structure):
    _fields_ = [("bytes_per_thread", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("tile_order", ctypes.c_int32)]


RESULT_FIELDS = ("status", "num_records", "num_fields", "first_invalid_offset", "final_state",
                 "num_conversion_errors", "num_ragged_records", "min_record_fields", "max_record_fields")

_lib = None


def lib():
    """The loaded C library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.pp_workspace_size.restype = ctypes.c_size_t
        L.pp_workspace_size.argtypes = [ctypes.c_int64, P]
        L.pp_parse.restype = ctypes.c_int32
        L.pp_parse.argtypes = [P, ctypes.c_int64, P, P, P, P, ctypes.c_size_t, P, P]
        L.pp_parse_utf16.restype = ctypes.c_int32
        L.pp_parse_utf16.argtypes = [P, ctypes.c_int64, P, P, P, P, ctypes.c_size_t, P, P]
        L.pp_materialize_strings_utf16.restype = ctypes.c_int32
        L.pp_materialize_strings_utf16.argtypes = [P, ctypes.c_int64, P, ctypes.c_int32, ctypes.c_int32, P, P,
                                                   ctypes.c_int64, P, ctypes.c_size_t, P]
        L.pp_workspace_size_utf16.restype = ctypes.c_size_t
        L.pp_workspace_size_utf16.argtypes = [ctypes.c_int64, P]
        L.pp_skip_records.restype = ctypes.c_int32
        L.pp_skip_records.argtypes = [P, ctypes.c_int32, P, P, ctypes.c_int32, P]
        L.pp_skip_rows_workspace_size.restype = ctypes.c_size_t
        L.pp_skip_rows_workspace_size.argtypes = [ctypes.c_int64]
        L.pp_skip_rows.restype = ctypes.c_int32
        L.pp_skip_rows.argtypes = [P, ctypes.c_int64, P, ctypes.c_int32, P, P, P, ctypes.c_size_t, P]
        L.pp_infer_types_workspace_size.restype = ctypes.c_size_t
        L.pp_infer_types_workspace_size.argtypes = [ctypes.c_int32]
        L.pp_infer_types.restype = ctypes.c_int32
        L.pp_infer_types.argtypes = [P, ctypes.c_int64, P, ctypes.c_int32, P, P, P, ctypes.c_size_t, P]
        L.pp_materialize_workspace_size.restype = ctypes.c_size_t
        L.pp_materialize_workspace_size.argtypes = [ctypes.c_int64, ctypes.c_int64]
        L.pp_materialize_strings.restype = ctypes.c_int32
        L.pp_materialize_strings.argtypes = [P, ctypes.c_int64, P, ctypes.c_int32, ctypes.c_int32, P, P,
                                             ctypes.c_int64, P, ctypes.c_size_t, P]
        L.pp_infer_columns.restype = ctypes.c_int32
        L.pp_infer_columns.argtypes = [P, ctypes.c_int64, P, P, P, ctypes.c_size_t, P, P]
        L.pp_parse_noalloc.restype = ctypes.c_int32
        L.pp_parse_noalloc.argtypes = [P, ctypes.c_int64, P, P, P, P, P]
        L.pp_status_str.restype = ctypes.c_char_p
        L.pp_status_str.argtypes = [ctypes.c_int32]
        L.pp_batch_create.restype = ctypes.c_int32
        L.pp_batch_create.argtypes = [P, ctypes.c_int32, P, ctypes.c_int32, P, ctypes.POINTER(P)]
        L.pp_batch_workspace_size.restype = ctypes.c_size_t
        L.pp_batch_workspace_size.argtypes = [P]
        L.pp_batch_num_tiles.restype = ctypes.c_int64
        L.pp_batch_num_tiles.argtypes = [P]
        L.pp_batch_bind.restype = ctypes.c_int32
        L.pp_batch_bind.argtypes = [P, P, ctypes.c_size_t, P]
        L.pp_batch_launch.restype = ctypes.c_int32
        L.pp_batch_launch.argtypes = [P, P]
        L.pp_batch_graph_create.restype = ctypes.c_int32
        L.pp_batch_graph_create.argtypes = [P, ctypes.POINTER(P)]
        L.pp_batch_graph_launch.restype = ctypes.c_int32
        L.pp_batch_graph_launch.argtypes = [P, P]
        L.pp_batch_graph_destroy.restype = None
        L.pp_batch_graph_destroy.argtypes = [P]
        L.pp_batch_destroy.restype = None
        L.pp_batch_destroy.argtypes = [P]
        L.pp_shape.restype = ctypes.c_int32
        L.pp_shape.argtypes = [ctypes.c_int32, P]
        L.pp_autotune_workspace_size.restype = ctypes.c_size_t
        L.pp_autotune_workspace_size.argtypes = [ctypes.c_int64]
        L.pp_parse_autotune.restype = ctypes.c_int32
        L.pp_parse_autotune.argtypes = [P, ctypes.c_int64, P, P, P, P, ctypes.c_size_t, ctypes.c_int32, P, P, P]
        L.pp_batch_autotune_workspace_size.restype = ctypes.c_size_t
        L.pp_batch_autotune_workspace_size.argtypes = [P, ctypes.c_int32, P, ctypes.c_int32]
        L.pp_batch_autotune.restype = ctypes.c_int32
        L.pp_batch_autotune.argtypes = [P, ctypes.c_int32, P, ctypes.c_int32, P, ctypes.c_size_t, ctypes.c_int32,
                                        P, P, P]
        L.pp_copy.restype = ctypes.c_int32
        L.pp_copy.argtypes = [P, P, ctypes.c_size_t, P]
        L.pp_stream_create.restype = ctypes.c_int32
        L.pp_stream_create.argtypes = [P, P, P, ctypes.POINTER(P)]
        L.pp_stream_parse.restype = ctypes.c_int32
        L.pp_stream_parse.argtypes = [P, P, ctypes.c_int64, P, P, P]
        L.pp_stream_destroy.restype = None
        L.pp_stream_destroy.argtypes = [P]
        L.pp_server_create.restype = ctypes.c_int32
        L.pp_server_create.argtypes = [P, P, ctypes.c_int32, ctypes.POINTER(P)]
        L.pp_server_submit.restype = ctypes.c_int32
        L.pp_server_submit.argtypes = [P, P, ctypes.POINTER(ctypes.c_uint64)]
        L.pp_server_poll.restype = ctypes.c_int32
        L.pp_server_poll.argtypes = [P, P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
        L.pp_server_wait.restype = ctypes.c_int32
        L.pp_server_wait.argtypes = [P, ctypes.c_int64]
        L.pp_server_release.restype = ctypes.c_int32
        L.pp_server_release.argtypes = [P, ctypes.c_uint64]
        L.pp_server_get_stats.restype = ctypes.c_int32
        L.pp_server_get_stats.argtypes = [P, P]
        L.pp_server_destroy.restype = None
        L.pp_server_destroy.argtypes = [P]
        _lib = L
    return _lib


def dfa_struct(dfa) -> PpDfa:
    """Marshal a datagen.dialects.Dfa-like object (fields num_states,
    num_groups, start_state, invalid_state, accept_mask, group_of,
    next_state[g][s], tag[g][s])."""
    d = PpDfa()
    d.num_states = dfa.num_states
    d.num_groups = dfa.num_groups
    d.start_state = dfa.start_state
    d.invalid_state = dfa.invalid_state
    d.accept_mask = dfa.accept_mask
    for b in range(256):
        d.group_of[b] = dfa.group_of[b]
    for g in range(dfa.num_groups):
        for s in range(dfa.num_states):
            d.next[g][s] = dfa.next_state[g][s]
            d.tag[g][s] = dfa.tag[g][s]
    return d


def options(bytes_per_thread: int = 0, block_threads: int = 0, tile_order: int = 0) -> PpOptions:
    """pp_options_t: launch shape (0: default) and the diagnostic tile order
    (0: input order; k > 0 permutes each block of 64 tiles)."""
    return PpOptions(bytes_per_thread, block_threads, tile_order)


def workspace_size(n: int, opts: Optional[PpOptions] = None) -> int:
    return int(lib().pp_workspace_size(n, ctypes.byref(opts) if opts else None))


class PpError(RuntimeError):
    pass


@dataclass
class Outputs:
    """Device output buffers (torch tensors) of one parse."""
    cap_records: int
    cap_fields: int
    record_offsets: "object"
    field_offsets: "object"
    column_ids: "object"
    values: List[Optional[object]]
    valid: List[Optional[object]]
    str_end: List[Optional[object]]
    result: "object"  # int64[len(RESULT_FIELDS)] on device: pp_result_t
    types: List[int]
    control_bitmap: Optional[object] = None  # int32[(n + 31) // 32]: control symbols, when requested

    def result_dict(self):
        r = self.result.cpu().tolist()
        return dict(zip(RESULT_FIELDS, r))


def alloc_outputs(types: Sequence[int], cap_records: int, cap_fields: int, device="cuda",
                  bitmap_bytes: int = -1) -> Outputs:
    """Device outputs; bitmap_bytes >= 0 also allocates the control-symbol
    bitmap of an input of that many bytes (for materialize())."""
    import torch
    vals, valid, ends = [], [], []
    for ty in types:
        if ty == SKIP:
            vals.append(None); valid.append(None); ends.append(None)
            continue
        vals.append(torch.empty(max(cap_records, 1), dtype=torch.float64 if ty == FLOAT64 else torch.int64,
                                device=device))
        valid.append(torch.empty(max(cap_records, 1), dtype=torch.uint8, device=device))
        ends.append(torch.empty(max(cap_records, 1), dtype=torch.int64, device=device) if ty == STRING else None)
    return Outputs(cap_records, cap_fields,
                   torch.empty(cap_records + 1, dtype=torch.int64, device=device),
                   torch.empty(cap_fields + 1, dtype=torch.int64, device=device),
                   torch.empty(max(cap_fields, 1), dtype=torch.int32, device=device),
                   vals, valid, ends, torch.zeros(len(RESULT_FIELDS), dtype=torch.int64, device=device), list(types),
                   torch.empty(max((bitmap_bytes + 31) // 32, 1), dtype=torch.int32, device=device)
                   if bitmap_bytes >= 0 else None)


def _ptr(t):
    return t.data_ptr() if t is not None else None


class Call:
    """The marshalled argument set of one pp_parse call; keeps the ctypes
    objects alive so the same call can be issued repeatedly (benchmarks)."""

    def __init__(self, d_in, n: int, dfa, types: Sequence[int], out: Outputs, workspace,
                 opts: Optional[PpOptions] = None, reject_ragged: bool = False):
        self.d_in = d_in
        self.n = n
        self.dfa = dfa_struct(dfa)
        nc = len(types)
        self.types = (ctypes.c_int32 * max(nc, 1))(*types)
        self.schema = PpSchema(nc, SCHEMA_REJECT_RAGGED if reject_ragged else 0, ctypes.cast(self.types, ctypes.c_void_p))
        self.vptr = (ctypes.c_void_p * max(nc, 1))(*[_ptr(t) for t in out.values])
        self.mptr = (ctypes.c_void_p * max(nc, 1))(*[_ptr(t) for t in out.valid])
        self.eptr = (ctypes.c_void_p * max(nc, 1))(*[_ptr(t) for t in out.str_end])
        self.outs = PpOutputs(out.cap_records, out.cap_fields, _ptr(out.record_offsets),
                              _ptr(out.field_offsets), _ptr(out.column_ids),
                              ctypes.cast(self.vptr, ctypes.c_void_p),
                              ctypes.cast(self.mptr, ctypes.c_void_p),
                              ctypes.cast(self.eptr, ctypes.c_void_p), _ptr(out.result), _ptr(out.control_bitmap))
        self.ws = workspace
        self.opts = opts
        self.out = out

    def launch_noalloc(self, stream=None) -> None:
        """The same call through pp_parse_noalloc (the library's static
        per-device workspace; self.ws is not used)."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        rc = lib().pp_parse_noalloc(self.d_in.data_ptr() if self.n else None, self.n, ctypes.byref(self.dfa),
                                    ctypes.byref(self.schema), ctypes.byref(self.outs),
                                    ctypes.byref(self.opts) if self.opts else None,
                                    ctypes.c_void_p(stream.cuda_stream))
        if rc != PP_OK:
            raise PpError(f"pp_parse_noalloc: {STATUS_TEXT.get(rc, rc)}")

    def launch(self, stream=None) -> None:
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        rc = lib().pp_parse(self.d_in.data_ptr() if self.n else None, self.n, ctypes.byref(self.dfa),
                            ctypes.byref(self.schema), ctypes.byref(self.outs), self.ws.data_ptr(),
                            self.ws.numel(), ctypes.byref(self.opts) if self.opts else None,
                            ctypes.c_void_p(stream.cuda_stream))
        if rc != PP_OK:
            raise PpError(f"pp_parse: {STATUS_TEXT.get(rc, rc)}")


def copy(dst, src, nbytes: Optional[int] = None, stream=None) -> None:
    """pp_copy: ``nbytes`` (default: all of ``src``) from device tensor
    ``src`` to device tensor ``dst`` with the library's streaming copy."""
    import torch
    n = src.numel() * src.element_size() if nbytes is None else int(nbytes)
    if n > dst.numel() * dst.element_size() or n > src.numel() * src.element_size():
        raise PpError("pp_copy: byte count beyond a tensor")
    if stream is None:
        stream = torch.cuda.current_stream()
    _check(lib().pp_copy(dst.data_ptr(), src.data_ptr(), n, ctypes.c_void_p(stream.cuda_stream)), "pp_copy")


def parse(d_in, dfa, types: Sequence[int], cap_records: int, cap_fields: int,
          opts: Optional[PpOptions] = None, stream=None, reject_ragged: bool = False,
          control_bitmap: bool = False) -> Outputs:
    """Parse the uint8 device tensor ``d_in`` (asynchronous on ``stream``).
    ``reject_ragged``: records whose field count differs from len(types)
    get the column defaults in every typed column (Sec. 4.3)."""
    import torch
    n = int(d_in.numel())
    out = alloc_outputs(types, cap_records, cap_fields, device=d_in.device, bitmap_bytes=n if control_bitmap else -1)
    ws = torch.empty(max(workspace_size(n, opts), 1), dtype=torch.uint8, device=d_in.device)
    call = Call(d_in, n, dfa, types, out, ws, opts, reject_ragged)
    call.launch(stream)
    out._call = call  # keep workspace alive until the caller synchronises
    return out


def parse_utf16(d_in, dfa, types: Sequence[int], cap_records: int, cap_fields: int,
                opts: Optional[PpOptions] = None, stream=None, reject_ragged: bool = False,
                control_bitmap: bool = False) -> Outputs:
    """pp_parse_utf16 (Sec. 4.2): parse the UTF-16LE text in the device
    tensor ``d_in`` (uint8 of even length, or int16/uint16 code units); every
    position in the outputs is a byte offset into it. ``control_bitmap``:
    also write the control-symbol bitmap (one bit per code unit), for
    materialize_utf16. Asynchronous."""
    import torch
    if d_in.dtype == torch.uint8:
        if d_in.numel() % 2:
            raise PpError("parse_utf16: UTF-16 text of odd byte length")
        n_units = int(d_in.numel()) // 2
    else:
        n_units = int(d_in.numel())
    if stream is None:
        stream = torch.cuda.current_stream()
    out = alloc_outputs(types, cap_records, cap_fields, device=d_in.device,
                        bitmap_bytes=n_units if control_bitmap else -1)
    ws = torch.empty(max(int(lib().pp_workspace_size_utf16(n_units, ctypes.byref(opts) if opts else None)), 1),
                     dtype=torch.uint8, device=d_in.device)
    call = Call(d_in, n_units, dfa, types, out, ws, opts, reject_ragged)
    _check(lib().pp_parse_utf16(d_in.data_ptr() if n_units else None, n_units, ctypes.byref(call.dfa),
                                ctypes.byref(call.schema), ctypes.byref(call.outs), ws.data_ptr(), ws.numel(),
                                ctypes.byref(opts) if opts else None, ctypes.c_void_p(stream.cuda_stream)),
           "pp_parse_utf16")
    out._call = call  # keep the workspace alive until the caller synchronises
    return out


def materialize_utf16(d_in, out: Outputs, column: int, cap_chars: Optional[int] = None, stream=None,
                      terminator: int = -1):
    """pp_materialize_strings_utf16: string column ``column`` of a
    parse_utf16 parse (with control_bitmap=True) of ``d_in``, as (offsets
    int64 [cap_records + 1] in code units, chars int16 code units).
    Asynchronous."""
    import torch
    n_units = int(d_in.numel()) // 2 if d_in.dtype == torch.uint8 else int(d_in.numel())
    if out.control_bitmap is None:
        raise PpError("materialize_utf16: the parse did not write the control-symbol bitmap")
    if stream is None:
        stream = torch.cuda.current_stream()
    cap_chars = (n_units + (out.cap_records if terminator >= 0 else 0)) if cap_chars is None else int(cap_chars)
    offsets = torch.empty(out.cap_records + 1, dtype=torch.int64, device=d_in.device)
    chars = torch.empty(max(cap_chars, 1), dtype=torch.int16, device=d_in.device)
    ws = torch.empty(max(int(lib().pp_materialize_workspace_size(n_units, out.cap_records)), 1), dtype=torch.uint8,
                     device=d_in.device)
    po, keep = _outputs_struct(out)
    _check(lib().pp_materialize_strings_utf16(d_in.data_ptr() if n_units else None, n_units, ctypes.byref(po), column,
                                              terminator, offsets.data_ptr(), chars.data_ptr(), cap_chars,
                                              ws.data_ptr(), ws.numel(), ctypes.c_void_p(stream.cuda_stream)),
           "pp_materialize_strings_utf16")
    offsets._keep = (ws, keep)  # alive until the caller synchronises
    return offsets, chars


def infer_columns(d_in, dfa, opts: Optional[PpOptions] = None, stream=None) -> dict:
    """pp_infer_columns: the result record of a structure-only parse of the
    uint8 device tensor ``d_in`` (Sec. 4.3): max_record_fields is the
    inferred number of columns. Synchronises ``stream``."""
    import torch
    n = int(d_in.numel())
    if stream is None:
        stream = torch.cuda.current_stream()
    res = torch.zeros(len(RESULT_FIELDS), dtype=torch.int64, device=d_in.device)
    ws = torch.empty(max(workspace_size(n, opts), 1), dtype=torch.uint8, device=d_in.device)
    d = dfa_struct(dfa)
    _check(lib().pp_infer_columns(d_in.data_ptr() if n else None, n, ctypes.byref(d), res.data_ptr(), ws.data_ptr(),
                                  ws.numel(), ctypes.byref(opts) if opts else None,
                                  ctypes.c_void_p(stream.cuda_stream)), "pp_infer_columns")
    stream.synchronize()
    return dict(zip(RESULT_FIELDS, res.cpu().tolist()))


def parse_schemaless(d_in, dfa, opts: Optional[PpOptions] = None, stream=None):
    """Without a schema: the column count inferred by pp_infer_columns (the
    most fields of any record), then pp_parse with that many string
    columns. Returns (Outputs, result of the inference)."""
    inf = infer_columns(d_in, dfa, opts, stream)
    ncols = int(inf["max_record_fields"])
    out = parse(d_in, dfa, [STRING] * ncols, inf["num_records"], inf["num_fields"], opts=opts, stream=stream)
    return out, inf


def materialize(d_in, out: Outputs, column: int, cap_chars: Optional[int] = None, stream=None,
                terminator: int = -1):
    """pp_materialize_strings: string column ``column`` of a parse of the
    device tensor ``d_in`` into ``out`` (parsed with control_bitmap=True)
    with every control symbol removed, as device tensors (offsets int64
    [cap_records + 1], chars uint8[cap_chars]). cap_chars defaults to the
    input size (a value is never longer than its span), plus one byte per
    record with a terminator (>= 0: written after every value, the
    inline-terminated form). Asynchronous."""
    import torch
    n = int(d_in.numel())
    if out.control_bitmap is None:
        raise PpError("materialize: the parse did not write the control-symbol bitmap")
    if stream is None:
        stream = torch.cuda.current_stream()
    cap_chars = (n + (out.cap_records if terminator >= 0 else 0)) if cap_chars is None else int(cap_chars)
    offsets = torch.empty(out.cap_records + 1, dtype=torch.int64, device=d_in.device)
    chars = torch.empty(max(cap_chars, 1), dtype=torch.uint8, device=d_in.device)
    ws = torch.empty(max(int(lib().pp_materialize_workspace_size(n, out.cap_records)), 1), dtype=torch.uint8,
                     device=d_in.device)
    nc = len(out.types)
    vp = (ctypes.c_void_p * max(nc, 1))(*[_ptr(x) for x in out.values])
    mp = (ctypes.c_void_p * max(nc, 1))(*[_ptr(x) for x in out.valid])
    ep = (ctypes.c_void_p * max(nc, 1))(*[_ptr(x) for x in out.str_end])
    po = PpOutputs(out.cap_records, out.cap_fields, _ptr(out.record_offsets), _ptr(out.field_offsets),
                   _ptr(out.column_ids), ctypes.cast(vp, ctypes.c_void_p), ctypes.cast(mp, ctypes.c_void_p),
                   ctypes.cast(ep, ctypes.c_void_p), _ptr(out.result), _ptr(out.control_bitmap))
    _check(lib().pp_materialize_strings(d_in.data_ptr() if n else None, n, ctypes.byref(po), column, terminator,
                                        offsets.data_ptr(), chars.data_ptr(), cap_chars, ws.data_ptr(), ws.numel(),
                                        ctypes.c_void_p(stream.cuda_stream)), "pp_materialize_strings")
    offsets._keep = (ws, vp, mp, ep)  # alive until the caller synchronises
    return offsets, chars


def _outputs_struct(out: Outputs):
    nc = len(out.types)
    vp = (ctypes.c_void_p * max(nc, 1))(*[_ptr(x) for x in out.values])
    mp = (ctypes.c_void_p * max(nc, 1))(*[_ptr(x) for x in out.valid])
    ep = (ctypes.c_void_p * max(nc, 1))(*[_ptr(x) for x in out.str_end])
    po = PpOutputs(out.cap_records, out.cap_fields, _ptr(out.record_offsets), _ptr(out.field_offsets),
                   _ptr(out.column_ids), ctypes.cast(vp, ctypes.c_void_p), ctypes.cast(mp, ctypes.c_void_p),
                   ctypes.cast(ep, ctypes.c_void_p), _ptr(out.result), _ptr(out.control_bitmap))
    return po, (vp, mp, ep)


def infer_types(d_in, out: Outputs, ncols: Optional[int] = None, stream=None):
    """pp_infer_types over the string columns of a parse of ``d_in`` into
    ``out``: (inferred type per column, non-empty fields per column).
    Synchronises ``stream``."""
    import torch
    n = int(d_in.numel())
    ncols = len(out.types) if ncols is None else ncols
    if stream is None:
        stream = torch.cuda.current_stream()
    types = torch.empty(max(ncols, 1), dtype=torch.int32, device=d_in.device)
    nonempty = torch.empty(max(ncols, 1), dtype=torch.int64, device=d_in.device)
    ws = torch.empty(max(int(lib().pp_infer_types_workspace_size(ncols)), 1), dtype=torch.uint8, device=d_in.device)
    po, keep = _outputs_struct(out)
    _check(lib().pp_infer_types(d_in.data_ptr() if n else None, n, ctypes.byref(po), ncols, types.data_ptr(),
                                nonempty.data_ptr(), ws.data_ptr(), ws.numel(), ctypes.c_void_p(stream.cuda_stream)),
           "pp_infer_types")
    stream.synchronize()
    return types[:ncols].cpu().tolist(), nonempty[:ncols].cpu().numpy()


def parse_inferred(d_in, dfa, opts: Optional[PpOptions] = None, stream=None):
    """No schema: the column count (pp_infer_columns), a parse into that many
    string columns, their types (pp_infer_types), then the typed parse.
    Returns (Outputs, inferred types)."""
    raw, inf = parse_schemaless(d_in, dfa, opts, stream)
    types, _ = infer_types(d_in, raw, stream=stream)
    out = parse(d_in, dfa, types, inf["num_records"], inf["num_fields"], opts=opts, stream=stream)
    return out, types


def skip_rows(d_in, ranges, stream=None):
    """pp_skip_rows: the uint8 device tensor ``d_in`` without the rows
    (line-feed separated lines) in the half-open ranges [(first, last), ...].
    Returns a device tensor of the kept bytes (synchronises ``stream``)."""
    import torch
    n = int(d_in.numel())
    if stream is None:
        stream = torch.cuda.current_stream()
    flat = (ctypes.c_int64 * max(2 * len(ranges), 1))(*[int(x) for pr in ranges for x in pr])
    out = torch.empty(max(n, 1), dtype=torch.uint8, device=d_in.device)
    out_len = torch.zeros(1, dtype=torch.int64, device=d_in.device)
    ws = torch.empty(max(int(lib().pp_skip_rows_workspace_size(n)), 1), dtype=torch.uint8, device=d_in.device)
    _check(lib().pp_skip_rows(d_in.data_ptr() if n else None, n, flat, len(ranges), out.data_ptr(),
                              out_len.data_ptr(), ws.data_ptr(), ws.numel(), ctypes.c_void_p(stream.cuda_stream)),
           "pp_skip_rows")
    stream.synchronize()
    return out[:int(out_len.item())]


def skip_records(out: Outputs, ranges, stream=None) -> None:
    """pp_skip_records: clear the typed values of the records in the
    half-open ranges [(first, last), ...] of a parse into ``out``
    (asynchronous on ``stream``)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    flat = (ctypes.c_int64 * max(2 * len(ranges), 1))(*[int(x) for pr in ranges for x in pr])
    po, keep = _outputs_struct(out)
    t = (ctypes.c_int32 * max(len(out.types), 1))(*out.types)
    _check(lib().pp_skip_records(ctypes.byref(po), len(out.types), t, flat, len(ranges),
                                 ctypes.c_void_p(stream.cuda_stream)), "pp_skip_records")


def parse_noalloc(d_in, dfa, types: Sequence[int], cap_records: int, cap_fields: int,
                  opts: Optional[PpOptions] = None, stream=None) -> Outputs:
    """Like parse(), through pp_parse_noalloc: the library's static
    per-device workspace (NOALLOC_SCRATCH_BYTES), no workspace tensor.
    Calls on one GPU must not overlap in time."""
    n = int(d_in.numel())
    out = alloc_outputs(types, cap_records, cap_fields, device=d_in.device)
    call = Call(d_in, n, dfa, types, out, None, opts)
    call.launch_noalloc(stream)
    out._call = call
    return out


NOALLOC_SCRATCH_BYTES = 16 << 20


class PpBatchItem(ctypes.Structure):
    _fields_ = [("d_in", ctypes.c_void_p), ("n", ctypes.c_int64), ("dialect", ctypes.c_int32),
                ("ncols", ctypes.c_int32), ("types", ctypes.c_void_p), ("out", PpOutputs)]


def _check(rc, what):
    if rc != PP_OK:
        raise PpError(f"{what}: {STATUS_TEXT.get(rc, rc)}")


def _batch_items(items):
    """Marshal (d_in, dialect index, types, Outputs) tuples into a
    pp_batch_item_t array; returns it with the ctypes objects it points to."""
    keep = []
    arr = (PpBatchItem * max(len(items), 1))()
    for i, (d_in, dialect, types, out) in enumerate(items):
        n = int(d_in.numel())
        nc = len(types)
        t = (ctypes.c_int32 * max(nc, 1))(*types)
        vp = (ctypes.c_void_p * max(nc, 1))(*[_ptr(x) for x in out.values])
        mp = (ctypes.c_void_p * max(nc, 1))(*[_ptr(x) for x in out.valid])
        ep = (ctypes.c_void_p * max(nc, 1))(*[_ptr(x) for x in out.str_end])
        keep += [t, vp, mp, ep]
        arr[i].d_in = d_in.data_ptr() if n else None
        arr[i].n = n
        arr[i].dialect = dialect
        arr[i].ncols = nc
        arr[i].types = ctypes.cast(t, ctypes.c_void_p)
        arr[i].out = PpOutputs(out.cap_records, out.cap_fields, _ptr(out.record_offsets),
                               _ptr(out.field_offsets), _ptr(out.column_ids),
                               ctypes.cast(vp, ctypes.c_void_p), ctypes.cast(mp, ctypes.c_void_p),
                               ctypes.cast(ep, ctypes.c_void_p), _ptr(out.result), _ptr(out.control_bitmap))
    return arr, keep


class Batch:
    """Many buffers with their own dialects and outputs in one
    launch (pp_batch_*). ``items`` is a list of (d_in, dialect index, types,
    Outputs); ``dfas`` the dialect list the indexes refer to."""

    def __init__(self, dfas, items, opts: Optional[PpOptions] = None, stream=None):
        import torch
        L = lib()
        self._dfas = (PpDfa * len(dfas))(*[dfa_struct(d) for d in dfas])
        arr, self._keep = _batch_items(items)
        self.opts = opts
        self.items = items
        h = ctypes.c_void_p()
        _check(L.pp_batch_create(self._dfas, len(dfas), arr, len(items),
                                 ctypes.byref(opts) if opts else None, ctypes.byref(h)), "pp_batch_create")
        self.handle = h
        self.num_tiles = int(L.pp_batch_num_tiles(h))
        size = int(L.pp_batch_workspace_size(h))
        dev = items[0][0].device if items else torch.device("cuda")
        self.ws = torch.empty(max(size, 1), dtype=torch.uint8, device=dev)
        if stream is None:
            stream = torch.cuda.current_stream()
        _check(L.pp_batch_bind(h, self.ws.data_ptr(), self.ws.numel(), ctypes.c_void_p(stream.cuda_stream)),
               "pp_batch_bind")
        self.graph = None

    def launch(self, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        _check(lib().pp_batch_launch(self.handle, ctypes.c_void_p(stream.cuda_stream)), "pp_batch_launch")

    def capture(self):
        g = ctypes.c_void_p()
        _check(lib().pp_batch_graph_create(self.handle, ctypes.byref(g)), "pp_batch_graph_create")
        self.graph = g

    def replay(self, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        _check(lib().pp_batch_graph_launch(self.graph, ctypes.c_void_p(stream.cuda_stream)), "pp_batch_graph_launch")

    def close(self):
        L = lib()
        if self.graph is not None:
            L.pp_batch_graph_destroy(self.graph)
            self.graph = None
        if self.handle:
            L.pp_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- end-to-end streaming form ---------------------------------------------------

class PpStreamConfig(ctypes.Structure):
    _fields_ = [("partition_bytes", ctypes.c_int64), ("max_record_bytes", ctypes.c_int64),
                ("cap_records", ctypes.c_int64), ("cap_fields", ctypes.c_int64), ("opts", PpOptions)]


class PpHostOutputs(ctypes.Structure):
    _fields_ = [("cap_records", ctypes.c_int64), ("cap_fields", ctypes.c_int64),
                ("h_record_offsets", ctypes.c_void_p), ("h_field_offsets", ctypes.c_void_p),
                ("h_column_ids", ctypes.c_void_p), ("h_values", ctypes.c_void_p), ("h_valid", ctypes.c_void_p),
                ("h_str_end", ctypes.c_void_p)]


STREAM_STATS = ("partitions", "structure_passes", "carried_bytes", "max_carry", "bytes_returned")


class PpStreamStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in STREAM_STATS]


@dataclass
class HostOutputs:
    """Host output arrays (torch CPU tensors, pinned when pin=True) of a
    streamed parse, in the layout of Outputs."""
    cap_records: int
    cap_fields: int
    record_offsets: "object"
    field_offsets: "object"
    column_ids: "object"
    values: List[Optional[object]]
    valid: List[Optional[object]]
    str_end: List[Optional[object]]
    types: List[int]
    result: Optional[dict] = None
    stats: Optional[dict] = None


def alloc_host_outputs(types: Sequence[int], cap_records: int, cap_fields: int, pin: bool = True) -> HostOutputs:
    import torch

    def e(n, dt):
        return torch.empty(max(n, 1), dtype=dt, pin_memory=pin)
    vals, valid, ends = [], [], []
    for ty in types:
        if ty == SKIP:
            vals.append(None); valid.append(None); ends.append(None)
            continue
        vals.append(e(cap_records, torch.float64 if ty == FLOAT64 else torch.int64))
        valid.append(e(cap_records, torch.uint8))
        ends.append(e(cap_records, torch.int64) if ty == STRING else None)
    return HostOutputs(cap_records, cap_fields, e(cap_records + 1, torch.int64), e(cap_fields + 1, torch.int64),
                       e(cap_fields, torch.int32), vals, valid, ends, list(types))


class Stream:
    """pp_stream_*: a host-resident input parsed partition by partition with
    transfers, parsing and the return of the columns overlapped (Sec. 4.4)."""

    def __init__(self, dfa, types: Sequence[int], partition_bytes: int = 0, max_record_bytes: int = 0,
                 cap_records: int = 0, cap_fields: int = 0, opts: Optional[PpOptions] = None,
                 reject_ragged: bool = False):
        self._dfa = dfa_struct(dfa)
        self.types = list(types)
        nc = len(self.types)
        self._types = (ctypes.c_int32 * max(nc, 1))(*self.types)
        sch = PpSchema(nc, SCHEMA_REJECT_RAGGED if reject_ragged else 0, ctypes.cast(self._types, ctypes.c_void_p))
        cfg = PpStreamConfig(partition_bytes, max_record_bytes, cap_records, cap_fields, opts or PpOptions())
        h = ctypes.c_void_p()
        _check(lib().pp_stream_create(ctypes.byref(cfg), ctypes.byref(self._dfa), ctypes.byref(sch), ctypes.byref(h)),
               "pp_stream_create")
        self.handle = h

    def parse(self, h_in, out: HostOutputs) -> HostOutputs:
        """Parse the uint8 host tensor ``h_in`` (pinned for the full rate)
        into ``out``; returns ``out`` with ``result`` and ``stats`` set."""
        n = int(h_in.numel())
        nc = len(self.types)
        vp = (ctypes.c_void_p * max(nc, 1))(*[_ptr(x) for x in out.values])
        mp = (ctypes.c_void_p * max(nc, 1))(*[_ptr(x) for x in out.valid])
        ep = (ctypes.c_void_p * max(nc, 1))(*[_ptr(x) for x in out.str_end])
        ho = PpHostOutputs(out.cap_records, out.cap_fields, _ptr(out.record_offsets), _ptr(out.field_offsets),
                           _ptr(out.column_ids), ctypes.cast(vp, ctypes.c_void_p), ctypes.cast(mp, ctypes.c_void_p),
                           ctypes.cast(ep, ctypes.c_void_p))
        res = PpResult()
        st = PpStreamStats()
        _check(lib().pp_stream_parse(self.handle, h_in.data_ptr() if n else None, n, ctypes.byref(ho),
                                     ctypes.byref(res), ctypes.byref(st)), "pp_stream_parse")
        out.result = {f: getattr(res, f) for f in RESULT_FIELDS}
        out.stats = {f: getattr(st, f) for f in STREAM_STATS}
        return out

    def close(self):
        if self.handle:
            lib().pp_stream_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- serving form ------------------------------------------------------------

class PpServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_slots", ctypes.c_int32),
                ("copy_streams", ctypes.c_int32), ("compute_streams", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("opts", PpOptions)]


class PpServerRequest(ctypes.Structure):
    _fields_ = [("h_in", ctypes.c_void_p), ("n", ctypes.c_int64), ("dialect", ctypes.c_int32),
                ("ncols", ctypes.c_int32), ("types", ctypes.c_void_p), ("cap_records", ctypes.c_int64),
                ("cap_fields", ctypes.c_int64)]


class PpResult(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in RESULT_FIELDS]


class PpServerCompletion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("n", ctypes.c_int64), ("result", PpResult), ("out", PpOutputs),
                ("t_arrival_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64),
                ("t_h2d_done_ns", ctypes.c_int64), ("t_parse_done_ns", ctypes.c_int64)]


class PpServerStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in
                ("submitted", "completed", "reparsed", "batches", "batched_requests", "max_batch",
                 "bytes_completed", "arena_bytes", "arena_used_bytes", "arena_peak_bytes", "pending",
                 "hip_error")]


_hip = None


def _hip_lib():
    """The HIP runtime torch has loaded (for reading server outputs)."""
    global _hip
    if _hip is None:
        import torch  # noqa: F401  (loads the runtime)
        h = ctypes.CDLL("libamdhip64.so")
        h.hipMemcpy.restype = ctypes.c_int
        h.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip = h
    return _hip


def device_to_numpy(ptr: int, count: int, dtype):
    """Synchronous copy of ``count`` elements at device address ``ptr``."""
    import numpy as np
    a = np.empty(count, dtype=dtype)
    if count:
        rc = _hip_lib().hipMemcpy(a.ctypes.data, ptr, a.nbytes, 2)  # device to host
        if rc != 0:
            raise PpError(f"hipMemcpy failed ({rc})")
    return a


@dataclass
class Completion:
    id: int
    n: int
    result: dict
    t_arrival_ns: int
    t_admit_ns: int
    t_h2d_done_ns: int
    t_parse_done_ns: int
    _out: "PpServerCompletion"
    types: List[int]

    @property
    def latency_ns(self) -> int:
        return self.t_parse_done_ns - self.t_arrival_ns

    def fetch(self):
        """The request's outputs as numpy arrays (copied from the server's
        device memory): record_offsets[R+1], field_offsets[F+1],
        column_ids[F], and per column values/valid/str_end of R entries."""
        import numpy as np
        o = self._out.out
        R = min(self.result["num_records"], o.cap_records)
        F = min(self.result["num_fields"], o.cap_fields)
        got = {"record_offsets": device_to_numpy(o.d_record_offsets, R + 1, np.int64),
               "field_offsets": device_to_numpy(o.d_field_offsets, F + 1, np.int64),
               "column_ids": device_to_numpy(o.d_column_ids, F, np.int32),
               "values": [], "valid": [], "str_end": []}
        nc = len(self.types)
        vals = ctypes.cast(o.d_values, ctypes.POINTER(ctypes.c_void_p))
        vmask = ctypes.cast(o.d_valid, ctypes.POINTER(ctypes.c_void_p))
        ends = ctypes.cast(o.d_str_end, ctypes.POINTER(ctypes.c_void_p))
        for c in range(nc):
            ty = self.types[c]
            if ty == SKIP:
                got["values"].append(None); got["valid"].append(None); got["str_end"].append(None)
                continue
            got["values"].append(device_to_numpy(vals[c], R, np.float64 if ty == FLOAT64 else np.int64))
            got["valid"].append(device_to_numpy(vmask[c], R, np.uint8))
            got["str_end"].append(device_to_numpy(ends[c], R, np.int64) if ty == STRING else None)
        return got


class Server:
    """Request loop over pinned host inputs (pp_server_*). ``dfas`` are the
    dialects requests refer to by index."""

    def __init__(self, dfas, hbm_budget_bytes: int, max_slots: int = 64, copy_streams: int = 4,
                 compute_streams: int = 2, max_batch: int = 0, opts: Optional[PpOptions] = None):
        self._dfas = (PpDfa * len(dfas))(*[dfa_struct(d) for d in dfas])
        cfg = PpServerConfig(hbm_budget_bytes, max_slots, copy_streams, compute_streams, max_batch,
                             opts if opts else PpOptions(0, 0))
        h = ctypes.c_void_p()
        _check(lib().pp_server_create(ctypes.byref(cfg), self._dfas, len(dfas), ctypes.byref(h)),
               "pp_server_create")
        self.handle = h
        self._live = {}  # id -> (pinned tensor, types array, types list) kept alive until completion
        # a request can complete before its submit returns: submit records it
        # under this lock, which poll takes too
        self._lock = threading.Lock()
        self._buf = (PpServerCompletion * 256)()

    def submit(self, h_in, dialect: int, types: Sequence[int], cap_records: int, cap_fields: int) -> int:
        """``h_in``: a pinned uint8 CPU tensor, unchanged until completion."""
        nc = len(types)
        t = (ctypes.c_int32 * max(nc, 1))(*types)
        n = int(h_in.numel())
        rq = PpServerRequest(h_in.data_ptr() if n else None, n, dialect, nc, ctypes.cast(t, ctypes.c_void_p),
                             cap_records, cap_fields)
        rid = ctypes.c_uint64()
        with self._lock:
            _check(lib().pp_server_submit(self.handle, ctypes.byref(rq), ctypes.byref(rid)), "pp_server_submit")
            self._live[rid.value] = (h_in, t, list(types))
        return rid.value

    def poll(self, max_items: int = 256) -> List[Completion]:
        arr = (PpServerCompletion * 256)()
        got = ctypes.c_int32()
        _check(lib().pp_server_poll(self.handle, arr, min(max_items, len(arr)), ctypes.byref(got)),
               "pp_server_poll")
        out = []
        for i in range(got.value):
            c = arr[i]
            with self._lock:
                keep = self._live.pop(c.id, (None, None, []))
            cc = PpServerCompletion.from_buffer_copy(c)
            out.append(Completion(c.id, c.n, {f: getattr(c.result, f) for f in RESULT_FIELDS},
                                  c.t_arrival_ns, c.t_admit_ns, c.t_h2d_done_ns, c.t_parse_done_ns,
                                  cc, keep[2]))
        return out

    def wait(self, timeout_us: int = 1000) -> None:
        _check(lib().pp_server_wait(self.handle, timeout_us), "pp_server_wait")

    def release(self, rid: int) -> None:
        _check(lib().pp_server_release(self.handle, rid), "pp_server_release")

    def stats(self) -> dict:
        st = PpServerStats()
        _check(lib().pp_server_get_stats(self.handle, ctypes.byref(st)), "pp_server_get_stats")
        return {f: getattr(st, f) for f, _ in PpServerStats._fields_}

    def close(self):
        if self.handle:
            lib().pp_server_destroy(self.handle)
            self.handle = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- launch-shape autotuner ----------------------------------------------------

def shapes() -> List[PpOptions]:
    out = []
    for i in range(5):
        o = PpOptions()
        _check(lib().pp_shape(i, ctypes.byref(o)), "pp_shape")
        out.append(o)
    return out


def _tune_cache_path(path=None):
    return path or os.environ.get("PARPARAW_TUNE_CACHE",
                                  os.path.join(os.path.expanduser("~"), ".cache", "parparaw", "tune.json"))


def _tune_lookup(key, path):
    import json
    try:
        with open(path) as f:
            hit = json.load(f).get(key)
    except (OSError, ValueError):
        return None
    if hit:
        return PpOptions(hit["bytes_per_thread"], hit["block_threads"]), hit
    return None


def _tune_store(key, best, ms, path):
    import json
    d = {}
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        d = {}
    d[key] = {"bytes_per_thread": best.bytes_per_thread, "block_threads": best.block_threads,
              "ms": [round(float(x), 5) for x in ms]}
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return d[key]


def _device_tag():
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{getattr(p, 'gcnArchName', p.name)}/{p.multi_processor_count}cu"


def _bucket(x: int) -> int:
    return max(int(x), 1).bit_length()


def batch_signature(dfas, items) -> str:
    """Cache key of a batch: device, buffer count and total bytes (powers of
    two), largest state count among the dialects used."""
    total = sum(int(it[0].numel()) for it in items)
    states = max((dfas[it[1]].num_states for it in items), default=0)
    return f"{_device_tag()}|batch|n{_bucket(len(items))}|b{_bucket(total)}|s{states}"


def autotune_batch(dfas, items, reps: int = 3, cache: Optional[str] = None, stream=None, retune: bool = False):
    """Fastest launch shape for this batch (pp_batch_autotune), cached in a
    JSON file by batch_signature(). Returns (PpOptions, record)."""
    import torch
    path = _tune_cache_path(cache)
    key = batch_signature(dfas, items)
    if not retune:
        hit = _tune_lookup(key, path)
        if hit:
            return hit
    L = lib()
    d = (PpDfa * len(dfas))(*[dfa_struct(x) for x in dfas])
    arr, keep = _batch_items(items)
    size = int(L.pp_batch_autotune_workspace_size(d, len(dfas), arr, len(items)))
    dev = items[0][0].device if items else torch.device("cuda")
    ws = torch.empty(max(size, 1), dtype=torch.uint8, device=dev)
    if stream is None:
        stream = torch.cuda.current_stream()
    best = PpOptions()
    ms = (ctypes.c_float * 5)()
    _check(L.pp_batch_autotune(d, len(dfas), arr, len(items), ws.data_ptr(), ws.numel(), reps,
                               ctypes.c_void_p(stream.cuda_stream), ctypes.byref(best), ms), "pp_batch_autotune")
    return best, _tune_store(key, best, list(ms), path)


def autotune_parse(d_in, dfa, types: Sequence[int], out: Outputs, reps: int = 3, cache: Optional[str] = None,
                   stream=None, retune: bool = False):
    """Fastest launch shape for pp_parse of this input (pp_parse_autotune),
    cached by device, size (power of two), state count and column count."""
    import torch
    path = _tune_cache_path(cache)
    n = int(d_in.numel())
    key = f"{_device_tag()}|parse|b{_bucket(n)}|s{dfa.num_states}|c{len(types)}"
    if not retune:
        hit = _tune_lookup(key, path)
        if hit:
            return hit
    L = lib()
    ws = torch.empty(max(int(L.pp_autotune_workspace_size(n)), 1), dtype=torch.uint8, device=d_in.device)
    call = Call(d_in, n, dfa, types, out, ws)
    if stream is None:
        stream = torch.cuda.current_stream()
    best = PpOptions()
    ms = (ctypes.c_float * 5)()
    _check(L.pp_parse_autotune(d_in.data_ptr() if n else None, n, ctypes.byref(call.dfa), ctypes.byref(call.schema),
                               ctypes.byref(call.outs), ws.data_ptr(), ws.numel(), reps,
                               ctypes.c_void_p(stream.cuda_stream), ctypes.byref(best), ms), "pp_parse_autotune")
    return best, _tune_store(key, best, list(ms), path)
