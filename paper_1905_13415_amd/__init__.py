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
from dataclasses import dataclass
from typing import List, Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
LIB_PATH = os.path.join(_HERE, "libparparaw.so")
SOURCES = [os.path.join(_HERE, "csrc", f) for f in ("parse.hip", "batch.hip", "serve.hip")]

PP_OK = 0
STATUS_TEXT = {0: "ok", -1: "invalid argument", -2: "invalid DFA", -3: "invalid schema",
               -4: "workspace too small", -5: "HIP launch failed", -6: "unsupported"}
INT64, FLOAT64, TIMESTAMP_S, DATE_DAYS, STRING, SKIP = 0, 1, 2, 3, 4, 5
RESULT_OK, RESULT_INVALID_INPUT, RESULT_NON_ACCEPTING_END, RESULT_CAPACITY = 0, 1, 2, 3
MAX_COLUMNS = 64

HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    """Compile the HIP sources for gfx950 into libparparaw.so (in-tree)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc] + HIPCC_FLAGS + ["-I", os.path.join(_ROOT, "include"),
                                   "-I", os.path.join(_HERE, "csrc")] + SOURCES + ["-o", LIB_PATH + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    if verbose:
        print(r.stderr)
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
                ("d_result", ctypes.c_void_p)]


class PpSchema(ctypes.Structure):
    _fields_ = [("ncols", ctypes.c_int32), ("types", ctypes.c_void_p)]


class PpOptions(ctypes.Structure):
    _fields_ = [("bytes_per_thread", ctypes.c_int32), ("block_threads", ctypes.c_int32)]


RESULT_FIELDS = ("status", "num_records", "num_fields", "first_invalid_offset", "final_state",
                 "num_conversion_errors", "num_ragged_records")

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


def options(bytes_per_thread: int = 0, block_threads: int = 0) -> PpOptions:
    return PpOptions(bytes_per_thread, block_threads)


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
    result: "object"  # int64[7] on device
    types: List[int]

    def result_dict(self):
        r = self.result.cpu().tolist()
        return dict(zip(RESULT_FIELDS, r))


def alloc_outputs(types: Sequence[int], cap_records: int, cap_fields: int, device="cuda") -> Outputs:
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
                   vals, valid, ends, torch.zeros(7, dtype=torch.int64, device=device), list(types))


def _ptr(t):
    return t.data_ptr() if t is not None else None


class Call:
    """The marshalled argument set of one pp_parse call; keeps the ctypes
    objects alive so the same call can be issued repeatedly (benchmarks)."""

    def __init__(self, d_in, n: int, dfa, types: Sequence[int], out: Outputs, workspace,
                 opts: Optional[PpOptions] = None):
        self.d_in = d_in
        self.n = n
        self.dfa = dfa_struct(dfa)
        nc = len(types)
        self.types = (ctypes.c_int32 * max(nc, 1))(*types)
        self.schema = PpSchema(nc, ctypes.cast(self.types, ctypes.c_void_p))
        self.vptr = (ctypes.c_void_p * max(nc, 1))(*[_ptr(t) for t in out.values])
        self.mptr = (ctypes.c_void_p * max(nc, 1))(*[_ptr(t) for t in out.valid])
        self.eptr = (ctypes.c_void_p * max(nc, 1))(*[_ptr(t) for t in out.str_end])
        self.outs = PpOutputs(out.cap_records, out.cap_fields, _ptr(out.record_offsets),
                              _ptr(out.field_offsets), _ptr(out.column_ids),
                              ctypes.cast(self.vptr, ctypes.c_void_p),
                              ctypes.cast(self.mptr, ctypes.c_void_p),
                              ctypes.cast(self.eptr, ctypes.c_void_p), _ptr(out.result))
        self.ws = workspace
        self.opts = opts
        self.out = out

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


def parse(d_in, dfa, types: Sequence[int], cap_records: int, cap_fields: int,
          opts: Optional[PpOptions] = None, stream=None) -> Outputs:
    """Parse the uint8 device tensor ``d_in`` (asynchronous on ``stream``)."""
    import torch
    n = int(d_in.numel())
    out = alloc_outputs(types, cap_records, cap_fields, device=d_in.device)
    ws = torch.empty(max(workspace_size(n, opts), 1), dtype=torch.uint8, device=d_in.device)
    call = Call(d_in, n, dfa, types, out, ws, opts)
    call.launch(stream)
    out._call = call  # keep workspace alive until the caller synchronises
    return out


class PpBatchItem(ctypes.Structure):
    _fields_ = [("d_in", ctypes.c_void_p), ("n", ctypes.c_int64), ("dialect", ctypes.c_int32),
                ("ncols", ctypes.c_int32), ("types", ctypes.c_void_p), ("out", PpOutputs)]


def _check(rc, what):
    if rc != PP_OK:
        raise PpError(f"{what}: {STATUS_TEXT.get(rc, rc)}")


class Batch:
    """Many buffers with their own dialects and outputs in one
    launch (pp_batch_*). ``items`` is a list of (d_in, dialect index, types,
    Outputs); ``dfas`` the dialect list the indexes refer to."""

    def __init__(self, dfas, items, opts: Optional[PpOptions] = None, stream=None):
        import torch
        L = lib()
        self._dfas = (PpDfa * len(dfas))(*[dfa_struct(d) for d in dfas])
        self._keep = []
        arr = (PpBatchItem * max(len(items), 1))()
        for i, (d_in, dialect, types, out) in enumerate(items):
            n = int(d_in.numel())
            nc = len(types)
            t = (ctypes.c_int32 * max(nc, 1))(*types)
            vp = (ctypes.c_void_p * max(nc, 1))(*[_ptr(x) for x in out.values])
            mp = (ctypes.c_void_p * max(nc, 1))(*[_ptr(x) for x in out.valid])
            ep = (ctypes.c_void_p * max(nc, 1))(*[_ptr(x) for x in out.str_end])
            self._keep += [t, vp, mp, ep]
            arr[i].d_in = d_in.data_ptr() if n else None
            arr[i].n = n
            arr[i].dialect = dialect
            arr[i].ncols = nc
            arr[i].types = ctypes.cast(t, ctypes.c_void_p)
            arr[i].out = PpOutputs(out.cap_records, out.cap_fields, _ptr(out.record_offsets),
                                   _ptr(out.field_offsets), _ptr(out.column_ids),
                                   ctypes.cast(vp, ctypes.c_void_p), ctypes.cast(mp, ctypes.c_void_p),
                                   ctypes.cast(ep, ctypes.c_void_p), _ptr(out.result))
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
