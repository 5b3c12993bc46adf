"""Oracle: a plain sequential CPU parser, and a plain model of the paper's
chunked formulation -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. The GPU library never loads it, and this package never
imports the GPU library.

``parse`` runs ``oracle.c``: one DFA instance from the start state, front to
back (Sec. 3.1), delimiters counted in order into record and column offsets
(Sec. 3.2), fields converted per column type (Sec. 3.3) with defaults for
empty and missing fields (Sec. 4.3). ``method_model`` restates the chunked
method itself (state-transition vectors, their composition and scans,
Sec. 3.1-3.2) for small inputs, so tests can check that it reaches the same
result as the sequential run.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

STATUS_OK, STATUS_INVALID_INPUT, STATUS_NON_ACCEPTING_END, STATUS_CAPACITY = 0, 1, 2, 3
INT64, FLOAT64, TIMESTAMP_S, DATE_DAYS, STRING, SKIP = 0, 1, 2, 3, 4, 5


def build() -> str:
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-o", _LIB,
                           _SRC, "-lm"])
    return _LIB


class _OrcDfa(ctypes.Structure):
    _fields_ = [("num_states", ctypes.c_int32), ("num_groups", ctypes.c_int32),
                ("start_state", ctypes.c_int32), ("invalid_state", ctypes.c_int32),
                ("accept_mask", ctypes.c_uint32), ("group_of", ctypes.c_uint8 * 256),
                ("next", (ctypes.c_uint8 * 16) * 16), ("tag", (ctypes.c_uint8 * 16) * 16)]


class _OrcResult(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "status", "num_records", "num_fields", "first_invalid_offset", "final_state",
        "num_conversion_errors", "num_ragged_records", "min_record_fields", "max_record_fields")]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.orc_parse.restype = ctypes.c_int
        lib.orc_parse.argtypes = [P, ctypes.c_int64, P, ctypes.c_int32, P, ctypes.c_int64,
                                  ctypes.c_int64, P, P, P, P, P, P, P]
        lib.orc_conv.restype = ctypes.c_int
        lib.orc_parse_utf16.restype = ctypes.c_int
        lib.orc_parse_utf16.argtypes = lib.orc_parse.argtypes
        lib.orc_skip_rows.restype = ctypes.c_int64
        lib.orc_skip_rows.argtypes = [P, ctypes.c_int64, P, ctypes.c_int32, P]
        lib.orc_infer_types.restype = None
        lib.orc_infer_types.argtypes = [P, ctypes.c_int64, P, ctypes.c_int32, P, P]
        lib.orc_materialize.restype = ctypes.c_int64
        lib.orc_materialize.argtypes = [P, ctypes.c_int64, P, ctypes.c_int32, ctypes.c_int64, P, P, ctypes.c_int64,
                                        ctypes.c_int32]
        lib.orc_materialize_utf16.restype = ctypes.c_int64
        lib.orc_materialize_utf16.argtypes = lib.orc_materialize.argtypes
        lib.orc_reject_ragged.restype = None
        lib.orc_reject_ragged.argtypes = [ctypes.c_int32, P, ctypes.c_int64, P, P, P, P]
        lib.orc_conv.argtypes = [ctypes.c_int32, P, ctypes.c_int64,
                                 ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]
        _lib = lib
    return _lib


def _dfa_struct(dfa) -> _OrcDfa:
    d = _OrcDfa()
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


@dataclass
class ParseResult:
    status: int
    num_records: int
    num_fields: int
    first_invalid_offset: int
    final_state: int
    num_conversion_errors: int
    num_ragged_records: int
    min_record_fields: int          # fewest fields in a record, -1 without records
    max_record_fields: int          # most fields in a record (the inferred column count)
    record_offsets: np.ndarray      # int64[R+1]
    field_offsets: np.ndarray       # int64[F+1]
    column_ids: np.ndarray          # int32[F]
    values: List[Optional[np.ndarray]]   # per column: int64 or float64 [R]
    valid: List[Optional[np.ndarray]]    # per column: uint8 [R]
    str_end: List[Optional[np.ndarray]]  # per STRING column: int64 [R]


def _as_u8(buf) -> np.ndarray:
    if isinstance(buf, (bytes, bytearray)):
        return np.frombuffer(bytes(buf), dtype=np.uint8)
    return np.ascontiguousarray(buf, dtype=np.uint8)


def _units(buf):
    """UTF-16LE bytes (even length) as little-endian 16-bit code units."""
    a = _as_u8(buf)
    if len(a) % 2:
        raise ValueError("oracle: UTF-16 input of odd length")
    return np.ascontiguousarray(a.view("<u2")).astype(np.uint16)


def count(buf, dfa, utf16: bool = False):
    """(R, F) of the sequential run, without writing outputs. ``utf16``: the
    bytes are UTF-16LE text (Sec. 4.2)."""
    lib = _load()
    a = _units(buf) if utf16 else _as_u8(buf)
    d = _dfa_struct(dfa)
    res = _OrcResult()
    fn = lib.orc_parse_utf16 if utf16 else lib.orc_parse
    rc = fn(a.ctypes.data, len(a), ctypes.byref(d), 0, None, 0, 0,
            None, None, None, None, None, None, ctypes.byref(res))
    if rc != 0:
        raise ValueError("oracle: rejected arguments (a DFA that starts in its invalid state?)")
    return res.num_records, res.num_fields


def parse(buf, dfa, schema_types, cap_records: Optional[int] = None,
          cap_fields: Optional[int] = None, reject_ragged: bool = False, utf16: bool = False) -> ParseResult:
    """Sequential parse of ``buf`` under ``dfa`` into the full output set.

    With no capacities given, the exact sizes are counted first.
    ``reject_ragged``: records whose field count differs from the schema's
    column count lose their typed values (Sec. 4.3). ``utf16``: ``buf`` is
    UTF-16LE text, parsed per code unit; positions stay byte offsets."""
    lib = _load()
    a = _units(buf) if utf16 else _as_u8(buf)
    types = list(schema_types)
    if cap_records is None or cap_fields is None:
        r, f = count(buf if utf16 else a, dfa, utf16=utf16)
        cap_records = r if cap_records is None else cap_records
        cap_fields = f if cap_fields is None else cap_fields
    ncols = len(types)
    rec = np.zeros(cap_records + 1, np.int64)
    fld = np.zeros(cap_fields + 1, np.int64)
    cid = np.zeros(max(cap_fields, 1), np.int32)
    values, valid, str_end = [], [], []
    vptr = (ctypes.c_void_p * max(ncols, 1))()
    mptr = (ctypes.c_void_p * max(ncols, 1))()
    eptr = (ctypes.c_void_p * max(ncols, 1))()
    for c, ty in enumerate(types):
        if ty == SKIP:
            values.append(None); valid.append(None); str_end.append(None)
            continue
        v = np.zeros(max(cap_records, 1), np.float64 if ty == FLOAT64 else np.int64)
        m = np.zeros(max(cap_records, 1), np.uint8)
        e = np.zeros(max(cap_records, 1), np.int64) if ty == STRING else None
        values.append(v); valid.append(m); str_end.append(e)
        vptr[c] = v.ctypes.data
        mptr[c] = m.ctypes.data
        eptr[c] = e.ctypes.data if e is not None else None
    tarr = np.array(types if types else [0], dtype=np.int32)
    d = _dfa_struct(dfa)
    res = _OrcResult()
    fn = lib.orc_parse_utf16 if utf16 else lib.orc_parse
    rc = fn(a.ctypes.data, len(a), ctypes.byref(d), ncols, tarr.ctypes.data,
            cap_records, cap_fields, rec.ctypes.data, fld.ctypes.data, cid.ctypes.data,
            vptr, mptr, eptr, ctypes.byref(res))
    if rc != 0:
        raise ValueError("oracle: rejected arguments (a DFA that starts in its invalid state?)")
    R = min(res.num_records, cap_records)
    F = min(res.num_fields, cap_fields)
    if reject_ragged:
        lib.orc_reject_ragged(ncols, tarr.ctypes.data, R, rec.ctypes.data, vptr, mptr, eptr)
    return ParseResult(res.status, res.num_records, res.num_fields, res.first_invalid_offset,
                       res.final_state, res.num_conversion_errors, res.num_ragged_records,
                       res.min_record_fields, res.max_record_fields,
                       rec[:R + 1], fld[:F + 1], cid[:F],
                       [x[:R] if x is not None else None for x in values],
                       [x[:R] if x is not None else None for x in valid],
                       [x[:R] if x is not None else None for x in str_end])


def convert(type_code: int, text: bytes):
    """One field through the oracle's conversion: (ok, int value, float value)."""
    lib = _load()
    iv = ctypes.c_int64(0)
    dv = ctypes.c_double(0.0)
    buf = ctypes.create_string_buffer(bytes(text), max(len(text), 1))
    ok = lib.orc_conv(type_code, buf, len(text), ctypes.byref(iv), ctypes.byref(dv))
    return bool(ok), iv.value, dv.value


def materialize(buf, dfa, column: int, terminator: int = -1, utf16: bool = False):
    """A string column's materialised values (all control symbols removed),
    as (offsets int64[R+1], chars uint8[total]) in the Arrow large-string
    layout; terminator >= 0 appends that byte to every value (the
    inline-terminated form). ``utf16``: UTF-16LE text; offsets count code
    units and chars are uint16 code units."""
    lib = _load()
    a = _units(buf) if utf16 else _as_u8(buf)
    R, _ = count(buf if utf16 else a, dfa, utf16=utf16)
    d = _dfa_struct(dfa)
    offs = np.zeros(R + 1, np.int64)
    fn = lib.orc_materialize_utf16 if utf16 else lib.orc_materialize
    total = fn(a.ctypes.data, len(a), ctypes.byref(d), column, R, offs.ctypes.data, None, 0, terminator)
    chars = np.zeros(max(total, 1), np.uint16 if utf16 else np.uint8)
    fn(a.ctypes.data, len(a), ctypes.byref(d), column, R, offs.ctypes.data, chars.ctypes.data, total, terminator)
    return offs, chars[:total]


def infer_types(buf, dfa, ncols: int):
    """Inferred column types (Sec. 4.3) of the first ncols columns and the
    number of non-empty fields of each: (types list, nonempty int64[ncols])."""
    lib = _load()
    a = _as_u8(buf)
    d = _dfa_struct(dfa)
    types = np.zeros(max(ncols, 1), np.int32)
    nonempty = np.zeros(max(ncols, 1), np.int64)
    lib.orc_infer_types(a.ctypes.data, len(a), ctypes.byref(d), ncols, types.ctypes.data, nonempty.ctypes.data)
    return [int(t) for t in types[:ncols]], nonempty[:ncols]


def skip_rows(buf, ranges):
    """The input without the rows (line-feed separated lines) in the
    half-open ranges [(first, last), ...] (Sec. 4.3, skipping rows)."""
    lib = _load()
    a = _as_u8(buf)
    r = np.array([x for pair in ranges for x in pair] or [0], dtype=np.int64)
    out = np.zeros(max(len(a), 1), np.uint8)
    m = lib.orc_skip_rows(a.ctypes.data, len(a), r.ctypes.data, len(ranges), out.ctypes.data)
    return out[:m]


def skip_records(res: ParseResult, types, ranges) -> ParseResult:
    """Skipping records (Sec. 4.3): the typed values of the records in the
    half-open ranges [(first, last), ...] become the column defaults (value
    0, valid 0, empty span); everything else is unchanged. Modifies and
    returns ``res``."""
    for c, ty in enumerate(types):
        if ty == SKIP:
            continue
        for a, b in ranges:
            res.values[c][a:b] = 0
            res.valid[c][a:b] = 0
            if ty == STRING:
                res.str_end[c][a:b] = 0
    return res
