"""Seeded synthetic inputs and dialects for the parse workloads.

The byte generator is C (``gen.c``, loaded with ctypes); blocks of records
are generated on a thread pool (ctypes releases the GIL) and concatenated.
Every block has its own random stream keyed by (seed, block index), so the
output does not depend on the thread count.

Workloads (sizes are bytes of whole records):
  c1   10,000 records x 8 columns, comma CSV, 20% of strings quoted with an
       embedded comma, LF and doubled quote                     (~1.4 MB)
  c2   numeric CSV, 18 columns, ~130 B per record, unquoted    (up to 2^30 B)
  c3   text-heavy CSV, 9 columns, 2 quoted free-text fields of lognormal
       length (mean ~300 B each), ~700 B per record            (up to 2^31 B)
  mixed  C1-like records in a given dialect (delimiter, quoting style)
  log  12-column extended web-server log, space delimited, quoted request
       strings with backslash escapes, bracketed timestamps
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

from . import dialects  # noqa: F401
from .dialects import (Dfa, Schema, SCHEMA_C1, SCHEMA_C2, SCHEMA_C3, SCHEMA_LOG12)
from .dialects import SCHEMA_C1 as SCHEMA_MIXED

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libdatagen.so")

K_C1, K_C2, K_C3, K_MIXED, K_LOG = 1, 2, 3, 4, 5
NCOLS = {K_C1: 8, K_C2: 18, K_C3: 9, K_MIXED: 8, K_LOG: 12}
# bytes per record, an upper estimate used to size block buffers
REC_BOUND = {K_C1: 400, K_C2: 220, K_C3: 140000, K_MIXED: 400, K_LOG: 800}
SEED_BASE = 190513415


def build() -> str:
    subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", _LIB, _SRC, "-lm"])
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.dg_block.restype = ctypes.c_int64
        lib.dg_block.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                 ctypes.c_int64, ctypes.c_int, ctypes.c_int, P, ctypes.c_int64,
                                 P, P, P, P, P, P, P]
        _lib = lib
    return _lib


@dataclass
class Truth:
    """What the generator wrote, per (record, column): raw field start,
    content span, drawn value. kind: 0 null text, 1 integer-like, 2 float
    (ival / 10**aux), 3 text."""
    fbeg: np.ndarray
    vbeg: np.ndarray
    vend: np.ndarray
    ival: np.ndarray
    aux: np.ndarray
    kind: np.ndarray


@dataclass
class Generated:
    data: np.ndarray          # uint8
    nrecords: int
    ncols: int
    truth: Optional[Truth]


def _ptr(a):
    return a.ctypes.data if a is not None else None


def _gen_block(kind, seed, block, nrec, max_bytes, delim, qstyle, with_truth):
    lib = _load()
    ncols = NCOLS[kind]
    cap = min(max_bytes, nrec * REC_BOUND[kind])
    out = np.empty(cap, dtype=np.uint8)
    t = None
    if with_truth:
        m = nrec * ncols
        t = [np.zeros(m, np.int64), np.zeros(m, np.int64), np.zeros(m, np.int64),
             np.zeros(m, np.int64), np.zeros(m, np.int32), np.zeros(m, np.int8)]
    nr = ctypes.c_int64(0)
    nb = lib.dg_block(kind, seed, block, nrec, max_bytes, delim, qstyle, out.ctypes.data, cap,
                      *([_ptr(a) for a in t] if t else [None] * 6), ctypes.byref(nr))
    assert nb >= 0
    nrec_got = nr.value
    if t:
        t = [a[: nrec_got * ncols] for a in t]
    return out[:nb], nrec_got, t


def generate(kind: int, seed: int, *, max_records: int = 1 << 62, max_bytes: int = 1 << 62,
                 delim: bytes = b",", qstyle: int = 1, with_truth: bool = False,
                 block_records: int = 16384, threads: int = 16) -> Generated:
    """Deterministic block-parallel generation.

    Blocks are generated in parallel with a per-block byte limit of
    ``max_bytes``; they are concatenated in order, and the block that would
    cross ``max_bytes`` is regenerated with the remaining room as its limit
    (its stream is keyed by its index, so it yields the same records up to
    the cut). Blocks after it are dropped.
    """
    ncols = NCOLS[kind]
    d = delim[0]
    chunks, truths = [], []
    total_b, total_r, block = 0, 0, 0
    done = False
    with ThreadPoolExecutor(max_workers=threads) as ex:
        while not done:
            jobs = []
            for _ in range(threads):
                nrec = int(min(block_records, max_records - total_r - sum(j[1] for j in jobs)))
                if nrec <= 0:
                    break
                jobs.append((block, nrec, ex.submit(_gen_block, kind, seed, block, nrec,
                                                    max_bytes, d, qstyle, with_truth)))
                block += 1
            if not jobs:
                break
            for blk, nrec, fut in jobs:
                out, nr, t = fut.result()
                if done:
                    continue
                if total_b + len(out) > max_bytes or nr < nrec:
                    out, nr, t = _gen_block(kind, seed, blk, nrec, max_bytes - total_b, d, qstyle,
                                            with_truth)
                    done = True
                if t:
                    t = list(t)
                    for i in range(3):
                        t[i] = t[i] + total_b
                    truths.append(t)
                chunks.append(out)
                total_b += len(out)
                total_r += nr
                if total_r >= max_records:
                    done = True
    data = np.concatenate(chunks) if chunks else np.zeros(0, np.uint8)
    truth = None
    if with_truth:
        if truths:
            cat = [np.concatenate([t[i] for t in truths]) for i in range(6)]
        else:
            cat = [np.zeros(0, np.int64)] * 4 + [np.zeros(0, np.int32), np.zeros(0, np.int8)]
        truth = Truth(*[c.reshape(-1, ncols) for c in cat])
    return Generated(data, total_r, ncols, truth)


# ---- named workloads ------------------------------------------------------

def c1(seed: int = SEED_BASE + 0, with_truth: bool = False) -> Generated:
    return generate(K_C1, seed, max_records=10000, with_truth=with_truth)


def c2(seed: int = SEED_BASE + 1, nbytes: int = 1 << 30, with_truth: bool = False) -> Generated:
    return generate(K_C2, seed, max_bytes=nbytes, with_truth=with_truth)


def c3(seed: int = SEED_BASE + 2, nbytes: int = 1 << 31, with_truth: bool = False) -> Generated:
    return generate(K_C3, seed, max_bytes=nbytes, with_truth=with_truth, block_records=1024)


def mixed(seed: int, nbytes: int, delim: bytes = b",", qstyle: int = 1,
          with_truth: bool = False) -> Generated:
    return generate(K_MIXED, seed, max_bytes=nbytes, delim=delim, qstyle=qstyle,
                        with_truth=with_truth, block_records=4096)


def log(seed: int, nbytes: int, delim: bytes = b" ", with_truth: bool = False) -> Generated:
    return generate(K_LOG, seed, max_bytes=nbytes, delim=delim, with_truth=with_truth,
                        block_records=4096)


SCHEMAS = {"c1": SCHEMA_C1, "c2": SCHEMA_C2, "c3": SCHEMA_C3, "log": SCHEMA_LOG12}


# ---- the batched workload: many buffers, mixed dialects -----------------------

# DFA family of 3 to 8 states and the content style each one parses:
# (dfa factory name, generator kind, quoting style)
C4_FAMILY = [("s3", K_MIXED, 3), ("csv4", K_MIXED, 1), ("s5", K_MIXED, 1),
             ("paper6", K_MIXED, 1), ("s7", K_MIXED, 2), ("s8", K_LOG, 0)]
C4_DELIMS = [b",", b"\t", b"|"]


@dataclass
class BufferSpec:
    index: int
    dfa_name: str
    delim: bytes
    kind: int
    qstyle: int
    nbytes: int   # size limit (whole records up to it)
    seed: int

    @property
    def dialect(self) -> int:
        return [n for n, _, _ in C4_FAMILY].index(self.dfa_name) * len(C4_DELIMS) + C4_DELIMS.index(self.delim)


def c4_dialects():
    """The 18 dialects (6 DFAs x 3 delimiters), in dialect-index order."""
    out = []
    for name, _, _ in C4_FAMILY:
        for d in C4_DELIMS:
            out.append(dialects.ALL_DFAS[name](d))
    return out


def c4_plan(seed: int = SEED_BASE + 3, count: int = 4096, lo: int = 1 << 10, hi: int = 64 << 20):
    """Buffer sizes log-uniform in [lo, hi] and a uniformly drawn dialect per
    buffer (numpy PCG64 seeded with ``seed``)."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(np.log(lo), np.log(hi), size=count)).astype(np.int64)
    fam = rng.integers(0, len(C4_FAMILY), size=count)
    dl = rng.integers(0, len(C4_DELIMS), size=count)
    plan = []
    for i in range(count):
        name, kind, q = C4_FAMILY[int(fam[i])]
        plan.append(BufferSpec(i, name, C4_DELIMS[int(dl[i])], kind, q, int(sizes[i]), seed * 7919 + i))
    return plan


def c4_buffer(spec: BufferSpec, threads: int = 16) -> Generated:
    if spec.kind == K_LOG:
        return generate(K_LOG, spec.seed, max_bytes=spec.nbytes, delim=spec.delim, block_records=4096,
                        threads=threads)
    return generate(K_MIXED, spec.seed, max_bytes=spec.nbytes, delim=spec.delim, qstyle=spec.qstyle,
                    block_records=4096, threads=threads)
