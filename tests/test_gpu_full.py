"""Parity at the full workload sizes, in the launch configuration the
benchmark times.

- The 1 GiB numeric CSV and the 2 GiB text-heavy CSV, parsed by one plain
  launch with the default shape (512 threads x 64 bytes), compared with the
  oracle element by element (every offset, column id, value and flag).
- The 4,096-buffer batch (sizes log-uniform up to 64 MiB, 18 dialects, 23.7
  GB), parsed by one captured batched launch with the shape the autotuner
  picks: every buffer's result record against the generator's record,
  field and column counts, and every buffer against the oracle element by
  element.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import datagen
import oracle
import paper_1905_13415_amd as pp
from datagen import dialects as D
from parity import assert_same, compare

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def test_full_numeric_1gib():
    g = datagen.c2()
    assert len(g.data) > (1 << 30) - 512
    ref, out, res = assert_same(g.data, D.csv4(), D.SCHEMA_C2.types)
    assert ref.num_records == g.nrecords and ref.num_fields == g.nrecords * g.ncols


def test_full_text_2gib():
    g = datagen.c3()
    assert len(g.data) > (1 << 31) - (1 << 18)
    ref, out, res = assert_same(g.data, D.csv4(), D.SCHEMA_C3.types)
    assert ref.num_records == g.nrecords


def test_full_batch_4096_buffers():
    dfas = datagen.c4_dialects()
    plan = datagen.c4_plan()
    gens = [datagen.c4_buffer(spec) for spec in plan]
    sizes = [len(g.data) for g in gens]
    dev = torch.device("cuda:0")
    offs, off = [], 0
    for n in sizes:
        offs.append(off)
        off += (n + 255) // 256 * 256
    arena = torch.empty(off, dtype=torch.uint8, device=dev)
    items, expect = [], []
    for spec, g, o in zip(plan, gens, offs):
        types = list(D.SCHEMA_LOG12.types if spec.kind == datagen.K_LOG else D.SCHEMA_C1.types)
        if len(g.data):
            arena[o:o + len(g.data)].copy_(torch.from_numpy(g.data))
        R, F = g.nrecords, g.nrecords * g.ncols
        items.append((arena[o:o + len(g.data)], spec.dialect, types, pp.alloc_outputs(types, R, F, device=dev)))
        expect.append((R, F, g.ncols))
    best, _ = pp.autotune_batch(dfas, items, reps=1)
    batch = pp.Batch(dfas, items, opts=best)
    batch.capture()
    batch.replay()
    torch.cuda.synchronize()
    res = torch.stack([it[3].result for it in items]).cpu().numpy()
    for i, (R, F, nc) in enumerate(expect):
        assert res[i, 0] == pp.RESULT_OK and res[i, 1] == R and res[i, 2] == F, (i, res[i].tolist())
        if R:  # every generated record has the schema's column count
            assert res[i, 7] == nc and res[i, 8] == nc, (i, res[i].tolist())

    # every buffer element by element against the oracle, on a host thread
    # pool (the oracle and the comparisons release the interpreter lock)
    def check(i):
        d_in, dialect, types, out = items[i]
        ref = oracle.parse(gens[i].data, dfas[dialect], types)
        compare(ref, out, out.result_dict(), types, tag=f"buffer {i} ({sizes[i]} bytes, {dfas[dialect].name})")
        return sizes[i]

    workers = min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(workers) as pool:
        checked = sum(pool.map(check, range(len(plan))))
    assert checked == sum(sizes)
    batch.close()
