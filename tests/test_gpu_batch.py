"""Batched form: one persistent launch over many buffers with mixed dialects
(3- to 8-state DFAs, comma/tab/pipe delimiters) and sizes from empty to
multi-tile, each buffer bit-exact against the oracle; a captured HIP graph
replayed several times gives the same outputs every time; the batched
outputs equal the single-buffer launches'."""
import random

import numpy as np
import pytest

import datagen
import oracle
import paper_1905_13415_amd as pp
from datagen import dialects as D
from parity import compare

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _schema(spec):
    return D.SCHEMA_LOG12.types if spec.kind == datagen.K_LOG else D.SCHEMA_C1.types


def _make_batch(nbuf, lo, hi, seed, extra=(), opts=None):
    dfas = datagen.c4_dialects()
    plan = datagen.c4_plan(seed=seed, count=nbuf, lo=lo, hi=hi)
    bufs = []
    for spec in plan:
        g = datagen.c4_buffer(spec, threads=4)
        bufs.append((g.data, spec.dialect, list(_schema(spec))))
    bufs.extend(extra)
    items, refs = [], []
    for data, dialect, types in bufs:
        ref = oracle.parse(data, dfas[dialect], types)
        d_in = torch.from_numpy(np.ascontiguousarray(data)).cuda() if len(data) else torch.empty(0, dtype=torch.uint8, device="cuda")
        out = pp.alloc_outputs(types, ref.num_records, ref.num_fields)
        items.append((d_in, dialect, types, out))
        refs.append(ref)
    return dfas, items, refs, pp.Batch(dfas, items, opts=opts)


def _extras():
    dfas = datagen.c4_dialects()
    csv4_comma = [d.name for d in dfas].index("csv4")
    rnd = random.Random(9)
    soup = bytes(rnd.choice(b'\n",ab1.-') for _ in range(70000))
    # numbers that begin tiles back (converted by the workgroup pass)
    digits = bytes(rnd.choice(b"0123456789") for _ in range(90000))
    longnum = b"1,2.5\n" + b"0" * 70000 + b"42,3." + digits + b"\n-" + b"0" * 40000 + b"7,1e" + b"0" * 50000 + b"5\n5,6\n"
    return [
        (np.frombuffer(longnum, np.uint8), csv4_comma, [D.INT64, D.FLOAT64]),        # long numbers
        (np.zeros(0, np.uint8), csv4_comma, [D.INT64, D.STRING]),                     # empty
        (np.frombuffer(b"7", np.uint8), csv4_comma, [D.INT64]),                       # one byte
        (np.frombuffer(b"," * 70000, np.uint8), csv4_comma, [D.INT64, D.STRING]),     # per-thread path
        (np.frombuffer(soup, np.uint8), csv4_comma, [D.STRING, D.INT64, D.FLOAT64]),  # symbol soup
        (np.frombuffer(soup, np.uint8), [d.name for d in dfas].index("paper6"), [D.STRING, D.INT64]),
    ]


def _check_all(items, refs, tag):
    for i, ((d_in, dialect, types, out), ref) in enumerate(zip(items, refs)):
        compare(ref, out, out.result_dict(), types, tag=f"{tag} buffer {i}")


@pytest.mark.parametrize("opts", [None, (32, 256), (16, 256)], ids=["512x64", "256x32", "256x16"])
def test_batch_mixed_dialects(opts):
    o = pp.options(*opts) if opts else None
    dfas, items, refs, batch = _make_batch(48, 1 << 10, 600 << 10, seed=11, extra=_extras(), opts=o)
    assert batch.num_tiles > len(items)
    batch.launch()
    torch.cuda.synchronize()
    _check_all(items, refs, "launch")
    batch.close()


def test_batch_graph_replays():
    dfas, items, refs, batch = _make_batch(24, 1 << 10, 300 << 10, seed=12, extra=_extras())
    batch.capture()
    for rep in range(3):
        for _, _, _, out in items:  # scribble over the outputs between replays
            out.field_offsets.fill_(-7)
            out.result.fill_(-7)
            for v in out.values:
                if v is not None:
                    v.view(torch.int64).fill_(-7)
        torch.cuda.synchronize()
        batch.replay()
        torch.cuda.synchronize()
        _check_all(items, refs, f"replay {rep}")
    batch.close()


def test_batch_equals_single_launches():
    dfas, items, refs, batch = _make_batch(16, 1 << 10, 200 << 10, seed=13)
    batch.launch()
    torch.cuda.synchronize()
    for i, (d_in, dialect, types, out) in enumerate(items):
        single = pp.parse(d_in, dfas[dialect], types, out.cap_records, out.cap_fields)
        torch.cuda.synchronize()
        assert single.result_dict() == out.result_dict()
        assert torch.equal(single.field_offsets, out.field_offsets)
        assert torch.equal(single.record_offsets, out.record_offsets)
        for a, b in zip(single.values, out.values):
            if a is not None:
                assert torch.equal(a.view(torch.int64), b.view(torch.int64))
    batch.close()


def test_autotune_batch_and_cache(tmp_path):
    cache = str(tmp_path / "tune.json")
    dfas, items, refs, batch = _make_batch(32, 1 << 10, 400 << 10, seed=14)
    batch.close()
    best, rec = pp.autotune_batch(dfas, items, reps=2, cache=cache)
    shapes = [(o.bytes_per_thread, o.block_threads) for o in pp.shapes()]
    assert (best.bytes_per_thread, best.block_threads) in shapes
    assert len(rec["ms"]) == 5 and all(m > 0 for m in rec["ms"])
    assert rec["ms"][shapes.index((best.bytes_per_thread, best.block_threads))] == min(rec["ms"])
    torch.cuda.synchronize()
    _check_all(items, refs, "after autotune")  # every shape gives the same outputs
    # second call: served from the cache file, same answer
    again, rec2 = pp.autotune_batch(dfas, items, cache=cache)
    assert (again.bytes_per_thread, again.block_threads) == (best.bytes_per_thread, best.block_threads)
    assert rec2["ms"] == rec["ms"]
    tuned = pp.Batch(dfas, items, opts=best)
    tuned.launch()
    torch.cuda.synchronize()
    _check_all(items, refs, "tuned launch")
    tuned.close()


def test_autotune_parse(tmp_path):
    g = datagen.c1()
    dfa = D.csv4()
    types = list(D.SCHEMA_C1.types)
    ref = oracle.parse(g.data, dfa, types)
    d_in = torch.from_numpy(g.data).cuda()
    out = pp.alloc_outputs(types, ref.num_records, ref.num_fields)
    best, rec = pp.autotune_parse(d_in, dfa, types, out, reps=2, cache=str(tmp_path / "t.json"))
    assert all(m > 0 for m in rec["ms"])
    torch.cuda.synchronize()
    compare(ref, out, out.result_dict(), types, tag="after parse autotune")
