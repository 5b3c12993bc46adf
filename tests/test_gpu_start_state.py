"""GPU parity for DFAs whose start state is not state 0, and for input made of
every byte value.

The DFAs are the library's dialects with their states renumbered (the same
automaton, so the same tags); the input's first field begins at byte 0 and is
a quoted field, or a quoted number, longer than one tile, so the tile where
it ends strips its opening quote by reading byte 0 in the start state (no
delimiter precedes it). Both the staged path and the per-thread path (a tile
of nothing but delimiters) close such a field. Every launch shape, and a
batch that mixes renumbered and original dialects.
"""
import random

import numpy as np
import pytest

import datagen
import oracle
import paper_1905_13415_amd as pp
from datagen import dialects as D
from parity import assert_same, compare

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

SHAPES = [None, (64, 256), (32, 256), (32, 512), (16, 256)]
SHAPE_IDS = ["512x64", "256x64", "256x32", "512x32", "256x16"]
RELABEL = [("csv4", [2, 0, 3, 1]), ("paper6", [3, 5, 0, 1, 4, 2]), ("log6", [5, 3, 0, 1, 2, 4]),
           ("s8", [6, 0, 1, 2, 3, 4, 5, 7])]
LONG = 40000  # longer than the largest tile (32 KiB)


def u8(b):
    return np.frombuffer(bytes(b), dtype=np.uint8)


def _inputs(name):
    """(bytes, types) cases whose first field is quoted and longer than a tile."""
    sp = b" " if name in ("log6", "s8") else b","
    rnd = random.Random(len(name))
    inner = bytes(rnd.choice(b"abc" + sp + b"\n") for _ in range(LONG))
    if name in ("csv4", "paper6"):
        inner = inner.replace(b'"', b"")
    tail = b"".join(b"%d%s%d%sx\n" % (i, sp, i * 3, sp) for i in range(3000))
    return [
        (b'"' + inner + b'"' + sp + b"5" + sp + b"y\n" + tail, [D.STRING, D.INT64, D.STRING]),
        (b'"' + b"0" * LONG + b'123"' + sp + b"9" + sp + b"z\n" + tail, [D.INT64, D.INT64, D.STRING]),
        # the tile where the long field ends holds nothing but delimiters (per-thread path)
        (b'"' + inner + b'"' + sp * LONG + b"\n" + tail, [D.STRING, D.INT64, D.STRING]),
        (b'"' + b"0" * LONG + b'77"' + sp * LONG + b"\n", [D.INT64, D.STRING]),
    ]


@pytest.mark.parametrize("shape", SHAPES, ids=SHAPE_IDS)
@pytest.mark.parametrize("name,perm", RELABEL, ids=[r[0] for r in RELABEL])
def test_relabelled_start_state(name, perm, shape):
    opts = pp.options(*shape) if shape else None
    base = D.ALL_DFAS[name]()
    rel = D.relabel(base, perm)
    assert rel.start_state != 0
    for data, types in _inputs(name):
        ref, _, res = assert_same(u8(data), rel, types, opts=opts)
        if types[0] == D.INT64:  # the quoted number converts: both quotes were control symbols
            assert ref.valid[0][0] == 1 and ref.values[0][0] in (123, 77)
        else:
            assert ref.values[0][0] == 1  # the span begins after the opening quote
        # the original numbering gives the same outputs
        assert_same(u8(data), base, types, opts=opts)


def test_batch_mixes_relabelled_and_original():
    dfas = []
    for name, perm in RELABEL:
        dfas += [D.ALL_DFAS[name](), D.relabel(D.ALL_DFAS[name](), perm)]
    items, refs = [], []
    for k, (name, _) in enumerate(RELABEL):
        for which in (2 * k, 2 * k + 1):
            for data, types in _inputs(name)[:2]:
                ref = oracle.parse(data, dfas[which], types)
                d_in = torch.from_numpy(u8(data).copy()).cuda()
                out = pp.alloc_outputs(types, ref.num_records, ref.num_fields)
                items.append((d_in, which, types, out))
                refs.append(ref)
    for opts in (None, pp.options(16, 256)):
        batch = pp.Batch(dfas, items, opts=opts)
        batch.launch()
        torch.cuda.synchronize()
        for i, ((_, which, types, out), ref) in enumerate(zip(items, refs)):
            compare(ref, out, out.result_dict(), types, tag=f"buffer {i} ({dfas[which].name})")
        batch.close()


def test_start_in_invalid_state_rejected():
    d = D.s5()
    d.invalid_state = d.start_state
    with pytest.raises(pp.PpError, match="DFA"):
        pp.parse(torch.zeros(4, dtype=torch.uint8, device="cuda"), d, [D.INT64], 4, 4)


# ---- every byte value ---------------------------------------------------------------

@pytest.mark.parametrize("shape", [None, (16, 256)], ids=["512x64", "256x16"])
@pytest.mark.parametrize("name", ["csv4", "s8", "paper6"])
def test_all_256_byte_values(name, shape):
    """Uniform random bytes over all 256 values (control bytes, NUL, bytes
    >= 0x80 in the catch-all group), then the same with every other byte a
    dialect symbol, so delimiters and quotes are dense."""
    opts = pp.options(*shape) if shape else None
    dfa = D.ALL_DFAS[name]()
    rng = np.random.default_rng(256 + len(name))
    types = [D.STRING, D.INT64, D.FLOAT64, D.STRING, D.DATE_DAYS]
    syms = np.frombuffer(b"".join(dfa.group_symbols), np.uint8)
    for n in (1000, 3 * 32768 + 123):
        data = rng.integers(0, 256, n, dtype=np.uint8)
        assert_same(data, dfa, types, opts=opts)
        dense = data.copy()
        dense[::2] = rng.choice(syms, size=len(dense[::2]))
        assert_same(dense, dfa, types, opts=opts)
