"""GPU parity on random DFAs: the library takes any DFA of up to 8 states and
16 symbol groups (Sec. 3.1: the method is defined for an arbitrary DFA and
tag table), so dialects drawn at random -- random transitions, tags of all
four kinds in any state (control symbols and delimiters where no real format
would put them), random start and accepting states, with or without an
absorbing invalid state -- are parsed through the plain launch (every launch
shape, and the tiles out of order) and the batched form, and every output
is compared with the oracle's bit for bit. Inputs are drawn over the
dialect's own symbols plus digits, signs and letters, so that delimiters,
control symbols and conversions all occur, at sizes from one byte to many
tiles. String materialisation and type inference run under random dialects
too."""
import random

import numpy as np
import pytest

import oracle
import paper_1905_13415_amd as pp
from datagen import dialects as D
from parity import assert_same, compare

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

SYMBOLS = b'\n",;|\t[]\\ :#'
FILLER = b"0123456789.-+eE:T abz"
SHAPES = [None, (64, 256), (32, 512), (16, 256)]


def random_dfa(rnd: random.Random, name: str) -> D.Dfa:
    ns = rnd.randint(2, 8)
    ng = rnd.randint(2, 8)
    syms = rnd.sample(list(SYMBOLS), ng - 1)  # one byte per explicit group; the last group takes the rest
    groups = [bytes([b]) for b in syms]
    kinds = [D.DATA] * 5 + [D.FIELD] * 2 + [D.RECORD] * 2 + [D.CONTROL] * 2
    nxt = [[rnd.randrange(ns) for _ in range(ns)] for _ in range(ng)]
    tag = [[rnd.choice(kinds) for _ in range(ns)] for _ in range(ng)]
    start = rnd.randrange(ns)
    invalid = D.NO_STATE
    if ns > 2 and rnd.random() < 0.5:
        invalid = rnd.choice([s for s in range(ns) if s != start])
        for g in range(ng):
            nxt[g][invalid] = invalid  # absorbing
    accept = [s for s in range(ns) if rnd.random() < 0.6] or [start]
    return D.Dfa(name, [f"S{i}" for i in range(ns)], groups, nxt, tag, start, accept, invalid)


def random_input(rnd: random.Random, dfa: D.Dfa, n: int) -> np.ndarray:
    alphabet = b"".join(dfa.group_symbols) * 3 + FILLER
    return np.frombuffer(bytes(rnd.choice(alphabet) for _ in range(n)), dtype=np.uint8)


def random_types(rnd: random.Random):
    return [rnd.choice([D.INT64, D.FLOAT64, D.TIMESTAMP_S, D.DATE_DAYS, D.STRING, D.SKIP])
            for _ in range(rnd.randint(0, 9))]


@pytest.mark.parametrize("seed", range(16))
def test_random_dfas_plain(seed):
    rnd = random.Random(1000 + seed)
    for k in range(5):
        dfa = random_dfa(rnd, f"r{seed}_{k}")
        types = random_types(rnd)
        for n in (1, 777, 3 * 32768 + 5):
            data = random_input(rnd, dfa, n)
            shape = SHAPES[(k + n) % len(SHAPES)]
            assert_same(data, dfa, types, opts=pp.options(*shape) if shape else None)
        # many tiles, parsed out of order
        data = random_input(rnd, dfa, 150 * 4096 + 99)
        assert_same(data, dfa, types, opts=pp.options(16, 256, 1 + k))


def test_random_dfas_batched():
    """One batch whose buffers each have their own random dialect."""
    rnd = random.Random(77)
    dfas = [random_dfa(rnd, f"b{i}") for i in range(12)]
    items, refs = [], []
    for i in range(40):
        d = i % len(dfas)
        types = random_types(rnd)
        data = random_input(rnd, dfas[d], rnd.choice([0, 5, 3000, 40000, 200000]))
        ref = oracle.parse(data, dfas[d], types)
        d_in = torch.from_numpy(np.ascontiguousarray(data)).cuda() if len(data) else \
            torch.empty(0, dtype=torch.uint8, device="cuda")
        out = pp.alloc_outputs(types, ref.num_records, ref.num_fields)
        items.append((d_in, d, types, out))
        refs.append(ref)
    batch = pp.Batch(dfas, items)
    batch.launch(torch.cuda.current_stream())
    torch.cuda.synchronize()
    for i, ((d_in, d, types, out), ref) in enumerate(zip(items, refs)):
        compare(ref, out, out.result_dict(), types, tag=f"buffer {i} dialect {d}")


@pytest.mark.parametrize("seed", range(6))
def test_random_dfas_materialize_and_infer(seed):
    """String columns materialised (control symbols removed, with and without
    a terminator) and column types inferred, under random dialects whose
    control symbols and delimiters sit anywhere."""
    rnd = random.Random(5000 + seed)
    for k in range(4):
        dfa = random_dfa(rnd, f"m{seed}_{k}")
        ncols = rnd.randint(1, 6)
        types = [D.STRING] * ncols
        data = random_input(rnd, dfa, rnd.choice([600, 70000, 200000]))
        R, F = oracle.count(data, dfa)
        d_in = torch.from_numpy(np.ascontiguousarray(data).copy()).cuda()
        out = pp.parse(d_in, dfa, types, R, F, control_bitmap=True)
        for c in range(ncols):
            for term in (-1, 0x1F):
                offs, chars = pp.materialize(d_in, out, c, terminator=term)
                torch.cuda.synchronize()
                want_o, want_c = oracle.materialize(data, dfa, c, terminator=term)
                go = offs.cpu().numpy()
                np.testing.assert_array_equal(go[:R + 1], want_o, err_msg=f"offsets {c} {term}")
                np.testing.assert_array_equal(chars.cpu().numpy()[:want_o[-1]], want_c, err_msg=f"chars {c} {term}")
        got_t, got_n = pp.infer_types(d_in, out)
        want_t, want_n = oracle.infer_types(data, dfa, ncols)
        assert got_t == want_t, (dfa.name, got_t, want_t)
        np.testing.assert_array_equal(got_n, want_n)
