"""Projection and inference on the GPU against the oracle (Sec. 4.3):
type inference over string-span columns (and the inferred typed parse),
skipping rows (stream compaction of the raw input, then the parse),
skipping records (typed values cleared), and multi-byte UTF-8 text, whose
bytes above 0x7f fall in the DFAs' catch-all group (every DFA symbol is
ASCII, so a byte-level DFA reads UTF-8 exactly)."""
import random

import numpy as np
import pytest

import datagen
import oracle
import paper_1905_13415_amd as pp
from datagen import dialects as D
from parity import compare

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

MiB = 1 << 20


def u8(b):
    return np.frombuffer(bytes(b), dtype=np.uint8)


def dev(arr):
    return torch.from_numpy(np.ascontiguousarray(arr).copy()).cuda() if len(arr) else \
        torch.empty(0, dtype=torch.uint8, device="cuda")


def typed_text(seed, nrows=4000):
    rng = random.Random(seed)
    kinds = {
        "int": lambda: str(rng.randrange(-10 ** 9, 10 ** 9)),
        "big": lambda: rng.choice(["9223372036854775807", "9223372036854775808"]),
        "float": lambda: f"{rng.uniform(-1e4, 1e4):.{rng.randrange(0, 4)}f}",
        "exp": lambda: f"{rng.uniform(1, 9):.2f}e{rng.randrange(-5, 5)}",
        "date": lambda: f"{rng.randrange(1900, 2100):04d}-{rng.randrange(1, 13):02d}-{rng.randrange(1, 29):02d}",
        "ts": lambda: f"2020-{rng.randrange(1, 13):02d}-{rng.randrange(1, 29):02d}T"
                      f"{rng.randrange(0, 24):02d}:{rng.randrange(0, 60):02d}:{rng.randrange(0, 60):02d}",
        "word": lambda: rng.choice(["abc", "x1", '"q,q"', '"7"']),
        "empty": lambda: "",
    }
    plans = [["int"], ["int", "empty"], ["int", "big"], ["float"], ["int", "float"], ["exp", "int"], ["date"],
             ["ts"], ["date", "ts"], ["word"], ["int", "word"], ["empty"]]
    rows = [",".join(kinds[rng.choice(p)]() for p in plans) for _ in range(nrows)]
    return ("\n".join(rows) + "\n").encode(), len(plans)


@pytest.mark.parametrize("seed", range(3))
def test_infer_types_matches_oracle(seed):
    text, ncols = typed_text(seed)
    arr = u8(text)
    R, F = oracle.count(arr, D.csv4())
    d = dev(arr)
    raw = pp.parse(d, D.csv4(), [D.STRING] * ncols, R, F)
    types, nonempty = pp.infer_types(d, raw)
    want, wn = oracle.infer_types(arr, D.csv4(), ncols)
    assert types == want and list(nonempty) == list(wn)
    assert types[:9] == [D.INT64, D.INT64, D.FLOAT64, D.FLOAT64, D.FLOAT64, D.FLOAT64, D.DATE_DAYS,
                         D.TIMESTAMP_S, D.STRING]


def test_infer_types_long_fields():
    """Fields of 4,096 bytes or more are checked by a whole workgroup: long
    integers (leading zeros, the 19-digit limit), long floats (many digits,
    exponents with leading zeros), long text and each way of breaking a
    grammar, alone in a column or beside short fields; with enough of them
    that some exceed the workgroup queue and are checked by their thread."""
    rnd = random.Random(21)
    z = lambda k: "0" * k
    digits = lambda k: "".join(rnd.choice("0123456789") for _ in range(k))
    cols = [
        [z(5000) + "42", "7", z(9000) + "9223372036854775807", "-" + z(4100) + "9223372036854775808"],  # INT64
        [z(5000) + "42", z(4200) + "9223372036854775808"],                              # FLOAT64 (overflow)
        ["1." + digits(6000), "2.5", digits(5000) + "e-" + z(4000) + "17", "." + digits(4500)],  # FLOAT64
        [digits(4000) + "x", "5"],                                                     # STRING
        ["1e" + z(4500), "1" + z(4200) + "e+5"],                                        # FLOAT64
        [z(4300) + "1.2.3", "1"],                                                      # STRING
        ["+" + z(4400) + "-1", "2"],                                                   # STRING
        ["-" + digits(4096), "3"],                                                     # FLOAT64 or INT64
        [z(4097) + "e", "1.5"],                                                        # STRING
    ]
    nrows = 3000
    rows = []
    for r in range(nrows):
        rows.append(",".join(c[r % len(c)] if r % 3 == 0 else c[1 % len(c)] for c in cols))
    text = ("\n".join(rows) + "\n").encode()
    arr = u8(text)
    R, F = oracle.count(arr, D.csv4())
    d = dev(arr)
    raw = pp.parse(d, D.csv4(), [D.STRING] * len(cols), R, F)
    types, nonempty = pp.infer_types(d, raw)
    want, wn = oracle.infer_types(arr, D.csv4(), len(cols))
    assert types == want and list(nonempty) == list(wn)
    assert types[:7] == [D.INT64, D.FLOAT64, D.FLOAT64, D.STRING, D.FLOAT64, D.STRING, D.STRING]


def test_parse_inferred_numeric_slice():
    """The numeric CSV without a schema: column count, string parse, types,
    typed parse; the inferred schema is the generator's."""
    g = datagen.c2(nbytes=32 * MiB)
    d = dev(g.data)
    out, types = pp.parse_inferred(d, D.csv4())
    torch.cuda.synchronize()
    assert types == list(D.SCHEMA_C2.types)
    ref = oracle.parse(g.data, D.csv4(), types)
    compare(ref, out, out.result_dict(), types, tag="inferred")


@pytest.mark.parametrize("seed", range(3))
def test_skip_rows_then_parse(seed):
    """Rows are raw lines: quoted records with embedded line feeds span
    several, so compaction can cut into records; the parse of the compacted
    input equals the oracle's parse of the oracle's compaction."""
    rng = random.Random(seed)
    data = datagen.c1().data
    nrows = int((data == 10).sum())
    ranges, k = [], rng.randrange(0, 3)
    while k < nrows and len(ranges) < 60:
        a = k + rng.randrange(0, 400)
        b = a + rng.randrange(1, 50)
        ranges.append((a, b))
        k = b + rng.randrange(1, 100)
    end = max(b for _, b in ranges) if ranges else 0
    ranges.append((max(end, nrows) + 5, max(end, nrows) + 9))  # beyond the input: nothing to drop
    d = dev(data)
    got = pp.skip_rows(d, ranges).cpu().numpy()
    want = oracle.skip_rows(data, ranges)
    np.testing.assert_array_equal(got, want)
    types = list(D.SCHEMA_C1.types)
    ref = oracle.parse(want, D.csv4(), types)
    out = pp.parse(dev(want), D.csv4(), types, ref.num_records, ref.num_fields)
    torch.cuda.synchronize()
    compare(ref, out, out.result_dict(), types, tag="after skip")


def test_skip_rows_large_and_edges():
    g = datagen.log(9, 64 * MiB)
    d = dev(g.data)
    for ranges in ([(0, 1)], [(0, 10 ** 9)], [], [(3, 4), (5, 100000), (200000, 200001)]):
        got = pp.skip_rows(d, ranges).cpu().numpy()
        np.testing.assert_array_equal(got, oracle.skip_rows(g.data, ranges), err_msg=str(ranges[:2]))
    assert pp.skip_rows(dev(u8(b"")), [(0, 1)]).numel() == 0
    with pytest.raises(pp.PpError):
        pp.skip_rows(d, [(5, 3)])  # empty range
    with pytest.raises(pp.PpError):
        pp.skip_rows(d, [(5, 9), (7, 12)])  # overlapping ranges


def test_skip_records():
    g = datagen.c1()
    types = list(D.SCHEMA_C1.types)
    R, F = g.nrecords, g.nrecords * g.ncols
    ranges = [(0, 1), (17, 400), (9000, 10 ** 6)]
    out = pp.parse(dev(g.data), D.csv4(), types, R, F)
    pp.skip_records(out, ranges)
    torch.cuda.synchronize()
    ref = oracle.skip_records(oracle.parse(g.data, D.csv4(), types), types, [(a, min(b, R)) for a, b in ranges])
    compare(ref, out, out.result_dict(), types, tag="skip records")


def test_utf8_text():
    """Multi-byte UTF-8 characters (2-4 bytes, all above 0x7f) inside quoted
    and unquoted fields: the structure, the typed columns and the
    materialised strings equal the oracle's."""
    rng = random.Random(3)
    words = ["é", "ß", "日本", "€5", "😀x", "naïve", "Ωmega", "a,b", "q\"\"q"]
    rows = []
    for i in range(20000):
        w = rng.choice(words)
        s = f'"{w}"' if ("," in w or '"' in w or rng.random() < 0.3) else w
        rows.append(f"{i},{s},{rng.uniform(0, 99):.2f},{rng.choice(words).replace(',', ';').replace(chr(34), '')}")
    arr = u8(("\n".join(rows) + "\n").encode("utf-8"))
    types = [D.INT64, D.STRING, D.FLOAT64, D.STRING]
    ref = oracle.parse(arr, D.csv4(), types)
    d = dev(arr)
    out = pp.parse(d, D.csv4(), types, ref.num_records, ref.num_fields, control_bitmap=True)
    offs, chars = pp.materialize(d, out, 1)
    torch.cuda.synchronize()
    compare(ref, out, out.result_dict(), types, tag="utf8")
    o_offs, o_chars = oracle.materialize(arr, D.csv4(), 1)
    np.testing.assert_array_equal(offs.cpu().numpy(), o_offs)
    np.testing.assert_array_equal(chars.cpu().numpy()[:o_offs[-1]], o_chars)
    vals = bytes(o_chars).decode("utf-8")  # whole characters, nothing cut
    assert "日本" in vals and "😀x" in vals
