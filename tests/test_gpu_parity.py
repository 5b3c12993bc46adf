"""GPU parity: the HIP path through the C ABI against the oracle, bit-exact.

Sizes span several tiles (32 KiB by default; 4-16 KiB for the other launch
shapes) with ragged tails; the edge cases cover empty input, inputs ending
at and off tile boundaries, fields and quotes spanning tiles, tiles of
nothing but delimiters or tiny records (the per-thread fallback path),
invalid input, unterminated quotes, capacity, an unaligned input pointer,
3- to 8-state DFAs, hard float conversions, the fewest and most fields per
record (a 70,000-field record across tiles), and a tile's first field of each
type beginning 0-71, 100 and 200 bytes before the tile.
"""
import random

import numpy as np
import pytest

import datagen
import oracle
import paper_1905_13415_amd as pp
from datagen import dialects as D
from parity import assert_same, gpu_parse

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

TILE = 32768  # default launch shape: 512 threads x 64 bytes
SHAPES = [None, (64, 256), (32, 256), (32, 512), (16, 256)]  # (bytes/thread, threads)
SHAPE_IDS = ["512x64", "256x64", "256x32", "512x32", "256x16"]


def opts_of(shape):
    return pp.options(*shape) if shape else None


def u8(b):
    return np.frombuffer(bytes(b), dtype=np.uint8)


# ---- worked examples ---------------------------------------------------------------

def test_quoted_example():
    assert_same(u8(b'a,"b,c"\n"d""e",f\n'), D.paper6(), [D.STRING, D.STRING])


def test_ragged_example():
    for dfa in (D.paper6(), D.csv4()):
        assert_same(u8(b"1,Apples\n2\n"), dfa, [D.INT64, D.STRING])


# ---- edge cases ----------------------------------------------------------------------

@pytest.mark.parametrize("text", [b"", b"a", b"\n", b",", b'"', b"1,2", b"1,", b"\n\n\n",
                                  b'"abc', b'a"b\n', b'"a""', b",,,\n,,\n"])
def test_tiny_inputs(text):
    for dfa in (D.csv4(), D.paper6()):
        assert_same(u8(text), dfa, [D.STRING, D.INT64, D.STRING])


@pytest.mark.parametrize("shape", SHAPES, ids=SHAPE_IDS)
def test_tile_boundaries(shape):
    tile = (shape[0] * shape[1]) if shape else TILE
    g = datagen.c1()
    for n in (tile - 1, tile, tile + 1, 2 * tile, 3 * tile + 17):
        data = g.data[:n].copy()
        assert_same(data, D.csv4(), D.SCHEMA_C1.types, opts=opts_of(shape))
        # the same length ending in a record delimiter exactly at the boundary
        data[-1] = ord("\n")
        assert_same(data, D.csv4(), D.SCHEMA_C1.types, opts=opts_of(shape))


@pytest.mark.parametrize("shape", SHAPES, ids=SHAPE_IDS)
def test_all_delimiters(shape):
    """Every byte a delimiter: more fields (and records) per tile than the
    LDS staging holds, so every tile takes the per-thread path."""
    for ch in (b",", b"\n"):
        assert_same(u8(ch * (3 * TILE + 5)), D.csv4(), [D.INT64, D.STRING, D.FLOAT64], opts=opts_of(shape))


@pytest.mark.parametrize("shape", SHAPES, ids=SHAPE_IDS)
def test_tiny_records_fallback_and_mixed_tiles(shape):
    """Records of 2-12 bytes exceed the per-tile record staging; longer ones
    in between keep some tiles on the staged path."""
    rnd = random.Random(11)
    c1 = bytes(datagen.c1().data[:20000])
    parts = []
    while sum(map(len, parts)) < 4 * TILE:
        if rnd.random() < 0.5:
            parts.append(b"1,2\n" * rnd.randint(1, 4000))
        else:
            parts.append(c1[:rnd.randint(1, 20000)])
    data = b"".join(parts)
    assert_same(u8(data), D.csv4(), D.SCHEMA_C1.types, opts=opts_of(shape))
    assert_same(u8(data), D.csv4(), [D.INT64, D.INT64], opts=opts_of(shape))


@pytest.mark.parametrize("shape", [None, (16, 256)], ids=["512x64", "256x16"])
def test_wide_records_column_ids_past_254(shape):
    """Records of 250-600 fields of 7 bytes: few enough fields per tile for
    the LDS staging, but column ids past 254 (the staged 8-bit ids' limit)
    send a tile to the per-thread path; records of exactly 255 fields (ids
    0-254) stay staged. Mixed with short records so both paths meet."""
    t = [D.INT64, D.STRING, D.FLOAT64, D.INT64]
    for nf in (250, 254, 255, 256, 257, 300, 600):
        rec = ",".join(f"{i:06d}" for i in range(nf)) + "\n"
        data = (rec * (3 * TILE // len(rec) + 2) + "1,a,2.5,3\n" * 4000 + rec * 7).encode()
        assert_same(u8(data), D.csv4(), t, opts=opts_of(shape))


def test_long_quoted_field_spanning_tiles():
    body = bytes(random.Random(1).choice(b'ab,\n ') for _ in range(5 * TILE))
    data = b'1,"' + body + b'",2\n3,"x",4\n'
    assert_same(u8(data), D.csv4(), [D.INT64, D.STRING, D.INT64])
    assert_same(u8(data), D.paper6(), [D.INT64, D.STRING, D.INT64])


def test_one_field_of_200mb():
    """The skewed input of the paper's evaluation: one record whose quoted
    field is 200 MB (doubled quotes, delimiters and line feeds inside),
    between short records, parsed into the same spans as the oracle's."""
    rng = np.random.default_rng(7)
    body = rng.integers(97, 123, size=200_000_000, dtype=np.uint8)
    body[rng.integers(0, len(body), 20000)] = ord(",")
    body[rng.integers(0, len(body), 20000)] = ord("\n")
    txt = body.tobytes().replace(b"qz", b'q""z')
    data = u8(b'1,"' + txt + b'",2.5\n2,"a""b",3\n3,short,4.25\n')
    assert txt.count(b'""') > 100000
    assert_same(data, D.csv4(), [D.INT64, D.STRING, D.FLOAT64])


def _long_numeric_fields(rnd):
    """Integer and float fields of 2,048 symbols or more (converted by the
    workgroup pass) in every form the grammar decides on: leading zeros,
    signs, overflow at the 19-digit boundary, long fractions, more than 800
    significant digits with and without a nonzero digit past the 800th,
    exponents with leading zeros or beyond 10^8, and each way of breaking the
    grammar."""
    z = lambda k: "0" * k
    digits = lambda k: "".join(rnd.choice("0123456789") for _ in range(k))
    ints = [z(5000) + "42", "-" + z(3000) + "7", "+" + z(2500), z(2047) + "1", "1" + z(2100),
            z(4000) + "9223372036854775807", z(4000) + "9223372036854775808",
            "-" + z(4000) + "9223372036854775808", "-" + z(4000) + "9223372036854775809",
            z(3000) + "12x4", z(2100) + "-5", z(3000) + "1.0", z(2600) + " "]
    floats = [z(5000) + "42.5", "-" + z(3000) + ".000" + z(2000) + "15", "0." + z(2400) + "1e2405",
              "1." + digits(3000), digits(2100) + "." + digits(900), digits(2500),
              "0.5" + z(2000) + "1", "0.5" + z(3000), "2." + z(850) + z(1500) + "1",
              "1.0000000000000002220446049250313080847263336181640625" + z(2500),
              "1.0000000000000002220446049250313080847263336181640625" + z(2500) + "1",
              "1e" + z(3000) + "22", "1e+" + z(2400) + "308", "1e-" + z(2400) + "330", "7e" + "9" * 2100,
              "-" + z(2300) + "e5", z(2200) + ".", "." + z(2200), "." + z(2200) + "3",
              z(2200) + "1..5", z(2200) + "1e5e5", z(2200) + "1e", z(2200) + "1e+", z(2200) + "1x",
              "+" + z(2200) + "-1", z(2300) + "E-" + z(5) + "3", digits(1000) + "." + digits(1500) + "e-" + z(2000) + "1200"]
    return ints, floats


@pytest.mark.parametrize("shape", [None, (16, 256)], ids=["512x64", "256x16"])
def test_long_numeric_fields_workgroup_pass(shape):
    """Numeric fields of 2,048 symbols or more: those that begin tiles back
    (a tile's first field) are converted by the whole workgroup after the
    tile's own conversion, those within a tile by their lane from LDS, and
    those in tiles with more fields than the staging holds by the per-thread
    path; every value, validity and the error count against the oracle."""
    rnd = random.Random(12)
    ints, floats = _long_numeric_fields(rnd)
    rows = []
    for k in range(max(len(ints), len(floats))):
        rows.append(f"{ints[k % len(ints)]},{floats[k % len(floats)]},{k}\n")
        rows.append(f"{k},{k}.5,{k}\n" * rnd.randint(0, 40))
    data = "".join(rows).encode()
    types = [D.INT64, D.FLOAT64, D.INT64]
    assert_same(u8(data), D.csv4(), types, opts=opts_of(shape))
    assert_same(u8(data), D.paper6(), types, opts=opts_of(shape))  # a 6-state DFA (8-state vectors)
    # a tile with more fields than it stages holds a long integer and float
    crowd = ("," * 9000 + "\n") + "".join(f"{i},{f},1\n" for i, f in zip(ints, floats))
    assert_same(u8(crowd.encode() * 3), D.csv4(), types, opts=opts_of(shape))
    # quoted long numbers (control symbols stripped before the conversion)
    quoted = "".join(f'"{i}","{f}",2\n' for i, f in zip(ints, floats)).encode()
    assert_same(u8(quoted), D.csv4(), types, opts=opts_of(shape))
    # a long number closed by the end of input, and records past the capacity
    tail = ("1,2.5,3\n" * 10 + "4,5.5," + "0" * 70000 + "6").encode()
    assert_same(u8(tail), D.csv4(), types, opts=opts_of(shape))
    assert_same(u8(data), D.csv4(), types, opts=opts_of(shape), cap_records=30, cap_fields=100)


def test_long_numeric_fields_utf16():
    """The same fields as UTF-16 text (the pass reads and narrows code units)."""
    rnd = random.Random(13)
    ints, floats = _long_numeric_fields(rnd)
    text = "".join(f"{i},{f},{k}\n" for k, (i, f) in enumerate(zip(ints * 2, floats)))
    b16 = text.encode("utf-16-le")
    ref = oracle.parse(b16, D.csv4(), [D.INT64, D.FLOAT64, D.INT64], utf16=True)
    d_in = torch.from_numpy(np.frombuffer(b16, dtype=np.uint8).copy()).cuda()
    out = pp.parse_utf16(d_in, D.csv4(), [D.INT64, D.FLOAT64, D.INT64], ref.num_records, ref.num_fields)
    torch.cuda.synchronize()
    from parity import compare
    compare(ref, out, out.result_dict(), [D.INT64, D.FLOAT64, D.INT64], tag="utf16 long numbers")


def test_one_numeric_field_of_20mb():
    """A float of 20 million digits and an integer of 20 million leading
    zeros, each one field spanning hundreds of tiles, converted by the
    workgroup of the tile that closes it, equal to the oracle's."""
    rng = np.random.default_rng(5)
    frac = rng.integers(48, 58, size=20_000_000, dtype=np.uint8).tobytes()
    data = b"1,2.5,3\n" + b"7," + b"3." + frac + b",9\n" + b"0" * 20_000_000 + b"42,1.25,8\n" + b"4,5,6\n"
    assert_same(u8(data), D.csv4(), [D.INT64, D.FLOAT64, D.INT64])
    assert_same(u8(data), D.csv4(), [D.FLOAT64, D.FLOAT64, D.INT64])


def test_one_numeric_field_of_200mb():
    """The skewed input of the paper's evaluation as a number: one float
    field of 200 million digits between short records, equal to the
    oracle's, and converted by the closing tile's workgroup within half a
    second (one lane reading it symbol by symbol from HBM takes seconds)."""
    rng = np.random.default_rng(6)
    frac = rng.integers(48, 58, size=200_000_000, dtype=np.uint8).tobytes()
    data = u8(b"1,2.5\n7,3." + frac + b"\n4,5.25\n")
    types = [D.INT64, D.FLOAT64]
    assert_same(data, D.csv4(), types)
    d_in = torch.from_numpy(data).cuda()
    out = pp.alloc_outputs(types, 3, 6)
    ws = torch.empty(pp.workspace_size(len(data)), dtype=torch.uint8, device="cuda")
    call = pp.Call(d_in, len(data), D.csv4(), types, out, ws)
    call.launch(torch.cuda.current_stream())
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    call.launch(torch.cuda.current_stream())
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    print(f"200 MB float field: {ms:.2f} ms")
    assert out.result_dict()["num_conversion_errors"] == 0
    assert ms < 500.0


def test_long_numeric_field_spanning_tiles():
    data = b"7," + b"0" * (2 * TILE + 100) + b"42,x\n" + b"1.5," + b"9" * 30000 + b",y\n"
    assert_same(u8(data), D.csv4(), [D.FLOAT64, D.INT64, D.STRING])


def test_invalid_and_unterminated():
    g = datagen.c1()
    data = bytearray(g.data[:5 * TILE])
    data[3 * TILE + 100] = ord('"')  # a quote in an unquoted field under paper6 -> INV
    ref, _, res = assert_same(u8(data), D.paper6(), D.SCHEMA_C1.types)
    assert res["status"] in (pp.RESULT_INVALID_INPUT, pp.RESULT_OK)
    assert_same(u8(b'1,2\n3,"unterminated\n' + b"x" * (2 * TILE)), D.csv4(), [D.INT64, D.STRING])
    assert_same(u8(b'1,2\n3,"unterminated\n' + b"x" * (2 * TILE)), D.paper6(), [D.INT64, D.STRING])


def test_capacity_exceeded():
    g = datagen.c1()
    data = g.data[:6 * TILE]
    assert_same(data, D.csv4(), D.SCHEMA_C1.types, cap_records=100, cap_fields=333)


def test_unaligned_input():
    g = datagen.c1()
    for off in (1, 3, 8):
        assert_same(g.data[:4 * TILE + 77], D.csv4(), D.SCHEMA_C1.types, offset=off)


@pytest.mark.parametrize("shape", SHAPES, ids=SHAPE_IDS)
def test_launch_shapes_c1(shape):
    g = datagen.c1()
    assert_same(g.data, D.csv4(), D.SCHEMA_C1.types, opts=opts_of(shape))
    assert_same(g.data, D.paper6(), D.SCHEMA_C1.types, opts=opts_of(shape))


def test_ragged_and_extra_fields():
    rnd = random.Random(5)
    lines = []
    for _ in range(5000):
        k = rnd.randint(0, 12)
        lines.append(",".join(str(rnd.randint(-99, 99)) for _ in range(k)))
    data = ("\n".join(lines) + "\n").encode()
    assert_same(u8(data), D.csv4(), [D.INT64] * 6)
    assert_same(u8(data), D.csv4(), [])


@pytest.mark.parametrize("shape", SHAPES, ids=SHAPE_IDS)
def test_column_counts(shape):
    """Fewest and most fields per record: a 70,000-field record spanning
    several tiles (its count needs the exact carried column), blank lines
    (one field each) at tile starts, and uniform stretches."""
    tile = (shape[0] * shape[1]) if shape else TILE
    rnd = random.Random(11)
    head = "1,2,3\n" * 3000 + "x," * 69999 + "y\n" + "7\n" + "4,5,6\n" * 2000
    head += ",".join("9" for _ in range(rnd.randint(1, 9))) + "\n"
    pad = -(len(head) + 1) % tile  # the blank line below begins a tile
    data = u8((head + "a" * pad + "\n" + "\n" + "1,2,3\n" * 1000).encode())
    assert (len(head) + pad + 1) % tile == 0
    ref, out, res = assert_same(data, D.csv4(), [D.INT64] * 3, opts=opts_of(shape))
    assert (res["min_record_fields"], res["max_record_fields"]) == (1, 70000)
    uniform = u8(b"1,2,3\n" * 20000)
    ref, out, res = assert_same(uniform, D.csv4(), [D.INT64] * 3, opts=opts_of(shape))
    assert (res["min_record_fields"], res["max_record_fields"], res["num_ragged_records"]) == (3, 3, 0)


# ---- random symbol soup over each dialect ------------------------------------------------

@pytest.mark.parametrize("name", ["csv4", "paper6", "log6", "s3", "s5", "s7", "s8"])
def test_random_symbol_soup(name):
    dfa = D.ALL_DFAS[name]()
    alphabet = b"".join(dfa.group_symbols) + b"a1.-"
    rnd = random.Random(sum(name.encode()))
    types = [D.STRING, D.INT64, D.FLOAT64, D.STRING, D.INT64]
    for n in (100, 5000, 3 * TILE + 11):
        data = bytes(rnd.choice(alphabet) for _ in range(n))
        for shape in (None, (16, 256)):
            assert_same(u8(data), dfa, types, opts=opts_of(shape))


# ---- workloads ------------------------------------------------------------------------------

def test_c1_full():
    g = datagen.c1()
    assert_same(g.data, D.csv4(), D.SCHEMA_C1.types)
    assert_same(g.data, D.paper6(), D.SCHEMA_C1.types)


@pytest.mark.parametrize("shape", SHAPES, ids=SHAPE_IDS)
def test_c2_c3_slices(shape):
    assert_same(datagen.c2(nbytes=24 << 20).data, D.csv4(), D.SCHEMA_C2.types, opts=opts_of(shape))
    assert_same(datagen.c3(nbytes=40 << 20).data, D.csv4(), D.SCHEMA_C3.types, opts=opts_of(shape))


@pytest.mark.parametrize("name,delim,qstyle", [("csv4", b"\t", 1), ("s5", b"|", 1), ("s3", b",", 3),
                                               ("s7", b",", 2), ("paper6", b",", 1)])
def test_mixed_dialects(name, delim, qstyle):
    dfa = D.ALL_DFAS[name](delim) if name != "paper6" else D.paper6()
    g = datagen.mixed(17, 3 << 20, delim=delim, qstyle=qstyle)
    assert_same(g.data, dfa, D.SCHEMA_C1.types)


def test_log_dialects():
    g = datagen.log(23, 3 << 20)
    assert_same(g.data, D.log6(), D.SCHEMA_LOG12.types)
    assert_same(g.data, D.s8(), D.SCHEMA_LOG12.types)


# ---- conversions ------------------------------------------------------------------------------

HARD_FLOATS = ["0", "-0.0", "1e10", "1E-5", "+3.25e+2", "0.1", "9007199254740993", "1e308", "1.8e308",
               "-1e400", "4.9406564584124654e-324", "2.4703282292062327e-324",
               "2.4703282292062328e-324", "1e-320", "2.2250738585072011e-308",
               "1.7976931348623157e308", "1.00000000000000011102230246251565404236316680908203125",
               "1.00000000000000011102230246251565404236316680908203124",
               "1.00000000000000011102230246251565404236316680908203126",
               "12345678901234567890123", "0.000000000000000000000000000000123456789",
               "123456789012345678901234567890e-10", "7.2057594037927933e16", "3.14159265358979323846264338",
               ".5", "5.", "", ".", "e5", "1e", "1e+", "--1", "inf", "nan", "1,0", "0x1p3",
               "1" * 400 + "e-400", "0." + "0" * 330 + "1", "179769313486231580793728971405301e276",
               "2.225073858507201136057409796709131975934819546351645648e-308"]


def test_hard_floats():
    rnd = random.Random(3)
    vals = list(HARD_FLOATS)
    for _ in range(4000):
        digits = "".join(rnd.choice("0123456789") for _ in range(rnd.randint(1, 25)))
        point = rnd.randint(0, len(digits))
        vals.append(digits[:point] + "." + digits[point:] + f"e{rnd.randint(-330, 310)}")
    data = "".join(f'"{v}",{i}\n' for i, v in enumerate(vals)).encode()
    assert_same(u8(data), D.csv4(), [D.FLOAT64, D.INT64])


def test_short_float_fields_every_form():
    """Float fields of at most 8 bytes take a word-parallel parse (a wavefront
    whose fields are all that short): every field of up to 4 symbols over
    digits, point, signs, an exponent letter and a space, and random fields of
    5-8 such symbols, with no longer field in the column, against the oracle
    (values, validity and the conversion-error count)."""
    import itertools
    alpha = "0123456789.-+e "
    vals = ["".join(t) for n in range(1, 4) for t in itertools.product(alpha, repeat=n)]
    rnd = random.Random(8)
    vals += ["".join(rnd.choice(alpha) for _ in range(4)) for _ in range(20000)]
    vals += ["".join(rnd.choice("0123456789.-+") for _ in range(rnd.randint(5, 8))) for _ in range(60000)]
    vals += ["-" + "".join(rnd.choice("0123456789") for _ in range(6)) + "." for _ in range(2000)]
    assert max(map(len, vals)) <= 8
    data = "".join(f"{v},{i}\n" for i, v in enumerate(vals)).encode()
    assert_same(u8(data), D.csv4(), [D.FLOAT64, D.INT64])


INTS = ["0", "-0", "+7", "9223372036854775807", "-9223372036854775808", "9223372036854775808",
        "-9223372036854775809", "00000000000000000000042", "", "+", "-", "1 ", " 1", "1.0", "12a",
        "99999999999999999999"]
TIMES = ["1970-01-01 00:00:00", "1969-12-31 23:59:59", "2000-02-29 12:00:00", "1900-02-29 00:00:00",
         "2001-02-29 00:00:00", "2018-13-01 00:00:00", "0001-01-01T00:00:00", "9999-12-31 23:59:59",
         "2018-01-01 24:00:00", "2018-01-01 00:00:60", "2018-01-01 00:00", "2018/01/01 00:00:00"]
DATES = ["1970-01-01", "1600-02-29", "1700-02-29", "2024-02-29", "2023-02-29", "2019-04-31", "0000-03-01",
         "2019-4-30", "20190430"]


def test_int_time_date_edge_cases():
    k = max(len(INTS), len(TIMES), len(DATES))
    rows = []
    for i in range(k):
        rows.append(",".join([INTS[i % len(INTS)], TIMES[i % len(TIMES)], DATES[i % len(DATES)]]))
    data = ("\n".join(rows) + "\n").encode()
    assert_same(u8(data), D.csv4(), [D.INT64, D.TIMESTAMP_S, D.DATE_DAYS])


def test_all_days_date_column():
    import datetime
    d0 = datetime.date(1600, 1, 1)
    data = "\n".join((d0 + datetime.timedelta(days=i)).isoformat() for i in range(300000)).encode()
    assert_same(u8(data), D.csv4(), [D.DATE_DAYS])


def test_repeated_runs_identical():
    g = datagen.c2(nbytes=8 << 20)
    out1, r1 = gpu_parse(g.data, D.csv4(), D.SCHEMA_C2.types)
    out2, r2 = gpu_parse(g.data, D.csv4(), D.SCHEMA_C2.types)
    assert r1 == r2
    assert torch.equal(out1.field_offsets, out2.field_offsets)
    for a, b in zip(out1.values, out2.values):
        assert torch.equal(a.view(torch.int64), b.view(torch.int64))


def test_int_every_length_and_sign():
    """Integers of 1 to 20 digits with and without signs (the register path
    accumulates the first nine bytes in 32 bits, the rest in 64)."""
    rnd = random.Random(5)
    rows = []
    for n in range(1, 21):
        for _ in range(40):
            digits = str(rnd.randint(1, 9)) + "".join(rnd.choice("0123456789") for _ in range(n - 1))
            sign = rnd.choice(["", "-", "+"])
            rows.append(sign + digits)
            rows.append(sign + "0" * rnd.randint(0, 3) + digits[: max(1, n // 2)])
    data = ("\n".join(f"{v},{i}" for i, v in enumerate(rows)) + "\n").encode()
    assert_same(u8(data), D.csv4(), [D.INT64, D.INT64])


def test_timestamps_all_years():
    """Timestamps and dates drawn over years 0000-9999 (four-digit years)."""
    rnd = random.Random(6)
    rows = []
    for _ in range(20000):
        y, mo, d = rnd.randint(0, 9999), rnd.randint(1, 12), rnd.randint(1, 31)
        h, mi, s = rnd.randint(0, 23), rnd.randint(0, 59), rnd.randint(0, 59)
        sep = rnd.choice([" ", "T"])
        rows.append(f"{y:04d}-{mo:02d}-{d:02d}{sep}{h:02d}:{mi:02d}:{s:02d},{y:04d}-{mo:02d}-{d:02d}")
    data = ("\n".join(rows) + "\n").encode()
    assert_same(u8(data), D.csv4(), [D.TIMESTAMP_S, D.DATE_DAYS])


# ---- the tile's first field, by how far before the tile it begins -------------------

HEAD_SCHEMA = [D.STRING, D.INT64, D.FLOAT64, D.TIMESTAMP_S, D.STRING]
HEAD_FIELDS = ["-1234567", "-12345.6789", "2019-03-04 05:06:07", '"q,u""o"']


@pytest.mark.parametrize("k", range(1, 5), ids=["int", "float", "timestamp", "quoted"])
def test_first_field_of_tile_at_every_offset(k):
    # Field k of the second record begins d bytes before the second tile: from
    # the tile boundary itself, through the 64 bytes the kernel keeps before a
    # tile, to beyond them (the general path). The bytes before the tile hold
    # no quote for k < 4 (the start-state guess from them is taken) and a
    # quote for k = 4 (it is not).
    tail = "".join(f"{i},{i * 7},{i}.25,2020-01-0{1 + i % 9} 00:00:0{i % 10},s{i}\n" for i in range(40))
    for d in list(range(0, 72)) + [100, 200]:
        rec = ["x", "7", "1.5", "2001-02-03 04:05:06", "y"]
        rec[k] = HEAD_FIELDS[k - 1]
        between = sum(len(f) + 1 for f in rec[1:k])  # fields 1..k-1 and their commas
        first = "p" * 10 + ",1,2.5,1999-12-31 23:59:59,z\n"
        pad = TILE - d - len(first) - 1 - between
        rec[0] = "w" * pad
        data = (first + ",".join(rec) + "\n" + tail * 3).encode()
        assert data.find(HEAD_FIELDS[k - 1].encode(), len(first)) == TILE - d
        assert_same(u8(data), D.csv4(), HEAD_SCHEMA)


# ---- tile order --------------------------------------------------------------------------------

@pytest.mark.parametrize("shape", SHAPES, ids=SHAPE_IDS)
def test_permuted_tile_order(shape):
    """Tiles parsed out of input order (each complete block of 64 permuted,
    the diagnostic tile_order option): the single-pass scans' lookbacks then
    meet predecessors that have not started, published only their aggregate,
    or finished. Outputs equal the oracle's under several permutations, for
    quoted text (state vectors that differ per start state), the numeric CSV,
    and an 8-state dialect; the inputs hold several complete blocks and an
    incomplete last one."""
    tile = (shape[0] * shape[1]) if shape else TILE
    b, t = shape if shape else (0, 0)
    c3 = datagen.c3(nbytes=200 * tile + 12345).data
    c2 = datagen.c2(nbytes=150 * tile + 77).data
    lg = datagen.log(29, 140 * tile + 5).data
    for order in (1, 5, 22):
        o = pp.options(b, t, order)
        assert_same(c3, D.csv4(), D.SCHEMA_C3.types, opts=o)
        assert_same(c2, D.csv4(), D.SCHEMA_C2.types, opts=o)
        assert_same(lg, D.log6(), D.SCHEMA_LOG12.types, opts=o)
