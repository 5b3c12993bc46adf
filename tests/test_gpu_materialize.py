"""Materialised string columns (pp_materialize_strings, Sec. 3.3) against
the oracle, byte for byte: offsets and chars of every string column.

Covers the hand-worked quoted example, the quoted 10,000-record CSV under
every launch shape (the control-symbol bitmap is written per chunk), the log
dialect's backslash escapes and brackets, ragged and rejected records (empty
values), a 64 MiB text slice, a single quoted field of 64 MiB with doubled
quotes (spread over thousands of wavefronts), and a chars capacity below the
total.
"""
import numpy as np
import pytest

import datagen
import oracle
import paper_1905_13415_amd as pp
from datagen import dialects as D

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

SHAPES = [None, (64, 256), (32, 256), (32, 512), (16, 256)]
SHAPE_IDS = ["512x64", "256x64", "256x32", "512x32", "256x16"]
MiB = 1 << 20


def u8(b):
    return np.frombuffer(bytes(b), dtype=np.uint8)


def gpu_materialize(data, dfa, types, columns, opts=None, reject_ragged=False, cap_chars=None, terminator=-1):
    R, F = oracle.count(data, dfa)
    d_in = torch.from_numpy(np.ascontiguousarray(data).copy()).cuda() if len(data) else \
        torch.empty(0, dtype=torch.uint8, device="cuda")
    out = pp.parse(d_in, dfa, types, R, F, opts=opts, reject_ragged=reject_ragged, control_bitmap=True)
    got = {c: pp.materialize(d_in, out, c, cap_chars=cap_chars, terminator=terminator) for c in columns}
    torch.cuda.synchronize()
    return {c: (o.cpu().numpy(), ch.cpu().numpy()) for c, (o, ch) in got.items()}, out


def check(data, dfa, types, opts=None, tag="", terminator=-1):
    cols = [c for c, t in enumerate(types) if t == D.STRING]
    got, _ = gpu_materialize(data, dfa, types, cols, opts, terminator=terminator)
    for c in cols:
        offs, chars = oracle.materialize(data, dfa, c, terminator=terminator)
        go, gc = got[c]
        np.testing.assert_array_equal(go, offs, err_msg=f"{tag} offsets {c}")
        np.testing.assert_array_equal(gc[:offs[-1]], chars, err_msg=f"{tag} chars {c}")


def test_quoted_example():
    data = u8(b'a,"b,c"\n"d""e",f\n')
    for dfa in (D.paper6(), D.csv4()):
        got, _ = gpu_materialize(data, dfa, [D.STRING, D.STRING], [0, 1])
        vals = {c: [bytes(got[c][1][got[c][0][r]:got[c][0][r + 1]]) for r in range(2)] for c in (0, 1)}
        assert vals == {0: [b"a", b'd"e'], 1: [b"b,c", b"f"]}, dfa.name


@pytest.mark.parametrize("shape", SHAPES, ids=SHAPE_IDS)
def test_quoted_csv_every_shape(shape):
    g = datagen.c1()
    check(g.data, D.csv4(), list(D.SCHEMA_C1.types), pp.options(*shape) if shape else None, "c1")


@pytest.mark.parametrize("term", [0x1E, 0x1F, 0])
def test_inline_terminated(term):
    """Every value followed by a terminator byte (Sec. 4.1), empty values and
    records without the column included."""
    g = datagen.c1()
    check(g.data, D.csv4(), list(D.SCHEMA_C1.types), tag=f"terminated {term}", terminator=term)
    check(u8(b'a,"x""y"\nb\n"z",\n'), D.csv4(), [D.STRING, D.STRING], tag="short", terminator=term)


def test_log_escapes_and_brackets():
    g = datagen.log(11, 3 * MiB)
    check(g.data, D.log6(), list(D.SCHEMA_LOG12.types), tag="log")


def test_ragged_and_rejected_records():
    text = b'a,"x""y",1\nb\nc,"p,q"\n,,,\n"z",\n' * 500
    data = u8(text)
    types = [D.STRING, D.STRING, D.INT64]
    check(data, D.csv4(), types, tag="ragged")
    got, out = gpu_materialize(data, D.csv4(), types, [0, 1], reject_ragged=True)
    R = out.result_dict()["num_records"]
    ro = out.record_offsets[:R + 1].cpu().numpy()
    keep = np.diff(ro) == 3
    for c in (0, 1):
        offs, _ = oracle.materialize(data, D.csv4(), c)
        lens = np.diff(offs)
        glens = np.diff(got[c][0])
        np.testing.assert_array_equal(glens[keep], lens[keep])
        assert (glens[~keep] == 0).all()


def test_text_slice_64mib():
    g = datagen.c3(nbytes=64 * MiB)
    check(g.data, D.csv4(), list(D.SCHEMA_C3.types), tag="c3 slice")


def test_one_field_of_64mib():
    """A single quoted field of 64 MiB with doubled quotes, embedded commas
    and line feeds, between short records."""
    rng = np.random.default_rng(5)
    body = rng.integers(97, 123, size=64 * MiB, dtype=np.uint8)
    body[rng.integers(0, len(body), 5000)] = ord(",")
    body[rng.integers(0, len(body), 5000)] = ord("\n")
    txt = body.tobytes().replace(b"qz", b'q""z')  # a doubled quote wherever "qz" occurs
    data = u8(b'1,"' + txt + b'",end\n2,"a""b",c\n3,short,d\n')
    assert len(data) > 64 * MiB and txt.count(b'""') > 10000
    check(data, D.csv4(), [D.INT64, D.STRING, D.STRING], tag="64 MiB field")


def test_chars_capacity():
    g = datagen.c1()
    offs, chars = oracle.materialize(g.data, D.csv4(), 5)
    cap = int(offs[-1]) // 3
    got, _ = gpu_materialize(g.data, D.csv4(), list(D.SCHEMA_C1.types), [5], cap_chars=cap)
    go, gc = got[5]
    np.testing.assert_array_equal(go, offs)  # the offsets report the full size
    np.testing.assert_array_equal(gc[:cap], chars[:cap])
