"""UTF-16 text (pp_parse_utf16, Sec. 4.2) against the oracle's UTF-16 run,
bit for bit: every output, with positions as byte offsets into the UTF-16
input.

Covers ASCII text (the quoted CSV, the numeric CSV, the log dialect) under
every launch shape, text with non-ASCII characters (accented Latin, CJK,
characters outside the BMP as surrogate pairs, a fullwidth comma that is
data) across many tiles, numerals with non-ASCII digits, invalid input,
empty and one-unit inputs, an input 2 bytes off 16-byte alignment, rejected
ragged records and the tiles parsed out of order; every path of the tile
kernel (per-thread fields, fields and numbers that begin before the tile's
LDS copy, invalid input); and materialised string columns of UTF-16 text
(pp_materialize_strings_utf16).
"""
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

SHAPES = [None, (64, 256), (32, 256), (32, 512), (16, 256)]
SHAPE_IDS = ["512x64", "256x64", "256x32", "512x32", "256x16"]


def same(b16: bytes, dfa, types, opts=None, offset=0, reject_ragged=False, tag=""):
    ref = oracle.parse(b16, dfa, types, utf16=True, reject_ragged=reject_ragged)
    host = torch.from_numpy(np.frombuffer(b16, dtype=np.uint8).copy())
    if offset:  # the text 'offset' bytes into a larger buffer
        buf = torch.zeros(len(b16) + offset, dtype=torch.uint8, device="cuda")
        buf[offset:] = host.cuda()
        d_in = buf[offset:]
    else:
        d_in = host.cuda()
    out = pp.parse_utf16(d_in, dfa, types, ref.num_records, ref.num_fields, opts=opts, reject_ragged=reject_ragged)
    torch.cuda.synchronize()
    compare(ref, out, out.result_dict(), types, tag=tag)
    return ref


def widen(data) -> bytes:
    return bytes(data).decode("latin-1").encode("utf-16-le")


@pytest.mark.parametrize("shape", SHAPES, ids=SHAPE_IDS)
def test_ascii_workloads(shape):
    o = pp.options(*shape) if shape else None
    same(widen(datagen.c1().data), D.csv4(), D.SCHEMA_C1.types, opts=o, tag="c1")
    same(widen(datagen.c2(nbytes=3 << 20).data), D.csv4(), D.SCHEMA_C2.types, opts=o, tag="c2 slice")
    same(widen(datagen.log(41, 2 << 20).data), D.log6(), D.SCHEMA_LOG12.types, opts=o, tag="log")


def _text(seed, nrec):
    rng = random.Random(seed)
    pieces = ["", "7", "-12", "2.5", "2020-02-29", "é", "漢字", "😀x", '"x,y"', '"a\nb"', '"say ""hi"""', '""',
              "a，b", "٣", "naïve café", '"日本,語"']
    recs = [",".join(rng.choice(pieces) for _ in range(rng.choice([3, 4, 4, 4, 5])))
            for _ in range(nrec)]
    return ("\n".join(recs) + "\n").encode("utf-16-le")


@pytest.mark.parametrize("shape", SHAPES, ids=SHAPE_IDS)
def test_non_ascii_text(shape):
    o = pp.options(*shape) if shape else None
    types = [D.STRING, D.INT64, D.FLOAT64, D.DATE_DAYS]
    for seed, nrec in ((1, 10), (2, 3000), (3, 60000)):
        ref = same(_text(seed, nrec), D.csv4(), types, opts=o, tag=f"seed {seed}")
        assert ref.num_conversion_errors > 0 or nrec < 100


def test_edges_alignment_rejection_and_order():
    types = [D.STRING, D.INT64, D.FLOAT64, D.DATE_DAYS]
    for text in ("", "7", "\n", "a", "😀", '"open', '1,"a""b"\n٣,x'):
        for dfa in (D.csv4(), D.paper6()):
            same(text.encode("utf-16-le"), dfa, types, tag=repr(text))
    b16 = _text(5, 20000)
    same(b16, D.csv4(), types, offset=2, tag="2 bytes off alignment")
    same(b16, D.csv4(), types, reject_ragged=True, tag="rejected ragged records")
    same(b16, D.paper6(), types, tag="paper6 (invalid input)")
    for order in (1, 9):
        same(b16, D.csv4(), types, opts=pp.options(16, 256, order), tag=f"tile order {order}")


TILE = 512 * 64  # code units per tile of the default launch shape


def test_tile_paths():
    """The code-unit form through every path of the tile kernel: every
    symbol a delimiter (more fields than a tile stages: the per-thread
    path), a quoted field of non-ASCII text spanning tiles, numbers spanning
    tiles (converted from units read and narrowed outside the tile's LDS
    copy), the first field of a tile beginning at offsets around the 64
    units kept before the tile, and invalid input deep in the text."""
    t3 = [D.INT64, D.STRING, D.FLOAT64]
    for ch in (",", "\n"):
        same((ch * (3 * TILE + 5)).encode("utf-16-le"), D.csv4(), t3, tag=f"all {ch!r}")
    body = "".join(random.Random(1).choice('ab,\n é漢😀""') for _ in range(2 * TILE))
    for dfa in (D.csv4(), D.paper6()):
        same(('1,"' + body + '",2\n3,"x",4\n').encode("utf-16-le"), dfa, t3, tag="long quoted field")
    same(("7," + "0" * (2 * TILE + 100) + "42,x\n1.5," + "9" * 30000 + ",y\n").encode("utf-16-le"), D.csv4(),
         [D.FLOAT64, D.INT64, D.STRING], tag="long numbers")
    first = "p" * 10 + ",1,2.5\n"
    for head in ("-1234567", '"q,u""o"', "é"):
        for d in (0, 1, 63, 64, 65, 100, 300):
            # field 1 of the second record begins d units before the second tile
            pad = TILE - d - len(first) - 1
            text = first + "漢" * pad + "," + head + ",2.5\n" + "1,2,3.5\n" * 50
            assert text.find(head, len(first)) == TILE - d
            for types in ([D.STRING, D.INT64, D.FLOAT64], [D.INT64, D.STRING, D.FLOAT64]):
                same(text.encode("utf-16-le"), D.csv4(), types, tag=f"{head!r} at -{d}")
    data = bytearray(datagen.c1().data[:5 * TILE])
    data[3 * TILE + 100] = ord('"')  # a quote in an unquoted field: invalid under paper6
    ref = same(widen(data), D.paper6(), D.SCHEMA_C1.types, tag="invalid")
    assert ref.first_invalid_offset >= 0


@pytest.mark.parametrize("shape", [None, (16, 256)], ids=["512x64", "256x16"])
def test_materialized_strings(shape):
    """String columns of UTF-16 text materialised (control symbols removed,
    code units kept), with and without a terminator code unit, against the
    oracle's, including one quoted field far longer than a tile."""
    o = pp.options(*shape) if shape else None
    big = '1,"' + ("漢a,\n" * 40000) + '""q😀",x\n'
    for b16 in (_text(7, 2000), _text(8, 40000), (big + "2,b,c\n").encode("utf-16-le")):
        types = [D.STRING, D.STRING, D.STRING, D.STRING]
        R, F = oracle.count(b16, D.csv4(), utf16=True)
        d_in = torch.from_numpy(np.frombuffer(b16, dtype=np.uint8).copy()).cuda()
        out = pp.parse_utf16(d_in, D.csv4(), types, R, F, opts=o, control_bitmap=True)
        for c in range(4):
            for term in (-1, 0x2028):
                offs, chars = pp.materialize_utf16(d_in, out, c, terminator=term)
                torch.cuda.synchronize()
                want_o, want_c = oracle.materialize(b16, D.csv4(), c, terminator=term, utf16=True)
                np.testing.assert_array_equal(offs.cpu().numpy()[:R + 1], want_o, err_msg=f"offsets {c} {term}")
                got = chars.cpu().numpy().view(np.uint16)[:want_o[-1]]
                np.testing.assert_array_equal(got, want_c, err_msg=f"chars {c} {term}")
