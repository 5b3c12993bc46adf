"""Validating and inferring the number of columns (Sec. 4.3) on the GPU,
against the oracle element by element:

- schema flag PP_SCHEMA_REJECT_RAGGED: records whose field count differs
  from the schema's lose their typed values (ragged text with quoted
  fields, a 70,000-field record spanning tiles, short and long records at
  tile starts, every launch shape);
- pp_infer_columns: the structure-only parse gives the result record (the
  most fields of any record is the inferred column count), never CAPACITY;
- the schema-less parse: that many string columns.
"""
import random

import numpy as np
import pytest

import oracle
import paper_1905_13415_amd as pp
from datagen import dialects as D
from parity import compare, expected_result

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

SHAPES = [None, (64, 256), (32, 256), (32, 512), (16, 256)]
SHAPE_IDS = ["512x64", "256x64", "256x32", "512x32", "256x16"]


def u8(b):
    return np.frombuffer(bytes(b), dtype=np.uint8)


def ragged_text(seed, nrec=6000):
    rnd = random.Random(seed)
    pieces = ["", "7", "-12", "3.25", "abc", '"x,y"', '"a\nb"', '"say ""hi"""', '""', "2020-02-29"]
    recs = []
    for _ in range(nrec):
        k = rnd.choice([4, 4, 4, 4, 3, 5, 1, 9])
        recs.append(",".join(rnd.choice(pieces) for _ in range(k)))
    return ("\n".join(recs) + "\n").encode()


TYPES4 = [D.INT64, D.STRING, D.FLOAT64, D.STRING]


@pytest.mark.parametrize("shape", SHAPES, ids=SHAPE_IDS)
def test_reject_ragged_matches_oracle(shape):
    opts = pp.options(*shape) if shape else None
    tile = shape[0] * shape[1] if shape else 32768
    long_rec = ",".join(["5"] * 70000) + "\n"  # spans several tiles
    data = ragged_text(1) + long_rec.encode() + ragged_text(2) + b"1,a,2.5,b\n" * 3000 + b"9,z"
    # a short record that begins exactly at a tile start
    pad = -len(data) % tile
    data = data + b"q" * max(pad - 1, 0) + b"\n" + b"1,x\n" + b"2,y,3.5,w\n" * 500
    arr = u8(data)
    for dfa in (D.csv4(), D.paper6()):
        ref = oracle.parse(arr, dfa, TYPES4, reject_ragged=True)
        assert ref.num_ragged_records > 0
        d_in = torch.from_numpy(arr.copy()).cuda()
        out = pp.parse(d_in, dfa, TYPES4, ref.num_records, ref.num_fields, opts=opts, reject_ragged=True)
        torch.cuda.synchronize()
        compare(ref, out, out.result_dict(), TYPES4, tag=f"{dfa.name} reject")


def test_reject_ragged_capacity_and_uniform():
    """Uniform input: nothing rejected (identical to the plain parse); a
    record capacity below R: only records within it are touched."""
    arr = u8(b"1,a,2.5,b\n" * 5000)
    ref = oracle.parse(arr, D.csv4(), TYPES4)
    d_in = torch.from_numpy(arr.copy()).cuda()
    out = pp.parse(d_in, D.csv4(), TYPES4, ref.num_records, ref.num_fields, reject_ragged=True)
    torch.cuda.synchronize()
    compare(ref, out, out.result_dict(), TYPES4)
    arr = u8(ragged_text(5, 3000))
    R, F = oracle.count(arr, D.csv4())
    ref = oracle.parse(arr, D.csv4(), TYPES4, cap_records=R // 2, cap_fields=F, reject_ragged=True)
    d_in = torch.from_numpy(arr.copy()).cuda()
    out = pp.parse(d_in, D.csv4(), TYPES4, R // 2, F, reject_ragged=True)
    torch.cuda.synchronize()
    compare(ref, out, out.result_dict(), TYPES4, tag="capacity")


@pytest.mark.parametrize("shape", [None, (16, 256)], ids=["512x64", "256x16"])
def test_infer_columns(shape):
    opts = pp.options(*shape) if shape else None
    cases = [u8(ragged_text(3)), u8(b"1,2,3\n" * 20000), u8(b""), u8(b"a"), u8(b'x,"unterminated'),
             u8(ragged_text(4) + (",".join(["1"] * 70000) + "\n").encode())]
    for dfa in (D.csv4(), D.paper6()):
        for arr in cases:
            ref = oracle.parse(arr, dfa, [])
            d_in = torch.from_numpy(arr.copy()).cuda() if len(arr) else torch.empty(0, dtype=torch.uint8,
                                                                                     device="cuda")
            got = pp.infer_columns(d_in, dfa, opts)
            want = expected_result(ref)
            assert got == want, (dfa.name, len(arr))
            assert got["status"] != pp.RESULT_CAPACITY


def test_schemaless_parse():
    arr = u8(ragged_text(7))
    ref_inf = oracle.parse(arr, D.csv4(), [])
    ncols = ref_inf.max_record_fields
    ref = oracle.parse(arr, D.csv4(), [D.STRING] * ncols)
    d_in = torch.from_numpy(arr.copy()).cuda()
    out, inf = pp.parse_schemaless(d_in, D.csv4())
    torch.cuda.synchronize()
    assert inf["max_record_fields"] == ncols == 9
    compare(ref, out, out.result_dict(), [D.STRING] * ncols, tag="schemaless")
