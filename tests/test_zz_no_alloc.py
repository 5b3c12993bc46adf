"""pp_parse_noalloc (the entry point for callers that cannot allocate: its
workspace is the library's static per-device array) against pp_parse with a
caller-allocated workspace, through the C ABI: two calls in a row on the
same GPU, the second on a smaller input (the array keeps the first call's
lookback words and tables), each compared element by element with pp_parse's
outputs on the same bytes, and with the oracle."""
import numpy as np
import pytest

import datagen
import oracle
import paper_1905_13415_amd as pp
from datagen import dialects as D
from parity import compare

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _same_outputs(a, b, types, tag):
    assert a.result_dict() == b.result_dict(), tag
    R = min(a.result_dict()["num_records"], a.cap_records)
    F = min(a.result_dict()["num_fields"], a.cap_fields)
    for x, y, k in ((a.record_offsets[:R + 1], b.record_offsets[:R + 1], "record_offsets"),
                    (a.field_offsets[:F + 1], b.field_offsets[:F + 1], "field_offsets"),
                    (a.column_ids[:F], b.column_ids[:F], "column_ids")):
        assert torch.equal(x, y), f"{tag}: {k}"
    for c, ty in enumerate(types):
        if ty == pp.SKIP:
            continue
        assert torch.equal(a.values[c][:R].view(torch.int64), b.values[c][:R].view(torch.int64)), f"{tag}: values {c}"
        assert torch.equal(a.valid[c][:R], b.valid[c][:R]), f"{tag}: valid {c}"
        if ty == pp.STRING:
            assert torch.equal(a.str_end[c][:R], b.str_end[c][:R]), f"{tag}: str_end {c}"


@pytest.mark.parametrize("opts", [None, pp.options(16, 256)], ids=["512x64", "256x16"])
def test_noalloc_matches_pp_parse_twice(opts):
    cases = [
        ("numeric 6 MiB", datagen.c2(nbytes=6 << 20).data, D.csv4(), list(D.SCHEMA_C2.types)),
        ("quoted 10k records", datagen.c1().data, D.csv4(), list(D.SCHEMA_C1.types)),
    ]
    assert len(cases[1][1]) < len(cases[0][1])  # the second call is the smaller one
    for tag, data, dfa, types in cases:
        print(f"[noalloc] {tag}: {len(data)} bytes, shape {opts and (opts.block_threads, opts.bytes_per_thread)}",
              flush=True)
        d_in = torch.from_numpy(np.ascontiguousarray(data)).cuda()
        R, F = oracle.count(data, dfa)
        ref_out = pp.parse(d_in, dfa, types, R, F, opts=opts)
        torch.cuda.synchronize()
        got = pp.parse_noalloc(d_in, dfa, types, R, F, opts=opts)
        torch.cuda.synchronize()
        _same_outputs(got, ref_out, types, tag)
        ref = oracle.parse(data, dfa, types)
        compare(ref, got, got.result_dict(), types, tag=tag)


def test_noalloc_rejects_inputs_beyond_its_scratch():
    dfa, types = D.csv4(), [D.INT64]
    d_in = torch.zeros(16, dtype=torch.uint8, device="cuda")
    out = pp.alloc_outputs(types, 4, 4, device=d_in.device)
    call = pp.Call(d_in, 16, dfa, types, out, None, pp.options(16, 256))
    # an input size whose workspace exceeds the static array (checked on the
    # host before any launch; nothing is read past the 16 real bytes)
    call.n = (pp.NOALLOC_SCRATCH_BYTES // 64 + 1) * 4096
    with pytest.raises(pp.PpError, match="workspace"):
        call.launch_noalloc()
    call.n = 16
    call.launch_noalloc()
    torch.cuda.synchronize()
    assert out.result_dict()["status"] == pp.RESULT_OK
