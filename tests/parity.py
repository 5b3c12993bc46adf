"""Element-by-element comparison of the GPU parse with the oracle."""
import numpy as np

import oracle
import paper_1905_13415_amd as pp


def gpu_parse(data, dfa, types, cap_records=None, cap_fields=None, opts=None, offset=0):
    """Run the GPU parse of ``data`` (numpy uint8); returns (Outputs, result dict).
    ``offset`` shifts the input inside a larger device buffer (unaligned start)."""
    import torch
    if cap_records is None or cap_fields is None:
        r, f = oracle.count(data, dfa)
        cap_records = r if cap_records is None else cap_records
        cap_fields = f if cap_fields is None else cap_fields
    host = torch.from_numpy(np.ascontiguousarray(data))
    if offset:
        buf = torch.zeros(len(data) + offset, dtype=torch.uint8, device="cuda")
        buf[offset:] = host.cuda()
        d_in = buf[offset:]
    else:
        d_in = host.cuda()
    out = pp.parse(d_in, dfa, types, cap_records, cap_fields, opts=opts)
    torch.cuda.synchronize()
    return out, out.result_dict()


def expected_result(ref):
    return {"status": ref.status, "num_records": ref.num_records, "num_fields": ref.num_fields,
            "first_invalid_offset": ref.first_invalid_offset, "final_state": ref.final_state,
            "num_conversion_errors": ref.num_conversion_errors,
            "num_ragged_records": ref.num_ragged_records,
            "min_record_fields": ref.min_record_fields, "max_record_fields": ref.max_record_fields}


def compare(ref, out, res, types, tag=""):
    """Every output of a GPU parse equals the oracle's, bit for bit."""
    assert res == expected_result(ref), tag
    R = min(ref.num_records, out.cap_records)
    F = min(ref.num_fields, out.cap_fields)
    np.testing.assert_array_equal(out.record_offsets[:R + 1].cpu().numpy(), ref.record_offsets[:R + 1], err_msg=tag)
    np.testing.assert_array_equal(out.field_offsets[:F + 1].cpu().numpy(), ref.field_offsets[:F + 1], err_msg=tag)
    np.testing.assert_array_equal(out.column_ids[:F].cpu().numpy(), ref.column_ids[:F], err_msg=tag)
    for c, ty in enumerate(types):
        if ty == pp.SKIP:
            continue
        gv = out.values[c][:R].cpu().numpy()
        rv = ref.values[c][:R]
        # floats compared bit for bit
        np.testing.assert_array_equal(gv.view(np.int64), rv.view(np.int64), err_msg=f"{tag} column {c}")
        np.testing.assert_array_equal(out.valid[c][:R].cpu().numpy(), ref.valid[c][:R], err_msg=f"{tag} valid {c}")
        if ty == pp.STRING:
            np.testing.assert_array_equal(out.str_end[c][:R].cpu().numpy(), ref.str_end[c][:R],
                                          err_msg=f"{tag} end {c}")


def assert_same(data, dfa, types, opts=None, offset=0, cap_records=None, cap_fields=None):
    """Bit-exact parity of every output and result field."""
    ref = oracle.parse(data, dfa, types, cap_records=cap_records, cap_fields=cap_fields)
    out, res = gpu_parse(data, dfa, types, cap_records=cap_records, cap_fields=cap_fields,
                         opts=opts, offset=offset)
    compare(ref, out, res, types)
    return ref, out, res
