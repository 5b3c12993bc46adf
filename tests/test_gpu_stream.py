"""End-to-end streaming form (pp_stream_*, Sec. 4.4) against the oracle run
over the whole input: every output (rebased to global byte, field and record
indices) and the result record, bit for bit.

Partitions as small as 4 KiB put partition boundaries inside quoted fields,
inside records with embedded line feeds and between a record delimiter and
its record; records longer than a partition are carried whole; the 2 GiB
text-heavy CSV is streamed in 256 MiB partitions from pinned host memory.
"""
import numpy as np
import pytest

import datagen
import oracle
import paper_1905_13415_amd as pp
from datagen import dialects as D
from parity import expected_result

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

KiB, MiB = 1 << 10, 1 << 20


def u8(b):
    return np.frombuffer(bytes(b), dtype=np.uint8)


def stream_parse(data, dfa, types, partition_bytes, max_record_bytes=64 * KiB, cap_records=0, cap_fields=0,
                 host_caps=None):
    R, F = oracle.count(data, dfa)
    hr, hf = host_caps or (R, F)
    st = pp.Stream(dfa, types, partition_bytes=partition_bytes, max_record_bytes=max_record_bytes,
                   cap_records=cap_records, cap_fields=cap_fields)
    h_in = torch.from_numpy(np.ascontiguousarray(data).copy()).pin_memory() if len(data) else \
        torch.empty(0, dtype=torch.uint8)
    out = pp.alloc_host_outputs(types, hr, hf)
    try:
        st.parse(h_in, out)
    finally:
        st.close()
    return out


def same_as_oracle(data, dfa, types, out, tag=""):
    ref = oracle.parse(data, dfa, types)
    assert out.result == expected_result(ref), tag
    R, F = ref.num_records, ref.num_fields
    np.testing.assert_array_equal(out.record_offsets[:R + 1].numpy(), ref.record_offsets[:R + 1], err_msg=tag)
    np.testing.assert_array_equal(out.field_offsets[:F + 1].numpy(), ref.field_offsets[:F + 1], err_msg=tag)
    np.testing.assert_array_equal(out.column_ids[:F].numpy(), ref.column_ids[:F], err_msg=tag)
    for c, ty in enumerate(types):
        if ty == D.SKIP:
            continue
        np.testing.assert_array_equal(out.values[c][:R].numpy().view(np.int64), ref.values[c][:R].view(np.int64),
                                      err_msg=f"{tag} column {c}")
        np.testing.assert_array_equal(out.valid[c][:R].numpy(), ref.valid[c][:R], err_msg=f"{tag} valid {c}")
        if ty == D.STRING:
            np.testing.assert_array_equal(out.str_end[c][:R].numpy(), ref.str_end[c][:R], err_msg=f"{tag} end {c}")
    return ref


@pytest.mark.parametrize("pbytes", [4096, 5000, 65536, 1 << 20])
def test_quoted_csv_in_small_partitions(pbytes):
    """The 10,000-record quoted CSV (embedded commas, line feeds and doubled
    quotes): partition boundaries fall inside quoted fields."""
    data = datagen.c1().data
    print(f"[stream] c1 {len(data)} bytes, partitions of {pbytes}", flush=True)
    out = stream_parse(data, D.csv4(), list(D.SCHEMA_C1.types), pbytes)
    same_as_oracle(data, D.csv4(), list(D.SCHEMA_C1.types), out, f"P={pbytes}")
    assert out.stats["partitions"] == (len(data) + pbytes - 1) // pbytes
    assert out.stats["carried_bytes"] > 0


@pytest.mark.parametrize("tail", [b"", b"\n", b"1,2", b"x,", b'"open'])
def test_endings(tail):
    """Inputs ending with and without a record delimiter, with a trailing
    field delimiter and inside an unterminated quote (NON_ACCEPTING_END)."""
    data = np.concatenate([datagen.c1().data[:50000], u8(tail)])
    for dfa in (D.csv4(), D.paper6()):
        out = stream_parse(data, dfa, list(D.SCHEMA_C1.types), 8192)
        same_as_oracle(data, dfa, list(D.SCHEMA_C1.types), out, f"tail {tail!r} {dfa.name}")


def test_empty_and_single_partition():
    for text in (b"", b"a", b"\n", b"1,2,3\n4,5,6\n"):
        out = stream_parse(u8(text), D.csv4(), [D.INT64, D.INT64, D.STRING], 4096)
        same_as_oracle(u8(text), D.csv4(), [D.INT64, D.INT64, D.STRING], out, repr(text))


def test_log_dialect_and_long_records():
    """The 6-state log dialect (brackets, escaped quotes) with records longer
    than a partition: a partition holding no record delimiter is carried
    whole into the next one."""
    g = datagen.log(7, 300 * KiB)
    long_rec = b'h - u [01/Jan/2020:00:00:00 +0000] "' + b"a" * 20000 + b'" 200 1 "-" "x" 0.001 80 s\n'
    cut = bytes(g.data[:100000]).rfind(b"\n") + 1  # at a record end
    data = np.concatenate([g.data[:cut], u8(long_rec), g.data[cut:]])
    types = list(D.SCHEMA_LOG12.types)
    out = stream_parse(data, D.log6(), types, 4096)
    same_as_oracle(data, D.log6(), types, out, "log")
    assert out.stats["max_carry"] > 4096


def test_record_longer_than_carry_region_fails():
    data = u8(b"1,2\n" + b"x" * 20000 + b"\n3,4\n")
    st = pp.Stream(D.csv4(), [D.INT64, D.INT64], partition_bytes=4096, max_record_bytes=8192)
    out = pp.alloc_host_outputs([D.INT64, D.INT64], 8, 8)
    with pytest.raises(pp.PpError, match="unsupported"):
        st.parse(torch.from_numpy(data.copy()), out)
    st.close()


def test_invalid_input_stops_at_its_partition():
    """paper6 (Table 1) enters its invalid state on a quote inside an
    unquoted field; the stream reports the offset of that transition."""
    good = datagen.c1().data[:40000]
    cut = bytes(good).rfind(b"\n") + 1
    data = np.concatenate([good[:cut], u8(b'1,2,ab"c,4\n'), good[:cut]])
    ref = oracle.parse(data, D.paper6(), list(D.SCHEMA_C1.types))
    assert ref.status == pp.RESULT_INVALID_INPUT
    out = stream_parse(data, D.paper6(), list(D.SCHEMA_C1.types), 8192)
    assert out.result["status"] == pp.RESULT_INVALID_INPUT
    assert out.result["first_invalid_offset"] == ref.first_invalid_offset
    R = out.result["num_records"]
    assert R == ref.num_records - 1  # the oracle's last record absorbs the rest of the input
    np.testing.assert_array_equal(out.record_offsets[:R + 1].numpy(), ref.record_offsets[:R + 1])


def test_capacity():
    data = datagen.c1().data[:60000]
    R, F = oracle.count(data, D.csv4())
    out = stream_parse(data, D.csv4(), list(D.SCHEMA_C1.types), 8192, host_caps=(R // 2, F))
    assert out.result["status"] == pp.RESULT_CAPACITY
    out = stream_parse(data, D.csv4(), list(D.SCHEMA_C1.types), 8192, cap_records=5)
    assert out.result["status"] == pp.RESULT_CAPACITY


def test_text_heavy_2gib_in_256mib_partitions():
    """The 2 GiB text-heavy CSV from pinned host memory in 256 MiB
    partitions (quoted fields with embedded delimiters span partitions)."""
    g = datagen.c3()
    types = list(D.SCHEMA_C3.types)
    print(f"[stream] c3 {len(g.data)} bytes", flush=True)
    out = stream_parse(g.data, D.csv4(), types, 256 * MiB, max_record_bytes=1 * MiB)
    ref = same_as_oracle(g.data, D.csv4(), types, out, "c3")
    assert ref.num_records == g.nrecords
    assert out.stats["partitions"] == 8


@pytest.mark.parametrize("seed", range(6))
def test_random_dialects_in_small_partitions(seed):
    """Random DFAs (tags of every kind anywhere) whose line feed ends a record
    from every state, and whose record delimiters all return to the start
    state, as the streaming form requires: partitions of a few KiB cut records, quoted-like regions and
    escapes at arbitrary points."""
    import random
    from test_gpu_random_dfa import random_dfa, random_input
    rnd = random.Random(900 + seed)
    dfa = random_dfa(rnd, f"st{seed}")
    dfa.invalid_state = D.NO_STATE
    lf = dfa.group_of[ord("\n")]
    if lf == dfa.num_groups - 1:  # the line feed fell into the catch-all group: give it a group of its own
        dfa.group_symbols = dfa.group_symbols + [b"\n"]
        dfa.next_state.insert(len(dfa.group_symbols) - 1, [0] * dfa.num_states)
        dfa.tag.insert(len(dfa.group_symbols) - 1, [0] * dfa.num_states)
        gm = bytearray(dfa.group_of)
        for b in range(256):
            if gm[b] >= len(dfa.group_symbols) - 1:
                gm[b] += 1
        gm[ord("\n")] = len(dfa.group_symbols) - 1
        dfa.group_of = bytes(gm)
        lf = len(dfa.group_symbols) - 1
    for s in range(dfa.num_states):
        dfa.next_state[lf][s] = dfa.start_state
        dfa.tag[lf][s] = D.RECORD
    for g in range(dfa.num_groups):  # every record delimiter restarts the DFA
        for s in range(dfa.num_states):
            if dfa.tag[g][s] == D.RECORD:
                dfa.next_state[g][s] = dfa.start_state
    types = [rnd.choice([D.INT64, D.FLOAT64, D.STRING, D.SKIP]) for _ in range(rnd.randint(1, 6))]
    data = random_input(rnd, dfa, 300_000)
    for pbytes in (4096, 5000, 65536):
        print(f"[stream] random dialect {seed}, partitions of {pbytes}", flush=True)
        # a random dialect may close a field or record at every byte: the
        # per-partition capacities cover that worst case
        cap = pbytes + 64 * KiB + 1
        out = stream_parse(data, dfa, types, pbytes, cap_records=cap, cap_fields=cap)
        same_as_oracle(data, dfa, types, out, f"seed {seed} P={pbytes}")
