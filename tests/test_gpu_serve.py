"""Serving form: requests streamed from pinned host memory through the
request loop give the same outputs as the oracle, and the same outputs
whether a request is served alone or in a mix where the budget forces
queueing, slots are shared, capacities overflow and launches batch several
requests together."""
import time

import numpy as np
import pytest

import datagen
import oracle
import paper_1905_13415_amd as pp
from datagen import dialects as D
from parity import expected_result

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

MiB = 1 << 20


def _dialects():
    return [D.log6(), D.csv4(b","), D.paper6(b"|")]


def _requests(count, seed):
    """(bytes, dialect index, types) with sizes log-uniform in 4 KiB..3 MiB."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(np.exp(rng.uniform(np.log(4096), np.log(3 * MiB))))
        which = int(rng.integers(0, 3))
        if which == 0:
            g = datagen.log(seed * 1000 + i, n)
            out.append((g.data, 0, list(D.SCHEMA_LOG12.types)))
        else:
            g = datagen.generate(datagen.K_MIXED, seed * 1000 + i, max_bytes=n,
                                 delim=b"," if which == 1 else b"|", qstyle=1, block_records=4096)
            out.append((g.data, which, list(D.SCHEMA_C1.types)))
    # edge cases: empty, one record without its LF, a 2 MiB single-record soup
    out.append((np.zeros(0, np.uint8), 1, [D.INT64, D.STRING]))
    out.append((np.frombuffer(b"1,abc", np.uint8).copy(), 1, [D.INT64, D.STRING]))
    return out


def _pinned(data):
    t = torch.empty(len(data), dtype=torch.uint8).pin_memory()
    if len(data):
        t.numpy()[:] = data
    return t


def _drain(srv, want, timeout_s=120):
    got = {}
    t0 = time.time()
    while len(got) < want:
        assert time.time() - t0 < timeout_s, f"server stalled: {srv.stats()}"
        srv.wait(2000)
        for c in srv.poll():
            got[c.id] = (c, c.fetch())
            srv.release(c.id)
    return got


def _same(a, b, tag):
    for k in ("record_offsets", "field_offsets", "column_ids"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=f"{tag} {k}")
    for k in ("values", "valid", "str_end"):
        for c, (x, y) in enumerate(zip(a[k], b[k])):
            if x is None:
                assert y is None
                continue
            np.testing.assert_array_equal(x.view(np.int64) if x.dtype == np.float64 else x,
                                          y.view(np.int64) if y.dtype == np.float64 else y,
                                          err_msg=f"{tag} {k}[{c}]")


def _as_fetch(ref, types):
    R, F = ref.num_records, ref.num_fields
    return {"record_offsets": ref.record_offsets[:R + 1], "field_offsets": ref.field_offsets[:F + 1],
            "column_ids": ref.column_ids[:F],
            "values": [None if t == D.SKIP else ref.values[c][:R] for c, t in enumerate(types)],
            "valid": [None if t == D.SKIP else ref.valid[c][:R] for c, t in enumerate(types)],
            "str_end": [ref.str_end[c][:R] if t == D.STRING else None for c, t in enumerate(types)]}


def test_server_alone_and_in_mix_match_oracle():
    dfas = _dialects()
    reqs = _requests(36, seed=5)
    pinned = [_pinned(d) for d, _, _ in reqs]
    refs = [oracle.parse(d, dfas[k], types) for d, k, types in reqs]

    # alone: one request in the server at a time, exact capacities
    alone = []
    srv = pp.Server(dfas, hbm_budget_bytes=256 * MiB, max_slots=4)
    for (d, k, types), h, ref in zip(reqs, pinned, refs):
        rid = srv.submit(h, k, types, ref.num_records, ref.num_fields)
        (c, out), = _drain(srv, 1).values()
        assert c.id == rid
        assert c.result == expected_result(ref)
        _same(out, _as_fetch(ref, types), f"alone request {rid}")
        assert c.t_arrival_ns <= c.t_admit_ns <= c.t_h2d_done_ns <= c.t_parse_done_ns
        alone.append((c.result, out))
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["arena_used_bytes"] == 0
    srv.close()

    # in the mix: everything submitted at once into a small budget with few
    # slots; every third request under-states its capacity
    srv = pp.Server(dfas, hbm_budget_bytes=64 * MiB, max_slots=12, max_batch=8)
    ids = []
    for i, ((d, k, types), h, ref) in enumerate(zip(reqs, pinned, refs)):
        cr, cf = ref.num_records, ref.num_fields
        if i % 3 == 0:
            cr, cf = cr // 3, cf // 4
        ids.append(srv.submit(h, k, types, cr, cf))
    got = _drain(srv, len(reqs))
    for i, rid in enumerate(ids):
        c, out = got[rid]
        assert c.result == alone[i][0], f"request {i}"
        _same(out, alone[i][1], f"mixed request {i}")
    st = srv.stats()
    assert st["completed"] == len(reqs)
    assert st["reparsed"] >= sum(1 for i, (_, _, _) in enumerate(reqs)
                                 if i % 3 == 0 and refs[i].num_records > 0)
    assert st["max_batch"] > 1 and st["batches"] < st["batched_requests"]
    assert st["arena_peak_bytes"] <= st["arena_bytes"] and st["arena_used_bytes"] == 0
    srv.close()


def test_server_rejects_oversized_and_bad_requests():
    dfas = _dialects()
    srv = pp.Server(dfas, hbm_budget_bytes=64 * MiB, max_slots=2)
    big = torch.empty(80 * MiB, dtype=torch.uint8).pin_memory()
    with pytest.raises(pp.PpError, match="budget"):
        srv.submit(big, 0, list(D.SCHEMA_LOG12.types), 1, 1)
    small = _pinned(np.frombuffer(b"1,2\n", np.uint8).copy())
    with pytest.raises(pp.PpError):
        srv.submit(small, 7, [D.INT64], 1, 2)  # no such dialect
    with pytest.raises(pp.PpError):
        srv.submit(small, 1, [42], 1, 2)  # no such type
    rid = srv.submit(small, 1, [D.INT64, D.INT64], 1, 2)
    (c, out), = _drain(srv, 1).values()
    assert c.id == rid and c.result["status"] == pp.RESULT_OK
    assert out["values"][1].tolist() == [2]
    with pytest.raises(pp.PpError):
        srv.release(rid)  # already released by _drain
    srv.close()


def test_server_c5_shaped_matches_oracle():
    """The serving workload's shape: the log dialect (12 columns), request
    sizes log-uniform from 4 KiB with several of 64-256 MiB among them,
    Poisson arrivals overlapping the work in flight, a 2 GiB budget. Every
    completion is compared with the oracle element by element."""
    dfas = [D.log6()]
    types = list(D.SCHEMA_LOG12.types)
    rng = np.random.default_rng(190513419)
    sizes = [int(np.exp(rng.uniform(np.log(4096), np.log(16 * MiB)))) for _ in range(28)]
    for k, big in enumerate((64, 96, 160, 256)):
        sizes.insert(3 + 7 * k, big * MiB)
    reqs = [datagen.log(7000 + i, n).data for i, n in enumerate(sizes)]
    assert max(len(d) for d in reqs) > 255 * MiB
    pinned = [_pinned(d) for d in reqs]
    arrivals = np.cumsum(rng.exponential(2e-3, len(reqs)))
    srv = pp.Server(dfas, hbm_budget_bytes=2048 * MiB, max_slots=16, max_batch=8)
    ids, got = {}, {}
    t0 = time.time()
    for i, (d, h) in enumerate(zip(reqs, pinned)):
        while time.time() - t0 < arrivals[i]:  # arrivals overlap the work in flight
            for c in srv.poll():
                got[c.id] = (c, c.fetch())
                srv.release(c.id)
            time.sleep(2e-4)
        # capacities from the request's byte count (log records average ~230
        # bytes); a request that needs more is parsed again with exact sizes
        cr = len(d) // 150 + 1
        ids[srv.submit(h, 0, types, cr, 12 * cr)] = i
    got.update(_drain(srv, len(reqs) - len(got), timeout_s=300))
    assert sorted(ids) == sorted(got)
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["arena_used_bytes"] == 0 and st["hip_error"] == 0
    assert st["arena_peak_bytes"] <= st["arena_bytes"]
    srv.close()
    for rid, i in ids.items():
        c, out = got[rid]
        ref = oracle.parse(reqs[i], dfas[0], types)
        assert c.result == expected_result(ref), f"request {i} ({len(reqs[i])} bytes)"
        _same(out, _as_fetch(ref, types), f"request {i} ({len(reqs[i])} bytes)")
