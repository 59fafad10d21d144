"""Serving loop through the C-ABI: continuous batching of uneven requests.

Each request's results inside the mix equal its results solved alone with
pinmpc_solve (bitwise: per-problem arithmetic does not depend on what shares
the launch), sampled problems match the FP64 oracle, the lanes really overlap
requests (fewer launches than requests), and warm-started problems still
certify.
"""
import numpy as np
import pytest

import mpcgen
from oracle import kkt, qp
from gpu_common import ACT_TOL_FP32

pytestmark = pytest.mark.gpu


def _requests(n_req, per_req, seed_offset=0):
    reqs = []
    for i in range(n_req):
        idx = np.arange(per_req) + (i + seed_offset) * per_req
        b = mpcgen.make_batch("serving_tick", indices=idx)
        reqs.append(b)
    return reqs


def test_mix_equals_alone_and_matches_oracle():
    import torch
    from paper_2606_05687_amd import binding
    reqs = _requests(12, 48)
    devs = [binding.to_device(r) for r in reqs]
    # alone: one pinmpc_solve per request
    solver = binding.Solver(0, graph=0)
    alone = []
    for d in devs:
        o = solver.solve(d)
        torch.cuda.synchronize()
        alone.append({k: v.cpu().numpy() for k, v in o.items()})
    solver.close()
    # in the mix: all requests queued at once on a 3-lane server
    srv = binding.Server(0, lanes=3, capacity=256)
    outs = [solver.alloc_out(d) for d in devs]
    tickets = [srv.submit(d, o) for d, o in zip(devs, outs)]
    lat = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    print("launches", st, "latency ms p50 %.2f p99 %.2f" % (np.percentile(lat, 50),
                                                              np.percentile(lat, 99)))
    assert st["problems"] == 12 * 48
    assert st["launches"] < 12          # requests were packed together
    for i, o in enumerate(outs):
        got = {k: v.cpu().numpy() for k, v in o.items()}
        for k in got:
            assert np.array_equal(got[k], alone[i][k]), (i, k)
        assert (got["status"] == 0).all()
    for i in (0, 7):
        for b in (0, 5, 11):
            p = mpcgen.problem_fp64(reqs[i], b)
            ref = qp.solve(p)
            N = p["N"]
            u = outs[i]["u"][b, :N].cpu().numpy().astype(np.float64)
            x = outs[i]["x"][b, :N + 1].cpu().numpy().astype(np.float64)
            eu, ex = kkt.rel_err(u, ref["u"], x, ref["x"], p["weight"])
            assert eu <= 1e-4 and ex <= 1e-4, (i, b, eu, ex)
            assert kkt.residuals(p, u, x, act_tol=ACT_TOL_FP32)["kkt"] <= 1e-5


def test_warm_start_round_trip():
    import torch
    from paper_2606_05687_amd import binding
    reqs = _requests(2, 32, seed_offset=40)
    devs = [binding.to_device(r) for r in reqs]
    srv = binding.Server(0, lanes=2, capacity=128, warm_slots=64)
    outs = []
    for tick in range(3):
        o = [binding.Solver.alloc_out(None, d) for d in devs]
        t = [srv.submit(d, oo, warm_base=32 * i) for i, (d, oo) in enumerate(zip(devs, o))]
        for tt in t:
            srv.wait(tt)
        outs.append(o)
    srv.close()
    for tick in range(3):
        for i in range(2):
            assert (outs[tick][i]["status"].cpu().numpy() == 0).all()
    # a warm start changes the ADMM iterates, not the certified optimum
    for i in range(2):
        a = outs[0][i]["u"].cpu().numpy()
        c = outs[2][i]["u"].cpu().numpy()
        assert np.max(np.abs(a - c)) <= 1e-4 * np.max(np.abs(a))


def test_overlapping_warm_slots_rejected_while_in_flight():
    """A warm slot serves one request at a time: a second request whose slot
    range overlaps a request still in flight is refused with PINMPC_EBUSY,
    a disjoint range is accepted, and the overlapping range is accepted again
    once the first request is done."""
    import ctypes
    from paper_2606_05687_amd import binding
    big = mpcgen.make_batch("uneven_b16384", indices=range(2048), n_max=60)
    small = mpcgen.make_batch("uneven_b16384", indices=range(64), n_max=60)
    dbig, dsmall = binding.to_device(big), binding.to_device(small)
    srv = binding.Server(0, lanes=2, capacity=2048, warm_slots=4096)
    lib = binding.load()
    obig = binding.Solver.alloc_out(None, dbig)
    osm = [binding.Solver.alloc_out(None, dsmall) for _ in range(2)]
    t = ctypes.c_int64()
    bbig, bsm = binding.make_batch_struct(dbig), binding.make_batch_struct(dsmall)
    assert lib.pinmpc_submit(srv._h, ctypes.byref(bbig), ctypes.byref(binding._out_struct(obig)),
                             0, ctypes.byref(t)) == 0
    first = t.value
    rc = lib.pinmpc_submit(srv._h, ctypes.byref(bsm), ctypes.byref(binding._out_struct(osm[0])),
                           2000, ctypes.byref(t))
    assert rc == -5, rc                              # overlaps slots 2000..2047
    assert lib.pinmpc_submit(srv._h, ctypes.byref(bsm), ctypes.byref(binding._out_struct(osm[0])),
                             2048, ctypes.byref(t)) == 0   # disjoint
    second = t.value
    srv.wait(first)
    assert lib.pinmpc_submit(srv._h, ctypes.byref(bsm), ctypes.byref(binding._out_struct(osm[1])),
                             2000, ctypes.byref(t)) == 0
    srv.wait(second)
    srv.wait(t.value)
    srv.close()
    assert (obig["status"].cpu().numpy() == 0).all()
    for o in osm:
        assert (o["status"].cpu().numpy() == 0).all()


def test_warm_state_export_import_resumes_bitwise():
    """Checkpoint and resume of warm slots through the C ABI: a server that
    imports another server's exported warm state continues exactly as the
    exporter does (the next tick's results are bitwise equal); malformed
    ranges and images are refused; an export while a request on those slots
    is in flight is refused with PINMPC_EBUSY."""
    import ctypes
    from paper_2606_05687_amd import binding
    reqs = _requests(2, 32, seed_offset=60)
    devs = [binding.to_device(r) for r in reqs]

    def tick(srv):
        o = [binding.Solver.alloc_out(None, d) for d in devs]
        t = [srv.submit(d, oo, warm_base=32 * i) for i, (d, oo) in enumerate(zip(devs, o))]
        for tt in t:
            srv.wait(tt)
        return [{k: v.cpu().numpy() for k, v in oo.items()} for oo in o]

    a = binding.Server(0, lanes=2, capacity=128, warm_slots=64)
    tick(a)
    image = a.export_state(0, 64)
    assert len(image) == binding.warm_image_bytes(64) and image[:4] == b"PMWS"
    next_a = tick(a)
    b = binding.Server(0, lanes=1, capacity=128, warm_slots=64)
    cold_b = tick(b)                      # b's slots now hold b's own state
    b.import_state(0, 64, image)
    next_b = tick(b)
    for i in range(2):
        for k in next_a[i]:
            assert np.array_equal(next_a[i][k], next_b[i][k]), (i, k)
        assert (next_b[i]["status"] == 0).all()
    # the import really replaced b's state: without it the iterates differ
    assert any(not np.array_equal(cold_b[i]["iters"], next_a[i]["iters"]) or
               not np.array_equal(cold_b[i]["u"], next_a[i]["u"]) for i in range(2))
    lib = binding.load()
    buf = ctypes.create_string_buffer(binding.warm_image_bytes(64))
    assert lib.pinmpc_server_export_state(a._h, 60, 8, buf, len(buf)) == -1    # past the slots
    assert lib.pinmpc_server_export_state(a._h, 0, 64, buf, 100) == -1        # short buffer
    bad = bytearray(image)
    bad[0:4] = b"XXXX"
    with pytest.raises(binding.PinmpcError):
        b.import_state(0, 64, bytes(bad))
    bad = bytearray(image)
    bad[8:12] = (63).to_bytes(4, "little")                                    # wrong count
    with pytest.raises(binding.PinmpcError):
        b.import_state(0, 64, bytes(bad))
    # a request in flight on slots 0..2047 blocks their export
    big = binding.to_device(mpcgen.make_batch("uneven_b16384", indices=range(2048), n_max=60))
    c = binding.Server(0, lanes=1, capacity=2048, warm_slots=2048)
    ob = binding.Solver.alloc_out(None, big)
    t = c.submit(big, ob, warm_base=0)
    buf2 = ctypes.create_string_buffer(binding.warm_image_bytes(16))
    rc = lib.pinmpc_server_export_state(c._h, 100, 16, buf2, len(buf2))
    done = c.poll(t) is not None
    assert rc == binding.E_BUSY or (rc == 0 and done), rc
    c.wait(t) if not done else None
    assert lib.pinmpc_server_export_state(c._h, 100, 16, buf2, len(buf2)) == 0
    for s in (a, b, c):
        s.close()


def test_mix_of_optional_arrays_and_horizons():
    """Requests with and without the optional arrays (e, u_ref, u_prev, weight,
    per-problem horizons) and with different padded horizons packed into one
    launch: the gather fills what a request leaves out exactly as
    pinmpc_solve defaults it, so every result equals its request solved alone
    (bitwise)."""
    import torch
    from paper_2606_05687_amd import binding
    reqs = [mpcgen.make_batch("serving_tick", indices=range(i * 16, i * 16 + 16), offsets=True)
            for i in range(2)]
    reqs += [mpcgen.make_batch("plain_b4096_n20", indices=range(i * 7, i * 7 + 7)) for i in range(2)]
    devs = []
    for i, r in enumerate(reqs):
        d = binding.to_device(r)
        if i >= 2:          # leave the optional arrays out
            for k in ("e", "u_ref", "u_prev", "weight", "N"):
                d.pop(k, None)
        devs.append(d)
    solver = binding.Solver(0, graph=0, iters=3, refine_passes=12, first_passes=0)
    alone = []
    for d in devs:
        o = solver.solve(d)
        torch.cuda.synchronize()
        alone.append({k: v.cpu().numpy() for k, v in o.items()})
    solver.close()
    srv = binding.Server(0, lanes=1, capacity=128, iters=3, refine_passes=12, first_passes=0)
    outs = [binding.Solver.alloc_out(None, d) for d in devs]
    for o in outs:
        for v in o.values():
            v.fill_(-7)
    tickets = [srv.submit(d, o) for d, o in zip(devs, outs)]
    for t in tickets:
        srv.wait(t)
    st = srv.stats()
    srv.close()
    assert st["launches"] < len(devs)
    for i, o in enumerate(outs):
        for k, v in o.items():
            assert np.array_equal(v.cpu().numpy(), alone[i][k]), (i, k)
        assert (alone[i]["status"] == 0).all()
