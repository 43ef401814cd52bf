"""Serving: concurrent requests of different grid sizes give the same results as
solving each alone, admission follows the HBM budget, and the served results match
the FP64 path."""
import time

import numpy as np
import pytest

from paper_1405_6456_amd import synth
from tests.gpu_util import ctx

pytestmark = pytest.mark.gpu


def requests():
    # four small systems of different grid sizes (21^3 .. 48^3)
    out = []
    for L, n, shift in ((16.0, 21, (0.11, -0.07, 0.05)), (17.6, 23, (-0.2, 0.1, 0.0)), (18.0, 25, (0.0, 0.0, 0.3))):
        S = synth.single_atom(L=L, n=n)
        S.R[0] += np.array(shift)
        out.append(S)
    out.append(synth.fcc_cluster(1, seed=10001, name="fcc1"))
    return out


@pytest.fixture(scope="module")
def alone():
    import paper_1405_6456_amd as lib

    c = ctx()
    c.set_tuning(target_blocks=lib.SERVER_SLOT_BLOCKS)  # the launch size of a server slot
    prm = lib.default_params(precision=lib.FP32_REFINED)
    res = [c.solve(S, prm, None) for S in requests()]
    c.close()
    return res


def test_same_alone_and_in_the_mix(alone):
    import paper_1405_6456_amd as lib

    ctx().close()  # skips without a GPU
    srv = lib.Server(0, max_slots=4)
    prm = lib.default_params(precision=lib.FP32_REFINED)
    reqs = requests()
    # submit twice in interleaved order so different sizes overlap on the device
    tickets = [(i, srv.submit(S, prm)) for _ in range(2) for i, S in enumerate(reqs)]
    for i, t in tickets:
        r = srv.wait(t)
        a = alone[i]
        assert r["status"] == 0 and a["status"] == 0
        assert abs(r["E_total"] - a["E_total"]) <= 1e-10 * max(1.0, abs(a["E_total"]))
        assert np.abs(r["forces"] - a["forces"]).max() <= 1e-10
        assert np.abs(r["u"] - a["u"]).max() <= 1e-10 * np.abs(a["u"]).max()
    st = srv.stats()
    assert st["completed"] == len(tickets) and st["rejected"] == 0 and st["queued"] == 0
    assert st["p50_ms"] > 0 and st["p99_ms"] >= st["p50_ms"] and st["solves_per_s"] > 0
    srv.close()


def test_fp64_requests_same_alone_and_in_the_mix():
    # FP64 requests on these small grids run the pipelined CG (one launch per iteration,
    # per-request state and partial buffers).  Overlapped on the device, each reaches the
    # result it reaches alone, to the same bounds as the FP32-refined requests
    import paper_1405_6456_amd as lib

    c = ctx()
    c.set_tuning(target_blocks=lib.SERVER_SLOT_BLOCKS)
    prm = lib.default_params(precision=lib.FP64)
    reqs = requests()
    single = [c.solve(S, prm, None) for S in reqs]
    c.close()
    srv = lib.Server(0, max_slots=4)
    tickets = [(i, srv.submit(S, prm)) for _ in range(2) for i, S in enumerate(reqs)]
    for i, t in tickets:
        r = srv.wait(t)
        a = single[i]
        assert r["status"] == 0 and a["status"] == 0
        assert r["cg_iters"] == a["cg_iters"], (i, r["cg_iters"], a["cg_iters"])
        assert abs(r["E_total"] - a["E_total"]) <= 1e-10 * max(1.0, abs(a["E_total"]))
        assert np.abs(r["forces"] - a["forces"]).max() <= 1e-10
        assert np.abs(r["u"] - a["u"]).max() <= 1e-10 * np.abs(a["u"]).max()
    srv.close()


def test_cluster_requests_same_alone_and_in_the_mix():
    # the serving stream's own sizes: fcc 1, 2 and 3 clusters (48^3, 63^3, 79^3 nodes),
    # FP32 stencil with FP64 refinement, overlapped with each other
    import paper_1405_6456_amd as lib

    reqs = [synth.fcc_cluster(m, seed=10000 + m, name=f"fcc{m}") for m in (1, 2, 3)]
    prm = lib.default_params(precision=lib.FP32_REFINED, initial_guess=lib.GUESS_ATOMIC)
    c = ctx()
    c.set_tuning(target_blocks=lib.SERVER_SLOT_BLOCKS)
    single = [c.solve(S, prm, None) for S in reqs]
    c.close()
    srv = lib.Server(0, max_slots=4)
    order = [2, 1, 0, 2, 1]
    tickets = [(i, srv.submit(reqs[i], prm)) for i in order]
    for i, t in tickets:
        r = srv.wait(t)
        a = single[i]
        assert r["status"] == 0 and a["status"] == 0
        assert abs(r["E_total"] - a["E_total"]) <= 1e-10 * max(1.0, abs(a["E_total"]))
        assert np.abs(r["forces"] - a["forces"]).max() <= 1e-10
        assert np.abs(r["u"] - a["u"]).max() <= 1e-10 * np.abs(a["u"]).max()
    srv.close()


def test_slot_launch_size_keeps_results_independent_of_the_mix():
    # with smaller stencil launches per slot (so the slots' kernels can share the device),
    # every served result still equals a standalone context with the same launch size; the
    # setting is refused while requests are queued or running
    import paper_1405_6456_amd as lib

    reqs = [synth.fcc_cluster(m, seed=10000 + m, name=f"fcc{m}") for m in (1, 2)]
    prm = lib.default_params(precision=lib.FP32_REFINED, initial_guess=lib.GUESS_ATOMIC)
    c = ctx()
    c.set_tuning(target_blocks=128)
    single = [c.solve(S, prm, None) for S in reqs]
    c.close()
    srv = lib.Server(0, max_slots=4)
    try:
        srv.set_tuning(128)
        tickets = [(i, srv.submit(S, prm)) for _ in range(2) for i, S in enumerate(reqs)]
        with pytest.raises(lib.AlofdftError):
            srv.set_tuning(0)
        for i, t in tickets:
            r = srv.wait(t)
            a = single[i]
            assert r["status"] == 0 and a["status"] == 0
            assert r["cg_iters"] == a["cg_iters"], (i, r["cg_iters"], a["cg_iters"])
            assert abs(r["E_total"] - a["E_total"]) <= 1e-10 * max(1.0, abs(a["E_total"]))
            assert np.abs(r["forces"] - a["forces"]).max() <= 1e-10
            assert np.abs(r["u"] - a["u"]).max() <= 1e-10 * np.abs(a["u"]).max()
    finally:
        srv.close()


def test_tight_budget_admits_every_request():
    # two small requests, then a larger one that fits the budget only alone: the idle
    # slots drop their cached arrays and every request completes
    import paper_1405_6456_amd as lib

    ctx().close()
    prm = lib.default_params(precision=lib.FP32_REFINED)
    small = synth.single_atom(L=16.0, n=21)
    big = synth.fcc_cluster(1, seed=10001, name="fcc1")
    fb = lib.footprint_bytes(big, prm)
    fs = lib.footprint_bytes(small, prm)
    assert fb + fs > fb * 1.1
    srv = lib.Server(0, hbm_budget_bytes=fb + fs // 2, max_slots=2)
    tickets = [srv.submit(small, prm), srv.submit(small, prm), srv.submit(big, prm)]
    t0 = time.time()
    for t in tickets:
        while srv.poll(t) is None:
            assert time.time() - t0 < 120, "a request was never admitted"
            time.sleep(0.005)
    st = srv.stats()
    assert st["completed"] == 3 and st["queued"] == 0
    srv.close()


def test_cancel_queued_and_running_requests():
    import paper_1405_6456_amd as lib

    ctx().close()
    prm = lib.default_params(precision=lib.FP64)
    S = synth.fcc_cluster(2, seed=10002, name="fcc2")
    srv = lib.Server(0, max_slots=1)
    t_run = srv.submit(S, prm)
    t_queued = srv.submit(S, prm)
    srv.cancel(t_queued)  # still queued behind the first
    r = srv.wait(t_queued)
    assert r["status"] == lib.CANCELLED
    time.sleep(0.3)  # the first is now running
    srv.cancel(t_run)
    r = srv.wait(t_run)
    assert r["status"] == lib.CANCELLED
    # the slot serves the next request normally
    t = srv.submit(synth.single_atom(L=16.0, n=21), prm)
    assert srv.wait(t)["status"] == 0
    st = srv.stats()
    assert st["cancelled"] == 2 and st["completed"] == 1
    srv.close()


def test_destroy_cancels_queued_requests():
    import paper_1405_6456_amd as lib

    ctx().close()
    prm = lib.default_params(precision=lib.FP64)
    S = synth.fcc_cluster(2, seed=10002, name="fcc2")
    srv = lib.Server(0, max_slots=1)
    for _ in range(6):
        srv.submit(S, prm)
    time.sleep(0.2)
    t0 = time.time()
    srv.close()  # one running request stops at its next check, five queued are cancelled
    assert time.time() - t0 < 5.0


def test_served_matches_fp64_path(alone):
    import paper_1405_6456_amd as lib

    c = ctx()
    for S, a in zip(requests(), alone):
        ref = c.solve(S, lib.default_params(precision=lib.FP64), None)
        assert abs(a["E_total"] - ref["E_total"]) / S.M <= 1e-5
        assert np.abs(a["forces"] - ref["forces"]).max() <= 1e-4
    c.close()


def test_admission_by_footprint():
    import paper_1405_6456_amd as lib

    ctx().close()
    reqs = requests()
    prm = lib.default_params(precision=lib.FP32_REFINED)
    fps = [lib.footprint_bytes(S, prm) for S in reqs]
    # a budget below the largest request rejects it; the rest still run, one at a time
    budget = max(fps) - 1
    srv = lib.Server(0, hbm_budget_bytes=budget, max_slots=4)
    with pytest.raises(lib.AlofdftError) as err:
        srv.submit(reqs[fps.index(max(fps))], prm)
    assert err.value.status == lib.REJECTED
    small = [S for S, f in zip(reqs, fps) if f <= budget]
    tickets = [srv.submit(S, prm) for S in small]
    peak = 0
    while True:
        st = srv.stats()
        peak = max(peak, st["hbm_reserved_bytes"])
        if st["completed"] == len(tickets):
            break
        time.sleep(0.002)
    assert peak <= budget
    for t in tickets:
        assert srv.wait(t)["status"] == 0
    st = srv.stats()
    assert st["rejected"] == 1 and st["completed"] == len(tickets)
    srv.close()


def test_invalid_requests_are_refused():
    import paper_1405_6456_amd as lib

    ctx().close()
    srv = lib.Server(0, max_slots=1)
    S = synth.single_atom(L=16.0, n=21)
    S.R[0] = [1.0, 8.0, 8.0]  # ball of radius 7 leaves the box
    with pytest.raises(lib.AlofdftError) as err:
        srv.submit(S, lib.default_params())
    assert err.value.status == lib.INVALID_ARGUMENT
    srv.close()
