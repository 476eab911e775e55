"""Scheduling logic of the shot server on a virtual clock (no GPU): overlap of calls admitted
while others run, admission by HBM footprint with backfill, batching of compatible requests,
failure isolation, and the latency percentiles."""
import numpy as np
import pytest

from paper_2311_02293_amd import inputs as I
from paper_2311_02293_amd.server import FakeBackend, Request, ShotServer, merge_requests


def tiny_job(name, nshot=1, n1=20, n2=30):
    g = I.Grid(ndim=2, n1=n1, n2=n2, nb=4, order=4, nt=10)
    vp = np.full((n2, n1), 2000.0, np.float32)
    sx = np.arange(nshot) * 10.0 + 50.0
    acq = I._surface_line(sx, 20.0, np.arange(n2) * 10.0, 20.0)
    stf = np.zeros((nshot, 10), np.float32)
    return I.Job(g, vp, vp.copy(), acq, stf, name=name)


def test_calls_overlap_and_queue_behind_busy_slots():
    be = FakeBackend(cost=lambda job, kind: 0.010)
    srv = ShotServer(be, budget_bytes=100, max_inflight=2)
    reqs = [Request("forward", tiny_job(f"j{k}"), arrival=0.0005 * k) for k in range(3)]
    out = srv.run(reqs)
    starts = {name: t for t, name, _ in be.launched}
    assert starts["j0"] == 0.0 and starts["j1"] == pytest.approx(0.0005)
    assert starts["j2"] == pytest.approx(0.010)           # waits for a free slot
    lat = [o.latency for o in out["outcomes"]]
    assert lat[0] == pytest.approx(0.010) and lat[1] == pytest.approx(0.010)
    assert lat[2] == pytest.approx(0.020 - 0.001)
    assert out["p50"] == pytest.approx(np.percentile(lat, 50))
    assert out["p99"] == pytest.approx(np.percentile(lat, 99))


def test_admission_by_footprint_with_backfill():
    fp = {"big0": 6, "big1": 6, "small": 3}
    be = FakeBackend(cost=lambda job, kind: 0.010, footprint=lambda job, kind: fp[job.name])
    srv = ShotServer(be, budget_bytes=10, max_inflight=4)
    reqs = [Request("forward", tiny_job("big0"), 0.0), Request("forward", tiny_job("big1"), 0.001),
            Request("forward", tiny_job("small"), 0.002)]
    srv.run(reqs)
    starts = {name: t for t, name, _ in be.launched}
    assert starts["big0"] == 0.0
    assert starts["small"] == pytest.approx(0.002)         # passes big1, which does not fit yet
    assert starts["big1"] == pytest.approx(0.010)


def test_compatible_requests_are_batched_into_one_call():
    be = FakeBackend(cost=lambda job, kind: 0.001 * job.acq.nshot)
    srv = ShotServer(be, budget_bytes=100, max_inflight=1)
    reqs = [Request("forward", tiny_job("a"), 0.0, model_key="m1")]
    reqs += [Request("forward", tiny_job(f"b{k}"), 0.0001, model_key="m1") for k in range(3)]
    reqs += [Request("forward", tiny_job("c"), 0.0001, model_key="m2")]
    out = srv.run(reqs)
    names = [name for _, name, _ in be.launched]
    assert names[0] == "a"
    assert "b0+b1+b2" in names                      # merged while "a" ran
    assert all(o.ok for o in out["outcomes"])
    assert [o.batch for o in out["outcomes"]][1:4] == [3, 3, 3]


def test_merge_keeps_every_shot_and_receiver():
    a, b = tiny_job("a", nshot=2), tiny_job("b", nshot=1)
    m = merge_requests([Request("forward", a, model_key="k"), Request("forward", b, model_key="k")])
    assert m.acq.nshot == 3
    assert list(m.acq.rec_off) == [0, 30, 60, 90]
    np.testing.assert_array_equal(m.stf, np.concatenate([a.stf, b.stf]))


def test_a_failing_request_fails_alone():
    be = FakeBackend(cost=lambda job, kind: 0.002, fail=lambda job, kind: job.name == "bad")
    srv = ShotServer(be, budget_bytes=100, max_inflight=2)
    reqs = [Request("forward", tiny_job(n), 0.0001 * k) for k, n in enumerate(["x", "bad", "y"])]
    out = srv.run(reqs)
    ok = {o.rid: o.ok for o in out["outcomes"]}
    assert ok == {0: True, 1: False, 2: True}
    assert out["failed"] == 1
    assert "injected" in out["outcomes"][1].error


def test_request_above_the_budget_is_rejected():
    be = FakeBackend(footprint=lambda job, kind: 50)
    srv = ShotServer(be, budget_bytes=10, max_inflight=2)
    out = srv.run([Request("forward", tiny_job("huge"), 0.0)])
    assert not out["outcomes"][0].ok and "budget" in out["outcomes"][0].error


def test_members_of_a_merged_call_get_their_own_shots():
    """Each member of a merged call gets the result of its own shots: the backend is told the
    request boundaries, and the server hands request k the k-th part."""
    be = FakeBackend(cost=lambda job, kind: 0.001 * job.acq.nshot)
    srv = ShotServer(be, budget_bytes=100, max_inflight=1)
    reqs = [Request("grad", tiny_job("a"), 0.0, model_key="m", dobs=np.zeros(1))]
    reqs += [Request("grad", tiny_job(f"b{k}", nshot=k + 1), 0.0001, model_key="m",
                     dobs=np.zeros(1)) for k in range(3)]
    out = srv.run(reqs)
    assert out["outcomes"][0].result == ("a", 0, 1)
    ranges = [o.result[1:] for o in out["outcomes"][1:]]
    assert ranges == [(0, 1), (1, 3), (3, 6)]
    assert {o.result[0] for o in out["outcomes"][1:]} == {"b0+b1+b2"}
    assert out["calls"] == 2 and out["merged_calls"] == 1
    assert out["requests_per_call"] == 2.0


def test_survey_pool_stream_shares_models_across_requests():
    jobs = I.stream_config5(njobs=40, rate=10.0, seed=7, scale=0.05, pool=3)
    keys = [sj.model_key for sj in jobs]
    assert all(k is not None for k in keys)
    assert len(set(keys)) < len(keys)               # several requests per survey
    by = {}
    for sj in jobs:
        by.setdefault(sj.model_key, []).append(sj)
    for key, grp in by.items():
        cls = key.rsplit("-", 1)[0]
        assert all(sj.kind == cls for sj in grp)
        g0 = grp[0].job
        for sj in grp[1:]:
            assert sj.job.grid is g0.grid and sj.job.vp is g0.vp and sj.job.rho is g0.rho
            np.testing.assert_array_equal(sj.job.stf, g0.stf)
        assert all(sj.job.acq.nshot == 1 for sj in grp)
    # the same seed gives the same stream; pool=0 keeps one model per request
    again = I.stream_config5(njobs=40, rate=10.0, seed=7, scale=0.05, pool=3)
    assert [(a.arrival, a.model_key, tuple(a.job.acq.src[0])) for a in jobs] == \
           [(b.arrival, b.model_key, tuple(b.job.acq.src[0])) for b in again]
    solo = I.stream_config5(njobs=10, rate=10.0, seed=7, scale=0.05)
    assert all(sj.model_key is None for sj in solo)
