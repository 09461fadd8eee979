"""Scheduler of the ensemble server on the CPU fake executor: admission by
HBM footprint (with backfill), continuous batching, eviction, statistics,
failure isolation."""
import numpy as np
import pytest

from paper_2605_16684_amd import serving as S


def _reqs(n=12, seed=1, steps=5, mean=1e-3):
    return S.request_stream(n=n, seed=seed, mean_interarrival=mean, steps=steps, kmin=2, kmax=6)


def test_request_stream_shape():
    rs = S.request_stream(n=400, seed=3, mean_interarrival=0.02)
    assert len(rs) == 400
    assert all(8 <= k <= 40 for r in rs for k in r.K)
    assert {r.N for r in rs} == {3, 4, 5, 7}
    assert {r.precision for r in rs} == {S.FP64, S.FP32_MIXED}
    assert {r.kind for r in rs} == {"bubble", "channel"}
    gaps = np.diff([0.0] + [r.arrival for r in rs])
    assert abs(gaps.mean() - 0.02) < 0.004          # Poisson arrivals, mean 0.02 s
    assert [r.seed for r in rs] == list(range(400))
    assert S.request_stream(n=5, seed=3) == S.request_stream(n=5, seed=3)


def test_all_requests_complete_and_budget_holds():
    rs = _reqs()
    budget = int(2.5 * max(S.footprint_bytes(r) for r in rs))
    srv = S.Server(budget, executor=S.FakeExecutor())
    st = srv.run(rs, realtime=False)
    assert st.n_completed == len(rs) and st.n_rejected == 0
    assert st.peak_footprint_bytes <= budget
    for r in rs:
        mb = srv.members[r.rid]
        assert mb.steps_done == r.steps and len(mb.latencies) == r.steps
        assert all(x > 0 for x in mb.latencies)
        assert mb.admitted >= r.arrival - 1e-12


def test_admission_binds_and_members_overlap():
    rs = _reqs(n=20, mean=1e-5)                       # burst: everyone arrives at once
    total = sum(S.footprint_bytes(r) for r in rs)
    srv = S.Server(total // 3, executor=S.FakeExecutor())
    st = srv.run(rs, realtime=False)
    assert st.n_completed == 20
    assert 1 < st.max_concurrent_members < 20         # batched, but not all at once
    assert st.queue_wait_p99_ms > 0
    # several (N, precision) buckets ran side by side
    assert st.buckets_seen >= 2


def test_backfill_small_requests_pass_a_blocked_large_one():
    big = S.Request(0, "bubble", (7, 7, 7), 7, S.FP64, 0, 3, 0.0)
    small = [S.Request(i, "bubble", (2, 2, 2), 3, S.FP64, i, 3, 1e-6 * i) for i in range(1, 5)]
    blocker = S.Request(9, "channel", (8, 8, 7), 7, S.FP64, 9, 40, 0.0)
    budget = S.footprint_bytes(blocker) + S.footprint_bytes(small[0]) * 4 + 1
    srv = S.Server(budget, executor=S.FakeExecutor())
    srv.run([blocker, big] + small, realtime=False)
    # the small requests were admitted while the big one still waited for the blocker
    assert max(srv.members[r.rid].admitted for r in small) < srv.members[0].admitted


def test_requests_larger_than_budget_are_rejected_not_hung():
    rs = _reqs(n=4)
    huge = S.Request(99, "bubble", (40, 40, 40), 7, S.FP64, 99, 2, 0.0)
    budget = 4 * max(S.footprint_bytes(r) for r in rs)
    st = S.Server(budget, executor=S.FakeExecutor()).run(rs + [huge], realtime=False)
    assert st.n_rejected == 1 and st.n_completed == 4


def test_requests_above_the_packable_order_are_rejected():
    rs = _reqs(n=4)
    high = S.Request(98, "bubble", (2, 2, 2), S.PACK_MAX_N + 1, S.FP64, 98, 2, 0.0)
    budget = 100 * max(S.footprint_bytes(r) for r in rs + [high])
    st = S.Server(budget, executor=S.FakeExecutor()).run(rs + [high], realtime=False)
    assert st.n_rejected == 1 and st.n_completed == 4


def test_failure_isolation():
    rs = _reqs(n=8)
    ex = S.FakeExecutor(fail_on={3})
    srv = S.Server(10 * max(S.footprint_bytes(r) for r in rs), executor=ex)
    st = srv.run(rs, realtime=False)
    assert st.n_rejected == 1 and st.n_completed == 7
    assert 3 not in srv.members


def test_nonphysical_member_is_evicted_and_others_complete():
    rs = _reqs(n=8, steps=6)
    ex = S.FakeExecutor(nonphysical_on={2: 3})      # request 2 goes bad in its third step
    srv = S.Server(10 * max(S.footprint_bytes(r) for r in rs), executor=ex)
    handles = {r.rid: S.RequestHandle(srv, r) for r in rs}
    st = srv.run(rs, realtime=False)
    assert st.n_failed == 1 and st.n_completed == 7 and st.n_rejected == 0
    h = handles[2]
    assert h.done() and isinstance(h.error(), S.NonPhysicalState)
    with pytest.raises(S.NonPhysicalState):
        h.result()
    assert srv.members[2].steps_done == 2            # evicted after its third step
    for r in rs:
        if r.rid != 2:
            assert handles[r.rid].error() is None
            assert srv.members[r.rid].steps_done == r.steps
    # its memory returned to the budget: nothing is left resident
    assert all(mb.handle is None or mb.error is None for mb in srv.members.values())


def test_statistics_are_computed_from_member_steps():
    rs = _reqs(n=6, steps=4)
    srv = S.Server(10 * max(S.footprint_bytes(r) for r in rs), executor=S.FakeExecutor())
    st = srv.run(rs, realtime=False)
    lat = np.array([x for r in rs for x in srv.members[r.rid].latencies])
    assert st.step_latency_p50_ms == pytest.approx(np.percentile(lat, 50) * 1e3)
    assert st.step_latency_p99_ms == pytest.approx(np.percentile(lat, 99) * 1e3)
    work = sum(r.nodes * 5 * r.steps for r in rs)
    assert st.aggregate_dof_rhs_per_s == pytest.approx(work / st.makespan_s)
    # fake cost model: a lone member's step latency is overhead + nodes * cost
    ex = S.FakeExecutor()
    one = S.Request(0, "bubble", (3, 3, 3), 4, S.FP64, 0, 3, 0.0)
    srv1 = S.Server(10 * S.footprint_bytes(one), executor=ex)
    srv1.run([one], realtime=False)
    lats = srv1.members[0].latencies
    assert lats[1] == pytest.approx(ex.overhead + one.nodes * ex.cost(4, S.FP64))


def test_buckets_advance_independently():
    # a bucket of one small member steps at its own pace next to a bucket of
    # a large member: its step latency is set by its own work (the device is
    # shared), not by the large member's step
    big = S.Request(0, "channel", (12, 12, 12), 7, S.FP64, 0, 4, 0.0)
    small = S.Request(1, "bubble", (2, 2, 2), 3, S.FP64, 1, 20, 0.0)
    ex = S.FakeExecutor()
    srv = S.Server(10 * (S.footprint_bytes(big) + S.footprint_bytes(small)), executor=ex)
    st = srv.run([big, small], realtime=False)
    assert st.n_completed == 2
    t_big = ex.overhead + big.nodes * ex.cost(7, S.FP64)
    t_small = ex.overhead + small.nodes * ex.cost(3, S.FP64)
    lat_small = srv.members[1].latencies[1:]
    assert max(lat_small) <= 2 * t_small + 1e-12       # shares the device with one other step
    assert max(lat_small) < 0.1 * t_big
    assert srv.members[1].finished < srv.members[0].finished
    assert st.bucket_steps == big.steps + small.steps


def test_submit_and_run_until_idle():
    rs = _reqs(n=5, steps=3)
    srv = S.Server(10 * max(S.footprint_bytes(r) for r in rs), executor=S.FakeExecutor())
    handles = [srv.submit(r) for r in rs]
    with pytest.raises(ValueError):
        srv.submit(rs[0])
    assert not any(h.done() for h in handles)
    with pytest.raises(RuntimeError):
        handles[0].result()
    st = srv.run_until_idle(realtime=False)
    assert st.n_completed == 5 and srv.stats()["n_completed"] == 5
    for h in handles:
        assert h.done()
        hs = h.stats()
        assert hs["steps"] == 3 and hs["e2e_latency_s"] >= hs["queue_wait_s"] >= 0
        assert hs["step_latency_p99_ms"] >= hs["step_latency_p50_ms"] > 0


def test_footprint_formula():
    r = S.Request(0, "bubble", (10, 10, 10), 4, S.FP64, 0, 1)
    assert S.footprint_bytes(r) >= 120 * r.nodes
    rm = S.Request(0, "bubble", (10, 10, 10), 4, S.FP32_MIXED, 0, 1)
    assert S.footprint_bytes(rm) - S.footprint_bytes(r) == 20 * r.nodes


def test_released_members_memory_is_counted_until_flushed():
    # released members keep part of their device memory (their meshes) until
    # the executor destroys them in a batch: admission must count it and
    # flush when a request would not fit otherwise
    reqs = S.request_stream(n=40, seed=5, mean_interarrival=1e-4, steps=3, kmin=2, kmax=8)
    budget = max(int(0.3 * sum(S.footprint_bytes(r) for r in reqs)),
                 max(S.footprint_bytes(r) for r in reqs))
    ex = S.FakeExecutor(retire_fraction=0.5)
    st = S.Server(budget, executor=ex).run(reqs, realtime=False)
    assert st.n_completed == len(reqs)
    assert ex.flushes >= 1
    assert ex.peak_bytes <= budget
    assert ex.retired == 0            # everything flushed at the end
