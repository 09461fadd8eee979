"""Ensemble serving on the GPU: packed launches reproduce single-mesh
stepping bit for bit, every request's result is the same alone and in the
mix (FP64 and FP32-mixed members; bitwise, the tolerance is 0), a member
that goes non-physical is evicted alone, and the pack's member table grows
and shrinks without changing any member's result."""
import numpy as np
import pytest

from paper_2605_16684_amd import serving as S
from paper_2605_16684_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_packed_steps_equal_single_mesh_steps():
    from paper_2605_16684_amd import esdg
    reqs = [S.Request(0, "bubble", (3, 2, 4), 4, S.FP64, 1, 3),
            S.Request(1, "channel", (5, 3, 2), 4, S.FP64, 2, 3),
            S.Request(2, "bubble", (2, 2, 2), 4, S.FP64, 3, 3)]
    members, ref = [], []
    for r in reqs:
        m, q, _ = S._make_member_mesh(r)
        dt = m.cfl_dt(q, 0.5)
        members.append((m, q.clone(), torch.empty_like(q), torch.zeros_like(q), dt))
        qa, dqa = q.clone(), torch.zeros_like(q)
        for _ in range(3):
            m.lsrk_step(qa, dqa, dt)
        ref.append(qa)
    pack = esdg.Pack()
    pack.set_members([x[0] for x in members], [x[1] for x in members], [x[2] for x in members],
                     [x[3] for x in members], [x[4] for x in members], [0, 0, 0])
    pack.step(3)
    torch.cuda.synchronize()
    for (m, q0, q1, dq, dt), qa in zip(members, ref):
        assert torch.equal(q1, qa)        # 3 steps: state is in buffer 0 ^ 1
    pack.close()


def test_alone_and_in_the_mix_give_identical_results(tmp_path):
    tuner = S.Autotuner(str(tmp_path / "epw.json"), target_nodes=1.5e5)
    # a burst (all arrive within microseconds) under a budget of half the
    # total footprint; enough steps that members prepared one after the other
    # on the admission thread overlap on the device
    reqs = S.request_stream(n=8, seed=7, mean_interarrival=1e-6, steps=100, kmin=2, kmax=5,
                            orders=(3, 4))
    budget = int(0.5 * sum(S.footprint_bytes(r) for r in reqs))
    budget = max(budget, max(S.footprint_bytes(r) for r in reqs))
    ex = S.GpuExecutor(tuner, keep_results=True)
    srv = S.Server(budget, executor=ex)
    st = srv.run(reqs)
    print("[serving mix]", st.as_dict(), flush=True)
    assert st.n_completed == len(reqs)
    assert st.max_concurrent_members > 1
    for r in reqs:
        alone = S.Server(10 * S.footprint_bytes(r), executor=S.GpuExecutor(tuner, keep_results=True))
        h = alone.submit(S.Request(r.rid, r.kind, r.K, r.N, r.precision, r.seed, r.steps, 0.0))
        alone.run_until_idle()
        a, b = srv.results[r.rid], h.result()
        assert a.shape == b.shape
        assert np.array_equal(a, b), (r, np.abs(a - b).max())
        assert np.all(np.isfinite(a))


def test_autotuner_caches_a_compiled_choice(tmp_path):
    from paper_2605_16684_amd import esdg
    path = tmp_path / "t.json"
    t = S.Autotuner(str(path), target_nodes=1e5)
    e = t.epw(4, S.FP64)
    assert e in esdg.epw_options(4, S.FP64)
    t2 = S.Autotuner(str(path))
    assert t2.table["N4_fp64"]["epw"] == e


def test_nonphysical_member_fails_alone_in_a_mix(tmp_path):
    """One member of a mixed stream starts with a negative density at one
    node: that request fails with NonPhysicalState, every other request ends
    bitwise equal to its solo run."""
    tuner = S.Autotuner(str(tmp_path / "epw.json"), target_nodes=1.5e5)
    # enough steps that members prepared one after the other on the
    # admission thread still overlap on the device
    reqs = S.request_stream(n=6, seed=11, mean_interarrival=1e-6, steps=100, kmin=2, kmax=4,
                            orders=(3, 4))
    bad = reqs[2]
    reqs[2] = S.Request(bad.rid, bad.kind, bad.K, bad.N, bad.precision, bad.seed, bad.steps,
                        bad.arrival, nonphysical_node=7)
    ex = S.GpuExecutor(tuner, keep_results=True)
    srv = S.Server(10 * sum(S.footprint_bytes(r) for r in reqs), executor=ex)
    handles = [srv.submit(r) for r in reqs]
    st = srv.run_until_idle()
    print("[serving nonphysical]", st.as_dict(), flush=True)
    assert st.n_failed == 1 and st.n_completed == len(reqs) - 1
    assert st.max_concurrent_members > 1
    assert isinstance(handles[2].error(), S.NonPhysicalState)
    with pytest.raises(S.NonPhysicalState):
        handles[2].result()
    for r, h in zip(reqs, handles):
        if r.rid == bad.rid:
            continue
        alone = S.Server(10 * S.footprint_bytes(r), executor=S.GpuExecutor(tuner, keep_results=True))
        ha = alone.submit(S.Request(r.rid, r.kind, r.K, r.N, r.precision, r.seed, r.steps, 0.0))
        alone.run_until_idle()
        a, b = h.result(), ha.result()
        assert np.array_equal(a, b), (r, np.abs(a - b).max())
        assert np.all(np.isfinite(a))


def test_pack_table_grows_and_shrinks():
    """Member sets of 1, 3, 2 and 5 meshes in a row (the device table grows
    geometrically and is reused when it shrinks): every member's two steps
    equal its single-mesh steps bit for bit, and the flags read clean."""
    from paper_2605_16684_amd import esdg
    reqs = [S.Request(i, "bubble" if i % 2 else "channel", (2 + i % 3, 2, 2), 3, S.FP64, i, 2)
            for i in range(5)]
    built = []
    for r in reqs:
        m, q, _ = S._make_member_mesh(r)
        dt = m.cfl_dt(q, 0.5)
        qa, dqa = q.clone(), torch.zeros_like(q)
        for _ in range(2):
            m.lsrk_step(qa, dqa, dt)
        built.append((m, q, dt, qa))
    pack = esdg.Pack()
    for sel in ([0], [0, 1, 2], [3, 4], [0, 1, 2, 3, 4]):
        bufs = [(built[i][1].clone(), torch.empty_like(built[i][1]), torch.zeros_like(built[i][1]))
                for i in sel]
        pack.set_members([built[i][0] for i in sel], [b[0] for b in bufs], [b[1] for b in bufs],
                         [b[2] for b in bufs], [built[i][2] for i in sel], [0] * len(sel))
        pack.step(2)
        torch.cuda.synchronize()
        assert pack.flags() == [False] * len(sel)
        for i, b in zip(sel, bufs):
            assert torch.equal(b[0], built[i][3]), (sel, i)   # 2 steps: back in buffer 0
    pack.close()


def test_async_flag_gathering_matches_the_synchronous_read():
    from paper_2605_16684_amd import esdg
    reqs = [S.Request(0, "bubble", (2, 2, 2), 4, S.FP64, 1, 1),
            S.Request(1, "bubble", (3, 2, 2), 4, S.FP64, 2, 1),
            S.Request(2, "bubble", (2, 3, 2), 4, S.FP64, 3, 1)]
    members = []
    for r in reqs:
        m, q, _ = S._make_member_mesh(r)
        dt = m.cfl_dt(q, 0.5)
        members.append((m, q, torch.empty_like(q), torch.zeros_like(q), dt))
    members[1][1][3, 0, 7] = -1.0   # one node of member 1 with rho < 0
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())  # the states were written there
    pack = esdg.Pack(stream)
    pack.set_members([x[0] for x in members], [x[1] for x in members], [x[2] for x in members],
                     [x[3] for x in members], [x[4] for x in members], [0, 0, 0])
    host = torch.full((8,), -7, dtype=torch.int32, pin_memory=True)
    with torch.cuda.stream(stream):
        pack.step(1)
        pack.flags_async(host)
        ev = torch.cuda.Event()
        ev.record(stream)
    ev.synchronize()
    got = [bool(x) for x in host[:3].tolist()]
    assert got == [False, True, False]
    assert host[3:].tolist() == [-7] * 5          # nothing written beyond n
    assert pack.flags() == [False, False, False]  # the async read cleared them
    with pytest.raises(ValueError):
        pack.flags_async(torch.zeros(2, dtype=torch.int32, pin_memory=True))
    pack.close()
