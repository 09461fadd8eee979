"""Checkpoint files: a CPU round trip of the integrator state and mesh
description, rejection of a mismatched state, and (GPU) a run resumed from a
checkpoint in a fresh mesh that reproduces the uninterrupted run bit for
bit."""
import numpy as np
import pytest

from paper_2605_16684_amd import checkpoint as CK
from paper_2605_16684_amd import workloads as W


def test_round_trip_on_the_host(tmp_path):
    spec = W.MeshSpec(3, (2, 3, 2), (0.0, 0.0, 0.0), (900.0, 700.0, 1100.0), (1, 0, 0),
                      coriolis_f=1e-4, surface_flux=2, warp=(0.05, 0.04, 0.03))
    rng = np.random.default_rng(7)
    q = rng.standard_normal((12, 5, 64))
    dq = rng.standard_normal((12, 5, 64))
    rr, pr = rng.random((12, 64)), rng.random((12, 64))
    p = str(tmp_path / "ck.npz")
    CK.save(p, spec, q, dq, t=1.25, step=17, dt=3e-3, precision=1, ref_rho=rr, ref_p=pr)
    ck = CK.load(p)
    assert ck.spec == spec
    assert (ck.t, ck.step, ck.dt, ck.precision) == (1.25, 17, 3e-3, 1)
    assert np.array_equal(ck.q, q) and np.array_equal(ck.dq, dq)
    assert np.array_equal(ck.ref_rho, rr) and np.array_equal(ck.ref_p, pr)


def test_mismatched_state_is_rejected(tmp_path):
    spec = W.MeshSpec(2, (2, 2, 2), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (1, 1, 0))
    p = str(tmp_path / "bad.npz")
    CK.save(p, spec, np.zeros((8, 5, 8)), np.zeros((8, 5, 8)), 0.0, 0, 1e-3)
    with pytest.raises(ValueError):
        CK.load(p)


@pytest.mark.gpu
def test_resumed_run_is_bitwise_the_uninterrupted_run(tmp_path):
    torch = pytest.importorskip("torch")
    from paper_2605_16684_amd import esdg
    spec = W.MeshSpec(4, (6, 4, 3), (0.0, 0.0, 0.0), (2.0e6, 6.0e6, 3.0e4), (1, 0, 0),
                      coriolis_f=1e-4)
    m = esdg.Mesh(spec)
    q0 = W.make_state("channel", m.coords(), spec, seed=2).contiguous()
    dt = m.cfl_dt(q0, 0.5)
    qa, dqa = q0.clone(), torch.zeros_like(q0)
    m.lsrk_run(qa, dqa, dt, 12)
    qb, dqb = q0.clone(), torch.zeros_like(q0)
    m.lsrk_run(qb, dqb, dt, 5)
    torch.cuda.synchronize()
    p = str(tmp_path / "run.npz")
    CK.save(p, spec, qb, dqb, t=5 * dt, step=5, dt=dt)
    m.close()
    ck = CK.load(p)
    m2 = esdg.Mesh(ck.spec)
    qc = torch.from_numpy(ck.q).cuda()
    dqc = torch.from_numpy(ck.dq).cuda()
    m2.lsrk_run(qc, dqc, ck.dt, 12 - ck.step, t0=ck.t)
    torch.cuda.synchronize()
    m2.check()
    assert torch.equal(qc, qa)
    m2.close()
