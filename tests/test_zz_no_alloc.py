"""The allocation-free LSRK step (esdg_lsrk_step_noalloc) against the
ordinary step (esdg_lsrk_step) through the C ABI: two calls in a row on the
library's per-device scratch array, the second on a smaller mesh, each
bitwise equal to the ordinary step on the same input; a mesh whose state
exceeds the array is rejected before any work is enqueued."""
import pytest

from paper_2605_16684_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NOALLOC_MAX_DOUBLES = 1 << 23


def _esdg():
    from paper_2605_16684_amd import esdg
    return esdg


def _both_steps(spec, kind, seed, nsteps):
    esdg = _esdg()
    m = esdg.Mesh(spec)
    assert m.state_len <= NOALLOC_MAX_DOUBLES
    q0 = W.make_state(kind, m.coords(), spec, seed=seed).contiguous()
    dt = m.cfl_dt(q0, 0.5)
    qa, dqa = q0.clone(), torch.zeros_like(q0)
    qb, dqb = q0.clone(), torch.full_like(q0, float("nan"))  # dq's contents must not matter
    for _ in range(nsteps):
        m.lsrk_step(qa, dqa, dt)
        m.lsrk_step_noalloc(qb, dqb, dt)
    torch.cuda.synchronize()
    m.check()
    print(f"[noalloc {kind} N={spec.N} K={spec.K}] state_len={m.state_len} "
          f"max|dq|={float(dqa.abs().max()):.3e}", flush=True)
    assert not torch.equal(qa, q0)
    assert torch.equal(qa, qb)
    assert torch.equal(dqa, dqb)
    m.close()


def test_noalloc_step_matches_lsrk_step_twice_in_a_row_shrinking():
    big = W.MeshSpec(4, (8, 4, 3), (0.0, 0.0, 0.0), (4.0e7 / 20, 6.0e6, 3.0e4), (1, 0, 0),
                     coriolis_f=1e-4)
    _both_steps(big, "channel", 3, 3)
    small = W.MeshSpec(3, (3, 3, 2), (0.0, 0.0, 0.0), (1000.0, 1000.0, 1000.0), (1, 1, 0))
    _both_steps(small, "iso_pert", 4, 2)


def test_noalloc_step_rejects_a_state_beyond_the_scratch():
    esdg = _esdg()
    spec = W.MeshSpec(7, (16, 16, 16), (0.0, 0.0, 0.0), (1000.0, 1000.0, 1000.0), (0, 0, 0))
    m = esdg.Mesh(spec)
    assert m.state_len > NOALLOC_MAX_DOUBLES
    q = torch.ones(m.shape, dtype=torch.float64, device="cuda")
    dq = torch.zeros_like(q)
    with pytest.raises(esdg.EsdgError) as ei:
        m.lsrk_step_noalloc(q, dq, 1e-3)
    assert ei.value.code == esdg.ESDG_EINVAL
    assert "exceeds" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((q == 1.0).all()) and bool((dq == 0.0).all())
    m.close()
