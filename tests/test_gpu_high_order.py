"""Parity of the high-order path (N = 9..15, node-per-thread kernels: the
element in LDS with the logarithms up to N = 12 and without them at N = 13,
14, the prim buffer at N = 15) with the CPU oracle, through the C ABI.

Same bars as the fused path (tests/_parity.py): per conserved variable the
RHS error is at most 2e-14 of the gross term scale and max(1e-12, 64 eps
kappa) of the RHS; the state after n LSRK(5,4) steps is within
max(1e-10, eps kappa_s / sqrt(5 n)).  The meshes are small (one to four
elements) but every order from 9 to 15 is covered, with walls and periodic
faces, the three surface fluxes and Coriolis.
"""
import numpy as np
import pytest

import oracle as O
from paper_2605_16684_amd import workloads as W
from tests._parity import check_rhs, check_state

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

_BOX = ((0, 0, 0), (900.0, 700.0, 1100.0))


def _esdg():
    from paper_2605_16684_amd import esdg
    return esdg


def _oracle_mesh(spec):
    return O.Mesh(spec.N, spec.K, spec.lo, spec.hi, spec.periodic, gamma=spec.gamma,
                  gas_R=spec.gas_R, grav=spec.grav, coriolis_f=spec.coriolis_f,
                  surface_flux=spec.surface_flux)


def _with_jumps(q, seed):
    rng = np.random.default_rng(seed)
    q = q.copy()
    q *= (1.0 + 0.02 * rng.uniform(-1, 1, size=q[:, 0].shape))[:, None, :]
    q[:, 1:4] += 5.0 * q[:, 0:1] * rng.uniform(-1, 1, size=q[:, 1:4].shape)
    return q


CASES = [
    # name, N, K, periodic, coriolis_f, surface flux
    ("N9_walls_rusanov", 9, (2, 1, 2), (0, 0, 0), 0.0, 0),
    ("N10_periodic_x_matrix", 10, (2, 1, 1), (1, 0, 0), 1e-4, 2),
    ("N11_ec", 11, (1, 2, 1), (0, 1, 0), 0.0, 1),
    ("N12_matrix", 12, (1, 1, 2), (1, 1, 0), 1e-4, 2),
    ("N13_rusanov", 13, (1, 1, 1), (0, 0, 0), 1e-4, 0),
    ("N14_no_gravity_periodic", 14, (1, 1, 2), (1, 1, 1), 0.0, 2),
    ("N15_matrix", 15, (1, 1, 2), (1, 0, 0), 1e-4, 2),
]


@pytest.mark.parametrize("name,N,K,periodic,f,surf", CASES, ids=[c[0] for c in CASES])
def test_high_order_rhs_parity(name, N, K, periodic, f, surf):
    esdg = _esdg()
    # a z-periodic box has no gravity (the geopotential g z is not periodic)
    grav = 0.0 if periodic[2] else W.MeshSpec.grav
    spec = W.MeshSpec(N, K, *_BOX, periodic, coriolis_f=f, surface_flux=surf, grav=grav)
    om = _oracle_mesh(spec)
    q = W.make_state("iso_pert", om.coords(), spec, seed=N)
    m = esdg.Mesh(spec)
    assert m.epw == 0
    for tag, qq in (("smooth", q), ("jumps", _with_jumps(q, N))):
        r_or, g = om.rhs(qq, gross=True)
        r = m.rhs(torch.from_numpy(qq).cuda()).cpu().numpy()
        check_rhs(f"{name} {tag}", r, r_or, g)
    m.check()


@pytest.mark.parametrize("mask", [1, 2, 4, 3, 5, 6])
def test_high_order_term_split_parity(mask):
    esdg = _esdg()
    spec = W.MeshSpec(10, (2, 1, 2), *_BOX, (1, 0, 0), coriolis_f=1e-4, surface_flux=2)
    om = _oracle_mesh(spec)
    q = _with_jumps(W.state_iso_pert(om.coords(), spec, seed=3), 3)
    r_or, _ = om.rhs(q, mask=mask, gross=True)
    _, g = om.rhs(q, gross=True)
    m = esdg.Mesh(spec)
    r = m.rhs_terms(torch.from_numpy(q).cuda(), mask).cpu().numpy()
    check_rhs(f"N10 mask{mask}", r, r_or, g)


@pytest.mark.parametrize("N,K,kind", [(9, (2, 2, 2), "bubble"), (12, (2, 1, 2), "iso_pert"),
                                      (13, (1, 1, 2), "iso_pert"), (14, (1, 1, 2), "bubble"),
                                      (15, (1, 1, 2), "iso_pert")])
def test_high_order_lsrk_steps_parity(N, K, kind):
    """Ten LSRK steps (eager, dq starting as NaN) and the graph-replayed run
    of the same steps, which must give the same bits."""
    esdg = _esdg()
    if kind == "bubble":
        spec = W.rising_bubble(N=N, K=K).mesh
    else:
        spec = W.MeshSpec(N, K, *_BOX, (1, 0, 0), coriolis_f=1e-4, surface_flux=2)
    om = _oracle_mesh(spec)
    q0 = W.make_state(kind, om.coords(), spec, seed=7)
    dt = om.cfl_dt(q0, 0.25)  # CFL 0.5 is unstable at high orders
    n = 10
    q_or = om.run(q0, dt, n)
    _, g0 = om.rhs(q0, gross=True)
    m = esdg.Mesh(spec)
    qe = torch.from_numpy(q0).cuda()
    dqe = torch.full_like(qe, float("nan"))
    for _ in range(n):
        m.lsrk_step(qe, dqe, dt)
    m.check()
    check_state(f"N{N} {kind} {n} steps", qe.cpu().numpy(), q_or, g0, n * dt, n)
    qg = torch.from_numpy(q0).cuda()
    dqg = torch.zeros_like(qg)
    m.lsrk_run(qg, dqg, dt, n)
    assert torch.equal(qg, qe)


def test_high_order_conservation_over_steps():
    """Periodic in x and y, walls in z: mass and total energy (with the
    geopotential) stay constant to rounding over 20 steps."""
    esdg = _esdg()
    spec = W.MeshSpec(11, (2, 2, 1), *_BOX, (1, 1, 0), coriolis_f=1e-4, surface_flux=2)
    om = _oracle_mesh(spec)
    q0 = _with_jumps(W.state_iso_pert(om.coords(), spec, seed=9), 9)
    dt = om.cfl_dt(q0, 0.25)  # CFL 0.5 is unstable at high orders
    m = esdg.Mesh(spec)
    qg = torch.from_numpy(q0).cuda()
    dq = torch.zeros_like(qg)
    e0 = m.entropy(qg)
    m.lsrk_run(qg, dq, dt, 20)
    e1 = m.entropy(qg)
    dm, de = abs(e1[1] - e0[1]) / e0[1], abs(e1[2] - e0[2]) / e0[2]
    print(f"[N11 conservation] mass {dm:.2e} energy {de:.2e}", flush=True)
    assert dm <= 1e-14 and de <= 1e-14


def test_high_order_nonphysical_state_is_reported():
    esdg = _esdg()
    spec = W.MeshSpec(9, (1, 1, 2), *_BOX, (0, 0, 0))
    om = _oracle_mesh(spec)
    q = W.state_iso_pert(om.coords(), spec, seed=1)
    q[1, 0, 17] = -1.0
    m = esdg.Mesh(spec)
    m.rhs(torch.from_numpy(q).cuda())
    with pytest.raises(esdg.NonPhysicalState):
        m.check()
    m.check()  # flag cleared


@pytest.mark.parametrize("N", [10, 14])
def test_high_order_diagnostics_match_oracle(N):
    """Entropy, mass and energy integrals, the entropy production and the CFL
    step at orders whose node loops run to 11-15 nodes per direction."""
    esdg = _esdg()
    spec = W.MeshSpec(N, (2, 1, 2), *_BOX, (1, 0, 0), coriolis_f=1e-4, surface_flux=0)
    om = _oracle_mesh(spec)
    q = W.state_iso_pert(om.coords(), spec, seed=N)
    m = esdg.Mesh(spec)
    qg = torch.from_numpy(q).cuda()
    eg, eo = m.entropy(qg), om.entropy(q)
    print(f"[N{N} entropy] gpu={eg} oracle={eo}", flush=True)
    for k in range(3):
        assert abs(eg[k] - eo[k]) <= 1e-13 * abs(eo[k])
    r, g = om.rhs(q, gross=True)
    v = np.stack([O.entropy_vars(q[e, :, n], om.phi()[e, n]) for e in range(om.ne)
                  for n in range(om.Np)]).reshape(om.ne, om.Np, 5).transpose(0, 2, 1)
    scale = np.abs(v * g).sum() * (om.h[0] * om.h[1] * om.h[2] / 8.0)
    assert abs(eg[3] - eo[3]) <= 1e-12 * scale
    assert eg[3] < 0.0  # Rusanov faces dissipate entropy
    dt = m.cfl_dt(qg, 0.25)
    assert abs(dt - om.cfl_dt(q, 0.25)) <= 1e-14 * dt


@pytest.mark.parametrize("N,K", [(12, (2, 1, 2)), (15, (1, 1, 2))])
def test_high_order_noalloc_step_matches_lsrk_step(N, K):
    """The allocation-free step on the LDS kernel (N = 12) and on the
    prim-buffer kernel (N = 15) gives the ordinary step's bits."""
    esdg = _esdg()
    spec = W.MeshSpec(N, K, *_BOX, (1, 0, 0), coriolis_f=1e-4, surface_flux=2)
    m = esdg.Mesh(spec)
    q0 = W.make_state("iso_pert", m.coords(), spec, seed=2).contiguous()
    dt = m.cfl_dt(q0, 0.25)
    qa, dqa = q0.clone(), torch.zeros_like(q0)
    qb, dqb = q0.clone(), torch.full_like(q0, float("nan"))
    for _ in range(2):
        m.lsrk_step(qa, dqa, dt)
        m.lsrk_step_noalloc(qb, dqb, dt)
    m.check()
    assert not torch.equal(qa, q0)
    assert torch.equal(qa, qb) and torch.equal(dqa, dqb)
