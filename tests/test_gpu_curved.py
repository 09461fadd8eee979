"""Curved hexahedra on the HIP path (the box warped by a displacement that
vanishes on its faces; Sec. 3 metric terms): parity with the curved oracle
to the FP64 bars, agreement of the curved code path with the affine one at
zero warp, and the properties the metric terms must keep (free stream,
isothermal balance, entropy conservation with EC faces)."""
from dataclasses import replace

import numpy as np
import pytest

import oracle as O
from paper_2605_16684_amd import workloads as W
from tests._parity import check_rhs, check_state, err_gross

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

WARP = (0.05, 0.04, 0.03)


def _esdg():
    from paper_2605_16684_amd import esdg
    return esdg


def _oracle_mesh(spec):
    return O.Mesh(spec.N, spec.K, spec.lo, spec.hi, spec.periodic, gamma=spec.gamma,
                  gas_R=spec.gas_R, grav=spec.grav, coriolis_f=spec.coriolis_f,
                  surface_flux=spec.surface_flux, warp=spec.warp)


def _with_jumps(q, seed):
    rng = np.random.default_rng(seed)
    q = q.copy()
    q *= (1.0 + 0.02 * rng.uniform(-1, 1, size=q[:, 0].shape))[:, None, :]
    q[:, 1:4] += 5.0 * q[:, 0:1] * rng.uniform(-1, 1, size=q[:, 1:4].shape)
    return q


_BOX = ((0, 0, 0), (900.0, 700.0, 1100.0))
CASES = [
    # name, N, K, periodic, coriolis_f, surface flux, state
    ("N1_walls", 1, (3, 2, 2), (0, 0, 0), 0.0, 0, "iso_pert"),
    ("N2_mixed", 2, (2, 3, 2), (1, 0, 0), 1e-4, 0, "jumps"),
    ("N3_ragged", 3, (3, 3, 2), (0, 1, 0), 0.0, 0, "jumps"),
    ("N4_periodic_xy", 4, (3, 2, 2), (1, 1, 0), 1e-4, 0, "jumps"),
    ("N4_ec", 4, (2, 2, 3), (1, 1, 0), 0.0, 1, "jumps"),
    ("N5", 5, (2, 2, 2), (1, 0, 0), 0.0, 0, "iso_pert"),
    ("N6", 6, (1, 2, 2), (0, 1, 0), 0.0, 0, "jumps"),
    ("N7", 7, (2, 1, 2), (1, 1, 0), 1e-4, 0, "jumps"),
    ("N8", 8, (1, 1, 2), (0, 0, 0), 0.0, 0, "iso_pert"),
    ("N2_matrix_walls", 2, (3, 2, 2), (0, 0, 0), 0.0, 2, "jumps"),
    ("N4_matrix", 4, (3, 2, 2), (1, 1, 0), 1e-4, 2, "jumps"),
    ("N7_matrix", 7, (2, 1, 2), (1, 0, 0), 0.0, 2, "jumps"),
]


@pytest.mark.parametrize("name,N,K,periodic,f,surf,state", CASES, ids=[c[0] for c in CASES])
def test_curved_rhs_parity(name, N, K, periodic, f, surf, state):
    esdg = _esdg()
    spec = W.MeshSpec(N, K, *_BOX, periodic, coriolis_f=f, surface_flux=surf, warp=WARP)
    om = _oracle_mesh(spec)
    q = W.state_iso_pert(om.coords(), spec, seed=6)
    if state == "jumps":
        q = _with_jumps(q, 6)
    r_or, g = om.rhs(q, gross=True)
    m = esdg.Mesh(spec)
    r = m.rhs(torch.from_numpy(q).cuda()).cpu().numpy()
    m.check()
    check_rhs(f"curved {name}", r, r_or, g)


def test_curved_node_coords_diagnostics_and_cfl_match_oracle():
    esdg = _esdg()
    spec = W.MeshSpec(3, (3, 2, 2), *_BOX, (1, 1, 0), warp=WARP)
    om = _oracle_mesh(spec)
    m = esdg.Mesh(spec)
    x, xo = m.coords().cpu().numpy(), om.coords()
    assert np.all(np.abs(x - xo) <= 1e-12 * np.abs(xo).max())
    q = _with_jumps(W.state_iso_pert(xo, spec, seed=3), 3)
    qg = torch.from_numpy(q).cuda()
    eg, eo = m.entropy(qg), om.entropy(q)
    for c in range(3):
        assert abs(eg[c] - eo[c]) <= 1e-12 * abs(eo[c])
    dt, dto = m.cfl_dt(qg, 0.5), om.cfl_dt(q, 0.5)
    assert abs(dt - dto) <= 1e-12 * dto


@pytest.mark.parametrize("N", [3, 4])
def test_zero_warp_curved_path_equals_affine_path(N):
    esdg = _esdg()
    spec = W.MeshSpec(N, (3, 2, 2), *_BOX, (1, 1, 0), coriolis_f=1e-4)
    om = _oracle_mesh(spec)
    q = _with_jumps(W.state_iso_pert(om.coords(), spec, seed=9), 9)
    _, g = om.rhs(q, gross=True)
    qg = torch.from_numpy(q).cuda()
    ra = esdg.Mesh(spec).rhs(qg).cpu().numpy()
    rc = esdg.Mesh(replace(spec, warp=(0.0, 0.0, 0.0))).rhs(qg).cpu().numpy()
    eg = err_gross(rc, ra, g)
    print(f"[zero warp N={N}] err/gross={np.array2string(eg, precision=2)}", flush=True)
    assert np.all(eg <= 1e-14), eg


@pytest.mark.parametrize("surf", [0, 2], ids=["rusanov", "matrix"])
def test_curved_lsrk_100_steps_parity(surf):
    esdg = _esdg()
    spec = W.MeshSpec(3, (4, 4, 4), (0, 0, 0), (1000.0, 1000.0, 1000.0), (1, 1, 0), warp=WARP,
                      surface_flux=surf)
    om = _oracle_mesh(spec)
    q0 = W.state_iso_pert(om.coords(), spec, seed=1)
    dt = om.cfl_dt(q0, 0.5)
    q_or = om.run(q0, dt, 100)
    _, g0 = om.rhs(q0, gross=True)
    m = esdg.Mesh(spec)
    qg = torch.from_numpy(q0).cuda()
    dq = torch.zeros_like(qg)
    m.lsrk_run(qg, dq, dt, 100)
    check_state(f"curved lsrk100 surf={surf}", qg.cpu().numpy(), q_or, g0, 100 * dt, 100)
    # eager steps give the graph's bits
    qe = torch.from_numpy(q0).cuda()
    dqe = torch.zeros_like(qe)
    for _ in range(100):
        m.lsrk_step(qe, dqe, dt)
    assert torch.equal(qe, qg)


@pytest.mark.parametrize("N", [2, 4, 7])
def test_curved_free_stream_balance_and_entropy(N):
    esdg = _esdg()
    # free stream without gravity, periodic
    spec = W.MeshSpec(N, (3, 2, 2), *_BOX, (1, 1, 1), grav=0.0, warp=WARP)
    om = _oracle_mesh(spec)
    q = W.constant_state(om.ne, om.Np)
    _, g = om.rhs(q, gross=True)
    r = esdg.Mesh(spec).rhs(torch.from_numpy(q).cuda()).cpu().numpy()
    assert np.all(err_gross(r, 0 * r, g) <= 1e-14), err_gross(r, 0 * r, g)
    # isothermal atmosphere at rest
    spec = W.MeshSpec(N, (2, 2, 4), (0, 0, 0), (2000.0, 2000.0, 30000.0), (1, 1, 0), warp=WARP)
    om = _oracle_mesh(spec)
    q = W.state_iso_rest(om.coords(), spec, T=250.0)
    _, g = om.rhs(q, gross=True)
    r = esdg.Mesh(spec).rhs(torch.from_numpy(q).cuda()).cpu().numpy()
    assert np.all(err_gross(r, 0 * r, g) <= 1e-14), err_gross(r, 0 * r, g)
    # entropy conservation with EC faces, periodic, no gravity, jumps everywhere
    spec = W.MeshSpec(N, (2, 3, 2), (0, 0, 0), (1000.0, 1000.0, 1000.0), (1, 1, 1), grav=0.0,
                      surface_flux=1, warp=WARP)
    om = _oracle_mesh(spec)
    q = _with_jumps(W.state_iso_pert(om.coords(), spec, seed=3, amp_rho=5e-2, amp_u=20.0), 3)
    e_gpu = esdg.Mesh(spec).entropy(torch.from_numpy(q).cuda())[3]
    e_ru = esdg.Mesh(replace(spec, surface_flux=0)).entropy(torch.from_numpy(q).cuda())[3]
    print(f"[curved entropy N={N}] EC {e_gpu:.3e} Rusanov {e_ru:.3e}", flush=True)
    assert e_ru < 0.0
    assert abs(e_gpu) <= 1e-10 * abs(e_ru)


def test_curved_matrix_dissipation_vanishes_exactly_where_states_agree():
    # a horizontally uniform wind over an isothermal column: both sides of
    # every face hold the same state, so matrix-dissipation faces give the
    # RHS of EC faces bit for bit; and the entropy production is ordered
    esdg = _esdg()
    base = W.MeshSpec(4, (3, 2, 3), (0, 0, 0), (2000.0, 2000.0, 6000.0), (1, 1, 0),
                      coriolis_f=1e-4, warp=WARP)
    om = _oracle_mesh(base)
    q = W.state_iso_rest(om.coords(), base)
    q[:, 1] = 10.0 * q[:, 0]
    q[:, 2] = -5.0 * q[:, 0]
    q[:, 4] += 0.5 * q[:, 0] * 125.0
    qg = torch.from_numpy(q).cuda()
    r1 = esdg.Mesh(replace(base, surface_flux=1)).rhs(qg)
    r2 = esdg.Mesh(replace(base, surface_flux=2)).rhs(qg)
    assert torch.equal(r1, r2)
    spec = W.MeshSpec(3, (3, 2, 2), (0, 0, 0), (1000.0, 1000.0, 1000.0), (1, 1, 1), grav=0.0,
                      warp=WARP)
    om = _oracle_mesh(spec)
    q = _with_jumps(W.state_iso_pert(om.coords(), spec, seed=8, amp_rho=5e-2, amp_u=20.0), 8)
    qg = torch.from_numpy(q).cuda()
    e = {s: esdg.Mesh(replace(spec, surface_flux=s)).entropy(qg)[3] for s in (0, 1, 2)}
    print(f"[curved entropy] EC {e[1]:.3e} matrix {e[2]:.3e} Rusanov {e[0]:.3e}", flush=True)
    assert e[0] < e[2] < 0.0
    assert abs(e[1]) < 1e-10 * abs(e[2])


@pytest.mark.parametrize("mask", [1, 2, 4, 3, 6])
def test_curved_term_split_parity(mask):
    # volume, face and source terms separately (and in pairs) against the
    # oracle's term split on the curved mesh
    esdg = _esdg()
    spec = W.MeshSpec(3, (3, 2, 2), *_BOX, (1, 0, 0), coriolis_f=1e-4, warp=WARP)
    om = _oracle_mesh(spec)
    q = _with_jumps(W.state_iso_pert(om.coords(), spec, seed=4), 4)
    r_or = om.rhs(q, mask=mask)
    _, g = om.rhs(q, gross=True)
    m = esdg.Mesh(spec)
    r = m.rhs_terms(torch.from_numpy(q).cuda(), mask).cpu().numpy()
    check_rhs(f"curved mask {mask}", r, r_or, g)


def test_curved_mesh_is_not_packed():
    esdg = _esdg()
    spec = W.MeshSpec(3, (2, 2, 2), *_BOX, (1, 1, 0), warp=WARP)
    m = esdg.Mesh(spec)
    q0 = m.empty()
    q0.copy_(torch.from_numpy(W.state_iso_pert(_oracle_mesh(spec).coords(), spec, seed=1)))
    pack = esdg.Pack()
    with pytest.raises(esdg.EsdgError, match="curved"):
        pack.set_members([m], [q0], [torch.empty_like(q0)], [torch.zeros_like(q0)], [1e-3], [0])
    pack.close()


def test_curved_mass_energy_conserved_over_steps():
    esdg = _esdg()
    spec = W.MeshSpec(4, (4, 3, 3), (0, 0, 0), (1000.0, 1000.0, 1000.0), (1, 1, 0),
                      coriolis_f=1e-4, warp=WARP)
    om = _oracle_mesh(spec)
    q = torch.from_numpy(_with_jumps(W.state_iso_pert(om.coords(), spec, seed=12), 12)).cuda()
    m = esdg.Mesh(spec)
    dq = torch.zeros_like(q)
    dt = m.cfl_dt(q, 0.5)
    e0 = m.entropy(q)
    q_start = q.clone()
    m.lsrk_run(q, dq, dt, 50)
    e1 = m.entropy(q)
    moved = (q - q_start).abs().max().item()
    assert moved > 1e-6 * q_start.abs().max().item()
    print(f"[curved conservation] moved {moved:.3e} mass {abs(e1[1]-e0[1])/e0[1]:.2e} "
          f"entropy {e1[0]-e0[0]:.3e} "
          f"energy {abs(e1[2]-e0[2])/e0[2]:.2e}", flush=True)
    assert e1[0] <= e0[0] + 1e-12 * abs(e0[0])
    assert abs(e1[1] - e0[1]) <= 1e-14 * e0[1]
    assert abs(e1[2] - e0[2]) <= 1e-14 * e0[2]


def test_folding_warp_is_rejected():
    esdg = _esdg()
    spec = W.MeshSpec(4, (2, 2, 2), *_BOX, (1, 1, 0), warp=(0.6, 0.6, 0.6))
    with pytest.raises(esdg.EsdgError, match="folds"):
        esdg.Mesh(spec)
