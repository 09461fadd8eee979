"""FP32-mixed path against the FP64 oracle.

Bars (stated per result, tests/_parity.py): per conserved variable, the RHS
error is at most 1e-5 of the gross term scale and at most
max(1e-5, eps32 kappa_v) of the RHS itself (one FP32 rounding of the gross
terms: where the RHS is a small residual of large terms, as for the
channel's density and energy, no FP32 evaluation of those terms can do
better); the state after 100 LSRK(5,4) steps is within
max(1e-4, eps32 kappa_s / sqrt(500)) relative L2 per Cartesian component;
mass and total-energy drift within 1e-10 (FP32 fluxes conserve to their own
rounding; the paper reports ~1e-7 for its FP32 runs); entropy drift
reported beside the oracle's.
"""
from dataclasses import replace

import numpy as np
import pytest

import oracle as O
from paper_2605_16684_amd import workloads as W
from tests._parity import check_rhs, check_state, err_gross

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _esdg():
    from paper_2605_16684_amd import esdg
    return esdg


def _oracle_mesh(spec):
    return O.Mesh(spec.N, spec.K, spec.lo, spec.hi, spec.periodic, gamma=spec.gamma,
                  gas_R=spec.gas_R, grav=spec.grav, coriolis_f=spec.coriolis_f,
                  surface_flux=spec.surface_flux)


def _mixed_mesh(spec, xyz, kind):
    esdg = _esdg()
    rr, pr = W.reference_state(xyz, spec, kind)
    rr_t = torch.from_numpy(np.ascontiguousarray(rr)).cuda()
    pr_t = torch.from_numpy(np.ascontiguousarray(pr)).cuda()
    return esdg.Mesh(spec, precision=esdg.FP32_MIXED, ref_rho=rr_t, ref_p=pr_t)


CASES = [
    ("c0_iso_pert", W.iso_pert_cube().mesh, "iso_pert"),
    ("bubble_small", W.rising_bubble(K=(4, 4, 4)).mesh, "bubble"),
    ("channel_small", W.channel(K=(8, 4, 3)).mesh, "channel"),
    ("channel_small_N7", W.channel(N=7, K=(4, 3, 2)).mesh, "channel"),
    ("N3_walls", W.MeshSpec(3, (3, 2, 2), (0, 0, 0), (900.0, 700.0, 1100.0), (0, 0, 0)), "iso_pert"),
    ("N5_ec", W.MeshSpec(5, (2, 2, 2), (0, 0, 0), (900.0, 700.0, 1100.0), (1, 0, 0),
                         surface_flux=1), "iso_pert"),
    ("N6_walls", W.MeshSpec(6, (2, 1, 2), (0, 0, 0), (900.0, 700.0, 1100.0), (0, 1, 0)),
     "iso_pert"),
    ("channel_small_N6", W.channel(N=6, K=(4, 3, 2)).mesh, "channel"),
]


@pytest.mark.parametrize("N", range(1, 9))
def test_default_epw_exists_for_every_order(N):
    # a mesh created with epw = 0 gets a compiled variant of its own
    # precision, and set_epw(0) returns to it
    esdg = _esdg()
    spec = W.MeshSpec(N, (2, 1, 1), (0, 0, 0), (900.0, 700.0, 1100.0), (1, 1, 0))
    xyz = _oracle_mesh(spec).coords()
    for m in (esdg.Mesh(spec), _mixed_mesh(spec, xyz, "iso_pert")):
        e = m.epw
        assert e in esdg.epw_options(N, m.precision)
        m.set_epw(0)
        assert m.epw == e
        m.close()


@pytest.mark.parametrize("name,spec,kind", CASES, ids=[c[0] for c in CASES])
def test_mixed_rhs_error(name, spec, kind):
    om = _oracle_mesh(spec)
    xyz = om.coords()
    q = W.make_state(kind, xyz, spec, seed=5)
    r_or, g = om.rhs(q, gross=True)
    m = _mixed_mesh(spec, xyz, kind)
    r = m.rhs(torch.from_numpy(q).cuda()).cpu().numpy()
    check_rhs(f"mixed {name}", r, r_or, g, mixed=True)


def _with_jumps(q, seed):
    """Seeded node-by-node perturbation so that states jump at every face."""
    rng = np.random.default_rng(seed)
    q = q.copy()
    q *= (1.0 + 0.02 * rng.uniform(-1, 1, size=q[:, 0].shape))[:, None, :]
    q[:, 1:4] += 5.0 * q[:, 0:1] * rng.uniform(-1, 1, size=q[:, 1:4].shape)
    return q


MATRIX_CASES = [
    ("channel_N7_matrix", replace(W.channel(N=7, K=(4, 3, 2)).mesh, surface_flux=2), "channel"),
    ("bubble_matrix", replace(W.rising_bubble(K=(4, 4, 4)).mesh, surface_flux=2), "bubble"),
    ("N2_walls_matrix", W.MeshSpec(2, (3, 2, 2), (0, 0, 0), (900.0, 700.0, 1100.0), (0, 0, 0),
                                   surface_flux=2), "iso_pert"),
]


@pytest.mark.parametrize("jumps", [False, True], ids=["smooth", "jumps"])
@pytest.mark.parametrize("name,spec,kind", MATRIX_CASES, ids=[c[0] for c in MATRIX_CASES])
def test_mixed_rhs_error_matrix_dissipation(name, spec, kind, jumps):
    om = _oracle_mesh(spec)
    xyz = om.coords()
    q = W.make_state(kind, xyz, spec, seed=5)
    if jumps:
        q = _with_jumps(q, 5)
    r_or, g = om.rhs(q, gross=True)
    m = _mixed_mesh(spec, xyz, kind)
    r = m.rhs(torch.from_numpy(q).cuda()).cpu().numpy()
    check_rhs(f"mixed {name} jumps={jumps}", r, r_or, g, mixed=True)


def test_mixed_full_size_sampled_channel_N7():
    """The precision comparison's own configuration (160 x 24 x 10 channel
    at N = 7, 19.7 M nodes) in the launch configuration bench.py times:
    sampled elements of the mixed RHS against the FP64 oracle."""
    from paper_2605_16684_amd import esdg
    wl = W.WORKLOADS["c3"]
    spec = wl.mesh
    om = _oracle_mesh(spec)
    xyz = om.coords()
    q = W.make_state(wl.kind, xyz, spec, seed=1)
    m = _mixed_mesh(spec, xyz, wl.kind)
    del xyz
    r = m.rhs(torch.from_numpy(q).cuda()).cpu().numpy()
    rng = np.random.default_rng(0)
    el = np.unique(np.concatenate([rng.choice(om.ne, 32, replace=False), [0, om.ne - 1]]))
    r_or, g = om.rhs_elems(q, el)
    print(f"[mixed c3-sampled] epw={m.epw}", flush=True)
    check_rhs("mixed c3-sampled", r[el], r_or, g, mixed=True)
    m.close()


def test_mixed_well_balanced_reference_state():
    spec = W.MeshSpec(4, (2, 2, 3), (0, 0, 0), (2000.0, 2000.0, 30000.0), (1, 1, 0))
    om = _oracle_mesh(spec)
    xyz = om.coords()
    q = W.state_iso_rest(xyz, spec)
    _, g = om.rhs(q, gross=True)
    m = _mixed_mesh(spec, xyz, "iso_rest")
    r = m.rhs(torch.from_numpy(q).cuda()).cpu().numpy()
    assert np.all(err_gross(r, 0 * r, g) <= 1e-14)


@pytest.mark.parametrize("name,wl", [
    ("channel_N7_small", W.channel(N=7, K=(6, 4, 3))),
    ("c0", W.iso_pert_cube()),
    ("channel_N4_matrix", replace(W.channel(K=(8, 4, 3)), mesh=replace(W.channel(K=(8, 4, 3)).mesh,
                                                                        surface_flux=2))),
])
def test_mixed_100_steps_against_oracle(name, wl):
    spec = wl.mesh
    om = _oracle_mesh(spec)
    xyz = om.coords()
    q0 = W.make_state(wl.kind, xyz, spec, seed=3)
    dt = om.cfl_dt(q0, wl.cfl)
    q_or = om.run(q0, dt, 100)
    _, g0 = om.rhs(q0, gross=True)
    m = _mixed_mesh(spec, xyz, wl.kind)
    q = torch.from_numpy(q0).cuda()
    dq = torch.zeros_like(q)
    e0 = m.entropy(q)
    m.lsrk_run(q, dq, dt, 100)
    e1 = m.entropy(q)
    eo0, eo1 = om.entropy(q0), om.entropy(q_or)
    qa = q.cpu().numpy()
    print(f"[mixed 100 steps {name}] "
          f"entropy change mixed {(e1[0]-e0[0])/abs(e0[0]):.3e} oracle {(eo1[0]-eo0[0])/abs(eo0[0]):.3e}; "
          f"mass drift {abs(e1[1]-e0[1])/e0[1]:.2e} energy drift {abs(e1[2]-e0[2])/e0[2]:.2e}",
          flush=True)
    check_state(f"mixed 100 steps {name}", qa, q_or, g0, 100 * dt, 100, mixed=True)
    assert abs(e1[1] - e0[1]) <= 1e-10 * e0[1]
    assert abs(e1[2] - e0[2]) <= 1e-10 * e0[2]
