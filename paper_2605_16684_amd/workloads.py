"""Seeded synthetic input states and the workload configurations.

This module is the only code shared by the HIP path and the CPU oracle's
tests: it turns node coordinates into initial states.  It holds no part of
the discretisation (no fluxes, no quadrature, no operators): the caller
passes the node coordinates xyz[e][3][n] of its own mesh, and every state is
returned in the boundary layout q[e][v][n] with v in (rho, rho u, rho v,
rho w, rho E) and E = p/(gamma-1) + rho |u|^2 / 2 + rho g z, the total energy
with geopotential of the governing equations (Sec. 2 of the paper).

The shapes follow the paper's test cases (Sec. 5): a rising thermal bubble
in a neutral atmosphere (smooth cosine perturbation of potential
temperature) and a zonal-jet channel in hydrostatic, geostrophically
balanced background with a Gaussian wind perturbation.  The paper's channel
benchmark state is not reproduced; the channel here is a self-constructed
stand-in of the same shape and size.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Tuple

import numpy as np


def _xp(a):
    """numpy for numpy arrays, torch for torch tensors (states can be built
    directly in device memory)."""
    if type(a).__module__.startswith("torch"):
        import torch
        return torch
    return np


GAMMA = 1.4
GAS_R = 287.0
GRAV = 9.81
P0 = 1.0e5
CP = GAS_R * GAMMA / (GAMMA - 1.0)


@dataclasses.dataclass(frozen=True)
class MeshSpec:
    """Box mesh description shared by the library and the oracle."""
    N: int
    K: Tuple[int, int, int]
    lo: Tuple[float, float, float]
    hi: Tuple[float, float, float]
    periodic: Tuple[int, int, int]
    gamma: float = GAMMA
    gas_R: float = GAS_R
    grav: float = GRAV
    coriolis_f: float = 0.0
    surface_flux: int = 0  # 0 Rusanov, 1 entropy-conservative, 2 matrix dissipation
    # curved hexahedra: warp amplitudes (fractions of the box lengths) of the
    # displacement that vanishes on the box faces; None = the affine box
    warp: Optional[Tuple[float, float, float]] = None

    @property
    def n_elem(self) -> int:
        return self.K[0] * self.K[1] * self.K[2]

    @property
    def n_nodes(self) -> int:
        return self.n_elem * (self.N + 1) ** 3


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    mesh: MeshSpec
    kind: str          # "iso_pert" | "bubble" | "channel"
    steps: int
    cfl: float = 0.5


def iso_pert_cube(N=3, K=(4, 4, 4)) -> Workload:
    """1 km cube, periodic x/y, walls z, perturbed isothermal atmosphere."""
    return Workload("iso_pert_4x4x4_N3", MeshSpec(N, tuple(K), (0.0, 0.0, 0.0),
                                                    (1000.0, 1000.0, 1000.0), (1, 1, 0)),
                    "iso_pert", 10)


def rising_bubble(N=4, K=(32, 32, 32)) -> Workload:
    """1 km cube, walls everywhere, neutral atmosphere with a warm bubble."""
    return Workload(f"rising_bubble_{K[0]}x{K[1]}x{K[2]}_N{N}",
                    MeshSpec(N, tuple(K), (0.0, 0.0, 0.0), (1000.0, 1000.0, 1000.0), (0, 0, 0)),
                    "bubble", 200)


def channel(N=4, K=(160, 24, 10)) -> Workload:
    """40000 x 6000 x 30 km channel, periodic x, walls y/z, f-plane."""
    return Workload(f"baroclinic_channel_{K[0]}x{K[1]}x{K[2]}_N{N}",
                    MeshSpec(N, tuple(K), (0.0, 0.0, 0.0), (4.0e7, 6.0e6, 3.0e4), (1, 0, 0),
                             coriolis_f=1.0e-4),
                    "channel", 100)


def high_order_box(N, K) -> Workload:
    """Perturbed isothermal box of 1 km elements, periodic x/y, walls z, for
    the orders 9..15 (CFL 0.25: the step rule's 0.5 is unstable from about
    N = 12 on)."""
    return Workload(f"iso_pert_box_{K[0]}x{K[1]}x{K[2]}_N{N}",
                    MeshSpec(N, tuple(K), (0.0, 0.0, 0.0),
                             (1000.0 * K[0], 1000.0 * K[1], 1000.0 * K[2]), (1, 1, 0)),
                    "iso_pert", 20, cfl=0.25)


WORKLOADS = {
    "c0": iso_pert_cube(),
    "c1": rising_bubble(),
    "c2": channel(),
    "c3": channel(N=7),
    # orders above the fused kernel's: LDS kernel (N = 12), prim buffer (N = 15)
    "h12": high_order_box(12, (10, 8, 8)),
    "h15": high_order_box(15, (8, 8, 8)),
}


# --------------------------------------------------------------------------
# Background atmospheres
# --------------------------------------------------------------------------

def _energy(rho, u, v, w, p, z, gamma=GAMMA, grav=GRAV):
    return p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w) + rho * grav * z


def _pack(rho, u, v, w, p, z, gamma=GAMMA, grav=GRAV):
    xp = _xp(rho)
    return xp.stack([rho, rho * u, rho * v, rho * w, _energy(rho, u, v, w, p, z, gamma, grav)],
                    axis=1)


def isothermal(z, T=300.0, p0=P0, gas_R=GAS_R, grav=GRAV):
    """Isothermal hydrostatic profile: p = p0 exp(-g z/(R T)), rho = p/(R T)."""
    p = p0 * _xp(z).exp(-grav * z / (gas_R * T))
    return p / (gas_R * T), p


def neutral(z, theta0=300.0, p0=P0, gas_R=GAS_R, grav=GRAV, gamma=GAMMA):
    """Constant potential temperature: Exner pi = 1 - g z/(cp theta0)."""
    cp = gas_R * gamma / (gamma - 1.0)
    pi = 1.0 - grav * z / (cp * theta0)
    p = p0 * pi ** (cp / gas_R)
    return pi, p


def _fourier(rng, x, y, z, L, nmodes=4):
    """Smooth seeded field: sum of nmodes plane waves with integer wavenumbers
    1..3 per direction over the box lengths L, random phases, amplitudes in
    [0.5, 1], normalised so that |field| <= 1 everywhere."""
    xp = _xp(x)
    out = xp.zeros_like(x)
    amps = rng.uniform(0.5, 1.0, nmodes)
    for m in range(nmodes):
        kx, ky, kz = rng.integers(1, 4, size=3)
        ph = rng.uniform(0.0, 2.0 * math.pi)
        out = out + float(amps[m]) * xp.cos(
            2 * math.pi * (float(kx) * x / L[0] + float(ky) * y / L[1] + float(kz) * z / L[2])
            + float(ph))
    return out / float(amps.sum())


def state_iso_pert(xyz, spec: MeshSpec, seed=0, T=300.0, amp_rho=1e-3, amp_u=1.0):
    """Isothermal hydrostatic state (T, p0 at z = 0) with seeded smooth
    perturbations: rho *= 1 + amp_rho * field, each velocity component
    += amp_u * field (independent fields); pressure unchanged."""
    rng = np.random.default_rng(seed)
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    L = [spec.hi[d] - spec.lo[d] for d in range(3)]
    rho, p = isothermal(z, T, gas_R=spec.gas_R, grav=spec.grav)
    rho = rho * (1.0 + amp_rho * _fourier(rng, x, y, z, L))
    u = amp_u * _fourier(rng, x, y, z, L)
    v = amp_u * _fourier(rng, x, y, z, L)
    w = amp_u * _fourier(rng, x, y, z, L)
    return _pack(rho, u, v, w, p, z, spec.gamma, spec.grav)


def state_iso_rest(xyz, spec: MeshSpec, T=300.0):
    """Isothermal hydrostatic state at rest (discretely well balanced)."""
    z = xyz[:, 2]
    rho, p = isothermal(z, T, gas_R=spec.gas_R, grav=spec.grav)
    zero = _xp(z).zeros_like(z)
    return _pack(rho, zero, zero, zero, p, z, spec.gamma, spec.grav)


def state_bubble(xyz, spec: MeshSpec, seed: Optional[int] = None, theta0=300.0, amp=0.5,
                 rc=250.0, centre=(500.0, 500.0, 350.0), shape="smooth"):
    """Neutral atmosphere with a warm bubble (Sec. 5.1): the smooth cosine
    bubble dtheta = amp (1 + cos(pi r/rc))/2 for r <= rc, or with
    shape="sharp" the discontinuous one, dtheta = amp for r <= rc, 0 outside;
    p is the background hydrostatic pressure, u = 0.  A seed jitters the
    centre (+-50 m) and the amplitude (x [0.8, 1.2])."""
    if seed is not None:
        rng = np.random.default_rng(seed)
        centre = tuple(c + float(rng.uniform(-50.0, 50.0)) for c in centre)
        amp = amp * float(rng.uniform(0.8, 1.2))
    xp = _xp(xyz)
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    pi, p = neutral(z, theta0, gas_R=spec.gas_R, grav=spec.grav, gamma=spec.gamma)
    r = xp.sqrt((x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2)
    if shape == "sharp":
        dth = amp * (r <= rc)
    elif shape == "smooth":
        rcl = xp.clip(r, None, rc) if xp is np else r.clamp(max=rc)
        dth = amp * 0.5 * (1.0 + xp.cos(math.pi * rcl / rc))
        dth = dth * (r <= rc)
    else:
        raise ValueError(shape)
    rho = p / (spec.gas_R * (theta0 + dth) * pi)
    zero = xp.zeros_like(z)
    return _pack(rho, zero, zero, zero, p, z, spec.gamma, spec.grav)


def channel_background(y, z, spec: MeshSpec, T0=300.0, dT=15.0):
    """Per-column isothermal hydrostatic background with
    T(y) = T0 - dT/2 (1 - cos(pi y/Ly)); returns (T, rho, p)."""
    xp = _xp(y)
    Ly = spec.hi[1] - spec.lo[1]
    T = T0 - 0.5 * dT * (1.0 - xp.cos(math.pi * (y - spec.lo[1]) / Ly))
    p = P0 * xp.exp(-spec.grav * z / (spec.gas_R * T))
    return T, p / (spec.gas_R * T), p


def state_channel(xyz, spec: MeshSpec, seed=0, T0=300.0, dT=15.0, bump=1.0, sigma=5.0e5):
    """Zonal jet in thermal-wind balance with the per-column isothermal
    background: f u = -g z T'(y)/T(y), zero at the walls, about 40 m/s at the
    top; plus a seeded Gaussian zonal-wind bump of `bump` m/s, width sigma."""
    rng = np.random.default_rng(seed)
    xp = _xp(xyz)
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    Ly = spec.hi[1] - spec.lo[1]
    Lx = spec.hi[0] - spec.lo[0]
    T, rho, p = channel_background(y, z, spec, T0, dT)
    dTdy = -0.5 * dT * (math.pi / Ly) * xp.sin(math.pi * (y - spec.lo[1]) / Ly)
    f = spec.coriolis_f if spec.coriolis_f != 0.0 else 1.0e-4
    u = -spec.grav * z * dTdy / (f * T)
    xc = spec.lo[0] + float(rng.uniform(0.25, 0.75)) * Lx
    yc = spec.lo[1] + float(rng.uniform(0.35, 0.65)) * Ly
    u = u + bump * xp.exp(-((x - xc) ** 2 + (y - yc) ** 2) / (2.0 * sigma ** 2))
    zero = xp.zeros_like(z)
    return _pack(rho, u, zero, zero, p, z, spec.gamma, spec.grav)


def reference_state(xyz, spec: MeshSpec, kind: str):
    """Hydrostatic reference (rho_r, p_r) per node for the mixed-precision
    path: [e][n] arrays."""
    z = xyz[:, 2]
    if kind in ("bubble", "bubble_sharp"):
        pi, p = neutral(z, gas_R=spec.gas_R, grav=spec.grav, gamma=spec.gamma)
        return p / (spec.gas_R * 300.0 * pi), p
    if kind == "channel":
        _, rho, p = channel_background(xyz[:, 1], z, spec)
        return rho, p
    rho, p = isothermal(z, gas_R=spec.gas_R, grav=spec.grav)
    return rho, p


def make_state(kind: str, xyz, spec: MeshSpec, seed=0):
    if kind == "iso_pert":
        return state_iso_pert(xyz, spec, seed)
    if kind == "bubble":
        return state_bubble(xyz, spec, None if seed == 0 else seed)
    if kind == "bubble_sharp":
        return state_bubble(xyz, spec, None if seed == 0 else seed, shape="sharp")
    if kind == "channel":
        return state_channel(xyz, spec, seed)
    if kind == "iso_rest":
        return state_iso_rest(xyz, spec)
    raise ValueError(kind)


def density_wave(xyz, spec: MeshSpec, t=0.0, rho0=1.0, amp=0.1, u0=1.0, p=1.0):
    """Exact solution of the Euler equations without gravity on a periodic
    cube of side L: rho = rho0 (1 + amp sin(2 pi (x + y + z - 3 u0 t)/L)),
    u = v = w = u0, p constant."""
    L = spec.hi[0] - spec.lo[0]
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    rho = rho0 * (1.0 + amp * np.sin(2 * math.pi * (x + y + z - 3.0 * u0 * t) / L))
    u = np.full_like(x, u0)
    q = np.empty((rho.shape[0], 5, rho.shape[1]))
    q[:, 0] = rho
    q[:, 1] = rho * u
    q[:, 2] = rho * u
    q[:, 3] = rho * u
    q[:, 4] = p / (spec.gamma - 1.0) + 0.5 * rho * 3.0 * u0 * u0
    return q


def constant_state(ne, Np, rho=1.2, u=(3.0, -2.0, 1.0), p=9.0e4, gamma=GAMMA):
    """Uniform state without gravity (free stream)."""
    q = np.empty((ne, 5, Np))
    q[:, 0] = rho
    for c in range(3):
        q[:, 1 + c] = rho * u[c]
    q[:, 4] = p / (gamma - 1.0) + 0.5 * rho * sum(c * c for c in u)
    return q
