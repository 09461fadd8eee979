"""Shared helpers of the parity tests: error norms and the stated tolerances.

RHS (per conserved variable v, over all compared nodes):
    err_gross_v = ||R_gpu,v - R_oracle,v||_2 / ||A_v||_2 <= TOL_RHS,
where A_v is the oracle's sum of the absolute values of every term that
enters R_v at a node (volume pair terms, face terms, source).  Near
hydrostatic balance the momentum RHS is a sum of terms up to ~1e6-1e16 times
larger than the result, so two correct FP64 evaluations that add the same
terms in a different order differ by ~1e-16 of A, not of R.  The net
relative error is asserted too, against the larger of the literal bar and
the cancellation bound:
    err_net_v = ||dR_v|| / ||R_v|| <= max(TOL_RHS_NET, C_RHS eps kappa_v),
    kappa_v = ||A_v|| / ||R_v||.
(The second is err_gross_v <= C_RHS eps; with C_RHS = 64 it is the tighter of
the two gross bars.)

State after n LSRK steps (per conserved variable, relative L2):
    err_v = ||q_gpu,v - q_oracle,v|| / ||q_oracle,v||
          <= max(TOL_STATE, eps kappa_s,v / sqrt(n_rhs)),
    kappa_s,v = T ||A_v(q_0)|| / ||q_oracle,v(T)||,   T = n dt,
with n_rhs = 5 n right-hand-side evaluations.  This is the state analogue of
the RHS bound: each evaluation differs by about one rounding of its gross
terms, and those differences, taken at different states, add in quadrature
over the n_rhs evaluations.  Where the state is not cancellation-dominated
(density, energy, a jet's zonal momentum) the literal 1e-10 binds; for a
momentum component that grows from rest out of cancelling pressure and
gravity terms (a bubble's horizontal momentum, a channel's vertical
momentum) the cancellation bound does.

FP32-mixed path (same norms, single-precision unit): RHS
    err_gross_v <= 1e-5,  err_net_v <= max(1e-5, C_RHS32 eps32 kappa_v),
and the state after n steps within max(1e-4, eps32 kappa_s,v / sqrt(n_rhs)),
eps32 = 2^-23.  Where kappa_v eps32 exceeds 1e-5 (the channel's density and
energy at N = 7, kappa ~ 1e4-1e5) no FP32 evaluation of the gross terms can
meet the literal 1e-5: one rounding of each term already leaves more.
"""
import numpy as np

EPS = 2.0 ** -52
EPS32 = 2.0 ** -23
TOL_RHS = 2e-14      # FP64 RHS vs oracle, relative to the gross term scale
TOL_RHS_NET = 1e-12  # FP64 RHS vs oracle, plain relative L2 (where cancellation allows)
C_RHS = 64
TOL_STATE = 1e-10    # FP64 state after 100 LSRK(5,4) steps, relative L2 per variable
TOL_RHS_MIXED = 1e-5     # FP32-mixed RHS: gross scale, and plain where cancellation allows
C_RHS32 = 1
TOL_STATE_MIXED = 1e-4   # FP32-mixed state after 100 steps, relative L2 per variable


def _norm(a):
    return np.sqrt((np.asarray(a) ** 2).sum(axis=(0, 2)))


def err_gross(a, b, gross):
    return _norm(a - b) / np.maximum(_norm(gross), 1e-300)


def err_net(a, b):
    return _norm(a - b) / np.maximum(_norm(b), 1e-300)


def kappa(r, gross):
    return _norm(gross) / np.maximum(_norm(r), 1e-300)


def rhs_net_bar(r_or, gross, mixed=False):
    if mixed:
        return np.maximum(TOL_RHS_MIXED, C_RHS32 * EPS32 * kappa(r_or, gross))
    return np.maximum(TOL_RHS_NET, C_RHS * EPS * kappa(r_or, gross))


def check_rhs(tag, r_gpu, r_or, gross, mixed=False):
    """Print and assert both RHS bars per conserved variable (FP64, or the
    FP32-mixed path's with mixed=True)."""
    tol_gross = TOL_RHS_MIXED if mixed else TOL_RHS
    eg, en, k = err_gross(r_gpu, r_or, gross), err_net(r_gpu, r_or), kappa(r_or, gross)
    bar = rhs_net_bar(r_or, gross, mixed)
    print(f"[{tag}] err/gross={np.array2string(eg, precision=2)} "
          f"err/net={np.array2string(en, precision=2)} kappa={np.array2string(k, precision=1)} "
          f"net bar={np.array2string(bar, precision=1)}", flush=True)
    assert np.all(eg <= tol_gross), (tag, eg)
    assert np.all(en <= bar), (tag, en, bar)
    return eg


def state_kappa(q_or, gross0, t_total):
    return t_total * _norm(gross0) / np.maximum(_norm(q_or), 1e-300)


def state_bar(q_or, gross0, t_total, nsteps, mixed=False):
    n_rhs = 5 * nsteps
    tol, eps = (TOL_STATE_MIXED, EPS32) if mixed else (TOL_STATE, EPS)
    return np.maximum(tol, eps * state_kappa(q_or, gross0, t_total) / np.sqrt(n_rhs))


def check_state(tag, q_gpu, q_or, gross0, t_total, nsteps, mixed=False):
    """Print and assert the per-variable state bar after nsteps LSRK steps."""
    e = err_net(q_gpu, q_or)
    ks = state_kappa(q_or, gross0, t_total)
    bar = state_bar(q_or, gross0, t_total, nsteps, mixed)
    print(f"[{tag}] state rel L2 per var {np.array2string(e, precision=2)} "
          f"kappa_s={np.array2string(ks, precision=1)} bar={np.array2string(bar, precision=1)}",
          flush=True)
    assert np.all(e <= bar), (tag, e, bar)
    return e
