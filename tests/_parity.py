"""Shared helpers of the parity tests: error norms and the stated tolerances.

Parity norm (per conserved variable v, over all compared nodes):
    err_v = ||R_gpu,v - R_oracle,v||_2 / ||A_v||_2,
where A_v is the oracle's sum of the absolute values of every term that
enters R_v at a node (volume pair terms, face terms, source).  The RHS is a
sum of terms up to ~1e6 times larger than the result (momentum near
hydrostatic balance), so two correct FP64 evaluations that add the same
terms in different orders differ by ~1e-16 of A, not of R: relative error
against ||R|| is not a well-posed target there, relative error against the
terms' own magnitude is.  The net relative error ||dR||/||R|| is reported
beside it.
"""
import numpy as np

TOL_RHS = 1e-12      # FP64 RHS vs oracle, relative to the gross term scale
TOL_STATE = 1e-10    # FP64 state after 100 LSRK(5,4) steps, relative L2 per variable


def err_gross(a, b, gross):
    d = np.sqrt(((a - b) ** 2).sum(axis=(0, 2)))
    s = np.sqrt((gross ** 2).sum(axis=(0, 2)))
    return d / np.maximum(s, 1e-300)


def err_net(a, b):
    d = np.sqrt(((a - b) ** 2).sum(axis=(0, 2)))
    s = np.sqrt((b ** 2).sum(axis=(0, 2)))
    return d / np.maximum(s, 1e-300)


def kappa(r, gross):
    return np.sqrt((gross ** 2).sum(axis=(0, 2))) / np.maximum(np.sqrt((r ** 2).sum(axis=(0, 2))), 1e-300)
