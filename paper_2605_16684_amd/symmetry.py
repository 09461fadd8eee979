"""Mirror-symmetry defect of a state on the box (a measurement, not part of
the right-hand side).

The rising-bubble problems of the paper's Sec. 5.1 are symmetric about the
vertical planes through the bubble centre, and the exact solution keeps
that symmetry; the paper observes that FP64 runs keep it better than FP32
runs, since rounding errors are not made symmetrically.  On a box of K
elements per direction with the mirror plane at the box centre, mirroring
about x maps element ex to K_x - 1 - ex and LGL node i to N - i (the nodes
are symmetric), and negates the x momentum; likewise for y.

States use the boundary layout q[e][v][n], e = ex + Kx (ey + Ky ez),
n = i + Nq (j + Nq k); numpy arrays or torch tensors (on any device).
"""
from __future__ import annotations


def _xp(a):
    if type(a).__module__.startswith("torch"):
        import torch
        return torch
    import numpy as np
    return np


def mirror(q, K, N, axis):
    """The state mirrored about the box's mid-plane normal to `axis` (0 = x,
    1 = y, 2 = z), with that momentum component negated."""
    xp = _xp(q)
    Nq = N + 1
    a = q.reshape(K[2], K[1], K[0], 5, Nq, Nq, Nq)    # ez, ey, ex, v, k, j, i
    dims = {0: (2, 6), 1: (1, 5), 2: (0, 4)}[axis]
    if xp.__name__ == "torch":
        m = xp.flip(a, dims=dims).clone()
    else:
        m = xp.flip(a, axis=dims).copy()
    m[:, :, :, 1 + axis] = -m[:, :, :, 1 + axis]
    return m.reshape(q.shape)


def defect(q, K, N, axis, q_ref=None):
    """Per conserved variable: ||q_v - (M q)_v|| / ||q_v - q_ref,v|| (the
    deviation from a symmetric reference, e.g. the hydrostatic background,
    so that the defect is measured against the flow and not against the
    atmosphere at rest), or / ||q_v|| without a reference.  Returns a list of
    five floats."""
    xp = _xp(q)
    d = q - mirror(q, K, N, axis)
    base = q if q_ref is None else q - q_ref
    out = []
    for v in range(5):
        num = float((d[:, v] ** 2).sum()) ** 0.5
        den = float((base[:, v] ** 2).sum()) ** 0.5
        out.append(num / den if den > 0 else 0.0)
    return out
