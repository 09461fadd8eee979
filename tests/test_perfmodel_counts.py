"""The roofline's algorithmic flop constants (paper_2605_16684_amd.perfmodel)
trace to the oracle's operation counter: each constant is recomputed here
from oracle_op_count (the oracle's pointwise physics compiled over a
counting scalar) through the mapping stated in perfmodel's docstring.  The
counter's values must be the FP64 oracle's, so that the counts are those of
the arithmetic the oracle executes."""
import numpy as np
import pytest

import oracle as O
from paper_2605_16684_amd import perfmodel as PM

G = 1.4


def _state(rho, u, p, phi):
    u = np.asarray(u, dtype=float)
    return np.array([rho, *(rho * u), p / (G - 1) + 0.5 * rho * u @ u + rho * phi])


QA = _state(1.1, [3.0, -2.0, 1.0], 9.0e4, 1000.0)
QB = _state(1.1005, [3.1, -2.05, 1.02], 9.003e4, 1010.0)      # series branch of both means
QC = _state(0.9, [1.0, 2.0, 3.0], 7.0e4, 1100.0)              # log branch of both means


def _flops(*args, **kw):
    c, _ = O.op_count(*args, **kw)
    return O.flops(c)


def test_counter_values_are_the_oracles():
    for r in range(3):
        _, v = O.op_count(O.OP_FLUX, r, QA, QB, 1000.0, 1010.0)
        assert np.array_equal(v, O.two_point_flux(r, QA, QB, 1000.0, 1010.0))
        for surf in (O.SURF_RUSANOV, O.SURF_MATRIX):
            _, v = O.op_count(O.OP_SURFACE, r, QA, QB, 1000.0, 1000.0, surf=surf)
            assert np.array_equal(v, O.surface_flux(r, 1, QA, QB, 1000.0, 1000.0, surf=surf))
    _, v = O.op_count(O.OP_LOGMEAN, 0, QA, QC)
    assert v[0] == O.logmean(QA[0], QC[0])


def test_branch_selection_is_the_one_counted():
    # the two branches of the log-mean cost differently: the series has no log
    cs, _ = O.op_count(O.OP_LOGMEAN, 0, QA, QB)
    cl, _ = O.op_count(O.OP_LOGMEAN, 0, QA, QC)
    assert cs["log"] == 0 and cl["log"] == 2
    c, _ = O.op_count(O.OP_FLUX, 2, QA, QB, 1000.0, 1010.0)
    assert c["log"] == 0


def test_perfmodel_constants_follow_from_the_counts():
    c_node = _flops(O.OP_NODE, 0, QA, QA, 1000.0, 1000.0)
    c_flux = {r: _flops(O.OP_FLUX, r, QA, QB, 1000.0, 1010.0) for r in range(3)}
    assert len(set(c_flux.values())) == 1          # the same arithmetic in every direction
    c_flux = c_flux[0]
    # the gravity term and its addition into the normal momentum flux
    c_grav = _flops(O.OP_GRAVITY, 2, QA, QB, 1000.0, 1010.0) + 1
    c_face = _flops(O.OP_SURFACE, 0, QA, QB, 1000.0, 1000.0, surf=O.SURF_RUSANOV)
    c_upd = _flops(O.OP_UPDATE, 0, np.array([0.3, 0.2, 1e-3, 5.0, 0.0]),
                   np.array([1.0, 2.0, 0.0, 0.0, 0.0]))
    c_src = _flops(O.OP_SOURCE, 0, QA, QA, 1e-4, 0.0)
    assert (PM.C_NODE, PM.C_FLUX, PM.C_GRAV, PM.C_FACE, PM.C_UPDATE, PM.C_SOURCE) == \
        (c_node, c_flux, c_grav, c_face, c_upd, c_src)
    assert PM.PRECOMP == c_node
    assert PM.PAIR_XY == c_flux - 2 * c_node - c_grav + PM.SCATTER
    assert PM.PAIR_Z == c_flux - 2 * c_node + c_grav + PM.SCATTER
    assert PM.FACE_NODE == c_face - c_node - c_grav + PM.LIFT
    assert PM.FINISH_STAGE == 5 * c_upd + c_src + PM.PHASE
    assert PM.FINISH_RHS == c_src + PM.PHASE
    # kernel-structure terms: multiply-and-add per variable
    assert PM.SCATTER == 2 * 5 * 2 and PM.LIFT == 5 * 2 and PM.PHASE == 5 * (3 + 2)


@pytest.mark.parametrize("N", [3, 4, 7])
def test_flops_per_node_from_the_constants(N):
    Nq = N + 1
    pair = (2 * PM.PAIR_XY + PM.PAIR_Z) / 3.0
    want = pair * 1.5 * N + PM.FACE_NODE * 6.0 / Nq + PM.PRECOMP + PM.FINISH_STAGE
    assert PM.flops_per_node(N) == pytest.approx(want)
