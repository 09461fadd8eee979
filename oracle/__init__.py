"""CPU oracle for the ES-DGSEM right-hand side -- TEST INFRASTRUCTURE ONLY.

This package wraps liboracle.so (plain FP64 C, see esdg_oracle.c) with
ctypes and numpy.  It is imported only by tests/, by
``__graft_entry__.smoke()`` and by the ``cpu_baseline`` leg of bench.py; the
product path (paper_2605_16684_amd) never imports it, and the two share no
code.  Arrays use the layout q[e][v][n]: element e = ex + Kx (ey + Ky ez),
variable v in (rho, rho u, rho v, rho w, rho E), node n = i + Nq (j + Nq k).
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

TERM_VOL, TERM_FACE, TERM_SRC = 1, 2, 4
TERM_ALL = TERM_VOL | TERM_FACE | TERM_SRC
SURF_RUSANOV, SURF_EC, SURF_MATRIX = 0, 1, 2

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_i64p = C.POINTER(C.c_int64)


def _stale(lib, sources):
    return not os.path.exists(lib) or any(os.path.getmtime(lib) < os.path.getmtime(f)
                                          for f in sources)


_POINTWISE = os.path.join(_HERE, "esdg_pointwise.h")


def _load():
    if _stale(_LIB_PATH, (_build.SRC, _POINTWISE)) or \
            _stale(_build.OPC_LIB, (_build.OPC_SRC, _POINTWISE)):
        _build.build()
    lib = C.CDLL(_LIB_PATH)
    sig = {
        "oracle_lgl": (None, [C.c_int, _dp, _dp, _dp]),
        "oracle_mesh_create": (C.c_void_p, [C.c_int, _ip, _dp, _dp, _ip, C.c_double,
                                            C.c_double, C.c_double, C.c_double, C.c_int]),
        "oracle_mesh_create_warped": (C.c_void_p, [C.c_int, _ip, _dp, _dp, _ip, C.c_double,
                                                   C.c_double, C.c_double, C.c_double, C.c_int,
                                                   _dp]),
        "oracle_metrics": (None, [C.c_void_p, _dp, _dp]),
        "oracle_surface_flux_vec": (None, [_dp, _dp, _dp, C.c_double, C.c_double, C.c_double,
                                           C.c_int, _dp]),
        "oracle_mesh_destroy": (None, [C.c_void_p]),
        "oracle_mesh_nelem": (C.c_int64, [C.c_void_p]),
        "oracle_node_coords": (None, [C.c_void_p, _dp]),
        "oracle_get_phi": (None, [C.c_void_p, _dp]),
        "oracle_set_phi": (None, [C.c_void_p, _dp]),
        "oracle_tables": (None, [C.c_void_p, _dp, _dp, _dp, _dp]),
        "oracle_logmean": (C.c_double, [C.c_double, C.c_double]),
        "oracle_euler_flux": (None, [C.c_int, _dp, C.c_double, C.c_double, _dp]),
        "oracle_two_point_flux": (None, [C.c_int, _dp, _dp, C.c_double, C.c_double,
                                         C.c_double, _dp]),
        "oracle_surface_flux": (None, [C.c_int, C.c_int, _dp, _dp, C.c_double, C.c_double,
                                       C.c_double, C.c_int, _dp]),
        "oracle_entropy_vars": (None, [_dp, C.c_double, C.c_double, _dp]),
        "oracle_entropy_density": (C.c_double, [_dp, C.c_double, C.c_double]),
        "oracle_rhs_terms": (C.c_int, [C.c_void_p, _dp, _dp, _dp, C.c_int]),
        "oracle_rhs": (C.c_int, [C.c_void_p, _dp, _dp]),
        "oracle_rhs_elems": (C.c_int, [C.c_void_p, _dp, _dp, _dp, C.c_int, _i64p, C.c_int64]),
        "oracle_rhs_strong": (C.c_int, [C.c_void_p, _dp, _dp]),
        "oracle_lsrk_coeffs": (None, [_dp, _dp, _dp]),
        "oracle_lsrk_step": (C.c_int, [C.c_void_p, _dp, _dp, C.c_double, C.c_double]),
        "oracle_lsrk_linear": (C.c_int, [C.c_int, _dp, _dp, C.c_double, C.c_int]),
        "oracle_lsrk_poly": (C.c_double, [C.c_int, C.c_double, C.c_double, C.c_double, C.c_int]),
        "oracle_entropy": (C.c_int, [C.c_void_p, _dp, _dp]),
        "oracle_cfl_dt": (C.c_double, [C.c_void_p, _dp, C.c_double]),
        "oracle_num_threads": (C.c_int, []),
        "oracle_set_num_threads": (None, [C.c_int]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()
_opc = None

# operation classes of op_count (one flop each)
OP_CLASSES = ("add", "mul", "div", "sqrt", "log")
OP_NODE, OP_FLUX, OP_GRAVITY, OP_SURFACE, OP_SOURCE, OP_UPDATE, OP_LOGMEAN = range(7)


def op_count(what, r=0, qa=(1.0, 0, 0, 0, 2.5), qb=(1.0, 0, 0, 0, 2.5), phia=0.0, phib=0.0,
             gamma=1.4, surf=SURF_RUSANOV):
    """Operation counts of one call of the oracle's pointwise physics
    (libopcount.so: esdg_pointwise.h compiled over a counting scalar).

    what: OP_NODE (per-node quantities of qa), OP_FLUX (two-point flux
    F_r(qa, qb)), OP_GRAVITY (its gravity term), OP_SURFACE (face flux of
    qa, qb for the normal +e_r and surface flux `surf`), OP_SOURCE (Coriolis
    source of qa with f = phia), OP_UPDATE (LSRK update of one value with
    A, B, dt, R = qa[0:4] and dq, q = qb[0:2]), OP_LOGMEAN ({{qa[0], qb[0]}}_log).
    Returns (counts, values): counts maps each of OP_CLASSES to its count,
    values the up to five numbers the call computed."""
    global _opc
    if _opc is None:
        _opc = C.CDLL(_build.OPC_LIB)
        _opc.oracle_op_count.restype = C.c_int
        _opc.oracle_op_count.argtypes = [C.c_int, C.c_int, _dp, _dp, C.c_double, C.c_double,
                                         C.c_double, C.c_int, C.POINTER(C.c_longlong), _dp]
    a, b = _vec(qa), _vec(qb)
    out = (C.c_longlong * 5)()
    res = np.zeros(5)
    rc = _opc.oracle_op_count(int(what), int(r), _ptr(a), _ptr(b), float(phia), float(phib),
                              float(gamma), int(surf), out, _ptr(res))
    assert rc == 0, what
    return dict(zip(OP_CLASSES, [int(x) for x in out])), res


def flops(counts) -> int:
    """Flops of an op_count result: every class counts one."""
    return sum(counts.values())


def _ptr(a):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _vec(x, n=5):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    assert a.size == n
    return a


def num_threads() -> int:
    return _lib.oracle_num_threads()


def set_num_threads(n: int) -> None:
    _lib.oracle_set_num_threads(int(n))


def lgl(N: int):
    """LGL nodes, weights and differentiation matrix of order N."""
    x = np.zeros(N + 1)
    w = np.zeros(N + 1)
    D = np.zeros((N + 1) * (N + 1))
    _lib.oracle_lgl(N, _ptr(x), _ptr(w), _ptr(D))
    return x, w, D.reshape(N + 1, N + 1)


def logmean(a: float, b: float) -> float:
    return _lib.oracle_logmean(a, b)


def euler_flux(r, q, phi, gamma=1.4):
    out = np.zeros(5)
    _lib.oracle_euler_flux(r, _ptr(_vec(q)), phi, gamma, _ptr(out))
    return out


def two_point_flux(r, qa, qb, phia, phib, gamma=1.4):
    out = np.zeros(5)
    _lib.oracle_two_point_flux(r, _ptr(_vec(qa)), _ptr(_vec(qb)), phia, phib, gamma, _ptr(out))
    return out


def surface_flux(r, s, qm, qp, phim, phip, gamma=1.4, surf=SURF_RUSANOV):
    out = np.zeros(5)
    _lib.oracle_surface_flux(r, s, _ptr(_vec(qm)), _ptr(_vec(qp)), phim, phip, gamma, surf,
                             _ptr(out))
    return out


def surface_flux_vec(Nv, qm, qp, phim, phip, gamma=1.4, surf=SURF_RUSANOV):
    out = np.zeros(5)
    _lib.oracle_surface_flux_vec(_ptr(_vec(Nv, 3)), _ptr(_vec(qm)), _ptr(_vec(qp)), phim, phip,
                                 gamma, surf, _ptr(out))
    return out


def entropy_vars(q, phi, gamma=1.4):
    out = np.zeros(5)
    _lib.oracle_entropy_vars(_ptr(_vec(q)), phi, gamma, _ptr(out))
    return out


def entropy_density(q, phi, gamma=1.4):
    return _lib.oracle_entropy_density(_ptr(_vec(q)), phi, gamma)


def lsrk_coeffs():
    A, B, Cc = np.zeros(5), np.zeros(5), np.zeros(5)
    _lib.oracle_lsrk_coeffs(_ptr(A), _ptr(B), _ptr(Cc))
    return A, B, Cc


def lsrk_linear(M, y0, dt, nsteps=1):
    M = np.ascontiguousarray(M, dtype=np.float64)
    y = np.ascontiguousarray(np.array(y0, dtype=np.float64))
    n = y.size
    assert M.shape == (n, n)
    rc = _lib.oracle_lsrk_linear(n, _ptr(M), _ptr(y), dt, nsteps)
    assert rc == 0
    return y


def lsrk_poly(m, t0, y0, dt, nsteps):
    return _lib.oracle_lsrk_poly(m, t0, y0, dt, nsteps)


class Mesh:
    """Uniform box of K[0] x K[1] x K[2] affine hexahedra of order N."""

    def __init__(self, N, K, lo, hi, periodic, gamma=1.4, gas_R=287.0, grav=9.81,
                 coriolis_f=0.0, surface_flux=SURF_RUSANOV, warp=None):
        self.N, self.Nq, self.Np = N, N + 1, (N + 1) ** 3
        self.K = tuple(int(k) for k in K)
        self.lo, self.hi = tuple(map(float, lo)), tuple(map(float, hi))
        self.periodic = tuple(int(bool(p)) for p in periodic)
        self.gamma, self.gas_R, self.grav, self.coriolis_f = gamma, gas_R, grav, coriolis_f
        self.surface_flux = surface_flux
        Ka = (C.c_int * 3)(*self.K)
        Pa = (C.c_int * 3)(*self.periodic)
        lo_a = (C.c_double * 3)(*self.lo)
        hi_a = (C.c_double * 3)(*self.hi)
        self.warp = None if warp is None else tuple(map(float, warp))
        if warp is None:
            self._h = _lib.oracle_mesh_create(N, Ka, lo_a, hi_a, Pa, gamma, gas_R, grav,
                                              coriolis_f, surface_flux)
        else:
            wa = (C.c_double * 3)(*self.warp)
            self._h = _lib.oracle_mesh_create_warped(N, Ka, lo_a, hi_a, Pa, gamma, gas_R, grav,
                                                     coriolis_f, surface_flux, wa)
        if not self._h:
            raise ValueError("oracle_mesh_create rejected the mesh description")
        self.ne = int(_lib.oracle_mesh_nelem(self._h))
        self.nn = self.ne * self.Np
        self.h = tuple((self.hi[d] - self.lo[d]) / self.K[d] for d in range(3))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.oracle_mesh_destroy(h)
            self._h = None

    @property
    def shape(self):
        return (self.ne, 5, self.Np)

    def zeros(self):
        return np.zeros(self.shape)

    def coords(self):
        xyz = np.zeros((self.ne, 3, self.Np))
        _lib.oracle_node_coords(self._h, _ptr(xyz))
        return xyz

    def metrics(self):
        """Curved meshes: (Ja [e][r][d][n], J [e][n]) -- J a^r_d and J."""
        assert self.warp is not None
        Ja = np.zeros((self.ne, 3, 3, self.Np))
        Jd = np.zeros((self.ne, self.Np))
        _lib.oracle_metrics(self._h, _ptr(Ja), _ptr(Jd))
        return Ja, Jd

    def phi(self):
        out = np.zeros((self.ne, self.Np))
        _lib.oracle_get_phi(self._h, _ptr(out))
        return out

    def set_phi(self, phi):
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        assert phi.shape == (self.ne, self.Np)
        _lib.oracle_set_phi(self._h, _ptr(phi))

    def tables(self):
        n = self.Nq
        xi, w, D, S = np.zeros(n), np.zeros(n), np.zeros(n * n), np.zeros(n * n)
        _lib.oracle_tables(self._h, _ptr(xi), _ptr(w), _ptr(D), _ptr(S))
        return xi, w, D.reshape(n, n), S.reshape(n, n)

    def _q(self, q):
        q = np.ascontiguousarray(q, dtype=np.float64)
        assert q.shape == self.shape, (q.shape, self.shape)
        return q

    def rhs(self, q, mask=TERM_ALL, gross=False):
        q = self._q(q)
        r = np.zeros(self.shape)
        g = np.zeros(self.shape) if gross else None
        _lib.oracle_rhs_terms(self._h, _ptr(q), _ptr(r), _ptr(g) if gross else None, mask)
        return (r, g) if gross else r

    def rhs_elems(self, q, elems, mask=TERM_ALL):
        """R and its gross scale for the listed elements only: (len, 5, Np) arrays."""
        q = self._q(q)
        elems = np.ascontiguousarray(np.asarray(elems, dtype=np.int64))
        r = np.zeros(self.shape)
        g = np.zeros(self.shape)
        _lib.oracle_rhs_elems(self._h, _ptr(q), _ptr(r), _ptr(g), mask,
                              elems.ctypes.data_as(_i64p), elems.size)
        return r[elems], g[elems]

    def rhs_strong(self, q):
        q = self._q(q)
        r = np.zeros(self.shape)
        _lib.oracle_rhs_strong(self._h, _ptr(q), _ptr(r))
        return r

    def lsrk_step(self, q, dq, t, dt):
        """In place on q (and dq)."""
        assert q.dtype == np.float64 and q.flags["C_CONTIGUOUS"] and q.shape == self.shape
        assert dq.dtype == np.float64 and dq.flags["C_CONTIGUOUS"] and dq.shape == self.shape
        rc = _lib.oracle_lsrk_step(self._h, _ptr(q), _ptr(dq), t, dt)
        assert rc == 0

    def run(self, q, dt, nsteps, t0=0.0):
        q = np.array(self._q(q))
        dq = np.zeros_like(q)
        for s in range(nsteps):
            self.lsrk_step(q, dq, t0 + s * dt, dt)
        return q

    def entropy(self, q):
        out = np.zeros(4)
        rc = _lib.oracle_entropy(self._h, _ptr(self._q(q)), _ptr(out))
        assert rc == 0
        return out

    def cfl_dt(self, q, cfl):
        return _lib.oracle_cfl_dt(self._h, _ptr(self._q(q)), cfl)
