"""Thin ctypes binding of libesdg.so (the gfx950 ES-DGSEM library).

Argument marshalling only: every step of the right-hand side and of the
time step runs in the library's HIP kernels.  PyTorch provides device
memory and the stream.  There is no fallback: if the library is missing
or fails to load, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libesdg.so")

ESDG_OK, ESDG_EINVAL, ESDG_ENOMEM, ESDG_EHIP, ESDG_ENONPHYS, ESDG_ENOTIMPL = 0, -1, -2, -3, -4, -5
SURF_RUSANOV, SURF_EC, SURF_MATRIX = 0, 1, 2
FP64, FP32_MIXED = 0, 1
TERM_VOL, TERM_FACE, TERM_SRC, TERM_ALL = 1, 2, 4, 7


class EsdgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"esdg error {code}: {msg}")
        self.code = code


class NonPhysicalState(EsdgError):
    pass


class MeshDesc(C.Structure):
    _fields_ = [
        ("N", C.c_int32),
        ("K", C.c_int32 * 3),
        ("lo", C.c_double * 3),
        ("hi", C.c_double * 3),
        ("periodic", C.c_int32 * 3),
        ("gamma", C.c_double),
        ("gas_R", C.c_double),
        ("grav", C.c_double),
        ("coriolis_f", C.c_double),
        ("surface_flux", C.c_int32),
        ("precision", C.c_int32),
        ("ref_rho", C.c_void_p),
        ("ref_p", C.c_void_p),
        ("epw", C.c_int32),
        ("curved", C.c_int32),
        ("warp", C.c_double * 3),
    ]


_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)

# name -> (restype, argtypes); every function that include/esdg.h declares
SIGNATURES = {
    "esdg_mesh_create": (C.c_int, [C.POINTER(MeshDesc), C.c_void_p, C.POINTER(C.c_void_p)]),
    "esdg_mesh_destroy": (C.c_int, [C.c_void_p]),
    "esdg_mesh_info": (C.c_int, [C.c_void_p, _i64p, _i64p, _i64p, _i64p]),
    "esdg_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "esdg_set_epw": (C.c_int, [C.c_void_p, C.c_int32]),
    "esdg_get_epw": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "esdg_node_coords": (C.c_int, [C.c_void_p, C.c_void_p]),
    "esdg_rhs": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double]),
    "esdg_rhs_terms": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    "esdg_lsrk_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_double]),
    "esdg_lsrk_step_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                         C.c_double]),
    "esdg_lsrk_run": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_double,
                                C.c_int32]),
    "esdg_entropy": (C.c_int, [C.c_void_p, C.c_void_p, _dp]),
    "esdg_cfl_dt": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, _dp]),
    "esdg_check": (C.c_int, [C.c_void_p]),
    "esdg_last_error": (C.c_char_p, []),
    "esdg_version": (C.c_char_p, []),
    "esdg_lgl_tables": (C.c_int, [C.c_int32, _dp, _dp, _dp]),
    "esdg_copy": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "esdg_epw_options": (C.c_int, [C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.c_int32]),
    "esdg_pack_create": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p)]),
    "esdg_pack_destroy": (C.c_int, [C.c_void_p]),
    "esdg_pack_set_members": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p),
                                        C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                        C.POINTER(C.c_void_p), _dp, C.POINTER(C.c_int32)]),
    "esdg_pack_step": (C.c_int, [C.c_void_p, C.c_int32]),
    "esdg_pack_flags": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "esdg_pack_flags_async": (C.c_int, [C.c_void_p, C.c_void_p]),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    # refuse a library built from other sources than the ones in this tree
    from . import build as _build
    version = lib.esdg_version().decode()
    want = _build.source_hash()
    have = version.rsplit("src:", 1)[-1] if "src:" in version else "none"
    if have != want:
        raise ImportError(f"{LIB_PATH} was built from other sources (library {have}, "
                          f"tree {want}): rebuild it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    return lib


lib = _load()


def last_error() -> str:
    return lib.esdg_last_error().decode()


def _check(rc):
    if rc != ESDG_OK:
        msg = last_error()
        if rc == ESDG_ENONPHYS:
            raise NonPhysicalState(rc, msg)
        raise EsdgError(rc, msg)


def lgl_tables(N: int):
    """Host-side LGL nodes, weights, derivative matrix of the library."""
    x, w, D = np.zeros(N + 1), np.zeros(N + 1), np.zeros((N + 1) * (N + 1))
    _check(lib.esdg_lgl_tables(N, x.ctypes.data_as(_dp), w.ctypes.data_as(_dp),
                               D.ctypes.data_as(_dp)))
    return x, w, D.reshape(N + 1, N + 1)


def epw_options(N: int, precision: int = FP64):
    """Elements-per-workgroup values compiled for order N and a precision."""
    n = lib.esdg_epw_options(N, precision, None, 0)
    if n < 0:
        _check(n)
    buf = (C.c_int32 * max(n, 1))()
    lib.esdg_epw_options(N, precision, buf, n)
    return [buf[i] for i in range(n)]


def copy(src, dst):
    """dst <- src (same-size float64 CUDA tensors) with the library's copy kernel."""
    torch = _torch()
    assert src.dtype == dst.dtype == torch.float64 and src.numel() == dst.numel()
    assert src.is_contiguous() and dst.is_contiguous()
    _check(lib.esdg_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), src.numel(),
                         C.c_void_p(torch.cuda.current_stream().cuda_stream)))


def _torch():
    import torch
    return torch


class Mesh:
    """A box mesh on the current HIP device, bound to torch's current stream
    at every call.  States are torch float64 CUDA tensors of shape
    (n_elem, 5, (N+1)^3)."""

    def __init__(self, spec, precision: int = FP64, ref_rho=None, ref_p=None, epw: int = 0):
        torch = _torch()
        self.spec = spec
        d = MeshDesc()
        d.N = spec.N
        d.K[:] = list(spec.K)
        d.lo[:] = list(spec.lo)
        d.hi[:] = list(spec.hi)
        d.periodic[:] = list(spec.periodic)
        d.gamma, d.gas_R, d.grav, d.coriolis_f = spec.gamma, spec.gas_R, spec.grav, spec.coriolis_f
        d.surface_flux = spec.surface_flux
        d.precision = precision
        self._refs = (ref_rho, ref_p)  # keep alive
        d.ref_rho = ref_rho.data_ptr() if ref_rho is not None else None
        d.ref_p = ref_p.data_ptr() if ref_p is not None else None
        d.epw = epw
        warp = getattr(spec, "warp", None)
        d.curved = 0 if warp is None else 1
        d.warp[:] = [0.0, 0.0, 0.0] if warp is None else [float(x) for x in warp]
        self._desc = d
        h = C.c_void_p()
        stream = torch.cuda.current_stream().cuda_stream
        _check(lib.esdg_mesh_create(C.byref(d), C.c_void_p(stream), C.byref(h)))
        self._h = h
        ne, nn, sl, fp = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib.esdg_mesh_info(h, C.byref(ne), C.byref(nn), C.byref(sl), C.byref(fp)))
        self.n_elem, self.n_nodes, self.state_len, self.footprint = ne.value, nn.value, sl.value, fp.value
        self.N, self.Np = spec.N, (spec.N + 1) ** 3
        self.precision = precision

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            lib.esdg_mesh_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        return (self.n_elem, 5, self.Np)

    def _bind(self):
        torch = _torch()
        _check(lib.esdg_set_stream(self._h, C.c_void_p(torch.cuda.current_stream().cuda_stream)))

    def _state(self, t, name):
        torch = _torch()
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
                and t.is_contiguous() and tuple(t.shape) == self.shape):
            raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of shape {self.shape}")
        return C.c_void_p(t.data_ptr())

    def empty(self):
        torch = _torch()
        return torch.empty(self.shape, dtype=torch.float64, device="cuda")

    def set_epw(self, epw: int):
        _check(lib.esdg_set_epw(self._h, epw))

    @property
    def epw(self) -> int:
        v = C.c_int32()
        _check(lib.esdg_get_epw(self._h, C.byref(v)))
        return v.value

    def coords(self):
        torch = _torch()
        xyz = torch.empty((self.n_elem, 3, self.Np), dtype=torch.float64, device="cuda")
        self._bind()
        _check(lib.esdg_node_coords(self._h, C.c_void_p(xyz.data_ptr())))
        return xyz

    def rhs(self, q, out=None, t: float = 0.0):
        out = self.empty() if out is None else out
        self._bind()
        _check(lib.esdg_rhs(self._h, self._state(q, "q"), self._state(out, "out"), t))
        return out

    def rhs_terms(self, q, mask: int, out=None):
        out = self.empty() if out is None else out
        self._bind()
        _check(lib.esdg_rhs_terms(self._h, self._state(q, "q"), self._state(out, "out"), mask))
        return out

    def lsrk_step(self, q, dq, dt: float, t: float = 0.0):
        self._bind()
        _check(lib.esdg_lsrk_step(self._h, self._state(q, "q"), self._state(dq, "dq"), t, dt))

    def lsrk_step_noalloc(self, q, dq, dt: float, t: float = 0.0):
        """lsrk_step with the library's per-device scratch array in place of
        the mesh's ping-pong buffer (no device allocation)."""
        self._bind()
        _check(lib.esdg_lsrk_step_noalloc(self._h, self._state(q, "q"), self._state(dq, "dq"),
                                          t, dt))

    def lsrk_run(self, q, dq, dt: float, nsteps: int, t0: float = 0.0):
        self._bind()
        _check(lib.esdg_lsrk_run(self._h, self._state(q, "q"), self._state(dq, "dq"), t0, dt,
                                 nsteps))

    def entropy(self, q):
        out = np.zeros(4)
        self._bind()
        _check(lib.esdg_entropy(self._h, self._state(q, "q"), out.ctypes.data_as(_dp)))
        return out

    def cfl_dt(self, q, cfl: float) -> float:
        dt = C.c_double()
        self._bind()
        _check(lib.esdg_cfl_dt(self._h, self._state(q, "q"), cfl, C.byref(dt)))
        return dt.value

    def check(self):
        self._bind()
        _check(lib.esdg_check(self._h))


class Pack:
    """Packed multi-member LSRK stepping on one stream (ensemble serving).

    Members share N, precision and elements per workgroup.  Each member i
    has two state buffers (q0[i], q1[i]); after k steps its state is in
    buffer parity[i] ^ (k & 1)."""

    def __init__(self, stream=None):
        torch = _torch()
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        _check(lib.esdg_pack_create(C.c_void_p(self._stream.cuda_stream), C.byref(h)))
        self._h = h
        self._keep = None
        self.n = 0

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            lib.esdg_pack_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_members(self, meshes, q0, q1, dq, dts, parity):
        n = len(meshes)
        arr = lambda T, vals: (T * n)(*vals)
        mh = arr(C.c_void_p, [m._h.value for m in meshes])
        for m, a, b, d in zip(meshes, q0, q1, dq):
            m._state(a, "q0")
            m._state(b, "q1")
            m._state(d, "dq")
        p0 = arr(C.c_void_p, [t.data_ptr() for t in q0])
        p1 = arr(C.c_void_p, [t.data_ptr() for t in q1])
        pd = arr(C.c_void_p, [t.data_ptr() for t in dq])
        dt = (C.c_double * n)(*[float(x) for x in dts])
        par = arr(C.c_int32, [int(x) for x in parity])
        _check(lib.esdg_pack_set_members(self._h, n, mh, p0, p1, pd, dt, par))
        self._keep = (list(meshes), list(q0), list(q1), list(dq))
        self.n = n

    def step(self, nsteps: int = 1):
        _check(lib.esdg_pack_step(self._h, nsteps))

    def flags(self):
        """Per member (in set_members order): True if it met a non-physical
        state since the last read (the flags are cleared).  Synchronises the
        pack's stream."""
        buf = (C.c_int32 * max(self.n, 1))()
        _check(lib.esdg_pack_flags(self._h, buf))
        return [bool(buf[i]) for i in range(self.n)]

    def flags_async(self, out):
        """Enqueue the flag gathering into `out`, a pinned host int32 torch
        tensor of at least n entries, on the pack's stream (no
        synchronisation): out[:n] holds the flags once the stream has passed
        this call."""
        torch = _torch()
        if not (isinstance(out, torch.Tensor) and out.dtype == torch.int32 and not out.is_cuda
                and out.is_contiguous() and out.numel() >= self.n):
            raise ValueError("out must be a contiguous host int32 tensor of at least n entries")
        _check(lib.esdg_pack_flags_async(self._h, C.c_void_p(out.data_ptr())))
