"""Checkpoint and resume of a time integration (host files, no pickling).

A checkpoint holds everything needed to continue an LSRK(5,4) run exactly:
the state q and the LSRK register dq (both in the boundary layout
q[e][v][n], FP64), the time t, the step count, the time step dt, the
precision mode and the mesh description.  The kernels are deterministic, so
a run resumed from a checkpoint reproduces the uninterrupted run bit for
bit (the step itself does not read dq on entry, since the first LSRK stage
has A_1 = 0; dq is kept so that the file is the whole integrator state).

Files are numpy .npz archives whose arrays are plain float64 data plus one
JSON string; loading uses numpy without pickle.
"""
from __future__ import annotations

import dataclasses
import json
from typing import Optional

import numpy as np

from . import workloads as W

FORMAT = "esdg-checkpoint-1"


def _to_host(a):
    if type(a).__module__.startswith("torch"):
        return a.detach().cpu().numpy()
    return np.asarray(a)


def save(path: str, spec: W.MeshSpec, q, dq, t: float, step: int, dt: float,
         precision: int = 0, ref_rho=None, ref_p=None) -> None:
    """Write the integrator state to `path` (.npz).  q, dq (and, for the
    FP32-mixed mode, the reference ref_rho, ref_p) may be numpy arrays or
    torch tensors on any device; they are copied to the host."""
    meta = {"format": FORMAT, "t": float(t), "step": int(step), "dt": float(dt),
            "precision": int(precision), "spec": dataclasses.asdict(spec)}
    arrays = {"q": _to_host(q).astype(np.float64, copy=False),
              "dq": _to_host(dq).astype(np.float64, copy=False),
              "meta": np.array(json.dumps(meta))}
    if ref_rho is not None:
        arrays["ref_rho"] = _to_host(ref_rho).astype(np.float64, copy=False)
        arrays["ref_p"] = _to_host(ref_p).astype(np.float64, copy=False)
    with open(path, "wb") as fh:
        np.savez(fh, **arrays)


@dataclasses.dataclass
class Checkpoint:
    spec: W.MeshSpec
    q: np.ndarray
    dq: np.ndarray
    t: float
    step: int
    dt: float
    precision: int
    ref_rho: Optional[np.ndarray] = None
    ref_p: Optional[np.ndarray] = None


def load(path: str) -> Checkpoint:
    """Read a checkpoint written by save() (host numpy arrays)."""
    with np.load(path, allow_pickle=False) as z:
        meta = json.loads(str(z["meta"]))
        if meta.get("format") != FORMAT:
            raise ValueError(f"{path}: not an {FORMAT} file")
        sp = dict(meta["spec"])
        for k in ("K", "lo", "hi", "periodic"):
            sp[k] = tuple(sp[k])
        if sp.get("warp") is not None:
            sp["warp"] = tuple(sp["warp"])
        spec = W.MeshSpec(**sp)
        ck = Checkpoint(spec=spec, q=np.array(z["q"]), dq=np.array(z["dq"]), t=meta["t"],
                        step=meta["step"], dt=meta["dt"], precision=meta["precision"])
        if "ref_rho" in z.files:
            ck.ref_rho = np.array(z["ref_rho"])
            ck.ref_p = np.array(z["ref_p"])
    Np = (spec.N + 1) ** 3
    ne = spec.K[0] * spec.K[1] * spec.K[2]
    if ck.q.shape != (ne, 5, Np) or ck.dq.shape != ck.q.shape:
        raise ValueError(f"{path}: state shape {ck.q.shape} does not match the mesh "
                         f"({ne}, 5, {Np})")
    return ck
