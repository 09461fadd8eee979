"""Algorithmic work and traffic of the fused ES-DGSEM stage, and the MI355X
roofline it is measured against.

Algorithmic counts come from the formulas the kernels evaluate (each +, -,
*, /, sqrt and log counts one flop, an FMA two), not from executed
instructions:

  pair (x or y line, series branch of both log-means)   73 flops
      two log-means 11 + 11, f^rho 3, momentum 12, u_a.u_b 5,
      energy 11, accumulation into both nodes 20
  pair on a z line (adds the gravity term and its partner scaling) 87
  per-node precompute (primitives, rho/p, two logs, 1/z)            19
  face node (both states' primitives, log-means, flux, Rusanov
      dissipation, lift)                                             126
  per-node finish (phase sums, Coriolis, LSRK update)                 55

Pairs per node: 3N/2 (Nq(Nq-1)/2 pairs per line, Nq^2 lines per direction,
three directions, Nq^3 nodes).  Face nodes per node: 6/Nq.

Algorithmic HBM bytes per node and stage (FP64): read q and dq, write q_out
and dq (4 x 40 B) plus the neighbours' face traces (6 faces of Nq^2 nodes of
40 B per element: 240/Nq B per node).  The first of the five LSRK(5,4)
stages has A_1 = 0 and reads no dq, so a stage launch moves on average
(4 - 1/5) x 40 + 240/Nq B per node (200 B at N = 4).  One RHS evaluation
without the update moves 40 + 40 + 240/Nq B per node.
"""
from __future__ import annotations

import hashlib
import os
import re

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_VECTOR_TFLOPS = 78.6      # MI355X FP64 vector peak
FP32_VECTOR_TFLOPS = 157.3     # MI355X FP32 vector peak (packed)

PAIR_XY, PAIR_Z, PRECOMP, FACE_NODE, FINISH_STAGE, FINISH_RHS = 73, 87, 19, 126, 55, 20


def pairs_per_node(N: int) -> float:
    return 1.5 * N


def flops_per_node(N: int, stage: bool = True) -> float:
    Nq = N + 1
    pair = (2 * PAIR_XY + PAIR_Z) / 3.0
    return (pair * pairs_per_node(N) + FACE_NODE * 6.0 / Nq + PRECOMP
            + (FINISH_STAGE if stage else FINISH_RHS))


def bytes_per_node(N: int, stage: bool = True, word: int = 8) -> float:
    Nq = N + 1
    own = (4.0 - 0.2 if stage else 2.0) * 5 * word
    return own + 6.0 * 5 * word / Nq


# Curved hexahedra: per node the metric terms J a^r_d (9 words), 1/J and phi
# are read once per stage (each phase reads the three J a^r of its own
# direction).
CURVED_GEOM_WORDS = 11


def bytes_per_node_curved(N: int, stage: bool = True, word: int = 8) -> float:
    return bytes_per_node(N, stage, word) + CURVED_GEOM_WORDS * word


def ridge_fp64() -> float:
    return FP64_VECTOR_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)


_SRC_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")


def _code_only(text: str) -> str:
    """Source text without comments and whitespace (string literals in the
    kernels hold no comment markers)."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return re.sub(r"\s+", "", text)


# Sources the FP64 stage kernel is built from (the mixed-precision kernel
# lives in esdg_mixed.hpp and does not change it).
FP64_STAGE_SOURCES = ("esdg_api.hip", "esdg_device.hpp")


def kernel_sources(kernel_name: str):
    """The sources a stage kernel is built from: the FP64 kernel's, plus the
    curved or mixed-precision kernel's own header."""
    if "stage_curved" in kernel_name:
        return FP64_STAGE_SOURCES + ("esdg_curved.hpp",)
    if "stage_mixed" in kernel_name:
        return FP64_STAGE_SOURCES + ("esdg_mixed.hpp",)
    return FP64_STAGE_SOURCES


def kernel_source_hash(src_dir: str = _SRC_DIR, names=FP64_STAGE_SOURCES) -> str:
    """Hash of the code of the FP64 stage kernel's sources (comments and
    whitespace ignored): hardware counters taken for an older kernel are not
    reported for the current one."""
    h = hashlib.sha256()
    for name in sorted(names):
        if name.endswith((".hip", ".hpp")):
            with open(os.path.join(src_dir, name), encoding="utf-8") as f:
                h.update(name.encode())
                h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]
