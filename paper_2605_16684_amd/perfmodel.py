"""Algorithmic work and traffic of the fused ES-DGSEM stage, and the MI355X
roofline it is measured against.

Algorithmic flops are the operation counts of the oracle's own pointwise
physics (each +, -, *, /, sqrt and log one flop; the oracle has no FMA),
mapped onto the work a node, a node pair and a face node need once:

  PRECOMP    = C_node                                   per node: u, p, rho/p, b
  PAIR_XY    = C_flux - 2 C_node - C_grav + SCATTER     unordered pair, x or y line
  PAIR_Z     = C_flux - 2 C_node + C_grav + SCATTER     unordered pair, z line
  FACE_NODE  = C_face - C_node - C_grav + LIFT          face node, Rusanov
  FINISH     = 5 C_update + C_source + PHASE            per node, stage
  FINISH_RHS = C_source + PHASE                         per node, RHS only

with C_node the per-node quantities of the two-point flux, C_flux one
two-point flux evaluation (series branch of both log-means), C_grav its
gravity term with the addition into the normal momentum, C_face one face
flux with Rusanov dissipation, C_update one value of the LSRK stage update
and C_source the Coriolis source of one node.  The flux evaluates both
nodes' quantities, which a node needs only once (the precompute); a pair of
an x or y line has no gravity term (phi is constant along it), and on a z
line the partner's flux differs from the own node's only in its gravity
term; at a face the own node's quantities come from the precompute and the
geopotential is continuous.  The kernel-structure terms are
  SCATTER = 20  a pair's flux into both nodes' sums: 2 x 5 x (mul + add)
  LIFT    = 10  a face flux into its node's sum: 5 x (mul + add)
  PHASE   = 25  per node the three directions' sums, each scaled by 2/h_r
                and added: 5 x (3 mul + 2 add).
tests/test_perfmodel_counts.py recomputes every constant from the oracle's
operation counter (oracle_op_count) through this mapping.

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

# oracle operation counts (series branch of both log-means) and the mapping above
C_NODE, C_FLUX, C_GRAV, C_FACE, C_UPDATE, C_SOURCE = 18, 104, 8, 163, 5, 4
SCATTER, LIFT, PHASE = 20, 10, 25
PRECOMP = C_NODE
PAIR_XY = C_FLUX - 2 * C_NODE - C_GRAV + SCATTER
PAIR_Z = C_FLUX - 2 * C_NODE + C_GRAV + SCATTER
FACE_NODE = C_FACE - C_NODE - C_GRAV + LIFT
FINISH_STAGE = 5 * C_UPDATE + C_SOURCE + PHASE
FINISH_RHS = C_SOURCE + PHASE


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
