// esdg_high.hpp -- FP64 stage kernels for orders N = 9..15 on the affine box.
//
// The line-per-lane kernel of esdg_device.hpp holds a whole LGL line (its
// primitives and sums) in one lane's registers; from N = 9 on that no longer
// fits.  These orders take a node-per-thread path instead, in two launches
// per stage (or RHS):
//   1. prim_kernel: every node's primitives (rho, u/2, p/2, rho/p, p/rho,
//      the quantities of the two-point flux, Sec. 4.1) into a per-mesh
//      buffer prim[e][7][n] (56 B per node);
//   2. stage_high_kernel: one thread per node evaluates the same semi-discrete
//      right-hand side as the fused kernel -- for each direction r the full
//      sweep over the node's r-line partners b != a, T_ab (S_ab + G_ab) with
//      the entropy-conservative flux and the gravity term, the face flux and
//      lift where the node lies on a face, the Coriolis source -- and writes
//      R or applies the LSRK(5,4) stage update.
// The partners' primitives come from the prim buffer (L2); each ordered
// pair is evaluated by both of its nodes (no flux-symmetry saving: a thread
// owns one node's sum).  Log-means take the branch rule of the fused kernel
// with logarithms only on the log branch.
#pragma once

#include "esdg_device.hpp"

namespace esdg {

constexpr int HIGH_THREADS = 256;
constexpr int PRIM_VARS = 7;  // r, h0, h1, h2, hp, z, zi

__device__ __forceinline__ double phi_node(const StageParams &P, const OrderTables &tb, int ez,
                                           int k)
{
    const double dz = P.zhi - P.zlo;
    const double ZL = P.zlo + dz * ((double)ez / (double)P.K[2]);
    const double ZR = P.zlo + dz * ((double)(ez + 1) / (double)P.K[2]);
    const double s = tb.xi[k];
    return P.grav * (0.5 * (1.0 - s) * ZL + 0.5 * (1.0 + s) * ZR);
}

// Primitives of every node of q_in.
__global__ void __launch_bounds__(HIGH_THREADS)
    prim_kernel(const StageParams P, int N, double *__restrict__ prim)
{
    const int NQ = N + 1, NP = NQ * NQ * NQ;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= P.ne * NP) return;
    const int64_t e = gid / NP;
    const int n = (int)(gid - e * NP);
    const int ez = (int)(e / ((int64_t)P.K[0] * P.K[1]));
    const OrderTables &tb = c_tab[N - 1];
    Cons c;
    load_cons(P.q_in, e, NP, n, c);
    const Node nd = primitives(c, phi_node(P, tb, ez, n / (NQ * NQ)), P.gamma - 1.0);
    double *o = prim + e * PRIM_VARS * NP + n;
    o[0] = nd.r;
    o[NP] = nd.h0;
    o[2 * NP] = nd.h1;
    o[3 * NP] = nd.h2;
    o[4 * NP] = nd.hp;
    o[5 * NP] = nd.z;
    o[6 * NP] = nd.zi;
}

__device__ __forceinline__ Node load_prim(const double *__restrict__ prim, int64_t e, int NP,
                                          int n)
{
    const double *p = prim + e * PRIM_VARS * NP + n;
    Node nd;
    nd.r = p[0];
    nd.h0 = p[NP];
    nd.h1 = p[2 * NP];
    nd.h2 = p[3 * NP];
    nd.hp = p[4 * NP];
    nd.z = p[5 * NP];
    nd.zi = p[6 * NP];
    return nd;
}

// {{x}}_log and 1/{{x}}_log of one pair with the branch rule of the fused
// kernel, logarithms (of x scaled by `scale`) only on the log branch.
__device__ __forceinline__ double log_mean_lazy(double xa, double xb)
{
    const double d = xb - xa, s = xa + xb;
    const bool ser = fabs(d) < LM_SQRT_EPS * s;
    double den = s;
    if (!ser) den = log(xb) - log(xa);
    const double x = fdiv(d, den);
    const double u = x * x;
    return ser ? 0.5 * s * (1.0 - u * (S1 + u * (S2 + u * S3))) : x;
}

__device__ __forceinline__ double inv_log_mean_lazy(double xa, double xb, double scale)
{
    const double d = xb - xa, s = xa + xb;
    const bool ser = fabs(d) < LM_SQRT_EPS * s;
    double num = 1.0, den = s;
    if (!ser) {
        num = log(xb * scale) - log(xa * scale);
        den = d;
    }
    const double x = fdiv(num, den);
    const double dx = d * x;
    const double u = dx * dx;
    return ser ? 2.0 * x * (1.0 + u * (I1 + u * (I2 + u * I3))) : x;
}

// Node of the r-line through node (i, j, k) at position t.
template <int R>
__device__ __forceinline__ int line_pos_node(int NQ, int i, int j, int k, int t)
{
    if (R == 0) return t + NQ * (j + NQ * k);
    if (R == 1) return i + NQ * (t + NQ * k);
    return i + NQ * (j + NQ * t);
}

// Sum over direction R of the node's volume pairs and, on a face, its face
// flux (unscaled: the caller multiplies by 2/h_R).
template <int R>
__device__ __forceinline__ void node_terms(const StageParams &P, const OrderTables &tb, int N,
                                           const double *__restrict__ prim, int64_t e,
                                           const int ec[3], int i, int j, int k,
                                           const Node &a, const Cons &qa, double phi_a,
                                           double acc[5])
{
    const int NQ = N + 1, NP = NQ * NQ * NQ;
    const int ia = R == 0 ? i : (R == 1 ? j : k);
    const double gm1i = P.gm1i;
#pragma unroll
    for (int v = 0; v < 5; ++v) acc[v] = 0.0;
    if (P.mask & TERM_FACE) {
        for (int side = 0; side < 2; ++side) {
            if (ia != (side ? N : 0)) continue;
            int nb = ec[R] + (side ? 1 : -1);
            const bool wall = (nb < 0 || nb >= P.K[R]) && !P.periodic[R];
            Cons qp;
            if (!wall) {
                if (nb < 0) nb += P.K[R];
                if (nb >= P.K[R]) nb -= P.K[R];
                int cc[3] = {ec[0], ec[1], ec[2]};
                cc[R] = nb;
                const int64_t en = cc[0] + (int64_t)P.K[0] * (cc[1] + (int64_t)P.K[1] * cc[2]);
                load_cons(P.q_in, en, NP, line_pos_node<R>(NQ, i, j, k, side ? 0 : N), qp);
            } else {
                qp = qa;
                qp.v[1 + R] = -qp.v[1 + R];
            }
            double Fn[5];
            face_flux<R>(a, qa, qp, phi_a, side ? 1.0 : -1.0, P, Fn);
            const double wi = tb.winv[ia];
#pragma unroll
            for (int v = 0; v < 5; ++v) acc[v] -= wi * Fn[v];
        }
    }
    if (!(P.mask & TERM_VOL)) return;
    const int ez = ec[2];
    for (int t = 0; t < NQ; ++t) {
        if (t == ia) continue;
        const Node b = load_prim(prim, e, NP, line_pos_node<R>(NQ, i, j, k, t));
        const double phi_b = R == 2 ? phi_node(P, tb, ez, t) : phi_a;
        const double rho_ln = log_mean_lazy(a.r, b.r);
        const double izln = inv_log_mean_lazy(a.z, b.z, P.lnz_scale);
        const double hRa = hcomp<R>(a), hRb = hcomp<R>(b);
        const double frho = rho_ln * (hRa + hRb);
        double S[5];
        S[0] = frho;
        S[1] = frho * (a.h0 + b.h0);
        S[2] = frho * (a.h1 + b.h1);
        S[3] = frho * (a.h2 + b.h2);
        S[1 + R] += a.hp + b.hp;
        const double hh = a.h0 * b.h0 + a.h1 * b.h1 + a.h2 * b.h2;
        const double cross = a.hp * hRb + b.hp * hRa;
        S[4] = frho * (izln * gm1i + 2.0 * hh + 0.5 * (phi_a + phi_b)) + 2.0 * cross;
        const double tab = tb.T[ia][t];
#pragma unroll
        for (int v = 0; v < 5; ++v) acc[v] -= tab * S[v];
        if (R == 2) {
            // own share of the gravity term, rho_hat = {{b}} {{rho}}_log / b_a
            const double X = 0.25 * rho_ln * (a.z + b.z) * (phi_b - phi_a);
            acc[3] -= tab * (X * a.zi);
        }
    }
}

template <int MODE>
__global__ void __launch_bounds__(HIGH_THREADS)
    stage_high_kernel(const StageParams P, int N, const double *__restrict__ prim)
{
    const int NQ = N + 1, NQ2 = NQ * NQ, NP = NQ2 * NQ;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= P.ne * NP) return;
    const int64_t e = gid / NP;
    const int n = (int)(gid - e * NP);
    const int i = n % NQ, j = (n / NQ) % NQ, k = n / NQ2;
    int ec[3];
    ec[0] = (int)(e % P.K[0]);
    ec[1] = (int)((e / P.K[0]) % P.K[1]);
    ec[2] = (int)(e / ((int64_t)P.K[0] * P.K[1]));
    const OrderTables &tb = c_tab[N - 1];
    Cons qa;
    load_cons(P.q_in, e, NP, n, qa);
    const Node a = load_prim(prim, e, NP, n);
    const double phi_a = phi_node(P, tb, ec[2], k);
    double Rv[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (P.mask & (TERM_VOL | TERM_FACE)) {
        double acc[5];
        node_terms<0>(P, tb, N, prim, e, ec, i, j, k, a, qa, phi_a, acc);
#pragma unroll
        for (int v = 0; v < 5; ++v) Rv[v] += P.two_h[0] * acc[v];
        node_terms<1>(P, tb, N, prim, e, ec, i, j, k, a, qa, phi_a, acc);
#pragma unroll
        for (int v = 0; v < 5; ++v) Rv[v] += P.two_h[1] * acc[v];
        node_terms<2>(P, tb, N, prim, e, ec, i, j, k, a, qa, phi_a, acc);
#pragma unroll
        for (int v = 0; v < 5; ++v) Rv[v] += P.two_h[2] * acc[v];
    }
    if (P.mask & TERM_SRC) {
        Rv[1] += P.cor_f * qa.v[2];
        Rv[2] -= P.cor_f * qa.v[1];
    }
    const int64_t o = e * 5 * NP + n;
    if (MODE == MODE_RHS) {
#pragma unroll
        for (int v = 0; v < 5; ++v) store_f64<true>(&P.r_out[o + v * NP], Rv[v]);
    } else {
        const bool use_dq = P.A != 0.0;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            const double d = use_dq ? P.A * P.dq[o + v * NP] + P.dt * Rv[v] : P.dt * Rv[v];
            P.dq[o + v * NP] = d;
            P.q_out[o + v * NP] = qa.v[v] + P.B * d;
        }
    }
    if (P.flag) {
        const double r = qa.v[0];
        const double kin = qa.v[1] * qa.v[1] + qa.v[2] * qa.v[2] + qa.v[3] * qa.v[3];
        const double eint = qa.v[4] - 0.5 * kin / r - r * phi_a;
        if (!(r > 0.0) || !(eint > 0.0)) atomicOr(P.flag, 1);
    }
}

}  // namespace esdg
