// esdg_high.hpp -- FP64 stage kernels for orders N = 9..15 on the affine box.
//
// The line-per-lane kernel of esdg_device.hpp holds a whole LGL line (its
// primitives and sums) in one lane's registers; from N = 9 on that no longer
// fits.  These orders take a node-per-thread path instead: one thread per
// node evaluates the same semi-discrete right-hand side as the fused kernel
// -- for each direction r the full sweep over the node's r-line partners
// b != a, T_ab (S_ab + G_ab) with the entropy-conservative flux and the
// gravity term, the face flux and lift where the node lies on a face, the
// Coriolis source -- and writes R or applies the LSRK(5,4) stage update.
// Each ordered pair is evaluated by both of its nodes (no flux-symmetry
// saving: a thread owns one node's sum).  Log-means take the branch rule of
// the fused kernel, with the per-node logarithms on the log branch; in the
// LDS kernel, waves whose lines all stay inside the series range take the
// series-only flux.
//
// The partners' primitives (rho, u/2, p/2, rho/p: the quantities of the
// two-point flux, Sec. 4.1) are formed once per node and per stage:
//   - stage_high_lds: one workgroup per element; the element's partner
//     quantities (with the per-node logarithms up to N = 12: 64 B per node;
//     without them, taken per pair on the log branch, at N = 13, 14: 48 B)
//     go to LDS, then every thread sweeps its nodes' lines out of LDS.  Used
//     where the element fits the workgroup's LDS (N <= 14 on gfx950).
//   - prim_kernel + stage_high_kernel: otherwise, a per-mesh buffer
//     prim[e][9][n] (72 B per node) written by a first launch and read by the
//     node-per-thread launch through L2.
#pragma once

#include "esdg_device.hpp"

namespace esdg {

constexpr int HIGH_THREADS = 256;
// Per-node quantities of the partners: r, h0, h1, h2, hp, z and the
// logarithms ln(r), ln(z z_s^-1) of the log branch (the paper's per-node logs,
// Sec. 4.1), laid out [var][n] per element.  The prim buffer adds p/rho.
constexpr int PARTNER_VARS = 8;
constexpr int PRIM_VARS = 9;
// Orders whose element, logarithms included, fits gfx950's 160 KB of LDS per
// workgroup; up to N = 14 the LDS kernel holds the six quantities without the
// logarithms and takes them per pair on the log branch.
constexpr int HIGH_LDS_LOGS_MAX_N = 12;

__device__ __forceinline__ double phi_node(const StageParams &P, const OrderTables &tb, int ez,
                                           int k)
{
    const double dz = P.zhi - P.zlo;
    const double ZL = P.zlo + dz * ((double)ez / (double)P.K[2]);
    const double ZR = P.zlo + dz * ((double)(ez + 1) / (double)P.K[2]);
    const double s = tb.xi[k];
    return P.grav * (0.5 * (1.0 - s) * ZL + 0.5 * (1.0 + s) * ZR);
}

// The partner quantities of one node into an element block [var][NP], with
// or without the two logarithms.
__device__ __forceinline__ void store_partner(double *__restrict__ pb, int NP, const Node &nd,
                                              double lnz_scale, bool logs = true)
{
    pb[0] = nd.r;
    pb[NP] = nd.h0;
    pb[2 * NP] = nd.h1;
    pb[3 * NP] = nd.h2;
    pb[4 * NP] = nd.hp;
    pb[5 * NP] = nd.z;
    if (logs) {
        pb[6 * NP] = log(nd.r);
        pb[7 * NP] = log(nd.z * lnz_scale);
    }
}

// {{x}}_log and 1/{{x}}_log of one pair with the branch rule of the fused
// kernel, logarithms (of x scaled by `scale`) taken here on the log branch.
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

// Primitives and logarithms of every node of q_in.
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
    store_partner(o, NP, nd, P.lnz_scale);
    o[8 * NP] = nd.zi;
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
    nd.zi = p[8 * NP];
    return nd;
}

// Partner primitives from an element block laid out [var][NP] (global prim
// buffer or LDS); the partner's p/rho is not needed, its logarithms are read
// where a pair takes the log branch.
__device__ __forceinline__ Node load_partner(const double *__restrict__ pb, int NP, int n)
{
    Node nd;
    nd.r = pb[n];
    nd.h0 = pb[NP + n];
    nd.h1 = pb[2 * NP + n];
    nd.h2 = pb[3 * NP + n];
    nd.hp = pb[4 * NP + n];
    nd.z = pb[5 * NP + n];
    nd.zi = 0.0;
    return nd;
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
// flux (unscaled: the caller multiplies by 2/h_R).  lflag (or NULL) marks
// the lines of the element that can reach the log branch of a log-mean;
// where no line of the wave's nodes can, the pairs take the series-only flux.
template <int R, bool LOGS>
__device__ __forceinline__ void node_terms(const StageParams &P, const OrderTables &tb, int N,
                                           const double *__restrict__ pb,
                                           const unsigned char *lflag, const int ec[3], int i,
                                           int j, int k, const Node &a, const Cons &qa,
                                           double phi_a, double acc[5])
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
    if (lflag) {
        const int line = R == 0 ? j + NQ * k : (R == 1 ? i + NQ * k : i + NQ * j);
        if (__ballot(lflag[R * NQ * NQ + line] != 0) == 0) {
            // every pair of these lines takes the series branch of both log-means
            for (int t = 0; t < NQ; ++t) {
                if (t == ia) continue;
                const Node b = load_partner(pb, NP, line_pos_node<R>(NQ, i, j, k, t));
                const double phi_b = R == 2 ? phi_node(P, tb, ez, t) : phi_a;
                double S[5];
                const double rho_ln =
                    sym_flux_series<R>(a, b, 0.5 * (phi_a + phi_b), gm1i, S);
                const double tab = tb.T[ia][t];
#pragma unroll
                for (int v = 0; v < 5; ++v) acc[v] -= tab * S[v];
                if (R == 2) {
                    const double X = 0.25 * rho_ln * (a.z + b.z) * (phi_b - phi_a);
                    acc[3] -= tab * (X * a.zi);
                }
            }
            return;
        }
    }
    const int na = line_pos_node<R>(NQ, i, j, k, ia);
    const double lra = LOGS ? pb[6 * NP + na] : 0.0, lza = LOGS ? pb[7 * NP + na] : 0.0;
    for (int t = 0; t < NQ; ++t) {
        if (t == ia) continue;
        const int nb = line_pos_node<R>(NQ, i, j, k, t);
        const Node b = load_partner(pb, NP, nb);
        const double phi_b = R == 2 ? phi_node(P, tb, ez, t) : phi_a;
        double rho_ln, izln;
        if constexpr (LOGS) {
            rho_ln = log_mean(a.r, b.r, lra, pb[6 * NP + nb]);
            izln = inv_log_mean(a.z, b.z, lza, pb[7 * NP + nb]);
        } else {
            rho_ln = log_mean_lazy(a.r, b.r);
            izln = inv_log_mean_lazy(a.z, b.z, P.lnz_scale);
        }
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

// R at node n = (i, j, k) of element e (partner primitives in pb), then the
// RHS store or the LSRK stage update of that node, and the flag check.
template <int MODE, bool LOGS = true>
__device__ __forceinline__ void high_node(const StageParams &P, const OrderTables &tb, int N,
                                          const double *__restrict__ pb,
                                          const unsigned char *lflag, int64_t e,
                                          const int ec[3], int n, const Cons &qa, const Node &a)
{
    const int NQ = N + 1, NQ2 = NQ * NQ, NP = NQ2 * NQ;
    const int i = n % NQ, j = (n / NQ) % NQ, k = n / NQ2;
    const double phi_a = phi_node(P, tb, ec[2], k);
    double Rv[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (P.mask & (TERM_VOL | TERM_FACE)) {
        double acc[5];
        node_terms<0, LOGS>(P, tb, N, pb, lflag, ec, i, j, k, a, qa, phi_a, acc);
#pragma unroll
        for (int v = 0; v < 5; ++v) Rv[v] += P.two_h[0] * acc[v];
        node_terms<1, LOGS>(P, tb, N, pb, lflag, ec, i, j, k, a, qa, phi_a, acc);
#pragma unroll
        for (int v = 0; v < 5; ++v) Rv[v] += P.two_h[1] * acc[v];
        node_terms<2, LOGS>(P, tb, N, pb, lflag, ec, i, j, k, a, qa, phi_a, acc);
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

__device__ __forceinline__ void elem_coords(const StageParams &P, int64_t e, int ec[3])
{
    ec[0] = (int)(e % P.K[0]);
    ec[1] = (int)((e / P.K[0]) % P.K[1]);
    ec[2] = (int)(e / ((int64_t)P.K[0] * P.K[1]));
}

// Node-per-thread stage reading the partners from the prim buffer.
template <int MODE>
__global__ void __launch_bounds__(HIGH_THREADS)
    stage_high_kernel(const StageParams P, int N, const double *__restrict__ prim)
{
    const int NQ = N + 1, NP = NQ * NQ * NQ;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= P.ne * NP) return;
    const int64_t e = gid / NP;
    const int n = (int)(gid - e * NP);
    int ec[3];
    elem_coords(P, e, ec);
    const OrderTables &tb = c_tab[N - 1];
    Cons qa;
    load_cons(P.q_in, e, NP, n, qa);
    const Node a = load_prim(prim, e, NP, n);
    high_node<MODE>(P, tb, N, prim + e * PRIM_VARS * NP, nullptr, e, ec, n, qa, a);
}

// Partner quantities per node that stage_high_lds holds in LDS at order N.
__host__ __device__ inline int high_lds_vars(int N)
{
    return N <= HIGH_LDS_LOGS_MAX_N ? PARTNER_VARS : PARTNER_VARS - 2;
}

// Bytes of LDS stage_high_lds needs for one element of order N: the partner
// quantities, then one flag per line.
inline size_t high_lds_bytes(int N)
{
    const size_t nq = (size_t)(N + 1);
    return sizeof(double) * high_lds_vars(N) * nq * nq * nq + 3 * nq * nq;
}

// One workgroup per element: the element's partner quantities are formed
// once into LDS (with the logarithms when LOGS), the lines that can reach the
// log branch are marked, then each thread finishes its nodes n = tid,
// tid + THREADS, ...
template <int MODE, int THREADS, bool LOGS>
__device__ __forceinline__ void stage_high_lds_body(const StageParams &P, int N, int64_t e,
                                                    double *sprim)
{
    const int NQ = N + 1, NQ2 = NQ * NQ, NP = NQ2 * NQ;
    int ec[3];
    elem_coords(P, e, ec);
    const OrderTables &tb = c_tab[N - 1];
    const double gm1 = P.gamma - 1.0;
    for (int n = threadIdx.x; n < NP; n += THREADS) {
        Cons c;
        load_cons(P.q_in, e, NP, n, c);
        const Node nd = primitives(c, phi_node(P, tb, ec[2], n / NQ2), gm1);
        store_partner(sprim + n, NP, nd, P.lnz_scale, LOGS);
    }
    __syncthreads();
    // lines whose extreme pair leaves the series range of a log-mean (the
    // fused kernel's per-line test)
    unsigned char *sflag = reinterpret_cast<unsigned char *>(sprim + high_lds_vars(N) * NP);
    for (int l = threadIdx.x; l < 3 * NQ2; l += THREADS) {
        const int R = l / NQ2, li = l - R * NQ2;
        const int n0 = R == 0 ? NQ * li : (R == 1 ? li % NQ + NQ2 * (li / NQ) : li);
        const int st = R == 0 ? 1 : (R == 1 ? NQ : NQ2);
        double rmn = sprim[n0], rmx = rmn, zmn = sprim[5 * NP + n0], zmx = zmn;
        for (int t = 1; t < NQ; ++t) {
            const double r = sprim[n0 + t * st], z = sprim[5 * NP + n0 + t * st];
            rmn = fmin(rmn, r);
            rmx = fmax(rmx, r);
            zmn = fmin(zmn, z);
            zmx = fmax(zmx, z);
        }
        sflag[l] = (!(rmx - rmn < LM_SQRT_EPS_LINE * (rmx + rmn)) ||
                    !(zmx - zmn < LM_SQRT_EPS_LINE * (zmx + zmn))) ? 1 : 0;
    }
    __syncthreads();
    for (int n = threadIdx.x; n < NP; n += THREADS) {
        Cons qa;
        load_cons(P.q_in, e, NP, n, qa);
        const Node a = primitives(qa, phi_node(P, tb, ec[2], n / NQ2), gm1);
        high_node<MODE, LOGS>(P, tb, N, sprim, sflag, e, ec, n, qa, a);
    }
}

// The grid has one block per element; blocks are dealt to the XCDs so that
// each walks a contiguous range of elements.
template <int MODE, int THREADS, int WAVES>
__global__ void __launch_bounds__(THREADS, WAVES) stage_high_lds(const StageParams P, int N)
{
    extern __shared__ double sprim[];  // [high_lds_vars(N)][NP], then the line flags
    const int64_t e = xcd_remap(blockIdx.x, P.nblocks);
    if (N <= HIGH_LDS_LOGS_MAX_N)
        stage_high_lds_body<MODE, THREADS, true>(P, N, e, sprim);
    else
        stage_high_lds_body<MODE, THREADS, false>(P, N, e, sprim);
}

}  // namespace esdg
