// esdg_mixed.hpp -- FP32-mixed variant of the fused ES-DGSEM stage kernel.
//
// The right-hand side is split exactly as R(q) = R(q_r) + R'(q), where q_r is
// a hydrostatic reference state at rest (rho_r, u = 0, p_r).  For a state at
// rest the two-point flux reduces to the pressure-gravity momentum term, so
// R(q_r) holds only that term; it is evaluated once in FP64 by the FP64
// kernel and stored (momentum components, FP32).  R'(q) is the ES-DGSEM
// right-hand side with the normal-momentum pair term
//     {{p}} + rho_hat [[phi]]/2
// replaced by its deviation from the reference,
//     {{p'}} + (rho_hat - rho_hat_r) [[phi]]/2,   p' = p - p_r,
// and the face pressure {{p}} by {{p'}} -- the identity
//     {{p}} + G = ({{p_r}} + G_r) + {{p'}} + (G - G_r)
// is exact, so R = R(q_r) + R' holds for any reference.  FP64 is kept where
// cancellation would otherwise destroy the perturbation: p', rho' and the
// relative b perturbation beta = b/b_r - 1 are formed per node in FP64 from
// the FP64 state; rho_hat - rho_hat_r is then evaluated from those
// perturbations (no difference of two nearly equal FP32 numbers); face jumps
// q+ - q- are formed in FP64; the LSRK accumulation is FP64.  Everything
// else -- log-means, fluxes, dissipation, accumulation -- is FP32 with the
// hardware reciprocal and logarithm.
#pragma once

#include "esdg_device.hpp"

namespace esdg {

struct MixedParams {
    StageParams s;          // geometry, coefficients, FP64 state pointers
    const float *ref_r;     // [e][n] reference density (FP32 values)
    const float *ref_p;     // [e][n] reference pressure (FP32 values)
    const float *rr_mom;    // [e][3][n] R(q_r) momentum components
};

// Per-node quantities of one line (FP32), plus the perturbation data.
struct NodeF {
    float r, h0, h1, h2, hp, z, zi;  // full-variable primitives (halved u, p)
    float lr, lz;                    // ln rho, ln(z * scale)
    float hpp;                       // p'/2
    float rp;                        // rho' = rho - rho_r
    float rr;                        // rho_r
    float zr, izr;                   // z_r = rho_r / p_r and its reciprocal
    float beta, ib1;                 // b/b_r - 1 and 1/(1 + beta)
};

template <int R>
__device__ __forceinline__ float hcompf(const NodeF &n)
{
    return R == 0 ? n.h0 : (R == 1 ? n.h1 : n.h2);
}

// FP32 log-mean rule: series for |b-a| < 0.1 (b+a) (u < 1e-2), with terms to
// u^4 (truncation below 2e-12 relative), else [[x]] / [[ln x]].
constexpr float LMF_SQRT = 0.1f;
constexpr float GF1 = 1.0f / 3.0f, GF2 = 4.0f / 45.0f, GF3 = 44.0f / 945.0f,
                GF4 = 428.0f / 14175.0f;
constexpr float IF1 = 1.0f / 3.0f, IF2 = 1.0f / 5.0f, IF3 = 1.0f / 7.0f, IF4 = 1.0f / 9.0f;
constexpr float LN2F = 0.693147180559945309f;

__device__ __forceinline__ float rcpf(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float lnf(float x) { return __builtin_amdgcn_logf(x) * LN2F; }

__device__ __forceinline__ float gser(float u)
{
    return 1.0f - u * (GF1 + u * (GF2 + u * (GF3 + u * GF4)));
}

// {{x}}_log with one reciprocal: series x = d/s, else d/(ln b - ln a).
__device__ __forceinline__ float log_mean_f(float a, float b, float la, float lb)
{
    const float d = b - a, s = a + b;
    const bool ser = fabsf(d) < LMF_SQRT * s;
    const float x = d * rcpf(ser ? s : lb - la);
    return ser ? 0.5f * s * gser(x * x) : x;
}

// 1/{{x}}_log with one reciprocal; the per-node logarithms are of x*scale ~ 1
// (the log-mean is 1-homogeneous), which keeps their FP32 rounding small.
__device__ __forceinline__ float inv_log_mean_f(float a, float b, float la, float lb)
{
    const float d = b - a, s = a + b;
    const bool ser = fabsf(d) < LMF_SQRT * s;
    const float r = rcpf(ser ? s : d);
    const float f = d * r;
    const float u = f * f;
    return ser ? 2.0f * r * (1.0f + u * (IF1 + u * (IF2 + u * (IF3 + u * IF4)))) : (lb - la) * r;
}

// {{rho}}_log - {{rho_r}}_log from the perturbations rho', in one of three
// forms, none of which subtracts two nearly equal FP32 numbers:
//  - both pairs in the series branch:  L = s g(u)/2,
//    L - L_r = (s - s_r) g(u)/2 + s_r (g(u) - g(u_r))/2,
//    g(u) - g(u_r) = -(u - u_r) [1/3 + 4(u+u_r)/45 + 44(u^2+u u_r+u_r^2)/945],
//    u - u_r = (f - f_r)(f + f_r),  f - f_r = (d' s_r - d_r s') / (s s_r);
//  - both pairs in the log branch: with l = [[ln rho]], l_r = [[ln rho_r]]
//    and l' = l - l_r = [[ln(1 + x)]], x = rho'/rho_r,
//    L - L_r = (d + d')/(l_r + l') - d_r/l_r = (d' l_r - d_r l') / (l l_r),
//    whose numerator holds only perturbation-sized products; l' is one
//    log1p of the relative jump (x_b - x_a)/(1 + x_a), l comes from the
//    per-node logs of rho and l_r = l - l' (|l|, |l_r| >= 0.2 outside the
//    series range);
//  - one pair in each branch (a perturbation as large as the reference's
//    own variation over the pair): FP64.
// At N = 5 the kernel holds 250 of the 256 registers that keep two waves per
// SIMD, and the FP32 log-branch form's per-node temporaries would cost it a
// wave: there both log-branch cases take the FP64 form.
template <int NQ>
constexpr bool fp32_log_branch()
{
    return NQ != 6;
}

template <int NQ>
__device__ __forceinline__ float dlog_mean_f(const NodeF &a, const NodeF &b)
{
    const float dr = b.rr - a.rr, sr = a.rr + b.rr;
    const float dp = b.rp - a.rp, sp = a.rp + b.rp;
    const float d = dr + dp, s = sr + sp;
    const bool ser = fabsf(d) < LMF_SQRT * s, ser_r = fabsf(dr) < LMF_SQRT * sr;
    if (fp32_log_branch<NQ>() && !ser && !ser_r) {
        const float xa = a.rp * rcpf(a.rr), xb = b.rp * rcpf(b.rr);
        const float y = (xb - xa) * rcpf(1.0f + xa);
        // ln(1 + y) to a few ulp also for small y: the rounding of 1 + y is
        // undone by the factor y / ((1 + y) - 1)
        const float u1 = 1.0f + y;
        const float lp = (u1 == 1.0f) ? y : lnf(u1) * (y * rcpf(u1 - 1.0f));
        const float l = b.lr - a.lr;
        const float l_r = l - lp;
        return (dp * l_r - dr * lp) * rcpf(l * l_r);
    }
    if (ser && ser_r) {
        const float rs = rcpf(s), rsr = rcpf(sr);
        const float f = d * rs, fr = dr * rsr;
        const float u = f * f, ur = fr * fr;
        const float df = (dp * sr - dr * sp) * rs * rsr;
        const float du = df * (f + fr);
        const float h = GF1 + (GF2 * (u + ur) + GF3 * (u * u + u * ur + ur * ur));
        return 0.5f * (sp * gser(u) - sr * du * h);
    }
    const double ra = (double)a.rr + (double)a.rp, rb = (double)b.rr + (double)b.rp;
    const double l = (rb - ra) / (log(rb) - log(ra));
    const double lr = (b.rr == a.rr) ? (double)a.rr
                                     : ((double)b.rr - (double)a.rr) /
                                           (log((double)b.rr) - log((double)a.rr));
    return (float)(l - lr);
}

// Node primitives: FP64 pressure and perturbations, FP32 storage.
__device__ __forceinline__ NodeF primitives_mixed(const Cons &c, double phi, double gm1,
                                                  float rr_f, float pr_f, float zscale)
{
    NodeF n;
    const double r = c.v[0];
    const double ri = frcp(r);
    const double u0 = c.v[1] * ri, u1 = c.v[2] * ri, u2 = c.v[3] * ri;
    const double p = gm1 * (c.v[4] - 0.5 * (c.v[1] * u0 + c.v[2] * u1 + c.v[3] * u2) - r * phi);
    const double rr = rr_f, pr = pr_f;
    const double rp = r - rr, pp = p - pr;
    n.r = (float)r;
    n.h0 = (float)(0.5 * u0);
    n.h1 = (float)(0.5 * u1);
    n.h2 = (float)(0.5 * u2);
    n.hp = (float)(0.5 * p);
    n.hpp = (float)(0.5 * pp);
    n.rp = (float)rp;
    n.rr = rr_f;
    const float zf = n.r * rcpf((float)p);
    n.z = zf;
    n.zi = (float)(p * ri);
    n.zr = rr_f * rcpf(pr_f);
    n.izr = pr_f * rcpf(rr_f);
    // beta = b/b_r - 1 = (rho p_r)/(rho_r p) - 1 = (rho' p_r - rho_r p')/(rho_r p)
    n.beta = (float)(fdiv(rp * pr - rr * pp, rr * p));
    n.ib1 = rcpf(1.0f + n.beta);
    n.lr = lnf(n.r);
    n.lz = lnf(zf * zscale);
    return n;
}

// Symmetric part of the two-point flux (FP32) with the perturbation
// pressure in the normal momentum.  Returns {{rho}}_log.
template <int R>
__device__ __forceinline__ float sym_flux_mixed(const NodeF &a, const NodeF &b, float phi_m,
                                                float gm1i, float zscale, float S[5])
{
    const float rho_ln = log_mean_f(a.r, b.r, a.lr, b.lr);
    const float izln = inv_log_mean_f(a.z, b.z, a.lz, b.lz);
    const float hRa = hcompf<R>(a), hRb = hcompf<R>(b);
    const float frho = rho_ln * (hRa + hRb);
    S[0] = frho;
    S[1] = frho * (a.h0 + b.h0);
    S[2] = frho * (a.h1 + b.h1);
    S[3] = frho * (a.h2 + b.h2);
    S[1 + R] += a.hpp + b.hpp;
    const float hh = a.h0 * b.h0 + a.h1 * b.h1 + a.h2 * b.h2;
    const float cross = a.hp * hRb + b.hp * hRa;
    S[4] = frho * (izln * gm1i + 2.0f * hh + phi_m) + 2.0f * cross;
    return rho_ln;
}

// Matrix dissipation (FP32), the operator of matrix_dissipation() with the
// same averaged state and eigen-structure.  The jumps of z = rho/p, z u and
// z |u|^2 / 2 are formed in FP64 from the two conservative states and then
// rounded: an FP32 difference of the rounded z would carry an error of one
// FP32 ulp of z, which the enthalpy h_hat ~ 1/{{z}}_log and phi scale up to
// about 1e-4 of the energy flux.
template <int R>
__device__ __forceinline__ void matrix_dissipation_mixed(const NodeF &a, const NodeF &b,
                                                         const Cons &qm, const Cons &qp,
                                                         float rho_ln, float izln, double phi,
                                                         double gm1, const StageParams &P,
                                                         float D[5])
{
    constexpr int T1 = (R + 1) % 3, T2 = (R + 2) % 3;
    const float g = (float)P.gamma, gm1i = (float)P.gm1i;
    float dv[5];
    {
        // No FMA contraction here: the jumps are differences of products, and
        // a contracted fma(x_b, y_b, -x_a y_a) leaves the rounding error of
        // x_a y_a where the states are equal; the dissipation must vanish
        // there exactly.
#pragma clang fp contract(off)
        double zj[2], zuj[2][3], kj[2];
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const Cons &c = side ? qp : qm;
            const double ri = frcp(c.v[0]);
            const double mu = (c.v[1] * c.v[1] + c.v[2] * c.v[2] + c.v[3] * c.v[3]) * ri;
            const double p = gm1 * (c.v[4] - 0.5 * mu - c.v[0] * phi);
            const double ip = frcp(p);
            zj[side] = c.v[0] * ip;
#pragma unroll
            for (int d = 0; d < 3; ++d) zuj[side][d] = c.v[1 + d] * ip;
            kj[side] = 0.5 * mu * ip;  // z |u|^2 / 2
        }
        const float dz = (float)(zj[1] - zj[0]);
        dv[0] = (float)(qp.v[0] - qm.v[0]) * rcpf(rho_ln) + gm1i * (dz * izln) -
                (float)(kj[1] - kj[0]);
#pragma unroll
        for (int d = 0; d < 3; ++d) dv[1 + d] = (float)(zuj[1][d] - zuj[0][d]);
        dv[4] = -dz;
    }

    const float u[3] = {a.h0 + b.h0, a.h1 + b.h1, a.h2 + b.h2};
    const float ka = a.h0 * a.h0 + a.h1 * a.h1 + a.h2 * a.h2;
    const float kb = b.h0 * b.h0 + b.h1 * b.h1 + b.h2 * b.h2;
    const float u2bar = 2.0f * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) - 2.0f * (ka + kb);
    const float phat = (a.r + b.r) * rcpf(a.z + b.z);
    const float hhat = g * gm1i * izln + 0.5f * u2bar;
    const float ahat = sqrtf(g * phat * rcpf(rho_ln));
    const float un = u[R];
    const float c0 = dv[0] + u[0] * dv[1] + u[1] * dv[2] + u[2] * dv[3] + hhat * dv[4];
    const float an = ahat * (dv[1 + R] + un * dv[4]);
    const float ta = rho_ln * (0.5f / g);
    const float te = rho_ln * (g - 1.0f) / g;
    const float aun = fabsf(un);
    const float s0 = fabsf(un - ahat) * ta * (c0 - an);
    const float s4 = fabsf(un + ahat) * ta * (c0 + an);
    const float s1 = aun * te * (c0 - (hhat - 0.5f * u2bar) * dv[4]);
    const float s2 = aun * phat * (dv[1 + T1] + u[T1] * dv[4]);
    const float s3 = aun * phat * (dv[1 + T2] + u[T2] * dv[4]);
    const float sa = s0 + s1 + s4, sd = s4 - s0;
    D[0] = sa;
    D[1] = u[0] * sa;
    D[2] = u[1] * sa;
    D[3] = u[2] * sa;
    D[1 + R] += ahat * sd;
    D[1 + T1] += s2;
    D[1 + T2] += s3;
    D[4] = hhat * (s0 + s4) + ahat * un * sd + 0.5f * u2bar * s1 + u[T1] * s2 + u[T2] * s3 +
           (float)phi * sa;
}

// Face flux (FP32) with the perturbation pressure; the reference is
// continuous across faces (and mirrored at walls), so p'+ uses the own
// node's reference.  Jumps q+ - q- are formed in FP64.
template <int R>
__device__ __forceinline__ void face_flux_mixed(const NodeF &a, const Cons &qm, const Cons &qp,
                                                double phi, double s, const StageParams &P,
                                                float rr_f, float pr_f, float Fn[5])
{
    const double gm1 = P.gamma - 1.0;
    const float g = (float)P.gamma, gm1i = (float)P.gm1i;
    const float zscale = (float)P.lnz_scale;
    const NodeF b = primitives_mixed(qp, phi, gm1, rr_f, pr_f, zscale);
    const float rho_ln = log_mean_f(a.r, b.r, a.lr, b.lr);
    const float izln = inv_log_mean_f(a.z, b.z, a.lz, b.lz);
    const float hRa = hcompf<R>(a), hRb = hcompf<R>(b);
    const float frho = rho_ln * (hRa + hRb);
    float S[5];
    S[0] = frho;
    S[1] = frho * (a.h0 + b.h0);
    S[2] = frho * (a.h1 + b.h1);
    S[3] = frho * (a.h2 + b.h2);
    S[1 + R] += a.hpp + b.hpp;
    const float hh = a.h0 * b.h0 + a.h1 * b.h1 + a.h2 * b.h2;
    const float cross = a.hp * hRb + b.hp * hRa;
    S[4] = frho * (izln * gm1i + 2.0f * hh + (float)phi) + 2.0f * cross;
    const float sf = (float)s;
    if (P.surf == SURF_MATRIX) {
        float D[5];
        matrix_dissipation_mixed<R>(a, b, qm, qp, rho_ln, izln, phi, gm1, P, D);
#pragma unroll
        for (int v = 0; v < 5; ++v) Fn[v] = sf * S[v] - 0.5f * D[v];
        return;
    }
    float hl = 0.0f;
    if (P.surf == SURF_RUSANOV) {
        const float la = 2.0f * fabsf(hRa) + sqrtf(g * a.zi);
        const float lb = 2.0f * fabsf(hRb) + sqrtf(g * b.zi);
        hl = 0.5f * (la > lb ? la : lb);
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) Fn[v] = sf * S[v] - hl * (float)(qp.v[v] - qm.v[v]);
}

template <int NQ>
__device__ __forceinline__ void load_ref(const MixedParams &M, int64_t e, int n, float &rr,
                                         float &pr)
{
    constexpr int NQ3 = NQ * NQ * NQ;
    rr = M.ref_r[e * NQ3 + n];
    pr = M.ref_p[e * NQ3 + n];
}

template <int NQ, int R, bool KEEP = false>
__device__ __forceinline__ void line_terms_mixed(const MixedParams &M, const OrderTables &tb,
                                                 int m, int64_t e, const int ec[3],
                                                 const double phi_k[NQ], float acc[NQ][5],
                                                 double (*qkeep)[5] = nullptr)
{
    constexpr int NQ3 = NQ * NQ * NQ;
    const StageParams &P = M.s;
    const double gm1 = P.gamma - 1.0;
    const float gm1i = (float)P.gm1i;
    const float zscale = (float)P.lnz_scale;
    const double *__restrict__ qin = P.q_in;
#pragma unroll
    for (int a = 0; a < NQ; ++a)
#pragma unroll
        for (int v = 0; v < 5; ++v) acc[a][v] = 0.0f;

    Cons qc[NQ];
    float rrf[NQ], prf[NQ];
#pragma unroll
    for (int t = 0; t < NQ; ++t) {
        const int n = line_node<NQ, R>(m, t);
        load_cons(qin, e, NQ3, n, qc[t]);
        load_ref<NQ>(M, e, n, rrf[t], prf[t]);
    }
    Cons qp[2];
    const bool faces = (P.mask & TERM_FACE) != 0;
    if (faces) {
#pragma unroll
        for (int side = 0; side < 2; ++side)
            plus_state<NQ, R>(P, m, ec, side, qc[side ? NQ - 1 : 0], qp[side]);
    }
    if (KEEP) {
#pragma unroll
        for (int t = 0; t < NQ; ++t)
#pragma unroll
            for (int v = 0; v < 5; ++v) qkeep[t][v] = qc[t].v[v];
    }
    NodeF nd[NQ];
#pragma unroll
    for (int t = 0; t < NQ; ++t)
        nd[t] = primitives_mixed(qc[t], R == 2 ? phi_k[t] : phi_k[0], gm1, rrf[t], prf[t],
                                 zscale);

    // face terms first: the conservative states die before the pair loop
    if (faces) {
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int t = side ? NQ - 1 : 0;
            float Fn[5];
            face_flux_mixed<R>(nd[t], qc[t], qp[side], R == 2 ? phi_k[t] : phi_k[0],
                               side ? 1.0 : -1.0, P, rrf[t], prf[t], Fn);
            const float wi = tb.winvf[t];
#pragma unroll
            for (int v = 0; v < 5; ++v) acc[t][v] -= wi * Fn[v];
        }
    }

    if (P.mask & TERM_VOL) {
#pragma unroll
        for (int a = 0; a < NQ; ++a) {
#pragma unroll
            for (int b = a + 1; b < NQ; ++b) {
                const float phi_m = (float)(R == 2 ? 0.5 * (phi_k[a] + phi_k[b]) : phi_k[0]);
                float S[5];
                const float rho_ln = sym_flux_mixed<R>(nd[a], nd[b], phi_m, gm1i, zscale, S);
                const float tab = tb.Tf[a][b], tba = tb.Tf[b][a];
#pragma unroll
                for (int v = 0; v < 5; ++v) {
                    acc[a][v] -= tab * S[v];
                    acc[b][v] -= tba * S[v];
                }
                if (R == 2) {
                    // G - G_r with rho_hat_ab = (1 + B) L / 2, B = b_b/b_a = z_b/z_a:
                    // rho_hat - rho_hat_r = [(B - B_r) L + (1 + B_r)(L - L_r)] / 2,
                    // B - B_r = B_r (beta_b - beta_a)/(1 + beta_a); partner likewise
                    // with a and b exchanged and [[phi]] negated.
                    const float dphi = (float)(phi_k[b] - phi_k[a]);
                    const float dL = dlog_mean_f<NQ>(nd[a], nd[b]);
                    const float Br = nd[b].zr * nd[a].izr;
                    const float Bri = nd[a].zr * nd[b].izr;
                    const float dB = Br * (nd[b].beta - nd[a].beta) * nd[a].ib1;
                    const float dBi = Bri * (nd[a].beta - nd[b].beta) * nd[b].ib1;
                    const float drh_ab = 0.5f * (dB * rho_ln + (1.0f + Br) * dL);
                    const float drh_ba = 0.5f * (dBi * rho_ln + (1.0f + Bri) * dL);
                    acc[a][3] -= tab * (0.5f * drh_ab * dphi);
                    acc[b][3] -= tba * (-0.5f * drh_ba * dphi);
                }
            }
        }
    }

}

template <int NQ, int EPW, int MODE>
__device__ __forceinline__ void stage_mixed_body(const MixedParams &M, int lb)
{
    constexpr int NQ2 = NQ * NQ, NQ3 = NQ2 * NQ;
    __shared__ float sacc[5][EPW][NQ3];
    const StageParams &P = M.s;

    const OrderTables &tb = c_tab[NQ - 2];
    const int tid = threadIdx.x;
    const int el = tid / NQ2;
    const int m = tid - el * NQ2;
    const int64_t it = (int64_t)lb * EPW + el;  // traversal position
    const bool act = (el < EPW) && (it < P.ne);

    int ec[3] = {0, 0, 0};
    int64_t e = 0;
    if (act) e = tile_element(P, it, ec);
    double phi_k[NQ];
    {
        const double dz = P.zhi - P.zlo;
        const double ZL = P.zlo + dz * ((double)ec[2] / (double)P.K[2]);
        const double ZR = P.zlo + dz * ((double)(ec[2] + 1) / (double)P.K[2]);
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            const double s = tb.xi[k];
            phi_k[k] = P.grav * (0.5 * (1.0 - s) * ZL + 0.5 * (1.0 + s) * ZR);
        }
    }

    float acc[NQ][5];
    const bool vol_or_face = (P.mask & (TERM_VOL | TERM_FACE)) != 0;

    if (act) {
        if (vol_or_face) {
            double phl[NQ];
#pragma unroll
            for (int t = 0; t < NQ; ++t) phl[t] = phi_k[m / NQ];
            line_terms_mixed<NQ, 0>(M, tb, m, e, ec, phl, acc);
        } else {
#pragma unroll
            for (int t = 0; t < NQ; ++t)
#pragma unroll
                for (int v = 0; v < 5; ++v) acc[t][v] = 0.0f;
        }
        const float th = (float)P.two_h[0];
#pragma unroll
        for (int t = 0; t < NQ; ++t) {
            const int n = line_node<NQ, 0>(m, t);
#pragma unroll
            for (int v = 0; v < 5; ++v) sacc[v][el][n] = th * acc[t][v];
        }
    }
    __syncthreads();

    if (act && vol_or_face) {
        double phl[NQ];
#pragma unroll
        for (int t = 0; t < NQ; ++t) phl[t] = phi_k[m / NQ];
        line_terms_mixed<NQ, 1>(M, tb, m, e, ec, phl, acc);
        const float th = (float)P.two_h[1];
#pragma unroll
        for (int t = 0; t < NQ; ++t) {
            const int n = line_node<NQ, 1>(m, t);
#pragma unroll
            for (int v = 0; v < 5; ++v) sacc[v][el][n] += th * acc[t][v];
        }
    }
    __syncthreads();

    if (!act) return;
    const int64_t base0 = e * 5 * NQ3 + m;
    const double *__restrict__ qin = P.q_in;
    // the z line's states stay in registers for the update
    double qv[NQ][5];
    if (vol_or_face) {
        line_terms_mixed<NQ, 2, true>(M, tb, m, e, ec, phi_k, acc, qv);
    } else {
#pragma unroll
        for (int t = 0; t < NQ; ++t)
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                acc[t][v] = 0.0f;
                qv[t][v] = qin[base0 + v * NQ3 + NQ2 * t];
            }
    }
    const bool src = (P.mask & TERM_SRC) != 0;
    // the reference part R(q_r) belongs to the pressure-gravity terms
    const bool with_ref = (P.mask & (TERM_VOL | TERM_FACE)) == (TERM_VOL | TERM_FACE);
    float rrm[NQ][3];
#pragma unroll
    for (int t = 0; t < NQ; ++t) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
            rrm[t][c] = with_ref ? M.rr_mom[(e * 3 + c) * NQ3 + m + NQ2 * t] : 0.0f;
    }
    const float th = (float)P.two_h[2];
    if (MODE == MODE_RHS) {
        double *__restrict__ rout = P.r_out;
#pragma unroll
        for (int t = 0; t < NQ; ++t) {
            const int n = m + NQ2 * t;
            double Rv[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) Rv[v] = (double)(sacc[v][el][n] + th * acc[t][v]);
#pragma unroll
            for (int c = 0; c < 3; ++c) Rv[1 + c] += (double)rrm[t][c];
            if (src) {
                Rv[1] += P.cor_f * qv[t][2];
                Rv[2] -= P.cor_f * qv[t][1];
            }
#pragma unroll
            for (int v = 0; v < 5; ++v) store_f64<true>(&rout[base0 + v * NQ3 + NQ2 * t], Rv[v]);
        }
    } else {
        double *__restrict__ dqp = P.dq;
        double *__restrict__ qout = P.q_out;
        constexpr bool nts = NQ >= NT_STAGE_MIN_NQ;
        // the first LSRK stage (A = 0) does not read dq
        const bool use_dq = P.A != 0.0;
        double dv[NQ][5];
        if (use_dq) {
#pragma unroll
            for (int t = 0; t < NQ; ++t)
#pragma unroll
                for (int v = 0; v < 5; ++v) dv[t][v] = load_f64<nts>(&dqp[base0 + v * NQ3 + NQ2 * t]);
        }
#pragma unroll
        for (int t = 0; t < NQ; ++t) {
            const int n = m + NQ2 * t;
            double Rv[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) Rv[v] = (double)(sacc[v][el][n] + th * acc[t][v]);
#pragma unroll
            for (int c = 0; c < 3; ++c) Rv[1 + c] += (double)rrm[t][c];
            if (src) {
                Rv[1] += P.cor_f * qv[t][2];
                Rv[2] -= P.cor_f * qv[t][1];
            }
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const double d = use_dq ? P.A * dv[t][v] + P.dt * Rv[v] : P.dt * Rv[v];
                store_f64<nts>(&dqp[base0 + v * NQ3 + NQ2 * t], d);
                store_f64<nts>(&qout[base0 + v * NQ3 + NQ2 * t], qv[t][v] + P.B * d);
            }
        }
    }
    if (P.flag) {
        bool bad = false;
#pragma unroll
        for (int t = 0; t < NQ; ++t) {
            const double r = qv[t][0];
            const double kin = qv[t][1] * qv[t][1] + qv[t][2] * qv[t][2] + qv[t][3] * qv[t][3];
            const double eint = qv[t][4] - 0.5 * kin / r - r * phi_k[t];
            bad |= !(r > 0.0) || !(eint > 0.0);
        }
        if (bad) atomicOr(P.flag, 1);
    }
}

template <int NQ, int EPW, int MODE>
__global__ void __launch_bounds__((block_threads<NQ, EPW>())) stage_mixed(const MixedParams M)
{
    stage_mixed_body<NQ, EPW, MODE>(M, xcd_remap(blockIdx.x, M.s.nblocks));
}

struct PackMemberMixed {
    MixedParams M;
    double *bufs[2];
    int block_begin;
    int pad;
};

struct PackLaunchMixed {
    const PackMemberMixed *members;
    const int *parity;
    int n_members;
    int nblocks;
    int stage;
    int mode;
    double A, B;
};

template <int NQ, int EPW, int MODE>
__global__ void __launch_bounds__((block_threads<NQ, EPW>()))
    stage_mixed_packed(const PackLaunchMixed L)
{
    const int gb = xcd_remap(blockIdx.x, L.nblocks);
    int lo = 0, hi = L.n_members - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (L.members[mid].block_begin <= gb) lo = mid;
        else hi = mid - 1;
    }
    const PackMemberMixed &pm = L.members[lo];
    MixedParams M = pm.M;
    const int par = L.parity[lo];
    M.s.q_in = pm.bufs[par ^ (L.stage & 1)];
    M.s.q_out = pm.bufs[par ^ ((L.stage + 1) & 1)];
    M.s.A = L.A;
    M.s.B = L.B;
    stage_mixed_body<NQ, EPW, MODE>(M, gb - pm.block_begin);
}

// Reference state as a conservative FP64 state (rho_r, 0, 0, 0, p_r/(gamma-1)
// + rho_r phi) from the FP32-rounded reference, and the rounding itself.
__global__ void reference_state_kernel(const GeomParams G, const double *__restrict__ rho_in,
                                       const double *__restrict__ p_in, float *__restrict__ rr,
                                       float *__restrict__ pr, double *__restrict__ q_ref)
{
    const int NQ = G.N + 1, NP = NQ * NQ * NQ;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= G.ne * NP) return;
    const int64_t e = gid / NP;
    const int n = (int)(gid - e * NP);
    const int k = n / (NQ * NQ);
    const OrderTables &tb = c_tab[G.N - 1];
    const int ez = (int)(e / ((int64_t)G.K[0] * G.K[1]));
    const double s = tb.xi[k];
    const double ZL = vertex(G, 2, ez), ZR = vertex(G, 2, ez + 1);
    const double phi = G.grav * (0.5 * (1.0 - s) * ZL + 0.5 * (1.0 + s) * ZR);
    const float rf = (float)rho_in[gid], pf = (float)p_in[gid];
    rr[gid] = rf;
    pr[gid] = pf;
    const int64_t base = e * 5 * NP + n;
    q_ref[base] = (double)rf;
    q_ref[base + NP] = 0.0;
    q_ref[base + 2 * NP] = 0.0;
    q_ref[base + 3 * NP] = 0.0;
    q_ref[base + 4 * NP] = (double)pf / (G.gamma - 1.0) + (double)rf * phi;
}

// Keep the momentum components of R(q_r) in FP32.
__global__ void reference_rhs_kernel(int64_t ne, int np, const double *__restrict__ r_ref,
                                     float *__restrict__ rr_mom)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= ne * np) return;
    const int64_t e = gid / np;
    const int n = (int)(gid - e * np);
#pragma unroll
    for (int c = 0; c < 3; ++c)
        rr_mom[(e * 3 + c) * np + n] = (float)r_ref[(e * 5 + 1 + c) * np + n];
}

}  // namespace esdg
