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

// Per-node quantities of one line (FP32), plus the perturbation data.  The
// per-node logarithms of the log-mean branch live in arrays of their own,
// filled only where the general pair loop runs.
struct NodeF {
    float r, h0, h1, h2, hp, z, zi;  // full-variable primitives (halved u, p)
    float hpp;                       // p'/2
    float rp;                        // rho' = rho - rho_r
    float rr;                        // rho_r
    float zr;                        // z_r = rho_r / p_r
    float beta;                      // b/b_r - 1
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

// A line whose extreme pair satisfies |b-a| < 0.09999 (b+a) has every pair in
// the series range of the FP32 rule (slightly tighter, so that no pair of a
// line declared series-only would select the log branch by itself).
constexpr float LMF_SQRT_LINE = 0.09999f;

template <int NQ>
__device__ __forceinline__ bool line_spread_f(const float x[NQ])
{
    float mn = x[0], mx = x[0];
#pragma unroll
    for (int t = 1; t < NQ; ++t) {
        mn = fminf(mn, x[t]);
        mx = fmaxf(mx, x[t]);
    }
    return !(mx - mn < LMF_SQRT_LINE * (mx + mn));
}

// Series forms with the 1/2 of the mean folded into the coefficients.
constexpr float GH0 = 0.5f, GH1 = 0.5f * GF1, GH2 = 0.5f * GF2, GH3 = 0.5f * GF3,
                GH4 = 0.5f * GF4;

__device__ __forceinline__ float log_mean_series_f(float a, float b)
{
    const float d = b - a, s = a + b;
    const float x = d * rcpf(s);
    const float u = x * x;
    return s * (GH0 - u * (GH1 + u * (GH2 + u * (GH3 + u * GH4))));
}

__device__ __forceinline__ float inv_log_mean_series_f(float a, float b)
{
    const float d = b - a, s = a + b;
    const float r = rcpf(s);
    const float f = d * r;
    const float u = f * f;
    return (r + r) * (1.0f + u * (IF1 + u * (IF2 + u * (IF3 + u * IF4))));
}

// {{rho}}_log - {{rho_r}}_log from the perturbations rho' (never a difference
// of two nearly equal FP32 log-means):
//  - both pairs in the series range, L = s g(u)/2 with g(u) = f/atanh f:
//    L - L_r = (s - s_r) g(u)/2 + s_r (g(u) - g(u_r))/2,
//    g(u) - g(u_r) = -(u - u_r) [GF1 + GF2 (u + u_r) + ...],
//    u - u_r = (f - f_r)(f + f_r),  f - f_r = (d' s_r - d_r s') / (s s_r);
//  - both pairs in the log range: with l = [[ln rho]], l_r = [[ln rho_r]]
//    and l' = l - l_r = [[ln(1 + x)]], x = rho'/rho_r,
//    L - L_r = (d + d')/(l_r + l') - d_r/l_r = (d' l_r - d_r l') / (l l_r),
//    whose numerator holds only perturbation-sized products; l' is one
//    log1p of the relative jump (x_b - x_a)/(1 + x_a), l comes from the
//    per-node logs of rho and l_r = l - l'.
// Series form (both log-means in the series range), to u^4:
//   L - L_r = [s' g(u) - s_r (u - u_r) h] / 2,
//   h = GF1 + GF2 (u + u_r) + GF3 (u^2 + u u_r + u_r^2)
//       + GF4 (u^3 + u^2 u_r + u u_r^2 + u_r^3).
__device__ __forceinline__ float dlog_mean_series_f(const NodeF &a, const NodeF &b)
{
    const float dr = b.rr - a.rr, sr = a.rr + b.rr;
    const float dp = b.rp - a.rp, sp = a.rp + b.rp;
    const float d = dr + dp, s = sr + sp;
    const float rs = rcpf(s), rsr = rcpf(sr);
    const float f = d * rs, fr = dr * rsr;
    const float u = f * f, ur = fr * fr;
    const float df = (dp * sr - dr * sp) * rs * rsr;
    const float du = df * (f + fr);
    const float u2 = u * u + u * ur + ur * ur;
    const float h = GF1 + (GF2 * (u + ur) + (GF3 * u2 + GF4 * (u + ur) * (u * u + ur * ur)));
    return 0.5f * (sp * gser(u) - sr * du * h);
}

// {{rho}}_log - {{rho_r}}_log for a pair, chosen by the spreads f = |[[rho]]|/(2{{rho}})
// and f_r of the full and the reference density:
//  - both below 0.2: the series form (u, u_r < 0.04, where the u^4 series is
//    exact to FP32 rounding);
//  - otherwise, both at least 0.1: the log form;
//  - otherwise (one spread below 0.1, the other at least 0.2: a perturbation
//    as large as the reference's own variation over the pair): the plain
//    difference of the two FP32 log-means, which is then itself of the size
//    of the log-means, so that its rounding stays near eps32 relative.
// la, lb are the per-node ln rho of the two nodes.
constexpr float DLM_SER = 0.2f, DLM_LOG = 0.1f;

__device__ __forceinline__ float dlog_mean_f(const NodeF &a, const NodeF &b, float la, float lb)
{
    const float dr = b.rr - a.rr, sr = a.rr + b.rr;
    const float dp = b.rp - a.rp, sp = a.rp + b.rp;
    const float d = dr + dp, s = sr + sp;
    const float ad = fabsf(d), adr = fabsf(dr);
    if (ad < DLM_SER * s && adr < DLM_SER * sr) return dlog_mean_series_f(a, b);
    if (ad >= DLM_LOG * s && adr >= DLM_LOG * sr) {
        const float xa = a.rp * rcpf(a.rr), xb = b.rp * rcpf(b.rr);
        const float y = (xb - xa) * rcpf(1.0f + xa);
        // ln(1 + y) to a few ulp also for small y: the rounding of 1 + y is
        // undone by the factor y / ((1 + y) - 1)
        const float u1 = 1.0f + y;
        const float lp = (u1 == 1.0f) ? y : lnf(u1) * (y * rcpf(u1 - 1.0f));
        const float l = lb - la;
        const float l_r = l - lp;
        return (dp * l_r - dr * lp) * rcpf(l * l_r);
    }
    return log_mean_f(a.r, b.r, la, lb) - log_mean_f(a.rr, b.rr, lnf(a.rr), lnf(b.rr));
}

// Node primitives: FP64 pressure and perturbations, FP32 storage.
__device__ __forceinline__ NodeF primitives_mixed(const Cons &c, double phi, double gm1,
                                                  float rr_f, float pr_f)
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
    // beta = b/b_r - 1 = (rho p_r)/(rho_r p) - 1 = (rho' p_r - rho_r p')/(rho_r p)
    n.beta = (float)(fdiv(rp * pr - rr * pp, rr * p));
    return n;
}

// Symmetric part of the two-point flux (FP32) with the perturbation
// pressure in the normal momentum, from the two log-means.
template <int R>
__device__ __forceinline__ void sym_flux_f(const NodeF &a, const NodeF &b, float rho_ln,
                                           float izln, float phi_m, float gm1i, float S[5])
{
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
    const NodeF b = primitives_mixed(qp, phi, gm1, rr_f, pr_f);
    float rho_ln, izln;
    {
        const float d = b.r - a.r, sm = a.r + b.r;
        float den = sm;
        if (!(fabsf(d) < LMF_SQRT * sm)) den = lnf(b.r) - lnf(a.r);
        const float x = d * rcpf(den);
        rho_ln = (fabsf(d) < LMF_SQRT * sm) ? 0.5f * sm * gser(x * x) : x;
    }
    {
        const float d = b.z - a.z, sm = a.z + b.z;
        const bool ser = fabsf(d) < LMF_SQRT * sm;
        float num = 1.0f, den = sm;
        if (!ser) {
            num = lnf(b.z * zscale) - lnf(a.z * zscale);
            den = d;
        }
        const float r = num * rcpf(den);
        const float f = d * r;
        const float u = f * f;
        izln = ser ? 2.0f * r * (1.0f + u * (IF1 + u * (IF2 + u * (IF3 + u * IF4)))) : r;
    }
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

// Waves per SIMD the mixed kernel is compiled for: from N = 6 on, two waves
// with a few spilled registers beat one wave without spills.
template <int NQ>
constexpr int mixed_min_waves()
{
    return NQ >= 7 ? 2 : 1;
}

// Whether the z phase of the mixed kernel holds its line's FP64 states in
// registers for the finish (else the finish reads them again).
template <int NQ>
constexpr bool mixed_holds_states()
{
    return NQ < 6;
}

// Geopotential at LGL level k of an element spanning [zl, zr] in z.
__device__ __forceinline__ double phi_level(const StageParams &P, const OrderTables &tb,
                                            double zl, double zr, int k)
{
    const double s = tb.xi[k];
    return P.grav * (0.5 * (1.0 - s) * zl + 0.5 * (1.0 + s) * zr);
}

// Accumulates the symmetric-flux shares of one pair (a, b) of a line.
__device__ __forceinline__ void flux_shares_f(float tab, float tba, const float S[5],
                                              float acc_a[5], float acc_b[5])
{
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        acc_a[v] -= tab * S[v];
        acc_b[v] -= tba * S[v];
    }
}

// Accumulates the shares of one z-line pair (a, b) in the deviation of the
// gravity term from the reference's,
//   G - G_r = [[phi]]/4 [(B - B_r) L + (1 + B_r)(L - L_r)],
//   B = z_b/z_a, B_r = z_r,b/z_r,a, L = {{rho}}_log,
//   B - B_r = z_r,b (beta_b - beta_a) / z_a   (z = z_r (1 + beta)),
// and for the partner a and b exchanged with [[phi]] negated.
__device__ __forceinline__ void gravity_shares_f(const NodeF &na, const NodeF &nb, float tab,
                                                 float tba, float rho_ln, float dL, float dphi,
                                                 float &acc_a, float &acc_b)
{
    const float dbeta = nb.beta - na.beta;
    const float dB = nb.zr * dbeta * na.zi;
    const float dBi = -(na.zr * dbeta * nb.zi);
    // 1/z_r = (1 + beta)/z
    const float izr_a = fmaf(na.beta, na.zi, na.zi), izr_b = fmaf(nb.beta, nb.zi, nb.zi);
    const float drh_ab = dB * rho_ln + (1.0f + nb.zr * izr_a) * dL;
    const float drh_ba = dBi * rho_ln + (1.0f + na.zr * izr_b) * dL;
    const float q = 0.25f * dphi;
    acc_a -= tab * (q * drh_ab);
    acc_b += tba * (q * drh_ba);
}

template <int NQ, int R, bool KEEP = false>
__device__ __forceinline__ void line_terms_mixed(const MixedParams &M, const OrderTables &tb,
                                                 int m, int64_t e, const int ec[3], double zl,
                                                 double zr, float acc[NQ][5],
                                                 double (*qkeep)[5] = nullptr)
{
    constexpr int NQ3 = NQ * NQ * NQ;
    const StageParams &P = M.s;
    const double gm1 = P.gamma - 1.0;
    const float gm1i = (float)P.gm1i;
    const float zscale = (float)P.lnz_scale;
    const double *__restrict__ qin = P.q_in;
    // geopotential of node t of the line (constant along x- and y-lines)
    auto phi = [&](int t) -> double { return phi_level(P, tb, zl, zr, R == 2 ? t : m / NQ); };

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
    for (int t = 0; t < NQ; ++t) nd[t] = primitives_mixed(qc[t], phi(t), gm1, rrf[t], prf[t]);

#pragma unroll
    for (int a = 0; a < NQ; ++a)
#pragma unroll
        for (int v = 0; v < 5; ++v) acc[a][v] = 0.0f;
    // face terms first: the conservative states die before the pair loop
    if (faces) {
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int t = side ? NQ - 1 : 0;
            float Fn[5];
            face_flux_mixed<R>(nd[t], qc[t], qp[side], phi(t), side ? 1.0 : -1.0, P, rrf[t],
                               prf[t], Fn);
            const float wi = tb.winvf[t];
#pragma unroll
            for (int v = 0; v < 5; ++v) acc[t][v] -= wi * Fn[v];
        }
    }
    if (!(P.mask & TERM_VOL)) return;

    float phf[NQ];
#pragma unroll
    for (int t = 0; t < NQ; ++t) phf[t] = (float)phi(t);
    float xr[NQ], xz[NQ];
#pragma unroll
    for (int t = 0; t < NQ; ++t) {
        xr[t] = nd[t].r;
        xz[t] = nd[t].z;
    }
    const bool need_r = line_spread_f<NQ>(xr), need_z = line_spread_f<NQ>(xz);
    // x- and y-lines take a wave-uniform series-only loop when no line of the
    // wave can reach the log branch of either log-mean; z-lines, which also
    // carry the gravity deviation, take the general loop
    if (R != 2 && __ballot(need_r || need_z) == 0) {
#pragma unroll
        for (int a = 0; a < NQ; ++a) {
#pragma unroll
            for (int b = a + 1; b < NQ; ++b) {
                const float rho_ln = log_mean_series_f(nd[a].r, nd[b].r);
                const float izln = inv_log_mean_series_f(nd[a].z, nd[b].z);
                const float phi_m = R == 2 ? 0.5f * (phf[a] + phf[b]) : phf[0];
                float S[5];
                sym_flux_f<R>(nd[a], nd[b], rho_ln, izln, phi_m, gm1i, S);
                flux_shares_f(tb.Tf[a][b], tb.Tf[b][a], S, acc[a], acc[b]);
            }
        }
    } else {
        float lr[NQ], lz[NQ];
#pragma unroll
        for (int t = 0; t < NQ; ++t) {
            lr[t] = lnf(nd[t].r);
            lz[t] = lnf(nd[t].z * zscale);
        }
#pragma unroll
        for (int a = 0; a < NQ; ++a) {
#pragma unroll
            for (int b = a + 1; b < NQ; ++b) {
                const float rho_ln = log_mean_f(nd[a].r, nd[b].r, lr[a], lr[b]);
                const float izln = inv_log_mean_f(nd[a].z, nd[b].z, lz[a], lz[b]);
                const float phi_m = R == 2 ? 0.5f * (phf[a] + phf[b]) : phf[0];
                float S[5];
                sym_flux_f<R>(nd[a], nd[b], rho_ln, izln, phi_m, gm1i, S);
                flux_shares_f(tb.Tf[a][b], tb.Tf[b][a], S, acc[a], acc[b]);
            }
        }
        if (R == 2) {
            // the gravity deviation in a pass of its own: the flux-only
            // quantities of the nodes are dead here
#pragma unroll
            for (int a = 0; a < NQ; ++a) {
#pragma unroll
                for (int b = a + 1; b < NQ; ++b) {
                    const float rho_ln = log_mean_f(nd[a].r, nd[b].r, lr[a], lr[b]);
                    const float dL = dlog_mean_f(nd[a], nd[b], lr[a], lr[b]);
                    gravity_shares_f(nd[a], nd[b], tb.Tf[a][b], tb.Tf[b][a], rho_ln, dL,
                                     phf[b] - phf[a], acc[a][3], acc[b][3]);
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
    // vertical extent of the element (geopotential of its LGL levels)
    const double dzb = P.zhi - P.zlo;
    const double ZL = P.zlo + dzb * ((double)ec[2] / (double)P.K[2]);
    const double ZR = P.zlo + dzb * ((double)(ec[2] + 1) / (double)P.K[2]);

    float acc[NQ][5];
    const bool vol_or_face = (P.mask & (TERM_VOL | TERM_FACE)) != 0;

    if (act) {
        if (vol_or_face) {
            line_terms_mixed<NQ, 0>(M, tb, m, e, ec, ZL, ZR, acc);
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
        line_terms_mixed<NQ, 1>(M, tb, m, e, ec, ZL, ZR, acc);
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
    constexpr bool HOLD = mixed_holds_states<NQ>();
    double qv[HOLD ? NQ : 1][5];
    if (vol_or_face) {
        line_terms_mixed<NQ, 2, HOLD>(M, tb, m, e, ec, ZL, ZR, acc, qv);
    } else {
#pragma unroll
        for (int t = 0; t < NQ; ++t)
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                acc[t][v] = 0.0f;
                if constexpr (HOLD) qv[t][v] = qin[base0 + v * NQ3 + NQ2 * t];
            }
    }
    auto qs = [&](int t, int v) -> double {
        if constexpr (HOLD)
            return qv[t][v];
        else
            return qin[base0 + v * NQ3 + NQ2 * t];
    };
    const bool src = (P.mask & TERM_SRC) != 0;
    // the reference part R(q_r) belongs to the pressure-gravity terms
    const bool with_ref = (P.mask & (TERM_VOL | TERM_FACE)) == (TERM_VOL | TERM_FACE);
    const float th = (float)P.two_h[2];
    constexpr bool nts = NQ >= NT_STAGE_MIN_NQ;
    // the first LSRK stage (A = 0) does not read dq
    const bool use_dq = MODE == MODE_STAGE && P.A != 0.0;
    double *__restrict__ rout = P.r_out;
    double *__restrict__ dqp = P.dq;
    double *__restrict__ qout = P.q_out;
    bool bad = false;
#pragma unroll
    for (int t = 0; t < NQ; ++t) {
        const int n = m + NQ2 * t;
        const int64_t o = base0 + NQ2 * t;
        double qn[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) qn[v] = qs(t, v);
        double Rv[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) Rv[v] = (double)(sacc[v][el][n] + th * acc[t][v]);
        if (with_ref) {
#pragma unroll
            for (int c = 0; c < 3; ++c) Rv[1 + c] += (double)M.rr_mom[(e * 3 + c) * NQ3 + n];
        }
        if (src) {
            Rv[1] += P.cor_f * qn[2];
            Rv[2] -= P.cor_f * qn[1];
        }
        if (MODE == MODE_RHS) {
#pragma unroll
            for (int v = 0; v < 5; ++v) store_f64<true>(&rout[o + v * NQ3], Rv[v]);
        } else {
            double dv[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) dv[v] = use_dq ? load_f64<nts>(&dqp[o + v * NQ3]) : 0.0;
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const double d = use_dq ? P.A * dv[v] + P.dt * Rv[v] : P.dt * Rv[v];
                store_f64<nts>(&dqp[o + v * NQ3], d);
                store_f64<nts>(&qout[o + v * NQ3], qn[v] + P.B * d);
            }
        }
        if (P.flag) {
            const double r = qn[0];
            const double kin = qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3];
            const double eint = qn[4] - 0.5 * kin / r - r * phi_level(P, tb, ZL, ZR, t);
            bad |= !(r > 0.0) || !(eint > 0.0);
        }
    }
    if (P.flag && bad) atomicOr(P.flag, 1);
}

template <int NQ, int EPW, int MODE>
__global__ void __launch_bounds__((block_threads<NQ, EPW>()), (mixed_min_waves<NQ>()))
    stage_mixed(const MixedParams M)
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
__global__ void __launch_bounds__((block_threads<NQ, EPW>()), (mixed_min_waves<NQ>()))
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
