// esdg_curved.hpp -- fused ES-DGSEM stage kernel on curved hexahedra.
//
// The affine kernel's metric factors 2/h_r become per-node metric terms
// (Sec. 3: the metric terms G and the Jacobian of the semi-discrete form).
// With J a^r the contravariant basis vector of direction r times the
// Jacobian J:
//   volume:  R_a += -(1/J_a) sum_r (1/w_i) sum_b S_ab sum_d {{J a^r_d}}_ab F_d(a, b),
//            where F_d is the two-point flux of direction d, whose momentum
//            part carries the pressure and the gravity term G_ab = rho_hat
//            [[phi]]/2 in component d; the sum over d is taken in closed form
//            (the flux along the averaged vector n = {{J a^r}});
//   faces:   R_a += -(1/(J_a w_0)) F*(q-, q+; s J a^r(a)), the face flux
//            along the unnormalised outward normal s J a^r, with the Rusanov
//            speed of the unit normal scaled by |J a^r|.
// The geopotential varies along every line of a curved element, so the
// gravity term appears in all three directions.  The line-per-lane layout,
// the LDS accumulator of the affine kernel and the face handling are kept;
// the metric terms and 1/J are read per node from HBM, and phi once per
// element by the x phase, which leaves it in LDS for the other phases and
// the finish (88 B per node per stage beyond the state).
#pragma once

#include "esdg_device.hpp"

namespace esdg {

struct CurvedParams {
    StageParams s;
    const double *Ja;   // [e][r][d][n]  J a^r_d
    const double *iJ;   // [e][n]        1/J
    const double *phi;  // [e][n]        geopotential
};

// Symmetric two-point flux along the vector n (the averaged J a^r of a pair,
// or a face normal): f^rho = {{rho}}_log (n.{{u}}),
// f^m = f^rho {{u}} + n {{p}},
// f^E = f^rho (1/((gamma-1) {{rho/p}}_log) + u_a.u_b/2 + phi_m)
//       + (p_a (n.u_b) + p_b (n.u_a))/2.   Returns {{rho}}_log.
__device__ __forceinline__ double sym_flux_vec(const Node &a, const Node &b, double rho_ln,
                                               double izln, const double n[3], double phi_m,
                                               double gm1i, double S[5])
{
    const double una = n[0] * a.h0 + n[1] * a.h1 + n[2] * a.h2;  // (n.u_a)/2
    const double unb = n[0] * b.h0 + n[1] * b.h1 + n[2] * b.h2;
    const double frho = rho_ln * (una + unb);
    const double pm = a.hp + b.hp;  // {{p}}
    S[0] = frho;
    S[1] = frho * (a.h0 + b.h0) + n[0] * pm;
    S[2] = frho * (a.h1 + b.h1) + n[1] * pm;
    S[3] = frho * (a.h2 + b.h2) + n[2] * pm;
    const double hh = a.h0 * b.h0 + a.h1 * b.h1 + a.h2 * b.h2;
    const double cross = a.hp * unb + b.hp * una;
    S[4] = frho * (izln * gm1i + 2.0 * hh + phi_m) + 2.0 * cross;
    return rho_ln;
}

// Both log-means of a pair with the branch rule; logarithms taken here only
// on the log branch.
__device__ __forceinline__ void pair_log_means(const Node &a, const Node &b,
                                               const StageParams &P, double &rho_ln,
                                               double &izln)
{
    {
        const double d = b.r - a.r, sm = a.r + b.r;
        const bool ser = fabs(d) < LM_SQRT_EPS * sm;
        double den = sm;
        if (!ser) den = log(b.r) - log(a.r);
        const double x = fdiv(d, den);
        const double u = x * x;
        rho_ln = ser ? 0.5 * sm * (1.0 - u * (S1 + u * (S2 + u * S3))) : x;
    }
    {
        const double d = b.z - a.z, sm = a.z + b.z;
        const bool ser = fabs(d) < LM_SQRT_EPS * sm;
        double num = 1.0, den = sm;
        if (!ser) {
            num = log(b.z * P.lnz_scale) - log(a.z * P.lnz_scale);
            den = d;
        }
        const double x = fdiv(num, den);
        const double dx = d * x;
        const double u = dx * dx;
        izln = ser ? 2.0 * x * (1.0 + u * (I1 + u * (I2 + u * I3))) : x;
    }
}

// Both log-means of a pair whose line stays inside the series range of both
// (the caller has checked the whole line): no branch, no logarithm.
__device__ __forceinline__ void pair_log_means_series(const Node &a, const Node &b,
                                                      double &rho_ln, double &izln)
{
    const double dr = b.r - a.r, sr = a.r + b.r;
    const double xr = dr * frcp1(sr);  // enters only through u < 1e-4
    const double ur = xr * xr;
    rho_ln = sr * (0.5 - ur * (H1 + ur * (H2 + ur * H3)));
    const double dz = b.z - a.z, sz = a.z + b.z;
    const double rz = frcp(sz);
    const double fz = dz * rz;
    const double uz = fz * fz;
    izln = (rz + rz) * (1.0 + uz * (I1 + uz * (I2 + uz * I3)));
}

// Shares of one pair (a, b) of a line: the flux along the averaged J a^r and
// the gravity term along it (partner G_ba = -G_ab z_a / z_b).  jh holds the
// halved metric terms J a^r / 2 of the line's nodes.
template <int NQ>
__device__ __forceinline__ void curved_pair_shares(const OrderTables &tb, const Node nd[NQ],
                                                   const double ph[NQ],
                                                   const double jh[NQ][3], int a, int b,
                                                   double rho_ln, double izln, double gm1i,
                                                   double acc[NQ][5])
{
    const double n[3] = {jh[a][0] + jh[b][0], jh[a][1] + jh[b][1], jh[a][2] + jh[b][2]};
    double S[5];
    sym_flux_vec(nd[a], nd[b], rho_ln, izln, n, 0.5 * (ph[a] + ph[b]), gm1i, S);
    const double tab = tb.T[a][b], tba = tb.T[b][a];
    const double X = 0.25 * rho_ln * (nd[a].z + nd[b].z) * (ph[b] - ph[a]);
    const double tga = tab * (X * nd[a].zi), tgb = tba * (X * nd[b].zi);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        acc[a][v] -= tab * S[v];
        acc[b][v] -= tba * S[v];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        acc[a][1 + d] -= tga * n[d];
        acc[b][1 + d] += tgb * n[d];
    }
}

// Matrix dissipation for a general unit normal nu: the operator of
// matrix_dissipation<R> with nu in place of e_R; the two shear waves enter
// through the tangent projector P = I - nu nu^T,
//   |u_n| p_hat (0, P w, u_hat . P w),  w = [[v]]_m + u_hat [[v]]_5,
// which does not depend on the tangents one would choose.
__device__ __forceinline__ void matrix_dissipation_vec(const Node &a, const Node &b,
                                                       double rho_ln, double izln, double phi,
                                                       const double nu[3],
                                                       const StageParams &P, double D[5])
{
    const double g = P.gamma, gm1i = P.gm1i;
    const double u[3] = {a.h0 + b.h0, a.h1 + b.h1, a.h2 + b.h2};
    const double ka = a.h0 * a.h0 + a.h1 * a.h1 + a.h2 * a.h2;
    const double kb = b.h0 * b.h0 + b.h1 * b.h1 + b.h2 * b.h2;
    const double u2bar = 2.0 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) - 2.0 * (ka + kb);
    const double phat = fdiv(a.r + b.r, a.z + b.z);
    const double hhat = g * gm1i * izln + 0.5 * u2bar;
    const double ahat = sqrt_pos(g * fdiv(phat, rho_ln));
    const double dz = b.z - a.z;
    double dv[5];
    {
        // jumps of products without FMA contraction (they must vanish
        // exactly where the two sides agree)
#pragma clang fp contract(off)
        const double zk_a = a.z * ka, zk_b = b.z * kb;
        dv[0] = fdiv(b.r - a.r, rho_ln) + gm1i * (dz * izln) - 2.0 * (zk_b - zk_a);
        dv[1] = 2.0 * (b.z * b.h0 - a.z * a.h0);
        dv[2] = 2.0 * (b.z * b.h1 - a.z * a.h1);
        dv[3] = 2.0 * (b.z * b.h2 - a.z * a.h2);
    }
    dv[4] = -dz;
    const double un = u[0] * nu[0] + u[1] * nu[1] + u[2] * nu[2];
    const double dvn = dv[1] * nu[0] + dv[2] * nu[1] + dv[3] * nu[2];
    const double c0 = dv[0] + u[0] * dv[1] + u[1] * dv[2] + u[2] * dv[3] + hhat * dv[4];
    const double an = ahat * (dvn + un * dv[4]);
    const double ta = rho_ln * (0.5 / g);
    const double te = rho_ln * (g - 1.0) / g;
    const double aun = fabs(un);
    const double s0 = fabs(un - ahat) * ta * (c0 - an);
    const double s4 = fabs(un + ahat) * ta * (c0 + an);
    const double s1 = aun * te * (c0 - (hhat - 0.5 * u2bar) * dv[4]);
    const double sa = s0 + s1 + s4, sd = s4 - s0;
    double w[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) w[c] = dv[1 + c] + u[c] * dv[4];
    const double nw = w[0] * nu[0] + w[1] * nu[1] + w[2] * nu[2];
    const double sh = aun * phat;
    double uPw = 0.0;
    D[0] = sa;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double Pw = w[c] - nu[c] * nw;
        D[1 + c] = u[c] * sa + ahat * nu[c] * sd + sh * Pw;
        uPw += u[c] * Pw;
    }
    D[4] = hhat * (s0 + s4) + ahat * un * sd + 0.5 * u2bar * s1 + sh * uPw + phi * sa;
}

// Face flux along the unnormalised outward normal Nv = s J a^r at a face
// node (phi on both sides): the EC flux along Nv minus the Rusanov term
// |Nv| lambda/2 (q+ - q-), lambda = max(|u.n| + c) with n = Nv/|Nv|, or
// minus |Nv| D(n)/2 with the matrix dissipation, or nothing (EC).
__device__ __forceinline__ void face_flux_vec(const Node &a, const Cons &qm, const Cons &qp,
                                              double phi, const double Nv[3],
                                              const StageParams &P, double Fn[5])
{
    const double g = P.gamma, gm1 = g - 1.0;
    const Node b = primitives(qp, phi, gm1);
    double rho_ln, izln;
    pair_log_means(a, b, P, rho_ln, izln);
    double S[5];
    sym_flux_vec(a, b, rho_ln, izln, Nv, phi, P.gm1i, S);
    if (P.surf == SURF_MATRIX) {
        const double nrm = sqrt_pos(Nv[0] * Nv[0] + Nv[1] * Nv[1] + Nv[2] * Nv[2]);
        const double inrm = frcp(nrm);
        const double nu[3] = {Nv[0] * inrm, Nv[1] * inrm, Nv[2] * inrm};
        double D[5];
        matrix_dissipation_vec(a, b, rho_ln, izln, phi, nu, P, D);
#pragma unroll
        for (int v = 0; v < 5; ++v) Fn[v] = S[v] - 0.5 * nrm * D[v];
        return;
    }
    double hl = 0.0;
    if (P.surf == SURF_RUSANOV) {
        const double n2 = Nv[0] * Nv[0] + Nv[1] * Nv[1] + Nv[2] * Nv[2];
        const double nrm = sqrt_pos(n2);
        const double una = 2.0 * fabs(Nv[0] * a.h0 + Nv[1] * a.h1 + Nv[2] * a.h2);
        const double unb = 2.0 * fabs(Nv[0] * b.h0 + Nv[1] * b.h1 + Nv[2] * b.h2);
        // |u.Nv| + c |Nv| = |Nv| (|u.n| + c)
        const double la = una + sqrt_pos(g * a.zi) * nrm;
        const double lb = unb + sqrt_pos(g * b.zi) * nrm;
        hl = 0.5 * (la > lb ? la : lb);
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) Fn[v] = S[v] - hl * (qp.v[v] - qm.v[v]);
}

// Volume and face sums of one R-line of a curved element (without the 1/J
// of the finish).  KEEP copies the line's conservative states to qkeep.
template <int NQ, int R, bool KEEP = false>
__device__ __forceinline__ void line_terms_curved(const CurvedParams &C, const OrderTables &tb,
                                                  int m, int64_t e, const int ec[3],
                                                  double *sphi, double acc[NQ][5],
                                                  double (*qkeep)[5] = nullptr)
{
    constexpr int NQ3 = NQ * NQ * NQ;
    const StageParams &P = C.s;
    const double gm1 = P.gamma - 1.0;
#pragma unroll
    for (int a = 0; a < NQ; ++a)
#pragma unroll
        for (int v = 0; v < 5; ++v) acc[a][v] = 0.0;

    Cons qc[NQ];
    double ph[NQ], jr[NQ][3];
#pragma unroll
    for (int t = 0; t < NQ; ++t) {
        const int n = line_node<NQ, R>(m, t);
        load_cons(P.q_in, e, NQ3, n, qc[t]);
        if (R == 0) {
            // the x lines cover the element: its geopotential goes to LDS
            // for the other phases and the finish
            ph[t] = C.phi[e * NQ3 + n];
            sphi[n] = ph[t];
        } else {
            ph[t] = sphi[n];
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) jr[t][d] = 0.5 * C.Ja[((e * 3 + R) * 3 + d) * NQ3 + n];
    }
    const bool faces = (P.mask & TERM_FACE) != 0;
    Cons qp[2];
    if (faces) {
#pragma unroll
        for (int side = 0; side < 2; ++side)
            plus_state<NQ, R>(P, m, ec, side, qc[side ? NQ - 1 : 0], qp[side]);
    }
    if constexpr (KEEP) {
#pragma unroll
        for (int t = 0; t < NQ; ++t)
#pragma unroll
            for (int v = 0; v < 5; ++v) qkeep[t][v] = qc[t].v[v];
    }
    Node nd[NQ];
#pragma unroll
    for (int t = 0; t < NQ; ++t) nd[t] = primitives(qc[t], ph[t], gm1);

    if (faces) {
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int t = side ? NQ - 1 : 0;
            const double s = side ? 2.0 : -2.0;  // jr holds J a^r / 2
            const double Nv[3] = {s * jr[t][0], s * jr[t][1], s * jr[t][2]};
            double Fn[5];
            face_flux_vec(nd[t], qc[t], qp[side], ph[t], Nv, P, Fn);
            const double wi = tb.winv[t];
#pragma unroll
            for (int v = 0; v < 5; ++v) acc[t][v] -= wi * Fn[v];
        }
    }

    if (P.mask & TERM_VOL) {
        double xr[NQ], xz[NQ];
#pragma unroll
        for (int t = 0; t < NQ; ++t) {
            xr[t] = nd[t].r;
            xz[t] = nd[t].z;
        }
        const bool need_r = line_spread<NQ>(xr), need_z = line_spread<NQ>(xz);
        // wave-uniform choice: the series-only loop when no line of the wave
        // can reach the log branch
        if (__ballot(need_r || need_z) == 0) {
#pragma unroll
            for (int a = 0; a < NQ; ++a) {
#pragma unroll
                for (int b = a + 1; b < NQ; ++b) {
                    double rho_ln, izln;
                    pair_log_means_series(nd[a], nd[b], rho_ln, izln);
                    curved_pair_shares<NQ>(tb, nd, ph, jr, a, b, rho_ln, izln, P.gm1i, acc);
                }
            }
        } else {
            double lr[NQ], lz[NQ];
            line_logs<NQ>(xr, need_r, 1.0, lr);
            line_logs<NQ>(xz, need_z, P.lnz_scale, lz);
#pragma unroll
            for (int a = 0; a < NQ; ++a) {
#pragma unroll
                for (int b = a + 1; b < NQ; ++b) {
                    const double rho_ln = log_mean(nd[a].r, nd[b].r, lr[a], lr[b]);
                    const double izln = inv_log_mean(nd[a].z, nd[b].z, lz[a], lz[b]);
                    curved_pair_shares<NQ>(tb, nd, ph, jr, a, b, rho_ln, izln, P.gm1i, acc);
                }
            }
        }
    }
}

// Whether the z phase holds its line's states in registers for the finish
// (HOLD) or the finish reads them again (L2 or last-level cache hits).  The
// metric terms and phi take 8 NQ registers per lane beyond the affine
// kernel's.  Up to N=3 the kernel fits two waves per SIMD either way and
// holding saves the second read (1-8% faster on the warped bubble).  At N=4
// holding costs half the occupancy (256 VGPRs plus 22 AGPRs against 242;
// reading again is 15% faster), and from N=5 on it costs AGPR copies and, at
// N=8, scratch spills (reading again is 6% faster at N=5 and 19% at N=8,
// even at N=6 and N=7).
template <int NQ>
constexpr bool curved_holds_states()
{
    return NQ <= 4;
}

// Waves per SIMD the curved kernel is compiled for (1: the compiler's
// choice).  At N=5 two waves spill 80 B per lane and run 28% faster than one
// wave with AGPR copies (warped 26^3 bubble); at N=6 two waves would spill
// 416 B, at N=4 the kernel fits two waves without spills.
template <int NQ>
constexpr int curved_min_waves()
{
    return NQ == 6 ? 2 : 1;
}

template <int NQ, int EPW, int MODE>
__device__ __forceinline__ void stage_curved_body(const CurvedParams &C, int lb)
{
    constexpr int NQ2 = NQ * NQ, NQ3 = NQ2 * NQ;
    __shared__ double sacc[5][EPW][NQ3];
    __shared__ double sphi[EPW][NQ3];
    const StageParams &P = C.s;
    const OrderTables &tb = c_tab[NQ - 2];
    const int tid = threadIdx.x;
    const int el = tid / NQ2;
    const int m = tid - el * NQ2;
    const int64_t it = (int64_t)lb * EPW + el;
    const bool act = (el < EPW) && (it < P.ne);
    int ec[3] = {0, 0, 0};
    int64_t e = 0;
    if (act) e = tile_element(P, it, ec);
    double acc[NQ][5];
    const bool vol_or_face = (P.mask & (TERM_VOL | TERM_FACE)) != 0;
    const int64_t base0 = e * 5 * NQ3 + m;

    // x phase
    if (act) {
        if (vol_or_face) {
            line_terms_curved<NQ, 0>(C, tb, m, e, ec, sphi[el], acc);
        } else {
#pragma unroll
            for (int t = 0; t < NQ; ++t) {
                const int n = line_node<NQ, 0>(m, t);
                sphi[el][n] = C.phi[e * NQ3 + n];
#pragma unroll
                for (int v = 0; v < 5; ++v) acc[t][v] = 0.0;
            }
        }
#pragma unroll
        for (int t = 0; t < NQ; ++t) {
            const int n = line_node<NQ, 0>(m, t);
#pragma unroll
            for (int v = 0; v < 5; ++v) sacc[v][el][n] = acc[t][v];
        }
    }
    __syncthreads();
    // y phase
    if (act && vol_or_face) {
        line_terms_curved<NQ, 1>(C, tb, m, e, ec, sphi[el], acc);
#pragma unroll
        for (int t = 0; t < NQ; ++t) {
            const int n = line_node<NQ, 1>(m, t);
#pragma unroll
            for (int v = 0; v < 5; ++v) sacc[v][el][n] += acc[t][v];
        }
    }
    __syncthreads();
    // z phase and finish
    if (!act) return;
    const bool src = (P.mask & TERM_SRC) != 0;
    constexpr bool HOLD = curved_holds_states<NQ>();
    double qv[HOLD ? NQ : 1][5];
    if (vol_or_face) {
        line_terms_curved<NQ, 2, HOLD>(C, tb, m, e, ec, sphi[el], acc, qv);
    } else {
#pragma unroll
        for (int t = 0; t < NQ; ++t)
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                acc[t][v] = 0.0;
                if constexpr (HOLD) qv[t][v] = P.q_in[base0 + v * NQ3 + NQ2 * t];
            }
    }
    const bool use_dq = P.A != 0.0;
    double dv[NQ][5];
    if (MODE == MODE_STAGE && use_dq) {
#pragma unroll
        for (int t = 0; t < NQ; ++t)
#pragma unroll
            for (int v = 0; v < 5; ++v) dv[t][v] = P.dq[base0 + v * NQ3 + NQ2 * t];
    }
    bool bad = false;
#pragma unroll
    for (int t = 0; t < NQ; ++t) {
        const int n = m + NQ2 * t;
        double qn[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            if constexpr (HOLD)
                qn[v] = qv[t][v];
            else
                qn[v] = P.q_in[base0 + v * NQ3 + NQ2 * t];
        }
        const double iJ = C.iJ[e * NQ3 + n];
        double Rv[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) Rv[v] = (sacc[v][el][n] + acc[t][v]) * iJ;
        if (src) {
            Rv[1] += P.cor_f * qn[2];
            Rv[2] -= P.cor_f * qn[1];
        }
        if (MODE == MODE_RHS) {
#pragma unroll
            for (int v = 0; v < 5; ++v) store_f64<true>(&P.r_out[base0 + v * NQ3 + NQ2 * t], Rv[v]);
        } else {
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const double d = use_dq ? P.A * dv[t][v] + P.dt * Rv[v] : P.dt * Rv[v];
                P.dq[base0 + v * NQ3 + NQ2 * t] = d;
                P.q_out[base0 + v * NQ3 + NQ2 * t] = qn[v] + P.B * d;
            }
        }
        if (P.flag) {
            const double r = qn[0];
            const double kin = qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3];
            const double eint = qn[4] - 0.5 * kin / r - r * sphi[el][n];
            bad |= !(r > 0.0) || !(eint > 0.0);
        }
    }
    if (bad) atomicOr(P.flag, 1);
}

template <int NQ, int EPW, int MODE>
__global__ void __launch_bounds__((block_threads<NQ, EPW>()), (curved_min_waves<NQ>()))
    stage_curved(const CurvedParams C)
{
    stage_curved_body<NQ, EPW, MODE>(C, xcd_remap(blockIdx.x, C.s.nblocks));
}

}  // namespace esdg
