/*
 * esdg_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.
 *
 * A plain, slow, FP64 CPU statement of the entropy-stable DGSEM right-hand
 * side R(q) for the 3-D compressible Euler equations with gravity (and an
 * f-plane Coriolis source) on a uniform box of affine hexahedra with
 * Legendre-Gauss-Lobatto (LGL) nodes, the Carpenter-Kennedy LSRK(5,4)
 * time step, and the entropy / conservation diagnostics.
 *
 * Only tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py
 * load this library.  It shares no source, table or constant with the HIP
 * library: every quantity below is computed here from its definition.
 *
 * Paper references (Waterhouse, Waruszewski, Wilcox, Warburton, Giraldo,
 * "GPU Performance of an Entropy-Stable Discontinuous Galerkin Euler Solver
 * with Non-Conservative Terms"):
 *   - governing equations, total energy with geopotential, pressure:
 *     Sec. 2, Eqs. (Eq:euler) and the pressure definition that follows;
 *   - semi-discrete form: Sec. 3, Eq. (nm:semi) and the operator list after
 *     it (G, D, F, F*, M, M^s); the printed equation is read as the
 *     Jacobian-weighted skew (flux-differencing) form, see rhs_element();
 *   - averages, log-mean, jump and the momentum flux with the gravity term
 *     rho_hat [[phi]]/2: Sec. 4.1 (GPU optimizations), the displayed
 *     definitions of {{a}}, {{a}}_log, [[a]] and of the momentum flux;
 *   - Horner-series log-mean with per-node logarithms: Sec. 4.1 text;
 *   - LSRK(5,4) time stepping: Sec. 3, last paragraph.
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - mass/energy components of the entropy-conservative flux: Ranocha-type
 *     flux, with {{phi}} f^rho added to the energy flux because E contains
 *     rho*phi, and p* = {{p}};
 *   - log-mean series branch: u = ((b-a)/(b+a))^2 < 1e-4 uses
 *     (a+b) / (2 + u(2/3 + u(2/5 + u 2/7))), else (b-a)/(ln b - ln a);
 *   - face flux: entropy-conservative flux plus Rusanov (local Lax-Friedrichs)
 *     dissipation 0.5*lambda*(q+ - q-), lambda = max over both sides of
 *     |u.n| + c; ESDG_SURF_EC drops the dissipation; ESDG_SURF_MATRIX uses
 *     the entropy-stable matrix dissipation of matrix_dissipation() (the
 *     paper's choice, Sec. 3, whose formula it cites but does not print);
 *   - reflecting walls: mirror state (rho, m - 2 (m.n) n, E), phi+ = phi-;
 *   - Coriolis: f-plane, h = (0, f m_y, -f m_x, 0, 0);
 *   - curved hexahedra (oracle_mesh_create_warped): the box warped by a
 *     smooth displacement that vanishes on the box faces; metric terms in
 *     Kopriva's conservative curl form, volume flux with averaged metrics,
 *     face flux along the contravariant normal (Sec. 3: the metric terms G
 *     and the surface terms of the semi-discrete form), with the matrix
 *     dissipation written for a general unit normal;
 *   - time step: dt = CFL / ((N+1) max_a sum_r (|u_r| + c) / h_r).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NQMAX 16
#define SURF_RUSANOV 0
#define SURF_EC 1
#define SURF_MATRIX 2
#define TERM_VOL 1
#define TERM_FACE 2
#define TERM_SRC 4

/* the scalar of the pointwise physics in esdg_pointwise.h: plain FP64 here */
typedef double real;

typedef struct {
    int N, Nq, Np;
    int K[3];
    int periodic[3];
    int surf;
    double lo[3], hi[3], h[3];
    double gamma, gas_R, grav, cor_f;
    double xi[NQMAX], w[NQMAX];
    double D[NQMAX][NQMAX];
    double S[NQMAX][NQMAX]; /* S = W D - (W D)^T, skew */
    int64_t ne, nn;
    double *xyz; /* [e][3][Np] node coordinates */
    double *phi; /* [e][Np] geopotential at the nodes */
    /* curved meshes only (NULL for the affine box): */
    double *Ja;  /* [e][r][d][Np] J a^r_d, the contravariant basis times J */
    double *Jd;  /* [e][Np] Jacobian determinant J */
} omesh;

/* ------------------------------------------------------------------------ */
/* LGL nodes, weights and differentiation matrix (textbook definitions)      */
/* ------------------------------------------------------------------------ */

/* Legendre P_n(x) and P_{n-1}(x) by the three-term recurrence. */
static void legendre_pair(int n, long double x, long double *pn, long double *pnm1)
{
    long double p0 = 1.0L, p1 = x;
    if (n == 0) { *pn = 1.0L; *pnm1 = 0.0L; return; }
    for (int k = 2; k <= n; ++k) {
        long double p2 = ((2.0L * k - 1.0L) * x * p1 - (k - 1.0L) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    *pn = p1;
    *pnm1 = p0;
}

/* LGL nodes are -1, +1 and the N-1 roots of P_N'(x).  Interior roots by
 * Newton's method on P_N' using P_N'' from the Legendre ODE
 * (1-x^2) P'' = 2x P' - N(N+1) P, started at Chebyshev-Lobatto points.
 * Weights w_i = 2 / (N(N+1) P_N(x_i)^2).  D_ij = P_N(x_i)/(P_N(x_j)(x_i-x_j))
 * for i != j, D_00 = -N(N+1)/4, D_NN = N(N+1)/4, other diagonals 0. */
void oracle_lgl(int N, double *x, double *w, double *D)
{
    int Nq = N + 1;
    long double X[NQMAX];
    X[0] = -1.0L;
    X[N] = 1.0L;
    for (int i = 1; i < N; ++i) {
        long double t = -cosl(3.14159265358979323846264338327950288L * i / N);
        for (int it = 0; it < 100; ++it) {
            long double pn, pnm1;
            legendre_pair(N, t, &pn, &pnm1);
            /* P_N'(t) = N (t P_N - P_{N-1}) / (t^2 - 1) */
            long double dp = N * (t * pn - pnm1) / (t * t - 1.0L);
            long double d2p = (2.0L * t * dp - N * (N + 1.0L) * pn) / (1.0L - t * t);
            long double dt = dp / d2p;
            t -= dt;
            if (fabsl(dt) < 1e-19L) break;
        }
        X[i] = t;
    }
    /* exact symmetry of the node set */
    for (int i = 0; i < Nq / 2; ++i) {
        long double s = 0.5L * (X[N - i] - X[i]);
        X[N - i] = s;
        X[i] = -s;
    }
    if (N % 2 == 0) X[N / 2] = 0.0L;
    long double P[NQMAX];
    for (int i = 0; i < Nq; ++i) {
        long double pnm1;
        legendre_pair(N, X[i], &P[i], &pnm1);
        x[i] = (double)X[i];
        w[i] = (double)(2.0L / (N * (N + 1.0L) * P[i] * P[i]));
    }
    for (int i = 0; i < Nq; ++i)
        for (int j = 0; j < Nq; ++j) {
            long double v;
            if (i != j) v = P[i] / (P[j] * (X[i] - X[j]));
            else if (i == 0) v = -N * (N + 1.0L) / 4.0L;
            else if (i == N) v = N * (N + 1.0L) / 4.0L;
            else v = 0.0L;
            D[i * Nq + j] = (double)v;
        }
}

/* ------------------------------------------------------------------------ */
/* Mesh                                                                      */
/* ------------------------------------------------------------------------ */

static inline int64_t elem_index(const omesh *m, int ex, int ey, int ez)
{
    return ex + (int64_t)m->K[0] * (ey + (int64_t)m->K[1] * ez);
}

/* Vertex d-coordinate of element boundary e (0..K): lo + (hi-lo)*e/K. */
static double vertex(const omesh *m, int d, int e)
{
    return m->lo[d] + (m->hi[d] - m->lo[d]) * ((double)e / (double)m->K[d]);
}

void *oracle_mesh_create(int N, const int *K, const double *lo, const double *hi,
                         const int *periodic, double gamma, double gas_R, double grav,
                         double cor_f, int surf)
{
    if (N < 1 || N >= NQMAX) return NULL;
    for (int d = 0; d < 3; ++d)
        if (K[d] < 1 || !(hi[d] > lo[d])) return NULL;
    omesh *m = (omesh *)calloc(1, sizeof(omesh));
    if (!m) return NULL;
    m->N = N;
    m->Nq = N + 1;
    m->Np = m->Nq * m->Nq * m->Nq;
    for (int d = 0; d < 3; ++d) {
        m->K[d] = K[d];
        m->lo[d] = lo[d];
        m->hi[d] = hi[d];
        m->periodic[d] = periodic[d] ? 1 : 0;
        m->h[d] = (hi[d] - lo[d]) / K[d];
    }
    m->gamma = gamma;
    m->gas_R = gas_R;
    m->grav = grav;
    m->cor_f = cor_f;
    m->surf = surf;
    double Dm[NQMAX * NQMAX];
    oracle_lgl(N, m->xi, m->w, Dm);
    for (int i = 0; i < m->Nq; ++i)
        for (int j = 0; j < m->Nq; ++j) m->D[i][j] = Dm[i * m->Nq + j];
    for (int i = 0; i < m->Nq; ++i)
        for (int j = 0; j < m->Nq; ++j)
            m->S[i][j] = m->w[i] * m->D[i][j] - m->w[j] * m->D[j][i];
    m->ne = (int64_t)K[0] * K[1] * K[2];
    m->nn = m->ne * m->Np;
    m->xyz = (double *)malloc(sizeof(double) * 3 * m->nn);
    m->phi = (double *)malloc(sizeof(double) * m->nn);
    if (!m->xyz || !m->phi) {
        free(m->xyz);
        free(m->phi);
        free(m);
        return NULL;
    }
    const int Nq = m->Nq, Np = m->Np;
    for (int ez = 0; ez < K[2]; ++ez)
        for (int ey = 0; ey < K[1]; ++ey)
            for (int ex = 0; ex < K[0]; ++ex) {
                int64_t e = elem_index(m, ex, ey, ez);
                int ee[3] = {ex, ey, ez};
                double XL[3], XR[3];
                for (int d = 0; d < 3; ++d) {
                    XL[d] = vertex(m, d, ee[d]);
                    XR[d] = vertex(m, d, ee[d] + 1);
                }
                for (int k = 0; k < Nq; ++k)
                    for (int j = 0; j < Nq; ++j)
                        for (int i = 0; i < Nq; ++i) {
                            int n = i + Nq * (j + Nq * k);
                            int ii[3] = {i, j, k};
                            for (int d = 0; d < 3; ++d) {
                                double s = m->xi[ii[d]];
                                /* affine map from the shared vertices: the face
                                 * nodes of two neighbours coincide bitwise */
                                double x = 0.5 * (1.0 - s) * XL[d] + 0.5 * (1.0 + s) * XR[d];
                                m->xyz[(e * 3 + d) * Np + n] = x;
                            }
                            m->phi[e * Np + n] = grav * m->xyz[(e * 3 + 2) * Np + n];
                        }
            }
    return m;
}

void oracle_mesh_destroy(void *mp)
{
    omesh *m = (omesh *)mp;
    if (!m) return;
    free(m->xyz);
    free(m->phi);
    free(m->Ja);
    free(m->Jd);
    free(m);
}

/* sin(2 pi k s), exactly 0 at s = 0 and s = 1 (the box faces). */
static double sin2pik(int k, double s)
{
    if (s == 0.0 || s == 1.0) return 0.0;
    return sin(2.0 * 3.14159265358979323846 * k * s);
}

/* Derivative along reference direction j of the nodal field f of one
 * element, at node n: sum_l D[i_j(n)][l] f(n with i_j = l). */
static double dref(const omesh *m, const double *f, int n, int j)
{
    const int Nq = m->Nq;
    int ii[3] = {n % Nq, (n / Nq) % Nq, n / (Nq * Nq)};
    double acc = 0.0;
    for (int l = 0; l < Nq; ++l) {
        int jj[3] = {ii[0], ii[1], ii[2]};
        jj[j] = l;
        acc += m->D[ii[j]][l] * f[jj[0] + Nq * (jj[1] + Nq * jj[2])];
    }
    return acc;
}

/* Metric terms of one element from its nodal coordinates X (Sec. 3, the
 * metric terms G of the semi-discrete form), in the conservative curl form
 *   J a^i_n = -e_i . curl_xi( X_l grad_xi X_m ),   (n, m, l) cyclic,
 * with every derivative the LGL derivative D.  This form satisfies the
 * discrete metric identities sum_i d/dxi_i (J a^i_n) = 0, which keep a
 * uniform flow uniform.  J = det(dX/dxi). */
static void element_metrics(const omesh *m, int64_t e, double *Ja, double *Jd)
{
    const int Np = m->Np;
    const double *X[3];
    for (int d = 0; d < 3; ++d) X[d] = m->xyz + (e * 3 + d) * Np;
    double *dX = (double *)malloc(sizeof(double) * 9 * Np); /* [m][j][n] */
    double *Y = (double *)malloc(sizeof(double) * 3 * Np);  /* [j][n] */
    for (int mm = 0; mm < 3; ++mm)
        for (int j = 0; j < 3; ++j)
            for (int n = 0; n < Np; ++n) dX[(mm * 3 + j) * Np + n] = dref(m, X[mm], n, j);
    for (int n = 0; n < Np; ++n) {
        const double *a0 = dX, *a1 = dX + 3 * Np, *a2 = dX + 6 * Np;
        /* rows: d X_0/d xi_j, d X_1/d xi_j, d X_2/d xi_j */
        double A[3][3];
        for (int j = 0; j < 3; ++j) {
            A[0][j] = a0[j * Np + n];
            A[1][j] = a1[j * Np + n];
            A[2][j] = a2[j * Np + n];
        }
        Jd[n] = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    }
    for (int nn = 0; nn < 3; ++nn) {
        int mm = (nn + 1) % 3, l = (nn + 2) % 3;
        for (int j = 0; j < 3; ++j)
            for (int n = 0; n < Np; ++n) Y[j * Np + n] = X[l][n] * dX[(mm * 3 + j) * Np + n];
        for (int i = 0; i < 3; ++i) {
            int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
            for (int n = 0; n < Np; ++n) {
                double curl = dref(m, Y + i2 * Np, n, i1) - dref(m, Y + i1 * Np, n, i2);
                Ja[(i * 3 + nn) * Np + n] = -curl;
            }
        }
    }
    free(dX);
    free(Y);
}

/* Curved mesh: the box of oracle_mesh_create with every node displaced by
 *   X_d = x_d + warp_d L_d prod_c sin(2 pi k_dc s_c),   s = (x - lo)/L,
 * k_dc = 2 for c = d > 0 and 1 otherwise (each coordinate gets a field of
 * its own, so that the metric terms are not the special case of a
 * displacement along one fixed direction).  The displacement vanishes on
 * the box faces, so walls stay planar and periodic faces still match;
 * interior faces are curved.  With warp = (0, 0, 0) the curved code path
 * runs on the affine box. */
void *oracle_mesh_create_warped(int N, const int *K, const double *lo, const double *hi,
                                const int *periodic, double gamma, double gas_R, double grav,
                                double cor_f, int surf, const double *warp)
{
    omesh *m = (omesh *)oracle_mesh_create(N, K, lo, hi, periodic, gamma, gas_R, grav, cor_f,
                                           surf);
    if (!m) return NULL;
    const int Np = m->Np;
    m->Ja = (double *)malloc(sizeof(double) * 9 * m->nn);
    m->Jd = (double *)malloc(sizeof(double) * m->nn);
    if (!m->Ja || !m->Jd) {
        oracle_mesh_destroy(m);
        return NULL;
    }
    double L[3];
    for (int d = 0; d < 3; ++d) L[d] = hi[d] - lo[d];
    for (int64_t e = 0; e < m->ne; ++e)
        for (int n = 0; n < Np; ++n) {
            double x[3], sv[3];
            for (int c = 0; c < 3; ++c) {
                x[c] = m->xyz[(e * 3 + c) * Np + n];
                sv[c] = (x[c] - lo[c]) / L[c];
            }
            for (int d = 0; d < 3; ++d) {
                double sn = 1.0;
                for (int c = 0; c < 3; ++c) sn *= sin2pik((c == d && d > 0) ? 2 : 1, sv[c]);
                m->xyz[(e * 3 + d) * Np + n] = x[d] + warp[d] * L[d] * sn;
            }
            m->phi[e * Np + n] = grav * m->xyz[(e * 3 + 2) * Np + n];
        }
    for (int64_t e = 0; e < m->ne; ++e)
        element_metrics(m, e, m->Ja + e * 9 * Np, m->Jd + e * Np);
    for (int64_t i = 0; i < m->nn; ++i)
        if (!(m->Jd[i] > 0.0)) {
            oracle_mesh_destroy(m);
            return NULL;
        }
    return m;
}

void oracle_metrics(void *mp, double *Ja, double *Jd)
{
    omesh *m = (omesh *)mp;
    if (!m->Ja) return;
    memcpy(Ja, m->Ja, sizeof(double) * 9 * m->nn);
    memcpy(Jd, m->Jd, sizeof(double) * m->nn);
}

int64_t oracle_mesh_nelem(void *mp) { return ((omesh *)mp)->ne; }

void oracle_node_coords(void *mp, double *xyz)
{
    omesh *m = (omesh *)mp;
    memcpy(xyz, m->xyz, sizeof(double) * 3 * m->nn);
}

void oracle_get_phi(void *mp, double *phi)
{
    omesh *m = (omesh *)mp;
    memcpy(phi, m->phi, sizeof(double) * m->nn);
}

/* Replace the nodal geopotential (used to test entropy conservation with a
 * gravity term on a fully periodic box, where phi = g z is not periodic). */
void oracle_set_phi(void *mp, const double *phi)
{
    omesh *m = (omesh *)mp;
    memcpy(m->phi, phi, sizeof(double) * m->nn);
}

void oracle_tables(void *mp, double *xi, double *w, double *D, double *S)
{
    omesh *m = (omesh *)mp;
    for (int i = 0; i < m->Nq; ++i) {
        xi[i] = m->xi[i];
        w[i] = m->w[i];
        for (int j = 0; j < m->Nq; ++j) {
            D[i * m->Nq + j] = m->D[i][j];
            S[i * m->Nq + j] = m->S[i][j];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Pointwise physics                                                         */
/* ------------------------------------------------------------------------ */
#include "esdg_pointwise.h"

/* Physical Euler flux in direction r (conservative form of Eq:euler). */
void oracle_euler_flux(int r, const double q[5], double phi, double gamma, double f[5])
{
    double p = pressure(q, phi, gamma);
    double ur = q[1 + r] / q[0];
    f[0] = q[1 + r];
    for (int c = 0; c < 3; ++c) f[1 + c] = q[1 + c] * ur + (c == r ? p : 0.0);
    f[4] = (q[4] + p) * ur;
}


/* The matrix dissipation above for a general unit normal n (curved faces).
 * The acoustic and entropy eigenvectors keep their form with n in place of
 * e_r.  The two shear eigenvectors (0, t, u_hat.t) span the tangent plane;
 * whatever tangents are chosen, together they contribute
 *   |u_n| p_hat (0, P w, u_hat . P w),   w = [[v]]_m + u_hat [[v]]_5,
 * with P = I - n n^T the projector onto the tangent plane, so no tangents are
 * formed.  For n = e_r this is matrix_dissipation(r, ...). */
static void matrix_dissipation_vec(const double nv[3], const double qm[5], const double qp[5],
                                   double phi, double gamma, double D[5])
{
    double gm1 = gamma - 1.0;
    double rm = qm[0], rp = qp[0], um[3], up[3];
    for (int c = 0; c < 3; ++c) {
        um[c] = qm[1 + c] / rm;
        up[c] = qp[1 + c] / rp;
    }
    double pm = pressure(qm, phi, gamma), pp = pressure(qp, phi, gamma);
    double bm = rm / (2.0 * pm), bp = rp / (2.0 * pp);
    double uum = um[0] * um[0] + um[1] * um[1] + um[2] * um[2];
    double uup = up[0] * up[0] + up[1] * up[1] + up[2] * up[2];
    double rho_hat = oracle_logmean(rm, rp);
    double b_ln = oracle_logmean(bm, bp);
    double uh[3];
    for (int c = 0; c < 3; ++c) uh[c] = 0.5 * (um[c] + up[c]);
    double p_hat = 0.5 * (rm + rp) / (2.0 * 0.5 * (bm + bp));
    double u2bar = 2.0 * (uh[0] * uh[0] + uh[1] * uh[1] + uh[2] * uh[2]) - 0.5 * (uum + uup);
    double h_hat = gamma / (2.0 * gm1 * b_ln) + 0.5 * u2bar;
    double a_hat = sqrt(gamma * p_hat / rho_hat);
    double ds = log(pp / pm) - gamma * log(rp / rm);
    double dv[5];
    dv[0] = -ds / gm1 - (bp * uup - bm * uum);
    for (int c = 0; c < 3; ++c) dv[1 + c] = 2.0 * (bp * up[c] - bm * um[c]);
    dv[4] = -2.0 * (bp - bm);

    double un = uh[0] * nv[0] + uh[1] * nv[1] + uh[2] * nv[2];
    /* acoustic (-), entropy and acoustic (+) eigenvectors as columns */
    double Rm[5][3];
    Rm[0][0] = Rm[0][1] = Rm[0][2] = 1.0;
    for (int c = 0; c < 3; ++c) {
        Rm[1 + c][0] = uh[c] - a_hat * nv[c];
        Rm[1 + c][1] = uh[c];
        Rm[1 + c][2] = uh[c] + a_hat * nv[c];
    }
    Rm[4][0] = h_hat - a_hat * un;
    Rm[4][1] = 0.5 * u2bar;
    Rm[4][2] = h_hat + a_hat * un;
    double lam[3] = {fabs(un - a_hat), fabs(un), fabs(un + a_hat)};
    double tsc[3] = {rho_hat / (2.0 * gamma), rho_hat * gm1 / gamma, rho_hat / (2.0 * gamma)};
    double w[3];
    for (int k = 0; k < 3; ++k) {
        double acc = 0.0;
        for (int v = 0; v < 5; ++v) acc += Rm[v][k] * dv[v];
        w[k] = lam[k] * tsc[k] * acc;
    }
    for (int v = 0; v < 5; ++v) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += Rm[v][k] * w[k];
        D[v] = acc;
    }
    /* shear waves through the tangent projector */
    double wv[3], Pw[3];
    for (int c = 0; c < 3; ++c) wv[c] = dv[1 + c] + uh[c] * dv[4];
    double nw = wv[0] * nv[0] + wv[1] * nv[1] + wv[2] * nv[2];
    for (int c = 0; c < 3; ++c) Pw[c] = wv[c] - nv[c] * nw;
    double sh = fabs(un) * p_hat;
    for (int c = 0; c < 3; ++c) D[1 + c] += sh * Pw[c];
    D[4] += sh * (uh[0] * Pw[0] + uh[1] * Pw[1] + uh[2] * Pw[2]);
    D[4] += phi * D[0];
}


/* Face flux along a general (unnormalised) normal Nv = s J a^r of a curved
 * element: sum_d Nv_d f_d(q-, q+) minus the Rusanov dissipation
 * |Nv| lambda/2 (q+ - q-), lambda = max(|u.n| + c) with n = Nv/|Nv|, minus
 * |Nv| D(n)/2 with the matrix dissipation for the unit normal n, or without
 * dissipation (EC).  Faces have phi+ = phi-. */
void oracle_surface_flux_vec(const double Nv[3], const double qm[5], const double qp[5],
                             double phim, double phip, double gamma, int surf, double Fn[5])
{
    for (int v = 0; v < 5; ++v) Fn[v] = 0.0;
    for (int d = 0; d < 3; ++d) {
        double F[5];
        oracle_two_point_flux(d, qm, qp, phim, phip, gamma, F);
        for (int v = 0; v < 5; ++v) Fn[v] += Nv[d] * F[v];
    }
    if (surf == SURF_EC) return;
    double nrm = sqrt(Nv[0] * Nv[0] + Nv[1] * Nv[1] + Nv[2] * Nv[2]);
    if (surf == SURF_MATRIX) {
        double nu[3] = {Nv[0] / nrm, Nv[1] / nrm, Nv[2] / nrm}, D[5];
        matrix_dissipation_vec(nu, qm, qp, phim, gamma, D);
        for (int v = 0; v < 5; ++v) Fn[v] -= 0.5 * nrm * D[v];
        return;
    }
    double lam = 0.0;
    const double *qs[2] = {qm, qp};
    double phis[2] = {phim, phip};
    for (int t = 0; t < 2; ++t) {
        const double *q = qs[t];
        double p = pressure(q, phis[t], gamma);
        double un = (q[1] * Nv[0] + q[2] * Nv[1] + q[3] * Nv[2]) / (q[0] * nrm);
        double l = fabs(un) + sqrt(gamma * p / q[0]);
        if (l > lam) lam = l;
    }
    for (int v = 0; v < 5; ++v) Fn[v] -= 0.5 * lam * nrm * (qp[v] - qm[v]);
}

/* Entropy variables of eta = -rho s/(gamma-1), s = ln p - gamma ln rho, for
 * total energy including rho*phi:
 * v = ((gamma - s)/(gamma-1) - b|u|^2 + 2 b phi, 2 b u, -2 b), b = rho/(2p). */
void oracle_entropy_vars(const double q[5], double phi, double gamma, double v[5])
{
    double rho = q[0];
    double p = pressure(q, phi, gamma);
    double b = rho / (2.0 * p);
    double u[3] = {q[1] / rho, q[2] / rho, q[3] / rho};
    double s = log(p) - gamma * log(rho);
    v[0] = (gamma - s) / (gamma - 1.0) - b * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) +
           2.0 * b * phi;
    v[1] = 2.0 * b * u[0];
    v[2] = 2.0 * b * u[1];
    v[3] = 2.0 * b * u[2];
    v[4] = -2.0 * b;
}

double oracle_entropy_density(const double q[5], double phi, double gamma)
{
    double p = pressure(q, phi, gamma);
    double s = log(p) - gamma * log(q[0]);
    return -q[0] * s / (gamma - 1.0);
}

/* ------------------------------------------------------------------------ */
/* Right-hand side                                                           */
/* ------------------------------------------------------------------------ */

static inline void load_node(const double *q, int64_t e, int Np, int n, double out[5])
{
    for (int v = 0; v < 5; ++v) out[v] = q[(e * 5 + v) * Np + n];
}

/* Neighbour across the face of element (ex,ey,ez) in direction r, side s.
 * Returns the neighbour element index, or -1 at a reflecting wall. */
static int64_t neighbour(const omesh *m, const int ee[3], int r, int s)
{
    int nb[3] = {ee[0], ee[1], ee[2]};
    nb[r] += s;
    if (nb[r] < 0 || nb[r] >= m->K[r]) {
        if (!m->periodic[r]) return -1;
        nb[r] = (nb[r] + m->K[r]) % m->K[r];
    }
    return elem_index(m, nb[0], nb[1], nb[2]);
}

/* Plus-side state at face node n of element e (own node index ii[]) in
 * direction r, side s: the neighbour's coincident node, or the mirror state
 * (rho, m - 2 (m.n) n, E) with phi+ = phi- at a wall. */
static void plus_state(const omesh *m, const double *q, int64_t e, const int ee[3],
                       const int ii[3], int r, int s, double qp[5], double *phip)
{
    int64_t en = neighbour(m, ee, r, s);
    const int Nq = m->Nq, Np = m->Np;
    int n = ii[0] + Nq * (ii[1] + Nq * ii[2]);
    if (en < 0) {
        load_node(q, e, Np, n, qp);
        qp[1 + r] = -qp[1 + r];
        *phip = m->phi[e * Np + n];
        return;
    }
    int jj[3] = {ii[0], ii[1], ii[2]};
    jj[r] = (s < 0) ? m->N : 0;
    int nn = jj[0] + Nq * (jj[1] + Nq * jj[2]);
    load_node(q, en, Np, nn, qp);
    *phip = m->phi[en * Np + nn];
}

/* R for one element of a curved mesh: the skew form with averaged metrics,
 *   R_a = h_a - (1/J_a) sum_r (1/w_{i_r(a)}) sum_{b on the r-line of a}
 *                 S_{i_r(a) i_r(b)} sum_d {{J a^r_d}}_ab F_d(a, b)
 *         - sum over faces of a: (1/(J_a w_0)) F*(q_a, q+; s J a^r(a)),
 * where F_d is the two-point flux of direction d (gravity term included) and
 * {{.}}_ab the average of the two nodes' metric terms.  On the affine box
 * J a^r_d = J (2/h_r) delta_rd and this is rhs_element's sum. */
static void rhs_element_curved(const omesh *m, const double *q, double *R, double *gross,
                               int64_t e, int mask)
{
    const int N = m->N, Nq = m->Nq, Np = m->Np;
    int ee[3];
    ee[0] = (int)(e % m->K[0]);
    ee[1] = (int)((e / m->K[0]) % m->K[1]);
    ee[2] = (int)(e / ((int64_t)m->K[0] * m->K[1]));
    const double *Ja = m->Ja + e * 9 * Np;
    for (int a = 0; a < Np; ++a) {
        int ii[3] = {a % Nq, (a / Nq) % Nq, a / (Nq * Nq)};
        double qa[5], acc[5] = {0, 0, 0, 0, 0}, gacc[5] = {0, 0, 0, 0, 0};
        load_node(q, e, Np, a, qa);
        double phia = m->phi[e * Np + a];
        double iJ = 1.0 / m->Jd[e * Np + a];
        if (mask & TERM_VOL) {
            for (int r = 0; r < 3; ++r) {
                int ia = ii[r];
                for (int l = 0; l < Nq; ++l) {
                    if (l == ia) continue;
                    int jj[3] = {ii[0], ii[1], ii[2]};
                    jj[r] = l;
                    int b = jj[0] + Nq * (jj[1] + Nq * jj[2]);
                    double qb[5], Ft[5] = {0, 0, 0, 0, 0};
                    load_node(q, e, Np, b, qb);
                    for (int d = 0; d < 3; ++d) {
                        double F[5];
                        oracle_two_point_flux(d, qa, qb, phia, m->phi[e * Np + b], m->gamma, F);
                        double jav = 0.5 * (Ja[(r * 3 + d) * Np + a] + Ja[(r * 3 + d) * Np + b]);
                        for (int v = 0; v < 5; ++v) Ft[v] += jav * F[v];
                    }
                    double coef = -iJ * m->S[ia][l] / m->w[ia];
                    for (int v = 0; v < 5; ++v) {
                        acc[v] += coef * Ft[v];
                        gacc[v] += fabs(coef * Ft[v]);
                    }
                }
            }
        }
        if (mask & TERM_FACE) {
            for (int r = 0; r < 3; ++r) {
                int sides[2] = {0, 0}, ns = 0;
                if (ii[r] == 0) sides[ns++] = -1;
                if (ii[r] == N) sides[ns++] = +1;
                for (int t = 0; t < ns; ++t) {
                    int s = sides[t];
                    double qp[5], phip, Fn[5], Nv[3];
                    plus_state(m, q, e, ee, ii, r, s, qp, &phip);
                    for (int d = 0; d < 3; ++d) Nv[d] = s * Ja[(r * 3 + d) * Np + a];
                    oracle_surface_flux_vec(Nv, qa, qp, phia, phip, m->gamma, m->surf, Fn);
                    double coef = -iJ / m->w[ii[r]];
                    for (int v = 0; v < 5; ++v) {
                        acc[v] += coef * Fn[v];
                        gacc[v] += fabs(coef * Fn[v]);
                    }
                }
            }
        }
        if (mask & TERM_SRC) {
            coriolis_source(m->cor_f, qa, acc);
            gacc[1] += fabs(m->cor_f * qa[2]);
            gacc[2] += fabs(m->cor_f * qa[1]);
        }
        for (int v = 0; v < 5; ++v) {
            R[(e * 5 + v) * Np + a] = acc[v];
            if (gross) gross[(e * 5 + v) * Np + a] = gacc[v];
        }
    }
}

/* R for one element in the skew (flux-differencing) form that the printed
 * semi-discrete equation (nm:semi) stands for on affine hexahedra:
 *   R_a = h_a - sum_r (2/h_r)(1/w_{i_r(a)}) sum_{b on the r-line of a}
 *                   S_{i_r(a) i_r(b)} F_r(a, b)
 *         - sum over faces of a: (2/h_r)(1/w_0) F*.n
 * with S = W D - (W D)^T.  Every ordered pair (a, b) is evaluated; nothing
 * uses the flux symmetry.  `gross` (if not NULL) receives the sum of the
 * absolute values of all terms, used as the scale of roundoff. */
static void rhs_element(const omesh *m, const double *q, double *R, double *gross,
                        int64_t e, int mask)
{
    if (m->Ja) {
        rhs_element_curved(m, q, R, gross, e, mask);
        return;
    }
    const int N = m->N, Nq = m->Nq, Np = m->Np;
    int ee[3];
    ee[0] = (int)(e % m->K[0]);
    ee[1] = (int)((e / m->K[0]) % m->K[1]);
    ee[2] = (int)(e / ((int64_t)m->K[0] * m->K[1]));
    for (int k = 0; k < Nq; ++k)
        for (int j = 0; j < Nq; ++j)
            for (int i = 0; i < Nq; ++i) {
                int ii[3] = {i, j, k};
                int a = i + Nq * (j + Nq * k);
                double qa[5], acc[5] = {0, 0, 0, 0, 0}, gacc[5] = {0, 0, 0, 0, 0};
                load_node(q, e, Np, a, qa);
                double phia = m->phi[e * Np + a];
                if (mask & TERM_VOL) {
                    for (int r = 0; r < 3; ++r) {
                        int ia = ii[r];
                        for (int l = 0; l < Nq; ++l) {
                            if (l == ia) continue;
                            int jj[3] = {i, j, k};
                            jj[r] = l;
                            int b = jj[0] + Nq * (jj[1] + Nq * jj[2]);
                            double qb[5], F[5];
                            load_node(q, e, Np, b, qb);
                            oracle_two_point_flux(r, qa, qb, phia, m->phi[e * Np + b], m->gamma, F);
                            double coef = -(2.0 / m->h[r]) * m->S[ia][l] / m->w[ia];
                            for (int v = 0; v < 5; ++v) {
                                acc[v] += coef * F[v];
                                gacc[v] += fabs(coef * F[v]);
                            }
                        }
                    }
                }
                if (mask & TERM_FACE) {
                    for (int r = 0; r < 3; ++r) {
                        int sides[2] = {0, 0}, ns = 0;
                        if (ii[r] == 0) sides[ns++] = -1;
                        if (ii[r] == N) sides[ns++] = +1;
                        for (int t = 0; t < ns; ++t) {
                            int s = sides[t];
                            double qp[5], phip, Fn[5];
                            plus_state(m, q, e, ee, ii, r, s, qp, &phip);
                            oracle_surface_flux(r, s, qa, qp, phia, phip, m->gamma, m->surf, Fn);
                            double coef = -(2.0 / m->h[r]) / m->w[ii[r]];
                            for (int v = 0; v < 5; ++v) {
                                acc[v] += coef * Fn[v];
                                gacc[v] += fabs(coef * Fn[v]);
                            }
                        }
                    }
                }
                if (mask & TERM_SRC) {
                    coriolis_source(m->cor_f, qa, acc);
                    gacc[1] += fabs(m->cor_f * qa[2]);
                    gacc[2] += fabs(m->cor_f * qa[1]);
                }
                for (int v = 0; v < 5; ++v) {
                    R[(e * 5 + v) * Np + a] = acc[v];
                    if (gross) gross[(e * 5 + v) * Np + a] = gacc[v];
                }
            }
}

int oracle_rhs_terms(void *mp, const double *q, double *R, double *gross, int mask)
{
    omesh *m = (omesh *)mp;
    int64_t e;
#pragma omp parallel for schedule(static)
    for (e = 0; e < m->ne; ++e) rhs_element(m, q, R, gross, e, mask);
    return 0;
}

int oracle_rhs(void *mp, const double *q, double *R)
{
    return oracle_rhs_terms(mp, q, R, NULL, TERM_VOL | TERM_FACE | TERM_SRC);
}

/* R (and gross) only for the listed elements; other entries untouched. */
int oracle_rhs_elems(void *mp, const double *q, double *R, double *gross, int mask,
                     const int64_t *elems, int64_t nelems)
{
    omesh *m = (omesh *)mp;
    int64_t t;
#pragma omp parallel for schedule(dynamic, 1)
    for (t = 0; t < nelems; ++t) rhs_element(m, q, R, gross, elems[t], mask);
    return 0;
}

/* Brute-force strong form, written independently of the skew form:
 *   R_a = h_a - sum_r (2/h_r) [ sum_l 2 D_{i l} F_r(a, b_l)              (l = i included)
 *                              + (F*.n - s f_r(q_a)) / w_{i}  at faces ]
 * where f_r is the physical Euler flux.  Exactly equal to the skew form in
 * exact arithmetic (summation by parts); used to pin it on tiny meshes. */
int oracle_rhs_strong(void *mp, const double *q, double *R)
{
    omesh *m = (omesh *)mp;
    if (m->Ja) return -1; /* affine boxes only */
    const int N = m->N, Nq = m->Nq, Np = m->Np;
    for (int64_t e = 0; e < m->ne; ++e) {
        int ee[3];
        ee[0] = (int)(e % m->K[0]);
        ee[1] = (int)((e / m->K[0]) % m->K[1]);
        ee[2] = (int)(e / ((int64_t)m->K[0] * m->K[1]));
        for (int a = 0; a < Np; ++a) {
            int ii[3] = {a % Nq, (a / Nq) % Nq, a / (Nq * Nq)};
            double qa[5], acc[5] = {0, 0, 0, 0, 0};
            load_node(q, e, Np, a, qa);
            double phia = m->phi[e * Np + a];
            for (int r = 0; r < 3; ++r) {
                double sum[5] = {0, 0, 0, 0, 0};
                for (int l = 0; l < Nq; ++l) {
                    int jj[3] = {ii[0], ii[1], ii[2]};
                    jj[r] = l;
                    int b = jj[0] + Nq * (jj[1] + Nq * jj[2]);
                    double qb[5], F[5];
                    load_node(q, e, Np, b, qb);
                    oracle_two_point_flux(r, qa, qb, phia, m->phi[e * Np + b], m->gamma, F);
                    for (int v = 0; v < 5; ++v) sum[v] += 2.0 * m->D[ii[r]][l] * F[v];
                }
                for (int s = -1; s <= 1; s += 2) {
                    if ((s < 0 && ii[r] != 0) || (s > 0 && ii[r] != N)) continue;
                    double qp[5], phip, Fn[5], f[5];
                    plus_state(m, q, e, ee, ii, r, s, qp, &phip);
                    oracle_surface_flux(r, s, qa, qp, phia, phip, m->gamma, m->surf, Fn);
                    oracle_euler_flux(r, qa, phia, m->gamma, f);
                    for (int v = 0; v < 5; ++v) sum[v] += (Fn[v] - s * f[v]) / m->w[ii[r]];
                }
                for (int v = 0; v < 5; ++v) acc[v] -= (2.0 / m->h[r]) * sum[v];
            }
            acc[1] += m->cor_f * qa[2];
            acc[2] -= m->cor_f * qa[1];
            for (int v = 0; v < 5; ++v) R[(e * 5 + v) * Np + a] = acc[v];
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* LSRK(5,4), 2N-storage (Carpenter & Kennedy 1994)                          */
/* ------------------------------------------------------------------------ */

static const double LSRK_A[5] = {
    0.0,
    -567301805773.0 / 1357537059087.0,
    -2404267990393.0 / 2016746695238.0,
    -3550918686646.0 / 2091501179385.0,
    -1275806237668.0 / 842570457699.0,
};
static const double LSRK_B[5] = {
    1432997174477.0 / 9575080441755.0,
    5161836677717.0 / 13612068292357.0,
    1720146321549.0 / 2090206949498.0,
    3134564353537.0 / 4481467310338.0,
    2277821191437.0 / 14882151754819.0,
};
static const double LSRK_C[5] = {
    0.0,
    1432997174477.0 / 9575080441755.0,
    2526269341429.0 / 6820363962896.0,
    2006345519317.0 / 3224310063776.0,
    2802321613138.0 / 2924317926251.0,
};

void oracle_lsrk_coeffs(double *A, double *B, double *C)
{
    for (int s = 0; s < 5; ++s) {
        A[s] = LSRK_A[s];
        B[s] = LSRK_B[s];
        C[s] = LSRK_C[s];
    }
}

typedef void (*rhs_fn)(void *ctx, const double *q, double *r, double t);

/* One 2N-storage step: for s = 1..5,
 *   dq <- A_s dq + dt R(q, t + C_s dt);  q <- q + B_s dq. */
static void lsrk_advance(int64_t n, double *q, double *dq, double *R, double t, double dt,
                         rhs_fn f, void *ctx)
{
    for (int s = 0; s < 5; ++s) {
        f(ctx, q, R, t + LSRK_C[s] * dt);
        for (int64_t i = 0; i < n; ++i) lsrk_update(LSRK_A[s], LSRK_B[s], dt, R[i], &dq[i], &q[i]);
    }
}

static void mesh_rhs_cb(void *ctx, const double *q, double *r, double t)
{
    (void)t;
    oracle_rhs(ctx, q, r);
}

/* One LSRK(5,4) step of the mesh ODE dq/dt = R(q), in place.  dq is the
 * caller's second register (its contents on entry are irrelevant: A_1 = 0). */
int oracle_lsrk_step(void *mp, double *q, double *dq, double t, double dt)
{
    omesh *m = (omesh *)mp;
    int64_t n = m->nn * 5;
    double *R = (double *)malloc(sizeof(double) * n);
    if (!R) return -1;
    lsrk_advance(n, q, dq, R, t, dt, mesh_rhs_cb, m);
    free(R);
    return 0;
}

typedef struct {
    int n;
    const double *M;
} lin_ctx;

static void lin_rhs_cb(void *ctx, const double *q, double *r, double t)
{
    (void)t;
    const lin_ctx *c = (const lin_ctx *)ctx;
    for (int i = 0; i < c->n; ++i) {
        double s = 0.0;
        for (int j = 0; j < c->n; ++j) s += c->M[i * c->n + j] * q[j];
        r[i] = s;
    }
}

typedef struct {
    int m;
} poly_ctx;

static void poly_rhs_cb(void *ctx, const double *q, double *r, double t)
{
    (void)q;
    const poly_ctx *c = (const poly_ctx *)ctx;
    r[0] = (c->m == 0) ? 1.0 : (double)c->m * pow(t, c->m - 1);
}

/* The same stepping routine applied to the linear ODE y' = M y (n <= 16),
 * used to read off the stability polynomial. */
int oracle_lsrk_linear(int n, const double *M, double *y, double dt, int nsteps)
{
    double dq[16] = {0}, R[16];
    if (n > 16) return -1;
    lin_ctx c = {n, M};
    for (int s = 0; s < nsteps; ++s) lsrk_advance(n, y, dq, R, 0.0, dt, lin_rhs_cb, &c);
    return 0;
}

/* The same stepping routine applied to y' = m t^(m-1), y(t0) = y0. */
double oracle_lsrk_poly(int mpow, double t0, double y0, double dt, int nsteps)
{
    double y = y0, dq = 0.0, R;
    poly_ctx c = {mpow};
    double t = t0;
    for (int s = 0; s < nsteps; ++s) {
        lsrk_advance(1, &y, &dq, &R, t, dt, poly_rhs_cb, &c);
        t += dt;
    }
    return y;
}

/* ------------------------------------------------------------------------ */
/* Diagnostics                                                               */
/* ------------------------------------------------------------------------ */

/* out[0] = sum_K int eta, out[1] = sum_K int rho, out[2] = sum_K int E,
 * out[3] = sum_a J w_a v_a . R_a(q) (the discrete entropy production),
 * all with the LGL quadrature and J = h_x h_y h_z / 8. */
int oracle_entropy(void *mp, const double *q, double *out)
{
    omesh *m = (omesh *)mp;
    const int Nq = m->Nq, Np = m->Np;
    double J = m->h[0] * m->h[1] * m->h[2] / 8.0;
    double *R = (double *)malloc(sizeof(double) * m->nn * 5);
    if (!R) return -1;
    oracle_rhs(mp, q, R);
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (int64_t e = 0; e < m->ne; ++e)
        for (int a = 0; a < Np; ++a) {
            int i = a % Nq, j = (a / Nq) % Nq, k = a / (Nq * Nq);
            double Jn = m->Jd ? m->Jd[e * Np + a] : J;
            double wq = Jn * m->w[i] * m->w[j] * m->w[k];
            double qa[5], v[5];
            load_node(q, e, Np, a, qa);
            double phi = m->phi[e * Np + a];
            oracle_entropy_vars(qa, phi, m->gamma, v);
            double vr = 0.0;
            for (int c = 0; c < 5; ++c) vr += v[c] * R[(e * 5 + c) * Np + a];
            s0 += wq * oracle_entropy_density(qa, phi, m->gamma);
            s1 += wq * qa[0];
            s2 += wq * qa[4];
            s3 += wq * vr;
        }
    free(R);
    out[0] = s0;
    out[1] = s1;
    out[2] = s2;
    out[3] = s3;
    return 0;
}

/* dt = CFL / ((N+1) max_a sum_r (|u_r| + c)/h_r). */
double oracle_cfl_dt(void *mp, const double *q, double cfl)
{
    omesh *m = (omesh *)mp;
    const int Np = m->Np;
    double smax = 0.0;
    for (int64_t e = 0; e < m->ne; ++e)
        for (int a = 0; a < Np; ++a) {
            double qa[5];
            load_node(q, e, Np, a, qa);
            double p = pressure(qa, m->phi[e * Np + a], m->gamma);
            double c = sqrt(m->gamma * p / qa[0]);
            double s = 0.0;
            if (m->Ja) {
                /* (|u . J a^r| + c |J a^r|) / (2 J): the affine (|u_r| + c) / h_r */
                const double *Ja = m->Ja + e * 9 * Np;
                for (int r = 0; r < 3; ++r) {
                    double un = 0.0, n2 = 0.0;
                    for (int d = 0; d < 3; ++d) {
                        double jv = Ja[(r * 3 + d) * Np + a];
                        un += qa[1 + d] / qa[0] * jv;
                        n2 += jv * jv;
                    }
                    s += (fabs(un) + c * sqrt(n2)) / (2.0 * m->Jd[e * Np + a]);
                }
            } else {
                for (int r = 0; r < 3; ++r) s += (fabs(qa[1 + r] / qa[0]) + c) / m->h[r];
            }
            if (s > smax) smax = s;
        }
    return cfl / ((m->N + 1) * smax);
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the parallel loops that follow (the CPU baseline times the
 * oracle on all host cores and on one). */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
