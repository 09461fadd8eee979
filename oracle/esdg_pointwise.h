/*
 * esdg_pointwise.h -- TEST INFRASTRUCTURE (part of the oracle): its
 * pointwise physics, written over the scalar type `real`.
 *
 * The oracle (esdg_oracle.c) includes this file with `typedef double real;`
 * and these functions are plain FP64 C.  The operation counter
 * (opcount.cpp) includes the same file with `real` an instrumented type
 * that counts every +, -, *, /, sqrt and log, so that the counts are those
 * of the arithmetic the oracle itself executes.  Nothing here is shared
 * with the HIP library.
 */
#ifndef ORACLE_FN
#define ORACLE_FN /* exported by the oracle library */
#endif

/* Pressure from the conservative state, with E containing rho*phi:
 * P = (gamma-1) (E - |U|^2/(2 rho) - rho phi)   (Sec. 2). */
static real pressure(const real q[5], real phi, real gamma)
{
    real ke = 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0];
    return (gamma - 1.0) * (q[4] - ke - q[0] * phi);
}

/* Logarithmic mean {{a}}_log = [[a]] / [[ln a]] (Sec. 4.1), with the
 * near-equal branch by the Taylor series of 2 atanh(f)/f in u = f^2,
 * f = (b-a)/(b+a). */
ORACLE_FN real oracle_logmean(real a, real b)
{
    real f = (b - a) / (b + a);
    real u = f * f;
    if (u < 1e-4)
        return (a + b) / (2.0 + u * (2.0 / 3.0 + u * (2.0 / 5.0 + u * (2.0 / 7.0))));
    return (b - a) / (log(b) - log(a));
}

/* Per-node quantities of the two-point flux: the velocity u = m/rho, the
 * pressure p, z = rho/p (the argument of the second log-mean) and
 * b = rho/(2 p). */
static void node_quantities(const real q[5], real phi, real gamma, real u[3], real *p, real *z,
                            real *b)
{
    real rho = q[0];
    for (int c = 0; c < 3; ++c) u[c] = q[1 + c] / rho;
    *p = pressure(q, phi, gamma);
    *z = rho / *p;
    *b = rho / (2.0 * *p);
}

/* Gravity part of the normal momentum flux of own node a (Sec. 4.1):
 * rho_hat [[phi]]/2 with rho_hat = {{b}} {{rho}}_log / b_a. */
static real gravity_term(real rho_ln, real ba, real bb, real phia, real phib)
{
    real rho_hat = 0.5 * (ba + bb) * rho_ln / ba;
    return 0.5 * rho_hat * (phib - phia);
}

/* Two-point volume flux F_r(a, b) for own node a and partner b.
 * Mass and momentum follow the paper's momentum flux
 *   f^m_c = f^rho {{u_c}} + delta_cr (p* + rho_hat [[phi]] / 2),
 *   rho_hat = {{b}} {{rho}}_log / b_a,  b = rho / (2 p)   (Sec. 4.1)
 * with f^rho = {{rho}}_log {{u_r}} and p* = {{p}}; the energy flux is the
 * Ranocha-type form plus {{phi}} f^rho (E contains rho*phi).  The result is
 * not symmetric in (a, b) because of the gravity term. */
ORACLE_FN void oracle_two_point_flux(int r, const real qa[5], const real qb[5], real phia,
                                     real phib, real gamma, real F[5])
{
    real ua[3], ub[3], pa, pb, za, zb, ba, bb;
    node_quantities(qa, phia, gamma, ua, &pa, &za, &ba);
    node_quantities(qb, phib, gamma, ub, &pb, &zb, &bb);
    real rho_ln = oracle_logmean(qa[0], qb[0]);
    real z_ln = oracle_logmean(za, zb); /* {{rho/p}}_log */
    real frho = rho_ln * 0.5 * (ua[r] + ub[r]);
    real grav_term = gravity_term(rho_ln, ba, bb, phia, phib);
    real pmean = 0.5 * (pa + pb);
    F[0] = frho;
    for (int c = 0; c < 3; ++c)
        F[1 + c] = frho * 0.5 * (ua[c] + ub[c]) + (c == r ? pmean + grav_term : 0.0);
    real uaub = ua[0] * ub[0] + ua[1] * ub[1] + ua[2] * ub[2];
    F[4] = frho * (1.0 / ((gamma - 1.0) * z_ln) + 0.5 * uaub + 0.5 * (phia + phib)) +
           0.5 * (pa * ub[r] + pb * ua[r]);
}

/* Entropy-stable matrix dissipation D for a face normal along axis r (the
 * Roe-type dissipation the paper adds to the entropy-conservative face flux,
 * Sec. 3; the formula is cited there, not printed, and is read here as the
 * standard construction).  With the averaged state
 *   rho_hat = {{rho}}_log,  u_hat = {{u}},  p_hat = {{rho}} / (2 {{b}}),
 *   |u|^2_bar = 2 |u_hat|^2 - {{|u|^2}},
 *   h_hat = gamma / (2 (gamma - 1) {{b}}_log) + |u|^2_bar / 2,
 *   a_hat = sqrt(gamma p_hat / rho_hat),
 * R holds the right eigenvectors of the normal flux Jacobian (acoustic,
 * entropy, two shear, acoustic), |lambda| the moduli of their eigenvalues
 * u_n -+ a, u_n, u_n, u_n, and t the diagonal scaling for which
 * R diag(t) R^T = dq/dv at equal states:
 *   D = R diag(|lambda| t) R^T [[v]],   [[v]] = v(q+) - v(q-).
 * D is symmetric positive semi-definite in [[v]], so it only removes
 * entropy, and it does not depend on the sign of the normal.  Both sides of
 * a face share phi and E contains rho*phi: D is formed for the state without
 * the potential energy, (rho, m, E - rho phi), whose entropy variables lack
 * the 2 b phi term, and the energy component then gains phi times the mass
 * component (that map is linear with unit diagonal, so this is the same
 * operator written for the total energy).
 * Pins: the small-jump limit |A| [[q]], entropy stability, antisymmetry and
 * an exactly kept stationary contact (which fixes the log-mean in h_hat).
 * The averages chosen for p_hat, |u|^2_bar and a_hat enter only at second
 * order in the jump: beyond that they are a reading, parity unpinned. */
static void matrix_dissipation(int r, const real qm[5], const real qp[5], real phi,
                               real gamma, real D[5])
{
    real gm1 = gamma - 1.0;
    real rm = qm[0], rp = qp[0], um[3], up[3];
    for (int c = 0; c < 3; ++c) {
        um[c] = qm[1 + c] / rm;
        up[c] = qp[1 + c] / rp;
    }
    real pm = pressure(qm, phi, gamma), pp = pressure(qp, phi, gamma);
    real bm = rm / (2.0 * pm), bp = rp / (2.0 * pp);
    real uum = um[0] * um[0] + um[1] * um[1] + um[2] * um[2];
    real uup = up[0] * up[0] + up[1] * up[1] + up[2] * up[2];

    /* averaged state */
    real rho_hat = oracle_logmean(rm, rp);
    real b_ln = oracle_logmean(bm, bp);
    real uh[3];
    for (int c = 0; c < 3; ++c) uh[c] = 0.5 * (um[c] + up[c]);
    real p_hat = 0.5 * (rm + rp) / (2.0 * 0.5 * (bm + bp));
    real u2bar = 2.0 * (uh[0] * uh[0] + uh[1] * uh[1] + uh[2] * uh[2]) - 0.5 * (uum + uup);
    real h_hat = gamma / (2.0 * gm1 * b_ln) + 0.5 * u2bar;
    real a_hat = sqrt(gamma * p_hat / rho_hat);

    /* jump of the entropy variables without the potential energy,
     * v = ((gamma - s)/(gamma - 1) - b |u|^2, 2 b u, -2 b), s = ln p - gamma ln rho;
     * a jump of logarithms is taken as the logarithm of the ratio */
    real ds = log(pp / pm) - gamma * log(rp / rm);
    real dv[5];
    dv[0] = -ds / gm1 - (bp * uup - bm * uum);
    for (int c = 0; c < 3; ++c) dv[1 + c] = 2.0 * (bp * up[c] - bm * um[c]);
    dv[4] = -2.0 * (bp - bm);

    /* eigenvectors (columns), normal e_r, tangents the other two axes */
    int t1 = (r + 1) % 3, t2 = (r + 2) % 3;
    real un = uh[r];
    real Rm[5][5];
    memset(Rm, 0, sizeof(Rm));
    Rm[0][0] = 1.0;
    Rm[0][1] = 1.0;
    Rm[0][4] = 1.0;
    for (int c = 0; c < 3; ++c) {
        Rm[1 + c][0] = uh[c] - (c == r ? a_hat : 0.0);
        Rm[1 + c][1] = uh[c];
        Rm[1 + c][4] = uh[c] + (c == r ? a_hat : 0.0);
    }
    Rm[1 + t1][2] = 1.0;
    Rm[1 + t2][3] = 1.0;
    Rm[4][0] = h_hat - a_hat * un;
    Rm[4][1] = 0.5 * u2bar;
    Rm[4][2] = uh[t1];
    Rm[4][3] = uh[t2];
    Rm[4][4] = h_hat + a_hat * un;
    real lam[5] = {fabs(un - a_hat), fabs(un), fabs(un), fabs(un), fabs(un + a_hat)};
    real tsc[5] = {rho_hat / (2.0 * gamma), rho_hat * gm1 / gamma, p_hat, p_hat,
                     rho_hat / (2.0 * gamma)};

    real w[5];
    for (int k = 0; k < 5; ++k) {
        real acc = 0.0;
        for (int v = 0; v < 5; ++v) acc += Rm[v][k] * dv[v];
        w[k] = lam[k] * tsc[k] * acc;
    }
    for (int v = 0; v < 5; ++v) {
        real acc = 0.0;
        for (int k = 0; k < 5; ++k) acc += Rm[v][k] * w[k];
        D[v] = acc;
    }
    D[4] += phi * D[0];
}

/* Normal face flux F* . n for the face with outward normal n = s e_r (s = +-1):
 * s f_r(q-, q+) - lambda/2 (q+ - q-) with lambda = max(|u.n| + c) (Rusanov),
 * s f_r(q-, q+) - D/2 with the matrix dissipation above, or without
 * dissipation for the entropy-conservative face flux.  Faces have
 * phi+ = phi-. */
ORACLE_FN void oracle_surface_flux(int r, int s, const real qm[5], const real qp[5], real phim,
                         real phip, real gamma, int surf, real Fn[5])
{
    real F[5];
    oracle_two_point_flux(r, qm, qp, phim, phip, gamma, F);
    if (surf == SURF_MATRIX) {
        real D[5];
        matrix_dissipation(r, qm, qp, phim, gamma, D);
        for (int v = 0; v < 5; ++v) Fn[v] = s * F[v] - 0.5 * D[v];
        return;
    }
    real lam = 0.0;
    if (surf == SURF_RUSANOV) {
        real pm = pressure(qm, phim, gamma), pp = pressure(qp, phip, gamma);
        real cm = sqrt(gamma * pm / qm[0]), cp = sqrt(gamma * pp / qp[0]);
        real lm = fabs(qm[1 + r] / qm[0]) + cm;
        real lp = fabs(qp[1 + r] / qp[0]) + cp;
        lam = lm > lp ? lm : lp;
    }
    for (int v = 0; v < 5; ++v) Fn[v] = s * F[v] - 0.5 * lam * (qp[v] - qm[v]);
}

/* f-plane Coriolis source -Omega x U, Omega = f z_hat (Sec. 2), added to the
 * momentum components of acc. */
static void coriolis_source(real f, const real q[5], real acc[5])
{
    acc[1] += f * q[2];
    acc[2] -= f * q[1];
}

/* One value of the 2N-storage LSRK stage update (Sec. 3):
 * dq <- A dq + dt R;  q <- q + B dq. */
static void lsrk_update(real A, real B, real dt, real R, real *dq, real *q)
{
    *dq = A * *dq + dt * R;
    *q = *q + B * *dq;
}
