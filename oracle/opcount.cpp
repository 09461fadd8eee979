/*
 * opcount.cpp -- TEST INFRASTRUCTURE (part of the oracle): operation counts
 * of the oracle's pointwise physics.
 *
 * esdg_pointwise.h is compiled here with `real` an instrumented scalar that
 * carries a double and counts every binary +, -, *, / and every sqrt and log
 * it evaluates (fabs, comparisons and negation are not arithmetic and are
 * not counted).  Calling a function of the header on given inputs therefore
 * yields the exact operation count of that call in the oracle, branch by
 * branch, with the values it computes (checked against the FP64 oracle by
 * the tests).  These counts are the algorithmic work of the roofline model.
 */
#include <cmath>
#include <cstdint>
#include <cstring>

namespace opc {

struct Counts {
    long long add, mul, div, sqrt, log;
};
static Counts g_counts;

struct real {
    double v;
    real() = default;
    real(double x) : v(x) {}
};

inline real operator+(real a, real b) { ++g_counts.add; return real(a.v + b.v); }
inline real operator-(real a, real b) { ++g_counts.add; return real(a.v - b.v); }
inline real operator*(real a, real b) { ++g_counts.mul; return real(a.v * b.v); }
inline real operator/(real a, real b) { ++g_counts.div; return real(a.v / b.v); }
inline real operator-(real a) { return real(-a.v); }
inline real &operator+=(real &a, real b) { a = a + b; return a; }
inline real &operator-=(real &a, real b) { a = a - b; return a; }
inline real &operator*=(real &a, real b) { a = a * b; return a; }
inline real &operator/=(real &a, real b) { a = a / b; return a; }
inline bool operator<(real a, real b) { return a.v < b.v; }
inline bool operator>(real a, real b) { return a.v > b.v; }
inline bool operator<=(real a, real b) { return a.v <= b.v; }
inline bool operator>=(real a, real b) { return a.v >= b.v; }
inline bool operator==(real a, real b) { return a.v == b.v; }
inline bool operator!=(real a, real b) { return a.v != b.v; }
inline real log(real a) { ++g_counts.log; return real(std::log(a.v)); }
inline real sqrt(real a) { ++g_counts.sqrt; return real(std::sqrt(a.v)); }
inline real fabs(real a) { return real(std::fabs(a.v)); }

#define SURF_RUSANOV 0
#define SURF_EC 1
#define SURF_MATRIX 2
#define ORACLE_FN static
#include "esdg_pointwise.h"

}  // namespace opc

namespace {

enum {
    OP_NODE = 0,      // node_quantities(qa, phia)
    OP_FLUX = 1,      // oracle_two_point_flux(r, qa, qb, phia, phib)
    OP_GRAVITY = 2,   // gravity_term of own node a in that flux
    OP_SURFACE = 3,   // oracle_surface_flux(r, +1, qa, qb, phia, phia, surf)
    OP_SOURCE = 4,    // coriolis_source(f = phia, qa)
    OP_UPDATE = 5,    // lsrk_update of one value (A = qa[0], B = qa[1], dt = qa[2], R = qa[3])
    OP_LOGMEAN = 6    // oracle_logmean(qa[0], qb[0])
};

void load(opc::real *dst, const double *src, int n)
{
    for (int i = 0; i < n; ++i) dst[i] = opc::real(src[i]);
}

}  // namespace

extern "C" {

/* Counts of one call: out[0..4] = additions/subtractions, multiplications,
 * divisions, square roots, logarithms; res (may be NULL) receives up to five
 * values the call computed.  Returns 0, or -1 for an unknown `what`. */
int oracle_op_count(int what, int r, const double *qa, const double *qb, double phia,
                    double phib, double gamma, int surf, long long *out, double *res)
{
    using opc::real;
    opc::g_counts = opc::Counts{0, 0, 0, 0, 0};
    real a[5], b[5], F[5];
    load(a, qa, 5);
    load(b, qb, 5);
    const real g(gamma), pa(phia), pb(phib);
    double vals[5] = {0, 0, 0, 0, 0};
    switch (what) {
    case OP_NODE: {
        real u[3], p, z, bb;
        opc::node_quantities(a, pa, g, u, &p, &z, &bb);
        vals[0] = u[0].v; vals[1] = u[1].v; vals[2] = u[2].v; vals[3] = p.v; vals[4] = bb.v;
        break;
    }
    case OP_FLUX:
        opc::oracle_two_point_flux(r, a, b, pa, pb, g, F);
        for (int v = 0; v < 5; ++v) vals[v] = F[v].v;
        break;
    case OP_GRAVITY: {
        // the inputs of the gravity term as the flux forms them
        real ua[3], ub[3], p1, p2, z1, z2, b1, b2;
        opc::node_quantities(a, pa, g, ua, &p1, &z1, &b1);
        opc::node_quantities(b, pb, g, ub, &p2, &z2, &b2);
        const real rho_ln = opc::oracle_logmean(a[0], b[0]);
        opc::g_counts = opc::Counts{0, 0, 0, 0, 0};
        vals[0] = opc::gravity_term(rho_ln, b1, b2, pa, pb).v;
        break;
    }
    case OP_SURFACE:
        opc::oracle_surface_flux(r, 1, a, b, pa, pa, g, surf, F);
        for (int v = 0; v < 5; ++v) vals[v] = F[v].v;
        break;
    case OP_SOURCE: {
        real acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        opc::coriolis_source(pa, a, acc);
        for (int v = 0; v < 5; ++v) vals[v] = acc[v].v;
        break;
    }
    case OP_UPDATE: {
        real dq = b[0], q = b[1];
        opc::lsrk_update(a[0], a[1], a[2], a[3], &dq, &q);
        vals[0] = dq.v;
        vals[1] = q.v;
        break;
    }
    case OP_LOGMEAN:
        vals[0] = opc::oracle_logmean(a[0], b[0]).v;
        break;
    default:
        return -1;
    }
    out[0] = opc::g_counts.add;
    out[1] = opc::g_counts.mul;
    out[2] = opc::g_counts.div;
    out[3] = opc::g_counts.sqrt;
    out[4] = opc::g_counts.log;
    if (res)
        for (int v = 0; v < 5; ++v) res[v] = vals[v];
    return 0;
}

}  // extern "C"
