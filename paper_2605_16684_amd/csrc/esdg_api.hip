// esdg_api.hip -- C ABI of the gfx950 ES-DGSEM library (see include/esdg.h).
//
// Host side: argument validation, per-device LGL tables, the mesh object
// (tables, scratch, captured graphs) and kernel launches.  All arithmetic of
// the method runs in the kernels of esdg_device.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "esdg.h"
#include "esdg_device.hpp"
#include "esdg_mixed.hpp"
#include "esdg_curved.hpp"
#include "esdg_high.hpp"

using namespace esdg;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t _e = (expr);                                                              \
        if (_e != hipSuccess)                                                                \
            return fail(ESDG_EHIP, "%s failed: %s", #expr, hipGetErrorString(_e));           \
    } while (0)

// ---------------------------------------------------------------------------
// LGL tables (host).  Interior nodes are the roots of the Jacobi polynomial
// P^(1,1)_{N-1} (proportional to P_N'), found by Newton's method on its
// three-term recurrence in extended precision; weights 2/(N(N+1) P_N^2);
// the derivative matrix from barycentric weights with the negative-sum
// diagonal.
// ---------------------------------------------------------------------------

void jacobi11(int n, long double x, long double *p, long double *dp)
{
    long double pm2 = 1.0L, dpm2 = 0.0L;
    if (n == 0) { *p = 1.0L; *dp = 0.0L; return; }
    long double pm1 = 2.0L * x, dpm1 = 2.0L;
    for (int k = 2; k <= n; ++k) {
        const long double a = 4.0L * k * k * (k + 2.0L);
        const long double b = (2.0L * k + 1.0L) * (2.0L * k + 2.0L) * (2.0L * k);
        const long double c = 2.0L * k * k * (2.0L * k + 2.0L);
        const long double pk = (b * x * pm1 - c * pm2) / a;
        const long double dpk = (b * (x * dpm1 + pm1) - c * dpm2) / a;
        pm2 = pm1; dpm2 = dpm1;
        pm1 = pk; dpm1 = dpk;
    }
    *p = pm1;
    *dp = dpm1;
}

long double legendre(int n, long double x)
{
    long double a = 1.0L, b = x;
    if (n == 0) return 1.0L;
    for (int k = 2; k <= n; ++k) {
        const long double c = ((2.0L * k - 1.0L) * x * b - (k - 1.0L) * a) / k;
        a = b;
        b = c;
    }
    return b;
}

void lgl_tables(int N, double *xi_out, double *w_out, double *D_out)
{
    const int Nq = N + 1;
    long double x[NQ_MAX];
    x[0] = -1.0L;
    x[N] = 1.0L;
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 1; i < N; ++i) {
        long double t = -std::cos(pi * (long double)i / (long double)N);
        for (int it = 0; it < 200; ++it) {
            long double p, dp;
            jacobi11(N - 1, t, &p, &dp);
            const long double step = p / dp;
            t -= step;
            if (std::fabs(step) <= 1e-21L) break;
        }
        x[i] = t;
    }
    for (int i = 0; i < Nq / 2; ++i) {  // exact mirror symmetry
        const long double s = 0.5L * (x[N - i] - x[i]);
        x[i] = -s;
        x[N - i] = s;
    }
    if (N % 2 == 0) x[N / 2] = 0.0L;
    long double lam[NQ_MAX];
    for (int j = 0; j < Nq; ++j) {
        long double prod = 1.0L;
        for (int k = 0; k < Nq; ++k)
            if (k != j) prod *= (x[j] - x[k]);
        lam[j] = 1.0L / prod;
    }
    for (int i = 0; i < Nq; ++i) {
        const long double pn = legendre(N, x[i]);
        xi_out[i] = (double)x[i];
        w_out[i] = (double)(2.0L / ((long double)N * (N + 1.0L) * pn * pn));
        long double diag = 0.0L;
        for (int j = 0; j < Nq; ++j) {
            if (j == i) continue;
            const long double d = (lam[j] / lam[i]) / (x[i] - x[j]);
            D_out[i * Nq + j] = (double)d;
            diag -= d;
        }
        D_out[i * Nq + i] = (double)diag;
    }
}

OrderTables make_order_tables(int N)
{
    OrderTables t;
    std::memset(&t, 0, sizeof t);
    const int Nq = N + 1;
    double D[NQ_MAX * NQ_MAX];
    lgl_tables(N, t.xi, t.w, D);
    for (int i = 0; i < Nq; ++i) t.winv[i] = 1.0 / t.w[i];
    for (int a = 0; a < Nq; ++a)
        for (int b = 0; b < Nq; ++b)
            t.T[a][b] = (a == b) ? 0.0 : D[a * Nq + b] - (t.w[b] / t.w[a]) * D[b * Nq + a];
    for (int a = 0; a < Nq; ++a) {
        t.winvf[a] = (float)t.winv[a];
        for (int b = 0; b < Nq; ++b) t.Tf[a][b] = (float)t.T[a][b];
    }
    return t;
}

std::mutex g_init_mu;
bool g_dev_init[64];
double *g_scratch[64];  // device address of `scratch` on each device (set at init)

}  // namespace

// Device memory of the allocation-free step (esdg_lsrk_step_noalloc): the
// ping-pong state of its five stages.  One array per device, held until the
// process ends; host code reaches it only through g_scratch[device].
constexpr int64_t kNoallocMaxDoubles = (int64_t)1 << 23;  // 64 MiB
static __device__ __align__(256) double scratch[kNoallocMaxDoubles];

namespace {

int ensure_tables(int dev)
{
    std::lock_guard<std::mutex> lk(g_init_mu);
    if (dev < 0 || dev >= 64) return fail(ESDG_EINVAL, "device id %d out of range", dev);
    if (g_dev_init[dev]) return ESDG_OK;
    OrderTables tabs[NQ_MAX];
    for (int N = 1; N <= NQ_MAX - 1; ++N) tabs[N - 1] = make_order_tables(N);
    std::memset(&tabs[NQ_MAX - 1], 0, sizeof(OrderTables));
    HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(c_tab), tabs, sizeof tabs, 0, hipMemcpyHostToDevice));
    void *sp = nullptr;
    HIP_TRY(hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)));
    g_scratch[dev] = (double *)sp;
    g_dev_init[dev] = true;
    return ESDG_OK;
}

bool aligned8(const void *p) { return ((uintptr_t)p & 7u) == 0; }

// Two arrays of n doubles overlap.
bool overlaps(const double *a, const double *b, int64_t n)
{
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b, len = (uintptr_t)n * sizeof(double);
    return x < y + len && y < x + len;
}

}  // namespace

// ---------------------------------------------------------------------------
// Mesh object
// ---------------------------------------------------------------------------

struct esdg_mesh {
    esdg_mesh_desc desc;
    int device;
    hipStream_t stream;
    int N, Nq, Np;
    int64_t ne, nn, state_len;
    int epw;
    double h[3];
    double *d_q2;        // ping-pong state
    double *d_prim;      // N > 8 without the LDS kernel: per-node partner quantities [e][9][n]
    bool high_lds;       // N > 8: one workgroup per element, primitives in LDS
    double *d_r;         // RHS scratch (entropy production)
    double *d_partials;  // reduction partials
    double *d_red_out;   // 4 doubles
    int *d_flag;
    double *h_out;       // pinned, 4 doubles
    int *h_flag;         // pinned
    float *d_ref_r;      // FP32_MIXED: reference density (FP32 values)
    float *d_ref_p;      // FP32_MIXED: reference pressure
    float *d_rr_mom;     // FP32_MIXED: momentum components of R(q_r)
    bool curved;         // curved hexahedra: per-node metric terms below
    double *d_Ja;        // [e][r][d][n] J a^r_d
    double *d_iJ;        // [e][n] 1/J
    double *d_J;         // [e][n] J
    double *d_phi;       // [e][n] geopotential
    double *d_xyz;       // [e][3][n] node coordinates
    int64_t red_blocks;
    int64_t footprint;
    // captured two-step graph for esdg_lsrk_run
    hipGraphExec_t graph_exec;
    const double *g_q;
    const double *g_dq;
    double g_dt;
    hipStream_t g_stream;
    int g_epw;
};

namespace {

// Compiled (N, EPW) variants of the fused stage kernel.
typedef void (*stage_kernel_t)(StageParams);

typedef void (*packed_kernel_t)(PackLaunch);

struct Variant {
    int N, epw, threads;
    stage_kernel_t rhs, stage;
    packed_kernel_t packed;
};

#define V(NN, E)                                                                             \
    {NN, E, block_threads<NN + 1, E>(), stage_fp64<NN + 1, E, MODE_RHS>,                    \
     stage_fp64<NN + 1, E, MODE_STAGE>, stage_fp64_packed<NN + 1, E, MODE_STAGE>}
const Variant kVariants[] = {
    V(1, 8), V(1, 16), V(1, 32),
    V(2, 4), V(2, 7), V(2, 14),
    V(3, 2), V(3, 4), V(3, 8),
    V(4, 1), V(4, 2), V(4, 5),
    V(5, 1), V(5, 3),
    V(6, 1), V(6, 2),
    V(7, 1), V(7, 2),
    V(8, 1),
};
#undef V

typedef void (*mixed_kernel_t)(MixedParams);
typedef void (*mixed_packed_kernel_t)(PackLaunchMixed);

struct MixedVariant {
    int N, epw, threads;
    mixed_kernel_t rhs, stage;
    mixed_packed_kernel_t packed;
};

#define VM(NN, E)                                                                            \
    {NN, E, block_threads<NN + 1, E>(), stage_mixed<NN + 1, E, MODE_RHS>,                   \
     stage_mixed<NN + 1, E, MODE_STAGE>, stage_mixed_packed<NN + 1, E, MODE_STAGE>}
const MixedVariant kMixedVariants[] = {
    VM(1, 16), VM(2, 7), VM(3, 4), VM(3, 8), VM(4, 2), VM(4, 5),
    VM(5, 3), VM(6, 2), VM(7, 1), VM(7, 2), VM(8, 1),
};
#undef VM

typedef void (*curved_kernel_t)(CurvedParams);

struct CurvedVariant {
    int N, epw, threads;
    curved_kernel_t rhs, stage;
};

#define VC(NN, E)                                                                            \
    {NN, E, block_threads<NN + 1, E>(), stage_curved<NN + 1, E, MODE_RHS>,                  \
     stage_curved<NN + 1, E, MODE_STAGE>}
const CurvedVariant kCurvedVariants[] = {
    VC(1, 16), VC(2, 7), VC(3, 4), VC(4, 5), VC(5, 3), VC(6, 1), VC(7, 1), VC(8, 1),
};
#undef VC

const CurvedVariant *find_curved_variant(int N, int epw)
{
    for (const CurvedVariant &v : kCurvedVariants)
        if (v.N == N && v.epw == epw) return &v;
    return nullptr;
}

const Variant *find_variant(int N, int epw)
{
    for (const Variant &v : kVariants)
        if (v.N == N && v.epw == epw) return &v;
    return nullptr;
}

const MixedVariant *find_mixed_variant(int N, int epw)
{
    for (const MixedVariant &v : kMixedVariants)
        if (v.N == N && v.epw == epw) return &v;
    return nullptr;
}

bool has_variant(int precision, int N, int epw)
{
    return precision == ESDG_FP32_MIXED ? find_mixed_variant(N, epw) != nullptr
                                        : find_variant(N, epw) != nullptr;
}

int default_epw(int N)
{
    switch (N) {
    case 1: return 16;
    case 2: return 7;
    case 3: return 4;
    case 4: return 5;
    case 5: return 3;
    case 6: return 1;
    case 7: return 1;
    default: return 1;
    }
}

// The default of one precision: the measured FP64 choice where that
// precision compiles it, else its first compiled variant for N.
int default_epw(int N, int precision)
{
    const int e = default_epw(N);
    if (has_variant(precision, N, e)) return e;
    if (precision == ESDG_FP32_MIXED) {
        for (const MixedVariant &v : kMixedVariants)
            if (v.N == N) return v.epw;
    } else {
        for (const Variant &v : kVariants)
            if (v.N == N) return v.epw;
    }
    return e;
}

GeomParams geom(const esdg_mesh *m)
{
    GeomParams G;
    G.ne = m->ne;
    G.N = m->N;
    for (int d = 0; d < 3; ++d) {
        G.K[d] = m->desc.K[d];
        G.lo[d] = m->desc.lo[d];
        G.hi[d] = m->desc.hi[d];
        G.h[d] = m->h[d];
    }
    G.gamma = m->desc.gamma;
    G.grav = m->desc.grav;
    G.lnz_scale = m->desc.gas_R * 300.0;
    G.Jn = m->curved ? m->d_J : nullptr;
    G.Ja = m->curved ? m->d_Ja : nullptr;
    G.phi = m->curved ? m->d_phi : nullptr;
    return G;
}

// Traversal bricks (elements): y and z neighbours of an element are visited
// within about one brick of it.  Bricks of 32 x 4 x 4 elements up to N = 4
// and 8 x 4 x 4 above (larger elements, fewer of them in flight per XCD)
// measured best on the bubble and channel workloads.
void traversal_tiles(const esdg_mesh *m, int tile[3])
{
    tile[0] = std::min(m->desc.K[0], m->N <= 4 ? 32 : 8);
    tile[1] = std::min(m->desc.K[1], 4);
    tile[2] = std::min(m->desc.K[2], 4);
}

StageParams base_params(const esdg_mesh *m)
{
    StageParams P;
    std::memset(&P, 0, sizeof P);
    P.ne = m->ne;
    for (int d = 0; d < 3; ++d) {
        P.K[d] = m->desc.K[d];
        P.periodic[d] = m->desc.periodic[d] ? 1 : 0;
        P.two_h[d] = 2.0 / m->h[d];
    }
    P.zlo = m->desc.lo[2];
    P.zhi = m->desc.hi[2];
    P.gamma = m->desc.gamma;
    P.gm1i = 1.0 / (m->desc.gamma - 1.0);
    P.grav = m->desc.grav;
    P.cor_f = m->desc.coriolis_f;
    P.lnz_scale = m->desc.gas_R * 300.0;
    P.surf = m->desc.surface_flux;
    P.flag = m->d_flag;
    P.mask = TERM_VOL | TERM_FACE | TERM_SRC;
    traversal_tiles(m, P.tile);
    return P;
}

int launch_stage_fp64(esdg_mesh *m, StageParams P, int epw)
{
    const Variant *v = find_variant(m->N, epw);
    if (!v) return fail(ESDG_EINVAL, "no FP64 kernel variant for N=%d epw=%d", m->N, epw);
    const int64_t nb = (m->ne + epw - 1) / epw;
    if (nb > 0x7fffffff) return fail(ESDG_EINVAL, "mesh too large");
    P.nblocks = (int)nb;
    hipLaunchKernelGGL(P.mode == MODE_RHS ? v->rhs : v->stage, dim3((unsigned)nb),
                       dim3(v->threads), 0, m->stream, P);
    HIP_TRY(hipGetLastError());
    return ESDG_OK;
}

int launch_stage_curved(esdg_mesh *m, StageParams P)
{
    const CurvedVariant *v = find_curved_variant(m->N, m->epw);
    if (!v) return fail(ESDG_EINVAL, "no curved kernel variant for N=%d epw=%d", m->N, m->epw);
    const int64_t nb = (m->ne + m->epw - 1) / m->epw;
    if (nb > 0x7fffffff) return fail(ESDG_EINVAL, "mesh too large");
    P.nblocks = (int)nb;
    CurvedParams C;
    C.s = P;
    C.Ja = m->d_Ja;
    C.iJ = m->d_iJ;
    C.phi = m->d_phi;
    hipLaunchKernelGGL(P.mode == MODE_RHS ? v->rhs : v->stage, dim3((unsigned)nb),
                       dim3(v->threads), 0, m->stream, C);
    HIP_TRY(hipGetLastError());
    return ESDG_OK;
}

// Launch shape of stage_high_lds: waves per SIMD it is compiled for, and the
// workgroup size below and from N = 10 on, where one element's LDS leaves
// room for two workgroups per CU (N = 9) or one.
constexpr int HIGH_LDS_WAVES = 1;
constexpr int HIGH_LDS_T_SMALL = 256, HIGH_LDS_T_LARGE = 512;
constexpr int high_lds_threads(int N)
{
    return N <= 9 ? HIGH_LDS_T_SMALL : HIGH_LDS_T_LARGE;
}

template <int MODE, int T>
void *high_lds_fn()
{
    return reinterpret_cast<void *>(&stage_high_lds<MODE, T, HIGH_LDS_WAVES>);
}

// Whether stage_high_lds can hold an element of order N on device dev: the
// element's primitives must fit the workgroup's LDS, and the kernels accept
// that much dynamic LDS.
bool high_lds_fits(int dev, int N)
{
    int lim = 0;
    if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return false;
    const size_t need = high_lds_bytes(N);
    if (need > (size_t)lim) return false;
    void *fns[] = {high_lds_fn<MODE_RHS, HIGH_LDS_T_SMALL>(),
                   high_lds_fn<MODE_STAGE, HIGH_LDS_T_SMALL>(),
                   high_lds_fn<MODE_RHS, HIGH_LDS_T_LARGE>(),
                   high_lds_fn<MODE_STAGE, HIGH_LDS_T_LARGE>()};
    for (void *f : fns)
        if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)need) !=
            hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
    return true;
}

// Orders above N_FUSED_MAX: one workgroup per element with the primitives in
// LDS, or, where an element does not fit, the primitives of the stage input
// into the prim buffer and then the node-per-thread kernel.
int launch_stage_high(esdg_mesh *m, StageParams P)
{
    if (m->high_lds) {
        if (m->ne > 0x7fffffff) return fail(ESDG_EINVAL, "mesh too large");
        P.nblocks = (int)m->ne;
        const size_t lds = high_lds_bytes(m->N);
        const int T = high_lds_threads(m->N);
        constexpr int TS = HIGH_LDS_T_SMALL, TL = HIGH_LDS_T_LARGE, W = HIGH_LDS_WAVES;
        void (*k)(StageParams, int);
        if (T == TS) k = P.mode == MODE_RHS ? stage_high_lds<MODE_RHS, TS, W>
                                            : stage_high_lds<MODE_STAGE, TS, W>;
        else k = P.mode == MODE_RHS ? stage_high_lds<MODE_RHS, TL, W>
                                    : stage_high_lds<MODE_STAGE, TL, W>;
        hipLaunchKernelGGL(k, dim3((unsigned)m->ne), dim3(T), lds, m->stream, P, m->N);
        HIP_TRY(hipGetLastError());
        return ESDG_OK;
    }
    const int64_t nb = (m->nn + HIGH_THREADS - 1) / HIGH_THREADS;
    if (nb > 0x7fffffff) return fail(ESDG_EINVAL, "mesh too large");
    hipLaunchKernelGGL(prim_kernel, dim3((unsigned)nb), dim3(HIGH_THREADS), 0, m->stream, P, m->N,
                       m->d_prim);
    HIP_TRY(hipGetLastError());
    if (P.mode == MODE_RHS)
        hipLaunchKernelGGL(stage_high_kernel<MODE_RHS>, dim3((unsigned)nb), dim3(HIGH_THREADS), 0,
                           m->stream, P, m->N, (const double *)m->d_prim);
    else
        hipLaunchKernelGGL(stage_high_kernel<MODE_STAGE>, dim3((unsigned)nb), dim3(HIGH_THREADS),
                           0, m->stream, P, m->N, (const double *)m->d_prim);
    HIP_TRY(hipGetLastError());
    return ESDG_OK;
}

int launch_stage(esdg_mesh *m, StageParams P)
{
    if (m->N > N_FUSED_MAX) return launch_stage_high(m, P);
    if (m->curved) return launch_stage_curved(m, P);
    if (m->desc.precision != ESDG_FP32_MIXED) return launch_stage_fp64(m, P, m->epw);
    const MixedVariant *v = find_mixed_variant(m->N, m->epw);
    if (!v) return fail(ESDG_EINVAL, "no mixed kernel variant for N=%d epw=%d", m->N, m->epw);
    const int64_t nb = (m->ne + m->epw - 1) / m->epw;
    if (nb > 0x7fffffff) return fail(ESDG_EINVAL, "mesh too large");
    P.nblocks = (int)nb;
    MixedParams M;
    M.s = P;
    M.ref_r = m->d_ref_r;
    M.ref_p = m->d_ref_p;
    M.rr_mom = m->d_rr_mom;
    hipLaunchKernelGGL(P.mode == MODE_RHS ? v->rhs : v->stage, dim3((unsigned)nb),
                       dim3(v->threads), 0, m->stream, M);
    HIP_TRY(hipGetLastError());
    return ESDG_OK;
}

// LSRK(5,4) coefficients of Carpenter and Kennedy (published rationals).
const double kA[5] = {0.0, -567301805773.0 / 1357537059087.0,
                      -2404267990393.0 / 2016746695238.0, -3550918686646.0 / 2091501179385.0,
                      -1275806237668.0 / 842570457699.0};
const double kB[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                      1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                      2277821191437.0 / 14882151754819.0};

// Enqueue the 5 stages of one step: stage s reads a, writes b (ping-pong).
int enqueue_step(esdg_mesh *m, double *q, double *q2, double *dq, double dt, bool start_in_q)
{
    StageParams P = base_params(m);
    P.mode = MODE_STAGE;
    P.dq = dq;
    P.dt = dt;
    double *bufs[2] = {start_in_q ? q : q2, start_in_q ? q2 : q};
    for (int s = 0; s < 5; ++s) {
        P.q_in = bufs[s & 1];
        P.q_out = bufs[(s + 1) & 1];
        P.A = kA[s];
        P.B = kB[s];
        int rc = launch_stage(m, P);
        if (rc) return rc;
    }
    return ESDG_OK;
}

int check_mesh(esdg_mesh_t m)
{
    if (!m) return fail(ESDG_EINVAL, "NULL mesh");
    return ESDG_OK;
}

int check_ptr(const void *p, const char *name)
{
    if (!p) return fail(ESDG_EINVAL, "%s is NULL", name);
    if (!aligned8(p)) return fail(ESDG_EINVAL, "%s is not 8-byte aligned", name);
    return ESDG_OK;
}

int set_device(esdg_mesh *m)
{
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != m->device) HIP_TRY(hipSetDevice(m->device));
    return ESDG_OK;
}

void drop_graph(esdg_mesh *m)
{
    if (m->graph_exec) {
        (void)hipGraphExecDestroy(m->graph_exec);
        m->graph_exec = nullptr;
    }
    m->g_q = m->g_dq = nullptr;
}

// State-sized scratch of the mesh, allocated on first use: the ping-pong
// buffer of esdg_lsrk_step/run and the RHS buffer of esdg_entropy.
int ensure_scratch(esdg_mesh *m, double **buf)
{
    if (*buf) return ESDG_OK;
    const size_t sb = sizeof(double) * (size_t)m->state_len;
    if (hipMalloc(buf, sb) != hipSuccess) {
        *buf = nullptr;
        return fail(ESDG_ENOMEM, "device allocation of %.1f MB failed", sb / 1e6);
    }
    m->footprint += (int64_t)sb;
    return ESDG_OK;
}

void release_scratch(esdg_mesh *m, double **buf)
{
    if (!*buf) return;
    (void)hipFree(*buf);
    *buf = nullptr;
    m->footprint -= (int64_t)(sizeof(double) * (size_t)m->state_len);
}

// sin(2 pi k s), exactly 0 at s = 0 and s = 1 (the box faces).
double sin2pik(int k, double s)
{
    if (s == 0.0 || s == 1.0) return 0.0;
    return std::sin(2.0 * 3.14159265358979323846 * k * s);
}

// Curved set-up (host, once per mesh): node coordinates of the warped box
//   X_d = x_d + warp_d L_d prod_c sin(2 pi k_dc s_c),  s = (x - lo)/L,
//   k_dc = 2 for c = d > 0, else 1,
// which vanishes on the box faces; the metric terms J a^r_d in the
// conservative curl form J a^i_n = -e_i . curl_xi(X_l grad_xi X_m) ((n, m, l)
// cyclic), which satisfies the discrete metric identities; J = det(dX/dxi);
// phi = g z.  Derivatives are the library's LGL derivative matrix applied
// along one reference direction.
int setup_curved(esdg_mesh *m)
{
    const int N = m->N, Nq = m->Nq, Np = m->Np;
    const esdg_mesh_desc &d = m->desc;
    std::vector<double> xi(Nq), wts(Nq), Dm(Nq * Nq);
    lgl_tables(N, xi.data(), wts.data(), Dm.data());
    const size_t nn = (size_t)m->nn;
    std::vector<double> xyz(3 * nn), Ja(9 * nn), iJ(nn), Jd(nn), phi(nn);
    double L[3];
    for (int c = 0; c < 3; ++c) L[c] = d.hi[c] - d.lo[c];
    std::vector<double> X(3 * Np), dX(9 * Np), Y(3 * Np);
    auto deriv = [&](const double *f, int n, int j) {
        int ii[3] = {n % Nq, (n / Nq) % Nq, n / (Nq * Nq)};
        const int row = ii[j];
        double acc = 0.0;
        for (int l = 0; l < Nq; ++l) {
            ii[j] = l;
            acc += Dm[row * Nq + l] * f[ii[0] + Nq * (ii[1] + Nq * ii[2])];
        }
        return acc;
    };
    for (int64_t e = 0; e < m->ne; ++e) {
        const int ec[3] = {(int)(e % d.K[0]), (int)((e / d.K[0]) % d.K[1]),
                           (int)(e / ((int64_t)d.K[0] * d.K[1]))};
        for (int n = 0; n < Np; ++n) {
            const int ii[3] = {n % Nq, (n / Nq) % Nq, n / (Nq * Nq)};
            double xh[3], sv[3];
            for (int c = 0; c < 3; ++c) {
                const double XL = d.lo[c] + (d.hi[c] - d.lo[c]) * ((double)ec[c] / (double)d.K[c]);
                const double XR =
                    d.lo[c] + (d.hi[c] - d.lo[c]) * ((double)(ec[c] + 1) / (double)d.K[c]);
                const double t = xi[ii[c]];
                xh[c] = 0.5 * (1.0 - t) * XL + 0.5 * (1.0 + t) * XR;
                sv[c] = (xh[c] - d.lo[c]) / L[c];
            }
            for (int c = 0; c < 3; ++c) {
                double sn = 1.0;
                for (int b = 0; b < 3; ++b) sn *= sin2pik((b == c && c > 0) ? 2 : 1, sv[b]);
                X[c * Np + n] = xh[c] + d.warp[c] * L[c] * sn;
            }
        }
        for (int c = 0; c < 3; ++c)
            for (int j = 0; j < 3; ++j)
                for (int n = 0; n < Np; ++n) dX[(c * 3 + j) * Np + n] = deriv(&X[c * Np], n, j);
        const size_t eo = (size_t)e * Np;
        for (int n = 0; n < Np; ++n) {
            auto a = [&](int c, int j) { return dX[(c * 3 + j) * Np + n]; };
            const double J = a(0, 0) * (a(1, 1) * a(2, 2) - a(1, 2) * a(2, 1)) -
                             a(0, 1) * (a(1, 0) * a(2, 2) - a(1, 2) * a(2, 0)) +
                             a(0, 2) * (a(1, 0) * a(2, 1) - a(1, 1) * a(2, 0));
            if (!(J > 0.0)) return fail(ESDG_EINVAL, "warp folds element %lld (J <= 0)", (long long)e);
            Jd[eo + n] = J;
            iJ[eo + n] = 1.0 / J;
            for (int c = 0; c < 3; ++c) xyz[((size_t)e * 3 + c) * Np + n] = X[c * Np + n];
            phi[eo + n] = d.grav * X[2 * Np + n];
        }
        for (int nc = 0; nc < 3; ++nc) {
            const int mc = (nc + 1) % 3, lc = (nc + 2) % 3;
            for (int j = 0; j < 3; ++j)
                for (int n = 0; n < Np; ++n) Y[j * Np + n] = X[lc * Np + n] * dX[(mc * 3 + j) * Np + n];
            for (int i = 0; i < 3; ++i) {
                const int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
                for (int n = 0; n < Np; ++n)
                    Ja[(((size_t)e * 3 + i) * 3 + nc) * Np + n] =
                        deriv(&Y[i1 * Np], n, i2) - deriv(&Y[i2 * Np], n, i1);
            }
        }
    }
    struct Buf {
        double **dst;
        const std::vector<double> *src;
    } bufs[] = {{&m->d_Ja, &Ja}, {&m->d_iJ, &iJ}, {&m->d_J, &Jd}, {&m->d_phi, &phi},
                {&m->d_xyz, &xyz}};
    for (const Buf &b : bufs) {
        const size_t bytes = sizeof(double) * b.src->size();
        if (hipMalloc(b.dst, bytes) != hipSuccess)
            return fail(ESDG_ENOMEM, "curved geometry (%.1f MB)", bytes / 1e6);
        m->footprint += (int64_t)bytes;
        HIP_TRY(hipMemcpy(*b.dst, b.src->data(), bytes, hipMemcpyHostToDevice));
    }
    return ESDG_OK;
}

// FP32_MIXED set-up: round the caller's reference to FP32, build the FP64
// reference state q_r (rho_r, 0, 0, 0, p_r/(gamma-1) + rho_r phi) and keep
// the momentum components of R(q_r), evaluated once by the FP64 kernel.
int setup_reference(esdg_mesh *m)
{
    const size_t nn = (size_t)m->nn;
    if (hipMalloc(&m->d_ref_r, sizeof(float) * nn) != hipSuccess ||
        hipMalloc(&m->d_ref_p, sizeof(float) * nn) != hipSuccess ||
        hipMalloc(&m->d_rr_mom, sizeof(float) * 3 * nn) != hipSuccess)
        return fail(ESDG_ENOMEM, "reference buffers (%.1f MB)", 20.0 * nn / 1e6);
    m->footprint += (int64_t)(20 * nn);
    // the FP64 reference state and its RHS are temporaries, allocated and
    // freed in the stream's order: freeing them does not wait for what other
    // streams have in flight on the device (hipFree would)
    const size_t sb = sizeof(double) * (size_t)m->state_len;
    double *tq = nullptr, *tr = nullptr;
    if (hipMallocAsync((void **)&tq, sb, m->stream) != hipSuccess ||
        hipMallocAsync((void **)&tr, sb, m->stream) != hipSuccess) {
        if (tq) (void)hipFreeAsync(tq, m->stream);
        (void)hipGetLastError();
        return fail(ESDG_ENOMEM, "reference temporaries (%.1f MB)", 2.0 * sb / 1e6);
    }
    GeomParams G = geom(m);
    const unsigned blocks = (unsigned)((nn + 255) / 256);
    hipLaunchKernelGGL(reference_state_kernel, dim3(blocks), dim3(256), 0, m->stream, G,
                       m->desc.ref_rho, m->desc.ref_p, m->d_ref_r, m->d_ref_p, tq);
    hipError_t el = hipGetLastError();
    int rc = ESDG_OK;
    if (el == hipSuccess) {
        StageParams P = base_params(m);
        P.mode = MODE_RHS;
        P.q_in = tq;
        P.r_out = tr;
        P.flag = nullptr;
        const int epw = find_variant(m->N, m->epw) ? m->epw : default_epw(m->N);
        rc = launch_stage_fp64(m, P, epw);
        if (!rc) {
            hipLaunchKernelGGL(reference_rhs_kernel, dim3(blocks), dim3(256), 0, m->stream, m->ne,
                               m->Np, (const double *)tr, m->d_rr_mom);
            el = hipGetLastError();
        }
    }
    (void)hipFreeAsync(tq, m->stream);
    (void)hipFreeAsync(tr, m->stream);
    if (rc) return rc;
    if (el != hipSuccess) return fail(ESDG_EHIP, "%s", hipGetErrorString(el));
    // the caller's reference arrays are read by then
    HIP_TRY(hipStreamSynchronize(m->stream));
    return ESDG_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

const char *esdg_last_error(void) { return g_err.c_str(); }

#ifndef ESDG_SOURCE_HASH
#define ESDG_SOURCE_HASH "unknown"
#endif

const char *esdg_version(void) { return "esdg-gfx950 0.2 src:" ESDG_SOURCE_HASH; }

int esdg_lgl_tables(int32_t N, double *xi, double *w, double *D)
{
    if (N < 1 || N > NQ_MAX - 1) return fail(ESDG_EINVAL, "N=%d outside 1..%d", N, NQ_MAX - 1);
    if (!xi || !w || !D) return fail(ESDG_EINVAL, "NULL output");
    lgl_tables(N, xi, w, D);
    return ESDG_OK;
}

int esdg_copy(const double *src, double *dst, int64_t n, void *hip_stream)
{
    if (n < 0) return fail(ESDG_EINVAL, "n < 0");
    if (n == 0) return ESDG_OK;
    int rc;
    if ((rc = check_ptr(src, "src")) || (rc = check_ptr(dst, "dst"))) return rc;
    if (((uintptr_t)src & 15u) || ((uintptr_t)dst & 15u))
        return fail(ESDG_EINVAL, "src/dst must be 16-byte aligned");
    if ((src < dst + n) && (dst < src + n)) return fail(ESDG_EINVAL, "src and dst overlap");
    const int64_t n2 = n / 2;
    hipStream_t s = (hipStream_t)hip_stream;
    if (n2 > 0) {
        const int64_t blocks = std::min<int64_t>((n2 + 255) / 256, 256 * 64);
        hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                           (const double2 *)src, (double2 *)dst, n2);
        HIP_TRY(hipGetLastError());
    }
    if (n & 1) {
        hipLaunchKernelGGL(copy_tail_kernel, dim3(1), dim3(64), 0, s, src, dst, n);
        HIP_TRY(hipGetLastError());
    }
    return ESDG_OK;
}

int esdg_mesh_create(const esdg_mesh_desc *d, void *hip_stream, esdg_mesh_t *out)
{
    if (!d || !out) return fail(ESDG_EINVAL, "NULL argument");
    *out = nullptr;
    if (d->N < 1 || d->N > NQ_MAX - 1)
        return fail(ESDG_EINVAL, "N=%d outside 1..%d", d->N, NQ_MAX - 1);
    const bool high = d->N > N_FUSED_MAX;
    if (high && (d->precision != ESDG_FP64 || d->curved))
        return fail(ESDG_EINVAL, "orders above %d run in FP64 on the affine box only", N_FUSED_MAX);
    if (high && d->epw != 0)
        return fail(ESDG_EINVAL, "orders above %d have no elements-per-workgroup variants",
                    N_FUSED_MAX);
    for (int k = 0; k < 3; ++k) {
        if (d->K[k] < 1) return fail(ESDG_EINVAL, "K[%d]=%d < 1", k, d->K[k]);
        if (!(d->hi[k] > d->lo[k])) return fail(ESDG_EINVAL, "hi[%d] <= lo[%d]", k, k);
    }
    if ((int64_t)d->K[0] * d->K[1] * d->K[2] >= ((int64_t)1 << 31))
        return fail(ESDG_EINVAL, "K[0]*K[1]*K[2] must be below 2^31 elements");
    if (d->periodic[2] && d->grav != 0.0)
        return fail(ESDG_EINVAL, "periodic z with grav != 0 (phi = g z is not periodic)");
    if (!(d->gamma > 1.0) || !(d->gas_R > 0.0))
        return fail(ESDG_EINVAL, "gamma must be > 1 and gas_R > 0");
    if (d->surface_flux != ESDG_SURF_RUSANOV && d->surface_flux != ESDG_SURF_EC &&
        d->surface_flux != ESDG_SURF_MATRIX)
        return fail(ESDG_EINVAL, "unknown surface flux %d", d->surface_flux);
    if (d->precision != ESDG_FP64 && d->precision != ESDG_FP32_MIXED)
        return fail(ESDG_EINVAL, "unknown precision %d", d->precision);
    if (d->curved != 0 && d->curved != 1) return fail(ESDG_EINVAL, "curved must be 0 or 1");
    if (d->curved) {
        if (d->precision != ESDG_FP64)
            return fail(ESDG_EINVAL, "curved meshes run in FP64 only");
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(d->warp[k])) return fail(ESDG_EINVAL, "warp[%d] is not finite", k);
    }
    if (d->precision == ESDG_FP32_MIXED) {
        int rc0;
        if ((rc0 = check_ptr(d->ref_rho, "ref_rho")) || (rc0 = check_ptr(d->ref_p, "ref_p")))
            return rc0;
    }
    const int epw = high ? 0 : (d->epw ? d->epw : default_epw(d->N, d->precision));
    if (!high &&
        (d->curved ? !find_curved_variant(d->N, epw) : !has_variant(d->precision, d->N, epw)))
        return fail(ESDG_EINVAL, "no kernel variant for N=%d epw=%d", d->N, epw);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    int rc = ensure_tables(dev);
    if (rc) return rc;

    esdg_mesh *m = new (std::nothrow) esdg_mesh();
    if (!m) return fail(ESDG_ENOMEM, "host allocation failed");
    std::memset(m, 0, sizeof *m);
    m->desc = *d;
    m->device = dev;
    m->stream = (hipStream_t)hip_stream;
    m->N = d->N;
    m->Nq = d->N + 1;
    m->Np = m->Nq * m->Nq * m->Nq;
    m->ne = (int64_t)d->K[0] * d->K[1] * d->K[2];
    m->nn = m->ne * m->Np;
    m->state_len = m->nn * 5;
    m->epw = epw;
    for (int k = 0; k < 3; ++k) m->h[k] = (d->hi[k] - d->lo[k]) / d->K[k];
    m->red_blocks = (m->nn + RED_THREADS - 1) / RED_THREADS;
    hipError_t e1 = hipSuccess, e2 = hipSuccess;  // state-sized scratch is allocated on first use
    hipError_t e3 = hipMalloc(&m->d_partials, sizeof(double) * 4 * (size_t)m->red_blocks);
    hipError_t e4 = hipMalloc(&m->d_red_out, sizeof(double) * 4);
    hipError_t e5 = hipMalloc(&m->d_flag, sizeof(int));
    hipError_t e6 = hipHostMalloc(&m->h_out, sizeof(double) * 4, hipHostMallocDefault);
    hipError_t e7 = hipHostMalloc(&m->h_flag, sizeof(int), hipHostMallocDefault);
    if (e1 || e2 || e3 || e4 || e5 || e6 || e7) {
        esdg_mesh_destroy(m);
        return fail(ESDG_ENOMEM, "device allocation of the mesh tables failed");
    }
    m->footprint = (int64_t)(sizeof(double) * 4 * m->red_blocks) + 64;
    m->high_lds = high && high_lds_fits(dev, m->N);
    if (high && !m->high_lds) {
        const size_t pb = sizeof(double) * PRIM_VARS * (size_t)m->nn;
        if (hipMalloc(&m->d_prim, pb) != hipSuccess) {
            m->d_prim = nullptr;
            esdg_mesh_destroy(m);
            return fail(ESDG_ENOMEM, "device allocation of %.1f MB failed", pb / 1e6);
        }
        m->footprint += (int64_t)pb;
    }
    hipError_t e8 = hipMemsetAsync(m->d_flag, 0, sizeof(int), m->stream);
    if (e8 != hipSuccess) {
        esdg_mesh_destroy(m);
        return fail(ESDG_EHIP, "hipMemsetAsync: %s", hipGetErrorString(e8));
    }
    m->curved = d->curved != 0;
    if (m->curved) {
        rc = setup_curved(m);
        if (rc) {
            const std::string msg = g_err;
            esdg_mesh_destroy(m);
            return fail(rc, "%s", msg.c_str());
        }
    }
    if (d->precision == ESDG_FP32_MIXED) {
        rc = setup_reference(m);
        if (rc) {
            const std::string msg = g_err;
            esdg_mesh_destroy(m);
            return fail(rc, "%s", msg.c_str());
        }
    }
    *out = m;
    return ESDG_OK;
}

int esdg_mesh_destroy(esdg_mesh_t m)
{
    if (!m) return ESDG_OK;
    int rc = ESDG_OK;
    if (m->stream || m->d_q2) {
        hipError_t e = hipStreamSynchronize(m->stream);
        if (e != hipSuccess) rc = fail(ESDG_EHIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
    }
    drop_graph(m);
    if (m->d_q2) (void)hipFree(m->d_q2);
    if (m->d_prim) (void)hipFree(m->d_prim);
    if (m->d_r) (void)hipFree(m->d_r);
    if (m->d_partials) (void)hipFree(m->d_partials);
    if (m->d_red_out) (void)hipFree(m->d_red_out);
    if (m->d_flag) (void)hipFree(m->d_flag);
    if (m->d_ref_r) (void)hipFree(m->d_ref_r);
    if (m->d_ref_p) (void)hipFree(m->d_ref_p);
    if (m->d_rr_mom) (void)hipFree(m->d_rr_mom);
    for (double *b : {m->d_Ja, m->d_iJ, m->d_J, m->d_phi, m->d_xyz})
        if (b) (void)hipFree(b);
    if (m->h_out) (void)hipHostFree(m->h_out);
    if (m->h_flag) (void)hipHostFree(m->h_flag);
    delete m;
    return rc;
}

int esdg_mesh_info(esdg_mesh_t m, int64_t *n_elem, int64_t *n_nodes, int64_t *state_len,
                   int64_t *footprint_bytes)
{
    int rc = check_mesh(m);
    if (rc) return rc;
    if (n_elem) *n_elem = m->ne;
    if (n_nodes) *n_nodes = m->nn;
    if (state_len) *state_len = m->state_len;
    if (footprint_bytes) *footprint_bytes = m->footprint;
    return ESDG_OK;
}

int esdg_set_stream(esdg_mesh_t m, void *hip_stream)
{
    int rc = check_mesh(m);
    if (rc) return rc;
    m->stream = (hipStream_t)hip_stream;
    return ESDG_OK;
}

int esdg_set_epw(esdg_mesh_t m, int32_t epw)
{
    int rc = check_mesh(m);
    if (rc) return rc;
    if (m->N > N_FUSED_MAX) {
        if (epw != 0)
            return fail(ESDG_EINVAL, "orders above %d have no elements-per-workgroup variants",
                        N_FUSED_MAX);
        return ESDG_OK;
    }
    const int e = epw ? epw : default_epw(m->N, m->desc.precision);
    if (m->curved ? !find_curved_variant(m->N, e) : !has_variant(m->desc.precision, m->N, e))
        return fail(ESDG_EINVAL, "no kernel variant for N=%d epw=%d", m->N, e);
    m->epw = e;
    drop_graph(m);
    return ESDG_OK;
}

int esdg_get_epw(esdg_mesh_t m, int32_t *epw)
{
    int rc = check_mesh(m);
    if (rc) return rc;
    if (!epw) return fail(ESDG_EINVAL, "epw is NULL");
    *epw = m->epw;
    return ESDG_OK;
}

int esdg_node_coords(esdg_mesh_t m, double *xyz)
{
    int rc = check_mesh(m);
    if (rc || (rc = check_ptr(xyz, "xyz")) || (rc = set_device(m))) return rc;
    if (m->curved) {
        HIP_TRY(hipMemcpyAsync(xyz, m->d_xyz, sizeof(double) * 3 * (size_t)m->nn,
                               hipMemcpyDeviceToDevice, m->stream));
        return ESDG_OK;
    }
    GeomParams G = geom(m);
    const int64_t n = m->nn;
    hipLaunchKernelGGL(node_coords_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       m->stream, G, xyz);
    HIP_TRY(hipGetLastError());
    return ESDG_OK;
}

int esdg_rhs_terms(esdg_mesh_t m, const double *q, double *r, int32_t mask)
{
    int rc = check_mesh(m);
    if (rc || (rc = check_ptr(q, "q")) || (rc = check_ptr(r, "r")) || (rc = set_device(m)))
        return rc;
    if (overlaps(q, r, m->state_len)) return fail(ESDG_EINVAL, "q and r must not overlap");
    if (mask & ~ESDG_TERM_ALL) return fail(ESDG_EINVAL, "bad term mask %d", mask);
    StageParams P = base_params(m);
    P.mode = MODE_RHS;
    P.mask = mask;
    P.q_in = q;
    P.r_out = r;
    return launch_stage(m, P);
}

int esdg_rhs(esdg_mesh_t m, const double *q, double *r, double t)
{
    (void)t;
    return esdg_rhs_terms(m, q, r, ESDG_TERM_ALL);
}

int esdg_lsrk_step(esdg_mesh_t m, double *q, double *dq, double t, double dt)
{
    (void)t;
    int rc = check_mesh(m);
    if (rc || (rc = check_ptr(q, "q")) || (rc = check_ptr(dq, "dq")) || (rc = set_device(m)))
        return rc;
    if (overlaps(q, dq, m->state_len)) return fail(ESDG_EINVAL, "q and dq must not overlap");
    if ((rc = ensure_scratch(m, &m->d_q2))) return rc;
    rc = enqueue_step(m, q, m->d_q2, dq, dt, true);
    if (rc) return rc;
    // five stages end in the mesh's second buffer
    HIP_TRY(hipMemcpyAsync(q, m->d_q2, sizeof(double) * (size_t)m->state_len,
                           hipMemcpyDeviceToDevice, m->stream));
    return ESDG_OK;
}

int esdg_lsrk_step_noalloc(esdg_mesh_t m, double *q, double *dq, double t, double dt)
{
    (void)t;
    int rc = check_mesh(m);
    if (rc || (rc = check_ptr(q, "q")) || (rc = check_ptr(dq, "dq"))) return rc;
    if (overlaps(q, dq, m->state_len)) return fail(ESDG_EINVAL, "q and dq must not overlap");
    if (m->state_len > kNoallocMaxDoubles)
        return fail(ESDG_EINVAL,
                    "state of %lld doubles exceeds the %lld-double device scratch of "
                    "esdg_lsrk_step_noalloc",
                    (long long)m->state_len, (long long)kNoallocMaxDoubles);
    if ((rc = set_device(m))) return rc;
    double *s = g_scratch[m->device];
    if (!s) return fail(ESDG_EINVAL, "device scratch of device %d is not set up", m->device);
    rc = enqueue_step(m, q, s, dq, dt, true);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(q, s, sizeof(double) * (size_t)m->state_len, hipMemcpyDeviceToDevice,
                           m->stream));
    return ESDG_OK;
}

int esdg_lsrk_run(esdg_mesh_t m, double *q, double *dq, double t0, double dt, int32_t nsteps)
{
    int rc = check_mesh(m);
    if (rc || (rc = check_ptr(q, "q")) || (rc = check_ptr(dq, "dq")) || (rc = set_device(m)))
        return rc;
    if (overlaps(q, dq, m->state_len)) return fail(ESDG_EINVAL, "q and dq must not overlap");
    if (nsteps < 0) return fail(ESDG_EINVAL, "nsteps < 0");
    if ((rc = ensure_scratch(m, &m->d_q2))) return rc;
    const int pairs = nsteps / 2;
    if (pairs > 0) {
        if (!m->graph_exec || m->g_q != q || m->g_dq != dq || m->g_dt != dt ||
            m->g_stream != m->stream || m->g_epw != m->epw) {
            drop_graph(m);
            // capture two steps (10 stages: q -> q2 -> q -> ... -> q) on a
            // private stream, then replay on the mesh stream
            hipStream_t cs;
            HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            hipStream_t saved = m->stream;
            m->stream = cs;
            hipError_t eb = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            int rc1 = ESDG_OK, rc2 = ESDG_OK;
            if (eb == hipSuccess) {
                rc1 = enqueue_step(m, q, m->d_q2, dq, dt, true);
                if (!rc1) rc2 = enqueue_step(m, q, m->d_q2, dq, dt, false);
            }
            hipGraph_t graph = nullptr;
            hipError_t ee = (eb == hipSuccess) ? hipStreamEndCapture(cs, &graph) : eb;
            m->stream = saved;
            (void)hipStreamDestroy(cs);
            if (eb != hipSuccess) return fail(ESDG_EHIP, "capture: %s", hipGetErrorString(eb));
            if (rc1 || rc2) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc1 ? rc1 : rc2;
            }
            if (ee != hipSuccess) return fail(ESDG_EHIP, "end capture: %s", hipGetErrorString(ee));
            hipError_t ei = hipGraphInstantiate(&m->graph_exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ei != hipSuccess) {
                m->graph_exec = nullptr;
                return fail(ESDG_EHIP, "graph instantiate: %s", hipGetErrorString(ei));
            }
            m->g_q = q;
            m->g_dq = dq;
            m->g_dt = dt;
            m->g_stream = m->stream;
            m->g_epw = m->epw;
        }
        for (int p = 0; p < pairs; ++p) HIP_TRY(hipGraphLaunch(m->graph_exec, m->stream));
    }
    if (nsteps & 1) return esdg_lsrk_step(m, q, dq, t0 + dt * (nsteps - 1), dt);
    return ESDG_OK;
}

int esdg_check(esdg_mesh_t m)
{
    int rc = check_mesh(m);
    if (rc || (rc = set_device(m))) return rc;
    HIP_TRY(hipMemcpyAsync(m->h_flag, m->d_flag, sizeof(int), hipMemcpyDeviceToHost, m->stream));
    HIP_TRY(hipStreamSynchronize(m->stream));
    if (*m->h_flag) {
        HIP_TRY(hipMemsetAsync(m->d_flag, 0, sizeof(int), m->stream));
        HIP_TRY(hipStreamSynchronize(m->stream));
        return fail(ESDG_ENONPHYS, "non-physical state (rho <= 0, p <= 0 or NaN) met");
    }
    return ESDG_OK;
}

int esdg_entropy(esdg_mesh_t m, const double *q, double out[4])
{
    int rc = check_mesh(m);
    if (rc || (rc = check_ptr(q, "q")) || (rc = set_device(m))) return rc;
    if (!out) return fail(ESDG_EINVAL, "out is NULL");
    if ((rc = ensure_scratch(m, &m->d_r))) return rc;
    rc = esdg_rhs(m, q, m->d_r, 0.0);
    if (rc) return rc;
    GeomParams G = geom(m);
    hipLaunchKernelGGL(entropy_partials_kernel, dim3((unsigned)m->red_blocks), dim3(RED_THREADS),
                       0, m->stream, G, q, (const double *)m->d_r, m->d_partials, m->d_flag);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(RED_THREADS), 0, m->stream,
                       (const double *)m->d_partials, (int)m->red_blocks, m->d_red_out);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(m->h_out, m->d_red_out, sizeof(double) * 4, hipMemcpyDeviceToHost,
                           m->stream));
    rc = esdg_check(m);  // synchronises
    for (int k = 0; k < 4; ++k) out[k] = m->h_out[k];
    return rc;
}

int esdg_cfl_dt(esdg_mesh_t m, const double *q, double cfl, double *dt_out)
{
    int rc = check_mesh(m);
    if (rc || (rc = check_ptr(q, "q")) || (rc = set_device(m))) return rc;
    if (!dt_out) return fail(ESDG_EINVAL, "dt_out is NULL");
    GeomParams G = geom(m);
    hipLaunchKernelGGL(wavespeed_partials_kernel, dim3((unsigned)m->red_blocks),
                       dim3(RED_THREADS), 0, m->stream, G, q, m->d_partials);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(reduce_max_kernel, dim3(1), dim3(RED_THREADS), 0, m->stream,
                       (const double *)m->d_partials, (int)m->red_blocks, m->d_red_out);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(m->h_out, m->d_red_out, sizeof(double), hipMemcpyDeviceToHost,
                           m->stream));
    HIP_TRY(hipStreamSynchronize(m->stream));
    const double smax = m->h_out[0];
    if (!(smax > 0.0) || !std::isfinite(smax))
        return fail(ESDG_ENONPHYS, "wave speed bound is %g", smax);
    *dt_out = cfl / ((m->N + 1) * smax);
    return ESDG_OK;
}

// ---------------------------------------------------------------------------
// Packed multi-member stepping (ensemble serving)
// ---------------------------------------------------------------------------

}  // extern "C"

struct esdg_pack {
    int device;
    hipStream_t stream;
    int n, N, precision, epw, nblocks, capacity;
    void *d_members;     // PackMember[] or PackMemberMixed[]
    int *d_parity;
    int **d_flagptrs;    // each member mesh's non-physical flag
    int *d_flags;        // gathered flags
    int *h_flags;        // pinned copy of d_flags
    char *h_stage;       // pinned staging of the uploads: table, parity, flag pointers
    hipGraphExec_t graph;
};

// Byte offsets of the parity and flag-pointer uploads in a staging buffer for
// cap members, and its size.
static inline size_t pack_stage_parity(int cap)
{
    return std::max(sizeof(PackMember), sizeof(PackMemberMixed)) * cap;
}
static inline size_t pack_stage_fptrs(int cap)
{
    return (pack_stage_parity(cap) + sizeof(int) * cap + 15) & ~(size_t)15;
}
static inline size_t pack_stage_bytes(int cap) { return pack_stage_fptrs(cap) + sizeof(int *) * cap; }

namespace {

void pack_drop_graph(esdg_pack *p)
{
    if (p->graph) {
        (void)hipGraphExecDestroy(p->graph);
        p->graph = nullptr;
    }
}

int pack_enqueue_step(esdg_pack *p, hipStream_t s)
{
    for (int st = 0; st < 5; ++st) {
        if (p->precision == ESDG_FP32_MIXED) {
            const MixedVariant *v = find_mixed_variant(p->N, p->epw);
            if (!v) return fail(ESDG_EINVAL, "no mixed kernel variant for N=%d epw=%d", p->N, p->epw);
            PackLaunchMixed L;
            L.members = (const PackMemberMixed *)p->d_members;
            L.parity = p->d_parity;
            L.n_members = p->n;
            L.nblocks = p->nblocks;
            L.stage = st;
            L.mode = MODE_STAGE;
            L.A = kA[st];
            L.B = kB[st];
            hipLaunchKernelGGL(v->packed, dim3((unsigned)p->nblocks), dim3(v->threads), 0, s, L);
        } else {
            const Variant *v = find_variant(p->N, p->epw);
            if (!v) return fail(ESDG_EINVAL, "no kernel variant for N=%d epw=%d", p->N, p->epw);
            PackLaunch L;
            L.members = (const PackMember *)p->d_members;
            L.parity = p->d_parity;
            L.n_members = p->n;
            L.nblocks = p->nblocks;
            L.stage = st;
            L.mode = MODE_STAGE;
            L.A = kA[st];
            L.B = kB[st];
            hipLaunchKernelGGL(v->packed, dim3((unsigned)p->nblocks), dim3(v->threads), 0, s, L);
        }
        HIP_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(pack_flip_kernel, dim3((unsigned)((p->n + 255) / 256)), dim3(256), 0, s,
                       p->d_parity, p->n);
    HIP_TRY(hipGetLastError());
    return ESDG_OK;
}

}  // namespace

extern "C" {

int esdg_epw_options(int32_t N, int32_t precision, int32_t *out, int32_t cap)
{
    if (N < 1 || N > NQ_MAX - 1) return fail(ESDG_EINVAL, "N=%d outside 1..%d", N, NQ_MAX - 1);
    int cnt = 0;
    if (N > N_FUSED_MAX) return 0;  // the node-per-thread kernels of higher orders
    if (precision == ESDG_FP32_MIXED) {
        for (const MixedVariant &v : kMixedVariants)
            if (v.N == N) {
                if (out && cnt < cap) out[cnt] = v.epw;
                ++cnt;
            }
    } else if (precision == ESDG_FP64) {
        for (const Variant &v : kVariants)
            if (v.N == N) {
                if (out && cnt < cap) out[cnt] = v.epw;
                ++cnt;
            }
    } else {
        return fail(ESDG_EINVAL, "unknown precision %d", precision);
    }
    return cnt;
}

int esdg_pack_create(void *hip_stream, esdg_pack_t *out)
{
    if (!out) return fail(ESDG_EINVAL, "NULL argument");
    esdg_pack *p = new (std::nothrow) esdg_pack();
    if (!p) return fail(ESDG_ENOMEM, "host allocation failed");
    std::memset(p, 0, sizeof *p);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        delete p;
        return fail(ESDG_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    }
    p->device = dev;
    p->stream = (hipStream_t)hip_stream;
    *out = p;
    return ESDG_OK;
}

int esdg_pack_destroy(esdg_pack_t p)
{
    if (!p) return ESDG_OK;
    int rc = ESDG_OK;
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) rc = fail(ESDG_EHIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
    pack_drop_graph(p);
    if (p->d_members) (void)hipFree(p->d_members);
    if (p->d_parity) (void)hipFree(p->d_parity);
    if (p->d_flagptrs) (void)hipFree(p->d_flagptrs);
    if (p->d_flags) (void)hipFree(p->d_flags);
    if (p->h_flags) (void)hipHostFree(p->h_flags);
    if (p->h_stage) (void)hipHostFree(p->h_stage);
    delete p;
    return rc;
}

int esdg_pack_set_members(esdg_pack_t p, int32_t n, const esdg_mesh_t *meshes, double *const *q0,
                          double *const *q1, double *const *dq, const double *dt,
                          const int32_t *parity)
{
    if (!p) return fail(ESDG_EINVAL, "NULL pack");
    if (n < 1) return fail(ESDG_EINVAL, "a pack needs at least one member");
    if (!meshes || !q0 || !q1 || !dq || !dt || !parity) return fail(ESDG_EINVAL, "NULL array");
    const esdg_mesh *m0 = meshes[0];
    if (!m0) return fail(ESDG_EINVAL, "NULL mesh");
    const int N = m0->N, prec = m0->desc.precision, epw = m0->epw;
    if (N > N_FUSED_MAX)
        return fail(ESDG_EINVAL, "packed stepping supports orders up to %d", N_FUSED_MAX);
    int64_t blocks = 0;
    const bool mixed = prec == ESDG_FP32_MIXED;
    std::string tab(mixed ? sizeof(PackMemberMixed) * n : sizeof(PackMember) * n, '\0');
    std::vector<int *> flagptrs(n);
    for (int i = 0; i < n; ++i) {
        esdg_mesh *m = meshes[i];
        if (!m) return fail(ESDG_EINVAL, "member %d: NULL mesh", i);
        if (m->N != N || m->desc.precision != prec || m->epw != epw || m->device != p->device)
            return fail(ESDG_EINVAL, "member %d: N, precision, epw and device must match", i);
        if (m->curved) return fail(ESDG_EINVAL, "member %d: curved meshes are not packed", i);
        int rc;
        if ((rc = check_ptr(q0[i], "q0")) || (rc = check_ptr(q1[i], "q1")) ||
            (rc = check_ptr(dq[i], "dq")))
            return rc;
        if (overlaps(q0[i], q1[i], m->state_len) || overlaps(q0[i], dq[i], m->state_len) ||
            overlaps(q1[i], dq[i], m->state_len))
            return fail(ESDG_EINVAL, "member %d: q0, q1 and dq must not overlap", i);
        if (parity[i] != 0 && parity[i] != 1)
            return fail(ESDG_EINVAL, "member %d: parity must be 0 or 1", i);
        StageParams P = base_params(m);
        P.mode = MODE_STAGE;
        P.dq = dq[i];
        P.dt = dt[i];
        P.nblocks = (int)((m->ne + epw - 1) / epw);
        flagptrs[i] = m->d_flag;
        if (mixed) {
            PackMemberMixed pm;
            std::memset(&pm, 0, sizeof pm);
            pm.M.s = P;
            pm.M.ref_r = m->d_ref_r;
            pm.M.ref_p = m->d_ref_p;
            pm.M.rr_mom = m->d_rr_mom;
            pm.bufs[0] = q0[i];
            pm.bufs[1] = q1[i];
            pm.block_begin = (int)blocks;
            std::memcpy(&tab[sizeof(pm) * i], &pm, sizeof pm);
        } else {
            PackMember pm;
            std::memset(&pm, 0, sizeof pm);
            pm.P = P;
            pm.bufs[0] = q0[i];
            pm.bufs[1] = q1[i];
            pm.block_begin = (int)blocks;
            std::memcpy(&tab[sizeof(pm) * i], &pm, sizeof pm);
        }
        blocks += P.nblocks;
        if (blocks > 0x7fffffff) return fail(ESDG_EINVAL, "pack too large");
    }
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != p->device) HIP_TRY(hipSetDevice(p->device));
    // the previous step may still read the old table
    HIP_TRY(hipStreamSynchronize(p->stream));
    pack_drop_graph(p);
    if (n > p->capacity) {
        // grow geometrically; the new tables are allocated before the old
        // ones are freed, so a failed allocation leaves the pack as it was
        const int cap = std::max(n, 2 * p->capacity);
        void *members = nullptr;
        int *par = nullptr, *flags = nullptr, *hflags = nullptr;
        int **fptrs = nullptr;
        char *stage = nullptr;
        const bool ok =
            hipMalloc(&members, std::max(sizeof(PackMember), sizeof(PackMemberMixed)) * cap) ==
                hipSuccess &&
            hipMalloc(&par, sizeof(int) * cap) == hipSuccess &&
            hipMalloc(&fptrs, sizeof(int *) * cap) == hipSuccess &&
            hipMalloc(&flags, sizeof(int) * cap) == hipSuccess &&
            hipHostMalloc(&hflags, sizeof(int) * cap, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc(&stage, pack_stage_bytes(cap), hipHostMallocDefault) == hipSuccess;
        if (!ok) {
            if (members) (void)hipFree(members);
            if (par) (void)hipFree(par);
            if (fptrs) (void)hipFree(fptrs);
            if (flags) (void)hipFree(flags);
            if (hflags) (void)hipHostFree(hflags);
            if (stage) (void)hipHostFree(stage);
            return fail(ESDG_ENOMEM, "pack table allocation failed");
        }
        if (p->d_members) (void)hipFree(p->d_members);
        if (p->d_parity) (void)hipFree(p->d_parity);
        if (p->d_flagptrs) (void)hipFree(p->d_flagptrs);
        if (p->d_flags) (void)hipFree(p->d_flags);
        if (p->h_flags) (void)hipHostFree(p->h_flags);
        if (p->h_stage) (void)hipHostFree(p->h_stage);
        p->d_members = members;
        p->d_parity = par;
        p->d_flagptrs = fptrs;
        p->d_flags = flags;
        p->h_flags = hflags;
        p->h_stage = stage;
        p->capacity = cap;
    }
    // from here on the device table no longer matches the old member set:
    // a failed upload leaves an empty pack, whose step() is rejected
    p->n = 0;
    // uploads from the pinned staging buffer, ordered on the pack's stream
    // before the next step; the stream was idle when the buffer was filled,
    // and the next call waits for it before refilling
    char *st_par = p->h_stage + pack_stage_parity(p->capacity);
    char *st_fp = p->h_stage + pack_stage_fptrs(p->capacity);
    std::memcpy(p->h_stage, tab.data(), tab.size());
    std::memcpy(st_par, parity, sizeof(int32_t) * n);
    std::memcpy(st_fp, flagptrs.data(), sizeof(int *) * n);
    HIP_TRY(hipMemcpyAsync(p->d_members, p->h_stage, tab.size(), hipMemcpyHostToDevice,
                           p->stream));
    HIP_TRY(hipMemcpyAsync(p->d_parity, st_par, sizeof(int32_t) * n, hipMemcpyHostToDevice,
                           p->stream));
    HIP_TRY(hipMemcpyAsync(p->d_flagptrs, st_fp, sizeof(int *) * n, hipMemcpyHostToDevice,
                           p->stream));
    p->n = n;
    p->N = N;
    p->precision = prec;
    p->epw = epw;
    p->nblocks = (int)blocks;
    return ESDG_OK;
}

int esdg_pack_step(esdg_pack_t p, int32_t nsteps)
{
    if (!p) return fail(ESDG_EINVAL, "NULL pack");
    if (nsteps < 0) return fail(ESDG_EINVAL, "nsteps < 0");
    if (p->n < 1) return fail(ESDG_EINVAL, "pack has no members");
    if (nsteps == 0) return ESDG_OK;
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != p->device) HIP_TRY(hipSetDevice(p->device));
    if (!p->graph) {
        hipStream_t cs;
        HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipError_t eb = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        int rc = ESDG_OK;
        hipGraph_t graph = nullptr;
        if (eb == hipSuccess) rc = pack_enqueue_step(p, cs);
        hipError_t ee = (eb == hipSuccess) ? hipStreamEndCapture(cs, &graph) : eb;
        (void)hipStreamDestroy(cs);
        if (eb != hipSuccess) return fail(ESDG_EHIP, "capture: %s", hipGetErrorString(eb));
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (ee != hipSuccess) return fail(ESDG_EHIP, "end capture: %s", hipGetErrorString(ee));
        hipError_t ei = hipGraphInstantiate(&p->graph, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) {
            p->graph = nullptr;
            return fail(ESDG_EHIP, "graph instantiate: %s", hipGetErrorString(ei));
        }
    }
    for (int s = 0; s < nsteps; ++s) HIP_TRY(hipGraphLaunch(p->graph, p->stream));
    return ESDG_OK;
}

int esdg_pack_flags(esdg_pack_t p, int32_t *out)
{
    if (!p) return fail(ESDG_EINVAL, "NULL pack");
    if (!out) return fail(ESDG_EINVAL, "out is NULL");
    if (p->n < 1) return fail(ESDG_EINVAL, "pack has no members");
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != p->device) HIP_TRY(hipSetDevice(p->device));
    hipLaunchKernelGGL(pack_flags_kernel, dim3((unsigned)((p->n + 255) / 256)), dim3(256), 0,
                       p->stream, (int *const *)p->d_flagptrs, p->n, p->d_flags);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(p->h_flags, p->d_flags, sizeof(int) * p->n, hipMemcpyDeviceToHost,
                           p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    for (int i = 0; i < p->n; ++i) out[i] = p->h_flags[i] ? 1 : 0;
    return ESDG_OK;
}

int esdg_pack_flags_async(esdg_pack_t p, int32_t *out_host)
{
    if (!p) return fail(ESDG_EINVAL, "NULL pack");
    if (!out_host) return fail(ESDG_EINVAL, "out_host is NULL");
    if (p->n < 1) return fail(ESDG_EINVAL, "pack has no members");
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != p->device) HIP_TRY(hipSetDevice(p->device));
    hipLaunchKernelGGL(pack_flags_kernel, dim3((unsigned)((p->n + 255) / 256)), dim3(256), 0,
                       p->stream, (int *const *)p->d_flagptrs, p->n, p->d_flags);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(out_host, p->d_flags, sizeof(int) * p->n, hipMemcpyDeviceToHost,
                           p->stream));
    return ESDG_OK;
}

}  // extern "C"
