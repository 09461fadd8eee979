/*
 * esdg.h -- C ABI of the MI355X (gfx950) entropy-stable DGSEM library.
 *
 * The library evaluates the semi-discrete entropy-stable discontinuous
 * Galerkin spectral-element discretisation dq/dt = R(q) of the 3-D
 * compressible Euler equations with gravity (paper Sec. 3, Eq. nm:semi) on a
 * uniform box of affine hexahedra with (N+1)^3 Legendre-Gauss-Lobatto nodes
 * per element, and advances it with the low-storage RK(5,4) scheme of
 * Carpenter and Kennedy (paper Sec. 3).  Every step runs in hand-written
 * HIP kernels on the device; the host side only validates and launches.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * State layout (FP64, device memory, caller owned):
 *     q[e][v][n],  e = ex + Kx*(ey + Ky*ez),
 *                  v in (rho, rho*u, rho*v, rho*w, rho*E),
 *                  n = i + Nq*(j + Nq*k), Nq = N+1, i/j/k along x/y/z.
 * E is the total energy including the geopotential: E = p/(gamma-1)
 * + rho|u|^2/2 + rho*phi, phi = grav*z (paper Sec. 2).  Gravity points in -z.
 * The boundary is FP64 also for the mixed-precision mode.
 * Node coordinates: x = (1-xi)/2 * X_L + (1+xi)/2 * X_R on each axis, with
 * the element vertices X_e = lo + (hi-lo)*e/K, so that the nodes that two
 * neighbouring elements share on a face coincide bitwise.
 *
 * Ownership: the caller owns every array passed in (device pointers that
 * must stay valid until the mesh's stream has passed the call); the mesh
 * owns its tables, scratch buffers and captured graphs.  All work is
 * enqueued on the mesh's HIP stream and is asynchronous unless stated.
 * Pointers must be 8-byte aligned.  Calls on one mesh must not overlap
 * from several host threads; different meshes are independent.
 *
 * Errors: every entry point returns ESDG_OK (0) or a negative code and
 * never aborts; esdg_last_error() returns a thread-local message for the
 * last failure in the calling thread.
 */
#ifndef ESDG_H
#define ESDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ESDG_OK = 0,
    ESDG_EINVAL = -1,    /* bad argument: N outside 1..15, K < 1, K[0]K[1]K[2] >= 2^31,
                            hi <= lo, NULL/misaligned pointer, periodic z with
                            grav != 0, no compiled kernel variant */
    ESDG_ENOMEM = -2,    /* device allocation failed */
    ESDG_EHIP = -3,      /* HIP runtime error; the message carries its text */
    ESDG_ENONPHYS = -4,  /* rho <= 0, p <= 0 or NaN met in a state */
    ESDG_ENOTIMPL = -5
};

enum { ESDG_SURF_RUSANOV = 0, ESDG_SURF_EC = 1, ESDG_SURF_MATRIX = 2 };
enum { ESDG_FP64 = 0, ESDG_FP32_MIXED = 1 };
enum { ESDG_TERM_VOL = 1, ESDG_TERM_FACE = 2, ESDG_TERM_SRC = 4, ESDG_TERM_ALL = 7 };

typedef struct esdg_mesh *esdg_mesh_t;

/* Mesh description (paper Sec. 3 and the test-case geometry of Sec. 5).
 *   N            polynomial order, 1..15 (Nq = N+1 nodes per direction).
 *                Orders 1..8 run the fused line-per-lane stage kernels;
 *                orders 9..15 run a node-per-thread path, FP64 on the
 *                affine box only, without elements-per-workgroup variants
 *                (epw must be 0) and not packable: one workgroup per element
 *                with the element's primitives in LDS where they fit the
 *                device's LDS per workgroup (N <= 14 on gfx950), else two
 *                launches per stage through a per-node buffer of 72 B held
 *                by the mesh (counted in its footprint)
 *   K[3]         elements per direction
 *   lo/hi[3]     box corners in metres
 *   periodic[3]  1 = periodic in that direction, 0 = reflecting walls
 *   gamma, gas_R ideal gas (1.4, 287.0)
 *   grav         gravitational acceleration in -z (9.81)
 *   coriolis_f   f-plane Coriolis parameter (0 or e.g. 1e-4 s^-1)
 *   surface_flux ESDG_SURF_RUSANOV (EC flux + local Lax-Friedrichs
 *                dissipation), ESDG_SURF_EC (no dissipation) or
 *                ESDG_SURF_MATRIX (EC flux + entropy-stable matrix
 *                dissipation R |Lambda| T R^T [[v]], the Roe-type dissipation
 *                of the paper's surface flux, Sec. 3)
 *   precision    ESDG_FP64 or ESDG_FP32_MIXED
 *   ref_rho/ref_p  FP32_MIXED only: device arrays [e][n] (FP64) holding the
 *                hydrostatic reference state; NULL for FP64
 *   epw          elements per workgroup; 0 = the library's choice
 *   curved       0: the affine box.  1: curved hexahedra (paper Sec. 3,
 *                metric terms G): the box warped by
 *                X_d = x_d + warp[d] L_d prod_c sin(2 pi k_dc s_c),
 *                s = (x - lo)/L, k_dc = 2 for c = d > 0 and 1 otherwise,
 *                which vanishes on the box faces (planar walls, matching
 *                periodic faces).  Metric terms in the conservative curl
 *                form, built on the host at creation (88 B per node of
 *                device geometry plus 24 B of coordinates).  FP64 only,
 *                not packable; a warp that folds an element (J <= 0) is
 *                rejected (ESDG_EINVAL).
 *   warp[3]      the warp amplitudes (fractions of the box lengths) */
typedef struct {
    int32_t N;
    int32_t K[3];
    double lo[3];
    double hi[3];
    int32_t periodic[3];
    double gamma;
    double gas_R;
    double grav;
    double coriolis_f;
    int32_t surface_flux;
    int32_t precision;
    const double *ref_rho;
    const double *ref_p;
    int32_t epw;
    int32_t curved;
    double warp[3];
} esdg_mesh_desc;

/* Create a mesh bound to `hip_stream` (a hipStream_t; NULL = the default
 * stream) on the current device.  Allocates the mesh's tables and scratch
 * (see esdg_mesh_info footprint).  *out receives the handle. */
int esdg_mesh_create(const esdg_mesh_desc *desc, void *hip_stream, esdg_mesh_t *out);

/* Synchronise the mesh's stream, release everything the mesh owns. */
int esdg_mesh_destroy(esdg_mesh_t mesh);

/* Sizes: elements, nodes (= DOF, N_e (N+1)^3), doubles in one state
 * (5 * nodes), and the device bytes the mesh itself holds. */
int esdg_mesh_info(esdg_mesh_t mesh, int64_t *n_elem, int64_t *n_nodes, int64_t *state_len,
                   int64_t *footprint_bytes);

/* Rebind the mesh to another stream (e.g. torch's current stream). */
int esdg_set_stream(esdg_mesh_t mesh, void *hip_stream);

/* Elements per workgroup the launches use (for autotuning); 0 restores the
 * default.  ESDG_EINVAL if the value has no compiled variant (curved meshes
 * compile only the default of each order). */
int esdg_set_epw(esdg_mesh_t mesh, int32_t epw);

/* Elements per workgroup currently used by the mesh's launches. */
int esdg_get_epw(esdg_mesh_t mesh, int32_t *epw);

/* Node coordinates into xyz_dev[e][3][n] (device, caller owned). */
int esdg_node_coords(esdg_mesh_t mesh, double *xyz_dev);

/* r = R(q): the full semi-discrete right-hand side of Eq. (nm:semi) --
 * flux-differencing volume term with the entropy-conservative two-point
 * flux and its gravity term, face flux and lift, Coriolis source.  q and r
 * are device arrays of state_len doubles and must not overlap (ESDG_EINVAL).  t is the
 * time (the operator is autonomous; kept for the dq/dt = R(q, t) form). */
int esdg_rhs(esdg_mesh_t mesh, const double *q_dev, double *r_dev, double t);

/* Debug split of R: only the terms selected by mask (ESDG_TERM_VOL: volume
 * flux differencing; ESDG_TERM_FACE: face flux + lift; ESDG_TERM_SRC:
 * Coriolis source).  The three parts add up to esdg_rhs. */
int esdg_rhs_terms(esdg_mesh_t mesh, const double *q_dev, double *r_dev, int32_t mask);

/* One LSRK(5,4) step in place: for s = 1..5, dq <- A_s dq + dt R(q),
 * q <- q + B_s dq (paper Sec. 3).  dq is caller-owned scratch of
 * state_len doubles (its contents on entry do not matter).  Each stage is
 * one fused kernel (volume + face + source + update); the mesh's own
 * second state buffer holds the ping-pong copy. */
int esdg_lsrk_step(esdg_mesh_t mesh, double *q_dev, double *dq_dev, double t, double dt);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the step
 * of esdg_lsrk_step, same kernels and the same bits, with its ping-pong
 * state in a library-owned device array of 8,388,608 doubles (64 MiB) per
 * device instead of the mesh's lazily allocated buffer.  It calls no
 * hipMalloc/hipFree.  The array is set up once per device when the first
 * mesh is created there and is held until the process ends.  Meshes whose
 * state_len exceeds 8,388,608 doubles are rejected (ESDG_EINVAL) before
 * any work is enqueued.  Every call on a device shares that device's
 * array: calls that overlap on one device (several host threads, or meshes
 * on different streams whose steps can run concurrently) race and must be
 * serialised by the caller.  The array's contents between calls are
 * meaningless (each step writes it before reading it). */
int esdg_lsrk_step_noalloc(esdg_mesh_t mesh, double *q_dev, double *dq_dev, double t, double dt);

/* nsteps LSRK(5,4) steps in place, replayed from a captured HIP graph of
 * two steps (re-captured when q, dq or dt change). */
int esdg_lsrk_run(esdg_mesh_t mesh, double *q_dev, double *dq_dev, double t0, double dt,
                  int32_t nsteps);

/* Diagnostics (paper Sec. 5.2 tracks mass and total energy):
 * out[0] = sum_K int eta dV (eta = -rho s/(gamma-1), s = ln p - gamma ln rho),
 * out[1] = sum_K int rho dV, out[2] = sum_K int rho*E dV,
 * out[3] = sum_a J w_a v_a . R_a(q) (discrete entropy production),
 * with LGL quadrature.  Deterministic two-pass reduction; synchronises the
 * stream and writes the four doubles to host memory `out`.  Returns
 * ESDG_ENONPHYS if a non-physical state was met since the last check. */
int esdg_entropy(esdg_mesh_t mesh, const double *q_dev, double out[4]);

/* dt = cfl / ((N+1) max_a sum_r (|u_r| + c)/h_r), computed on the device;
 * synchronises and writes the host double *dt_out. */
int esdg_cfl_dt(esdg_mesh_t mesh, const double *q_dev, double cfl, double *dt_out);

/* Synchronise and report ESDG_ENONPHYS if any kernel met rho <= 0, p <= 0
 * or NaN since the last check (the flag is cleared). */
int esdg_check(esdg_mesh_t mesh);

/* dst[i] = src[i] for i < n doubles with a plain vectorised copy kernel on
 * `hip_stream` (device pointers, caller owned, must not overlap).  Used to
 * snapshot states and to calibrate hardware byte counters against a copy
 * of known size (reads 8n bytes, writes 8n bytes). */
int esdg_copy(const double *src, double *dst, int64_t n, void *hip_stream);

/* Thread-local text of the last error in this thread ("" if none). */
const char *esdg_last_error(void);

/* Library version string, "esdg-gfx950 <version> src:<hash>", where <hash>
 * identifies the sources the library was built from (the first 16 hex
 * digits of a SHA-256 over the HIP sources and this header). */
const char *esdg_version(void);

/* Host-only: the library's LGL nodes xi[N+1], weights w[N+1] and
 * differentiation matrix D[(N+1)*(N+1)] (row-major, D[i][j] = l_j'(xi_i))
 * for order N in 1..15 (paper Sec. 3: collocated LGL quadrature, matrix-free
 * tensor-product derivatives).  No device work; usable without a GPU. */
int esdg_lgl_tables(int32_t N, double *xi, double *w, double *D);

/* Elements-per-workgroup values compiled for order N and a precision
 * (ESDG_FP64 or ESDG_FP32_MIXED) on the affine box: writes up to cap of them
 * to out (may be NULL) and returns their count (0 for N above 8, whose
 * kernels have no such variants), or a negative error.
 * Curved meshes use the FP64 default of each order only.  Host-only. */
int esdg_epw_options(int32_t N, int32_t precision, int32_t *out, int32_t cap);

/* ---- Packed multi-member stepping (ensemble serving) --------------------
 * A pack advances several independent meshes ("members") of the same order
 * N, precision and elements-per-workgroup with one fused stage launch per
 * LSRK stage: every member's elements are dealt to the workgroups of a
 * single grid through a device descriptor table, so small members share the
 * device with large ones.  One step = 5 packed stage launches + a parity
 * flip, captured once in a HIP graph and replayed (paper Sec. 3: LSRK(5,4);
 * each member evolves exactly as esdg_lsrk_step would evolve it alone).
 * Each member owns two caller-allocated state buffers q0/q1 and dq; its
 * state lives in q0 (parity 0) or q1 (parity 1) and moves to the other
 * buffer after every step, so after k steps it is in q[parity ^ (k & 1)].
 * Members and buffers must stay valid until the pack's stream has passed
 * the last step; calls on one pack must not overlap. */
typedef struct esdg_pack *esdg_pack_t;

/* Create an empty pack bound to hip_stream (NULL = default stream). */
int esdg_pack_create(void *hip_stream, esdg_pack_t *out);

/* Synchronise the pack's stream and free it (members are not touched). */
int esdg_pack_destroy(esdg_pack_t pack);

/* Replace the member set: n meshes (same N <= 8, precision, epw, device), each
 * with q0[i], q1[i], dq[i] (device arrays of its state_len doubles, not
 * overlapping), time step dt[i], and parity[i] in {0, 1} naming the buffer
 * that holds its current state.  Waits for the pack's stream (a step in
 * flight still reads the old table), then uploads the new table on that
 * stream, ordered before the next step, from pinned host memory the pack
 * owns; drops the captured graph. */
int esdg_pack_set_members(esdg_pack_t pack, int32_t n, const esdg_mesh_t *meshes,
                          double *const *q0, double *const *q1, double *const *dq,
                          const double *dt, const int32_t *parity);

/* nsteps LSRK(5,4) steps of every member (graph replay, asynchronous). */
int esdg_pack_step(esdg_pack_t pack, int32_t nsteps);

/* Failure isolation for ensemble serving: out[i] = 1 if member i (in the
 * order of the last esdg_pack_set_members) met rho <= 0, p <= 0 or NaN in
 * a stage since its flag was last read, else 0; the flags are cleared.  Each
 * member's flag is its mesh's own (also read by esdg_check).  Synchronises
 * the pack's stream; out is host memory of at least n int32.  The other
 * members' states are unaffected by a failing one (members share no data). */
int esdg_pack_flags(esdg_pack_t pack, int32_t *out);

/* esdg_pack_flags without synchronising: enqueues on the pack's stream the
 * gathering (and clearing) of every member's flag into out_host[i] (nonzero:
 * member i met rho <= 0, p <= 0 or NaN since its flag was last read).  The
 * values are there once the stream has passed this call (e.g. when an event
 * recorded after it has completed); out_host must hold n int32 of host
 * memory and stay valid until then, and should be pinned (hipHostMalloc),
 * since a copy into pageable memory may complete synchronously.  For a
 * serving loop that must not block on a bucket whose stream queues behind
 * other streams' launches. */
int esdg_pack_flags_async(esdg_pack_t pack, int32_t *out_host);

#ifdef __cplusplus
}
#endif

#endif /* ESDG_H */
