/*
 * pcexp.h -- C ABI of libpcexp, the MI355X (gfx950) implementation of the
 * hot path of the PCEXP predictor-corrector exponential integrator for the
 * DG-discretised Euler equations (Li, Luo, Wang, Ju, arXiv 1801.06300).
 *
 * Problem statement followed (paper Sec. 2.1, eq. (starteq)): du/dt = R(u),
 * u in R^K, K = (number of elements) x (variables d+2) x (basis functions).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * Vectors u, R, v, w, b, out are FP64 device pointers of K entries in the
 *    element-major layout [E][k][i]: element E (in the order of the mesh
 *    descriptor), conserved variable k = (rho, rho u, rho v, [rho w], rho E),
 *    basis function i of the paper's orthonormal basis (Sec. 4.3, eqs.
 *    (basis2), (basis), Alg. 1: centred and scaled global monomials in graded
 *    order, x before y before z, modified Gram-Schmidt with s_i > 0).
 *  * `stream` is a hipStream_t passed as void*; NULL is the default stream.
 *    All work is enqueued on it and is asynchronous unless stated otherwise.
 *  * The caller owns every array and the stream.  The context owns its
 *    geometry, tables and a fixed scratch area allocated at creation; no
 *    other entry point allocates device memory.  Host descriptor arrays are
 *    copied by pcexp_create and not retained.
 *  * One host thread and one stream at a time per context: the single-shot
 *    calls (residual, JVP, VJP, functional, dt, totals, projection) work in
 *    the context's scratch, so calls on two streams would race on it; use one
 *    context per stream.  The stepping calls work in the caller's workspace
 *    and share only the context's flag word.
 *  * Errors: argument/mesh/workspace validation returns before any work is
 *    enqueued; HIP failures return PCEXP_E_HIP.  pcexp_last_error() returns a
 *    message for the last failing call on the context.  Kernels record
 *    non-finite values and rho <= 0 or p <= 0 at quadrature points in a
 *    device flag word, reported by the next call that synchronises
 *    (pcexp_stable_dt, or any call given a non-NULL info) as
 *    PCEXP_E_NONFINITE / PCEXP_E_UNPHYSICAL and in info->flags.
 */
#ifndef PCEXP_H
#define PCEXP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pcexp_ctx pcexp_ctx;

typedef enum {
  PCEXP_OK = 0,
  PCEXP_E_ARG = -1,         /* invalid argument */
  PCEXP_E_MESH = -2,        /* malformed mesh (orientation, unmatched face, ...) */
  PCEXP_E_HIP = -3,         /* HIP runtime / launch failure */
  PCEXP_E_WORKSPACE = -4,   /* workspace NULL or smaller than pcexp_workspace_bytes */
  PCEXP_E_NONFINITE = -5,   /* NaN/Inf seen by a kernel */
  PCEXP_E_UNPHYSICAL = -6,  /* rho <= 0 or p <= 0 at a quadrature point */
  PCEXP_E_UNSUPPORTED = -7  /* valid request the library does not implement */
} pcexp_status;

typedef enum { PCEXP_FLUX_LF = 0, PCEXP_FLUX_ROE = 1 } pcexp_flux_kind;

/* F64: everything in FP64.  MIXED: JVP (inputs, arithmetic, output) and the
 * Krylov basis in FP32; Gram-Schmidt projections (FP64 accumulation), the
 * Hessenberg matrix, phi, the Krylov combination, the corrector and the
 * stage residuals R(u_n), R(u*) in FP64. */
typedef enum { PCEXP_PREC_F64 = 0, PCEXP_PREC_MIXED = 1 } pcexp_prec_kind;

/* TANGENT: exact J(u)v (paper Sec. 4.4, eqs. (jac1), (jac2), applied matrix-free).
 * FD: (R(u + eps v) - R(u)) / eps with eps = sqrt(2^-52)(1 + |u|_2)/|v|_2 (FP64 only).
 * ZERO: J = 0 (test mode: PCEXP reduces to Heun's method, eq. (rk2)). */
typedef enum { PCEXP_JVP_TANGENT = 0, PCEXP_JVP_FD = 1, PCEXP_JVP_ZERO = 2 } pcexp_jvp_kind;

/* PCEXP: eqs. (s9)-(s10).  EXP1: first stage only, eq. (s8). */
typedef enum { PCEXP_SCHEME_PCEXP = 0, PCEXP_SCHEME_EXP1 = 1, PCEXP_SCHEME_ETD2 = 2 /* pcexp_step_etd2 only */ }
    pcexp_scheme_kind;

/* Boundary tags: slip wall (mirror ghost state), Riemann-invariant far field. */
typedef enum { PCEXP_BC_SLIP = 1, PCEXP_BC_FARFIELD = 2 } pcexp_bc_kind;

/* Flags reported in info->flags. */
#define PCEXP_FLAG_NONFINITE 1u
#define PCEXP_FLAG_UNPHYSICAL 2u

typedef struct {
  int32_t dim;               /* 2 (triangles) or 3 (tetrahedra) */
  int64_t n_vert;
  const double* vert;        /* host [n_vert][dim] */
  int64_t n_elem;
  const int32_t* elem;       /* host [n_elem][dim+1], positively oriented simplices */
  const int32_t* vert_canon; /* host [n_vert] periodic identification (index of the
                                vertex this one is an image of), or NULL */
  int64_t n_bface;
  const int32_t* bface;      /* host [n_bface][dim] vertex ids of boundary faces */
  const int32_t* bface_tag;  /* host [n_bface] pcexp_bc */
} pcexp_mesh_desc;

typedef struct {
  int32_t p;                 /* polynomial degree, 0..3 in 2D, 0..2 in 3D */
  int32_t flux;              /* pcexp_flux_kind */
  double gamma;              /* ratio of specific heats (paper: 7/5) */
  double farfield_prim[5];   /* rho, u, v, [w], p of the far field (dim+2 used) */
} pcexp_disc_desc;

typedef struct {
  double beta;               /* |b|_2 */
  double h_last;             /* h_{m_eff+1, m_eff} */
  int32_t m_eff;             /* Krylov dimension used (< m after breakdown or an adaptive stop; 0 if b = 0) */
  int32_t breakdown;         /* 1 if the Arnoldi process broke down */
  double err_est;            /* a-posteriori relative error estimate (with a Krylov tolerance set) */
  int32_t dt_halvings;       /* times dt was halved to meet the tolerance */
  int32_t pad;
} pcexp_krylov_info;

typedef struct {
  pcexp_krylov_info k1, k2;  /* predictor and corrector Arnoldi runs */
  double dt;                 /* time step used (by the last step of the call) */
  double res_rho_norm;       /* |R(rho_n)| of eq. (cfl) at u_n */
  uint32_t flags;            /* PCEXP_FLAG_* seen since the previous report */
  double t_advanced;         /* time advanced by the whole call: the sum of the dt each step used */
} pcexp_step_info;

typedef struct {
  int32_t iterations;     /* pseudo-time steps taken */
  int32_t converged;      /* 1 if ||R(rho)|| <= tol was reached */
  double res_rho_norm0;   /* ||R(rho)|| of eq. (cfl) at the initial state */
  double res_rho_norm;    /* ... at the returned state */
} pcexp_steady_info;

/* Create a context for a mesh and discretisation (Sec. 4.2-4.3): builds faces,
 * periodic pairing, geometry, quadrature and basis tables on the host and
 * uploads them.  Synchronises `stream`.  *out is NULL on failure.
 * Quadrature (Sec. 4.3 asks for Gaussian rules): conical-product Gauss-Jacobi
 * rules with p + 1 points per collapsed direction, (p+1)^dim in the volume and
 * (p+1)^(dim-1) per face, except dim = 3, p = 2, which takes fully symmetric
 * rules of the same degree 5 (14 points on the tetrahedron, 7 per face);
 * pcexp_sizes reports both counts. */
pcexp_status pcexp_create(const pcexp_mesh_desc* mesh, const pcexp_disc_desc* disc,
                          void* stream, pcexp_ctx** out);

/* Test operator context: R(u) = A_res u and J v = A_jac v with device row-major
 * n x n FP64 matrices (copied), 1 <= n <= 4096.  Vectors are plain length-n.
 * Lets the same Arnoldi/step code be checked on linear systems and on the
 * scalar split model of Sec. 3 (A_jac = [J], A_res = [J + lambda]). */
pcexp_status pcexp_create_dense(int64_t n, const double* A_jac, const double* A_res,
                                void* stream, pcexp_ctx** out);

void pcexp_destroy(pcexp_ctx* ctx);

/* sizes[0..7] = K, n_elem, dim, n_var, n_basis, n_quad, n_face_quad, p. */
pcexp_status pcexp_sizes(const pcexp_ctx* ctx, int64_t* sizes);

const char* pcexp_last_error(const pcexp_ctx* ctx);

/* Bytes of caller workspace needed by pcexp_arnoldi_phi / pcexp_step for
 * Krylov dimension m (1..64), phi index k (0..3), precision and JVP kind. */
size_t pcexp_workspace_bytes(const pcexp_ctx* ctx, int32_t m, int32_t k, int32_t prec,
                             int32_t jvp);

/* Physical volume quadrature points, device [n_elem][n_quad][dim]. */
pcexp_status pcexp_quad_points(pcexp_ctx* ctx, double* xyz, void* stream);

/* L2 projection (mass = I, Sec. 4.2): u_{E,k,i} = int_E psi_i U_k from values
 * U_qp, device [n_elem][n_quad][n_var] at pcexp_quad_points. */
pcexp_status pcexp_project(pcexp_ctx* ctx, const double* U_qp, double* u, void* stream);

/* U_h at the volume quadrature points, device [n_elem][n_quad][n_var]. */
pcexp_status pcexp_evaluate(pcexp_ctx* ctx, const double* u, double* U_qp, void* stream);

/* R(u) of eq. (euler3) with identity mass and omega = 0 (Sec. 4.2, 4.4). R != u. */
pcexp_status pcexp_residual(pcexp_ctx* ctx, const double* u, double* R, void* stream);

/* Jv = J(u) v, J = dR/du (Sec. 4.4).  u is FP64.  PCEXP_PREC_F64: v and Jv are
 * double*.  PCEXP_PREC_MIXED: v and Jv are float* (FP32 arithmetic and
 * accumulation inside the JVP, the precision of the Krylov basis in a mixed
 * step).  FD is FP64 only.  Jv != v.  Uses the context's scratch. */
pcexp_status pcexp_jvp(pcexp_ctx* ctx, const double* u, const void* v, void* Jv,
                       int32_t jvp, int32_t prec, void* stream);

/* JTw = J(u)^T w, the transpose of the exact Jacobian of Sec. 4.4 (FP64).
 * Dense contexts: A_jac^T w. */
pcexp_status pcexp_vjp(pcexp_ctx* ctx, const double* u, const double* w, double* JTw,
                       void* stream);

/* Second-order adjoint term (reverse mode through an operator that depends on
 * u; not part of the paper, which has no adjoint): in one pass
 * JTw = J(u)^T w and dJTw = d/deps [J(u + eps v)^T w] = (d_u [J(u) v])^T w,
 * by nested forward-mode differentiation of the VJP.  All arrays device FP64,
 * ABI layout, distinct from w and from each other.  Dense contexts: dJTw = 0. */
pcexp_status pcexp_vjp2(pcexp_ctx* ctx, const double* u, const double* v, const double* w,
                        double* JTw, double* dJTw, void* stream);

/* dt of eq. (x3d): CFL min_E h_E / ((2p+1)(|v| + c)), h_E = 2d|E|/|dE|, with v and c
 * at the element centroid.  Synchronises; result on the host. */
pcexp_status pcexp_stable_dt(pcexp_ctx* ctx, const double* u, double cfl, double* dt_host,
                             void* stream);

/* Conserved totals int_Omega U_k dx, host out[n_var].  Synchronises. */
pcexp_status pcexp_conserved_totals(pcexp_ctx* ctx, const double* u, double* out_host,
                                    void* stream);

/* out = Phi_k(dt J(u_lin)) b by the Krylov projection of dimension m (Sec. 2.2,
 * eqs. (vm)-(final)): Arnoldi with classical Gram-Schmidt and a delayed
 * re-orthogonalisation pass, phi_k(dt H_m) e_1 from the exponential of the
 * augmented (m+k) matrix (scaled Taylor polynomial and squaring, on the device).
 * No dt prefactor (k = 0 gives exp(dt J) b).  out != b.  info may be NULL; if
 * not, the call synchronises and fills it.  Breakdown is not an error. */
pcexp_status pcexp_arnoldi_phi(pcexp_ctx* ctx, const double* u_lin, const double* b, double dt,
                               int32_t k, int32_t m, int32_t prec, int32_t jvp, double* out,
                               void* ws, size_t ws_bytes, pcexp_krylov_info* info, void* stream);

/* One step u_n -> u_{n+1} in place: PCEXP (eqs. (s9)-(s10), both stages with J_n)
 * or EXP1 (eq. (s8)).  If dt > 0 it is used; otherwise cfl > 0 gives dt from
 * eq. (x3d) at u_n, computed on the device (no synchronisation).  info as above. */
pcexp_status pcexp_step(pcexp_ctx* ctx, double* u, double dt, double cfl, int32_t m,
                        int32_t scheme, int32_t prec, int32_t jvp, void* ws, size_t ws_bytes,
                        pcexp_step_info* info, void* stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): pcexp_step with its
 * workspace taken from a fixed device array owned by the library, of
 * PCEXP_NOALLOC_WS_BYTES (64 MiB) on each GPU the library runs on, held until
 * the process ends, instead of a caller-provided one.  The caller passes u
 * and info as for pcexp_step; the call allocates nothing.  The context must
 * be used on the device it was created on (PCEXP_E_ARG otherwise).
 * PCEXP_E_WORKSPACE, before any work is enqueued, when
 * pcexp_workspace_bytes(ctx, m, 1, prec, jvp) exceeds the fixed size (for the
 * 2D P2 FP64 step with m = 30 that is about 230 000 unknowns).  All calls on
 * one GPU share its array, which keeps the last call's contents: the step
 * clears what must start at zero, and calls that overlap on one GPU (other
 * streams, other host threads, other contexts) race and must be serialised
 * by the caller.  With info non-NULL the call synchronises as pcexp_step. */
#define PCEXP_NOALLOC_WS_BYTES (64u << 20)
pcexp_status pcexp_step_noalloc(pcexp_ctx* ctx, double* u, double dt, double cfl, int32_t m,
                                int32_t scheme, int32_t prec, int32_t jvp, pcexp_step_info* info,
                                void* stream);

/* nsteps (>= 1) steps as by pcexp_step, in place, with u kept in the internal
 * basis between them: one change of basis in and one out instead of one pair
 * per step, so the result equals nsteps calls of pcexp_step up to the rounding
 * of those basis changes (an orthogonal transform per element).  dt > 0 is
 * the step each step starts from; otherwise each step takes dt from eq. (x3d)
 * at its own u_n with the given cfl.  With a Krylov tolerance set
 * (pcexp_set_krylov_tol) the predictor of each step may halve that dt, so the
 * steps need not be equal.  Same workspace as pcexp_step.  info, if not NULL,
 * describes the last step (its Krylov runs, dt, and ||R(rho)|| of the state it
 * started from), gives in t_advanced the time advanced by all nsteps steps
 * (summed on the device when the steps can differ, else nsteps dt), and
 * reports PCEXP_E_NONFINITE / PCEXP_E_UNPHYSICAL flags raised in any of the
 * steps.  PCEXP_E_ARG for nsteps < 1 or as pcexp_step. */
pcexp_status pcexp_advance(pcexp_ctx* ctx, double* u, int32_t nsteps, double dt, double cfl,
                           int32_t m, int32_t scheme, int32_t prec, int32_t jvp, void* ws,
                           size_t ws_bytes, pcexp_step_info* info, void* stream);

/* ETD2 step, eq. (s7) (the second-order exponential time differencing
 * variant of Sec. 2, not the PCEXP scheme):
 *   u_{n+1} = u_n + dt Phi_1(dt J_n) R_n + dt Phi_2(dt J_n) (N_n - N_{n-1}),
 * with N = R - J_n u on the step (the split of eq. (s3)), so
 * N_n - N_{n-1} = R_n - R_{n-1} - J_n (u_n - u_{n-1}): two Arnoldi runs (phi_1
 * of R_n, phi_2 of the difference) and one JVP.  u (in/out), u_prev and
 * r_prev are device FP64 arrays in ABI layout, K entries each, caller-owned
 * and distinct.  With have_prev != 0 they hold u_{n-1} and R(u_{n-1}) on entry;
 * with have_prev == 0 the step is ETD1, eq. (s8).  On return they hold u_n and
 * R(u_n) for the next call.  dt > 0 fixed (the difference quotient assumes a
 * constant step); FP64 only (prec is implied); jvp as for pcexp_step.
 * Workspace as for pcexp_step with the same m (pcexp_workspace_bytes with
 * k = 1, FP64).  info (optional): k1 the phi_1 run, k2 the phi_2 run (zero
 * without history); synchronises when given.  Errors: PCEXP_E_ARG for
 * missing, aliased or bad arguments, PCEXP_E_WORKSPACE as pcexp_step. */
pcexp_status pcexp_step_etd2(pcexp_ctx* ctx, double* u, double* u_prev, double* r_prev, int32_t have_prev,
                             double dt, int32_t m, int32_t jvp, void* ws, size_t ws_bytes,
                             pcexp_step_info* info, void* stream);

/* Objective for reverse-mode tests: value_host = int_Omega (p_h - p_ref)^2 dx
 * by the volume quadrature rule, p = (gamma-1)(rho E - |rho v|^2 / (2 rho))
 * (Sec. 4.1); grad (optional, device, ABI layout, != u) = d value / d u.
 * Synchronises. */
pcexp_status pcexp_pressure_functional(pcexp_ctx* ctx, const double* u, double p_ref,
                                       double* value_host, double* grad, void* stream);

/* Device-side accumulation for the adjoint workload (asynchronous, no
 * synchronisation), with P(u) the functional of pcexp_pressure_functional:
 *   *value_acc += scale P(u)      value_acc: device FP64 scalar, or NULL;
 *   grad_acc   += scale dP/du(u)  grad_acc: device FP64 vector, ABI layout, or NULL.
 * At least one of them must be given; neither may alias u or the other.
 * The checkpointed gradient of J = sum_n dt P(u_n) seeds and accumulates
 * with it (scale = dt times the incoming cotangent) so that no arithmetic of
 * the sweep happens outside the library.  Uses the context's scratch (one
 * stream at a time per context).  PCEXP_E_ARG for NULL u, no accumulator,
 * aliasing or a non-finite scale / p_ref; PCEXP_E_UNSUPPORTED on dense contexts. */
pcexp_status pcexp_pressure_functional_acc(pcexp_ctx* ctx, const double* u, double p_ref, double scale,
                                           double* value_acc, double* grad_acc, void* stream);

/* Reverse mode of one step (the discrete adjoint of pcexp_step in FP64 with
 * the tangent JVP; not part of the paper): ubar_n = (d u_{n+1} / d u_n)^T
 * ubar_np1 for the step u_n -> u_{n+1} of eqs. (s9)-(s10) (scheme PCEXP) or
 * (s8) (EXP1) with the fixed time step dt > 0 and Krylov dimension m.  The
 * step is recomputed from u_n with both Krylov bases kept in the workspace,
 * then swept backwards: reverse Arnoldi (Gram-Schmidt relations, the adjoint
 * of the Frechet derivative of the Hessenberg exponential, J^T and the
 * second-order term of pcexp_vjp2 per basis vector) and the reverse glue.
 * The result is the exact derivative of the Krylov approximation (not of the
 * exact exponential).  Arrays device FP64, ABI layout; ubar_n != ubar_np1.
 * Workspace: pcexp_step_vjp_workspace_bytes (3(m+1) + 14 vectors of K plus
 * small state), 256-byte aligned, caller-owned.  Synchronises once (to read
 * the Krylov dimensions reached).  The Krylov controls of
 * pcexp_set_krylov_tol / pcexp_set_krylov_adapt do not apply: it
 * differentiates the fixed-dimension, fixed-dt step. */
size_t pcexp_step_vjp_workspace_bytes(const pcexp_ctx* ctx, int32_t m);
pcexp_status pcexp_step_vjp(pcexp_ctx* ctx, const double* u_n, double dt, int32_t m,
                            int32_t scheme, const double* ubar_np1, double* ubar_n, void* ws,
                            size_t ws_bytes, void* stream);

/* Krylov tolerance for pcexp_step / pcexp_steady (0, the default, disables
 * it).  With tol > 0 the predictor's phi_1 is evaluated together with phi_2
 * and the a-posteriori estimate of the relative Krylov error (Saad 1992),
 *   err(dt) = dt h_{m+1,m} |[phi_2(dt H_m) e_1]_m| / |phi_1(dt H_m) e_1|,
 * and dt is halved on the device until err <= tol; the step (both stages)
 * then uses that dt (reported in pcexp_step_info.dt).  The paper sets a
 * Krylov convergence tolerance of 1e-5 (Sec. 5) without defining the
 * control; this is one reading of it. */
pcexp_status pcexp_set_krylov_tol(pcexp_ctx* ctx, double tol);

/* Adaptive Krylov dimension for pcexp_step / pcexp_steady (the paper's
 * Krylov tolerance of Sec. 5 read as a stopping rule for the Arnoldi process;
 * the paper finds EXP1 with it the faster steady solver, Sec. 5).  With
 * check_every = c > 0 and a tolerance tol > 0 set by pcexp_set_krylov_tol,
 * each Arnoldi run of a step (predictor and corrector) evaluates, after
 * every iteration j with j % c == 0 (1 <= j < m), the estimate above for
 * dimension j at the current dt and stops with m_eff = j when it is <= tol;
 * m is the upper bound.  Only the predictor may then halve dt (when even
 * dimension m misses tol).  Each check is one small launch on the stream (no
 * synchronisation); the dimension reached is in pcexp_step_info.
 * check_every = 0 (the default) keeps the dimension fixed at m.  Errors:
 * PCEXP_E_ARG for check_every outside [0, 64]. */
pcexp_status pcexp_set_krylov_adapt(pcexp_ctx* ctx, int32_t check_every);

/* Steady state by pseudo-time stepping (Sec. 5: PCEXP or EXP1 with the CFL
 * ramp of eq. (cfl), CFL(n) = min{CFL_max, max[||R(rho_n)||^-3, 1 + (n-1)/(2p+1)]},
 * ||R(rho)|| = (1/|Omega|)(sum of squared rho coefficients)^(1/2), dt from eq.
 * (x3d) at u_n with CFL(n); the ramp and dt are computed on the device).
 * u (device, ABI layout) is updated in place until ||R(rho)|| <= tol or
 * max_iter steps; the norm is read back every check_every steps (one
 * synchronisation each).  Workspace as pcexp_step.  Not for dense contexts. */
pcexp_status pcexp_steady(pcexp_ctx* ctx, double* u, double cfl_max, double tol, int32_t max_iter,
                          int32_t check_every, int32_t m, int32_t scheme, int32_t prec, int32_t jvp,
                          void* ws, size_t ws_bytes, pcexp_steady_info* info, void* stream);

/* Kernel-class timing with HIP events for the launches made by pcexp_step /
 * pcexp_arnoldi_phi (for roofline reports).  Each timed operation is one
 * kernel; its event pair is passed to that kernel's dispatch on the caller's
 * stream, so the interval is the kernel's own execution time.
 * op = 1: enable and reset (pre-creates the events; call outside timed code);
 * op = 0: disable; op = 2: synchronise and write, for each class c in
 * [0, PCEXP_PROF_NCLASS), out[3c] = total milliseconds, out[3c+1] = launches,
 * out[3c+2] = algorithmic bytes moved (reads + writes the operation needs).
 * Classes: 0 residual, 1 JVP, 2 Gram-Schmidt reduction pass (V^T [U W]),
 * 3 the one-block closing of the last Hessenberg column (no HBM bytes),
 * 4 Gram-Schmidt finalise-and-update pass, 5 Hessenberg phi, 6 Krylov
 * combination, 7 other. */
#define PCEXP_PROF_NCLASS 8
pcexp_status pcexp_profile(pcexp_ctx* ctx, int32_t op, double* out);

#ifdef __cplusplus
}
#endif
#endif /* PCEXP_H */
