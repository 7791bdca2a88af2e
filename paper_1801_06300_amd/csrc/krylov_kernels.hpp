// Krylov / Arnoldi kernels for gfx950 (paper Sec. 2.2, eqs. (vm), (vm1),
// (vm2), (final1), (final)) and small utility kernels.
//
// Arnoldi with classical Gram-Schmidt and delayed re-orthogonalisation
// (CGS with the second pass of vector j folded into iteration j+1, as in the
// low-synchronisation DCGS2 schemes): per iteration one fused reduction pass
// and one fused update pass over the basis.  The Krylov basis lives in the
// caller's workspace as m+1 vectors V_0..V_m of stride ld; V_j is stored
// unnormalised and used as sigma_j V_j, which removes normalisation passes:
// the JVP writes w = J (sigma_j V_j) straight into the slot V_{j+1}.  Dot
// products accumulate in FP64 whatever the storage type of V; every grid
// reduction is a per-block partial followed by a fixed-order reduction in a
// one-block kernel (no float atomics, so results are bitwise reproducible).
// After a breakdown every later launch of the iteration is a no-op (device
// flag `done`).
#pragma once

#include <hip/hip_runtime.h>

namespace pcexp {

constexpr int KMAX = 64;          // largest Krylov dimension
constexpr int KLD = KMAX + 1;     // leading dimension of H
constexpr int GS_THREADS = 256;
// dimension of the zero-padded matrices of the small exponential (a multiple
// of the 16 x 16 matrix-core tile)
__host__ __device__ constexpr int pad16(int n) { return (n + 15) & ~15; }
// Leading dimension of the Hessenberg exponential's np x np matrices: one
// padding row, so that the rows of one column lie in different LDS banks.
__host__ __device__ constexpr int phi_ld(int np) { return np + 1; }
// Doubles of scratch the exponential of an n x n matrix needs (7 matrices).
__host__ __device__ constexpr size_t phi_scratch_doubles(int n) { return (size_t)7 * pad16(n) * phi_ld(pad16(n)); }

// Arnoldi state.  Quantities that iteration j reads and iteration j writes
// are kept apart (tentative values indexed by iteration, H's tentative column
// double-buffered), because every block of the fused finalise-and-update pass
// recomputes the iteration's small algebra while block 0 publishes it.
struct KState {
  double H[KLD * KMAX];    // column-major Hessenberg, H[j*KLD + i] (final columns, and the tentative last one)
  double htent[2 * KLD];   // tentative column j in htent[(j & 1) * KLD + i]
  double sigma[KMAX + 2];  // final scale of each stored basis vector (v_i = sigma_i V_i)
  double sig_t[KMAX + 2];  // tentative scale of slot j while it holds the once-orthogonalised vector
  double nu_t[KMAX + 2];   // tentative norm estimate of slot j
  double wn_t[KMAX + 2];   // |J q_{j-1}| (breakdown threshold of iteration j)
  double y[KMAX + 4];      // beta * phi_k(dt H) e_1
  double beta;
  double hlast;
  double fd_eps;           // FD increment for a unit direction
  double eta;              // breakdown threshold
  double norm_tmp[4];
  int m_eff;
  int done;                // nonzero once the run has stopped (read by later kernels)
  int done_at;             // iteration at which it stopped (INT_MAX while running)
  int breakdown;
  unsigned counter[8];
};

// State of the reverse sweep through one Arnoldi run.
struct RState {
  double Hbar[KLD * KMAX];   // adjoint of H (same layout), entries i <= j + 1 of column j
  double a[KMAX + 2], b[KMAX + 2], c[KMAX + 2];   // per-iteration coefficients
  double dots[KMAX + 2];     // dot-product results
  double t[4];               // scalar dot results
  double alpha, gamma;       // two-term combination coefficients
  double betabar;            // adjoint of beta = |b|
};

// --- host-side launchers (krylov_kernels.hip) -------------------------------
size_t gs_blocks(size_t n);
void k_init_state(KState* ks, double eta, hipStream_t st);
template <typename TV>
void k_start(const double* b, TV* V0, size_t n, KState* ks, double* part, hipStream_t st);
// Iteration j, after the JVP has written W = J(sig_t[j] V_j) into slot j+1:
// reduce (one pass over V_0..V_{j+1}; or, when the DG JVP launch formed the
// partials per tile, k_gs_colsum), then the fused pass that finalises the
// iteration (every block recomputes the small algebra from the partials,
// block 0 publishes it) and rewrites V_j and V_{j+1}.  After the last
// iteration, reduce with close = true and k_gs_close complete column m-1 of H.
// nt: read the basis with non-temporal loads (for a basis larger than the
// Infinity Cache).
template <typename TV>
void k_gs_reduce(const TV* V, size_t ld, int j, size_t n, KState* ks, double* part, bool close, hipStream_t st,
                 bool nt = false);
template <typename TV>
void k_gs_update(TV* V, size_t ld, int j, size_t n, KState* ks, const double* part, hipStream_t st,
                 bool nt = false);
// The same pass when the reduction left one partial per column (part[c * 512]).
template <typename TV>
void k_gs_update_one(TV* V, size_t ld, int j, size_t n, KState* ks, const double* part, hipStream_t st,
                     bool nt = false);
// Fixed-order sums of columns [0, ncol) of fp (nblk partials each, stride pld)
// into part[c * 512]; a no-op once ks->done is set.
void k_gs_colsum(const double* fp, int pld, int nblk, int ncol, const KState* ks, double* part, hipStream_t st);
void k_gs_close(KState* ks, const double* part, int m, size_t n, hipStream_t st);
// scratch: >= phi_scratch_doubles(m + k) doubles (used when that exceeds the LDS path)
void k_hess_phi(KState* ks, const double* dt, int k, int m, double* scratch, hipStream_t st);
// phi_1 with the Krylov error estimate: halves *dt on the device until the
// estimated relative error is <= tol; scratch >= phi_scratch_doubles(m + 2) doubles.
void k_hess_phi_adapt(KState* ks, double* dt, double tol, int m, double* scratch, hipStream_t st);
// Adaptive dimension: after iteration j (1 <= j < m), stop the run with
// m_eff = j when the error estimate for dimension j at *dt is <= tol;
// scratch >= phi_scratch_doubles(j + 2) doubles.
void k_krylov_check(KState* ks, const double* dt, double tol, int j, double* scratch, hipStream_t st);
template <typename TV, typename TX>
void k_combine(const TV* V, size_t ld, const KState* ks, const double* base, double* out,
               TX* xout, double fac, const double* dtp, size_t n, hipStream_t st);

// reverse sweep (FP64 basis V, v_i = sigma_i V_i)
struct RvComb {
  const double* x;
  const double* axp;
  double axc;
  const double* y;
  const double* ayp;
  double ayc;
  const double* V;
  size_t ld;
  const double* sigma;
  const double* coef;
  int i0, nvec;
};
// out[c] = (sigma_{i0+c} V_{i0+c}) . x (sigma may be null: 1), c < nvec
void k_rv_dots(const double* V, size_t ld, const double* sigma, int i0, int nvec, const double* x, size_t n,
               double* part, double* out, hipStream_t st);
void k_rv_combine(const RvComb& a, double* out, size_t n, hipStream_t st);
// Iteration j < M - 1 of the reverse sweep in one pass (coefficients from
// k_rv_dots_coef; v_i = sigma_i V_i):
//   r = alpha v_{j+1}_bar + gamma v_{j+1},  wb = r + sum_{i<=j} b_i v_i,
//   wj = sum_{i<=j+1} c_i v_i,  Vb_i += a_i r + b_i wj (i <= j); writes wb.
void k_rv_iter(const double* vb1, const RState* rs, const double* V, size_t ld, const double* sigma, int j,
               double* Vb, double* wb, size_t n, hipStream_t st);
// o1 += y1, o2 += (*s2) y2
void k_rv_acc2(double* o1, const double* y1, double* o2, const double* y2, const double* s2, size_t n,
               hipStream_t st);
void k_rv_rank(double* Vb, size_t ld, int nvec, const double* r, const double* w, const double* a, const double* b,
               bool set, size_t n, hipStream_t st);
void k_rv_init(const KState* ks, RState* rs, double fac, const double* dtp, hipStream_t st);
void k_rv_phi_adjoint(const KState* ks, RState* rs, const double* dots, double fac, const double* dtp, double* mem,
                      hipStream_t st);
void k_rv_coef_w(const KState* ks, RState* rs, int j, const double* cdots, hipStream_t st);
// Iteration j < M - 1: d_i = v_i . v_{j+1}_bar (i <= j + 1) in one pass, then
// alpha, gamma and the coefficients a, b, c into rs
void k_rv_dots_coef(const double* V, size_t ld, const double* sigma, int j, const double* vb1, size_t n, double* part,
                    const KState* ks, RState* rs, hipStream_t st);
void k_rv_coef_b(const KState* ks, RState* rs, const double* tdot, hipStream_t st);
void k_gemv_t(const double* A, const double* v, double* out, int n, hipStream_t st);

// utilities
template <typename T> void k_fill(T* p, T v, size_t n, const int* skip, hipStream_t st);
template <typename TA, typename TB> void k_cast(const TA* a, TB* b, size_t n, hipStream_t st);
// out = sum x^2 over n entries (mode 0) or sqrt of it (mode 1); deterministic.
void k_sumsq(const double* x, size_t n, double* out, int mode, double* part, unsigned* counter,
             hipStream_t st);
// eps = c0 * (1 + *unorm) / *vnorm, or c0*(1 + *unorm) if vnorm == NULL
void k_fd_eps(const double* unorm, const double* vnorm, double c0, double* eps, hipStream_t st);
// out = a - b - c  (double a, b; c of type TC, or NULL for 0)
template <typename TC>
void k_glue_d(const double* a, const double* b, const TC* c, double* out, size_t n, hipStream_t st);
void k_set_scalar(double* p, double v, hipStream_t st);
// *acc += *x (one thread)
void k_add_scalar(double* acc, const double* x, hipStream_t st);
// dense operator: out = A (scale * v)
template <typename T>
void k_gemv(const T* A, const T* v, T* out, int n, const double* vscale, const int* skip,
            hipStream_t st);

}  // namespace pcexp
