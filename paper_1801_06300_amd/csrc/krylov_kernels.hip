// Krylov / Arnoldi and utility kernels (see krylov_kernels.hpp).
#include "krylov_kernels.hpp"

#include <hip/hip_runtime.h>

#include <cmath>

namespace pcexp {

constexpr int RT = 512;          // threads per reduction block
constexpr int RW = RT / 64;      // waves per reduction block
constexpr int MAXB = 512;        // max reduction blocks (partials per column)
constexpr int PLD = MAXB;        // partials are column-major: part[col * PLD + block]

size_t gs_blocks(size_t n) {
  size_t b = (n + RT - 1) / RT;
  if (b > MAXB) b = MAXB;
  if (b < 1) b = 1;
  return b;
}

__device__ __forceinline__ double wave_sum(double a) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
  return a;
}

__device__ __forceinline__ double wave_min(double a) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) a = fmin(a, __shfl_xor(a, off, 64));
  return a;
}

// Reductions: every kernel writes one partial per block and column
// (part[col * PLD + block]); the next kernel on the stream -- which sees them
// by kernel-boundary ordering -- sums each column in a fixed order.  No
// grid-wide fences or atomics: on gfx950 an agent-scope fence writes back
// the L2 and costs far more than the streaming work of these kernels.

// Fixed-order sum of column c over nblk partials, by one wave (all lanes get it).
__device__ __forceinline__ double col_sum(const double* part, int c, int nblk) {
  const int lane = threadIdx.x & 63;
  double a = 0.0;
  for (int b = lane; b < nblk; b += 64) a += part[(size_t)c * PLD + b];
  return wave_sum(a);
}

// Block-reduce NV per-thread accumulators into part[c * PLD + blockIdx.x].
template <int NV>
__device__ __forceinline__ void block_partials(const double* acc, int nvec, double* part) {
  __shared__ double red[RW][NV];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    if (i < nvec) {
      double a = wave_sum(acc[i]);
      if (lane == 0) red[wid][i] = a;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nvec; i += RT) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < RW; ++w) s += red[w][i];
    part[(size_t)i * PLD + blockIdx.x] = s;
  }
}

// ------------------------------------------------------------------ state
__global__ void init_state_kernel(KState* ks, double eta) {
  const int t = threadIdx.x;
  for (int i = t; i < KLD * KMAX; i += blockDim.x) ks->H[i] = 0.0;
  for (int i = t; i < KMAX + 2; i += blockDim.x) {
    ks->sigma[i] = 0.0;
    ks->hcol[i] = 0.0;
  }
  for (int i = t; i < KMAX + 4; i += blockDim.x) ks->y[i] = 0.0;
  if (t < 8) ks->counter[t] = 0u;
  if (t == 0) {
    ks->beta = ks->wnorm = ks->hlast = ks->fd_eps = 0.0;
    ks->eta = eta;
    ks->m_eff = 0;
    ks->done = 0;
    ks->breakdown = 0;
  }
}

void k_init_state(KState* ks, double eta, hipStream_t st) {
  hipLaunchKernelGGL(init_state_kernel, dim3(1), dim3(256), 0, st, ks, eta);
}

// Partial buffers of one Arnoldi run: three column blocks of (KMAX+2) columns.
__device__ __forceinline__ double* pbuf(double* part, int which) { return part + (size_t)which * (KMAX + 2) * PLD; }
__device__ __forceinline__ const double* pbuf(const double* part, int which) {
  return part + (size_t)which * (KMAX + 2) * PLD;
}

// ------------------------------------------------- start: V_0 = b, beta = |b|
template <typename TV>
__global__ __launch_bounds__(RT) void start_kernel(const double* __restrict__ b, TV* __restrict__ V0,
                                                   size_t n, double* part) {
  double acc[1] = {0.0};
  for (size_t i = (size_t)blockIdx.x * RT + threadIdx.x; i < n; i += (size_t)gridDim.x * RT) {
    double x = b[i];
    V0[i] = (TV)x;
    acc[0] += x * x;
  }
  block_partials<1>(acc, 1, pbuf(part, 2));
}

__global__ __launch_bounds__(64) void start_finalize(KState* ks, const double* part, int nblk) {
  const double s = col_sum(pbuf(part, 2), 0, nblk);
  if (threadIdx.x == 0) {
    const double beta = sqrt(s);
    ks->beta = beta;
    if (beta > 0.0) {
      ks->sigma[0] = 1.0 / beta;
    } else {
      ks->done = 1;
      ks->m_eff = 0;
    }
  }
}

template <typename TV>
void k_start(const double* b, TV* V0, size_t n, KState* ks, double* part, hipStream_t st) {
  const int nb = (int)gs_blocks(n);
  hipLaunchKernelGGL(start_kernel<TV>, dim3(nb), dim3(RT), 0, st, b, V0, n, part);
  hipLaunchKernelGGL(start_finalize, dim3(1), dim3(64), 0, st, ks, part, nb);
}

// Vector loads of the Gram-Schmidt kernels are unconditional: slots beyond
// the live vectors re-read the last live vector (an L1/L2 hit) and get a zero
// coefficient, so the compiler can keep all NV loads of an element in flight.
__device__ __forceinline__ int clampv(int i, int nvec) { return i < nvec ? i : nvec - 1; }

// Iteration j (vectors V_0..V_j live, w stored in slot V_{j+1}):
//   dots:         raw1_i = V_i . w, |w|^2                         -> partials 0
//   coeff:        hcol_i = sigma_i^2 raw1_i                          (one block)
//   update_dots:  w -= sum hcol_i V_i;  raw2_i = V_i . w             -> partials 1
//   coeff:        hcol_i = sigma_i^2 raw2_i                          (one block)
//   update_norm:  w -= sum hcol_i V_i;  |w|^2                        -> partials 2
//   finalize:     H[i][j] = sigma_i (raw1_i + raw2_i), h_{j+1,j} = |w|,
//                 breakdown test, sigma_{j+1} = 1/h_{j+1,j}          (one block)
template <typename TV, int NV>
__global__ __launch_bounds__(RT) void dots_kernel(const TV* __restrict__ V, size_t ld, int j, size_t n,
                                                  const KState* ks, double* part) {
  if (ks->done) return;
  const int nvec = j + 1;
  const TV* w = V + (size_t)(j + 1) * ld;
  double acc[NV];
  double aw = 0.0;
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  for (size_t idx = (size_t)blockIdx.x * RT + threadIdx.x; idx < n; idx += (size_t)gridDim.x * RT) {
    const double wv = (double)w[idx];
    TV vr[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) vr[i] = V[(size_t)clampv(i, nvec) * ld + idx];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] += (double)vr[i] * wv;
    aw += wv * wv;
  }
  // block partials: columns 0..nvec-1 = projections, column nvec = |w|^2
  double* out = pbuf(part, 0);
  __shared__ double red[RW][NV + 1];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    if (i < nvec) {
      double a = wave_sum(acc[i]);
      if (lane == 0) red[wid][i] = a;
    }
  }
  double a = wave_sum(aw);
  if (lane == 0) red[wid][NV] = a;
  __syncthreads();
  for (int i = threadIdx.x; i <= nvec; i += RT) {
    const int src = (i == nvec) ? NV : i;
    double s = 0.0;
#pragma unroll
    for (int w2 = 0; w2 < RW; ++w2) s += red[w2][src];
    out[(size_t)i * PLD + blockIdx.x] = s;
  }
}

template <typename TV, int NV, int IN, int OUT, bool DOTS>
__global__ __launch_bounds__(RT) void update_kernel(TV* __restrict__ V, size_t ld, int j, size_t n,
                                                    const KState* ks, double* part) {
  if (ks->done) return;
  const int nvec = j + 1;
  __shared__ double hs[NV];
  for (int i = threadIdx.x; i < NV; i += RT) hs[i] = (i < nvec) ? ks->hcol[i] : 0.0;
  __syncthreads();
  TV* w = V + (size_t)(j + 1) * ld;
  double acc[DOTS ? NV : 1];
#pragma unroll
  for (int i = 0; i < (DOTS ? NV : 1); ++i) acc[i] = 0.0;
  for (size_t idx = (size_t)blockIdx.x * RT + threadIdx.x; idx < n; idx += (size_t)gridDim.x * RT) {
    TV vr[NV];
    double wv = (double)w[idx];
#pragma unroll
    for (int i = 0; i < NV; ++i) vr[i] = V[(size_t)clampv(i, nvec) * ld + idx];
#pragma unroll
    for (int i = 0; i < NV; ++i) wv -= hs[i] * (double)vr[i];
    const TV ws = (TV)wv;
    w[idx] = ws;
    const double wq = (double)ws;
    if constexpr (DOTS) {
#pragma unroll
      for (int i = 0; i < NV; ++i) acc[i] += (double)vr[i] * wq;
    } else {
      acc[0] += wq * wq;
    }
  }
  if constexpr (DOTS) block_partials<NV>(acc, nvec, pbuf(part, OUT));
  else block_partials<1>(acc, 1, pbuf(part, OUT));
}

__global__ __launch_bounds__(RT) void finalize_kernel(KState* ks, const double* part, int j, int nblk) {
  if (ks->done) return;
  const int nvec = j + 1;
  __shared__ double r1[KMAX + 1], r2[KMAX + 1];
  __shared__ double nrm;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int c = wid; c <= nvec; c += RW) {
    const double s = col_sum(pbuf(part, 0), c, nblk);
    if (lane == 0) r1[c] = s;
  }
  for (int c = wid; c <= nvec; c += RW) {
    const double s = (c < nvec) ? col_sum(pbuf(part, 1), c, nblk) : col_sum(pbuf(part, 2), 0, nblk);
    if (lane == 0) {
      if (c < nvec) r2[c] = s;
      else nrm = s;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int c = 0; c < nvec; ++c) ks->H[(size_t)j * KLD + c] = ks->sigma[c] * (r1[c] + r2[c]);
    ks->wnorm = sqrt(r1[nvec]);
    const double h = sqrt(nrm);
    ks->H[(size_t)j * KLD + j + 1] = h;
    ks->hlast = h;
    ks->m_eff = j + 1;
    if (!(h > ks->eta * ks->wnorm)) {
      ks->breakdown = 1;
      ks->done = 1;
    } else {
      ks->sigma[j + 1] = 1.0 / h;
    }
  }
}

// Launch with the smallest vector-count bucket that holds j + 1 vectors.
#define PCEXP_GS_DISPATCH(KERNEL, ...)                                                          \
  do {                                                                                          \
    const int nv_ = j + 1;                                                                      \
    dim3 g_(gs_blocks(n)), b_(RT);                                                              \
    if (nv_ <= 4) hipLaunchKernelGGL((KERNEL(4)), g_, b_, 0, st, __VA_ARGS__);                  \
    else if (nv_ <= 8) hipLaunchKernelGGL((KERNEL(8)), g_, b_, 0, st, __VA_ARGS__);             \
    else if (nv_ <= 12) hipLaunchKernelGGL((KERNEL(12)), g_, b_, 0, st, __VA_ARGS__);           \
    else if (nv_ <= 16) hipLaunchKernelGGL((KERNEL(16)), g_, b_, 0, st, __VA_ARGS__);           \
    else if (nv_ <= 20) hipLaunchKernelGGL((KERNEL(20)), g_, b_, 0, st, __VA_ARGS__);           \
    else if (nv_ <= 24) hipLaunchKernelGGL((KERNEL(24)), g_, b_, 0, st, __VA_ARGS__);           \
    else if (nv_ <= 28) hipLaunchKernelGGL((KERNEL(28)), g_, b_, 0, st, __VA_ARGS__);           \
    else if (nv_ <= 32) hipLaunchKernelGGL((KERNEL(32)), g_, b_, 0, st, __VA_ARGS__);           \
    else if (nv_ <= 40) hipLaunchKernelGGL((KERNEL(40)), g_, b_, 0, st, __VA_ARGS__);           \
    else if (nv_ <= 48) hipLaunchKernelGGL((KERNEL(48)), g_, b_, 0, st, __VA_ARGS__);           \
    else if (nv_ <= 56) hipLaunchKernelGGL((KERNEL(56)), g_, b_, 0, st, __VA_ARGS__);           \
    else hipLaunchKernelGGL((KERNEL(64)), g_, b_, 0, st, __VA_ARGS__);                          \
  } while (0)

#define PCEXP_K_DOTS(NV) dots_kernel<TV, NV>
#define PCEXP_K_UPD(NV) update_kernel<TV, NV, 0, 1, true>
#define PCEXP_K_NRM(NV) update_kernel<TV, NV, 1, 2, false>

// One block: the coefficients on the stored vectors for the next update,
// hcol[c] = sigma_c^2 * (V_c . w), from the partials of buffer `which`.
__global__ __launch_bounds__(RT) void coeff_kernel(KState* ks, const double* part, int which, int nvec, int nblk) {
  if (ks->done) return;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int c = wid; c < nvec; c += RW) {
    const double s = col_sum(pbuf(part, which), c, nblk);
    if (lane == 0) ks->hcol[c] = s * ks->sigma[c] * ks->sigma[c];
  }
}

template <typename TV>
void k_dots(const TV* V, size_t ld, int j, size_t n, KState* ks, double* part, hipStream_t st) {
  PCEXP_GS_DISPATCH(PCEXP_K_DOTS, V, ld, j, n, ks, part);
  hipLaunchKernelGGL(coeff_kernel, dim3(1), dim3(RT), 0, st, ks, part, 0, j + 1, (int)gs_blocks(n));
}
template <typename TV>
void k_update_dots(TV* V, size_t ld, int j, size_t n, KState* ks, double* part, hipStream_t st) {
  PCEXP_GS_DISPATCH(PCEXP_K_UPD, V, ld, j, n, ks, part);
  hipLaunchKernelGGL(coeff_kernel, dim3(1), dim3(RT), 0, st, ks, part, 1, j + 1, (int)gs_blocks(n));
}
template <typename TV>
void k_update_norm(TV* V, size_t ld, int j, size_t n, KState* ks, double* part, hipStream_t st) {
  PCEXP_GS_DISPATCH(PCEXP_K_NRM, V, ld, j, n, ks, part);
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(RT), 0, st, ks, part, j, (int)gs_blocks(n));
}

// ------------------------------------------------------------ Hessenberg phi
// y = beta * phi_k(dt H_m) e_1, m = m_eff, from the exponential of the
// augmented (m+k) x (m+k) matrix [[dt H, e_1, 0], [0, 0, I_{k-1}], [0, 0, 0]]
// (k = 0: exp(dt H) e_1).  exp(A) by scaling and squaring of the degree-18
// Taylor polynomial: A is scaled by 2^-s so that |A|_1 <= 1, where the
// truncation error is below 1/19! ~ 8e-18 relative; the polynomial is
// evaluated by the Paterson-Stockmeyer scheme in powers of X^4 (7 matrix
// products), then squared s times.  Matrix products only: no pivoting, few
// barriers.  One workgroup; matrices column-major in `mem` (LDS or global).
constexpr int PHI_T = 256;

__device__ void mat_mul(const double* A, const double* B, double* C, int n) {
  for (int t = threadIdx.x; t < n * n; t += PHI_T) {
    const int i = t % n, jj = t / n;
    double s = 0.0;
    for (int l = 0; l < n; ++l) s += A[l * n + i] * B[jj * n + l];
    C[jj * n + i] = s;
  }
  __syncthreads();
}

// C = A * B + D  (D may alias neither A nor B nor C)
__device__ void mat_mul_add(const double* A, const double* B, const double* D, double* C, int n) {
  for (int t = threadIdx.x; t < n * n; t += PHI_T) {
    const int i = t % n, jj = t / n;
    double s = D[t];
    for (int l = 0; l < n; ++l) s += A[l * n + i] * B[jj * n + l];
    C[jj * n + i] = s;
  }
  __syncthreads();
}

__device__ void phi_body(KState* ks, const double* dtp, int k, double* mem) {
  const int m = ks->m_eff;
  const int tid = threadIdx.x;
  if (m == 0) {
    for (int i = tid; i < KMAX + 4; i += PHI_T) ks->y[i] = 0.0;
    return;
  }
  const int n = (k >= 1) ? m + k : m;
  const int nn = n * n;
  double* X = mem;          // scaled A
  double* X2 = X + nn;
  double* X3 = X2 + nn;
  double* X4 = X3 + nn;
  double* Bq = X4 + nn;     // current block polynomial
  double* T0 = Bq + nn;     // ping-pong accumulators
  double* T1 = T0 + nn;
  const double dt = *dtp;
  for (int t = tid; t < nn; t += PHI_T) {
    const int i = t % n, jj = t / n;
    double v = 0.0;
    if (i < m && jj < m) {
      if (i <= jj + 1) v = dt * ks->H[(size_t)jj * KLD + i];
    } else if (k >= 1 && jj == m && i == 0) {
      v = 1.0;
    } else if (k >= 2 && jj >= m + 1 && i == jj - 1) {
      v = 1.0;
    }
    X[t] = v;
  }
  __syncthreads();
  __shared__ double colsum[KMAX + 4];
  __shared__ int s_sq;
  for (int jj = tid; jj < n; jj += PHI_T) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += fabs(X[jj * n + i]);
    colsum[jj] = s;
  }
  __syncthreads();
  if (tid == 0) {
    double nrm = 0.0;
    for (int jj = 0; jj < n; ++jj) nrm = fmax(nrm, colsum[jj]);
    int s = 0;
    if (nrm > 1.0) s = (int)ceil(log2(nrm));
    s_sq = s;
  }
  __syncthreads();
  const int s = s_sq;
  const double sc = ldexp(1.0, -s);
  for (int t = tid; t < nn; t += PHI_T) X[t] *= sc;
  __syncthreads();
  mat_mul(X, X, X2, n);
  mat_mul(X2, X, X3, n);
  mat_mul(X2, X2, X4, n);
  // Taylor coefficients c_k = 1/k!, k = 0..18; blocks B_i = sum_{r<4} c_{4i+r} X^r,
  // T(X) = B_0 + X^4 (B_1 + X^4 (B_2 + X^4 (B_3 + X^4 B_4))), B_4 = c_16 + c_17 X + c_18 X^2
  double c[19];
  c[0] = 1.0;
  for (int q = 1; q < 19; ++q) c[q] = c[q - 1] / q;
  auto block = [&](int i, double* dst) {
    const double a0 = c[4 * i], a1 = (4 * i + 1 < 19) ? c[4 * i + 1] : 0.0;
    const double a2 = (4 * i + 2 < 19) ? c[4 * i + 2] : 0.0, a3 = (4 * i + 3 < 19) ? c[4 * i + 3] : 0.0;
    for (int t = tid; t < nn; t += PHI_T) {
      const int r = t % n, jj = t / n;
      dst[t] = a1 * X[t] + a2 * X2[t] + a3 * X3[t] + (r == jj ? a0 : 0.0);
    }
    __syncthreads();
  };
  block(4, T0);                      // T0 = B_4
  block(3, Bq);
  mat_mul_add(X4, T0, Bq, T1, n);    // T1 = B_3 + X^4 B_4
  block(2, Bq);
  mat_mul_add(X4, T1, Bq, T0, n);    // T0 = B_2 + X^4 T1
  block(1, Bq);
  mat_mul_add(X4, T0, Bq, T1, n);    // T1 = B_1 + X^4 T0
  block(0, Bq);
  mat_mul_add(X4, T1, Bq, T0, n);    // T0 = B_0 + X^4 T1 = T(X)
  double* P = T0;
  double* Q = T1;
  for (int it = 0; it < s; ++it) {
    mat_mul(P, P, Q, n);
    double* t = P; P = Q; Q = t;
  }
  const int col = (k >= 1) ? n - 1 : 0;
  const double beta = ks->beta;
  for (int i = tid; i < KMAX + 4; i += PHI_T) ks->y[i] = (i < m) ? beta * P[col * n + i] : 0.0;
}

__global__ __launch_bounds__(PHI_T) void hess_phi_lds(KState* ks, const double* dtp, int k) {
  extern __shared__ double smem[];
  phi_body(ks, dtp, k, smem);
}
__global__ __launch_bounds__(PHI_T) void hess_phi_glb(KState* ks, const double* dtp, int k, double* mem) {
  phi_body(ks, dtp, k, mem);
}

void k_hess_phi(KState* ks, const double* dt, int k, int m, double* scratch, hipStream_t st) {
  const int n = m + (k >= 1 ? k : 0);
  const size_t bytes = (size_t)7 * n * n * sizeof(double);
  if (bytes <= 60 * 1024) {
    hipLaunchKernelGGL(hess_phi_lds, dim3(1), dim3(PHI_T), bytes, st, ks, dt, k);
  } else {
    hipLaunchKernelGGL(hess_phi_glb, dim3(1), dim3(PHI_T), 0, st, ks, dt, k, scratch);
  }
}

// -------------------------------------- x = fac dt sum_i y_i sigma_i V_i
template <typename TV, typename TX>
__global__ __launch_bounds__(256) void combine_kernel(const TV* __restrict__ V, size_t ld, const KState* ks,
                                                      const double* base, double* out, TX* xout, double fac,
                                                      const double* dtp, size_t n) {
  __shared__ double c[KMAX];
  __shared__ int meff;
  const double f = fac * (dtp ? *dtp : 1.0);
  if (threadIdx.x == 0) meff = ks->m_eff;
  for (int i = threadIdx.x; i < KMAX; i += blockDim.x) c[i] = f * ks->y[i] * ks->sigma[i];
  __syncthreads();
  const int m = meff;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x) {
    double x = 0.0;
    for (int i = 0; i < m; ++i) x += c[i] * (double)V[(size_t)i * ld + idx];
    if (xout) xout[idx] = (TX)x;
    if (out) out[idx] = (base ? base[idx] : 0.0) + x;
  }
}

template <typename TV, typename TX>
void k_combine(const TV* V, size_t ld, const KState* ks, const double* base, double* out, TX* xout,
               double fac, const double* dtp, size_t n, hipStream_t st) {
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL((combine_kernel<TV, TX>), dim3(blocks), dim3(256), 0, st, V, ld, ks, base, out, xout,
                     fac, dtp, n);
}

// ----------------------------------------------------------------- utilities
template <typename T>
__global__ void fill_kernel(T* p, T v, size_t n, const int* skip) {
  if (skip && *skip) return;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
template <typename T>
void k_fill(T* p, T v, size_t n, const int* skip, hipStream_t st) {
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((fill_kernel<T>), dim3(blocks), dim3(256), 0, st, p, v, n, skip);
}

template <typename TA, typename TB>
__global__ void cast_kernel(const TA* a, TB* b, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) b[i] = (TB)a[i];
}
template <typename TA, typename TB>
void k_cast(const TA* a, TB* b, size_t n, hipStream_t st) {
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((cast_kernel<TA, TB>), dim3(blocks), dim3(256), 0, st, a, b, n);
}

__global__ __launch_bounds__(RT) void sumsq_kernel(const double* __restrict__ x, size_t n, double* part) {
  double acc[1] = {0.0};
  for (size_t i = (size_t)blockIdx.x * RT + threadIdx.x; i < n; i += (size_t)gridDim.x * RT) acc[0] += x[i] * x[i];
  block_partials<1>(acc, 1, part);
}
__global__ __launch_bounds__(64) void sumsq_finalize(const double* part, int nblk, double* out, int mode) {
  const double s = col_sum(part, 0, nblk);
  if (threadIdx.x == 0) *out = mode ? sqrt(s) : s;
}
void k_sumsq(const double* x, size_t n, double* out, int mode, double* part, unsigned* counter,
             hipStream_t st) {
  (void)counter;
  const int nb = (int)gs_blocks(n);
  hipLaunchKernelGGL(sumsq_kernel, dim3(nb), dim3(RT), 0, st, x, n, part);
  hipLaunchKernelGGL(sumsq_finalize, dim3(1), dim3(64), 0, st, part, nb, out, mode);
}

__global__ void fd_eps_kernel(const double* unorm, const double* vnorm, double c0, double* eps) {
  double e = c0 * (1.0 + *unorm);
  if (vnorm) e /= *vnorm;
  *eps = e;
}
void k_fd_eps(const double* unorm, const double* vnorm, double c0, double* eps, hipStream_t st) {
  hipLaunchKernelGGL(fd_eps_kernel, dim3(1), dim3(1), 0, st, unorm, vnorm, c0, eps);
}

template <typename TC>
__global__ void glue_kernel(const double* a, const double* b, const TC* c, double* out, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = a[i] - b[i] - (double)c[i];
}
template <typename TC>
void k_glue_d(const double* a, const double* b, const TC* c, double* out, size_t n, hipStream_t st) {
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL((glue_kernel<TC>), dim3(blocks), dim3(256), 0, st, a, b, c, out, n);
}

__global__ void set_scalar_kernel(double* p, double v) { *p = v; }
void k_set_scalar(double* p, double v, hipStream_t st) {
  hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(1), 0, st, p, v);
}

template <typename T>
__global__ void gemv_kernel(const T* A, const T* v, T* out, int n, const double* vscale, const int* skip) {
  if (skip && *skip) return;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  double s = 0.0;
  for (int c = lane; c < n; c += 64) s += (double)A[(size_t)row * n + c] * (double)v[c];
  s = wave_sum(s);
  if (lane == 0) out[row] = (T)(s * (vscale ? *vscale : 1.0));
}
template <typename T>
void k_gemv(const T* A, const T* v, T* out, int n, const double* vscale, const int* skip, hipStream_t st) {
  hipLaunchKernelGGL((gemv_kernel<T>), dim3((n + 3) / 4), dim3(256), 0, st, A, v, out, n, vscale, skip);
}

// explicit instantiations
template void k_start<double>(const double*, double*, size_t, KState*, double*, hipStream_t);
template void k_start<float>(const double*, float*, size_t, KState*, double*, hipStream_t);
template void k_dots<double>(const double*, size_t, int, size_t, KState*, double*, hipStream_t);
template void k_dots<float>(const float*, size_t, int, size_t, KState*, double*, hipStream_t);
template void k_update_dots<double>(double*, size_t, int, size_t, KState*, double*, hipStream_t);
template void k_update_dots<float>(float*, size_t, int, size_t, KState*, double*, hipStream_t);
template void k_update_norm<double>(double*, size_t, int, size_t, KState*, double*, hipStream_t);
template void k_update_norm<float>(float*, size_t, int, size_t, KState*, double*, hipStream_t);
template void k_combine<double, double>(const double*, size_t, const KState*, const double*, double*, double*,
                                        double, const double*, size_t, hipStream_t);
template void k_combine<float, float>(const float*, size_t, const KState*, const double*, double*, float*,
                                      double, const double*, size_t, hipStream_t);
template void k_combine<float, double>(const float*, size_t, const KState*, const double*, double*, double*,
                                       double, const double*, size_t, hipStream_t);
template void k_fill<double>(double*, double, size_t, const int*, hipStream_t);
template void k_fill<float>(float*, float, size_t, const int*, hipStream_t);
template void k_fill<unsigned>(unsigned*, unsigned, size_t, const int*, hipStream_t);
template void k_cast<double, float>(const double*, float*, size_t, hipStream_t);
template void k_cast<float, double>(const float*, double*, size_t, hipStream_t);
template void k_glue_d<double>(const double*, const double*, const double*, double*, size_t, hipStream_t);
template void k_glue_d<float>(const double*, const double*, const float*, double*, size_t, hipStream_t);
template void k_gemv<double>(const double*, const double*, double*, int, const double*, const int*, hipStream_t);
template void k_gemv<float>(const float*, const float*, float*, int, const double*, const int*, hipStream_t);

}  // namespace pcexp
