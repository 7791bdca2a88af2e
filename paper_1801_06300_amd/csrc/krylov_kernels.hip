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

// Called by all threads after the block has written its partials.  Returns
// true (in every thread) in the last block to arrive.
__device__ __forceinline__ bool arrive_last(unsigned* counter) {
  __shared__ int amlast;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    amlast = (prev == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  if (amlast) __threadfence();
  return amlast != 0;
}

// Fixed-order sum of column c of the partials over nblk blocks, computed by
// one wave; the result is returned in every lane.
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

// ------------------------------------------------- start: V_0 = b, beta = |b|
template <typename TV>
__global__ __launch_bounds__(RT) void start_kernel(const double* __restrict__ b, TV* __restrict__ V0,
                                                   size_t n, KState* ks, double* part) {
  double acc[1] = {0.0};
  for (size_t i = (size_t)blockIdx.x * RT + threadIdx.x; i < n; i += (size_t)gridDim.x * RT) {
    double x = b[i];
    V0[i] = (TV)x;
    acc[0] += x * x;
  }
  block_partials<1>(acc, 1, part);
  if (arrive_last(&ks->counter[0])) {
    if (threadIdx.x < 64) {
      double s = col_sum(part, 0, gridDim.x);
      if (threadIdx.x == 0) {
        double beta = sqrt(s);
        ks->beta = beta;
        if (beta > 0.0) {
          ks->sigma[0] = 1.0 / beta;
        } else {
          ks->done = 1;
          ks->m_eff = 0;
        }
        ks->counter[0] = 0u;
      }
    }
  }
}

template <typename TV>
void k_start(const double* b, TV* V0, size_t n, KState* ks, double* part, hipStream_t st) {
  hipLaunchKernelGGL(start_kernel<TV>, dim3(gs_blocks(n)), dim3(RT), 0, st, b, V0, n, ks, part);
}

// Vector loads of the Gram-Schmidt kernels are unconditional: slots beyond
// the live vectors re-read the last live vector (an L1/L2 hit) and get a zero
// coefficient, so the compiler can keep all NV loads of an element in flight.
__device__ __forceinline__ int clampv(int i, int nvec) { return i < nvec ? i : nvec - 1; }

// ------------------------------------------ pass-1 projections h = V^T w, |w|
template <typename TV, int NV>
__global__ __launch_bounds__(RT) void dots_kernel(const TV* __restrict__ V, size_t ld, int j, size_t n,
                                                  KState* ks, double* part) {
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
  {
    // block partials: columns 0..nvec-1 = projections, column nvec = |w|^2
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
      part[(size_t)i * PLD + blockIdx.x] = s;
    }
  }
  if (arrive_last(&ks->counter[1])) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int c = wid; c <= nvec; c += RW) {
      double s = col_sum(part, c, gridDim.x);
      if (lane == 0) {
        if (c < nvec) ks->hcol[c] = ks->sigma[c] * s;
        else ks->wnorm = sqrt(s);
      }
    }
    if (threadIdx.x == 0) ks->counter[1] = 0u;
  }
}

// ---------------- w -= V (sigma .* h1), then pass-2 projections h2 = V^T w
template <typename TV, int NV>
__global__ __launch_bounds__(RT) void update_dots_kernel(TV* __restrict__ V, size_t ld, int j, size_t n,
                                                         KState* ks, double* part) {
  if (ks->done) return;
  const int nvec = j + 1;
  __shared__ double hs[NV];
  for (int i = threadIdx.x; i < NV; i += RT) hs[i] = (i < nvec) ? ks->hcol[i] * ks->sigma[i] : 0.0;
  __syncthreads();
  TV* w = V + (size_t)(j + 1) * ld;
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
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
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] += (double)vr[i] * wq;
  }
  block_partials<NV>(acc, nvec, part);
  if (arrive_last(&ks->counter[2])) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int c = wid; c < nvec; c += RW) {
      double s = col_sum(part, c, gridDim.x);
      if (lane == 0) {
        ks->H[(size_t)j * KLD + c] = ks->hcol[c];   // pass-1 coefficient
        ks->hcol[c] = ks->sigma[c] * s;              // pass-2 coefficient
      }
    }
    if (threadIdx.x == 0) ks->counter[2] = 0u;
  }
}

// -------- w -= V (sigma .* h2); h_{j+1,j} = |w|; breakdown test; sigma_{j+1}
template <typename TV, int NV>
__global__ __launch_bounds__(RT) void update_norm_kernel(TV* __restrict__ V, size_t ld, int j, size_t n,
                                                         KState* ks, double* part) {
  if (ks->done) return;
  const int nvec = j + 1;
  __shared__ double hs[NV];
  for (int i = threadIdx.x; i < NV; i += RT) hs[i] = (i < nvec) ? ks->hcol[i] * ks->sigma[i] : 0.0;
  __syncthreads();
  TV* w = V + (size_t)(j + 1) * ld;
  double acc[1] = {0.0};
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
    acc[0] += wq * wq;
  }
  block_partials<1>(acc, 1, part);
  if (arrive_last(&ks->counter[3])) {
    if (threadIdx.x < 64) {
      double s = col_sum(part, 0, gridDim.x);
      if (threadIdx.x == 0) {
        for (int c = 0; c < nvec; ++c) ks->H[(size_t)j * KLD + c] += ks->hcol[c];
        double h = sqrt(s);
        ks->H[(size_t)j * KLD + j + 1] = h;
        ks->hlast = h;
        ks->m_eff = j + 1;
        if (!(h > ks->eta * ks->wnorm)) {
          ks->breakdown = 1;
          ks->done = 1;
        } else {
          ks->sigma[j + 1] = 1.0 / h;
        }
        ks->counter[3] = 0u;
      }
    }
  }
}

// Launch with the smallest vector-count bucket that holds j + 1 vectors.
#define PCEXP_GS_DISPATCH(KERNEL, ...)                                                          \
  do {                                                                                          \
    const int nv_ = j + 1;                                                                      \
    dim3 g_(gs_blocks(n)), b_(RT);                                                              \
    if (nv_ <= 4) hipLaunchKernelGGL((KERNEL<TV, 4>), g_, b_, 0, st, __VA_ARGS__);              \
    else if (nv_ <= 8) hipLaunchKernelGGL((KERNEL<TV, 8>), g_, b_, 0, st, __VA_ARGS__);         \
    else if (nv_ <= 12) hipLaunchKernelGGL((KERNEL<TV, 12>), g_, b_, 0, st, __VA_ARGS__);       \
    else if (nv_ <= 16) hipLaunchKernelGGL((KERNEL<TV, 16>), g_, b_, 0, st, __VA_ARGS__);       \
    else if (nv_ <= 20) hipLaunchKernelGGL((KERNEL<TV, 20>), g_, b_, 0, st, __VA_ARGS__);       \
    else if (nv_ <= 24) hipLaunchKernelGGL((KERNEL<TV, 24>), g_, b_, 0, st, __VA_ARGS__);       \
    else if (nv_ <= 28) hipLaunchKernelGGL((KERNEL<TV, 28>), g_, b_, 0, st, __VA_ARGS__);       \
    else if (nv_ <= 32) hipLaunchKernelGGL((KERNEL<TV, 32>), g_, b_, 0, st, __VA_ARGS__);       \
    else if (nv_ <= 40) hipLaunchKernelGGL((KERNEL<TV, 40>), g_, b_, 0, st, __VA_ARGS__);       \
    else if (nv_ <= 48) hipLaunchKernelGGL((KERNEL<TV, 48>), g_, b_, 0, st, __VA_ARGS__);       \
    else if (nv_ <= 56) hipLaunchKernelGGL((KERNEL<TV, 56>), g_, b_, 0, st, __VA_ARGS__);       \
    else hipLaunchKernelGGL((KERNEL<TV, 64>), g_, b_, 0, st, __VA_ARGS__);                      \
  } while (0)

template <typename TV>
void k_dots(const TV* V, size_t ld, int j, size_t n, KState* ks, double* part, hipStream_t st) {
  PCEXP_GS_DISPATCH(dots_kernel, V, ld, j, n, ks, part);
}
template <typename TV>
void k_update_dots(TV* V, size_t ld, int j, size_t n, KState* ks, double* part, hipStream_t st) {
  PCEXP_GS_DISPATCH(update_dots_kernel, V, ld, j, n, ks, part);
}
template <typename TV>
void k_update_norm(TV* V, size_t ld, int j, size_t n, KState* ks, double* part, hipStream_t st) {
  PCEXP_GS_DISPATCH(update_norm_kernel, V, ld, j, n, ks, part);
}

// ------------------------------------------------------------ Hessenberg phi
// y = beta * phi_k(dt H_m) e_1, m = m_eff, from the exponential of the
// augmented (m+k) x (m+k) matrix [[dt H, e_1, 0], [0, 0, I_{k-1}], [0, 0, 0]]
// (k = 0: exp(dt H) e_1).  exp by the degree-13 Pade approximant with scaling
// and squaring (Higham 2005).  One workgroup; matrices column-major in `mem`
// (LDS or global scratch), n <= KMAX + 3.
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

__device__ void phi_body(KState* ks, const double* dtp, int k, double* mem) {
  const int m = ks->m_eff;
  const int tid = threadIdx.x;
  if (m == 0) {
    for (int i = tid; i < KMAX + 4; i += PHI_T) ks->y[i] = 0.0;
    return;
  }
  const int n = (k >= 1) ? m + k : m;
  const int nn = n * n;
  double* A = mem;
  double* A2 = A + nn;
  double* A4 = A2 + nn;
  double* A6 = A4 + nn;
  double* T1 = A6 + nn;
  double* U = T1 + nn;
  double* Vm = U + nn;
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
    A[t] = v;
  }
  __syncthreads();
  // 1-norm and scaling
  __shared__ double colsum[KMAX + 4];
  __shared__ int s_sq;
  for (int jj = tid; jj < n; jj += PHI_T) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += fabs(A[jj * n + i]);
    colsum[jj] = s;
  }
  __syncthreads();
  if (tid == 0) {
    double nrm = 0.0;
    for (int jj = 0; jj < n; ++jj) nrm = fmax(nrm, colsum[jj]);
    const double theta13 = 5.371920351148152;
    int s = 0;
    if (nrm > theta13) s = (int)ceil(log2(nrm / theta13));
    if (s < 0) s = 0;
    s_sq = s;
  }
  __syncthreads();
  const int s = s_sq;
  const double sc = ldexp(1.0, -s);
  for (int t = tid; t < nn; t += PHI_T) A[t] *= sc;
  __syncthreads();
  const double b[14] = {64764752532480000.0, 32382376266240000.0, 7771770303897600.0,
                        1187353796428800.0, 129060195264000.0,  10559470521600.0,
                        670442572800.0,     33522128640.0,      1323241920.0,
                        40840800.0,         960960.0,           16380.0,
                        182.0,              1.0};
  mat_mul(A, A, A2, n);
  mat_mul(A2, A2, A4, n);
  mat_mul(A4, A2, A6, n);
  for (int t = tid; t < nn; t += PHI_T) T1[t] = b[13] * A6[t] + b[11] * A4[t] + b[9] * A2[t];
  __syncthreads();
  mat_mul(A6, T1, U, n);
  for (int t = tid; t < nn; t += PHI_T) {
    const int i = t % n, jj = t / n;
    T1[t] = U[t] + b[7] * A6[t] + b[5] * A4[t] + b[3] * A2[t] + (i == jj ? b[1] : 0.0);
  }
  __syncthreads();
  mat_mul(A, T1, U, n);  // U = A (A6 (b13 A6 + b11 A4 + b9 A2) + b7 A6 + b5 A4 + b3 A2 + b1 I)
  for (int t = tid; t < nn; t += PHI_T) T1[t] = b[12] * A6[t] + b[10] * A4[t] + b[8] * A2[t];
  __syncthreads();
  mat_mul(A6, T1, Vm, n);
  for (int t = tid; t < nn; t += PHI_T) {
    const int i = t % n, jj = t / n;
    const double v = Vm[t] + b[6] * A6[t] + b[4] * A4[t] + b[2] * A2[t] + (i == jj ? b[0] : 0.0);
    // P = V - U (in A2), Q = V + U (in A4)
    A2[t] = v - U[t];
    A4[t] = v + U[t];
  }
  __syncthreads();
  // Solve P X = Q by Gaussian elimination with partial pivoting (X in A4).
  double* P = A2;
  double* Q = A4;
  __shared__ int piv;
  for (int c = 0; c < n; ++c) {
    if (tid < 64) {
      // wave-parallel pivot search; ties go to the lowest row
      int best = n;
      double bv = -1.0;
      for (int r = c + tid; r < n; r += 64) {
        const double v = fabs(P[c * n + r]);
        if (v > bv) { bv = v; best = r; }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off, 64);
        const int ob = __shfl_xor(best, off, 64);
        if (ov > bv || (ov == bv && ob < best)) { bv = ov; best = ob; }
      }
      if (tid == 0) piv = best;
    }
    __syncthreads();
    const int pr = piv;
    if (pr != c) {
      for (int jj = tid; jj < n; jj += PHI_T) {
        double t1 = P[jj * n + c]; P[jj * n + c] = P[jj * n + pr]; P[jj * n + pr] = t1;
        double t2 = Q[jj * n + c]; Q[jj * n + c] = Q[jj * n + pr]; Q[jj * n + pr] = t2;
      }
    }
    __syncthreads();
    const double inv = 1.0 / P[c * n + c];
    const int rem = n - c - 1;
    // eliminate rows r > c: columns > c of P and all columns of Q
    for (int t = tid; t < rem * (n - c - 1 + n); t += PHI_T) {
      const int r = c + 1 + t % rem;
      const int cc = t / rem;  // 0..(n-c-2) -> P column c+1+cc ; then Q columns
      const double l = P[c * n + r] * inv;
      if (cc < n - c - 1) {
        const int col = c + 1 + cc;
        P[col * n + r] -= l * P[col * n + c];
      } else {
        const int col = cc - (n - c - 1);
        Q[col * n + r] -= l * Q[col * n + c];
      }
    }
    __syncthreads();
  }
  for (int c = n - 1; c >= 0; --c) {
    const double inv = 1.0 / P[c * n + c];
    for (int jj = tid; jj < n; jj += PHI_T) Q[jj * n + c] *= inv;
    __syncthreads();
    for (int t = tid; t < c * n; t += PHI_T) {
      const int r = t % c, jj = t / c;
      Q[jj * n + r] -= P[c * n + r] * Q[jj * n + c];
    }
    __syncthreads();
  }
  // squaring: X <- X^2, s times (ping-pong between Q and T1)
  double* X = Q;
  double* Y = T1;
  for (int it = 0; it < s; ++it) {
    mat_mul(X, X, Y, n);
    double* t = X; X = Y; Y = t;
  }
  const int col = (k >= 1) ? n - 1 : 0;
  const double beta = ks->beta;
  for (int i = tid; i < KMAX + 4; i += PHI_T) ks->y[i] = (i < m) ? beta * X[col * n + i] : 0.0;
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

__global__ __launch_bounds__(RT) void sumsq_kernel(const double* __restrict__ x, size_t n, double* out, int mode,
                                                   double* part, unsigned* counter) {
  double acc[1] = {0.0};
  for (size_t i = (size_t)blockIdx.x * RT + threadIdx.x; i < n; i += (size_t)gridDim.x * RT) acc[0] += x[i] * x[i];
  block_partials<1>(acc, 1, part);
  if (arrive_last(counter)) {
    if (threadIdx.x < 64) {
      double s = col_sum(part, 0, gridDim.x);
      if (threadIdx.x == 0) {
        *out = mode ? sqrt(s) : s;
        *counter = 0u;
      }
    }
  }
}
void k_sumsq(const double* x, size_t n, double* out, int mode, double* part, unsigned* counter,
             hipStream_t st) {
  hipLaunchKernelGGL(sumsq_kernel, dim3(gs_blocks(n)), dim3(RT), 0, st, x, n, out, mode, part, counter);
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
