// Krylov / Arnoldi and utility kernels (see krylov_kernels.hpp).
#include "krylov_kernels.hpp"
#include "launch.hpp"
#include "wave_reduce.hpp"

#include <hip/hip_runtime.h>

#include <cmath>

namespace pcexp {

constexpr int RT = 512;          // threads per reduction block
constexpr int RW = RT / 64;      // waves per reduction block
constexpr int PLD = 512;         // partials are column-major: part[col * PLD + block]
#ifndef PCEXP_RED_BLOCKS
#define PCEXP_RED_BLOCKS 256
#endif
// One 8-wave block per compute unit: the fused Gram-Schmidt passes hold
// 2 NV + 3 FP64 accumulators per lane, so a second resident block per CU
// would only add a tail round.
constexpr int MAXB = PCEXP_RED_BLOCKS;
static_assert(MAXB <= PLD, "partials per column exceed the partial stride");

size_t gs_blocks(size_t n) {
  size_t b = (n + 2 * RT - 1) / (2 * RT);   // the Gram-Schmidt passes take two entries per lane
  if (b > (size_t)MAXB) b = MAXB;
  if (b < 1) b = 1;
  return b;
}

// Two consecutive entries per lane: one 16-byte (FP64) or 8-byte (FP32) load.
// With NTL the load carries the non-temporal hint, which raises the rate of
// a pass streaming many vectors far larger than the Infinity Cache (3D P2
// vortex, 133 MB per FP32 vector: reduction and update passes -10 % and
// -4 %); where the cache serves part of a pass the hint costs more than it
// gains, so the caller chooses it per pass by the bytes streamed.
template <typename T> struct Pair;
template <> struct Pair<double> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct Pair<float> { typedef float type __attribute__((ext_vector_type(2))); };
template <typename T, bool NTL>
__device__ __forceinline__ typename Pair<T>::type ld_pair(const T* base, size_t p) {
  const typename Pair<T>::type* q = reinterpret_cast<const typename Pair<T>::type*>(base) + p;
  if constexpr (NTL) return __builtin_nontemporal_load(q);
  else return *q;
}
template <typename T, bool NTL>
__device__ __forceinline__ T ld_one(const T* base, size_t p) {
  if constexpr (NTL) return __builtin_nontemporal_load(base + p);
  else return base[p];
}
template <typename T, bool NTL = false>
__device__ __forceinline__ void load_pair(const T* base, size_t p, size_t n, double& a, double& b) {
  const typename Pair<T>::type v = ld_pair<T, NTL>(base, p);
  a = (double)v[0];
  b = (2 * p + 1 < n) ? (double)v[1] : 0.0;   // the slot stride is even, so the load stays in the slot
}

// Stores of the update pass, with the non-temporal hint under NTL (3D P2
// vortex: update passes a further -2 %).
template <typename T, bool NTL>
__device__ __forceinline__ void store_pair(T* base, size_t p, size_t n, double a, double b) {
  if (2 * p + 1 < n) {
    typename Pair<T>::type v;
    v[0] = (T)a;
    v[1] = (T)b;
    typename Pair<T>::type* q = reinterpret_cast<typename Pair<T>::type*>(base) + p;
    if constexpr (NTL) __builtin_nontemporal_store(v, q);
    else *q = v;
  } else {
    if constexpr (NTL) __builtin_nontemporal_store((T)a, base + 2 * p);
    else base[2 * p] = (T)a;
  }
}
template <typename T, bool NTL>
__device__ __forceinline__ void store_one(T* base, size_t p, double a) {
  if constexpr (NTL) __builtin_nontemporal_store((T)a, base + p);
  else base[p] = (T)a;
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

// Fixed-order sums of columns [0, ncol) of part into col[] by a whole
// RT-thread block: 8 lanes per column, lane `sub` summing partials sub,
// sub + 8, ... in ascending order, then a butterfly over the 8 lanes.  The
// loads of one round (64 columns) are split from the adds so that a caller
// can issue them together with its other loads.  They are unconditional --
// column clamped to ncol - 1, slot < MAXB <= PLD, inside every partial
// buffer -- and slots at or past nblk are dropped by a select at the sum.
constexpr int CS_PER = MAXB / 8;
constexpr int CS_COLS = RT / 8;
// NR partials per lane (CS_PER covers MAXB blocks; NR = 1 covers the one
// partial per column that the fused reduction's column sums leave).
template <int NR = CS_PER>
__device__ __forceinline__ void col_sums_load(const double* part, int c0, int ncol, double (&x)[NR]) {
  const int c = c0 + (threadIdx.x >> 3), sub = threadIdx.x & 7;
  const int cc = c < ncol ? c : ncol - 1;
#pragma unroll
  for (int r = 0; r < NR; ++r) x[r] = part[(size_t)cc * PLD + sub + 8 * r];
}
template <int NR = CS_PER>
__device__ __forceinline__ void col_sums_finish(const double (&x)[NR], int c0, int ncol, int nblk, double* col) {
  const int c = c0 + (threadIdx.x >> 3), sub = threadIdx.x & 7;
  double a = 0.0;
#pragma unroll
  for (int r = 0; r < NR; ++r) a += (sub + 8 * r < nblk) ? x[r] : 0.0;
  a += __shfl_xor(a, 4, 64);
  a += __shfl_xor(a, 2, 64);
  a += __shfl_xor(a, 1, 64);
  if (c < ncol && sub == 0) col[c] = a;
}
template <int NR = CS_PER>
__device__ __forceinline__ void block_col_sums(const double* part, int ncol, int nblk, double* col) {
  for (int c0 = 0; c0 < ncol; c0 += CS_COLS) {
    double x[NR];
    col_sums_load<NR>(part, c0, ncol, x);
    col_sums_finish<NR>(x, c0, ncol, nblk, col);
  }
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
  for (int i = t; i < 2 * KLD; i += blockDim.x) ks->htent[i] = 0.0;
  for (int i = t; i < KMAX + 2; i += blockDim.x) {
    ks->sigma[i] = 0.0;
    ks->sig_t[i] = 0.0;
    ks->nu_t[i] = 0.0;
    ks->wn_t[i] = 0.0;
  }
  for (int i = t; i < KMAX + 4; i += blockDim.x) ks->y[i] = 0.0;
  if (t < 8) ks->counter[t] = 0u;
  if (t < 4) ks->norm_tmp[t] = 0.0;
  if (t == 0) {
    ks->beta = ks->hlast = ks->fd_eps = 0.0;
    ks->eta = eta;
    ks->m_eff = 0;
    ks->done = 0;
    ks->done_at = 0x7fffffff;
    ks->breakdown = 0;
  }
}

void k_init_state(KState* ks, double eta, hipStream_t st) {
  launch(init_state_kernel, dim3(1), dim3(256), 0, st, ks, eta);
}

// The partial buffer of an Arnoldi run holds 3 (KMAX + 2) columns of PLD:
// the fused pass writes at most 2 (KMAX - 1) + 3 of them.
static_assert(2 * (KMAX - 1) + 3 <= 3 * (KMAX + 2), "partial columns exceed the buffer");

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
  block_partials<1>(acc, 1, part);
}

__global__ __launch_bounds__(64) void start_finalize(KState* ks, const double* part, int nblk) {
  const double s = col_sum(part, 0, nblk);
  if (threadIdx.x == 0) {
    const double beta = sqrt(s);
    ks->beta = beta;
    if (beta > 0.0) {
      ks->sig_t[0] = 1.0 / beta;
    } else {
      ks->done = 1;
      ks->done_at = -1;
      ks->m_eff = 0;
    }
  }
}

template <typename TV>
void k_start(const double* b, TV* V0, size_t n, KState* ks, double* part, hipStream_t st) {
  const int nb = (int)gs_blocks(n);
  launch(start_kernel<TV>, dim3(nb), dim3(RT), 0, st, b, V0, n, part);
  launch(start_finalize, dim3(1), dim3(64), 0, st, ks, part, nb);
}

// Vector loads of the Gram-Schmidt kernels are unconditional: slots beyond
// the live vectors re-read the last live vector (an L1/L2 hit) and their
// results are discarded, so the compiler can keep all loads of an element in
// flight.
__device__ __forceinline__ int clampv(int i, int nq) { return i < nq ? i : (nq > 0 ? nq - 1 : 0); }

// Iteration j.  Final vectors q_i = sigma_i V_i (i < j) are orthonormal; slot j
// holds U, the once-orthogonalised next vector with tentative scale sigma_j
// (u = sigma_j U, |u| ~ 1); slot j+1 holds W = J u.
//   reduce:    V_i.U, V_i.W (i < j), U.U, U.W, W.W             (one pass, or
//              per tile in the DG tangent kernel that made W, whose
//              partials gs_colsum_kernel then sums)
//   finalize:  s = Q^T u, rho^2 = |u|^2 - |s|^2, q_j = (u - Q s)/rho;
//              column j-1 of H corrected by nu s and nu rho (nu = |U|
//              estimate of the previous iteration); J q_j = (W - J Q s)/rho
//              with J Q s from the Arnoldi relation of the finished columns;
//              h = [Q q_j]^T J q_j; next U' = J q_j - [Q q_j] h with
//              |U'|^2 = |J q_j|^2 - |h|^2 (Pythagoras, tentative)   (one block)
//   update:    V_j <- U - sum e_i V_i;  V_{j+1} <- W/rho - a U - sum b_i V_i
//              (one pass, both vectors from the same loads)
// Column j of H stays tentative until the next iteration (or the closing
// pass) adds nu' s'.
// Column sums over a wave use the butterfly of wave_reduce.hpp.
constexpr int pow2_ceil(int x) { return x <= 4 ? 4 : 2 * pow2_ceil((x + 1) / 2); }

// Largest number of basis vectors one reduction block handles; more live
// vectors are split over blockIdx.y (each chunk re-reads U and W).
constexpr int CHUNK = 32;

template <typename TV, int PW, bool NTL = false>
__device__ __forceinline__ void load_pw(const TV* base, size_t p, size_t n, double* x) {
  if (PW == 2) load_pair<TV, NTL>(base, p, n, x[0], x[1]);
  else x[0] = (double)ld_one<TV, NTL>(base, p);
}
// Unmasked variant for passes that write back what they read: past the end
// of the vector the second entry holds whatever the slot's padding holds,
// and store_pair never writes it.
template <typename TV, int PW, bool NTL = false>
__device__ __forceinline__ void load_pw_raw(const TV* base, size_t p, double* x) {
  if (PW == 2) {
    const typename Pair<TV>::type v = ld_pair<TV, NTL>(base, p);
    x[0] = (double)v[0];
    x[1] = (double)v[1];
  } else {
    x[0] = (double)ld_one<TV, NTL>(base, p);
  }
}

template <typename TV, int NV, int PW, bool CLOSE, bool NTL>
__global__ __launch_bounds__(RT) void dcgs_reduce(const TV* __restrict__ V, size_t ld, int j, size_t n,
                                                  const KState* ks, double* part) {
  if (ks->done) return;
  const int nq = j;                    // final vectors before U
  const int i0 = blockIdx.y * NV;      // this block's chunk of them
  const TV* U = V + (size_t)j * ld;
  const TV* W = V + (size_t)(j + 1) * ld;
  constexpr int NB = CLOSE ? NV : 2 * NV;   // V.U (and V.W) columns of the chunk
  constexpr int NP = pow2_ceil(NB);
  constexpr int NX = CLOSE ? 1 : 3;         // U.U (, U.W, W.W)
  static_assert(NP <= 64, "one butterfly column per lane at most");
  double acc[NP], ext[NX];
#pragma unroll
  for (int i = 0; i < NP; ++i) acc[i] = 0.0;
#pragma unroll
  for (int i = 0; i < NX; ++i) ext[i] = 0.0;
  const size_t np = PW == 2 ? (n + 1) / 2 : n;
  for (size_t p = (size_t)blockIdx.x * RT + threadIdx.x; p < np; p += (size_t)gridDim.x * RT) {
    double u[PW], w[PW], v[NV][PW];
    load_pw<TV, PW, NTL>(U, p, n, u);
    if (!CLOSE) load_pw<TV, PW, NTL>(W, p, n, w);
#pragma unroll
    for (int i = 0; i < NV; ++i) load_pw<TV, PW, NTL>(V + (size_t)clampv(i0 + i, nq) * ld, p, n, v[i]);
#pragma unroll
    for (int k = 0; k < PW; ++k) {
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        acc[i] += v[i][k] * u[k];
        if (!CLOSE) acc[NV + i] += v[i][k] * w[k];
      }
      ext[0] += u[k] * u[k];
      if (!CLOSE) {
        ext[1] += u[k] * w[k];
        ext[2] += w[k] * w[k];
      }
    }
  }
  __shared__ double red[RW][NP + NX];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int col = 0;
  Bfly<NP / 2, 32>::run(acc, lane, col);
#pragma unroll
  for (int i = 0; i < NX; ++i) ext[i] = wave_sum(ext[i]);
  if ((lane & (64 / NP - 1)) == 0) red[wid][col] = acc[0];
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NX; ++i) red[wid][NP + i] = ext[i];
  }
  __syncthreads();
  // partial columns: [0, nq) V.U, then (not CLOSE) [nq, 2nq) V.W, then the extras
  for (int c = threadIdx.x; c < NB + NX; c += RT) {
    int g, src;
    bool live;
    if (c < NV) {
      g = i0 + c; live = g < nq; src = c;
    } else if (c < NB) {
      g = nq + i0 + (c - NV); live = i0 + (c - NV) < nq; src = c;
    } else {
      g = (CLOSE ? nq : 2 * nq) + (c - NB); live = blockIdx.y == 0; src = NP + (c - NB);
    }
    if (live) {
      double t = 0.0;
#pragma unroll
      for (int w2 = 0; w2 < RW; ++w2) t += red[w2][src];
      part[(size_t)g * PLD + blockIdx.x] = t;
    }
  }
}

// Finalise iteration j and rewrite V_j, V_{j+1} in one pass.  Slot j holds U
// (once-orthogonalised q_j with tentative scale sig_t[j], u = sig_t[j] U),
// slot j+1 holds W = J u; the partials hold V_i.U, V_i.W (i < j), U.U, U.W, W.W.
//   s = Q^T u, rho^2 = |u|^2 - |s|^2, q_j = (u - Q s)/rho; column j-1 of H
//   gets nu s and nu rho (nu = nu_t[j]); J q_j = (W - J Q s)/rho with J Q s
//   from the Arnoldi relation of the finished columns; h = [Q q_j]^T J q_j;
//   next U' = J q_j - [Q q_j] h, |U'|^2 = |J q_j|^2 - |h|^2 (tentative).
//   V_j <- U - sum e_i V_i;  V_{j+1} <- W/rho - a U - sum b_i V_i.
// Every block computes the same algebra (same inputs, same order); block 0
// publishes H, the scales and the stop flags, into locations no block of this
// launch reads.
template <typename TV, int NV, int PW, int CV, int NR, bool NTL>
__global__ __launch_bounds__(RT) void dcgs_fin_update(TV* __restrict__ V, size_t ld, int j, size_t n, KState* ks,
                                                      const double* part, int nblk) {
  if (ks->done_at < j) return;
  const int nq = j;
  const bool writer = blockIdx.x == 0;
  __shared__ double col[2 * KMAX + 3];
  __shared__ double s[KMAX], z[KMAX], g[KMAX], hc[KMAX];
  __shared__ double Hs[KMAX * KMAX];   // H[l][i], l, i < nq; column nq-1 tentative
  __shared__ double e[NV], b[NV];
  __shared__ double sa, sir;
  __shared__ int go;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  TV* U = V + (size_t)j * ld;
  TV* W = V + (size_t)(j + 1) * ld;
  const size_t np = PW == 2 ? (n + 1) / 2 : n;

  // Every global load the small algebra needs is issued first (partials,
  // H, the scales), then the loads of the first entries this thread will
  // update, so that their HBM latency overlaps the algebra: vector loads
  // complete in issue order, and waiting for the first group does not wait
  // for the second.
  constexpr bool ONE_ROUND = 2 * NV + 3 <= CS_COLS;
  constexpr bool PREFETCH = ONE_ROUND && CV == NV;
  constexpr int HQ = (NV * NV + RT - 1) / RT;
  const double* Ht = ks->htent + (size_t)((j + 1) & 1) * KLD;
  // (addresses are selected, not the loads, so no load sits under a branch)
  double hq[HQ];
#pragma unroll
  for (int q = 0; q < HQ; ++q) {
    const int t = tid + q * RT;
    const int i = t / (nq > 0 ? nq : 1), l = t - i * nq;   // column i, row l
    const double* src = t >= nq * nq ? ks->H : (i == nq - 1) ? Ht + l : ks->H + (size_t)i * KLD + l;
    hq[q] = *src;
  }
  const double sgv = ks->sigma[tid < nq ? tid : 0];   // used by threads tid < nq only
  const double sj = ks->sig_t[j];
  const double nu = ks->nu_t[j];
  const double wnj = ks->wn_t[j];
  const double eta = ks->eta;
  double px[NR];
  if (ONE_ROUND) col_sums_load<NR>(part, 0, 2 * nq + 3, px);

  // Loaded unconditionally (index clamped into the vector, n >= 1): a load
  // under a branch would make the wait for the partials wait for it as well.
  const size_t p0 = (size_t)blockIdx.x * RT + threadIdx.x;
  const size_t pc = p0 < np ? p0 : np - 1;
  double pv[PREFETCH ? NV : 1][PW], pu[PW], pw[PW];
  if (PREFETCH) {
    load_pw_raw<TV, PW, NTL>(U, pc, pu);
    load_pw_raw<TV, PW, NTL>(W, pc, pw);
#pragma unroll
    for (int i = 0; i < (PREFETCH ? NV : 1); ++i) load_pw_raw<TV, PW, NTL>(V + (size_t)clampv(i, nq) * ld, pc, pv[i]);
  }
  __builtin_amdgcn_sched_barrier(0);   // keep both groups of loads ahead of the first use

  if (ONE_ROUND) col_sums_finish<NR>(px, 0, 2 * nq + 3, nblk, col);
  else block_col_sums<NR>(part, 2 * nq + 3, nblk, col);
#pragma unroll
  for (int q = 0; q < HQ; ++q) {
    const int t = tid + q * RT;
    const int i = t / (nq > 0 ? nq : 1), l = t - i * nq;
    if (t < nq * nq) Hs[l * KMAX + i] = hq[q];
  }
  for (int i = nq + tid; i < NV; i += RT) {
    e[i] = 0.0;
    b[i] = 0.0;
  }
  __syncthreads();
  // s = Q^T u and z = Q^T W (scaled), the corrected column j-1 of H
  if (tid < nq) {
    const int l = tid;
    const double sl = sgv * sj * col[l];
    s[l] = sl;
    z[l] = sgv * col[nq + l];
    hc[l] = Hs[l * KMAX + (nq - 1)] + nu * sl;
  }
  __syncthreads();
  // g = H_{0:nq, 0:nq} s with the corrected last column (J Q s), 8 lanes per row
  {
    const int l = tid >> 3, sub = tid & 7;
    for (int l0 = 0; l0 < nq; l0 += RT / 8) {
      const int row = l0 + l;
      double a = 0.0;
      if (row < nq) {
        for (int i = (row > 0 ? row - 1 : 0) + sub; i < nq - 1; i += 8) a += Hs[row * KMAX + i] * s[i];
        if (sub == 0) a += hc[row] * s[nq - 1];
      }
      a += __shfl_xor(a, 4, 64);
      a += __shfl_xor(a, 2, 64);
      a += __shfl_xor(a, 1, 64);
      if (row < nq && sub == 0) g[row] = a;
    }
  }
  __syncthreads();
  if (wid == 0) {   // scalar reductions and the coefficients, lane l <-> row l
    double* H = ks->H;
    const bool live = lane < nq;
    const double sl = live ? s[lane] : 0.0;
    const double zl = live ? z[lane] : 0.0;
    const double gl = live ? g[lane] : 0.0;
    const double sgl = sgv;   // lane == tid in wave 0
    const double ss = wave_sum(sl * sl);
    const double gz = wave_sum(gl * zl), gg = wave_sum(gl * gl), sz = wave_sum(sl * zl);
    const double alpha = sj * sj * col[2 * nq];
    const double zeta = sj * col[2 * nq + 1];
    const double omega = col[2 * nq + 2];
    double rho = 1.0;
    bool stop = false;
    if (j > 0) {
      const double r2 = alpha - ss;
      rho = r2 > 0.0 ? sqrt(r2) : 0.0;
      const double hjj1 = nu * rho;
      stop = !(hjj1 > eta * wnj);   // v_j lies in the span: stop with m_eff = j
      if (writer) {
        if (live) H[(size_t)(j - 1) * KLD + lane] = hc[lane];
        if (lane == 0) {
          H[(size_t)(j - 1) * KLD + j] = hjj1;
          ks->hlast = hjj1;
          if (stop) {
            ks->breakdown = 1;
            ks->done = 1;
            ks->done_at = j;
            ks->m_eff = j;
          }
        }
      }
    }
    if (stop) {
      if (lane == 0) go = 0;
    } else {
      const double c = (j > 0) ? nu * rho * s[j - 1] : 0.0;
      const double ir = 1.0 / rho;
      const double qW = (zeta - sz) * ir;
      const double hl = live ? (zl - gl) * ir : 0.0;
      const double hj = (qW - c) * ir;
      const double hh = wave_sum(hl * hl) + hj * hj;
      const double jq2 = (omega - 2.0 * (gz + c * qW) + gg + c * c) * ir * ir;
      const double wn = sqrt(jq2 > 0.0 ? jq2 : 0.0);
      const double t = c * ir + hj;
      if (live) {
        e[lane] = sl * sgl / sj;
        b[lane] = sgl * (gl * ir + hl - t * sl * ir);
      }
      const double nu2 = jq2 - hh;
      const bool stop2 = !(nu2 > (eta * wn) * (eta * wn));   // J q_j lies in the span: m_eff = j + 1
      if (writer) {
        double* Hn = ks->htent + (size_t)(j & 1) * KLD;
        if (live) {
          H[(size_t)j * KLD + lane] = hl;
          Hn[lane] = hl;
        }
        if (lane == 0) {
          H[(size_t)j * KLD + j] = hj;
          Hn[j] = hj;
          ks->sigma[j] = sj * ir;
          ks->wn_t[j + 1] = wn;
          ks->m_eff = j + 1;
          if (stop2) {
            ks->breakdown = 1;
            ks->done = 1;
            ks->done_at = j;
            ks->hlast = nu2 > 0.0 ? sqrt(nu2) : 0.0;
            H[(size_t)j * KLD + j + 1] = ks->hlast;
          } else {
            const double nup = sqrt(nu2);
            ks->nu_t[j + 1] = nup;
            ks->sig_t[j + 1] = 1.0 / nup;
            H[(size_t)j * KLD + j + 1] = nup;   // tentative; corrected by the next iteration
          }
        }
      }
      if (lane == 0) {
        sa = t * sj * ir;
        sir = ir;
        go = 1;
      }
    }
  }
  __syncthreads();
  if (!go) return;
  const double a = sa, ir = sir;
  const size_t stride = (size_t)gridDim.x * RT;
  if (PREFETCH && p0 < np) {   // the first point, from the registers loaded before the algebra
    double un[PW], wn[PW];
#pragma unroll
    for (int k = 0; k < PW; ++k) {
      un[k] = pu[k];
      wn[k] = pw[k] * ir - a * pu[k];
    }
#pragma unroll
    for (int i = 0; i < (PREFETCH ? NV : 1); ++i) {
      const double ei = e[i], bi = b[i];
#pragma unroll
      for (int k = 0; k < PW; ++k) {
        un[k] -= ei * pv[i][k];
        wn[k] -= bi * pv[i][k];
      }
    }
    if (PW == 2) {
      store_pair<TV, NTL>(U, p0, n, un[0], un[1]);
      store_pair<TV, NTL>(W, p0, n, wn[0], wn[1]);
    } else {
      store_one<TV, NTL>(U, p0, un[0]);
      store_one<TV, NTL>(W, p0, wn[0]);
    }
  }
  for (size_t p = p0 + (PREFETCH ? stride : 0); p < np; p += stride) {
    double u[PW], w[PW], un[PW], wn[PW];
    load_pw_raw<TV, PW, NTL>(U, p, u);
    load_pw_raw<TV, PW, NTL>(W, p, w);
#pragma unroll
    for (int k = 0; k < PW; ++k) {
      un[k] = u[k];
      wn[k] = w[k] * ir - a * u[k];
    }
#pragma unroll 1
    for (int c0 = 0; c0 < NV; c0 += CV) {
      if (CV < NV && c0 >= nq) break;
      double v[CV][PW];
#pragma unroll
      for (int i = 0; i < CV; ++i) load_pw_raw<TV, PW, NTL>(V + (size_t)clampv(c0 + i, nq) * ld, p, v[i]);
#pragma unroll
      for (int i = 0; i < CV; ++i) {
        const double ei = e[c0 + i], bi = b[c0 + i];
#pragma unroll
        for (int k = 0; k < PW; ++k) {
          un[k] -= ei * v[i][k];
          wn[k] -= bi * v[i][k];
        }
      }
    }
    if (PW == 2) {
      store_pair<TV, NTL>(U, p, n, un[0], un[1]);
      store_pair<TV, NTL>(W, p, n, wn[0], wn[1]);
    } else {
      store_one<TV, NTL>(U, p, un[0]);
      store_one<TV, NTL>(W, p, wn[0]);
    }
  }
}

__global__ __launch_bounds__(RT) void dcgs_close_finalize(KState* ks, const double* part, int m, int nblk) {
  if (ks->done) return;
  __shared__ double col[KMAX + 1];
  block_col_sums(part, m + 1, nblk, col);
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double sm = ks->sig_t[m], nu = ks->nu_t[m];
  double ss = 0.0;
  for (int i = 0; i < m; ++i) {
    const double si = ks->sigma[i] * sm * col[i];
    ks->H[(size_t)(m - 1) * KLD + i] += nu * si;
    ss += si * si;
  }
  const double r2 = sm * sm * col[m] - ss;
  const double h = nu * (r2 > 0.0 ? sqrt(r2) : 0.0);
  ks->H[(size_t)(m - 1) * KLD + m] = h;
  ks->hlast = h;
}

// Blocks per vector chunk of the reduction (the partials per column).
static int red_blocks(size_t n, int nq) {
  const int nc = nq > CHUNK ? (nq + CHUNK - 1) / CHUNK : 1;
  const int b = (int)gs_blocks(n) / nc;
  return b > 0 ? b : 1;
}

// Smallest vector-count bucket that holds nq (>= 1) vectors; two entries per
// lane while the registers allow it.
template <typename TV, bool CLOSE, bool NTL>
static void launch_reduce(const TV* V, size_t ld, int j, size_t n, KState* ks, double* part, hipStream_t st) {
  const int nq = j > 0 ? j : 1;
  const dim3 b(RT);
  const unsigned nb = (unsigned)red_blocks(n, nq);
  if (nq <= 4) launch((dcgs_reduce<TV, 4, 2, CLOSE, NTL>), dim3(nb), b, 0, st, V, ld, j, n, ks, part);
  else if (nq <= 8) launch((dcgs_reduce<TV, 8, 2, CLOSE, NTL>), dim3(nb), b, 0, st, V, ld, j, n, ks, part);
  else if (nq <= 12) launch((dcgs_reduce<TV, 12, 2, CLOSE, NTL>), dim3(nb), b, 0, st, V, ld, j, n, ks, part);
  else if (nq <= 16) launch((dcgs_reduce<TV, 16, 2, CLOSE, NTL>), dim3(nb), b, 0, st, V, ld, j, n, ks, part);
  else if (nq <= 20) launch((dcgs_reduce<TV, 20, 2, CLOSE, NTL>), dim3(nb), b, 0, st, V, ld, j, n, ks, part);
  else if (nq <= 24) launch((dcgs_reduce<TV, 24, 2, CLOSE, NTL>), dim3(nb), b, 0, st, V, ld, j, n, ks, part);
  else if (nq <= 28) launch((dcgs_reduce<TV, 28, 2, CLOSE, NTL>), dim3(nb), b, 0, st, V, ld, j, n, ks, part);
  else {
    // the closing pass forms V.U only, so its registers hold two entries per lane
    const unsigned nc = (unsigned)((nq + CHUNK - 1) / CHUNK);
    launch((dcgs_reduce<TV, CHUNK, CLOSE ? 2 : 1, CLOSE, NTL>), dim3(nb, nc), b, 0, st, V, ld, j, n, ks, part);
  }
}

template <typename TV, int NR, bool NTL>
static void launch_update(TV* V, size_t ld, int j, size_t n, KState* ks, const double* part, int nb,
                          hipStream_t st) {
  const int nq = j > 0 ? j : 1;
  // Few vectors per point leave one 8-wave block per CU latency-bound; the
  // one-partial instances up to 12 vectors fit two blocks per CU (measured:
  // update passes 18.4 us against 18.9 us on average; three blocks for up to
  // 4 vectors gain nothing more).
  const unsigned mult = (NR == 1 && nq <= 12) ? 2u : 1u;
  const dim3 g(mult * (unsigned)gs_blocks(n)), b(RT);
  if (nq <= 4) launch((dcgs_fin_update<TV, 4, 2, 4, NR, NTL>), g, b, 0, st, V, ld, j, n, ks, part, nb);
  else if (nq <= 8) launch((dcgs_fin_update<TV, 8, 2, 8, NR, NTL>), g, b, 0, st, V, ld, j, n, ks, part, nb);
  else if (nq <= 12) launch((dcgs_fin_update<TV, 12, 2, 12, NR, NTL>), g, b, 0, st, V, ld, j, n, ks, part, nb);
  else if (nq <= 16) launch((dcgs_fin_update<TV, 16, 2, 16, NR, NTL>), g, b, 0, st, V, ld, j, n, ks, part, nb);
  else if (nq <= 20) launch((dcgs_fin_update<TV, 20, 2, 20, NR, NTL>), g, b, 0, st, V, ld, j, n, ks, part, nb);
  else if (nq <= 24) launch((dcgs_fin_update<TV, 24, 2, 24, NR, NTL>), g, b, 0, st, V, ld, j, n, ks, part, nb);
  else if (nq <= 28) {
    constexpr int PW = sizeof(TV) == 8 ? 2 : 1;   // FP32 pairs would spill here
    launch((dcgs_fin_update<TV, 28, PW, 28, NR, NTL>), g, b, 0, st, V, ld, j, n, ks, part, nb);
  }
  else if (nq <= 32) launch((dcgs_fin_update<TV, 32, 1, 32, NR, NTL>), g, b, 0, st, V, ld, j, n, ks, part, nb);
  else launch((dcgs_fin_update<TV, KMAX, 1, 16, NR, NTL>), g, b, 0, st, V, ld, j, n, ks, part, nb);
}

template <typename TV>
void k_gs_reduce(const TV* V, size_t ld, int j, size_t n, KState* ks, double* part, bool close, hipStream_t st,
                 bool nt) {
  if (nt) {
    if (close) launch_reduce<TV, true, true>(V, ld, j, n, ks, part, st);
    else launch_reduce<TV, false, true>(V, ld, j, n, ks, part, st);
  } else {
    if (close) launch_reduce<TV, true, false>(V, ld, j, n, ks, part, st);
    else launch_reduce<TV, false, false>(V, ld, j, n, ks, part, st);
  }
}

template <typename TV>
void k_gs_update(TV* V, size_t ld, int j, size_t n, KState* ks, const double* part, hipStream_t st, bool nt) {
  const int nb = red_blocks(n, j > 0 ? j : 1);
  if (nt) launch_update<TV, CS_PER, true>(V, ld, j, n, ks, part, nb, st);
  else launch_update<TV, CS_PER, false>(V, ld, j, n, ks, part, nb, st);
}

template <typename TV>
void k_gs_update_one(TV* V, size_t ld, int j, size_t n, KState* ks, const double* part, hipStream_t st,
                     bool nt) {
  if (nt) launch_update<TV, 1, true>(V, ld, j, n, ks, part, 1, st);
  else launch_update<TV, 1, false>(V, ld, j, n, ks, part, 1, st);
}

// Column c < ncol of fp (nblk partials at stride pld) summed in a fixed order
// (thread t takes partials t, t + 256, ..., then waves in order) into
// part[c * PLD]: the one partial per column that k_gs_update_one reads.
__global__ __launch_bounds__(256) void gs_colsum_kernel(const double* __restrict__ fp, int pld, int nblk,
                                                        const KState* ks, double* __restrict__ part) {
  if (ks->done) return;
  const int c = blockIdx.x;
  double a = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) a += fp[(size_t)c * pld + b];
  a = wave_sum(a);
  __shared__ double r[4];
  if ((threadIdx.x & 63) == 0) r[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) part[(size_t)c * PLD] = ((r[0] + r[1]) + r[2]) + r[3];
}

void k_gs_colsum(const double* fp, int pld, int nblk, int ncol, const KState* ks, double* part, hipStream_t st) {
  launch(gs_colsum_kernel, dim3(ncol), dim3(256), 0, st, fp, pld, nblk, ks, part);
}

void k_gs_close(KState* ks, const double* part, int m, size_t n, hipStream_t st) {
  launch(dcgs_close_finalize, dim3(1), dim3(RT), 0, st, ks, part, m, red_blocks(n, m > 0 ? m : 1));
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

// Small dense products on the matrix cores: C = A B (+ D), np x np column-major
// (np a multiple of 16), one 16 x 16 output tile per wave at a time,
// accumulated over k in steps of 4 by v_mfma_f64_16x16x4f64.  Lane l holds
// A(i, k) with i = l % 16, k = l / 16, B(k, j) with k = l / 16, j = l % 16,
// and result rows l / 16 + 4 r, r < 4, of column l % 16.
typedef double mfma_d4 __attribute__((ext_vector_type(4)));
// NS steps of 4 along k with every operand load issued before the first
// product (the same products in the same order as the run-time loop).
template <int NS>
__device__ __forceinline__ void mfma_chain(const double* a, const double* b, int ld, mfma_d4& acc) {
  double av[NS], bv[NS];
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    av[q] = a[(size_t)(4 * q) * ld];
    bv[q] = b[4 * q];
  }
#pragma unroll
  for (int q = 0; q < NS; ++q) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], bv[q], acc, 0, 0, 0);
}
__device__ void mat_mul_mfma(const double* A, const double* B, const double* D, double* C, int np, int ld) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nt = np >> 4;
  const int li = lane & 15, lk = lane >> 4;
  for (int tile = wid; tile < nt * nt; tile += PHI_T / 64) {
    const int ti = tile % nt, tj = tile / nt;
    mfma_d4 acc = {0.0, 0.0, 0.0, 0.0};
    const double* a = A + (size_t)lk * ld + ti * 16 + li;
    const double* b = B + (size_t)(tj * 16 + li) * ld + lk;
    // chunks of 32 along k (np is a multiple of 16): the loads of a chunk
    // are in flight together, the products keep the order of k
    int k0 = 0;
    for (; k0 + 32 <= np; k0 += 32) mfma_chain<8>(a + (size_t)k0 * ld, b + k0, ld, acc);
    if (k0 < np) mfma_chain<4>(a + (size_t)k0 * ld, b + k0, ld, acc);
    const int col = tj * 16 + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const size_t t = (size_t)col * ld + ti * 16 + lk + 4 * r;
      C[t] = D ? acc[r] + D[t] : acc[r];
    }
  }
  __syncthreads();
}

// exp(X) for the n x n matrix X = mem[0, n^2) (column-major, leading
// dimension n), n <= 2 KMAX + 2.  The matrix is zero-padded to np = pad16(n)
// (exp of [X 0; 0 0] is [exp(X) 0; 0 I]); mem holds 7 np^2 doubles.  Returns
// a pointer to the result inside mem, with leading dimension *ld = np.
__device__ double* expm_core(double* mem, int n, int* ld) {
  const int tid = threadIdx.x;
  const int np = pad16(n), lm = phi_ld(np);
  const int nn = np * lm;   // rows np .. lm-1 of every matrix are padding, never read by the products
  double* X = mem + (size_t)6 * nn;   // scaled, padded A (the input region is read first)
  double* X2 = mem;
  double* X3 = X2 + nn;
  double* X4 = X3 + nn;
  double* Bq = X4 + nn;     // current block polynomial
  double* T0 = Bq + nn;     // ping-pong accumulators
  double* T1 = T0 + nn;
  __shared__ double colsum[pad16(2 * KMAX + 2)];
  __shared__ int s_sq;
  for (int t = tid; t < nn; t += PHI_T) {
    const int i = t % lm, jj = t / lm;
    X[t] = (i < n && jj < n) ? mem[jj * n + i] : 0.0;
  }
  __syncthreads();
  for (int jj = tid; jj < np; jj += PHI_T) {
    double s = 0.0;
    for (int i = 0; i < np; ++i) s += fabs(X[jj * lm + i]);
    colsum[jj] = s;
  }
  __syncthreads();
  if (tid == 0) {
    double nrm = 0.0;
    for (int jj = 0; jj < np; ++jj) nrm = fmax(nrm, colsum[jj]);
    // an infinite norm (overflow in H or dt) gets the largest exponent a
    // finite one can have, so the squaring loop stays bounded
    int s = 0;
    if (nrm > 1.0) s = isfinite(nrm) ? (int)ceil(log2(nrm)) : 1024;
    s_sq = s;
  }
  __syncthreads();
  const int s = s_sq;
  const double sc = ldexp(1.0, -s);
  for (int t = tid; t < nn; t += PHI_T) X[t] *= sc;
  __syncthreads();
  mat_mul_mfma(X, X, nullptr, X2, np, lm);
  mat_mul_mfma(X2, X, nullptr, X3, np, lm);
  mat_mul_mfma(X2, X2, nullptr, X4, np, lm);
  // Taylor coefficients c_k = 1/k!, k = 0..18; blocks B_i = sum_{r<4} c_{4i+r} X^r,
  // T(X) = B_0 + X^4 (B_1 + X^4 (B_2 + X^4 (B_3 + X^4 B_4))), B_4 = c_16 + c_17 X + c_18 X^2
  double c[19];
  c[0] = 1.0;
  for (int q = 1; q < 19; ++q) c[q] = c[q - 1] / q;
  auto block = [&](int i, double* dst) {
    const double a0 = c[4 * i], a1 = (4 * i + 1 < 19) ? c[4 * i + 1] : 0.0;
    const double a2 = (4 * i + 2 < 19) ? c[4 * i + 2] : 0.0, a3 = (4 * i + 3 < 19) ? c[4 * i + 3] : 0.0;
    for (int t = tid; t < nn; t += PHI_T) {
      const int r = t % lm, jj = t / lm;
      dst[t] = a1 * X[t] + a2 * X2[t] + a3 * X3[t] + (r == jj ? a0 : 0.0);
    }
    __syncthreads();
  };
  block(4, T0);                          // T0 = B_4
  block(3, Bq);
  mat_mul_mfma(X4, T0, Bq, T1, np, lm);      // T1 = B_3 + X^4 B_4
  block(2, Bq);
  mat_mul_mfma(X4, T1, Bq, T0, np, lm);      // T0 = B_2 + X^4 T1
  block(1, Bq);
  mat_mul_mfma(X4, T0, Bq, T1, np, lm);      // T1 = B_1 + X^4 T0
  block(0, Bq);
  mat_mul_mfma(X4, T1, Bq, T0, np, lm);      // T0 = B_0 + X^4 T1 = T(X)
  double* P = T0;
  double* Q = T1;
  for (int it = 0; it < s; ++it) {
    mat_mul_mfma(P, P, nullptr, Q, np, lm);
    double* t = P; P = Q; Q = t;
  }
  *ld = lm;
  return P;
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
  double* X = mem;
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
  int ld;
  const double* P = expm_core(mem, n, &ld);
  const int col = (k >= 1) ? n - 1 : 0;
  const double beta = ks->beta;
  for (int i = tid; i < KMAX + 4; i += PHI_T) ks->y[i] = (i < m) ? beta * P[col * ld + i] : 0.0;
}

// Step-size control by the a-posteriori error of the Krylov approximation of
// phi_1 (Saad 1992): the leading error term of beta V_M phi_1(dt H_M) e_1 is
// beta dt h_{M+1,M} [phi_2(dt H_M) e_1]_M v_{M+1}, so
//   err(dt) = dt h_{M+1,M} |[phi_2(dt H_M) e_1]_M| / |phi_1(dt H_M) e_1|
// estimates the relative error.  Both phi's come from one exponential of the
// augmented matrix [[dt H, e_1, 0], [0, 0, 1], [0, 0, 0]] (size M + 2).  The
// Krylov basis does not depend on dt, so dt is halved (here, on the device)
// until err <= tol (at most 40 times); *dtp returns the accepted dt, y the
// corresponding beta phi_1(dt H_M) e_1.  norm_tmp[2] = err, norm_tmp[3] =
// number of halvings.
// Saad's a-posteriori estimate of the Krylov approximation of phi_1(dt J) b
// with dimension m: err = dt h_{m+1,m} |[phi_2(dt H_m) e_1]_m| / |phi_1(dt H_m) e_1|,
// both phi from the exponential of the augmented (m+2) x (m+2) matrix, which
// is left in *P with leading dimension *ldp (phi_1(dt H_m) e_1 is its column
// m, rows < m).  Every thread returns err.
__device__ double krylov_estimate(const KState* ks, double dt, int m, double hnext, double* mem, const double** P,
                                  int* ldp) {
  const int tid = threadIdx.x;
  __shared__ double red[PHI_T / 64];
  const int n = m + 2, nn = n * n;
  for (int t = tid; t < nn; t += PHI_T) {
    const int i = t % n, jj = t / n;
    double v = 0.0;
    if (i < m && jj < m) {
      if (i <= jj + 1) v = dt * ks->H[(size_t)jj * KLD + i];
    } else if (jj == m && i == 0) {
      v = 1.0;
    } else if (jj == m + 1 && i == m) {
      v = 1.0;
    }
    mem[t] = v;
  }
  __syncthreads();
  int ld;
  const double* Q = expm_core(mem, n, &ld);
  double sq = 0.0;
  for (int i = tid; i < m; i += PHI_T) {
    const double x = Q[(size_t)m * ld + i];
    sq += x * x;
  }
  sq = wave_sum(sq);
  if ((tid & 63) == 0) red[tid >> 6] = sq;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int w = 0; w < PHI_T / 64; ++w) t += red[w];
    const double phi2m = fabs(Q[(size_t)(m + 1) * ld + (m - 1)]);
    red[0] = t > 0.0 ? dt * hnext * phi2m / sqrt(t) : 0.0;
  }
  __syncthreads();
  const double err = red[0];
  __syncthreads();
  *P = Q;
  *ldp = ld;
  return err;
}

__device__ void phi_adapt_body(KState* ks, double* dtp, double tol, double* mem) {
  const int m = ks->m_eff;
  const int tid = threadIdx.x;
  if (m == 0) {
    for (int i = tid; i < KMAX + 4; i += PHI_T) ks->y[i] = 0.0;
    if (tid == 0) { ks->norm_tmp[2] = 0.0; ks->norm_tmp[3] = 0.0; }
    return;
  }
  const double hnext = ks->breakdown ? 0.0 : ks->hlast;
  double dt = *dtp;
  int halvings = 0;
  double err = 0.0;
  const double* P = nullptr;
  int ld = 0;
  for (;;) {
    err = krylov_estimate(ks, dt, m, hnext, mem, &P, &ld);
    if (err <= tol || halvings >= 40) break;
    dt *= 0.5;
    ++halvings;
  }
  const double beta = ks->beta;
  for (int i = tid; i < KMAX + 4; i += PHI_T) ks->y[i] = (i < m) ? beta * P[(size_t)m * ld + i] : 0.0;
  if (tid == 0) {
    *dtp = dt;
    ks->norm_tmp[2] = err;
    ks->norm_tmp[3] = (double)halvings;
  }
}

// Dimension check of an adaptive run, after the finalise-and-update pass of
// iteration j, when H_j and h_{j+1,j} are final and V_0..V_{j-1} complete:
// the estimate for dimension j at the current dt; at or below tol the run
// stops with m_eff = j (the later launches of the run see `done`, as after
// a breakdown, but the breakdown flag stays clear).
__device__ void krylov_check_body(KState* ks, const double* dtp, double tol, int j, double* mem) {
  if (ks->done) return;
  const double hnext = ks->H[(size_t)(j - 1) * KLD + j];
  const double* P = nullptr;
  int ld;
  const double err = krylov_estimate(ks, *dtp, j, hnext, mem, &P, &ld);
  if (threadIdx.x == 0 && err <= tol) {
    ks->m_eff = j;
    ks->hlast = hnext;
    ks->done_at = j;
    ks->done = 1;
    ks->norm_tmp[2] = err;
  }
}

__global__ __launch_bounds__(PHI_T) void krylov_check_lds(KState* ks, const double* dtp, double tol, int j) {
  extern __shared__ double smem[];
  krylov_check_body(ks, dtp, tol, j, smem);
}
__global__ __launch_bounds__(PHI_T) void krylov_check_glb(KState* ks, const double* dtp, double tol, int j,
                                                          double* mem) {
  krylov_check_body(ks, dtp, tol, j, mem);
}

void k_krylov_check(KState* ks, const double* dt, double tol, int j, double* scratch, hipStream_t st) {
  const int n = j + 2;
  const size_t bytes = phi_scratch_doubles(n) * sizeof(double);
  if (bytes <= 60 * 1024) launch(krylov_check_lds, dim3(1), dim3(PHI_T), bytes, st, ks, dt, tol, j);
  else launch(krylov_check_glb, dim3(1), dim3(PHI_T), 0, st, ks, dt, tol, j, scratch);
}

__global__ __launch_bounds__(PHI_T) void hess_phi_adapt_lds(KState* ks, double* dtp, double tol) {
  extern __shared__ double smem[];
  phi_adapt_body(ks, dtp, tol, smem);
}
__global__ __launch_bounds__(PHI_T) void hess_phi_adapt_glb(KState* ks, double* dtp, double tol, double* mem) {
  phi_adapt_body(ks, dtp, tol, mem);
}

void k_hess_phi_adapt(KState* ks, double* dt, double tol, int m, double* scratch, hipStream_t st) {
  const int n = m + 2;
  const size_t bytes = phi_scratch_doubles(n) * sizeof(double);
  if (bytes <= 60 * 1024) launch(hess_phi_adapt_lds, dim3(1), dim3(PHI_T), bytes, st, ks, dt, tol);
  else launch(hess_phi_adapt_glb, dim3(1), dim3(PHI_T), 0, st, ks, dt, tol, scratch);
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
  const size_t bytes = phi_scratch_doubles(n) * sizeof(double);
  if (bytes <= 60 * 1024) {
    launch(hess_phi_lds, dim3(1), dim3(PHI_T), bytes, st, ks, dt, k);
  } else {
    launch(hess_phi_glb, dim3(1), dim3(PHI_T), 0, st, ks, dt, k, scratch);
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
  launch((combine_kernel<TV, TX>), dim3(blocks), dim3(256), 0, st, V, ld, ks, base, out, xout,
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
  launch((fill_kernel<T>), dim3(blocks), dim3(256), 0, st, p, v, n, skip);
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
  launch((cast_kernel<TA, TB>), dim3(blocks), dim3(256), 0, st, a, b, n);
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
  launch(sumsq_kernel, dim3(nb), dim3(RT), 0, st, x, n, part);
  launch(sumsq_finalize, dim3(1), dim3(64), 0, st, part, nb, out, mode);
}

__global__ void fd_eps_kernel(const double* unorm, const double* vnorm, double c0, double* eps) {
  double e = c0 * (1.0 + *unorm);
  if (vnorm) e /= *vnorm;
  *eps = e;
}
void k_fd_eps(const double* unorm, const double* vnorm, double c0, double* eps, hipStream_t st) {
  launch(fd_eps_kernel, dim3(1), dim3(1), 0, st, unorm, vnorm, c0, eps);
}

template <typename TC>
__global__ void glue_kernel(const double* a, const double* b, const TC* c, double* out, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = a[i] - b[i] - (c ? (double)c[i] : 0.0);
}
template <typename TC>
void k_glue_d(const double* a, const double* b, const TC* c, double* out, size_t n, hipStream_t st) {
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  launch((glue_kernel<TC>), dim3(blocks), dim3(256), 0, st, a, b, c, out, n);
}

__global__ void set_scalar_kernel(double* p, double v) { *p = v; }
void k_set_scalar(double* p, double v, hipStream_t st) {
  launch(set_scalar_kernel, dim3(1), dim3(1), 0, st, p, v);
}

__global__ void add_scalar_kernel(double* acc, const double* x) { *acc += *x; }
void k_add_scalar(double* acc, const double* x, hipStream_t st) {
  launch(add_scalar_kernel, dim3(1), dim3(1), 0, st, acc, x);
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
  launch((gemv_kernel<T>), dim3((n + 3) / 4), dim3(256), 0, st, A, v, out, n, vscale, skip);
}

// explicit instantiations
// ================================================================ reverse mode
// Kernels of the reverse sweep through one Arnoldi run (FP64 basis).  The
// basis vectors are v_i = sigma_i V_i; adjoint vectors are plain.

// Vectors per group of the read-modify-write passes over the adjoint basis.
constexpr int RK = 8;

// Partial dot products of x with sigma_i V_i, i in [i0, i0 + nvec): blockIdx.y
// selects a chunk of NV vectors (NV the smallest bucket of 4, 8, .., 32 that
// holds nvec, or 32 chunks beyond); column c of the partials is vector
// i0 + c.  Slots past the last vector re-read it (a cache hit) and are
// dropped, so that every load of a point is in flight together.
constexpr int RV_CHUNK = 32;

template <int NV>
__global__ __launch_bounds__(RT) void rv_dots_kernel(const double* __restrict__ V, size_t ld, int i0, int nvec,
                                                     const double* __restrict__ x, size_t n, double* part) {
  constexpr int NP = pow2_ceil(NV);
  const int c0 = blockIdx.y * NV;
  double acc[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) acc[i] = 0.0;
  const size_t np = (n + 1) / 2;
  for (size_t p = (size_t)blockIdx.x * RT + threadIdx.x; p < np; p += (size_t)gridDim.x * RT) {
    double x0, x1, v[NV][2];
    load_pair(x, p, n, x0, x1);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int c = c0 + i < nvec ? c0 + i : nvec - 1;
      load_pair(V + (size_t)(i0 + c) * ld, p, n, v[i][0], v[i][1]);
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] += v[i][0] * x0 + v[i][1] * x1;
  }
  __shared__ double red[RW][NP];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int col = 0;
  Bfly<NP / 2, 32>::run(acc, lane, col);
  if ((lane & (64 / NP - 1)) == 0) red[wid][col] = acc[0];
  __syncthreads();
  for (int c = threadIdx.x; c < NV; c += RT) {
    if (c0 + c < nvec) {
      double t = 0.0;
#pragma unroll
      for (int w2 = 0; w2 < RW; ++w2) t += red[w2][c];
      part[(size_t)(c0 + c) * PLD + blockIdx.x] = t;
    }
  }
}

// out[c] = scale_c * sum of column c, scale_c = sigma[i0 + c] (or 1).
__global__ __launch_bounds__(RT) void rv_dots_finalize(const double* part, int nvec, int nblk, const double* sigma,
                                                       int i0, double* out) {
  __shared__ double col[KMAX + 2];
  block_col_sums(part, nvec, nblk, col);
  __syncthreads();
  for (int c = threadIdx.x; c < nvec; c += RT) out[c] = (sigma ? sigma[i0 + c] : 1.0) * col[c];
}

// The partials of k_rv_dots; returns the blocks per chunk (partials per column).
static int rv_dots_partials(const double* V, size_t ld, int i0, int nvec, const double* x, size_t n, double* part,
                            hipStream_t st) {
  const unsigned nc = (unsigned)((nvec + RV_CHUNK - 1) / RV_CHUNK);
  int nb = (int)gs_blocks(n) / (int)nc;
  if (nb < 1) nb = 1;
  const dim3 g((unsigned)nb, nc), b(RT);
  if (nvec <= 4) launch(rv_dots_kernel<4>, g, b, 0, st, V, ld, i0, nvec, x, n, part);
  else if (nvec <= 8) launch(rv_dots_kernel<8>, g, b, 0, st, V, ld, i0, nvec, x, n, part);
  else if (nvec <= 12) launch(rv_dots_kernel<12>, g, b, 0, st, V, ld, i0, nvec, x, n, part);
  else if (nvec <= 16) launch(rv_dots_kernel<16>, g, b, 0, st, V, ld, i0, nvec, x, n, part);
  else if (nvec <= 20) launch(rv_dots_kernel<20>, g, b, 0, st, V, ld, i0, nvec, x, n, part);
  else if (nvec <= 24) launch(rv_dots_kernel<24>, g, b, 0, st, V, ld, i0, nvec, x, n, part);
  else if (nvec <= 28) launch(rv_dots_kernel<28>, g, b, 0, st, V, ld, i0, nvec, x, n, part);
  else launch(rv_dots_kernel<RV_CHUNK>, g, b, 0, st, V, ld, i0, nvec, x, n, part);
  return nb;
}

void k_rv_dots(const double* V, size_t ld, const double* sigma, int i0, int nvec, const double* x, size_t n,
               double* part, double* out, hipStream_t st) {
  if (nvec <= 0) return;
  const int nb = rv_dots_partials(V, ld, i0, nvec, x, n, part, st);
  launch(rv_dots_finalize, dim3(1), dim3(RT), 0, st, (const double*)part, nvec, nb, sigma, i0, out);
}

// out = ax * x + ay * y + sum_{i < nvec} coef[i] sigma[i0 + i] V_{i0 + i}; ax, ay
// are device scalars when the pointers are given, else the constants.
__global__ __launch_bounds__(256) void rv_combine_kernel(RvComb a, double* out, size_t n) {
  __shared__ double cf[KMAX + 2];
  __shared__ double sx, sy;
  for (int i = threadIdx.x; i < a.nvec; i += blockDim.x)
    cf[i] = a.coef[i] * (a.sigma ? a.sigma[a.i0 + i] : 1.0);
  if (threadIdx.x == 0) {
    sx = a.axp ? *a.axp : a.axc;
    sy = a.ayp ? *a.ayp : a.ayc;
  }
  __syncthreads();
  const double ax = sx, ay = sy;
  const int nv = a.nvec;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x) {
    double r = 0.0;
    if (a.x) r += ax * a.x[idx];
    if (a.y) r += ay * a.y[idx];
    const double* Vp = a.V + (size_t)a.i0 * a.ld + idx;
    int i = 0;
    for (; i + 4 <= nv; i += 4) {
      const double v0 = Vp[(size_t)i * a.ld], v1 = Vp[(size_t)(i + 1) * a.ld];
      const double v2 = Vp[(size_t)(i + 2) * a.ld], v3 = Vp[(size_t)(i + 3) * a.ld];
      r += cf[i] * v0 + cf[i + 1] * v1 + cf[i + 2] * v2 + cf[i + 3] * v3;
    }
    for (; i < nv; ++i) r += cf[i] * Vp[(size_t)i * a.ld];
    out[idx] = r;
  }
}

void k_rv_combine(const RvComb& a, double* out, size_t n, hipStream_t st) {
  size_t blocks = (n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  launch(rv_combine_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a, out, n);
}

// Iteration j < M - 1 in one pass over V_0 .. V_{j+1}, v_{j+1}_bar and the
// adjoint basis Vb_0 .. Vb_j (coefficients from k_rv_dots_coef):
//   r = alpha v_{j+1}_bar + gamma v_{j+1},  wb = r + sum_{i<=j} b_i v_i,
//   wj = sum_{i<=j+1} c_i v_i  (J v_j by the Arnoldi relation; v_i = sigma_i V_i),
//   Vb_i += a_i r + b_i wj  (i <= j);
// r and wj stay in registers, only wb is written.
__global__ __launch_bounds__(256) void rv_iter_kernel(const double* __restrict__ vb1, const RState* rs,
                                                      const double* __restrict__ V, size_t ld, const double* sigma,
                                                      int j, double* __restrict__ Vb, double* __restrict__ wb_out,
                                                      size_t n) {
  __shared__ double f1[KMAX + 2], f2[KMAX + 2], ra[KMAX + 2], rb[KMAX + 2];
  __shared__ double sa, sg, sc;
  const int nv = j + 1;
  for (int i = threadIdx.x; i < nv; i += blockDim.x) {
    const double s = sigma ? sigma[i] : 1.0;
    f1[i] = rs->b[i] * s;
    f2[i] = rs->c[i] * s;
    ra[i] = rs->a[i];
    rb[i] = rs->b[i];
  }
  if (threadIdx.x == 0) {
    const double s = sigma ? sigma[j + 1] : 1.0;
    sa = rs->alpha;
    sg = rs->gamma * s;
    sc = rs->c[j + 1] * s;
  }
  __syncthreads();
  const double al = sa, ga = sg, cj = sc;
  const double* Vj1 = V + (size_t)(j + 1) * ld;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x) {
    const double v1 = Vj1[idx];
    const double r = al * vb1[idx] + ga * v1;
    double r1 = r, r2 = cj * v1;
    const double* Vp = V + idx;
    int i = 0;
    for (; i + 4 <= nv; i += 4) {
      const double v0 = Vp[(size_t)i * ld], va = Vp[(size_t)(i + 1) * ld];
      const double vb = Vp[(size_t)(i + 2) * ld], vc = Vp[(size_t)(i + 3) * ld];
      r1 += f1[i] * v0 + f1[i + 1] * va + f1[i + 2] * vb + f1[i + 3] * vc;
      r2 += f2[i] * v0 + f2[i + 1] * va + f2[i + 2] * vb + f2[i + 3] * vc;
    }
    for (; i < nv; ++i) {
      const double v = Vp[(size_t)i * ld];
      r1 += f1[i] * v;
      r2 += f2[i] * v;
    }
    wb_out[idx] = r1;
    // the rank update, reads of a group of RK before its writes
    for (int g0 = 0; g0 < nv; g0 += RK) {
      double* p = Vb + (size_t)g0 * ld + idx;
      double old[RK];
#pragma unroll
      for (int k = 0; k < RK; ++k) old[k] = g0 + k < nv ? p[(size_t)k * ld] : 0.0;
#pragma unroll
      for (int k = 0; k < RK; ++k)
        if (g0 + k < nv) p[(size_t)k * ld] = old[k] + (ra[g0 + k] * r + rb[g0 + k] * r2);
    }
  }
}

void k_rv_iter(const double* vb1, const RState* rs, const double* V, size_t ld, const double* sigma, int j,
               double* Vb, double* wb, size_t n, hipStream_t st) {
  size_t blocks = (n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  launch(rv_iter_kernel, dim3((unsigned)blocks), dim3(256), 0, st, vb1, rs, V, ld, sigma, j, Vb, wb, n);
}

// o1 += y1 and o2 += (*s2) y2 in one pass.
__global__ __launch_bounds__(256) void rv_acc2_kernel(double* o1, const double* y1, double* o2, const double* y2,
                                                      const double* s2, size_t n) {
  const double s = *s2;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x) {
    o1[idx] = o1[idx] + y1[idx];
    o2[idx] = o2[idx] + s * y2[idx];
  }
}

void k_rv_acc2(double* o1, const double* y1, double* o2, const double* y2, const double* s2, size_t n,
               hipStream_t st) {
  size_t blocks = (n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  launch(rv_acc2_kernel, dim3((unsigned)blocks), dim3(256), 0, st, o1, y1, o2, y2, s2, n);
}

// Vb_i (=|+=) a[i] r + b[i] w for i < nvec (r or w may be null).  The
// vectors go in groups of RK: the reads of a group are issued before its
// writes (the compiler cannot reorder them through the run-time stride), so
// each lane has RK loads in flight at a small register cost.
__global__ __launch_bounds__(256) void rv_rank_kernel(double* __restrict__ Vb, size_t ld, int nvec,
                                                      const double* __restrict__ r, const double* __restrict__ w,
                                                      const double* ca, const double* cb, int set, size_t n) {
  __shared__ double sa[KMAX + 2], sb[KMAX + 2];
  for (int i = threadIdx.x; i < nvec; i += blockDim.x) {
    sa[i] = ca ? ca[i] : 0.0;
    sb[i] = cb ? cb[i] : 0.0;
  }
  __syncthreads();
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x) {
    const double rr = r ? r[idx] : 0.0, ww = w ? w[idx] : 0.0;
    for (int g0 = 0; g0 < nvec; g0 += RK) {
      double* p = Vb + (size_t)g0 * ld + idx;
      double old[RK];
#pragma unroll
      for (int i = 0; i < RK; ++i) old[i] = (!set && g0 + i < nvec) ? p[(size_t)i * ld] : 0.0;
#pragma unroll
      for (int i = 0; i < RK; ++i)
        if (g0 + i < nvec) p[(size_t)i * ld] = old[i] + (sa[g0 + i] * rr + sb[g0 + i] * ww);
    }
  }
}

void k_rv_rank(double* Vb, size_t ld, int nvec, const double* r, const double* w, const double* a, const double* b,
               bool set, size_t n, hipStream_t st) {
  if (nvec <= 0) return;
  size_t blocks = (n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  launch(rv_rank_kernel, dim3((unsigned)blocks), dim3(256), 0, st, Vb, ld, nvec, r, w, a, b, set ? 1 : 0, n);
}

// ---- one-block algebra of the reverse sweep
// a[i] = fac dt y_i (i < M): initial adjoints of the basis, v_i_bar = a_i x_bar.
__global__ void rv_init_kernel(const KState* ks, RState* rs, double fac, const double* dtp) {
  const double f = fac * *dtp;
  const int M = ks->m_eff;
  for (int i = threadIdx.x; i < KMAX + 2; i += blockDim.x) rs->a[i] = i < M ? f * ks->y[i] : 0.0;
}

// y_bar = fac dt V^T x_bar (dots given), then the adjoint of
// y = beta [exp(A^)]_{0:M, M}, A^ = [[dt H_M, e_1], [0, 0]]:
//   beta_bar = y_bar . y / beta,  z_bar = beta y_bar,
//   H_bar = dt [L(A^T, Z)]_{0:M, 0:M},  Z = [z_bar; 0] e_M^T,
// with the Frechet derivative L(X, E) = upper-right block of exp([[X, E], [0, X]]).
__global__ __launch_bounds__(PHI_T) void rv_phi_adjoint_kernel(const KState* ks, RState* rs, const double* dots,
                                                               double fac, const double* dtp, double* mem) {
  const int M = ks->m_eff;
  const int tid = threadIdx.x;
  const double dt = *dtp;
  const double beta = ks->beta;
  __shared__ double yb[KMAX + 2];
  for (int i = tid; i < KMAX + 2; i += PHI_T) yb[i] = i < M ? fac * dt * dots[i] : 0.0;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int i = 0; i < M; ++i) t += yb[i] * ks->y[i];
    rs->betabar = beta > 0.0 ? t / beta : 0.0;
  }
  for (int t = tid; t < KLD * KMAX; t += PHI_T) rs->Hbar[t] = 0.0;
  if (M == 0) return;
  const int n1 = M + 1, n = 2 * n1, nn = n * n;
  double* X = mem;
  for (int t = tid; t < nn; t += PHI_T) {
    const int i = t % n, jj = t / n;    // row i, column jj
    double v = 0.0;
    const bool top = i < n1, left = jj < n1;
    if (top == left || (top && !left)) {
      if (top && !left) {                 // Z block: column M of the upper-right block
        if (jj - n1 == M && i < M) v = beta * yb[i];
      } else {                            // A^T blocks on the diagonal
        const int r = top ? i : i - n1, cc = top ? jj : jj - n1;
        // A^T[r][cc] = A^[cc][r]
        if (cc < M && r < M) {
          if (cc <= r + 1) v = dt * ks->H[(size_t)r * KLD + cc];
        } else if (r == M && cc == 0) {
          v = 1.0;
        }
      }
    }
    X[t] = v;
  }
  __syncthreads();
  int ld;
  const double* P = expm_core(mem, n, &ld);
  for (int t = tid; t < M * M; t += PHI_T) {
    const int i = t % M, jj = t / M;
    if (i <= jj + 1) rs->Hbar[(size_t)jj * KLD + i] = dt * P[(size_t)(n1 + jj) * ld + i];
  }
}

// Iteration j: with c_i = v_i . r_bar (or 0), h_bar_i = H_bar_{i,j} - c_i;
//   b[i] = h_bar_i, a[i] = -h_{i,j} (i <= j); c[i] = h_{i,j} (i <= j + 1).
__global__ void rv_coef_w_kernel(const KState* ks, RState* rs, int j, const double* cdots) {
  for (int i = threadIdx.x; i < KMAX + 2; i += blockDim.x) {
    const bool in = i <= j;
    const double hij = (i <= j + 1 && i < KLD) ? ks->H[(size_t)j * KLD + i] : 0.0;
    rs->b[i] = in ? rs->Hbar[(size_t)j * KLD + i] - (cdots ? cdots[i] : 0.0) : 0.0;
    rs->a[i] = in ? -hij : 0.0;
    rs->c[i] = (i <= j + 1) ? hij : 0.0;
  }
}

// Iteration j < M - 1, from the partials of d_i = v_i . v_{j+1}_bar
// (i <= j + 1; column sums in a fixed order, as rv_dots_finalize):
//   r_bar = alpha v_{j+1}_bar + gamma v_{j+1},  alpha = 1 / h,
//   gamma = H_bar_{j+1,j} - d_{j+1} / h,  h = h_{j+1,j};
//   c_i = v_i . r_bar = alpha d_i (i <= j: the basis is orthonormal, the
//   reading under which the sweep differentiates the Arnoldi relations);
//   b[i] = H_bar_{i,j} - c_i, a[i] = -h_{i,j} (i <= j); c[i] = h_{i,j} (i <= j + 1).
__global__ __launch_bounds__(RT) void rv_coef_rw_kernel(const double* part, int nblk, const double* sigma,
                                                        const KState* ks, RState* rs, int j) {
  __shared__ double col[KMAX + 2];
  block_col_sums(part, j + 2, nblk, col);
  __syncthreads();
  const double h = ks->H[(size_t)j * KLD + j + 1];
  const double al = 1.0 / h;
  if (threadIdx.x == 0) {
    const double dj1 = (sigma ? sigma[j + 1] : 1.0) * col[j + 1];
    rs->alpha = al;
    rs->gamma = rs->Hbar[(size_t)j * KLD + j + 1] - dj1 / h;
  }
  for (int i = threadIdx.x; i < KMAX + 2; i += RT) {
    const bool in = i <= j;
    const double hij = (i <= j + 1 && i < KLD) ? ks->H[(size_t)j * KLD + i] : 0.0;
    const double di = in ? (sigma ? sigma[i] : 1.0) * col[i] : 0.0;
    rs->b[i] = in ? rs->Hbar[(size_t)j * KLD + i] - al * di : 0.0;
    rs->a[i] = in ? -hij : 0.0;
    rs->c[i] = (i <= j + 1) ? hij : 0.0;
  }
}

// b_bar = v_0_bar / beta + (beta_bar - t / beta) v_0, t = v_0_bar . v_0.
__global__ void rv_coef_b_kernel(const KState* ks, RState* rs, const double* tdot) {
  const double beta = ks->beta;
  rs->alpha = 1.0 / beta;
  rs->gamma = rs->betabar - *tdot / beta;
}

void k_rv_init(const KState* ks, RState* rs, double fac, const double* dtp, hipStream_t st) {
  launch(rv_init_kernel, dim3(1), dim3(64), 0, st, ks, rs, fac, dtp);
}
void k_rv_phi_adjoint(const KState* ks, RState* rs, const double* dots, double fac, const double* dtp, double* mem,
                      hipStream_t st) {
  launch(rv_phi_adjoint_kernel, dim3(1), dim3(PHI_T), 0, st, ks, rs, dots, fac, dtp, mem);
}
void k_rv_coef_w(const KState* ks, RState* rs, int j, const double* cdots, hipStream_t st) {
  launch(rv_coef_w_kernel, dim3(1), dim3(64), 0, st, ks, rs, j, cdots);
}
void k_rv_dots_coef(const double* V, size_t ld, const double* sigma, int j, const double* vb1, size_t n, double* part,
                    const KState* ks, RState* rs, hipStream_t st) {
  const int nb = rv_dots_partials(V, ld, 0, j + 2, vb1, n, part, st);
  launch(rv_coef_rw_kernel, dim3(1), dim3(RT), 0, st, (const double*)part, nb, sigma, ks, rs, j);
}
void k_rv_coef_b(const KState* ks, RState* rs, const double* tdot, hipStream_t st) {
  launch(rv_coef_b_kernel, dim3(1), dim3(1), 0, st, ks, rs, tdot);
}

// Dense test operator: out = A^T v (row-major A).
__global__ void gemv_t_kernel(const double* A, const double* v, double* out, int n) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += A[(size_t)i * n + j] * v[i];
    out[j] = s;
  }
}
void k_gemv_t(const double* A, const double* v, double* out, int n, hipStream_t st) {
  launch(gemv_t_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, A, v, out, n);
}

template void k_start<double>(const double*, double*, size_t, KState*, double*, hipStream_t);
template void k_start<float>(const double*, float*, size_t, KState*, double*, hipStream_t);
template void k_gs_reduce<double>(const double*, size_t, int, size_t, KState*, double*, bool, hipStream_t, bool);
template void k_gs_reduce<float>(const float*, size_t, int, size_t, KState*, double*, bool, hipStream_t, bool);
template void k_gs_update<double>(double*, size_t, int, size_t, KState*, const double*, hipStream_t, bool);
template void k_gs_update<float>(float*, size_t, int, size_t, KState*, const double*, hipStream_t, bool);
template void k_gs_update_one<double>(double*, size_t, int, size_t, KState*, const double*, hipStream_t, bool);
template void k_gs_update_one<float>(float*, size_t, int, size_t, KState*, const double*, hipStream_t, bool);
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
