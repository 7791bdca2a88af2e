// Element-level kernels at the ABI boundary: change of basis (paper basis,
// Sec. 4.3, <-> reference basis), quadrature points, L2 projection and
// evaluation (Sec. 4.2, mass = I), the time step of eq. (x3d) and conserved
// totals.  Sizes are run-time values; none of these is on the hot path.
#include <hip/hip_runtime.h>

#include "dg_dispatch.hpp"
#include "launch.hpp"

namespace pcexp {

constexpr int MAXNB = 20;
constexpr int EK_T = 256;

static dim3 grid_for(size_t n) {
  size_t b = (n + EK_T - 1) / EK_T;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}

__global__ void to_internal_kernel(ElemArgs a, const double* __restrict__ u_abi, double* __restrict__ u_int) {
  const size_t t = (size_t)blockIdx.x * EK_T + threadIdx.x;
  const int nb = a.nb, nv = a.nv;
  if (t >= (size_t)a.Epad * nv) return;
  const int e = (int)(t / nv), k = (int)(t % nv);
  if (e >= a.nE) {
    for (int i = 0; i < nb; ++i) u_int[(size_t)(k * nb + i) * a.Epad + e] = 0.0;
    return;
  }
  double x[MAXNB];
  for (int j = 0; j < nb; ++j) x[j] = u_abi[((size_t)e * nv + k) * nb + j];
  const double* Q = a.Q + (size_t)e * nb * nb;
  const int ie = a.perm[e];
  for (int i = 0; i < nb; ++i) {
    double s = 0.0;
    for (int j = 0; j < nb; ++j) s += Q[i * nb + j] * x[j];
    u_int[(size_t)(k * nb + i) * a.Epad + ie] = s;
  }
}

// u_abi = Q^T u_int, or u_abi += scale Q^T u_int when acc (the same rounding
// of Q^T u_int in both forms, then one multiply-add).
__global__ void to_abi_kernel(ElemArgs a, const double* __restrict__ u_int, double* __restrict__ u_abi, int acc,
                              double scale) {
  const size_t t = (size_t)blockIdx.x * EK_T + threadIdx.x;
  const int nb = a.nb, nv = a.nv;
  if (t >= (size_t)a.nE * nv) return;
  const int e = (int)(t / nv), k = (int)(t % nv);
  const int ie = a.perm[e];
  double x[MAXNB];
  for (int i = 0; i < nb; ++i) x[i] = u_int[(size_t)(k * nb + i) * a.Epad + ie];
  const double* Q = a.Q + (size_t)e * nb * nb;
  for (int j = 0; j < nb; ++j) {
    double s = 0.0;
    for (int i = 0; i < nb; ++i) s += Q[i * nb + j] * x[i];
    double* o = &u_abi[((size_t)e * nv + k) * nb + j];
    if (acc) *o = fma(scale, s, *o);
    else *o = s;
  }
}

__global__ void quad_points_kernel(ElemArgs a, double* xyz) {
  const size_t t = (size_t)blockIdx.x * EK_T + threadIdx.x;
  if (t >= (size_t)a.nE * a.nq) return;
  const int e = (int)(t / a.nq), q = (int)(t % a.nq);
  const int ie = a.perm[e], d = a.dim;
  for (int c = 0; c < d; ++c) {
    double x = a.x0[(size_t)c * a.Epad + ie];
    for (int j = 0; j < d; ++j) x += a.amat[(size_t)(c * d + j) * a.Epad + ie] * a.refp[q * d + j];
    xyz[t * d + c] = x;
  }
}

__global__ void project_kernel(ElemArgs a, const double* __restrict__ Uqp, double* __restrict__ u_abi) {
  const size_t t = (size_t)blockIdx.x * EK_T + threadIdx.x;
  const int nb = a.nb, nv = a.nv, nq = a.nq;
  if (t >= (size_t)a.nE * nv) return;
  const int e = (int)(t / nv), k = (int)(t % nv);
  const double s = a.sdet[a.perm[e]];
  double r[MAXNB];
  for (int i = 0; i < nb; ++i) r[i] = 0.0;
  for (int q = 0; q < nq; ++q) {
    const double U = Uqp[((size_t)e * nq + q) * nv + k] * a.wq[q] * s;
    for (int i = 0; i < nb; ++i) r[i] += U * a.B[q * nb + i];
  }
  const double* Q = a.Q + (size_t)e * nb * nb;
  for (int j = 0; j < nb; ++j) {
    double v = 0.0;
    for (int i = 0; i < nb; ++i) v += Q[i * nb + j] * r[i];
    u_abi[((size_t)e * nv + k) * nb + j] = v;
  }
}

__global__ void evaluate_kernel(ElemArgs a, const double* __restrict__ u_abi, double* __restrict__ Uqp) {
  const size_t t = (size_t)blockIdx.x * EK_T + threadIdx.x;
  const int nb = a.nb, nv = a.nv, nq = a.nq;
  if (t >= (size_t)a.nE * nv) return;
  const int e = (int)(t / nv), k = (int)(t % nv);
  const double rs = 1.0 / a.sdet[a.perm[e]];
  const double* Q = a.Q + (size_t)e * nb * nb;
  double r[MAXNB];
  for (int i = 0; i < nb; ++i) {
    double s = 0.0;
    for (int j = 0; j < nb; ++j) s += Q[i * nb + j] * u_abi[((size_t)e * nv + k) * nb + j];
    r[i] = s;
  }
  for (int q = 0; q < nq; ++q) {
    double U = 0.0;
    for (int i = 0; i < nb; ++i) U += r[i] * a.B[q * nb + i];
    Uqp[((size_t)e * nq + q) * nv + k] = U * rs;
  }
}

__device__ __forceinline__ double ek_wave_min(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ double ek_wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// dt = cfl * min_E h_E / ((2p+1)(|v| + c)), v and c at the centroid (eq. (x3d)).
// Per-block minima, then a one-block kernel takes the minimum (order-free).
__global__ void stable_dt_kernel(ElemArgs a, const double* __restrict__ u, double* part) {
  const int e = blockIdx.x * EK_T + threadIdx.x;
  const int nb = a.nb, d = a.dim;
  double lam = 1e300;
  if (e < a.nE) {
    double U[5];
    const double rs = 1.0 / a.sdet[e];
    for (int k = 0; k < d + 2; ++k) {
      double s = 0.0;
      for (int i = 0; i < nb; ++i) s += u[(size_t)(k * nb + i) * a.Epad + e] * a.Bc[i];
      U[k] = s * rs;
    }
    double q2 = 0.0;
    for (int c = 0; c < d; ++c) q2 += U[1 + c] * U[1 + c];
    const double rho = U[0];
    const double p = (a.gamma - 1.0) * (U[d + 1] - 0.5 * q2 / rho);
    const double speed = sqrt(q2) / rho + sqrt(a.gamma * p / rho);
    lam = a.hE[e] / ((2 * a.p + 1) * speed);
    if (!(lam > 0.0)) lam = -1.0;   // NaN or non-positive: propagate an invalid step
  }
  __shared__ double red[EK_T / 64];
  double m = ek_wave_min(lam);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mm = red[0];
    for (int w = 1; w < EK_T / 64; ++w) mm = fmin(mm, red[w]);
    part[blockIdx.x] = mm;
  }
}

__global__ void stable_dt_finalize(const double* part, int nblk, const double* cfl_dev, double cfl, double* dt) {
  double mm = 1e300;
  for (int b = threadIdx.x; b < nblk; b += 64) mm = fmin(mm, part[b]);
  mm = ek_wave_min(mm);
  if (threadIdx.x == 0) *dt = (cfl_dev ? *cfl_dev : cfl) * mm;
}

// Q_k = sum_E int_E U_k = sum_E s_E phi_hat_0 / d! * u_int[k][0][E]
__global__ void totals_kernel(ElemArgs a, const double* __restrict__ u, double* part) {
  const int e = blockIdx.x * EK_T + threadIdx.x;
  const int nv = a.nv;
  const double fact = (a.dim == 2) ? 0.5 : (1.0 / 6.0);
  __shared__ double red[EK_T / 64][5];
  for (int k = 0; k < nv; ++k) {
    double v = 0.0;
    if (e < a.nE) v = u[(size_t)(k * a.nb) * a.Epad + e] * a.sdet[e] * a.Bc[0] * fact;
    v = ek_wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < nv) {
    double s = 0.0;
    for (int w = 0; w < EK_T / 64; ++w) s += red[w][threadIdx.x];
    part[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = s;
  }
}

__global__ void totals_finalize(const double* part, int nblk, int nv, double* out) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int k = wid; k < nv; k += EK_T / 64) {
    double s = 0.0;
    for (int b = lane; b < nblk; b += 64) s += part[(size_t)k * nblk + b];
    s = ek_wave_sum(s);
    if (lane == 0) out[k] = s;
  }
}

// Pressure functional P(u) = int_Omega (p_h - p_ref)^2 dx by the volume rule,
// and its gradient with respect to the internal coefficients:
//   dP/du_{k,i,E} = sum_q w_q s_E 2 (p_q - p_ref) dp/dU_k(U_q) B_{q,i},
// U_q = sum_i u_{k,i,E} B_{q,i} / s_E, dx = s_E^2 dxi (s_E = sqrt(det A_E)).
// One thread per element; per-block partial sums of P (fixed order).
__global__ void pfun_kernel(ElemArgs a, const double* __restrict__ u, double p_ref, double* part, double* grad) {
  const int e = blockIdx.x * EK_T + threadIdx.x;
  const int nb = a.nb, nv = a.nv, d = a.dim;
  double val = 0.0;
  if (e < a.nE) {
    const double s = a.sdet[e], rs = 1.0 / s;
    const double gm1 = a.gamma - 1.0;
    double g[5 * MAXNB];
    for (int t = 0; t < nv * nb; ++t) g[t] = 0.0;
    for (int q = 0; q < a.nq; ++q) {
      double U[5];
      for (int k = 0; k < nv; ++k) {
        double x = 0.0;
        for (int i = 0; i < nb; ++i) x += u[(size_t)(k * nb + i) * a.Epad + e] * a.B[q * nb + i];
        U[k] = x * rs;
      }
      const double rho = U[0];
      double m2 = 0.0;
      for (int c = 0; c < d; ++c) m2 += U[1 + c] * U[1 + c];
      const double p = gm1 * (U[d + 1] - 0.5 * m2 / rho);
      const double dp = p - p_ref;
      val += a.wq[q] * s * s * dp * dp;
      // dp/dU: (gm1 |m|^2 / (2 rho^2), -gm1 m / rho, gm1)
      double dpdU[5];
      dpdU[0] = 0.5 * gm1 * m2 / (rho * rho);
      for (int c = 0; c < d; ++c) dpdU[1 + c] = -gm1 * U[1 + c] / rho;
      dpdU[d + 1] = gm1;
      const double f = a.wq[q] * s * 2.0 * dp;
      for (int k = 0; k < nv; ++k)
        for (int i = 0; i < nb; ++i) g[k * nb + i] += f * dpdU[k] * a.B[q * nb + i];
    }
    if (grad)
      for (int t = 0; t < nv * nb; ++t) grad[(size_t)t * a.Epad + e] = g[t];
  } else if (grad && e < a.Epad) {
    for (int t = 0; t < nv * nb; ++t) grad[(size_t)t * a.Epad + e] = 0.0;
  }
  __shared__ double red[EK_T / 64];
  const double wsum = ek_wave_sum(val);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = wsum;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < EK_T / 64; ++w) t += red[w];
    part[blockIdx.x] = t;
  }
}

// *out = P, or *out += scale P when acc.
__global__ void pfun_finalize(const double* part, int nblk, double* out, int acc, double scale) {
  double t = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) t += part[b];
  t = ek_wave_sum(t);
  if (threadIdx.x == 0) *out = acc ? fma(scale, t, *out) : t;
}

void ek_pressure_functional(const ElemArgs& a, const double* u_int, double p_ref, double* value, double* grad_int,
                            double* part, hipStream_t st, int acc, double scale) {
  const dim3 g = grid_for((size_t)a.Epad);
  launch(pfun_kernel, g, dim3(EK_T), 0, st, a, u_int, p_ref, part, grad_int);
  if (value) launch(pfun_finalize, dim3(1), dim3(64), 0, st, (const double*)part, (int)g.x, value, acc, scale);
}

void ek_to_internal(const ElemArgs& a, const double* u_abi, double* u_int, hipStream_t st) {
  launch(to_internal_kernel, grid_for((size_t)a.Epad * a.nv), dim3(EK_T), 0, st, a, u_abi, u_int);
}
void ek_to_abi(const ElemArgs& a, const double* u_int, double* u_abi, hipStream_t st) {
  launch(to_abi_kernel, grid_for((size_t)a.nE * a.nv), dim3(EK_T), 0, st, a, u_int, u_abi, 0, 0.0);
}
void ek_to_abi_axpy(const ElemArgs& a, const double* u_int, double scale, double* u_abi, hipStream_t st) {
  launch(to_abi_kernel, grid_for((size_t)a.nE * a.nv), dim3(EK_T), 0, st, a, u_int, u_abi, 1, scale);
}
void ek_quad_points(const ElemArgs& a, double* xyz, hipStream_t st) {
  launch(quad_points_kernel, grid_for((size_t)a.nE * a.nq), dim3(EK_T), 0, st, a, xyz);
}
void ek_project(const ElemArgs& a, const double* Uqp, double* u_abi, hipStream_t st) {
  launch(project_kernel, grid_for((size_t)a.nE * a.nv), dim3(EK_T), 0, st, a, Uqp, u_abi);
}
void ek_evaluate(const ElemArgs& a, const double* u_abi, double* Uqp, hipStream_t st) {
  launch(evaluate_kernel, grid_for((size_t)a.nE * a.nv), dim3(EK_T), 0, st, a, u_abi, Uqp);
}
void ek_stable_dt(const ElemArgs& a, const double* u_int, const double* cfl_dev, double cfl, double* dt,
                  double* part, unsigned* counter, hipStream_t st) {
  (void)counter;
  const dim3 g = grid_for((size_t)a.nE);
  launch(stable_dt_kernel, g, dim3(EK_T), 0, st, a, u_int, part);
  launch(stable_dt_finalize, dim3(1), dim3(64), 0, st, part, (int)g.x, cfl_dev, cfl, dt);
}
void ek_totals(const ElemArgs& a, const double* u_int, double* out, double* part, unsigned* counter,
               hipStream_t st) {
  (void)counter;
  const dim3 g = grid_for((size_t)a.nE);
  launch(totals_kernel, g, dim3(EK_T), 0, st, a, u_int, part);
  launch(totals_finalize, dim3(1), dim3(EK_T), 0, st, part, (int)g.x, a.nv, out);
}

}  // namespace pcexp
