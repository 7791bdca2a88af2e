// Device-side Euler physics for the DG kernels (paper Sec. 4.1 eq. (euler)
// with omega = 0, perfect gas p = (gamma-1) rho e; Sec. 4.2 numerical flux;
// Sec. 4.4 boundary ghost states).
//
// Every function is templated on the scalar type S, which is either the
// storage type T (value) or Dual<T, N> (value + N directional derivatives), so
// that the tangent (JVP) and the flux Jacobians used by the adjoint are the
// exact derivatives of the residual code.  Non-smooth points follow one
// convention everywhere: d|x| = sign(x) dx with sign(0) = 0, and max() takes
// the first argument on a tie.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace pcexp {

// Forward-mode number: value v and N directional derivatives d[].  T may
// itself be a Dual (nested forward mode: Dual<Dual<double, 1>, N> carries the
// N first derivatives and their derivative along one more direction, which is
// what the second-order adjoint term needs).
template <typename T, int N>
struct Dual {
  T v;
  T d[N];
  Dual() = default;
  // constant (all derivatives zero)
  __host__ __device__ Dual(double c) : v(c) {
#pragma unroll
    for (int i = 0; i < N; ++i) d[i] = T(0);
  }
};

template <typename U> struct IsPlain { static constexpr bool value = std::is_arithmetic<U>::value; };

template <typename T> struct ScalarOf { using type = T; };
template <typename T, int N> struct ScalarOf<Dual<T, N>> { using type = T; };

template <typename T> __device__ __forceinline__ T val(T x) { return x; }
template <typename T, int N> __device__ __forceinline__ T val(const Dual<T, N>& x) { return x.v; }

template <typename T, int N>
__device__ __forceinline__ Dual<T, N> mkconst(T c) {
  Dual<T, N> r;
  r.v = c;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = T(0);
  return r;
}

template <typename S> struct Make;
template <> struct Make<double> {
  __device__ static double zero() { return 0.0; }
  __device__ static double c(double x) { return x; }
};
template <> struct Make<float> {
  __device__ static float zero() { return 0.0f; }
  __device__ static float c(float x) { return x; }
};
template <typename T, int N> struct Make<Dual<T, N>> {
  __device__ static Dual<T, N> zero() { return mkconst<T, N>(T(0)); }
  __device__ static Dual<T, N> c(T x) { return mkconst<T, N>(x); }
};
template <typename S> __device__ __forceinline__ S mkzero() { return Make<S>::zero(); }
template <typename S, typename T> __device__ __forceinline__ S mkconst_s(T x) { return Make<S>::c(x); }

// ---- reciprocal
// 1/x from the hardware reciprocal estimate refined by Newton steps (two in
// FP64, one in FP32): within about an ulp of the IEEE quotient for finite,
// nonzero x of normal range.  Every reciprocal the flux kernels take is of a
// physical quantity of order one (density, the speed of sound squared, a sum
// of square roots of densities, sqrt(det A), a face length), so the
// special-case handling of IEEE division (denormals, overflow, infinities) is
// not needed; a zero or non-finite operand gives a non-finite result, which
// the kernels' flags report.
__device__ __forceinline__ double s_inv(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  return fma(fma(-x, r, 1.0), r, r);
}
__device__ __forceinline__ float s_inv(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(fmaf(-x, r, 1.0f), r, r);
}

// ---- Dual arithmetic
#define PCEXP_DUAL_BINOP(OP, VEXPR, DEXPR)                                                      \
  template <typename T, int N>                                                                  \
  __device__ __forceinline__ Dual<T, N> operator OP(const Dual<T, N>& a, const Dual<T, N>& b) { \
    Dual<T, N> r;                                                                               \
    r.v = VEXPR;                                                                                \
    _Pragma("unroll") for (int i = 0; i < N; ++i) r.d[i] = DEXPR;                               \
    return r;                                                                                   \
  }
PCEXP_DUAL_BINOP(+, a.v + b.v, a.d[i] + b.d[i])
PCEXP_DUAL_BINOP(-, a.v - b.v, a.d[i] - b.d[i])
PCEXP_DUAL_BINOP(*, a.v * b.v, a.d[i] * b.v + a.v * b.d[i])
#undef PCEXP_DUAL_BINOP

template <typename T, int N>
__device__ __forceinline__ Dual<T, N> operator/(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r;
  T ib = s_inv(b.v);
  r.v = a.v * ib;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * ib;
  return r;
}
template <typename T, int N>
__device__ __forceinline__ Dual<T, N> operator-(const Dual<T, N>& a) {
  Dual<T, N> r;
  r.v = -a.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
  return r;
}
template <typename T, int N>
__device__ __forceinline__ Dual<T, N> operator+(const Dual<T, N>& a, T b) {
  Dual<T, N> r = a;
  r.v += b;
  return r;
}
template <typename T, int N>
__device__ __forceinline__ Dual<T, N> operator+(T b, const Dual<T, N>& a) { return a + b; }
template <typename T, int N>
__device__ __forceinline__ Dual<T, N> operator-(const Dual<T, N>& a, T b) {
  Dual<T, N> r = a;
  r.v -= b;
  return r;
}
template <typename T, int N>
__device__ __forceinline__ Dual<T, N> operator-(T b, const Dual<T, N>& a) {
  Dual<T, N> r;
  r.v = b - a.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
  return r;
}
template <typename T, int N>
__device__ __forceinline__ Dual<T, N> operator*(const Dual<T, N>& a, T b) {
  Dual<T, N> r;
  r.v = a.v * b;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b;
  return r;
}
template <typename T, int N>
__device__ __forceinline__ Dual<T, N> operator*(T b, const Dual<T, N>& a) { return a * b; }
template <typename T, int N>
__device__ __forceinline__ Dual<T, N> operator/(const Dual<T, N>& a, T b) {
  Dual<T, N> r;
  T ib = s_inv(b);
  r.v = a.v * ib;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * ib;
  return r;
}
template <typename T, int N>
__device__ __forceinline__ Dual<T, N> operator/(T a, const Dual<T, N>& b) {
  Dual<T, N> r;
  T ib = s_inv(b.v);
  r.v = a * ib;
  T f = -r.v * ib;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = f * b.d[i];
  return r;
}

// Plain scalars (double, float, int) against a Dual whose component type is
// a different type (a nested Dual): applied to the value and every derivative.
#define PCEXP_DUAL_PLAIN(OP)                                                                   \
  template <typename T, int N, typename U,                                                     \
            typename std::enable_if<IsPlain<U>::value && !std::is_same<U, T>::value, int>::type = 0> \
  __device__ __forceinline__ Dual<T, N> operator OP(const Dual<T, N>& a, U b) {                \
    Dual<T, N> r;                                                                              \
    r.v = a.v OP b;                                                                            \
    _Pragma("unroll") for (int i = 0; i < N; ++i) r.d[i] = PCEXP_DUAL_PLAIN_D(a.d[i], b);     \
    return r;                                                                                  \
  }
#define PCEXP_DUAL_PLAIN_D(x, b) (x)
PCEXP_DUAL_PLAIN(+)
PCEXP_DUAL_PLAIN(-)
#undef PCEXP_DUAL_PLAIN_D
#define PCEXP_DUAL_PLAIN_D(x, b) ((x) * (b))
PCEXP_DUAL_PLAIN(*)
#undef PCEXP_DUAL_PLAIN_D
#define PCEXP_DUAL_PLAIN_D(x, b) ((x) * s_inv((double)(b)))
PCEXP_DUAL_PLAIN(/)
#undef PCEXP_DUAL_PLAIN_D
#undef PCEXP_DUAL_PLAIN

template <typename T, int N, typename U,
          typename std::enable_if<IsPlain<U>::value && !std::is_same<U, T>::value, int>::type = 0>
__device__ __forceinline__ Dual<T, N> operator+(U b, const Dual<T, N>& a) { return a + b; }
template <typename T, int N, typename U,
          typename std::enable_if<IsPlain<U>::value && !std::is_same<U, T>::value, int>::type = 0>
__device__ __forceinline__ Dual<T, N> operator*(U b, const Dual<T, N>& a) { return a * b; }
template <typename T, int N, typename U,
          typename std::enable_if<IsPlain<U>::value && !std::is_same<U, T>::value, int>::type = 0>
__device__ __forceinline__ Dual<T, N> operator-(U b, const Dual<T, N>& a) {
  Dual<T, N> r;
  r.v = b - a.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
  return r;
}
template <typename T, int N, typename U,
          typename std::enable_if<IsPlain<U>::value && !std::is_same<U, T>::value, int>::type = 0>
__device__ __forceinline__ Dual<T, N> operator/(U a, const Dual<T, N>& b) {
  Dual<T, N> r;
  T ib = s_inv(b.v);
  r.v = a * ib;
  T f = -r.v * ib;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = f * b.d[i];
  return r;
}

// Comparisons look at values only.
#define PCEXP_DUAL_CMP(OP)                                                                      \
  template <typename T, int N>                                                                  \
  __device__ __forceinline__ bool operator OP(const Dual<T, N>& a, const Dual<T, N>& b) {       \
    return a.v OP b.v;                                                                          \
  }                                                                                             \
  template <typename T, int N, typename U, typename std::enable_if<IsPlain<U>::value, int>::type = 0> \
  __device__ __forceinline__ bool operator OP(const Dual<T, N>& a, U b) {                       \
    return a.v OP b;                                                                            \
  }                                                                                             \
  template <typename T, int N, typename U, typename std::enable_if<IsPlain<U>::value, int>::type = 0> \
  __device__ __forceinline__ bool operator OP(U a, const Dual<T, N>& b) {                       \
    return a OP b.v;                                                                            \
  }
PCEXP_DUAL_CMP(>)
PCEXP_DUAL_CMP(<)
PCEXP_DUAL_CMP(>=)
PCEXP_DUAL_CMP(<=)
#undef PCEXP_DUAL_CMP

// ---- elementary functions (value and Dual)
__device__ __forceinline__ double s_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float s_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double s_abs(double x) { return fabs(x); }
__device__ __forceinline__ float s_abs(float x) { return fabsf(x); }
__device__ __forceinline__ double s_pow(double x, double e) { return pow(x, e); }
__device__ __forceinline__ float s_pow(float x, float e) { return powf(x, e); }
template <typename T> __device__ __forceinline__ T s_max(T a, T b) { return a >= b ? a : b; }
template <typename T> __device__ __forceinline__ T s_sign(T x) {
  return x > T(0) ? T(1) : (x < T(0) ? T(-1) : T(0));
}

template <typename T, int N>
__device__ __forceinline__ Dual<T, N> s_sqrt(const Dual<T, N>& a) {
  Dual<T, N> r;
  r.v = s_sqrt(a.v);
  T f = T(0.5) * s_inv(r.v);
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = f * a.d[i];
  return r;
}
template <typename T, int N>
__device__ __forceinline__ Dual<T, N> s_inv(const Dual<T, N>& a) {
  Dual<T, N> r;
  r.v = s_inv(a.v);
  T f = -r.v * r.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = f * a.d[i];
  return r;
}
template <typename T, int N>
__device__ __forceinline__ Dual<T, N> s_abs(const Dual<T, N>& a) {
  T s = s_sign(a.v);
  Dual<T, N> r;
  r.v = a.v * s;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * s;
  return r;
}
template <typename T, int N>
__device__ __forceinline__ Dual<T, N> s_max(const Dual<T, N>& a, const Dual<T, N>& b) {
  return a.v >= b.v ? a : b;
}
template <typename T, int N, typename E, typename std::enable_if<IsPlain<E>::value, int>::type = 0>
__device__ __forceinline__ Dual<T, N> s_pow(const Dual<T, N>& a, E e) {
  Dual<T, N> r;
  r.v = s_pow(a.v, e);
  T f = e * s_pow(a.v, e - E(1));
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = f * a.d[i];
  return r;
}

// ---- Euler fluxes.  U = (rho, m_1..m_D, rho E).
// Physical flux in the (not necessarily unit) direction a:
//   F.a = (m.a, m (m.a)/rho + p a, (rho E + p)(m.a)/rho).
template <int D, typename S, typename T>
__device__ __forceinline__ void normal_flux(const S* U, const T* a, T gm1, S* F, S* p_out = nullptr) {
  S rinv = s_inv(U[0]);
  S ma = U[1] * a[0];
  S m2 = U[1] * U[1];
#pragma unroll
  for (int c = 1; c < D; ++c) {
    ma = ma + U[1 + c] * a[c];
    m2 = m2 + U[1 + c] * U[1 + c];
  }
  S p = gm1 * (U[D + 1] - T(0.5) * m2 * rinv);
  S vn = ma * rinv;
  F[0] = ma;
#pragma unroll
  for (int c = 0; c < D; ++c) F[1 + c] = U[1 + c] * vn + p * a[c];
  F[D + 1] = (U[D + 1] + p) * vn;
  if (p_out) *p_out = p;
}

// Local Lax-Friedrichs (Rusanov): 1/2 (F_L + F_R).n - 1/2 alpha (U_R - U_L),
// alpha = max(|v_L.n| + c_L, |v_R.n| + c_R) at the point.
template <int D, typename S, typename T>
__device__ __forceinline__ void flux_lf(const S* UL, const S* UR, const T* n, T gamma, S* F) {
  const T gm1 = gamma - T(1);
  S FL[D + 2], FR[D + 2], pL, pR;
  normal_flux<D>(UL, n, gm1, FL, &pL);
  normal_flux<D>(UR, n, gm1, FR, &pR);
  const S riL = s_inv(UL[0]), riR = s_inv(UR[0]);
  S vnL = FL[0] * riL, vnR = FR[0] * riR;
  S aL = s_abs(vnL) + s_sqrt(gamma * pL * riL);
  S aR = s_abs(vnR) + s_sqrt(gamma * pR * riR);
  S al = s_max(aL, aR);
#pragma unroll
  for (int k = 0; k < D + 2; ++k) F[k] = T(0.5) * (FL[k] + FR[k]) - T(0.5) * al * (UR[k] - UL[k]);
}

// Roe (1981) flux without entropy fix:
//   1/2 (F_L + F_R).n - 1/2 sum_waves |lambda| alpha r.
template <int D, typename S, typename T>
__device__ __forceinline__ void flux_roe(const S* UL, const S* UR, const T* n, T gamma, S* F) {
  const T gm1 = gamma - T(1);
  S pL, pR;
  {
    // the central part 1/2 (F_L + F_R).n first, so that the two physical
    // fluxes are not held while the dissipation is formed
    S FR[D + 2];
    normal_flux<D>(UL, n, gm1, F, &pL);
    normal_flux<D>(UR, n, gm1, FR, &pR);
#pragma unroll
    for (int k = 0; k < D + 2; ++k) F[k] = T(0.5) * (F[k] + FR[k]);
  }
  S rLi = s_inv(UL[0]), rRi = s_inv(UR[0]);
  S sL = s_sqrt(UL[0]), sR = s_sqrt(UR[0]);
  S den = s_inv(sL + sR);
  S HL = (UL[D + 1] + pL) * rLi, HR = (UR[D + 1] + pR) * rRi;
  S ut[D], dv[D];
  S q2 = mkzero<S>(), vn = mkzero<S>(), dvn = mkzero<S>(), udv = mkzero<S>();
#pragma unroll
  for (int c = 0; c < D; ++c) {
    S vLc = UL[1 + c] * rLi, vRc = UR[1 + c] * rRi;
    ut[c] = (sL * vLc + sR * vRc) * den;
    dv[c] = vRc - vLc;
    q2 = q2 + ut[c] * ut[c];
    vn = vn + ut[c] * n[c];
    dvn = dvn + dv[c] * n[c];
    udv = udv + ut[c] * dv[c];
  }
  S Ht = (sL * HL + sR * HR) * den;
  S c2 = gm1 * (Ht - T(0.5) * q2);
  S ct = s_sqrt(c2);
  S rt = sL * sR;
  S dr = UR[0] - UL[0];
  S dp = pR - pL;
  S ic2 = s_inv(c2);
  S a1 = (dp - rt * ct * dvn) * (T(0.5) * ic2);
  S a3 = (dp + rt * ct * dvn) * (T(0.5) * ic2);
  S a2 = dr - dp * ic2;
  S l1 = s_abs(vn - ct), l2 = s_abs(vn), l3 = s_abs(vn + ct);
  S w1 = l1 * a1, w2 = l2 * a2, w3 = l3 * a3, ws = l2 * rt;
  S Dk = w1 + w2 + w3;
  F[0] = F[0] - T(0.5) * Dk;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    S Dc = w1 * (ut[c] - ct * n[c]) + w2 * ut[c] + ws * (dv[c] - dvn * n[c]) + w3 * (ut[c] + ct * n[c]);
    F[1 + c] = F[1 + c] - T(0.5) * Dc;
  }
  S DE = w1 * (Ht - ct * vn) + w2 * (T(0.5) * q2) + ws * (udv - vn * dvn) + w3 * (Ht + ct * vn);
  F[D + 1] = F[D + 1] - T(0.5) * DE;
}

// Slip wall: mirror state (rho, m - 2 (m.n) n, rho E).
template <int D, typename S, typename T>
__device__ __forceinline__ void ghost_slip(const S* UL, const T* n, S* G) {
  S mn = UL[1] * n[0];
#pragma unroll
  for (int c = 1; c < D; ++c) mn = mn + UL[1 + c] * n[c];
  G[0] = UL[0];
#pragma unroll
  for (int c = 0; c < D; ++c) G[1 + c] = UL[1 + c] - T(2) * mn * n[c];
  G[D + 1] = UL[D + 1];
}

// Riemann-invariant far field (prim_inf = rho, u, v, [w], p).  Supersonic
// outflow (v_L.n >= c_L): interior state; supersonic inflow (v_L.n <= -c_L):
// free stream; otherwise R+ = v_L.n + 2c_L/(g-1), R- = v_inf.n - 2c_inf/(g-1),
// v_n = (R+ + R-)/2, c = (g-1)(R+ - R-)/4, entropy and tangential velocity
// from the interior if v_n >= 0 else from the free stream.
template <int D, typename S, typename T>
__device__ __forceinline__ void ghost_farfield(const S* UL, const T* n, const T* prim, T gamma, S* G) {
  const T gm1 = gamma - T(1);
  S rinv = s_inv(UL[0]);
  S vL[D], vnL = mkzero<S>(), q2 = mkzero<S>();
#pragma unroll
  for (int c = 0; c < D; ++c) {
    vL[c] = UL[1 + c] * rinv;
    vnL = vnL + vL[c] * n[c];
    q2 = q2 + vL[c] * vL[c];
  }
  S pL = gm1 * (UL[D + 1] - T(0.5) * UL[0] * q2);
  S cL = s_sqrt(gamma * pL * rinv);
  const T rinf = prim[0], pinf = prim[D + 1];
  T vninf = T(0), q2inf = T(0);
#pragma unroll
  for (int c = 0; c < D; ++c) {
    vninf += prim[1 + c] * n[c];
    q2inf += prim[1 + c] * prim[1 + c];
  }
  if (val(vnL) >= val(cL)) {
#pragma unroll
    for (int k = 0; k < D + 2; ++k) G[k] = UL[k];
    return;
  }
  if (val(vnL) <= -val(cL)) {
    G[0] = mkconst_s<S>(rinf);
#pragma unroll
    for (int c = 0; c < D; ++c) G[1 + c] = mkconst_s<S>(rinf * prim[1 + c]);
    G[D + 1] = mkconst_s<S>(pinf / gm1 + T(0.5) * rinf * q2inf);
    return;
  }
  const T cinf = s_sqrt(gamma * pinf / rinf);
  S Rp = vnL + (T(2) / gm1) * cL;
  T Rm = vninf - T(2) * cinf / gm1;
  S vnb = T(0.5) * (Rp + Rm);
  S cb = (T(0.25) * gm1) * (Rp - Rm);
  S sb, vt[D];
  if (val(vnb) >= T(0)) {
    sb = pL / s_pow(UL[0], gamma);
#pragma unroll
    for (int c = 0; c < D; ++c) vt[c] = vL[c] - vnL * n[c];
  } else {
    sb = mkconst_s<S>(pinf / s_pow(rinf, gamma));
#pragma unroll
    for (int c = 0; c < D; ++c) vt[c] = mkconst_s<S>(prim[1 + c] - vninf * n[c]);
  }
  S rb = s_pow(cb * cb / (gamma * sb), T(1) / gm1);
  S pb = rb * cb * cb / gamma;
  S vb2 = mkzero<S>();
  G[0] = rb;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    S vb = vt[c] + vnb * n[c];
    G[1 + c] = rb * vb;
    vb2 = vb2 + vb * vb;
  }
  G[D + 1] = pb / gm1 + T(0.5) * rb * vb2;
}

}  // namespace pcexp
