// Element-tiled DG operator kernels for gfx950: residual R(u) (paper Sec. 4.2
// eq. (euler3), identity mass, omega = 0), its exact tangent J(u)v (Sec. 4.4,
// the Jacobian of eqs. (jac1)/(jac2) applied matrix-free), the
// finite-difference JVP baseline, and the transpose J(u)^T w.
//
// Internal basis: reference-orthonormal phi_hat mapped affinely, psi_i =
// phi_hat_i(xi)/s with s = sqrt(det A), x = X_0 + A xi.  For element E:
//   volume:  s * sum_q w_q sum_r G_kr(q) dphi_hat_i/dxi_r(xi_q),
//            G_kr = F_k(U_q) . a_r,  a_r = row r of A^{-1}
//   faces:   - sum_f sum_r w_r (|f|/s) phi_hat_i(xi_r) Ftilde_k(U_L, U_R, n_f)
// with |f| n_f = det(A) A^{-T} nref_f.
//
// Layout: vectors are [k][i][E] with element stride Epad (element-fastest, so
// every global access of a tile is coalesced).  One workgroup of 256 threads
// owns a tile of TE consecutive elements; the tile's coefficients are staged
// in LDS, threads map to (quadrature point, element) for the pointwise flux
// work and to (output, element) for the contractions.  Every face flux is
// computed by both of its elements (no atomics; bitwise deterministic).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "dg_physics.hpp"
#include "launch.hpp"
#include "wave_reduce.hpp"

namespace pcexp {

template <int D, int P>
struct Shape {
  static constexpr int NV = D + 2;
  static constexpr int NB = D == 2 ? (P + 1) * (P + 2) / 2 : (P + 1) * (P + 2) * (P + 3) / 6;
  // quadrature points, volume and per face: conical-product rules with P + 1
  // points per collapsed direction, except 3D P2, which takes symmetric rules
  // of the same degree 5 (14 points on the tetrahedron, 7 on each face)
  static constexpr int Q1 = P + 1;
  static constexpr bool SYM = D == 3 && P == 2;
  static constexpr int NQ = SYM ? 14 : D == 2 ? Q1 * Q1 : Q1 * Q1 * Q1;
  static constexpr int NFQ = SYM ? 7 : D == 2 ? Q1 : Q1 * Q1;
  static constexpr int NF = D + 1;
  static constexpr int NORI = D == 2 ? 2 : 6;
  static constexpr int NVB = NV * NB;
};

enum { MODE_RES = 0, MODE_TAN = 1, MODE_FD = 2 };
enum { FLUX_LF = 0, FLUX_ROE = 1 };

template <typename T>
struct DGParams {
  const T* B;      // [NQ][NB]
  const T* Dg;     // [NQ][NB][D]
  const T* wq;     // [NQ]
  const T* Bf;     // [NF][NORI][NFQ][NB]
  const T* wf;     // [NFQ]
  const T* nref;   // [NF][D]
  const T* ainv;   // [D*D][Epad]
  const T* sdet;   // [Epad]
  const int* nbr;  // [NF][Epad]
  const int* finfo;  // [NF][Epad]
  int nE, Epad;
  T gamma;
  T ff[5];
};

template <typename T>
struct DGIO {
  const T* u;
  const T* v;
  T* out;
  const double* vscale;  // optional: v is multiplied by *vscale
  const int* skip;       // optional: the launch is a no-op if *skip != 0
  const T* rbase;        // FD: R(u)
  const double* fd_eps;  // FD: increment eps for the (scaled) direction
  unsigned* flags;       // RES: PCEXP_FLAG_* bits
  // Optional (TAN, FD): the reduction pass of the Arnoldi iteration fused
  // into this launch.  With gsV set, the block that handles tile b also sums,
  // over its tile's live elements, V_i.U and V_i.W for the gsj basis vectors
  // V_i = gsV + i gsld, and U.U, U.W, W.W, where U = v (unscaled) and W = out,
  // and writes them to gspart[col * gspld + b]: columns [0, gsj) V.U,
  // [gsj, 2 gsj) V.W, then U.U, U.W, W.W.  gspld >= the launch's block count.
  const T* gsV;
  size_t gsld;
  int gsj;
  double* gspart;
  int gspld;
};

// LDS budget per workgroup (bytes) used to choose the tile size.
constexpr int kLdsBudget = 40 * 1024;

// Tile policy.  The two pointwise phases have NQ * TE (volume) and
// NF * NFQ * TE (faces) work items over NT threads; a partial last round
// leaves most lanes idle, so TE is chosen to minimise rounds per element
// under the LDS budget, and among equals the smallest TE: more workgroups
// per compute unit hide the phases' latency better (measured: the FP32 2D P2
// tangent at 28 elements instead of 56 makes the mixed-precision step 11 %
// faster on the 128 x 128 vortex).
template <int D, int P, typename T, bool DUAL>
struct Tile {
  using Sh = Shape<D, P>;
  static constexpr int NG = Sh::NQ * Sh::NV * D;
  static constexpr int FS = Sh::NV * (DUAL ? 2 : 1);   // LDS words per face point (neighbour trace)
  static constexpr int NFL = Sh::NF * Sh::NFQ * FS;
  static constexpr int NW = NG > NFL ? NG : NFL;
  // volume contraction on the matrix cores for 3D, p >= 2 (NB <= 16: one tile
  // of rows).  Measured: the 3D P2 FP64 residual gains 8 %, the 3D JVP is
  // unchanged, and the 2D P2 kernels (six basis functions pad to 16 rows)
  // lose 4 %, so 2D keeps the VALU contraction.
  static constexpr bool VMFMA = D == 3 && P >= 2 && Sh::NB <= 16;
  // basis-to-quadrature interpolation U_q = B u on the matrix cores, in the
  // same element class (3D P2: 14 points, one 16-row tile, x 10 basis
  // functions per (set, variable, element) column).  Measured with the
  // 27-point conical rule: the 3D P2 FP32 tangent JVP 1.13 -> 1.10 ms, the
  // FP64 residual 1.52 -> 1.43 ms; in 2D P2 (9 points x 6 basis functions
  // pad to 16 x 8) the JVPs got 1-6 % slower, so 2D keeps the VALU
  // interpolation.
  static constexpr bool VMFMA_IN = VMFMA;
  // per element: coefficients (and direction), flux scratch, geometry (det,
  // A^-1, neighbours, face codes) and the face orientation codes
  static constexpr int per_elem = (int)sizeof(T) * (Sh::NVB * (DUAL ? 2 : 1) + NW + 1 + D * D) + 8 * Sh::NF + Sh::NF;
  // reference tables B, Dg, Bf, wq, wf, nref, staged in LDS: every lane
  // reads an entry per multiply-add, and from global memory (L1) those reads
  // bound the kernel (3D P2: 2273 entries).  A 3D tile gets a larger LDS
  // budget so that the tables fit beside a tile that fills the pointwise
  // phases.
  static constexpr int NTAB = Sh::NQ * Sh::NB * (D + 1) + Sh::NF * Sh::NORI * Sh::NFQ * Sh::NB + Sh::NQ +
                              Sh::NFQ + Sh::NF * D;
  static constexpr bool STAGE_TAB = NTAB * (int)sizeof(T) <= 32768;
  static constexpr int fixed_lds = STAGE_TAB ? NTAB * (int)sizeof(T) : 0;
  static constexpr int budget = D == 3 ? 64 * 1024 : kLdsBudget;
  static constexpr int NT = 256;
  static constexpr int rounds(int te) {
    return (Sh::NQ * te + NT - 1) / NT + (Sh::NF * Sh::NFQ * te + NT - 1) / NT;
  }
  static constexpr int pick() {
    int best = 1;
    for (int te = 2; te <= 64; ++te) {
      if (te * per_elem + fixed_lds > budget) break;
      if (rounds(te) * best < rounds(best) * te) best = te;   // rounds/te smaller
    }
    return best;
  }
  static constexpr int TE = pick();
  // Outputs per thread in the contractions: the smallest divisor NI of NB
  // with NV * (NB / NI) * TE <= NT (one round); each thread then reuses every
  // flux value it reads from LDS for NI basis functions.
  static constexpr int pick_ni() {
    for (int ni = 1; ni <= Sh::NB; ++ni)
      if (Sh::NB % ni == 0 && Sh::NV * (Sh::NB / ni) * TE <= NT) return ni;
    return Sh::NB;
  }
  static constexpr int NI = pick_ni();
};

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of tiles so that neighbouring tiles share an L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int per = nb / 8, rem = nb % 8;
  const int x = b % 8, k = b / 8;
  return x * per + (x < rem ? x : rem) + k;
}

template <typename S> struct Part;
template <> struct Part<double> { __device__ static double get(double x) { return x; } };
template <> struct Part<float> { __device__ static float get(float x) { return x; } };
template <typename T> struct Part<Dual<T, 1>> { __device__ static T get(const Dual<T, 1>& x) { return x.d[0]; } };

template <int D, int FLUX, typename S, typename T>
__device__ __forceinline__ void num_flux(const S* UL, const S* UR, const T* n, T gamma, S* F) {
  if (FLUX == FLUX_LF) flux_lf<D>(UL, UR, n, gamma, F);
  else flux_roe<D>(UL, UR, n, gamma, F);
}

// One 16 x 16 x 4 product on the matrix cores, C += A B: lane l supplies
// A(l % 16, l / 16) and B(l / 16, l % 16) and holds C rows row(l, r), r < 4,
// of column l % 16 (layouts checked on the device for both precisions).
template <typename T> struct Mfma16;
template <> struct Mfma16<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __device__ static v4 mma(double a, double b, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct Mfma16<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ static v4 mma(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// The fused Arnoldi reduction of one tile (see DGIO::gsV).  Thread entries
// e < NE sit at offsets ix[e] of every vector, with U values u[e] and W
// values w[e] (zero for entries outside the tile's live elements).  Basis
// vectors go in chunks of CB: each lane loads its entries of the chunk's
// vectors together and the wave sums the 2 CB products by the butterfly into
// its own LDS row (red: NT / 64 rows of GS_ROW slots), so the chunk loop has
// no barrier; after one barrier, thread c sums column c over the rows in wave
// order and writes the block's partial.  Row slots: V.U of vector i at i,
// V.W at GS_SW + i (a chunk past nq writes up to 7 slots beyond, never read),
// then U.U, U.W, W.W.
constexpr int GS_MAXQ = 64;   // basis vectors before U, at most (the Krylov dimension bound)
constexpr int GS_SW = GS_MAXQ + 8;
constexpr int GS_ROW = 2 * GS_SW + 4;
template <int NT, int NE, int CB, typename T>
__device__ __forceinline__ void gs_tile_dots(const T* __restrict__ V, size_t ld, int nq, const int* ix,
                                             const double* u, const double* w, double* __restrict__ part,
                                             int pld, double* red) {
  constexpr int NC = 2 * CB, NWV = NT / 64, RL = GS_ROW;
  static_assert(CB <= 8, "chunk overhang within the row's slack");
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double* row = red + wid * RL;
  for (int i0 = 0; i0 < nq; i0 += CB) {
    T x[CB][NE];
#pragma unroll
    for (int i = 0; i < CB; ++i) {
      const int vi = i0 + i < nq ? i0 + i : nq - 1;   // past the last vector: re-read it, result dropped
      const T* Vi = V + (size_t)vi * ld;
#pragma unroll
      for (int e = 0; e < NE; ++e) x[i][e] = Vi[ix[e]];
    }
    double a[NC];
#pragma unroll
    for (int i = 0; i < CB; ++i) {
      double su = 0.0, sw = 0.0;
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        su += (double)x[i][e] * u[e];
        sw += (double)x[i][e] * w[e];
      }
      a[i] = su;
      a[CB + i] = sw;
    }
    int col = 0;
    Bfly<NC / 2, 32>::run(a, lane, col);
    if ((lane & (64 / NC - 1)) == 0) row[(col < CB ? 0 : GS_SW - CB) + i0 + col] = a[0];
  }
  double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    a[0] += u[e] * u[e];
    a[1] += u[e] * w[e];
    a[2] += w[e] * w[e];
  }
  int col = 0;
  Bfly<2, 32>::run(a, lane, col);
  if ((lane & 15) == 0) row[2 * GS_SW + col] = a[0];
  __syncthreads();
  for (int c = threadIdx.x; c < 2 * nq + 3; c += NT) {
    // partial column c: [0, nq) V.U, [nq, 2 nq) V.W, then U.U, U.W, W.W
    const int src = c < nq ? c : c < 2 * nq ? GS_SW + (c - nq) : 2 * GS_SW + (c - 2 * nq);
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < NWV; ++q) s += red[q * RL + src];
    part[(size_t)c * pld + blockIdx.x] = s;
  }
}

template <int D, int P, int FLUX, typename T, int MODE, int TE, int NT>
__global__ __launch_bounds__(NT) void dg_apply(DGParams<T> prm, DGIO<T> io) {
  using Sh = Shape<D, P>;
  constexpr int NV = Sh::NV, NB = Sh::NB, NVB = Sh::NVB, NQ = Sh::NQ, NFQ = Sh::NFQ;
  constexpr int NF = Sh::NF, NORI = Sh::NORI;
  constexpr bool DUAL = (MODE == MODE_TAN);
  using Tl = Tile<D, P, T, DUAL>;
  using S = typename std::conditional<DUAL, Dual<T, 1>, T>::type;
  // output items (k, g, e): basis functions i = g + NG c, c < NI
  constexpr int NI = Tl::NI, NG = NB / NI;
  constexpr int NITEM = NV * NG * TE;
  constexpr int NOUT = (NITEM + NT - 1) / NT;

  __shared__ T su[NVB * TE];
  __shared__ T sv[DUAL ? NVB * TE : 1];
  __shared__ __attribute__((aligned(16))) T sw[Tl::NW * TE];
  __shared__ unsigned char sori[NF * TE];
  __shared__ T stab[Tl::STAGE_TAB ? Tl::NTAB : 1];
  // Faces whose two elements both lie in the tile are evaluated once, by
  // the side of smaller index (see the face phase), in the FP32 kernels.
  // Measured: the mixed-precision JVP gains 9 % on the 3D P2 vortex and 2 %
  // on the 2D one; the FP64 kernels, with fewer resident waves and bound by
  // latency, lose 2-10 % to the indirection through the face list, so they
  // keep one item per face point of every element.
  constexpr bool DEDUP = sizeof(T) == 4;
  // Per-element geometry, neighbours and face codes, staged in LDS.  When
  // the pointwise phases that use the geometry are single rounds, thread tid
  // works on element e0 + tid % TE in them and keeps its det and A^-1 in
  // registers (with DEDUP the face phase reads them from LDS).
  constexpr bool PF = NQ * TE <= NT && (DEDUP || NF * NFQ * TE <= NT);
  constexpr int GTE = (PF && !DEDUP) ? 1 : TE;
  __shared__ T sg_det[GTE];
  __shared__ T sg_ainv[D * D * GTE];
  __shared__ int sg_nbr[NF * TE];
  __shared__ int sg_info[NF * TE];
  // With DEDUP, the face incidences (e, f) of the tile, entry f * TE + e, in
  // three classes: 0, the neighbour lies in the tile and has the larger
  // index (this side evaluates the flux for both); 1, the neighbour lies in
  // another tile; 2, a boundary face; 3, none (the neighbour in the tile
  // evaluates it, or a padding element).  flist holds classes 0, 1, 2 in
  // that order, each in entry order; fcnt the per-wave class counts.
  static_assert(!DEDUP || NF * TE <= NT, "one face incidence per thread");
  constexpr int NFL_ = DEDUP ? NF * TE : 1;
  __shared__ unsigned short flist[NFL_];
  __shared__ unsigned char fcls[NFL_];
  __shared__ int fcnt[NT / 64][3];
  // sw holds, in turn, the weighted volume fluxes (k, r, q, e) and the face
  // values (c, f, r, e), with the pointwise index (q or face point) next to
  // e: the threads of a pointwise phase, t = q * TE + e, then touch
  // consecutive words and the LDS banks without conflicts.
  constexpr int NFP = NF * NFQ;
  auto vix = [](int q, int k, int r, int e) { return ((k * D + r) * NQ + q) * TE + e; };
  auto fix = [](int c, int fp, int e) { return (c * NFP + fp) * TE + e; };

  const int Epad = prm.Epad, nE = prm.nE;
  const int e0 = xcd_tile(blockIdx.x, gridDim.x) * TE;
  const int tid = threadIdx.x;
  const T gm1 = prm.gamma - T(1);

  // Every global load the block needs before its first barrier is issued up
  // front, from clamped addresses and outside branches, so that the block
  // waits for one memory round trip: the skip flag and scales, the reference
  // tables, the tile's coefficients and its geometry.
  const bool skipped = io.skip ? (*io.skip != 0) : false;
  T scale = T(1);
  if (MODE != MODE_RES && io.vscale) scale = (T)(*io.vscale);
  T eps = T(0);
  if (MODE == MODE_FD) eps = (T)(*io.fd_eps);

  // reference tables: every lane reads them, so keep them in LDS when small
  constexpr int oDg = NQ * NB, oBf = oDg + NQ * NB * D, owq = oBf + NF * NORI * NFQ * NB, owf = owq + NQ,
                onr = owf + NFQ;
  constexpr int NTR = Tl::STAGE_TAB ? (Tl::NTAB + NT - 1) / NT : 1;
  T xt[NTR];
  if constexpr (Tl::STAGE_TAB) {
#pragma unroll
    for (int s = 0; s < NTR; ++s) {
      int t = tid + s * NT;
      t = t < Tl::NTAB ? t : Tl::NTAB - 1;
      const T* src = t < oDg   ? prm.B + t
                     : t < oBf ? prm.Dg + (t - oDg)
                     : t < owq ? prm.Bf + (t - oBf)
                     : t < owf ? prm.wq + (t - owq)
                     : t < onr ? prm.wf + (t - owf)
                               : prm.nref + (t - onr);
      xt[s] = *src;
    }
  }
  constexpr int NSTG = (NVB * TE + NT - 1) / NT;
  T ru[NSTG], rv[NSTG];
#pragma unroll
  for (int s = 0; s < NSTG; ++s) {
    const int t = tid + s * NT;
    const int tc = t < NVB * TE ? t : NVB * TE - 1;
    const int ki = tc / TE, ge = e0 + tc % TE;
    const int gc = ge < nE ? ge : nE - 1;
    ru[s] = io.u[(size_t)ki * Epad + gc];
    if constexpr (MODE != MODE_RES) rv[s] = io.v[(size_t)ki * Epad + gc];
    else rv[s] = T(0);
  }
  constexpr int NGT = PF ? 0 : (1 + D * D) * TE, NGI = 2 * NF * TE;
  static_assert(!PF || TE <= NT, "the register copy of the geometry covers the tile");
  constexpr int NGTL = (NGT + NT - 1) / NT, NGIL = (NGI + NT - 1) / NT;
  T gt[NGTL > 0 ? NGTL : 1];
  int gi[NGIL > 0 ? NGIL : 1];
#pragma unroll
  for (int s = 0; s < NGTL; ++s) {
    int t = tid + s * NT;
    t = t < NGT ? t : NGT - 1;
    const int c = t / TE, ge = e0 + t % TE, gc = ge < nE ? ge : nE - 1;
    gt[s] = c == 0 ? prm.sdet[gc] : prm.ainv[(size_t)(c - 1) * Epad + gc];
  }
#pragma unroll
  for (int s = 0; s < NGIL; ++s) {
    int t = tid + s * NT;
    t = t < NGI ? t : NGI - 1;
    const int c = t / TE, ge = e0 + t % TE, gc = ge < nE ? ge : nE - 1;
    gi[s] = c < NF ? prm.nbr[(size_t)c * Epad + gc] : prm.finfo[(size_t)(c - NF) * Epad + gc];
  }
  T pg_det = T(0), pg_ainv[D * D];
  if constexpr (PF) {
    const int ge = e0 + tid % TE, gc = ge < nE ? ge : nE - 1;
    pg_det = prm.sdet[gc];
#pragma unroll
    for (int c = 0; c < D * D; ++c) pg_ainv[c] = prm.ainv[(size_t)c * Epad + gc];
  }
  __builtin_amdgcn_sched_barrier(0);
  if (skipped) return;
  // geometry of element e of the tile (with PF: the thread's own element)
  auto g_det = [&](int e) -> T {
    if constexpr (PF) return pg_det;
    else return sg_det[e];
  };
  auto g_ainv = [&](int e, int c) -> T {
    if constexpr (PF) return pg_ainv[c];
    else return sg_ainv[c * TE + e];
  };
  auto l_det = [&](int e) -> T { return sg_det[e]; };
  auto l_ainv = [&](int e, int c) -> T { return sg_ainv[c * TE + e]; };
  auto g_nbr = [&](int e, int f) -> int { return sg_nbr[f * TE + e]; };
  auto g_info = [&](int e, int f) -> int { return sg_info[f * TE + e]; };

  const T *tB, *tDg, *tBf, *twq, *twf, *tnref;
  if constexpr (Tl::STAGE_TAB) {
#pragma unroll
    for (int s = 0; s < NTR; ++s)
      if (tid + s * NT < Tl::NTAB) stab[tid + s * NT] = xt[s];
    tB = stab; tDg = stab + oDg; tBf = stab + oBf; twq = stab + owq; twf = stab + owf; tnref = stab + onr;
  } else {
    tB = prm.B; tDg = prm.Dg; tBf = prm.Bf; twq = prm.wq; twf = prm.wf; tnref = prm.nref;
  }
#pragma unroll
  for (int s = 0; s < NGTL; ++s) {
    const int t = tid + s * NT;
    if (t < NGT) {
      const int c = t / TE, e = t % TE;
      if (c == 0) sg_det[e] = gt[s];
      else sg_ainv[(c - 1) * TE + e] = gt[s];
    }
  }
  if constexpr (PF && DEDUP) {
    if (tid < TE) {
      sg_det[tid] = pg_det;
#pragma unroll
      for (int c = 0; c < D * D; ++c) sg_ainv[c * TE + tid] = pg_ainv[c];
    }
  }
#pragma unroll
  for (int s = 0; s < NGIL; ++s) {
    const int t = tid + s * NT;
    if (t < NGI) {
      const int c = t / TE, e = t % TE;
      if (c < NF) sg_nbr[c * TE + e] = gi[s];
      else sg_info[(c - NF) * TE + e] = gi[s];
    }
  }
  // ---- the tile's coefficients (u, and the direction v for the tangent)
#pragma unroll
  for (int s = 0; s < NSTG; ++s) {
    const int t = tid + s * NT;
    if (t < NVB * TE) {
      const bool live = e0 + t % TE < nE;
      T uu = live ? ru[s] : T(0);
      const T vv = live ? rv[s] * scale : T(0);
      if (MODE == MODE_FD) uu = uu + eps * vv;
      su[t] = uu;
      if (DUAL) sv[t] = vv;
    }
  }
  __syncthreads();

  // ---- face incidences: class of thread tid's incidence, per-wave counts
  if constexpr (DEDUP) {
    const int f = tid / TE, e = tid % TE, ge = e0 + e;
    int cls = 3;
    if (tid < NF * TE && ge < nE) {
      const int nb = g_nbr(e, f);
      if (nb < 0) cls = 2;
      else if (nb >= e0 && nb < e0 + TE && nb != ge) cls = ge < nb ? 0 : 3;
      else cls = 1;
    }
    if (tid < NF * TE) fcls[tid] = (unsigned char)cls;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const unsigned long long m = __ballot(cls == c);
      if ((tid & 63) == 0) fcnt[tid >> 6][c] = __popcll(m);
    }
  }
  // class totals (after the barrier that follows the counts)
  auto ftot = [&](int c) -> int {
    int n = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) n += fcnt[w][c];
    return n;
  };

  T acc[NOUT][NI];
#pragma unroll
  for (int o = 0; o < NOUT; ++o)
#pragma unroll
    for (int c = 0; c < NI; ++c) acc[o][c] = T(0);

  // ---- volume: pointwise flux contracted with the rows of A^{-1}
  // (flags in residual mode, then the weighted normal fluxes of point q of
  // element e into the flux scratch)
  auto vol_flux = [&](int q, int e, const S* U) {
    if (MODE == MODE_RES && io.flags) {
      T rho = val(U[0]), m2 = T(0);
#pragma unroll
      for (int c = 0; c < D; ++c) m2 += val(U[1 + c]) * val(U[1 + c]);
      T p = gm1 * (val(U[D + 1]) - T(0.5) * m2 / rho);
      unsigned fl = 0;
      if (!isfinite(rho) || !isfinite(p)) fl |= 1u;
      else if (!(rho > T(0)) || !(p > T(0))) fl |= 2u;
      if (fl) atomicOr(io.flags, fl);
    }
    const T wgt = g_det(e) * twq[q];
#pragma unroll
    for (int r = 0; r < D; ++r) {
      T a[D];
#pragma unroll
      for (int c = 0; c < D; ++c) a[c] = g_ainv(e, r * D + c);
      S F[NV];
      normal_flux<D>(U, a, gm1, F);
#pragma unroll
      for (int k = 0; k < NV; ++k) sw[vix(q, k, r, e)] = wgt * Part<S>::get(F[k]);
    }
  };
  if constexpr (Tl::VMFMA_IN) {
    // U at the quadrature points on the matrix cores: C = B X with rows the
    // points q < NQ (tiles of 16), the contraction over the basis functions
    // i < NB in steps of 4, and columns c = (s, k, e): coefficient set s (the
    // state, and the direction for the tangent), variable k, element e.
    // The point values go to the flux scratch, then into registers, before
    // the scratch receives the fluxes.
    constexpr int NS = DUAL ? 2 : 1;
    constexpr int NCI = NS * NV * TE, NTI = (NCI + 15) / 16;
    constexpr int NRT = (NQ + 15) / 16, KB4 = (NB + 3) / 4;
    constexpr int NW_ = NT / 64, MTI = (NTI + NW_ - 1) / NW_;
    static_assert(NS * NV * NQ <= Tl::NW, "point values fit the flux scratch");
    auto uix = [](int s_, int k, int q, int e) { return ((s_ * NV + k) * NQ + q) * TE + e; };
    const int lane = tid & 63, li = lane & 15, lk = lane >> 4, wid = tid >> 6;
    T av[NRT][KB4];   // A operands of this lane: B(q = 16 rt + li, i = 4 kb + lk)
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
      for (int kb = 0; kb < KB4; ++kb) {
        const int q = 16 * rt + li, i = 4 * kb + lk;
        av[rt][kb] = (q < NQ && i < NB) ? tB[q * NB + i] : T(0);
      }
#pragma unroll
    for (int mt = 0; mt < MTI; ++mt) {
      const int tn = wid + mt * NW_;
      if (tn < NTI) {
        const int c = tn * 16 + li;
        const bool cv = c < NCI;
        const int cs_ = cv ? c / (NV * TE) : 0, ck = cv ? (c / TE) % NV : 0, ce = cv ? c % TE : 0;
        const T* X = (DUAL && cs_ == 1) ? sv : su;
        T bv[KB4];   // B operands of this lane: X(i = 4 kb + lk, c)
#pragma unroll
        for (int kb = 0; kb < KB4; ++kb) {
          const int i = 4 * kb + lk;
          bv[kb] = (cv && i < NB) ? X[(ck * NB + i) * TE + ce] : T(0);
        }
#pragma unroll
        for (int rt = 0; rt < NRT; ++rt) {
          typename Mfma16<T>::v4 cq = typename Mfma16<T>::v4{T(0), T(0), T(0), T(0)};
#pragma unroll
          for (int kb = 0; kb < KB4; ++kb) cq = Mfma16<T>::mma(av[rt][kb], bv[kb], cq);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int q = 16 * rt + Mfma16<T>::row(lane, r);
            if (cv && q < NQ) sw[uix(cs_, ck, q, ce)] = cq[r];
          }
        }
      }
    }
    __syncthreads();
    constexpr int NVI = (NQ * TE + NT - 1) / NT;
    S Ur[NVI][NV];
#pragma unroll
    for (int it = 0; it < NVI; ++it) {
      const int t = tid + it * NT;
      if (t < NQ * TE) {
        const int q = t / TE, e = t % TE;
        const T rs = s_inv(g_det(e));
#pragma unroll
        for (int k = 0; k < NV; ++k) {
          if constexpr (DUAL) {
            Ur[it][k].v = sw[uix(0, k, q, e)] * rs;
            Ur[it][k].d[0] = sw[uix(1, k, q, e)] * rs;
          } else {
            Ur[it][k] = sw[uix(0, k, q, e)] * rs;
          }
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < NVI; ++it) {
      const int t = tid + it * NT;
      if (t < NQ * TE) {
        const int q = t / TE, e = t % TE;
        if (e0 + e < nE) vol_flux(q, e, Ur[it]);
      }
    }
  } else {
    for (int t = tid; t < NQ * TE; t += NT) {
      const int q = t / TE, e = t % TE, ge = e0 + e;
      if (ge >= nE) continue;
      const T rs = s_inv(g_det(e));
      S U[NV];
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        T a = T(0), b = T(0);
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          const T bq = tB[q * NB + i];
          a += su[(k * NB + i) * TE + e] * bq;
          if (DUAL) b += sv[(k * NB + i) * TE + e] * bq;
        }
        if constexpr (DUAL) {
          U[k].v = a * rs;
          U[k].d[0] = b * rs;
        } else {
          U[k] = a * rs;
        }
      }
      vol_flux(q, e, U);
    }
  }
  __syncthreads();
  // ---- compact list of the face incidences (see flist)
  if constexpr (DEDUP) {
    const int lane = tid & 63, w = tid >> 6;
    const int cls = tid < NF * TE ? fcls[tid] : 3;
    int pos = 0, base = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      int before = 0;
#pragma unroll
      for (int q = 0; q < NT / 64; ++q) before += q < w ? fcnt[q][c] : 0;
      const unsigned long long m = __ballot(cls == c);
      if (cls == c) pos = base + before + __popcll(m & ((1ull << lane) - 1ull));
      base += ftot(c);
    }
    if (cls < 3) flist[pos] = (unsigned short)tid;
  }
  if constexpr (Tl::VMFMA) {
    // R_k = Dg^T F_k for every variable k: rows i < NB, columns c = k TE + e,
    // contraction over kappa = r NQ + q (F_k(kappa, e) = sw[vix(q, k, r, e)]),
    // one 16-column tile per wave at a time, 4 kappa per product.  The
    // results stay in registers until every wave has read the fluxes, then
    // go to the front of sw, from where the output threads take them.
    constexpr int KV = D * NQ, KV4 = (KV + 3) / 4 * 4, NCOL = NV * TE, NTN = (NCOL + 15) / 16;
    constexpr int NW_ = NT / 64, MT = (NTN + NW_ - 1) / NW_;
    static_assert(NVB * TE <= Tl::NW * TE, "contraction result must fit the flux scratch");
    const int lane = tid & 63, li = lane & 15, lk = lane >> 4, wid = tid >> 6;
    typename Mfma16<T>::v4 r4[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int tn = wid + mt * NW_;
      r4[mt] = typename Mfma16<T>::v4{T(0), T(0), T(0), T(0)};
      if (tn < NTN) {
        const int c = tn * 16 + li;
        const bool cv = c < NCOL;
        const int ck = cv ? c / TE : 0, ce = cv ? c % TE : 0;
        for (int k0 = 0; k0 < KV4; k0 += 4) {
          const int kap = k0 + lk, r = kap / NQ, q = kap % NQ;
          const bool kv = kap < KV;
          const T a = (li < NB && kv) ? tDg[(q * NB + li) * D + r] : T(0);
          const T b = (cv && kv) ? sw[(ck * KV + kap) * TE + ce] : T(0);
          r4[mt] = Mfma16<T>::mma(a, b, r4[mt]);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int tn = wid + mt * NW_;
      const int c = tn * 16 + li;
      if (tn < NTN && c < NCOL) {
        const int ck = c / TE, ce = c % TE;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = Mfma16<T>::row(lane, r);
          if (i < NB) sw[(ck * NB + i) * TE + ce] = r4[mt][r];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
      const int t = tid + o * NT;
      if (t < NITEM) {
        const int kg = t / TE, e = t % TE, k = kg / NG, g = kg % NG;
#pragma unroll
        for (int c = 0; c < NI; ++c) acc[o][c] = sw[(k * NB + g + NG * c) * TE + e];
      }
    }
  } else {
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
      const int t = tid + o * NT;
      if (t < NITEM) {
        const int kg = t / TE, e = t % TE, k = kg / NG, g = kg % NG;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
          for (int r = 0; r < D; ++r) {
            const T fv = sw[vix(q, k, r, e)];
#pragma unroll
            for (int c = 0; c < NI; ++c) acc[o][c] += fv * tDg[(q * NB + g + NG * c) * D + r];
          }
      }
    }
  }
  __syncthreads();

  // ---- neighbour traces: item (k, f, e) takes the coefficients of variable
  // k of the neighbour across face f of element e -- from LDS when it lies
  // in the tile, else from global memory -- and evaluates them at the face
  // points (the face items below read them from LDS).  With DEDUP the items
  // are (k, j) for the list entries j < nA + nB (classes 0 and 1).
  {
    const int nA = DEDUP ? ftot(0) : 0, nAB = DEDUP ? nA + ftot(1) : NF * TE;
    // rounds bounded at compile time (a loop with a run-time bound costs the
    // face phase below 30-60 registers)
    constexpr int NIT = (NV * NF * TE + NT - 1) / NT;
#pragma unroll 1
    for (int it = 0; it < NIT; ++it) {
      const int t = tid + it * NT;
      if (t >= NV * nAB) break;
      int k = 0, j = t, f, e;
      if constexpr (DEDUP) {
        while (j >= nAB) {
          j -= nAB;
          ++k;
        }
        const int ent = flist[j];
        f = ent / TE;
        e = ent % TE;
      } else {
        const int kf = t / TE;
        e = t % TE;
        k = kf / NF;
        f = kf % NF;
        if (e0 + e >= nE) continue;
      }
      const int nb = g_nbr(e, f);
      if (!DEDUP && nb < 0) continue;
      const int info = g_info(e, f);
      const int fN = info & 3, oN = (info >> 2) & 7;
      T cu[NB], cv[NB], rsn;
      if (DEDUP && j < nA) {
        const int en = nb - e0;
        rsn = s_inv(l_det(en));
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          cu[i] = su[(k * NB + i) * TE + en];
          cv[i] = DUAL ? sv[(k * NB + i) * TE + en] : T(0);
        }
      } else {
        rsn = s_inv(prm.sdet[nb]);
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          T uu = io.u[(size_t)(k * NB + i) * Epad + nb];
          T vv = T(0);
          if constexpr (MODE != MODE_RES) vv = io.v[(size_t)(k * NB + i) * Epad + nb] * scale;
          if (MODE == MODE_FD) uu = uu + eps * vv;
          cu[i] = uu;
          cv[i] = vv;
        }
      }
#pragma unroll
      for (int r = 0; r < NFQ; ++r) {
        const T* br = tBf + ((fN * NORI + oN) * NFQ + r) * NB;
        T a = T(0), b = T(0);
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          a += cu[i] * br[i];
          if (DUAL) b += cv[i] * br[i];
        }
        sw[fix(k, f * NFQ + r, e)] = a * rsn;
        if (DUAL) sw[fix(NV + k, f * NFQ + r, e)] = b * rsn;
      }
    }
  }
  __syncthreads();

  // ---- faces: traces and the numerical flux, item (f, r, e) for point r of
  // face f of element e (each face computed by both sides), or with DEDUP
  // item (r, j) for point r of list entry j: a face whose two elements lie
  // in the tile is then evaluated once, by the side of smaller index, which
  // also writes the neighbour's term: both sides parametrise the face by the
  // same points, the normals are opposite, and the Roe and Lax-Friedrichs
  // fluxes are antisymmetric, F(U_N, U_E, -n) = -F(U_E, U_N, n), so the
  // neighbour's value at point r is -F weighted by its own face weight.
  {
    const int nA = DEDUP ? ftot(0) : 0, nT = DEDUP ? nA + ftot(1) + ftot(2) : NF * TE;
    constexpr int NIT = (NF * NFQ * TE + NT - 1) / NT;
#pragma unroll 1
    for (int it = 0; it < NIT; ++it) {
      const int t = tid + it * NT;
      if (t >= NFQ * nT) break;
      int r = 0, j = t, f, e;
      if constexpr (DEDUP) {
        while (j >= nT) {
          j -= nT;
          ++r;
        }
        const int ent = flist[j];
        f = ent / TE;
        e = ent % TE;
      } else {
        const int fr_ = t / TE;
        e = t % TE;
        f = fr_ / NFQ;
        r = fr_ % NFQ;
        if (e0 + e >= nE) continue;
      }
      const int fr = f * NFQ + r;
      const int info = g_info(e, f);
      const int nb = g_nbr(e, f);
      const int oE = (info >> 5) & 7;
      const bool pair = DEDUP && j < nA;   // class 0: the neighbour's term too
      const int en = pair ? nb - e0 : 0, fN = info & 3, oN = (info >> 2) & 7;
      if (r == 0) {
        sori[f * TE + e] = (unsigned char)oE;
        if (pair) sori[fN * TE + en] = (unsigned char)oN;
      }
      const T sd = DEDUP ? l_det(e) : g_det(e);
      const T rs = s_inv(sd);
      const T* bl = tBf + ((f * NORI + oE) * NFQ + r) * NB;
      S UL[NV], UR[NV];
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        T a = T(0), b = T(0);
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          a += su[(k * NB + i) * TE + e] * bl[i];
          if (DUAL) b += sv[(k * NB + i) * TE + e] * bl[i];
        }
        if constexpr (DUAL) {
          UL[k].v = a * rs;
          UL[k].d[0] = b * rs;
        } else {
          UL[k] = a * rs;
        }
      }
      // |f| n = det(A) A^{-T} nref_f
      T nl[D];
      T len2 = T(0);
#pragma unroll
      for (int c = 0; c < D; ++c) {
        T s_ = T(0);
#pragma unroll
        for (int rr = 0; rr < D; ++rr) s_ += (DEDUP ? l_ainv(e, rr * D + c) : g_ainv(e, rr * D + c)) * tnref[f * D + rr];
        nl[c] = s_ * sd * sd;
        len2 += nl[c] * nl[c];
      }
      const T len = s_sqrt(len2);
      const T ilen = s_inv(len);
      T n[D];
#pragma unroll
      for (int c = 0; c < D; ++c) n[c] = nl[c] * ilen;
      if (nb >= 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
          if constexpr (DUAL) {
            UR[k].v = sw[fix(k, fr, e)];
            UR[k].d[0] = sw[fix(NV + k, fr, e)];
          } else {
            UR[k] = sw[fix(k, fr, e)];
          }
        }
      } else if (((info >> 8) & 3) == 1) {
        ghost_slip<D>(UL, n, UR);
      } else {
        ghost_farfield<D>(UL, n, prm.ff, prm.gamma, UR);
      }
      S F[NV];
      num_flux<D, FLUX>(UL, UR, n, prm.gamma, F);
      const T wl = twf[r] * len;
      const T wgt = wl * rs;
#pragma unroll
      for (int k = 0; k < NV; ++k) sw[fix(k, fr, e)] = wgt * Part<S>::get(F[k]);
      if (pair) {
        const T wgn = -(wl * s_inv(l_det(en)));
#pragma unroll
        for (int k = 0; k < NV; ++k) sw[fix(k, fN * NFQ + r, en)] = wgn * Part<S>::get(F[k]);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int o = 0; o < NOUT; ++o) {
    const int t = tid + o * NT;
    if (t < NITEM) {
      const int kg = t / TE, e = t % TE, k = kg / NG, g = kg % NG;
      if (e0 + e < nE) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          const T* bl = tBf + (f * NORI + sori[f * TE + e]) * NFQ * NB;
#pragma unroll
          for (int r = 0; r < NFQ; ++r) {
            const T fv = sw[fix(k, f * NFQ + r, e)];
#pragma unroll
            for (int c = 0; c < NI; ++c) acc[o][c] -= fv * bl[r * NB + g + NG * c];
          }
        }
      }
    }
  }

  // ---- write (padding elements get zeros)
  T wo[NOUT][NI];
#pragma unroll
  for (int o = 0; o < NOUT; ++o) {
    const int t = tid + o * NT;
#pragma unroll
    for (int c = 0; c < NI; ++c) wo[o][c] = T(0);
    if (t < NITEM) {
      const int kg = t / TE, e = t % TE, k = kg / NG, g = kg % NG, ge = e0 + e;
      if (ge < Epad) {
#pragma unroll
        for (int c = 0; c < NI; ++c) {
          const int ki = k * NB + g + NG * c;
          T v = ge < nE ? acc[o][c] : T(0);
          if (MODE == MODE_FD && ge < nE) v = (v - io.rbase[(size_t)ki * Epad + ge]) / eps;
          io.out[(size_t)ki * Epad + ge] = v;
          wo[o][c] = v;
        }
      }
    }
  }

  // ---- the Arnoldi reduction over this tile (DGIO::gsV)
  if constexpr (MODE != MODE_RES) {
    if (io.gsV != nullptr) {
      constexpr int NE = NOUT * NI;
      // chunk width: as wide as the epilogue's registers stay within the body's
      constexpr int CB = (MODE == MODE_TAN && sizeof(T) == 8 && NE <= 3) ? 8 : NE >= 8 ? 2 : 4;
      // the per-wave rows reuse the flux scratch, free once every wave has left the lift
      static_assert(sizeof(sw) >= (NT / 64) * GS_ROW * sizeof(double), "flux scratch holds the reduction rows");
      double* gsred = reinterpret_cast<double*>(sw);
      __syncthreads();
      int gix[NE];
      double gu[NE], gw[NE];
#pragma unroll
      for (int o = 0; o < NOUT; ++o) {
        const int t = tid + o * NT;
        const int tc = t < NITEM ? t : 0;
        const int kg = tc / TE, e = tc % TE, k = kg / NG, g = kg % NG, ge = e0 + e;
        const bool live = t < NITEM && ge < nE;
#pragma unroll
        for (int c = 0; c < NI; ++c) {
          const int ix = live ? (k * NB + g + NG * c) * Epad + ge : 0;
          gix[o * NI + c] = ix;
          gu[o * NI + c] = live ? (double)io.v[ix] : 0.0;
          gw[o * NI + c] = live ? (double)wo[o][c] : 0.0;
        }
      }
      gs_tile_dots<NT, NE, CB>(io.gsV, io.gsld, io.gsj, gix, gu, gw, io.gspart, io.gspld, gsred);
    }
  }
}

// ---------------------------------------------------------------------------
// Transpose: out = J(u)^T w, gathered element by element (no atomics).  For
// element E the contributions are (a) the adjoint of its own volume term,
// (b) the adjoint of its own face terms with respect to its trace U_L, and
// (c) for each interior face, the adjoint of the neighbour N's face term
// F~(U_N, U_E, n_N) with respect to its second argument, evaluated with N's
// own geometry exactly as N's forward residual does.  Flux Jacobians come from
// forward-mode Dual<ST, NV> numbers seeded on the state being differentiated.
//
// ST = double gives J(u)^T w.  ST = Dual<double, 1> runs the same code on the
// state u + eps v: the value part is J(u)^T w and the eps part is
// d/deps [J(u + eps v)^T w] = (d_u [J(u) v])^T w, the second-order term of the
// reverse sweep through an Arnoldi process whose operator depends on u.
template <typename ST> struct StateScalar;
template <> struct StateScalar<double> {
  static constexpr bool SECOND = false;
  __device__ static double make(double u, double) { return u; }
  __device__ static double value(double x) { return x; }
  __device__ static double deriv(double) { return 0.0; }
};
template <> struct StateScalar<Dual<double, 1>> {
  static constexpr bool SECOND = true;
  __device__ static Dual<double, 1> make(double u, double v) {
    Dual<double, 1> r;
    r.v = u;
    r.d[0] = v;
    return r;
  }
  __device__ static double value(const Dual<double, 1>& x) { return x.v; }
  __device__ static double deriv(const Dual<double, 1>& x) { return x.d[0]; }
};

template <int D, int P, int FLUX, typename ST>
struct VjpTile {
  using Sh = Shape<D, P>;
  static constexpr int NX = (Sh::NQ > Sh::NF * Sh::NFQ ? Sh::NQ : Sh::NF * Sh::NFQ) * Sh::NV;
  static constexpr int per_elem = (int)sizeof(ST) * (Sh::NVB + NX) + 8 * Sh::NVB + Sh::NF;
  // derivative directions per face-flux evaluation: the whole Jacobian at
  // once for first order; one column at a time for the nested second-order
  // scalars, whose NV-direction form of the numerical flux does not fit the
  // register file (the lighter physical flux of the volume term takes all
  // NV directions in one pass in both cases)
  static constexpr int NC = std::is_same<ST, double>::value ? Sh::NV : 1;
  // As for the forward tiles: the fewest rounds of the two pointwise phases
  // (NQ TE and NF NFQ TE items over 256 threads) per element under the LDS
  // budget, the smallest tile among equals (2D P2: 28 elements, one round
  // each, instead of 32 with a second round of 32 items).
  static constexpr int rounds(int te) {
    return (Sh::NQ * te + 255) / 256 + (Sh::NF * Sh::NFQ * te + 255) / 256;
  }
  static constexpr int pick() {
    int best = 1;
    for (int te = 2; te <= 64; ++te) {
      if (te * per_elem > kLdsBudget) break;
      if (rounds(te) * best < rounds(best) * te) best = te;
    }
    return best;
  }
  static constexpr int TE = pick();
};

template <int D, int P, int FLUX, typename ST>
__global__ __launch_bounds__(256) void dg_vjp_kernel(DGParams<double> prm, const double* __restrict__ u,
                                                     const double* __restrict__ vdir,
                                                     const double* __restrict__ w, double* __restrict__ out,
                                                     double* __restrict__ out_d, const double* acc_scale) {
  using T = double;
  using SS = StateScalar<ST>;
  using Sh = Shape<D, P>;
  constexpr int NV = Sh::NV, NB = Sh::NB, NVB = Sh::NVB, NQ = Sh::NQ, NFQ = Sh::NFQ;
  constexpr int NF = Sh::NF, NORI = Sh::NORI;
  constexpr int TE = VjpTile<D, P, FLUX, ST>::TE;
  constexpr int NX = VjpTile<D, P, FLUX, ST>::NX;
  constexpr int NT = 256;
  constexpr int NOUT = (NVB * TE + NT - 1) / NT;
  constexpr int NC = VjpTile<D, P, FLUX, ST>::NC;
  using SD = Dual<ST, NC>;
  // The face terms' passes over the derivative directions are kept apart
  // (not unrolled) so that only one pass's duals are live; Ub is indexed
  // through selects.
  auto add_dir = [](ST* Ub, int j, ST x) {
#pragma unroll
    for (int jj = 0; jj < NV; ++jj)
      if (jj == j) Ub[jj] = Ub[jj] + x;
  };
  // U_k with derivative directions j0 .. j0 + NC - 1 seeded on the state
  auto seed = [](const ST* val, int j0, SD* U) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      U[k].v = val[k];
#pragma unroll
      for (int c = 0; c < NC; ++c) U[k].d[c] = ST((k == j0 + c) ? 1.0 : 0.0);
    }
  };

  __shared__ ST su[NVB * TE];
  __shared__ T sw[NVB * TE];
  __shared__ ST sx[NX * TE];
  __shared__ unsigned char sori[NF * TE];

  const int Epad = prm.Epad, nE = prm.nE;
  const int e0 = xcd_tile(blockIdx.x, gridDim.x) * TE;
  const int tid = threadIdx.x;
  const T gm1 = prm.gamma - T(1);

  for (int t = tid; t < NVB * TE; t += NT) {
    const int ki = t / TE, e = t % TE, ge = e0 + e;
    const bool in = ge < nE;
    su[t] = SS::make(in ? u[(size_t)ki * Epad + ge] : T(0), (SS::SECOND && in) ? vdir[(size_t)ki * Epad + ge] : T(0));
    sw[t] = in ? w[(size_t)ki * Epad + ge] : T(0);
  }
  __syncthreads();
  ST acc[NOUT];
#pragma unroll
  for (int o = 0; o < NOUT; ++o) acc[o] = ST(0);

  // ---- (a) volume adjoint
  for (int t = tid; t < NQ * TE; t += NT) {
    const int q = t / TE, e = t % TE, ge = e0 + e;
    if (ge >= nE) continue;
    const T sd = prm.sdet[ge], rs = T(1) / sd;
    ST Uv[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      ST a = ST(0);
#pragma unroll
      for (int i = 0; i < NB; ++i) a = a + su[(k * NB + i) * TE + e] * prm.B[q * NB + i];
      Uv[k] = a * rs;
    }
    T gb[D][NV];   // test-function weights of the volume term
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        T g = T(0);
#pragma unroll
        for (int i = 0; i < NB; ++i) g += sw[(k * NB + i) * TE + e] * prm.Dg[(q * NB + i) * D + r];
        gb[r][k] = g * sd * prm.wq[q];
      }
    ST Ub[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) Ub[j] = ST(0);
    {
      // every state component seeded at once: the physical flux is light
      // enough for NV directions of the nested scalars
      using SDV = Dual<ST, NV>;
      SDV U[NV];
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        U[k].v = Uv[k];
#pragma unroll
        for (int c = 0; c < NV; ++c) U[k].d[c] = ST(k == c ? 1.0 : 0.0);
      }
#pragma unroll
      for (int r = 0; r < D; ++r) {
        T a[D];
#pragma unroll
        for (int c = 0; c < D; ++c) a[c] = prm.ainv[(size_t)(r * D + c) * Epad + ge];
        SDV F[NV];
        normal_flux<D>(U, a, gm1, F);
#pragma unroll
        for (int c = 0; c < NV; ++c) {
          ST x = ST(0);
#pragma unroll
          for (int k = 0; k < NV; ++k) x = x + F[k].d[c] * gb[r][k];
          Ub[c] = Ub[c] + x;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < NV; ++j) sx[(q * NV + j) * TE + e] = Ub[j] * rs;
  }
  __syncthreads();
#pragma unroll
  for (int o = 0; o < NOUT; ++o) {
    const int t = tid + o * NT;
    if (t < NVB * TE) {
      const int ki = t / TE, e = t % TE, k = ki / NB, i = ki % NB;
      ST s = ST(0);
#pragma unroll
      for (int q = 0; q < NQ; ++q) s = s + sx[(q * NV + k) * TE + e] * prm.B[q * NB + i];
      acc[o] = acc[o] + s;
    }
  }
  __syncthreads();

  // ---- (b) own face terms and (c) neighbours' face terms
  for (int t = tid; t < NF * NFQ * TE; t += NT) {
    const int fr = t / TE, e = t % TE, f = fr / NFQ, r = fr % NFQ, ge = e0 + e;
    if (ge >= nE) continue;
    const int info = prm.finfo[(size_t)f * Epad + ge];
    const int nb = prm.nbr[(size_t)f * Epad + ge];
    const int oE = (info >> 5) & 7;
    if (r == 0) sori[f * TE + e] = (unsigned char)oE;
    const T sd = prm.sdet[ge], rs = T(1) / sd;
    const T* bl = prm.Bf + ((f * NORI + oE) * NFQ + r) * NB;
    ST UEv[NV];
    T wl[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      ST a = ST(0);
      T b = T(0);
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        a = a + su[(k * NB + i) * TE + e] * bl[i];
        b += sw[(k * NB + i) * TE + e] * bl[i];
      }
      UEv[k] = a * rs;
      wl[k] = b;
    }
    T nl[D], len2 = T(0);
#pragma unroll
    for (int c = 0; c < D; ++c) {
      T s = T(0);
#pragma unroll
      for (int rr = 0; rr < D; ++rr) s += prm.ainv[(size_t)(rr * D + c) * Epad + ge] * prm.nref[f * D + rr];
      nl[c] = s * sd * sd;
      len2 += nl[c] * nl[c];
    }
    const T len = s_sqrt(len2);
    const T ilen = s_inv(len);
    T n[D];
#pragma unroll
    for (int c = 0; c < D; ++c) n[c] = nl[c] * ilen;
    ST Ub[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) Ub[j] = ST(0);
    const T cs = -prm.wf[r] * len * rs;   // seed scale of the own face term
    if (nb >= 0) {
      const int fN = info & 3, oN = (info >> 2) & 7;
      const T* br = prm.Bf + ((fN * NORI + oN) * NFQ + r) * NB;
      const T sN = prm.sdet[nb], rsN = T(1) / sN;
      ST UNv[NV];
      T wn[NV];
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        ST a = ST(0);
        T b = T(0);
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          const size_t g = (size_t)(k * NB + i) * Epad + nb;
          a = a + SS::make(u[g], SS::SECOND ? vdir[g] : T(0)) * br[i];
          b += w[g] * br[i];
        }
        UNv[k] = a * rsN;
        wn[k] = b;
      }
      // neighbour's own geometry: |f|_N n_N = det(A_N) A_N^{-T} nref_{fN}
      T nN[D], l2N = T(0);
#pragma unroll
      for (int c = 0; c < D; ++c) {
        T s = T(0);
#pragma unroll
        for (int rr = 0; rr < D; ++rr) s += prm.ainv[(size_t)(rr * D + c) * Epad + nb] * prm.nref[fN * D + rr];
        nN[c] = s * sN * sN;
        l2N += nN[c] * nN[c];
      }
      const T lenN = s_sqrt(l2N);
      const T cn = -prm.wf[r] * lenN * rsN;
      // The neighbour's term F~(U_N, U_E, n_N) at the same physical point,
      // with n_N = -n on the shared straight face, equals -F~(U_E, U_N, n)
      // (both fluxes are antisymmetric), so one flux evaluation seeded on
      // U_E serves the own term (weight cs wl) and the neighbour's (weight
      // -cn wn); the face lengths |f| and |f|_N stay each side's own.
      T wc[NV];
#pragma unroll
      for (int k = 0; k < NV; ++k) wc[k] = cs * wl[k] - cn * wn[k];
#pragma unroll 1
      for (int j0 = 0; j0 < NV; j0 += NC) {
        SD UE[NV], UN[NV], F[NV];
        seed(UEv, j0, UE);
#pragma unroll
        for (int k = 0; k < NV; ++k) UN[k] = mkconst<ST, NC>(UNv[k]);
        num_flux<D, FLUX>(UE, UN, n, prm.gamma, F);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          ST x = ST(0);
#pragma unroll
          for (int k = 0; k < NV; ++k) x = x + F[k].d[c] * wc[k];
          add_dir(Ub, j0 + c, x);
        }
      }
    } else {
#pragma unroll 1
      for (int j0 = 0; j0 < NV; j0 += NC) {
        SD UE[NV], G[NV], F[NV];
        seed(UEv, j0, UE);
        if (((info >> 8) & 3) == 1) ghost_slip<D>(UE, n, G);
        else ghost_farfield<D>(UE, n, prm.ff, prm.gamma, G);
        num_flux<D, FLUX>(UE, G, n, prm.gamma, F);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          ST x = ST(0);
#pragma unroll
          for (int k = 0; k < NV; ++k) x = x + F[k].d[c] * (cs * wl[k]);
          add_dir(Ub, j0 + c, x);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < NV; ++j) sx[((f * NFQ + r) * NV + j) * TE + e] = Ub[j] * rs;
  }
  __syncthreads();
#pragma unroll
  for (int o = 0; o < NOUT; ++o) {
    const int t = tid + o * NT;
    if (t < NVB * TE) {
      const int ki = t / TE, e = t % TE, k = ki / NB, i = ki % NB, ge = e0 + e;
      if (ge < nE) {
        ST s = ST(0);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          const T* bl = prm.Bf + (f * NORI + sori[f * TE + e]) * NFQ * NB;
#pragma unroll
          for (int r = 0; r < NFQ; ++r) s = s + sx[((f * NFQ + r) * NV + k) * TE + e] * bl[r * NB + i];
        }
        acc[o] = acc[o] + s;
      }
      if (acc_scale) {
        // accumulate (second order only): out += value, out_d += s deriv
        if (SS::SECOND && ge < nE) {
          const size_t g = (size_t)ki * Epad + ge;
          out[g] = out[g] + SS::value(acc[o]);
          out_d[g] = out_d[g] + (*acc_scale) * SS::deriv(acc[o]);
        }
      } else if (ge < Epad) {
        out[(size_t)ki * Epad + ge] = ge < nE ? SS::value(acc[o]) : T(0);
        if (SS::SECOND) out_d[(size_t)ki * Epad + ge] = ge < nE ? SS::deriv(acc[o]) : T(0);
      }
    }
  }
}

template <int D, int P, int FLUX>
void launch_vjp(const DGParams<double>& prm, const double* u, const double* w, double* out, hipStream_t st) {
  constexpr int TE = VjpTile<D, P, FLUX, double>::TE;
  launch((dg_vjp_kernel<D, P, FLUX, double>), dim3((prm.Epad + TE - 1) / TE), dim3(256), 0, st, prm, u,
         (const double*)nullptr, w, out, (double*)nullptr, (const double*)nullptr);
}

// out = J(u)^T w and out_d = d/deps [J(u + eps v)^T w] in one pass (with
// acc_scale: out += J(u)^T w, out_d += (*acc_scale) d/deps [...]).
template <int D, int P, int FLUX>
void launch_vjp2(const DGParams<double>& prm, const double* u, const double* v, const double* w, double* out,
                 double* out_d, const double* acc_scale, hipStream_t st) {
  constexpr int TE = VjpTile<D, P, FLUX, Dual<double, 1>>::TE;
  launch((dg_vjp_kernel<D, P, FLUX, Dual<double, 1>>), dim3((prm.Epad + TE - 1) / TE), dim3(256), 0, st, prm, u,
         v, w, out, out_d, acc_scale);
}

// Host launchers (defined in the per-dimension translation units).
template <int D, int P, int FLUX, typename T, int MODE>
void launch_dg(const DGParams<T>& prm, const DGIO<T>& io, hipStream_t st) {
  using Tl = Tile<D, P, T, MODE == MODE_TAN>;
  constexpr int TE = Tl::TE, NT = Tl::NT;
  const int nblk = (prm.Epad + TE - 1) / TE;   // the last tile may run past Epad: guarded in the kernel
  launch((dg_apply<D, P, FLUX, T, MODE, TE, NT>), dim3(nblk), dim3(NT), 0, st, prm, io);
}

}  // namespace pcexp
