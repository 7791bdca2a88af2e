// libpcexp: C ABI (include/pcexp.h) and host orchestration of the PCEXP step.
//
// Paper anchors: Sec. 2.1 eqs. (starteq), (s8), (s9), (s10) (PCEXP and EXP1);
// Sec. 2.2 eqs. (vm)-(final) (Krylov evaluation of phi_k); Sec. 4 (DG
// residual and exact Jacobian); Sec. 5 eq. (x3d) (time step).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/pcexp.h"
#include "dg_dispatch.hpp"
#include "krylov_kernels.hpp"
#include "launch.hpp"
#include "setup.hpp"

namespace pcexp {
thread_local LaunchTiming g_launch_timing;
}  // namespace pcexp

// Workspace of pcexp_step_noalloc: a fixed array in device memory, one copy
// per GPU the library runs on, held until the process ends.  Host code never
// uses this name as an address (on the host it is only a stand-in for the
// symbol); it takes the device address from hipGetSymbolAddress once per
// device, at context creation with that device current.
constexpr size_t kNoallocBytes = (size_t)PCEXP_NOALLOC_WS_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch` on each device

// Device address of this device's copy of `scratch` (looked up once per device).
hipError_t noalloc_scratch(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}
}  // namespace

using namespace pcexp;

namespace {

constexpr int TILE_PAD = 64;
constexpr size_t ALIGN = 256;

size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

template <typename T>
struct DevBuf {
  T* p = nullptr;
};

}  // namespace

struct pcexp_ctx {
  bool dense = false;
  int dim = 0, p = 0, nv = 1, nb = 1, nq = 0, nfq = 0, nf = 0, nori = 0, flux = 0;
  int64_t nE = 0, Epad = 0;
  size_t K = 0;      // ABI length
  size_t Kint = 0;   // internal length (nv * nb * Epad, or n for dense)
  size_t Kld = 0;    // stride of Krylov vectors
  double gamma = 1.4, ff[5] = {0, 0, 0, 0, 0};
  double volume_total = 0.0;
  double krylov_tol = 0.0;   // > 0: stage-1 dt control by the Krylov error estimate
  int krylov_every = 0;      // > 0 (with krylov_tol): adaptive dimension, checked every krylov_every iterations
  // tables and geometry
  double *B = nullptr, *Dg = nullptr, *wq = nullptr, *Bf = nullptr, *wf = nullptr, *nref = nullptr,
         *Bc = nullptr, *refp = nullptr;
  float *B32 = nullptr, *Dg32 = nullptr, *wq32 = nullptr, *Bf32 = nullptr, *wf32 = nullptr,
        *nref32 = nullptr;
  double *ainv = nullptr, *sdet = nullptr, *x0 = nullptr, *amat = nullptr, *hE = nullptr, *Q = nullptr;
  float *ainv32 = nullptr, *sdet32 = nullptr;
  int *nbr = nullptr, *finfo = nullptr, *perm = nullptr;
  // dense operator
  double *Ajac = nullptr, *Ares = nullptr;
  float* Ajac32 = nullptr;
  // context-owned scratch for single-shot calls
  double* io[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  float* io32[2] = {nullptr, nullptr};
  double* part = nullptr;
  size_t part_len = 0;
  KState* ks = nullptr;
  double* scal = nullptr;     // small device scalars
  unsigned* flags = nullptr;
  unsigned* counters = nullptr;
  std::vector<void*> allocs;
  std::string err;
  // kernel-class timing (pcexp_profile)
  bool prof = false;
  std::vector<hipEvent_t> ev;
  struct Rec { int cls; double bytes; int e0; };
  std::vector<Rec> recs;
  hipStream_t prof_stream = nullptr;
  // device the context was created on, and that device's no-allocation workspace
  int device = -1;
  void* noalloc_ws = nullptr;
};

namespace {

pcexp_status fail(pcexp_ctx* c, pcexp_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

template <typename T>
bool dalloc(pcexp_ctx* c, T** p, size_t n) {
  if (n == 0) n = 1;
  if (hipMalloc((void**)p, n * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    return false;
  }
  c->allocs.push_back((void*)*p);
  return true;
}

template <typename T>
bool upload(pcexp_ctx* c, T** p, const std::vector<T>& v, hipStream_t st) {
  if (!dalloc(c, p, v.size())) return false;
  return hipMemcpyAsync(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st) == hipSuccess;
}

template <typename T>
bool upload32(pcexp_ctx* c, float** p, const std::vector<T>& v, hipStream_t st) {
  std::vector<float> f(v.begin(), v.end());
  return upload(c, p, f, st);
}

pcexp_status hip_check(pcexp_ctx* c, const char* where) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, PCEXP_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
  return PCEXP_OK;
}

DGParams<double> params_d(const pcexp_ctx* c) {
  DGParams<double> p;
  p.B = c->B; p.Dg = c->Dg; p.wq = c->wq; p.Bf = c->Bf; p.wf = c->wf; p.nref = c->nref;
  p.ainv = c->ainv; p.sdet = c->sdet; p.nbr = c->nbr; p.finfo = c->finfo;
  p.nE = (int)c->nE; p.Epad = (int)c->Epad; p.gamma = c->gamma;
  for (int k = 0; k < 5; ++k) p.ff[k] = c->ff[k];
  return p;
}

DGParams<float> params_f(const pcexp_ctx* c) {
  DGParams<float> p;
  p.B = c->B32; p.Dg = c->Dg32; p.wq = c->wq32; p.Bf = c->Bf32; p.wf = c->wf32; p.nref = c->nref32;
  p.ainv = c->ainv32; p.sdet = c->sdet32; p.nbr = c->nbr; p.finfo = c->finfo;
  p.nE = (int)c->nE; p.Epad = (int)c->Epad; p.gamma = (float)c->gamma;
  for (int k = 0; k < 5; ++k) p.ff[k] = (float)c->ff[k];
  return p;
}

ElemArgs elem_args(const pcexp_ctx* c) {
  ElemArgs a;
  a.dim = c->dim; a.nv = c->nv; a.nb = c->nb; a.nq = c->nq; a.p = c->p;
  a.nE = (int)c->nE; a.Epad = (int)c->Epad;
  a.Q = c->Q; a.perm = c->perm; a.sdet = c->sdet; a.x0 = c->x0; a.amat = c->amat; a.B = c->B;
  a.wq = c->wq; a.Bc = c->Bc; a.refp = c->refp; a.hE = c->hE; a.gamma = c->gamma;
  return a;
}

const double kSqrtEps = 1.4901161193847656e-08;  // sqrt(2^-52)

enum { PC_RES = 0, PC_JVP = 1, PC_GSR = 2, PC_GSF = 3, PC_GSU = 4, PC_PHI = 5, PC_COMB = 6, PC_OTHER = 7 };

// Times the one kernel launched in its scope when profiling is on (no-op
// otherwise): the event pair is handed to that launch, so it measures the
// kernel's own execution.  If no launch consumed the pair (the operation was
// skipped on the host), both events are recorded here and the interval is ~0.
struct Prof {
  pcexp_ctx* c;
  hipStream_t st;
  int idx = -1;
  Prof(pcexp_ctx* c_, hipStream_t s, int cls, double bytes) : c(c_), st(s) {
    if (!c->prof) return;
    size_t k = c->recs.size();
    if (2 * k + 1 >= c->ev.size()) return;
    idx = (int)k;
    c->recs.push_back({cls, bytes, (int)(2 * k)});
    g_launch_timing.start = c->ev[2 * k];
    g_launch_timing.stop = c->ev[2 * k + 1];
  }
  ~Prof() {
    if (idx < 0 || !g_launch_timing.start) return;
    g_launch_timing.start = g_launch_timing.stop = nullptr;
    (void)hipEventRecord(c->ev[2 * idx], st);
    (void)hipEventRecord(c->ev[2 * idx + 1], st);
  }
};

double geo_bytes(const pcexp_ctx* c, size_t w) {
  // per element: A^{-1} (d^2), sqrt(det) (1) in the compute type, neighbour + face info (2 ints per face)
  return (double)c->nE * ((c->dim * c->dim + 1) * (double)w + c->nf * 8.0);
}

// ---- internal operators --------------------------------------------------
void to_int(pcexp_ctx* c, const double* abi, double* in, hipStream_t st) {
  if (c->dense) (void)hipMemcpyAsync(in, abi, c->K * sizeof(double), hipMemcpyDeviceToDevice, st);
  else ek_to_internal(elem_args(c), abi, in, st);
}
void to_abi(pcexp_ctx* c, const double* in, double* abi, hipStream_t st) {
  if (c->dense) (void)hipMemcpyAsync(abi, in, c->K * sizeof(double), hipMemcpyDeviceToDevice, st);
  else ek_to_abi(elem_args(c), in, abi, st);
}

bool residual_int(pcexp_ctx* c, const double* u, double* R, hipStream_t st) {
  Prof pr(c, st, PC_RES, 2.0 * c->K * 8 + (c->dense ? (double)c->K * c->K * 8 : geo_bytes(c, 8)));
  if (c->dense) {
    k_gemv<double>(c->Ares, u, R, (int)c->K, nullptr, nullptr, st);
    return true;
  }
  DGIO<double> io{};
  io.u = u; io.out = R; io.flags = c->flags;
  return dg_run_d(c->dim, c->p, c->flux, MODE_RES, params_d(c), io, st);
}

// Tiles (workgroups) of the DG tangent / FD launch: its partials per column
// when the Arnoldi reduction is fused into it.
template <int D, int P>
int tile_elems(int jvp, int prec) {
  if (prec == PCEXP_PREC_MIXED) return Tile<D, P, float, true>::TE;
  return jvp == PCEXP_JVP_FD ? Tile<D, P, double, false>::TE : Tile<D, P, double, true>::TE;
}
template <int D>
int tile_elems_p(int p, int jvp, int prec) {
  switch (p) {
    case 0: return tile_elems<D, 0>(jvp, prec);
    case 1: return tile_elems<D, 1>(jvp, prec);
    case 2: return tile_elems<D, 2>(jvp, prec);
    default: return tile_elems<D, 3>(jvp, prec);
  }
}
int jvp_tiles(const pcexp_ctx* c, int jvp, int prec) {
  const int te = c->dim == 2 ? tile_elems_p<2>(c->p, jvp, prec) : tile_elems_p<3>(c->p, jvp, prec);
  return (int)((c->Epad + te - 1) / te);
}
// The reduction pass of each Arnoldi iteration runs inside the DG JVP launch
// that produced W (its tiles write partial sums, a small kernel adds them up)
// when that launch leaves HBM idle while its tiles compute fluxes: at most
// kFuseMaxTiles tiles, about four rounds of resident workgroups on 256
// compute units.  Measured: the 128 x 128 P2 vortex (1171 tiles) gains 4 %
// per step and the 384 x 128 P2 channel in FP64 (3511 tiles) 7 %; the 3D P2
// vortex (36 864 tiles), whose FP32 JVP keeps the vector ALUs busy, loses
// 5 % (streaming does not overlap, and summing that many partials per column
// costs 0.1 ms).
static_assert(KMAX <= GS_MAXQ, "the fused reduction's LDS rows hold the basis of the largest Krylov dimension");
constexpr int kFuseMaxTiles = 4096;
bool fuse_gs(const pcexp_ctx* c, int jvp, int prec) {
  return !c->dense && jvp != PCEXP_JVP_ZERO && c->Kint < ((size_t)1 << 31) &&
         jvp_tiles(c, jvp, prec) <= kFuseMaxTiles;
}
// A Gram-Schmidt pass over nvec basis vectors reads them with non-temporal
// loads when they exceed twice the 256 MB Infinity Cache, which then keeps
// nothing of them for the next pass.  Measured: the 3D P2 vortex (133 MB
// per FP32 vector) step -4 %; with the hint on every pass, the 384 x 128
// channel (9.4 MB per FP32 vector, 31 vectors) lost 9 % per mixed-precision
// iteration and the 128 x 128 vortex (6.3 MB per FP64 vector) 11 % per
// step, whose passes the cache serves in part.
constexpr size_t kMallBytes = (size_t)256 << 20;
bool basis_streams(const pcexp_ctx* c, int nvec, size_t word) {
  return (size_t)nvec * c->Kld * word > 2 * kMallBytes;
}
// Partials region: the Gram-Schmidt passes' columns (3 * 512 * (KMAX + 2)
// doubles), then room for the fused reduction's 2m + 3 columns of one partial
// per tile (at most kFuseMaxTiles).
constexpr size_t kPartStd = (size_t)3 * 512 * (KMAX + 2);
size_t part_bytes(const pcexp_ctx* c, int m) {
  const size_t tiles = c->dense ? 0 : (size_t)kFuseMaxTiles;
  return (kPartStd + (size_t)(2 * m + 3) * tiles) * sizeof(double);
}

// JVP on internal vectors.  F64: v, out double.  MIXED: u32/v/out float.
// vscale/skip optional device pointers; fd_eps device pointer for FD.  With
// gsV set (a DG context), the launch also forms the Arnoldi reduction of
// iteration gsj over the basis gsV (stride Kld) into gspart (DGIO::gsV).
bool jvp_int(pcexp_ctx* c, int jvp, int prec, const double* u, const float* u32, const void* v, void* out,
             const double* vscale, const int* skip, const double* Rbase, const double* fd_eps, hipStream_t st,
             const void* gsV = nullptr, int gsj = 0, double* gspart = nullptr, int gspld = 0) {
  const size_t n = c->Kint;
  const size_t w = (prec == PCEXP_PREC_MIXED) ? 4 : 8;
  Prof pr(c, st, PC_JVP, (jvp == PCEXP_JVP_FD ? 4.0 : 3.0) * c->K * w + (c->dense ? 0.0 : geo_bytes(c, w)) +
                             (gsV ? (double)gsj * c->K * w : 0.0));
  if (jvp == PCEXP_JVP_ZERO) {
    if (prec == PCEXP_PREC_MIXED) k_fill<float>((float*)out, 0.0f, n, skip, st);
    else k_fill<double>((double*)out, 0.0, n, skip, st);
    return true;
  }
  if (c->dense) {
    if (prec == PCEXP_PREC_MIXED) k_gemv<float>(c->Ajac32, (const float*)v, (float*)out, (int)n, vscale, skip, st);
    else k_gemv<double>(c->Ajac, (const double*)v, (double*)out, (int)n, vscale, skip, st);
    return true;
  }
  if (prec == PCEXP_PREC_MIXED) {
    DGIO<float> io{};
    io.u = u32; io.v = (const float*)v; io.out = (float*)out; io.vscale = vscale; io.skip = skip;
    io.gsV = (const float*)gsV; io.gsld = c->Kld; io.gsj = gsj; io.gspart = gspart; io.gspld = gspld;
    return dg_run_f(c->dim, c->p, c->flux, MODE_TAN, params_f(c), io, st);
  }
  DGIO<double> io{};
  io.u = u; io.v = (const double*)v; io.out = (double*)out; io.vscale = vscale; io.skip = skip;
  io.gsV = (const double*)gsV; io.gsld = c->Kld; io.gsj = gsj; io.gspart = gspart; io.gspld = gspld;
  if (jvp == PCEXP_JVP_FD) {
    io.rbase = Rbase;
    io.fd_eps = fd_eps;
    return dg_run_d(c->dim, c->p, c->flux, MODE_FD, params_d(c), io, st);
  }
  return dg_run_d(c->dim, c->p, c->flux, MODE_TAN, params_d(c), io, st);
}


// ---- workspace layout ----------------------------------------------------
struct WsLayout {
  size_t ks1, ks2, part, phi, scal, cnt, un, Rn, us, Rs, x1, un32, V, total;
};

WsLayout ws_layout(const pcexp_ctx* c, int m, int k, int prec) {
  WsLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += align_up(bytes); return o; };
  const size_t vb = c->Kint * sizeof(double);
  L.ks1 = take(sizeof(KState));
  L.ks2 = take(sizeof(KState));
  L.part = take(part_bytes(c, m));
  const size_t nphi = (size_t)(m + (k > 2 ? k : 2));   // k = 1 steps may use the (m+2) error-estimate matrix
  L.phi = take(phi_scratch_doubles((int)nphi) * sizeof(double));
  L.scal = take(64 * sizeof(double));
  L.cnt = take(64 * sizeof(unsigned));
  L.un = take(vb);
  L.Rn = take(vb);
  L.us = take(vb);
  L.Rs = take(vb);
  L.x1 = take(vb);
  L.un32 = take(prec == PCEXP_PREC_MIXED ? c->Kint * sizeof(float) : 0);
  const size_t tv = (prec == PCEXP_PREC_MIXED) ? sizeof(float) : sizeof(double);
  L.V = take((size_t)(m + 1) * c->Kld * tv);
  L.total = off;
  return L;
}

template <typename TV>
void arnoldi_run(pcexp_ctx* c, int jvp, int prec, const double* u_lin, const float* u32, const double* b,
                 const double* Rlin, double* dtp, int k, int m, KState* ks, double* part, double* phi,
                 TV* V, hipStream_t st, double tol = 0.0, bool dt_control = false, int check_every = 0) {
  const size_t n = c->Kint, ld = c->Kld;
  const double eta = (prec == PCEXP_PREC_MIXED) ? 1e-5 : 1e-12;
  k_init_state(ks, eta, st);
  if (jvp == PCEXP_JVP_FD) {
    k_sumsq(u_lin, n, &ks->norm_tmp[0], 1, part, &ks->counter[4], st);
    k_fd_eps(&ks->norm_tmp[0], nullptr, kSqrtEps, &ks->fd_eps, st);
  }
  k_start<TV>(b, V, n, ks, part, st);
  const bool fuse = fuse_gs(c, jvp, prec);
  const int fpld = fuse ? jvp_tiles(c, jvp, prec) : 0;
  double* fpart = part + kPartStd;
  for (int j = 0; j < m; ++j) {
    const double vb = (double)c->K * sizeof(TV);
    const bool nt = basis_streams(c, j + 2, sizeof(TV));
    if (fuse) {
      // JVP + reduction in one launch (it reads V_0..V_{j-1} besides its operands),
      // then the column sums of its per-tile partials
      jvp_int(c, jvp, prec, u_lin, u32, V + (size_t)j * ld, V + (size_t)(j + 1) * ld, &ks->sig_t[j], &ks->done,
              Rlin, &ks->fd_eps, st, V, j, fpart, fpld);
      { Prof pr(c, st, PC_GSR, (2.0 * j + 3.0) * fpld * 8.0); k_gs_colsum(fpart, fpld, fpld, 2 * j + 3, ks, part, st); }
      { Prof pr(c, st, PC_GSU, (j + 4.0) * vb); k_gs_update_one<TV>(V, ld, j, n, ks, part, st, nt); }
    } else {
      jvp_int(c, jvp, prec, u_lin, u32, V + (size_t)j * ld, V + (size_t)(j + 1) * ld, &ks->sig_t[j], &ks->done,
              Rlin, &ks->fd_eps, st);
      // the reduction pass reads j + 2 vectors; the finalise-and-update pass reads j + 2 and writes 2
      { Prof pr(c, st, PC_GSR, (j + 2.0) * vb); k_gs_reduce<TV>(V, ld, j, n, ks, part, false, st, nt); }
      { Prof pr(c, st, PC_GSU, (j + 4.0) * vb); k_gs_update<TV>(V, ld, j, n, ks, part, st, nt); }
    }
    // adaptive dimension: H_j is final now; stop at m_eff = j if its estimate meets tol
    if (tol > 0.0 && check_every > 0 && k == 1 && j >= 1 && j % check_every == 0) {
      Prof pr(c, st, PC_PHI, 0.0);
      k_krylov_check(ks, dtp, tol, j, phi, st);
    }
  }
  {
    Prof pr(c, st, PC_GSR, (m + 1.0) * (double)c->K * sizeof(TV));
    k_gs_reduce<TV>(V, ld, m, n, ks, part, true, st, basis_streams(c, m + 1, sizeof(TV)));
  }
  { Prof pr(c, st, PC_GSF, 0.0); k_gs_close(ks, part, m, n, st); }
  {
    Prof pr(c, st, PC_PHI, 0.0);
    if (tol > 0.0 && dt_control && k == 1) k_hess_phi_adapt(ks, dtp, tol, m, phi, st);
    else k_hess_phi(ks, dtp, k, m, phi, st);
  }
}

// ---- reverse mode ----------------------------------------------------------
// J^T w on internal vectors (with res_jac on a dense context: the residual
// matrix); if out_d is given also out_d = d/deps [J(u + eps v)^T w] (zero for
// the constant dense operators).
bool vjp_int(pcexp_ctx* c, const double* u, const double* v, const double* w, double* out, double* out_d,
             bool res_jac, hipStream_t st) {
  if (c->dense) {
    k_gemv_t(res_jac ? c->Ares : c->Ajac, w, out, (int)c->Kint, st);
    if (out_d) k_fill<double>(out_d, 0.0, c->Kint, nullptr, st);
    return true;
  }
  return c->dim == 2 ? dg_vjp2(c->p, c->flux, params_d(c), u, v, w, out, out_d, st)
                     : dg_vjp3(c->p, c->flux, params_d(c), u, v, w, out, out_d, st);
}

struct RevBufs {
  double *r, *wb, *wj, *t1, *t2;   // K-vectors
  double* Vb;                       // m adjoint basis vectors, stride Kld
  RState* rs;
  double* part;
  double* mem;                      // expm scratch, 7 (2 KMAX + 2)^2 doubles
};

// Reverse sweep through one Arnoldi run of J = J(u_lin) with b, producing
// x = fac dt V_M y, y = beta phi_1(dt H_M) e_1 (the forward left its basis in
// V, its state in ks; M = m_eff).  Given x_bar: b_bar = (dx/db)^T x_bar, and
// ubar += the part of (dx/du_lin)^T x_bar that comes through J(u_lin).
// Differentiates the Arnoldi relations themselves (one classical Gram-Schmidt
// pass with exact orthogonality, which the re-orthogonalised forward
// realises to rounding): for j = M-1 .. 0,
//   r_bar = (v_{j+1}_bar - (v_{j+1}_bar . v_{j+1}) v_{j+1}) / h_{j+1,j} + H_bar_{j+1,j} v_{j+1}  (j < M-1)
//   h_bar_{ij} = H_bar_{ij} - v_i . r_bar,  w_bar = r_bar + sum_i h_bar_{ij} v_i
//   v_i_bar += -h_{ij} r_bar + h_bar_{ij} J v_j   (i <= j)
//   v_j_bar += J^T w_bar,  ubar += (d_u [J(u) v_j])^T w_bar
// and finally b = beta v_0: b_bar = (v_0_bar - (v_0_bar . v_0) v_0) / beta + beta_bar v_0.
void arnoldi_reverse(pcexp_ctx* c, const double* u_lin, const KState* ks, int M, const double* V, double fac,
                     const double* dtp, const double* xbar, double* bbar, double* ubar, const RevBufs& B,
                     hipStream_t st) {
  const size_t n = c->Kint, ld = c->Kld;
  const double* sig = ks->sigma;
  RState* rs = B.rs;
  if (M == 0) {
    k_fill<double>(bbar, 0.0, n, nullptr, st);
    return;
  }
  k_rv_init(ks, rs, fac, dtp, st);
  k_rv_rank(B.Vb, ld, M, xbar, nullptr, rs->a, nullptr, true, n, st);
  k_rv_dots(V, ld, sig, 0, M, xbar, n, B.part, rs->dots, st);
  k_rv_phi_adjoint(ks, rs, rs->dots, fac, dtp, B.mem, st);
  for (int j = M - 1; j >= 0; --j) {
    if (j < M - 1) {
      // d_i = v_i . v_{j+1}_bar (i <= j + 1) in one pass, then r_bar, w_bar = r_bar + sum_{i <= j}
      // h_bar_i v_i, J v_j = sum_{i <= j+1} c_i v_i (the Arnoldi relation) and the updates of
      // v_i_bar (i <= j) from one read of the basis
      double* vb1 = B.Vb + (size_t)(j + 1) * ld;
      k_rv_dots_coef(V, ld, sig, j, vb1, n, B.part, ks, rs, st);
      k_rv_iter(vb1, rs, V, ld, sig, j, B.Vb, B.wb, n, st);
    } else {
      k_rv_coef_w(ks, rs, j, nullptr, st);
      RvComb a{};
      a.x = nullptr; a.axc = 1.0; a.V = V; a.ld = ld; a.sigma = sig; a.coef = rs->b; a.i0 = 0; a.nvec = j + 1;
      k_rv_combine(a, B.wb, n, st);
      jvp_int(c, PCEXP_JVP_TANGENT, PCEXP_PREC_F64, u_lin, nullptr, V + (size_t)j * ld, B.wj, &sig[j], nullptr,
              nullptr, nullptr, st);
      k_rv_rank(B.Vb, ld, j + 1, nullptr, B.wj, rs->a, rs->b, false, n, st);
    }
    // v_j_bar += J^T w_bar, u_bar += sigma_j (d_u[J v_j])^T w_bar (accumulated by the DG
    // kernel itself; the dense test operators have no second-order term)
    if (c->dense) {
      vjp_int(c, u_lin, V + (size_t)j * ld, B.wb, B.t1, B.t2, false, st);
      k_rv_acc2(B.Vb + (size_t)j * ld, B.t1, ubar, B.t2, &sig[j], n, st);
    } else if (c->dim == 2) {
      dg_vjp2(c->p, c->flux, params_d(c), u_lin, V + (size_t)j * ld, B.wb, B.Vb + (size_t)j * ld, ubar, st, &sig[j]);
    } else {
      dg_vjp3(c->p, c->flux, params_d(c), u_lin, V + (size_t)j * ld, B.wb, B.Vb + (size_t)j * ld, ubar, st, &sig[j]);
    }
  }
  k_rv_dots(V, ld, sig, 0, 1, B.Vb, n, B.part, &rs->t[0], st);
  k_rv_coef_b(ks, rs, &rs->t[0], st);
  RvComb a{};
  a.x = B.Vb; a.axp = &rs->alpha; a.V = V; a.ld = ld; a.sigma = sig; a.coef = &rs->gamma; a.i0 = 0; a.nvec = 1;
  k_rv_combine(a, bbar, n, st);
}

struct RevLayout {
  size_t ks1, ks2, rs, part, mem, scal, un, Rn, us, Rs, x1, ub, acc, xb, db, r, wb, wj, t1, t2, V1, V2, Vb, total;
};

RevLayout rev_layout(const pcexp_ctx* c, int m) {
  RevLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += align_up(bytes); return o; };
  const size_t vb = c->Kint * sizeof(double), sb = c->Kld * sizeof(double);
  L.ks1 = take(sizeof(KState));
  L.ks2 = take(sizeof(KState));
  L.rs = take(sizeof(RState));
  L.part = take(part_bytes(c, m));
  const size_t nphi = (size_t)std::max(m + 1, 2 * (m + 1));
  L.mem = take(phi_scratch_doubles((int)nphi) * sizeof(double));
  L.scal = take(64 * sizeof(double));
  L.un = take(vb); L.Rn = take(vb); L.us = take(vb); L.Rs = take(vb); L.x1 = take(vb);
  L.ub = take(vb); L.acc = take(vb); L.xb = take(vb); L.db = take(vb);
  L.r = take(vb); L.wb = take(vb); L.wj = take(vb); L.t1 = take(vb); L.t2 = take(vb);
  L.V1 = take((size_t)(m + 1) * sb);
  L.V2 = take((size_t)(m + 1) * sb);
  L.Vb = take((size_t)m * sb);
  L.total = off;
  return L;
}

void fill_info(pcexp_krylov_info* out, const KState& h) {
  out->beta = h.beta;
  out->h_last = h.hlast;
  out->m_eff = h.m_eff;
  out->breakdown = h.breakdown;
  out->err_est = h.norm_tmp[2];
  out->dt_halvings = (int32_t)h.norm_tmp[3];
}

pcexp_status check_common(pcexp_ctx* c, int m, int k, int prec, int jvp, void* ws, size_t ws_bytes) {
  if (!c) return PCEXP_E_ARG;
  if (m < 1 || m > KMAX) return fail(c, PCEXP_E_ARG, "m must be in [1, 64]");
  if (k < 0 || k > 3) return fail(c, PCEXP_E_ARG, "k must be in [0, 3]");
  if (prec != PCEXP_PREC_F64 && prec != PCEXP_PREC_MIXED) return fail(c, PCEXP_E_ARG, "bad precision");
  if (jvp != PCEXP_JVP_TANGENT && jvp != PCEXP_JVP_FD && jvp != PCEXP_JVP_ZERO)
    return fail(c, PCEXP_E_ARG, "bad jvp kind");
  if (jvp == PCEXP_JVP_FD && prec == PCEXP_PREC_MIXED)
    return fail(c, PCEXP_E_UNSUPPORTED, "FD JVP is FP64 only");
  if (!ws || ws_bytes < ws_layout(c, m, k, prec).total)
    return fail(c, PCEXP_E_WORKSPACE, "workspace missing or too small");
  if (((uintptr_t)ws) % ALIGN != 0) return fail(c, PCEXP_E_WORKSPACE, "workspace must be 256-byte aligned");
  return PCEXP_OK;
}

pcexp_status report_flags(pcexp_ctx* c, uint32_t* out_flags) {
  unsigned f = 0;
  if (hipMemcpy(&f, c->flags, sizeof(unsigned), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(c, PCEXP_E_HIP, "flag read failed");
  unsigned z = 0;
  (void)hipMemcpy(c->flags, &z, sizeof(unsigned), hipMemcpyHostToDevice);
  if (out_flags) *out_flags = f;
  if (f & PCEXP_FLAG_NONFINITE) return fail(c, PCEXP_E_NONFINITE, "non-finite value at a quadrature point");
  if (f & PCEXP_FLAG_UNPHYSICAL) return fail(c, PCEXP_E_UNPHYSICAL, "rho <= 0 or p <= 0 at a quadrature point");
  return PCEXP_OK;
}

pcexp_status alloc_common(pcexp_ctx* c, hipStream_t st) {
  if (hipGetDevice(&c->device) != hipSuccess || c->device < 0 || c->device >= kMaxDevices)
    return fail(c, PCEXP_E_HIP, "hipGetDevice failed");
  {
    const hipError_t e = noalloc_scratch(c->device, &c->noalloc_ws);
    if (e != hipSuccess)
      return fail(c, PCEXP_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  }
  for (int i = 0; i < 5; ++i)
    if (!dalloc(c, &c->io[i], c->Kint)) return fail(c, PCEXP_E_HIP, "hipMalloc failed");
  for (int i = 0; i < 2; ++i)
    if (!dalloc(c, &c->io32[i], c->Kint)) return fail(c, PCEXP_E_HIP, "hipMalloc failed");
  c->part_len = (size_t)3 * 512 * (KMAX + 2);
  size_t eb = (size_t)(c->nE + 255) / 256 * 6;
  if (eb > c->part_len) c->part_len = eb;
  if (!dalloc(c, &c->part, c->part_len)) return fail(c, PCEXP_E_HIP, "hipMalloc failed");
  if (!dalloc(c, (char**)&c->ks, sizeof(KState))) return fail(c, PCEXP_E_HIP, "hipMalloc failed");
  if (!dalloc(c, &c->scal, 64)) return fail(c, PCEXP_E_HIP, "hipMalloc failed");
  if (!dalloc(c, &c->flags, 1)) return fail(c, PCEXP_E_HIP, "hipMalloc failed");
  if (!dalloc(c, &c->counters, 16)) return fail(c, PCEXP_E_HIP, "hipMalloc failed");
  k_fill<unsigned>(c->flags, 0u, 1, nullptr, st);
  k_fill<unsigned>(c->counters, 0u, 16, nullptr, st);
  k_init_state(c->ks, 1e-12, st);
  return PCEXP_OK;
}

}  // namespace

namespace pcexp {
bool dg_run_d(int dim, int p, int flux, int mode, const DGParams<double>& prm, const DGIO<double>& io,
              hipStream_t st) {
  return dim == 2 ? dg_run2_d(p, flux, mode, prm, io, st) : dg_run3_d(p, flux, mode, prm, io, st);
}
bool dg_run_f(int dim, int p, int flux, int mode, const DGParams<float>& prm, const DGIO<float>& io,
              hipStream_t st) {
  return dim == 2 ? dg_run2_f(p, flux, mode, prm, io, st) : dg_run3_f(p, flux, mode, prm, io, st);
}
}  // namespace pcexp

// Quadrature sizes (volume, per face) the DG kernels of (dim, p) are built
// for; the host set-up must generate rules of the same sizes.
template <int D, int P>
static void rule_sizes(int* nq, int* nfq) {
  *nq = Shape<D, P>::NQ;
  *nfq = Shape<D, P>::NFQ;
}
static bool kernel_rule_sizes(int dim, int p, int* nq, int* nfq) {
  switch (dim * 10 + p) {
    case 20: rule_sizes<2, 0>(nq, nfq); return true;
    case 21: rule_sizes<2, 1>(nq, nfq); return true;
    case 22: rule_sizes<2, 2>(nq, nfq); return true;
    case 23: rule_sizes<2, 3>(nq, nfq); return true;
    case 30: rule_sizes<3, 0>(nq, nfq); return true;
    case 31: rule_sizes<3, 1>(nq, nfq); return true;
    case 32: rule_sizes<3, 2>(nq, nfq); return true;
    default: return false;
  }
}

extern "C" {

pcexp_status pcexp_create(const pcexp_mesh_desc* mesh, const pcexp_disc_desc* disc, void* stream,
                          pcexp_ctx** out) {
  if (!out) return PCEXP_E_ARG;
  *out = nullptr;
  if (!mesh || !disc) return PCEXP_E_ARG;
  if (disc->flux != PCEXP_FLUX_LF && disc->flux != PCEXP_FLUX_ROE) return PCEXP_E_ARG;
  if (!(disc->gamma > 1.0)) return PCEXP_E_ARG;
  pcexp_ctx* c = new (std::nothrow) pcexp_ctx();
  if (!c) return PCEXP_E_ARG;
  MeshIn mi;
  mi.dim = mesh->dim; mi.n_vert = mesh->n_vert; mi.n_elem = mesh->n_elem; mi.n_bface = mesh->n_bface;
  mi.vert = mesh->vert; mi.elem = mesh->elem; mi.vert_canon = mesh->vert_canon;
  mi.bface = mesh->bface; mi.bface_tag = mesh->bface_tag;
  Setup S;
  std::string msg = build_setup(mi, disc->p, TILE_PAD, S);
  if (!msg.empty()) {
    pcexp_status s = PCEXP_E_ARG;
    if (msg.rfind("mesh:", 0) == 0) s = PCEXP_E_MESH;
    if (msg.rfind("unsupported:", 0) == 0) s = PCEXP_E_UNSUPPORTED;
    delete c;
    return s;
  }
  if (S.nb > 20 || S.nv > 5) { delete c; return PCEXP_E_UNSUPPORTED; }
  {
    int kq = 0, kfq = 0;
    if (!kernel_rule_sizes(S.dim, S.p, &kq, &kfq) || kq != S.nq || kfq != S.nfq) {
      delete c;
      return PCEXP_E_UNSUPPORTED;
    }
  }
  bool has_far = false;
  for (int64_t b = 0; b < mesh->n_bface; ++b) has_far |= (mesh->bface_tag[b] == PCEXP_BC_FARFIELD);
  if (has_far) {
    if (!(disc->farfield_prim[0] > 0.0) || !(disc->farfield_prim[S.nv - 1] > 0.0)) {
      delete c;
      return PCEXP_E_ARG;
    }
  }
  hipStream_t st = (hipStream_t)stream;
  c->dim = S.dim; c->p = S.p; c->nv = S.nv; c->nb = S.nb; c->nq = S.nq; c->nfq = S.nfq; c->nf = S.nf;
  c->nori = S.nori; c->flux = disc->flux; c->nE = S.nE; c->Epad = S.Epad;
  c->K = (size_t)S.nE * S.nv * S.nb;
  c->Kint = (size_t)S.Epad * S.nv * S.nb;
  c->Kld = (c->Kint + 63) / 64 * 64;
  c->gamma = disc->gamma;
  for (int k = 0; k < 5; ++k) c->ff[k] = disc->farfield_prim[k];
  c->volume_total = S.volume_total;
  bool ok = upload(c, &c->B, S.B, st) && upload(c, &c->Dg, S.Dg, st) && upload(c, &c->wq, S.wq, st) &&
            upload(c, &c->Bf, S.Bf, st) && upload(c, &c->wf, S.wf, st) && upload(c, &c->nref, S.nref, st) &&
            upload(c, &c->Bc, S.Bc, st) && upload(c, &c->refp, S.ref_pts, st) &&
            upload32(c, &c->B32, S.B, st) && upload32(c, &c->Dg32, S.Dg, st) && upload32(c, &c->wq32, S.wq, st) &&
            upload32(c, &c->Bf32, S.Bf, st) && upload32(c, &c->wf32, S.wf, st) &&
            upload32(c, &c->nref32, S.nref, st) && upload(c, &c->ainv, S.ainv, st) &&
            upload(c, &c->sdet, S.sdet, st) && upload(c, &c->x0, S.x0, st) && upload(c, &c->amat, S.amat, st) &&
            upload(c, &c->hE, S.hE, st) && upload(c, &c->Q, S.Q, st) && upload32(c, &c->ainv32, S.ainv, st) &&
            upload32(c, &c->sdet32, S.sdet, st) && upload(c, &c->nbr, S.nbr, st) &&
            upload(c, &c->finfo, S.finfo, st) && upload(c, &c->perm, S.perm, st);
  if (!ok) {
    c->err = "device upload failed";
    pcexp_destroy(c);
    return PCEXP_E_HIP;
  }
  if (alloc_common(c, st) != PCEXP_OK || hipStreamSynchronize(st) != hipSuccess) {
    pcexp_destroy(c);
    return PCEXP_E_HIP;
  }
  *out = c;
  return PCEXP_OK;
}

pcexp_status pcexp_create_dense(int64_t n, const double* A_jac, const double* A_res, void* stream,
                                pcexp_ctx** out) {
  if (!out) return PCEXP_E_ARG;
  *out = nullptr;
  if (n < 1 || n > 4096 || !A_jac || !A_res) return PCEXP_E_ARG;
  pcexp_ctx* c = new (std::nothrow) pcexp_ctx();
  if (!c) return PCEXP_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  c->dense = true;
  c->K = c->Kint = (size_t)n;
  c->Kld = (c->Kint + 63) / 64 * 64;
  c->nE = 1;
  c->nv = 1;
  c->nb = (int)n;
  bool ok = dalloc(c, &c->Ajac, (size_t)n * n) && dalloc(c, &c->Ares, (size_t)n * n) &&
            dalloc(c, &c->Ajac32, (size_t)n * n);
  if (ok) {
    ok = hipMemcpyAsync(c->Ajac, A_jac, (size_t)n * n * sizeof(double), hipMemcpyDeviceToDevice, st) ==
             hipSuccess &&
         hipMemcpyAsync(c->Ares, A_res, (size_t)n * n * sizeof(double), hipMemcpyDeviceToDevice, st) == hipSuccess;
  }
  if (ok) k_cast<double, float>(c->Ajac, c->Ajac32, (size_t)n * n, st);
  if (!ok || alloc_common(c, st) != PCEXP_OK || hipStreamSynchronize(st) != hipSuccess) {
    pcexp_destroy(c);
    return PCEXP_E_HIP;
  }
  *out = c;
  return PCEXP_OK;
}

void pcexp_destroy(pcexp_ctx* c) {
  if (!c) return;
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  for (void* p : c->allocs) (void)hipFree(p);
  delete c;
}

pcexp_status pcexp_sizes(const pcexp_ctx* c, int64_t* s) {
  if (!c || !s) return PCEXP_E_ARG;
  s[0] = (int64_t)c->K; s[1] = c->nE; s[2] = c->dim; s[3] = c->nv; s[4] = c->nb; s[5] = c->nq;
  s[6] = c->nfq; s[7] = c->p;
  return PCEXP_OK;
}

const char* pcexp_last_error(const pcexp_ctx* c) { return c ? c->err.c_str() : "null context"; }

size_t pcexp_workspace_bytes(const pcexp_ctx* c, int32_t m, int32_t k, int32_t prec, int32_t jvp) {
  (void)jvp;
  if (!c || m < 1 || m > KMAX || k < 0 || k > 3) return 0;
  return ws_layout(c, m, k, prec).total;
}

pcexp_status pcexp_quad_points(pcexp_ctx* c, double* xyz, void* stream) {
  if (!c || !xyz) return PCEXP_E_ARG;
  if (c->dense) return fail(c, PCEXP_E_UNSUPPORTED, "dense context has no mesh");
  ek_quad_points(elem_args(c), xyz, (hipStream_t)stream);
  return hip_check(c, "quad_points");
}

pcexp_status pcexp_project(pcexp_ctx* c, const double* U_qp, double* u, void* stream) {
  if (!c || !U_qp || !u) return PCEXP_E_ARG;
  if (c->dense) return fail(c, PCEXP_E_UNSUPPORTED, "dense context has no mesh");
  ek_project(elem_args(c), U_qp, u, (hipStream_t)stream);
  return hip_check(c, "project");
}

pcexp_status pcexp_evaluate(pcexp_ctx* c, const double* u, double* U_qp, void* stream) {
  if (!c || !U_qp || !u) return PCEXP_E_ARG;
  if (c->dense) return fail(c, PCEXP_E_UNSUPPORTED, "dense context has no mesh");
  ek_evaluate(elem_args(c), u, U_qp, (hipStream_t)stream);
  return hip_check(c, "evaluate");
}

pcexp_status pcexp_residual(pcexp_ctx* c, const double* u, double* R, void* stream) {
  if (!c || !u || !R || u == R) return c ? fail(c, PCEXP_E_ARG, "bad pointers") : PCEXP_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  to_int(c, u, c->io[0], st);
  if (!residual_int(c, c->io[0], c->io[1], st)) return fail(c, PCEXP_E_UNSUPPORTED, "no kernel");
  to_abi(c, c->io[1], R, st);
  return hip_check(c, "residual");
}

pcexp_status pcexp_jvp(pcexp_ctx* c, const double* u, const void* v_, void* Jv_, int32_t jvp, int32_t prec,
                       void* stream) {
  if (!c || !u || !v_ || !Jv_ || v_ == Jv_) return c ? fail(c, PCEXP_E_ARG, "bad pointers") : PCEXP_E_ARG;
  if (jvp != PCEXP_JVP_TANGENT && jvp != PCEXP_JVP_FD && jvp != PCEXP_JVP_ZERO)
    return fail(c, PCEXP_E_ARG, "bad jvp kind");
  if (prec != PCEXP_PREC_F64 && prec != PCEXP_PREC_MIXED) return fail(c, PCEXP_E_ARG, "bad precision");
  if (jvp == PCEXP_JVP_FD && prec == PCEXP_PREC_MIXED) return fail(c, PCEXP_E_UNSUPPORTED, "FD JVP is FP64 only");
  hipStream_t st = (hipStream_t)stream;
  const size_t n = c->Kint;
  to_int(c, u, c->io[0], st);
  bool ok;
  if (prec == PCEXP_PREC_MIXED) {
    // FP32 v and Jv at the boundary; the change of basis runs in FP64 on
    // widened copies (an orthogonal map per element), the JVP in FP32
    k_cast<float, double>((const float*)v_, c->io[4], c->K, st);
    to_int(c, c->io[4], c->io[1], st);
    k_cast<double, float>(c->io[0], c->io32[0], n, st);
    k_cast<double, float>(c->io[1], c->io32[1], n, st);
    // the FP32 result is written as float into io[2]'s storage
    ok = jvp_int(c, jvp, prec, nullptr, c->io32[0], c->io32[1], (void*)c->io[2], nullptr, nullptr, nullptr,
                 nullptr, st);
    k_cast<float, double>((const float*)c->io[2], c->io[3], n, st);
    to_abi(c, c->io[3], c->io[4], st);
    k_cast<double, float>(c->io[4], (float*)Jv_, c->K, st);
    return ok ? hip_check(c, "jvp") : fail(c, PCEXP_E_UNSUPPORTED, "no kernel");
  }
  const double* v = (const double*)v_;
  double* Jv = (double*)Jv_;
  to_int(c, v, c->io[1], st);
  const double* Rb = nullptr;
  double* eps = nullptr;
  if (jvp == PCEXP_JVP_FD) {
    if (!residual_int(c, c->io[0], c->io[3], st)) return fail(c, PCEXP_E_UNSUPPORTED, "no kernel");
    Rb = c->io[3];
    k_sumsq(c->io[0], n, &c->scal[0], 1, c->part, &c->counters[0], st);
    k_sumsq(c->io[1], n, &c->scal[1], 1, c->part, &c->counters[1], st);
    k_fd_eps(&c->scal[0], &c->scal[1], kSqrtEps, &c->scal[2], st);
    eps = &c->scal[2];
  }
  ok = jvp_int(c, jvp, prec, c->io[0], nullptr, c->io[1], c->io[2], nullptr, nullptr, Rb, eps, st);
  to_abi(c, c->io[2], Jv, st);
  return ok ? hip_check(c, "jvp") : fail(c, PCEXP_E_UNSUPPORTED, "no kernel");
}

pcexp_status pcexp_vjp(pcexp_ctx* c, const double* u, const double* w, double* JTw, void* stream) {
  if (!c || !u || !w || !JTw || w == JTw) return c ? fail(c, PCEXP_E_ARG, "bad pointers") : PCEXP_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  to_int(c, u, c->io[0], st);
  to_int(c, w, c->io[1], st);
  bool ok = vjp_int(c, c->io[0], nullptr, c->io[1], c->io[2], nullptr, false, st);
  to_abi(c, c->io[2], JTw, st);
  return ok ? hip_check(c, "vjp") : fail(c, PCEXP_E_UNSUPPORTED, "no kernel");
}

pcexp_status pcexp_stable_dt(pcexp_ctx* c, const double* u, double cfl, double* dt_host, void* stream) {
  if (!c || !u || !dt_host || !(cfl > 0.0)) return c ? fail(c, PCEXP_E_ARG, "bad arguments") : PCEXP_E_ARG;
  if (c->dense) return fail(c, PCEXP_E_UNSUPPORTED, "dense context has no mesh");
  hipStream_t st = (hipStream_t)stream;
  to_int(c, u, c->io[0], st);
  ek_stable_dt(elem_args(c), c->io[0], nullptr, cfl, &c->scal[8], c->part, &c->counters[2], st);
  if (hipMemcpyAsync(dt_host, &c->scal[8], sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(c, PCEXP_E_HIP, "stable_dt sync failed");
  if (!std::isfinite(*dt_host) || !(*dt_host > 0.0)) return fail(c, PCEXP_E_UNPHYSICAL, "invalid time step");
  return hip_check(c, "stable_dt");
}

pcexp_status pcexp_conserved_totals(pcexp_ctx* c, const double* u, double* out_host, void* stream) {
  if (!c || !u || !out_host) return PCEXP_E_ARG;
  if (c->dense) return fail(c, PCEXP_E_UNSUPPORTED, "dense context has no mesh");
  hipStream_t st = (hipStream_t)stream;
  to_int(c, u, c->io[0], st);
  ek_totals(elem_args(c), c->io[0], &c->scal[16], c->part, &c->counters[3], st);
  if (hipMemcpyAsync(out_host, &c->scal[16], c->nv * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(c, PCEXP_E_HIP, "totals sync failed");
  return hip_check(c, "totals");
}

pcexp_status pcexp_arnoldi_phi(pcexp_ctx* c, const double* u_lin, const double* b, double dt, int32_t k, int32_t m,
                               int32_t prec, int32_t jvp, double* out, void* ws, size_t ws_bytes,
                               pcexp_krylov_info* info, void* stream) {
  pcexp_status s = check_common(c, m, k, prec, jvp, ws, ws_bytes);
  if (s != PCEXP_OK) return s;
  if (!u_lin || !b || !out || out == b) return fail(c, PCEXP_E_ARG, "bad pointers");
  if (!std::isfinite(dt)) return fail(c, PCEXP_E_ARG, "dt must be finite");
  hipStream_t st = (hipStream_t)stream;
  const WsLayout L = ws_layout(c, m, k, prec);
  char* w = (char*)ws;
  KState* ks = (KState*)(w + L.ks1);
  double* part = (double*)(w + L.part);
  double* phi = (double*)(w + L.phi);
  double* scal = (double*)(w + L.scal);
  double* un = (double*)(w + L.un);
  double* Rn = (double*)(w + L.Rn);
  double* bb = (double*)(w + L.us);
  double* xo = (double*)(w + L.Rs);
  float* un32 = (float*)(w + L.un32);
  to_int(c, u_lin, un, st);
  to_int(c, b, bb, st);
  k_set_scalar(&scal[0], dt, st);
  if (jvp == PCEXP_JVP_FD && !residual_int(c, un, Rn, st)) return fail(c, PCEXP_E_UNSUPPORTED, "no kernel");
  if (prec == PCEXP_PREC_MIXED) {
    k_cast<double, float>(un, un32, c->Kint, st);
    float* V = (float*)(w + L.V);
    arnoldi_run<float>(c, jvp, prec, un, un32, bb, Rn, &scal[0], k, m, ks, part, phi, V, st);
    k_combine<float, double>(V, c->Kld, ks, nullptr, xo, (double*)nullptr, 1.0, nullptr, c->Kint, st);
  } else {
    double* V = (double*)(w + L.V);
    arnoldi_run<double>(c, jvp, prec, un, nullptr, bb, Rn, &scal[0], k, m, ks, part, phi, V, st);
    k_combine<double, double>(V, c->Kld, ks, nullptr, xo, (double*)nullptr, 1.0, nullptr, c->Kint, st);
  }
  to_abi(c, xo, out, st);
  s = hip_check(c, "arnoldi_phi");
  if (s != PCEXP_OK) return s;
  if (info) {
    KState h;
    if (hipMemcpyAsync(&h, ks, sizeof(KState), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return fail(c, PCEXP_E_HIP, "info sync failed");
    fill_info(info, h);
    uint32_t f;
    return report_flags(c, &f);
  }
  return PCEXP_OK;
}

}  // extern "C"

namespace {

// How a step chooses dt: fixed, from a constant CFL (eq. (x3d)), or from the
// CFL ramp of eq. (cfl) driven by ||R(rho_n)|| (pseudo-time iteration n).
struct DtMode {
  double dt = 0.0, cfl = 0.0, cfl_max = 0.0;
  int ramp_iter = 0;   // > 0: ramp at this iteration
};

// cfl = min(cfl_max, max(r^-3, 1 + (n-1)/(2p+1))), r = sqrt(sum R_rho^2) / |Omega| (eq. (cfl)).
__global__ void cfl_ramp_kernel(const double* rsqrt, double inv_vol, int n, int p, double cfl_max, double* cfl,
                                double* rnorm) {
  const double r = *rsqrt * inv_vol;
  const double big = r > 0.0 ? 1.0 / (r * r * r) : INFINITY;
  const double lin = 1.0 + (double)(n - 1) / (2 * p + 1);
  *cfl = fmin(cfl_max, fmax(big, lin));
  *rnorm = r;
}

// History of an ETD2 step (ABI layout, caller-owned): u_{n-1} and R(u_{n-1}),
// read when have_prev, then overwritten with u_n and R(u_n).
struct Etd2Hist {
  double* u_prev;
  double* r_prev;
  int have_prev;
};

// One step on internal vectors: un (u_n) is replaced by u_{n+1}.  scal[0] = dt,
// scal[4] = ||R(rho_n)|| (ramp mode), scal[5] = CFL used (ramp mode).
pcexp_status step_core(pcexp_ctx* c, double* un, const DtMode& dm, int m, int scheme, int prec, int jvp, char* w,
                       const WsLayout& L, hipStream_t st, const Etd2Hist* hist = nullptr) {
  KState* ks1 = (KState*)(w + L.ks1);
  KState* ks2 = (KState*)(w + L.ks2);
  double* part = (double*)(w + L.part);
  double* phi = (double*)(w + L.phi);
  double* scal = (double*)(w + L.scal);
  double* Rn = (double*)(w + L.Rn);
  double* us = (double*)(w + L.us);
  double* Rs = (double*)(w + L.Rs);
  void* x1 = (void*)(w + L.x1);
  float* un32 = (float*)(w + L.un32);
  unsigned* cnt = (unsigned*)(w + L.cnt);
  const size_t n = c->Kint;
  double* dtp = &scal[0];
  const bool exp1 = scheme == PCEXP_SCHEME_EXP1;

  if (!residual_int(c, un, Rn, st)) return fail(c, PCEXP_E_UNSUPPORTED, "no kernel");
  if (dm.dt > 0.0) {
    k_set_scalar(dtp, dm.dt, st);
  } else if (dm.ramp_iter > 0) {
    k_sumsq(Rn, (size_t)c->nb * c->Epad, &scal[6], 1, part, &cnt[3], st);
    launch(cfl_ramp_kernel, dim3(1), dim3(1), 0, st, (const double*)&scal[6], 1.0 / c->volume_total, dm.ramp_iter,
           c->p, dm.cfl_max, &scal[5], &scal[4]);
    ek_stable_dt(elem_args(c), un, &scal[5], 0.0, dtp, part, &cnt[0], st);
  } else {
    ek_stable_dt(elem_args(c), un, nullptr, dm.cfl, dtp, part, &cnt[0], st);
  }
  const bool mixed = (prec == PCEXP_PREC_MIXED);
  if (mixed) k_cast<double, float>(un, un32, n, st);

  // ETD2 (eq. (s7)): take u_{n-1}, R_{n-1} into internal storage (x1 is not
  // needed by the predictor of this scheme), then leave u_n, R_n as history
  const bool etd2 = scheme == PCEXP_SCHEME_ETD2;
  double* up = (double*)x1;
  if (etd2) {
    if (hist->have_prev) {
      to_int(c, hist->u_prev, up, st);
      to_int(c, hist->r_prev, Rs, st);
    }
    to_abi(c, un, hist->u_prev, st);
    to_abi(c, Rn, hist->r_prev, st);
  }

  // stage 1: x1 = dt Phi_1(dt J_n) R_n; u* = u_n + x1 (EXP1: the result, written over u_n)
  double* out1 = exp1 ? un : us;
  if (mixed) {
    float* V = (float*)(w + L.V);
    arnoldi_run<float>(c, jvp, prec, un, un32, Rn, Rn, dtp, 1, m, ks1, part, phi, V, st, c->krylov_tol, true,
                       c->krylov_every);
    Prof pr(c, st, PC_COMB, (double)c->K * (m * 4.0 + 8 + 8 + 4));
    k_combine<float, float>(V, c->Kld, ks1, un, out1, (exp1 || etd2) ? (float*)nullptr : (float*)x1, 1.0, dtp, n,
                            st);
  } else {
    double* V = (double*)(w + L.V);
    arnoldi_run<double>(c, jvp, prec, un, nullptr, Rn, Rn, dtp, 1, m, ks1, part, phi, V, st, c->krylov_tol, true,
                        c->krylov_every);
    Prof pr(c, st, PC_COMB, (double)c->K * (m * 8.0 + 8 + 8 + 8));
    k_combine<double, double>(V, c->Kld, ks1, un, out1, (exp1 || etd2) ? (double*)nullptr : (double*)x1, 1.0,
                              dtp, n, st);
  }
  if (exp1) return PCEXP_OK;

  if (etd2) {
    if (!hist->have_prev) {   // first step: ETD1, eq. (s8)
      if (hipMemcpyAsync(un, us, n * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess)
        return fail(c, PCEXP_E_HIP, "copy failed");
      return PCEXP_OK;
    }
    // N_n - N_{n-1} = R_n - R_{n-1} - J_n (u_n - u_{n-1}) (N = R - J_n u on this step)
    k_glue_d<double>(un, up, (const double*)nullptr, up, n, st);
    double* jx = (double*)(w + L.V);
    if (jvp == PCEXP_JVP_FD) {
      k_sumsq(un, n, &scal[1], 1, part, &cnt[1], st);
      k_sumsq(up, n, &scal[2], 1, part, &cnt[2], st);
      k_fd_eps(&scal[1], &scal[2], kSqrtEps, &scal[3], st);
    }
    jvp_int(c, jvp, prec, un, nullptr, up, jx, nullptr, nullptr, Rn, &scal[3], st);
    k_glue_d<double>(Rn, Rs, jx, Rs, n, st);
    // u_{n+1} = u* + dt Phi_2(dt J_n)(N_n - N_{n-1})
    double* V = (double*)(w + L.V);
    arnoldi_run<double>(c, jvp, prec, un, nullptr, Rs, Rn, dtp, 2, m, ks2, part, phi, V, st);
    Prof pr(c, st, PC_COMB, (double)c->K * (m * 8.0 + 8 + 8));
    k_combine<double, double>(V, c->Kld, ks2, us, un, (double*)nullptr, 1.0, dtp, n, st);
    return PCEXP_OK;
  }

  // N* - N_n = R(u*) - R_n - J_n x1
  if (!residual_int(c, us, Rs, st)) return fail(c, PCEXP_E_UNSUPPORTED, "no kernel");
  if (mixed) {
    float* jx = (float*)(w + L.V);  // Krylov storage is free between the two Arnoldi runs
    jvp_int(c, jvp, prec, un, un32, x1, jx, nullptr, nullptr, Rn, nullptr, st);
    k_glue_d<float>(Rs, Rn, jx, Rs, n, st);
  } else {
    double* jx = (double*)(w + L.V);
    if (jvp == PCEXP_JVP_FD) {
      k_sumsq(un, n, &scal[1], 1, part, &cnt[1], st);
      k_sumsq((const double*)x1, n, &scal[2], 1, part, &cnt[2], st);
      k_fd_eps(&scal[1], &scal[2], kSqrtEps, &scal[3], st);
    }
    jvp_int(c, jvp, prec, un, nullptr, x1, jx, nullptr, nullptr, Rn, &scal[3], st);
    k_glue_d<double>(Rs, Rn, jx, Rs, n, st);
  }
  // stage 2: u_{n+1} = u* + dt/2 Phi_1(dt J_n)(N* - N_n)
  if (mixed) {
    float* V = (float*)(w + L.V);
    arnoldi_run<float>(c, jvp, prec, un, un32, Rs, Rn, dtp, 1, m, ks2, part, phi, V, st, c->krylov_tol, false,
                       c->krylov_every);
    Prof pr(c, st, PC_COMB, (double)c->K * (m * 4.0 + 8 + 8));
    k_combine<float, double>(V, c->Kld, ks2, us, un, (double*)nullptr, 0.5, dtp, n, st);
  } else {
    double* V = (double*)(w + L.V);
    arnoldi_run<double>(c, jvp, prec, un, nullptr, Rs, Rn, dtp, 1, m, ks2, part, phi, V, st, c->krylov_tol, false,
                        c->krylov_every);
    Prof pr(c, st, PC_COMB, (double)c->K * (m * 8.0 + 8 + 8));
    k_combine<double, double>(V, c->Kld, ks2, us, un, (double*)nullptr, 0.5, dtp, n, st);
  }
  return PCEXP_OK;
}

pcexp_status check_step_args(pcexp_ctx* c, int m, int scheme, int prec, int jvp, void* ws, size_t ws_bytes) {
  pcexp_status s = check_common(c, m, 1, prec, jvp, ws, ws_bytes);
  if (s != PCEXP_OK) return s;
  if (scheme != PCEXP_SCHEME_PCEXP && scheme != PCEXP_SCHEME_EXP1) return fail(c, PCEXP_E_ARG, "bad scheme");
  return PCEXP_OK;
}

}  // namespace

extern "C" {

pcexp_status pcexp_set_krylov_tol(pcexp_ctx* c, double tol) {
  if (!c) return PCEXP_E_ARG;
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(c, PCEXP_E_ARG, "tol must be finite and >= 0");
  c->krylov_tol = tol;
  return PCEXP_OK;
}

pcexp_status pcexp_set_krylov_adapt(pcexp_ctx* c, int32_t check_every) {
  if (!c) return PCEXP_E_ARG;
  if (check_every < 0 || check_every > KMAX) return fail(c, PCEXP_E_ARG, "check_every must be in [0, 64]");
  c->krylov_every = check_every;
  return PCEXP_OK;
}

// nsteps steps with u in the internal basis between them (one basis change
// in, one out); pcexp_step is nsteps = 1.
static pcexp_status advance_impl(pcexp_ctx* c, double* u, int nsteps, double dt, double cfl, int32_t m,
                                 int32_t scheme, int32_t prec, int32_t jvp, void* ws, size_t ws_bytes,
                                 pcexp_step_info* info, void* stream) {
  pcexp_status s = check_step_args(c, m, scheme, prec, jvp, ws, ws_bytes);
  if (s != PCEXP_OK) return s;
  if (nsteps < 1) return fail(c, PCEXP_E_ARG, "nsteps must be >= 1");
  if (!u) return fail(c, PCEXP_E_ARG, "u is NULL");
  if (!(dt > 0.0) && !(cfl > 0.0)) return fail(c, PCEXP_E_ARG, "need dt > 0 or cfl > 0");
  if (!(dt > 0.0) && c->dense) return fail(c, PCEXP_E_ARG, "dense contexts need dt > 0");
  if (!std::isfinite(dt) || !std::isfinite(cfl)) return fail(c, PCEXP_E_ARG, "dt/cfl must be finite");
  hipStream_t st = (hipStream_t)stream;
  const WsLayout L = ws_layout(c, m, 1, prec);
  char* w = (char*)ws;
  double* scal = (double*)(w + L.scal);
  double* un = (double*)(w + L.un);
  double* Rn = (double*)(w + L.Rn);
  double* part = (double*)(w + L.part);
  unsigned* cnt = (unsigned*)(w + L.cnt);
  to_int(c, u, un, st);
  DtMode dm;
  dm.dt = dt > 0.0 ? dt : 0.0;
  dm.cfl = cfl;
  // the time advanced: nsteps dt when every step takes the given dt, else the
  // sum over the steps of the dt each one used (eq. (x3d) per step, or a dt
  // the Krylov tolerance halved on the device), summed in scal[16]
  const bool dt_varies = !(dt > 0.0) || c->krylov_tol > 0.0;
  if (dt_varies && info) k_set_scalar(&scal[16], 0.0, st);
  for (int i = 0; i < nsteps; ++i) {
    k_fill<unsigned>(cnt, 0u, 64, nullptr, st);
    s = step_core(c, un, dm, m, scheme, prec, jvp, w, L, st);
    if (s != PCEXP_OK) return s;
    if (dt_varies && info) k_add_scalar(&scal[16], &scal[0], st);
  }
  to_abi(c, un, u, st);
  s = hip_check(c, "step");
  if (s != PCEXP_OK) return s;
  if (info) {
    std::memset(info, 0, sizeof(*info));
    if (!c->dense) k_sumsq(Rn, (size_t)c->nb * c->Epad, &scal[4], 1, part, &cnt[3], st);
    KState h1, h2;
    double sc[17];
    if (hipMemcpyAsync(&h1, (KState*)(w + L.ks1), sizeof(KState), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(&h2, (KState*)(w + L.ks2), sizeof(KState), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(sc, scal, sizeof(sc), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return fail(c, PCEXP_E_HIP, "info sync failed");
    fill_info(&info->k1, h1);
    if (scheme == PCEXP_SCHEME_PCEXP) fill_info(&info->k2, h2);
    info->dt = sc[0];
    info->res_rho_norm = c->dense ? 0.0 : sc[4] / c->volume_total;
    info->t_advanced = dt_varies ? sc[16] : nsteps * dt;
    return report_flags(c, &info->flags);
  }
  return PCEXP_OK;
}

pcexp_status pcexp_step(pcexp_ctx* c, double* u, double dt, double cfl, int32_t m, int32_t scheme, int32_t prec,
                        int32_t jvp, void* ws, size_t ws_bytes, pcexp_step_info* info, void* stream) {
  return advance_impl(c, u, 1, dt, cfl, m, scheme, prec, jvp, ws, ws_bytes, info, stream);
}

pcexp_status pcexp_step_noalloc(pcexp_ctx* c, double* u, double dt, double cfl, int32_t m, int32_t scheme,
                                int32_t prec, int32_t jvp, pcexp_step_info* info, void* stream) {
  if (!c) return PCEXP_E_ARG;
  if (!c->noalloc_ws) return fail(c, PCEXP_E_HIP, "no-allocation workspace was not set up");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(c, PCEXP_E_HIP, "hipGetDevice failed");
  if (dev != c->device) return fail(c, PCEXP_E_ARG, "the current device is not the context's device");
  const size_t need = pcexp_workspace_bytes(c, m, 1, prec, jvp);
  if (need == 0) return fail(c, PCEXP_E_ARG, "bad m, prec or jvp");
  if (need > kNoallocBytes)
    return fail(c, PCEXP_E_WORKSPACE,
                "pcexp_step_noalloc: this mesh and Krylov dimension need " + std::to_string(need) +
                    " workspace bytes, more than the fixed " + std::to_string(kNoallocBytes) +
                    " (use pcexp_step with a caller workspace)");
  // every quantity the step needs at zero is cleared by the step itself
  // (counters at its start, accumulators by their first write), so the
  // contents left by an earlier call do not matter
  return advance_impl(c, u, 1, dt, cfl, m, scheme, prec, jvp, c->noalloc_ws, kNoallocBytes, info, stream);
}

pcexp_status pcexp_advance(pcexp_ctx* c, double* u, int32_t nsteps, double dt, double cfl, int32_t m,
                           int32_t scheme, int32_t prec, int32_t jvp, void* ws, size_t ws_bytes,
                           pcexp_step_info* info, void* stream) {
  return advance_impl(c, u, nsteps, dt, cfl, m, scheme, prec, jvp, ws, ws_bytes, info, stream);
}

pcexp_status pcexp_step_etd2(pcexp_ctx* c, double* u, double* u_prev, double* r_prev, int32_t have_prev, double dt,
                             int32_t m, int32_t jvp, void* ws, size_t ws_bytes, pcexp_step_info* info, void* stream) {
  pcexp_status s = check_common(c, m, 1, PCEXP_PREC_F64, jvp, ws, ws_bytes);
  if (s != PCEXP_OK) return s;
  if (!u || !u_prev || !r_prev) return fail(c, PCEXP_E_ARG, "u, u_prev and r_prev are required");
  if (u == u_prev || u == r_prev || u_prev == r_prev) return fail(c, PCEXP_E_ARG, "u, u_prev, r_prev must differ");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, PCEXP_E_ARG, "ETD2 needs a fixed dt > 0");
  hipStream_t st = (hipStream_t)stream;
  const WsLayout L = ws_layout(c, m, 1, PCEXP_PREC_F64);
  char* w = (char*)ws;
  double* scal = (double*)(w + L.scal);
  double* un = (double*)(w + L.un);
  unsigned* cnt = (unsigned*)(w + L.cnt);
  k_fill<unsigned>(cnt, 0u, 64, nullptr, st);
  to_int(c, u, un, st);
  DtMode dm;
  dm.dt = dt;
  const Etd2Hist hist{u_prev, r_prev, have_prev != 0};
  s = step_core(c, un, dm, m, PCEXP_SCHEME_ETD2, PCEXP_PREC_F64, jvp, w, L, st, &hist);
  if (s != PCEXP_OK) return s;
  to_abi(c, un, u, st);
  s = hip_check(c, "step_etd2");
  if (s != PCEXP_OK) return s;
  if (info) {
    std::memset(info, 0, sizeof(*info));
    KState h1, h2;
    double sc[8];
    if (hipMemcpyAsync(&h1, (KState*)(w + L.ks1), sizeof(KState), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(&h2, (KState*)(w + L.ks2), sizeof(KState), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(sc, scal, sizeof(sc), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return fail(c, PCEXP_E_HIP, "info sync failed");
    fill_info(&info->k1, h1);
    if (have_prev) fill_info(&info->k2, h2);
    info->dt = sc[0];
    return report_flags(c, &info->flags);
  }
  return PCEXP_OK;
}

pcexp_status pcexp_steady(pcexp_ctx* c, double* u, double cfl_max, double tol, int32_t max_iter,
                          int32_t check_every, int32_t m, int32_t scheme, int32_t prec, int32_t jvp, void* ws,
                          size_t ws_bytes, pcexp_steady_info* info, void* stream) {
  pcexp_status s = check_step_args(c, m, scheme, prec, jvp, ws, ws_bytes);
  if (s != PCEXP_OK) return s;
  if (!u) return fail(c, PCEXP_E_ARG, "u is NULL");
  if (c->dense) return fail(c, PCEXP_E_UNSUPPORTED, "the CFL ramp needs a mesh");
  if (!(cfl_max > 0.0) || !std::isfinite(cfl_max) || !(tol >= 0.0) || max_iter < 1 || check_every < 1)
    return fail(c, PCEXP_E_ARG, "need cfl_max > 0, tol >= 0, max_iter >= 1, check_every >= 1");
  hipStream_t st = (hipStream_t)stream;
  const WsLayout L = ws_layout(c, m, 1, prec);
  char* w = (char*)ws;
  double* scal = (double*)(w + L.scal);
  double* un = (double*)(w + L.un);
  double* Rn = (double*)(w + L.Rn);
  double* part = (double*)(w + L.part);
  unsigned* cnt = (unsigned*)(w + L.cnt);
  k_fill<unsigned>(cnt, 0u, 64, nullptr, st);
  to_int(c, u, un, st);
  double r0 = -1.0, r = -1.0;
  int it = 0;
  bool conv = false;
  while (it < max_iter) {
    DtMode dm;
    dm.cfl_max = cfl_max;
    dm.ramp_iter = it + 1;
    s = step_core(c, un, dm, m, scheme, prec, jvp, w, L, st);
    if (s != PCEXP_OK) return s;
    ++it;
    if (it == 1 || it % check_every == 0 || it == max_iter) {
      // scal[4] holds ||R(rho)|| at the start of the latest step
      double sc[8];
      if (hipMemcpyAsync(sc, scal, sizeof(sc), hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return fail(c, PCEXP_E_HIP, "steady sync failed");
      if (it == 1) r0 = sc[4];
      r = sc[4];
      if (!std::isfinite(r)) return fail(c, PCEXP_E_NONFINITE, "residual norm is not finite");
      if (r <= tol) {
        conv = true;
        break;
      }
    }
  }
  // residual norm of the final state
  if (!residual_int(c, un, Rn, st)) return fail(c, PCEXP_E_UNSUPPORTED, "no kernel");
  k_sumsq(Rn, (size_t)c->nb * c->Epad, &scal[6], 1, part, &cnt[3], st);
  double rf = 0.0;
  if (hipMemcpyAsync(&rf, &scal[6], sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(c, PCEXP_E_HIP, "steady sync failed");
  rf /= c->volume_total;
  to_abi(c, un, u, st);
  s = hip_check(c, "steady");
  if (s != PCEXP_OK) return s;
  if (info) {
    info->iterations = it;
    info->converged = (conv || rf <= tol) ? 1 : 0;
    info->res_rho_norm0 = r0;
    info->res_rho_norm = rf;
  }
  uint32_t f;
  return report_flags(c, &f);
}

pcexp_status pcexp_pressure_functional(pcexp_ctx* c, const double* u, double p_ref, double* value_host,
                                       double* grad, void* stream) {
  if (!c || !u || !value_host) return c ? fail(c, PCEXP_E_ARG, "bad pointers") : PCEXP_E_ARG;
  if (c->dense) return fail(c, PCEXP_E_UNSUPPORTED, "dense context has no mesh");
  if (grad == u) return fail(c, PCEXP_E_ARG, "grad must not alias u");
  hipStream_t st = (hipStream_t)stream;
  to_int(c, u, c->io[0], st);
  ek_pressure_functional(elem_args(c), c->io[0], p_ref, &c->scal[24], grad ? c->io[1] : nullptr, c->part, st);
  if (grad) to_abi(c, c->io[1], grad, st);
  if (hipMemcpyAsync(value_host, &c->scal[24], sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(c, PCEXP_E_HIP, "pressure functional sync failed");
  return hip_check(c, "pressure_functional");
}

pcexp_status pcexp_pressure_functional_acc(pcexp_ctx* c, const double* u, double p_ref, double scale,
                                           double* value_acc, double* grad_acc, void* stream) {
  if (!c || !u) return c ? fail(c, PCEXP_E_ARG, "u is NULL") : PCEXP_E_ARG;
  if (c->dense) return fail(c, PCEXP_E_UNSUPPORTED, "dense context has no mesh");
  if (!value_acc && !grad_acc) return fail(c, PCEXP_E_ARG, "nothing to accumulate");
  if (!std::isfinite(scale) || !std::isfinite(p_ref)) return fail(c, PCEXP_E_ARG, "scale and p_ref must be finite");
  if ((const double*)grad_acc == u || (const double*)value_acc == u || (value_acc && value_acc == grad_acc))
    return fail(c, PCEXP_E_ARG, "accumulators must not alias u or each other");
  hipStream_t st = (hipStream_t)stream;
  to_int(c, u, c->io[0], st);
  ek_pressure_functional(elem_args(c), c->io[0], p_ref, value_acc, grad_acc ? c->io[1] : nullptr, c->part, st, 1,
                         scale);
  if (grad_acc) ek_to_abi_axpy(elem_args(c), c->io[1], scale, grad_acc, st);
  return hip_check(c, "pressure_functional_acc");
}

size_t pcexp_step_vjp_workspace_bytes(const pcexp_ctx* c, int32_t m) {
  if (!c || m < 1 || m > KMAX) return 0;
  return rev_layout(c, m).total;
}

pcexp_status pcexp_vjp2(pcexp_ctx* c, const double* u, const double* v, const double* w, double* JTw,
                        double* dJTw, void* stream) {
  if (!c || !u || !v || !w || !JTw || !dJTw || w == JTw || w == dJTw || JTw == dJTw)
    return c ? fail(c, PCEXP_E_ARG, "bad pointers") : PCEXP_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  to_int(c, u, c->io[0], st);
  to_int(c, v, c->io[1], st);
  to_int(c, w, c->io[2], st);
  if (!vjp_int(c, c->io[0], c->io[1], c->io[2], c->io[3], c->io[4], false, st))
    return fail(c, PCEXP_E_UNSUPPORTED, "no kernel");
  to_abi(c, c->io[3], JTw, st);
  to_abi(c, c->io[4], dJTw, st);
  return hip_check(c, "vjp2");
}

pcexp_status pcexp_step_vjp(pcexp_ctx* c, const double* u_n, double dt, int32_t m, int32_t scheme,
                            const double* ubar_np1, double* ubar_n, void* ws, size_t ws_bytes, void* stream) {
  if (!c) return PCEXP_E_ARG;
  if (!u_n || !ubar_np1 || !ubar_n || ubar_np1 == ubar_n) return fail(c, PCEXP_E_ARG, "bad pointers");
  if (m < 1 || m > KMAX) return fail(c, PCEXP_E_ARG, "m must be in [1, 64]");
  if (scheme != PCEXP_SCHEME_PCEXP && scheme != PCEXP_SCHEME_EXP1) return fail(c, PCEXP_E_ARG, "bad scheme");
  if (!std::isfinite(dt) || !(dt > 0.0)) return fail(c, PCEXP_E_ARG, "step_vjp needs a fixed dt > 0");
  const RevLayout L = rev_layout(c, m);
  if (!ws || ws_bytes < L.total) return fail(c, PCEXP_E_WORKSPACE, "workspace missing or too small");
  if (((uintptr_t)ws) % ALIGN != 0) return fail(c, PCEXP_E_WORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  char* w = (char*)ws;
  auto vec = [&](size_t off) { return (double*)(w + off); };
  KState* ks1 = (KState*)(w + L.ks1);
  KState* ks2 = (KState*)(w + L.ks2);
  double* part = vec(L.part);
  double* mem = vec(L.mem);
  double* scal = vec(L.scal);
  double *un = vec(L.un), *Rn = vec(L.Rn), *us = vec(L.us), *Rs = vec(L.Rs), *x1 = vec(L.x1);
  double *ub = vec(L.ub), *acc = vec(L.acc), *xb = vec(L.xb), *db = vec(L.db);
  double *V1 = vec(L.V1), *V2 = vec(L.V2);
  RevBufs B{vec(L.r), vec(L.wb), vec(L.wj), vec(L.t1), vec(L.t2), vec(L.Vb), (RState*)(w + L.rs), part, mem};
  const size_t n = c->Kint;
  double* dtp = &scal[0];
  const bool pc = scheme == PCEXP_SCHEME_PCEXP;

  // ---- forward step, keeping both Krylov bases
  to_int(c, u_n, un, st);
  k_set_scalar(dtp, dt, st);
  if (!residual_int(c, un, Rn, st)) return fail(c, PCEXP_E_UNSUPPORTED, "no kernel");
  arnoldi_run<double>(c, PCEXP_JVP_TANGENT, PCEXP_PREC_F64, un, nullptr, Rn, Rn, dtp, 1, m, ks1, part, mem, V1, st);
  k_combine<double, double>(V1, c->Kld, ks1, un, us, x1, 1.0, dtp, n, st);
  if (pc) {
    if (!residual_int(c, us, Rs, st)) return fail(c, PCEXP_E_UNSUPPORTED, "no kernel");
    jvp_int(c, PCEXP_JVP_TANGENT, PCEXP_PREC_F64, un, nullptr, x1, B.wj, nullptr, nullptr, nullptr, nullptr, st);
    k_glue_d<double>(Rs, Rn, B.wj, Rs, n, st);   // Rs <- d = R(u*) - R_n - J_n x1
    arnoldi_run<double>(c, PCEXP_JVP_TANGENT, PCEXP_PREC_F64, un, nullptr, Rs, Rn, dtp, 1, m, ks2, part, mem, V2,
                        st);
  }
  int M1 = 0, M2 = 0;
  if (hipMemcpyAsync(&M1, &ks1->m_eff, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      (pc && hipMemcpyAsync(&M2, &ks2->m_eff, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(c, PCEXP_E_HIP, "step_vjp sync failed");

  // ---- reverse sweep; acc accumulates u_n_bar
  to_int(c, ubar_np1, ub, st);
  k_fill<double>(acc, 0.0, n, nullptr, st);
  if (pc) {
    // u_{n+1} = u* + x2 (x2 = 1/2 dt V2 y2): x2_bar = u*_bar = ub
    arnoldi_reverse(c, un, ks2, M2, V2, 0.5, dtp, ub, db, acc, B, st);   // db = d_bar
    // d = R(u*) - R_n - J(u_n) x1
    vjp_int(c, us, nullptr, db, B.t1, nullptr, true, st);                  // J(u*)^T d_bar
    RvComb a{};
    a.x = ub; a.axc = 1.0; a.y = B.t1; a.ayc = 1.0;
    k_rv_combine(a, xb, n, st);                                            // xb = u*_bar
    vjp_int(c, un, x1, db, B.t1, B.t2, false, st);                         // J^T d_bar, (d_u[J x1])^T d_bar
    a = RvComb{};
    a.x = xb; a.axc = 1.0; a.y = B.t1; a.ayc = -1.0;
    k_rv_combine(a, B.r, n, st);                                           // x1_bar = u*_bar - J^T d_bar
    a = RvComb{};
    a.x = acc; a.axc = 1.0; a.y = B.t2; a.ayc = -1.0;
    k_rv_combine(a, acc, n, st);
    a = RvComb{};
    a.x = acc; a.axc = 1.0; a.y = xb; a.ayc = 1.0;
    k_rv_combine(a, acc, n, st);                                           // u* = u_n + x1
    a = RvComb{};
    a.x = B.r; a.axc = 1.0;
    k_rv_combine(a, xb, n, st);                                            // xb = x1_bar
    arnoldi_reverse(c, un, ks1, M1, V1, 1.0, dtp, xb, Rs, acc, B, st);     // Rs = b1_bar
    a = RvComb{};
    a.x = Rs; a.axc = 1.0; a.y = db; a.ayc = -1.0;
    k_rv_combine(a, Rs, n, st);                                            // R_n_bar = b1_bar - d_bar
  } else {
    arnoldi_reverse(c, un, ks1, M1, V1, 1.0, dtp, ub, Rs, acc, B, st);     // Rs = R_n_bar
    RvComb a{};
    a.x = acc; a.axc = 1.0; a.y = ub; a.ayc = 1.0;
    k_rv_combine(a, acc, n, st);                                           // u_{n+1} = u_n + x1
  }
  vjp_int(c, un, nullptr, Rs, B.t1, nullptr, true, st);                    // R_n = R(u_n)
  RvComb a{};
  a.x = acc; a.axc = 1.0; a.y = B.t1; a.ayc = 1.0;
  k_rv_combine(a, acc, n, st);
  to_abi(c, acc, ubar_n, st);
  return hip_check(c, "step_vjp");
}

pcexp_status pcexp_profile(pcexp_ctx* c, int32_t op, double* out) {
  if (!c) return PCEXP_E_ARG;
  if (op == 0) {
    c->prof = false;
    return PCEXP_OK;
  }
  if (op == 1) {
    if (c->ev.empty()) {
      c->ev.resize(65536);
      for (auto& e : c->ev)
        if (hipEventCreate(&e) != hipSuccess) return fail(c, PCEXP_E_HIP, "hipEventCreate failed");
    }
    c->recs.clear();
    c->prof = true;
    return PCEXP_OK;
  }
  if (op == 2) {
    if (!out) return fail(c, PCEXP_E_ARG, "out is NULL");
    for (int i = 0; i < 3 * PCEXP_PROF_NCLASS; ++i) out[i] = 0.0;
    if (hipDeviceSynchronize() != hipSuccess) return fail(c, PCEXP_E_HIP, "sync failed");
    for (const auto& r : c->recs) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, c->ev[r.e0], c->ev[r.e0 + 1]) != hipSuccess) continue;
      out[3 * r.cls] += ms;
      out[3 * r.cls + 1] += 1.0;
      out[3 * r.cls + 2] += r.bytes;
    }
    return PCEXP_OK;
  }
  return fail(c, PCEXP_E_ARG, "bad profile op");
}

}  // extern "C"
