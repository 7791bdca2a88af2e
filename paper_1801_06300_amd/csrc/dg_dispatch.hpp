// Run-time dispatch to the compile-time instantiations of the DG kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "dg_kernels.hpp"

namespace pcexp {

// Returns false if (dim, p, flux, mode, precision) has no instantiation.
bool dg_run_d(int dim, int p, int flux, int mode, const DGParams<double>& prm, const DGIO<double>& io,
              hipStream_t st);
bool dg_run_f(int dim, int p, int flux, int mode, const DGParams<float>& prm, const DGIO<float>& io,
              hipStream_t st);
bool dg_run2_d(int p, int flux, int mode, const DGParams<double>& prm, const DGIO<double>& io, hipStream_t st);
bool dg_run3_d(int p, int flux, int mode, const DGParams<double>& prm, const DGIO<double>& io, hipStream_t st);
bool dg_run2_f(int p, int flux, int mode, const DGParams<float>& prm, const DGIO<float>& io, hipStream_t st);
bool dg_run3_f(int p, int flux, int mode, const DGParams<float>& prm, const DGIO<float>& io, hipStream_t st);

// Transpose J(u)^T w (FP64).
// out = J(u)^T w; if out_d is not null also out_d = d/deps [J(u + eps v)^T w].
// With acc_scale (device scalar s, only with out_d) both are accumulated
// instead: out += J(u)^T w, out_d += s d/deps [J(u + eps v)^T w].
bool dg_vjp2(int p, int flux, const DGParams<double>& prm, const double* u, const double* v, const double* w,
             double* out, double* out_d, hipStream_t st, const double* acc_scale = nullptr);
bool dg_vjp3(int p, int flux, const DGParams<double>& prm, const double* u, const double* v, const double* w,
             double* out, double* out_d, hipStream_t st, const double* acc_scale = nullptr);

// Element-level helpers (elem_kernels.hip); runtime sizes, not on the hot path.
struct ElemArgs {
  int dim, nv, nb, nq, p;
  int nE, Epad;
  const double* Q;      // [nE][nb][nb]
  const int* perm;      // [nE]
  const double* sdet;   // [Epad]
  const double* x0;     // [dim][Epad]
  const double* amat;   // [dim*dim][Epad]
  const double* B;      // [nq][nb]
  const double* wq;     // [nq]
  const double* Bc;     // [nb]
  const double* refp;   // [nq][dim]
  const double* hE;     // [Epad]
  double gamma;
};
void ek_to_internal(const ElemArgs& a, const double* u_abi, double* u_int, hipStream_t st);
// value = int (p_h - p_ref)^2 dx (device scalar; with acc, value += scale times
// it; may be NULL); grad_int (optional) its gradient with respect to the
// internal coefficients; part >= Epad/256 doubles.
void ek_pressure_functional(const ElemArgs& a, const double* u_int, double p_ref, double* value, double* grad_int,
                            double* part, hipStream_t st, int acc = 0, double scale = 1.0);
void ek_to_abi(const ElemArgs& a, const double* u_int, double* u_abi, hipStream_t st);
// u_abi += scale Q^T u_int
void ek_to_abi_axpy(const ElemArgs& a, const double* u_int, double scale, double* u_abi, hipStream_t st);
void ek_quad_points(const ElemArgs& a, double* xyz, hipStream_t st);
void ek_project(const ElemArgs& a, const double* Uqp, double* u_abi, hipStream_t st);
void ek_evaluate(const ElemArgs& a, const double* u_abi, double* Uqp, hipStream_t st);
// dt of eq. (x3d) from internal u; writes cfl * min_E h_E/((2p+1)(|v|+c)) to *dt.
void ek_stable_dt(const ElemArgs& a, const double* u_int, const double* cfl_dev, double cfl, double* dt,
                  double* part, unsigned* counter, hipStream_t st);
void ek_totals(const ElemArgs& a, const double* u_int, double* out, double* part, unsigned* counter,
               hipStream_t st);

}  // namespace pcexp
