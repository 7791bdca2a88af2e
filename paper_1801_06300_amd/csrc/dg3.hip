// Instantiations of the DG kernels for tetrahedra (dim = 3), p = 0..2.
#include "dg_dispatch.hpp"

namespace pcexp {

template <int P, typename T>
static bool run_p(int flux, int mode, const DGParams<T>& prm, const DGIO<T>& io, hipStream_t st) {
  if (flux == FLUX_LF) {
    if (mode == MODE_TAN) { launch_dg<3, P, FLUX_LF, T, MODE_TAN>(prm, io, st); return true; }
    if constexpr (std::is_same<T, double>::value) {
      if (mode == MODE_RES) { launch_dg<3, P, FLUX_LF, T, MODE_RES>(prm, io, st); return true; }
      if (mode == MODE_FD) { launch_dg<3, P, FLUX_LF, T, MODE_FD>(prm, io, st); return true; }
    }
  } else {
    if (mode == MODE_TAN) { launch_dg<3, P, FLUX_ROE, T, MODE_TAN>(prm, io, st); return true; }
    if constexpr (std::is_same<T, double>::value) {
      if (mode == MODE_RES) { launch_dg<3, P, FLUX_ROE, T, MODE_RES>(prm, io, st); return true; }
      if (mode == MODE_FD) { launch_dg<3, P, FLUX_ROE, T, MODE_FD>(prm, io, st); return true; }
    }
  }
  return false;
}

template <typename T>
static bool run(int p, int flux, int mode, const DGParams<T>& prm, const DGIO<T>& io, hipStream_t st) {
  switch (p) {
    case 0: return run_p<0, T>(flux, mode, prm, io, st);
    case 1: return run_p<1, T>(flux, mode, prm, io, st);
    case 2: return run_p<2, T>(flux, mode, prm, io, st);
  }
  return false;
}

bool dg_run3_d(int p, int flux, int mode, const DGParams<double>& prm, const DGIO<double>& io, hipStream_t st) {
  return run<double>(p, flux, mode, prm, io, st);
}
bool dg_run3_f(int p, int flux, int mode, const DGParams<float>& prm, const DGIO<float>& io, hipStream_t st) {
  return run<float>(p, flux, mode, prm, io, st);
}

template <int P>
static bool vjp_p(int flux, const DGParams<double>& prm, const double* u, const double* v, const double* w,
                  double* out, double* out_d, hipStream_t st, const double* acc_scale) {
  if (out_d) {
    if (flux == FLUX_LF) launch_vjp2<3, P, FLUX_LF>(prm, u, v, w, out, out_d, acc_scale, st);
    else launch_vjp2<3, P, FLUX_ROE>(prm, u, v, w, out, out_d, acc_scale, st);
  } else {
    if (flux == FLUX_LF) launch_vjp<3, P, FLUX_LF>(prm, u, w, out, st);
    else launch_vjp<3, P, FLUX_ROE>(prm, u, w, out, st);
  }
  return true;
}

bool dg_vjp3(int p, int flux, const DGParams<double>& prm, const double* u, const double* v, const double* w,
             double* out, double* out_d, hipStream_t st, const double* acc_scale) {
  switch (p) {
    case 0: return vjp_p<0>(flux, prm, u, v, w, out, out_d, st, acc_scale);
    case 1: return vjp_p<1>(flux, prm, u, v, w, out, out_d, st, acc_scale);
    case 2: return vjp_p<2>(flux, prm, u, v, w, out, out_d, st, acc_scale);
  }
  return false;
}

}  // namespace pcexp
