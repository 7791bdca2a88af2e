// Host-only entry points that expose the discretisation set-up for CPU tests
// (face matching, orientation tables, quadrature, change of basis).  Built
// into libpcexp_setup_probe.so, which needs no HIP runtime.
#include <cstring>

#include "setup.hpp"

extern "C" {

int pcexp_probe_gauss_jacobi(int n, double alpha, double beta, double* x, double* w) {
  std::vector<double> xx, ww;
  pcexp::gauss_jacobi(n, alpha, beta, xx, ww);
  for (int i = 0; i < n; ++i) { x[i] = xx[i]; w[i] = ww[i]; }
  return 0;
}

// sizes[0..7] = nb, nq, nfq, nori, nf, Epad, nE, dim.  Any output pointer may be NULL.
int pcexp_probe_setup(int dim, long long n_vert, const double* vert, long long n_elem, const int* elem,
                      const int* vert_canon, long long n_bface, const int* bface, const int* bface_tag, int p,
                      long long* sizes, double* ref_pts, double* wq, double* fpts, double* wf, double* Q,
                      int* nbr, int* finfo, double* sdet, double* B, double* Bf, char* err, int errlen) {
  pcexp::MeshIn m;
  m.dim = dim; m.n_vert = n_vert; m.vert = vert; m.n_elem = n_elem; m.elem = elem;
  m.vert_canon = vert_canon; m.n_bface = n_bface; m.bface = bface; m.bface_tag = bface_tag;
  pcexp::Setup S;
  std::string msg = pcexp::build_setup(m, p, 64, S);
  if (!msg.empty()) {
    if (err && errlen > 0) {
      std::strncpy(err, msg.c_str(), errlen - 1);
      err[errlen - 1] = 0;
    }
    return msg.rfind("mesh:", 0) == 0 ? -2 : -1;
  }
  if (sizes) {
    sizes[0] = S.nb; sizes[1] = S.nq; sizes[2] = S.nfq; sizes[3] = S.nori; sizes[4] = S.nf;
    sizes[5] = S.Epad; sizes[6] = S.nE; sizes[7] = S.dim;
  }
  auto cp = [](double* dst, const std::vector<double>& v) { if (dst) std::memcpy(dst, v.data(), v.size() * sizeof(double)); };
  auto cpi = [](int* dst, const std::vector<int32_t>& v) { if (dst) std::memcpy(dst, v.data(), v.size() * sizeof(int)); };
  cp(ref_pts, S.ref_pts); cp(wq, S.wq); cp(fpts, S.fpts); cp(wf, S.wf); cp(Q, S.Q); cp(sdet, S.sdet);
  cp(B, S.B); cp(Bf, S.Bf);
  cpi(nbr, S.nbr); cpi(finfo, S.finfo);
  return 0;
}

}  // extern "C"
