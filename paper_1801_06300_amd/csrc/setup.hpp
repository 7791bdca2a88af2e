// Host-side discretisation set-up: face connectivity, periodic pairing,
// geometry, Gauss-Jacobi quadrature, reference-element basis tables and the
// per-element change of basis to the paper's global-Cartesian basis.
// Plain C++17, no HIP; everything is FP64.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace pcexp {

// Number of basis functions of total degree <= p.
int n_basis(int dim, int p);
// Monomial exponents in graded order; within a degree descending power of the
// first coordinate, then of the second.  Row-major [N][dim].
std::vector<int> graded_exponents(int dim, int p);

// n-point Gauss-Jacobi rule on [-1,1] for (1-x)^alpha (1+x)^beta
// (Golub-Welsch with a cyclic Jacobi eigen-solver).  Nodes ascending.
void gauss_jacobi(int n, double alpha, double beta, std::vector<double>& x,
                  std::vector<double>& w);

// Conical-product rule on the reference simplex (vertices 0, e_1, .., e_d):
// q points per collapsed direction, weights summing to 1/d!.
void simplex_rule(int dim, int q, std::vector<double>& pts, std::vector<double>& w);

// Face rule in barycentric form: mu [nfq][dim] w.r.t. the face's ordered
// vertices, weights summing to 1.
void face_rule(int dim, int q, std::vector<double>& mu, std::vector<double>& w);

// The rules of the DG operator of degree p: the conical-product rules with
// q = p + 1, except dim = 3, p = 2, which takes the symmetric rules of the
// same degree 5 with fewer points (14 on the tetrahedron, Radon's 7 on each
// triangular face).  Volume rule as simplex_rule, face rule as face_rule.
void dg_rules(int dim, int p, std::vector<double>& pts, std::vector<double>& w, std::vector<double>& mu,
              std::vector<double>& wf);

struct MeshIn {
  int dim = 0;
  int64_t n_vert = 0, n_elem = 0, n_bface = 0;
  const double* vert = nullptr;
  const int32_t* elem = nullptr;
  const int32_t* vert_canon = nullptr;
  const int32_t* bface = nullptr;
  const int32_t* bface_tag = nullptr;
};

// Everything the device needs, in the internal layouts.
struct Setup {
  int dim = 0, p = 0, nv = 0, nb = 0, nq = 0, nfq = 0, nf = 0, nori = 0;
  int64_t nE = 0, Epad = 0;
  // reference tables (FP64)
  std::vector<double> B;     // [nq][nb]
  std::vector<double> Dg;    // [nq][nb][dim]
  std::vector<double> wq;    // [nq]
  std::vector<double> Bf;    // [nf][nori][nfq][nb]
  std::vector<double> fpts;  // [nf][nori][nfq][dim] reference coordinates of the face points
  std::vector<double> wf;    // [nfq]
  std::vector<double> nref;  // [nf][dim]
  std::vector<double> Bc;    // [nb] basis at the reference centroid
  std::vector<double> ref_pts;  // [nq][dim]
  // per element, internal order, SoA with stride Epad
  std::vector<double> ainv;  // [dim*dim][Epad]
  std::vector<double> sdet;  // [Epad] sqrt(det A)
  std::vector<double> x0;    // [dim][Epad] first vertex
  std::vector<double> amat;  // [dim*dim][Epad] A (columns = edges)
  std::vector<double> hE;    // [Epad] 2 d |E| / |dE|
  std::vector<int32_t> nbr;    // [nf][Epad] internal neighbour index or -1
  std::vector<int32_t> finfo;  // [nf][Epad] packed face info
  // ABI <-> internal
  std::vector<int32_t> perm;   // [nE] internal index of ABI element e
  std::vector<double> Q;       // [nE][nb][nb] u_ref_i = sum_j Q[e][i][j] u_paper_j (ABI order)
  double volume_total = 0.0;
};

// finfo bit fields
inline int finfo_nbr_face(int v) { return v & 3; }
inline int finfo_nbr_ori(int v) { return (v >> 2) & 7; }
inline int finfo_own_ori(int v) { return (v >> 5) & 7; }
inline int finfo_bc(int v) { return (v >> 8) & 3; }

// Returns an empty string on success, else an error message (mesh errors are
// prefixed "mesh:").  `tile` is the element padding granularity.
std::string build_setup(const MeshIn& mesh, int p, int tile, Setup& out);

// Reference basis evaluation (values [npts][nb], gradients [npts][nb][dim]).
void ref_basis_eval(int dim, int p, const std::vector<double>& pts, std::vector<double>* val,
                    std::vector<double>* grad);

}  // namespace pcexp
