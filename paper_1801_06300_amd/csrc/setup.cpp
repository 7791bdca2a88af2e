// Host-side discretisation set-up (see setup.hpp).
//
// Paper anchors: Sec. 4.2 (DG weak form, eq. (euler3)); Sec. 4.3 (orthonormal
// basis in global Cartesian coordinates, eqs. (basis2), (basis), Alg. 1);
// Sec. 5 eq. (x3d) (h_E = 2 d |E| / |dE|).
//
// The device works in a reference-element orthonormal basis: phi_hat_i on the
// reference simplex, orthonormal for d xi, mapped affinely and divided by
// sqrt(det A).  The paper's element basis psi^E spans the same polynomials and
// is orthonormal for the same inner product, so the two are related by an
// orthogonal Nb x Nb matrix Q_E per element; every PCEXP quantity (residual,
// JVP, 2-norms, dot products, phi-actions) transforms covariantly, and Q_E is
// applied only at the ABI boundary.
//
// Face quadrature points: a face shared by elements E and N is parametrised by
// the element of smaller index (a boundary face by its element); its ordered
// vertices are that element's local face vertices in increasing local order.
// Each side evaluates its basis at those points through a table indexed by
// (local face, permutation of the face vertices).
#include "setup.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <thread>
#include <unordered_map>

namespace pcexp {

int n_basis(int dim, int p) {
  return dim == 2 ? (p + 1) * (p + 2) / 2 : (p + 1) * (p + 2) * (p + 3) / 6;
}

std::vector<int> graded_exponents(int dim, int p) {
  std::vector<int> e;
  for (int deg = 0; deg <= p; ++deg) {
    if (dim == 1) {
      e.push_back(deg);
    } else if (dim == 2) {
      for (int a = deg; a >= 0; --a) { e.push_back(a); e.push_back(deg - a); }
    } else {
      for (int a = deg; a >= 0; --a)
        for (int b = deg - a; b >= 0; --b) {
          e.push_back(a); e.push_back(b); e.push_back(deg - a - b);
        }
    }
  }
  return e;
}

// Cyclic Jacobi eigenvalue iteration for a small symmetric matrix (row-major).
static void sym_eig(int n, std::vector<double>& A, std::vector<double>& V) {
  V.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
    if (off < 1e-300) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (apq == 0.0) continue;
        double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // rotate columns p, q
          double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rotate rows p, q
          double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
}

void gauss_jacobi(int n, double a, double b, std::vector<double>& x, std::vector<double>& w) {
  // Jacobi matrix of the monic Jacobi polynomials (three-term recurrence).
  std::vector<double> J(n * n, 0.0);
  for (int k = 0; k < n; ++k) {
    double s = 2.0 * k + a + b;
    J[k * n + k] = (k == 0) ? (b - a) / (a + b + 2.0) : (b * b - a * a) / (s * (s + 2.0));
    if (k >= 1) {
      double num = 4.0 * k * (k + a) * (k + b) * (k + a + b);
      double den = s * s * (s + 1.0) * (s - 1.0);
      double off = std::sqrt(num / den);
      J[k * n + k - 1] = J[(k - 1) * n + k] = off;
    }
  }
  std::vector<double> V;
  sym_eig(n, J, V);
  double mu0 = std::pow(2.0, a + b + 1.0) * std::tgamma(a + 1.0) * std::tgamma(b + 1.0) /
               std::tgamma(a + b + 2.0);
  std::vector<std::pair<double, double>> nw(n);
  for (int k = 0; k < n; ++k) nw[k] = {J[k * n + k], mu0 * V[0 * n + k] * V[0 * n + k]};
  std::sort(nw.begin(), nw.end());
  x.resize(n);
  w.resize(n);
  for (int k = 0; k < n; ++k) { x[k] = nw[k].first; w[k] = nw[k].second; }
}

void simplex_rule(int dim, int q, std::vector<double>& pts, std::vector<double>& w) {
  std::vector<double> xa, wa, xb, wb, xc, wc;
  gauss_jacobi(q, 0.0, 0.0, xa, wa);
  pts.clear();
  w.clear();
  if (dim == 1) {
    for (int i = 0; i < q; ++i) { pts.push_back(0.5 * (1 + xa[i])); w.push_back(0.5 * wa[i]); }
    return;
  }
  gauss_jacobi(q, 1.0, 0.0, xb, wb);
  if (dim == 2) {
    for (int ib = 0; ib < q; ++ib)
      for (int ia = 0; ia < q; ++ia) {
        double eta = 0.5 * (1 + xb[ib]);
        double xi = 0.5 * (1 + xa[ia]) * (1 - eta);
        pts.push_back(xi); pts.push_back(eta);
        w.push_back(wa[ia] * wb[ib] / 8.0);
      }
    return;
  }
  gauss_jacobi(q, 2.0, 0.0, xc, wc);
  for (int ic = 0; ic < q; ++ic)
    for (int ib = 0; ib < q; ++ib)
      for (int ia = 0; ia < q; ++ia) {
        double zeta = 0.5 * (1 + xc[ic]);
        double eta = 0.5 * (1 + xb[ib]) * (1 - zeta);
        double xi = 0.5 * (1 + xa[ia]) * (1 - eta - zeta);
        pts.push_back(xi); pts.push_back(eta); pts.push_back(zeta);
        w.push_back(wa[ia] * wb[ib] * wc[ic] / 64.0);
      }
}

void face_rule(int dim, int q, std::vector<double>& mu, std::vector<double>& w) {
  std::vector<double> pts, ww;
  simplex_rule(dim - 1, q, pts, ww);
  int n = (int)ww.size();
  double s = 0.0;
  for (double x : ww) s += x;
  mu.assign(n * dim, 0.0);
  w.resize(n);
  for (int r = 0; r < n; ++r) {
    double acc = 0.0;
    for (int j = 1; j < dim; ++j) { mu[r * dim + j] = pts[r * (dim - 1) + j - 1]; acc += mu[r * dim + j]; }
    mu[r * dim + 0] = 1.0 - acc;
    w[r] = ww[r] / s;
  }
}

// Radon's 7-point triangle rule, exact to degree 5: the centroid (weight
// 9/40 of the area) and the orbits of the barycentric point (a, a, 1 - 2a)
// for a = (6 -+ sqrt 15)/21 (weights (155 -+ sqrt 15)/1200).  bary [7][3],
// weights summing to 1; each orbit lists 1 - 2a at index 0, 1, 2 in turn.
static void radon7(std::vector<double>& bary, std::vector<double>& w) {
  const double r15 = std::sqrt(15.0);
  bary = {1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0};
  w = {9.0 / 40.0};
  const double av[2] = {(6.0 - r15) / 21.0, (6.0 + r15) / 21.0};
  const double wv[2] = {(155.0 - r15) / 1200.0, (155.0 + r15) / 1200.0};
  for (int o = 0; o < 2; ++o)
    for (int k = 0; k < 3; ++k) {
      for (int j = 0; j < 3; ++j) bary.push_back(j == k ? 1.0 - 2.0 * av[o] : av[o]);
      w.push_back(wv[o]);
    }
}

// The 14-point fully symmetric tetrahedron rule, exact to degree 5, with
// positive weights: two orbits of (a, a, a, 1 - 3a) (4 points each, 1 - 3a at
// index 0..3) and the orbit of (b, b, 1/2 - b, 1/2 - b) (6 points, b at the
// index pairs i < j in lexicographic order); the parameters solve the moment
// equations of degree <= 5.  bary [14][4], weights summing to 1/6.
static void tet14(std::vector<double>& bary, std::vector<double>& w) {
  const double av[2] = {0.0927352503108912, 0.3108859192633006};
  const double wv[3] = {0.01224884051939366, 0.01878132095300264, 0.007091003462846911};
  const double b = 0.0455037041256496;
  bary.clear();
  w.clear();
  for (int o = 0; o < 2; ++o)
    for (int k = 0; k < 4; ++k) {
      for (int j = 0; j < 4; ++j) bary.push_back(j == k ? 1.0 - 3.0 * av[o] : av[o]);
      w.push_back(wv[o]);
    }
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j) {
      for (int k = 0; k < 4; ++k) bary.push_back(k == i || k == j ? b : 0.5 - b);
      w.push_back(wv[2]);
    }
}

void dg_rules(int dim, int p, std::vector<double>& pts, std::vector<double>& w, std::vector<double>& mu,
              std::vector<double>& wf) {
  if (dim == 3 && p == 2) {
    std::vector<double> bary;
    tet14(bary, w);
    pts.clear();
    for (size_t q = 0; q < w.size(); ++q)
      for (int a = 1; a < 4; ++a) pts.push_back(bary[q * 4 + a]);
    radon7(mu, wf);
    return;
  }
  simplex_rule(dim, p + 1, pts, w);
  face_rule(dim, p + 1, mu, wf);
}

// ---------------------------------------------------------------- bases
static void monomials(int dim, const std::vector<int>& ex, const double* z, double* val,
                      double* grad /* [N][dim] or null */) {
  int N = (int)ex.size() / dim;
  for (int i = 0; i < N; ++i) {
    double v = 1.0;
    for (int a = 0; a < dim; ++a) v *= std::pow(z[a], ex[i * dim + a]);
    val[i] = v;
    if (grad) {
      for (int a = 0; a < dim; ++a) {
        int e = ex[i * dim + a];
        double g = 0.0;
        if (e > 0) {
          g = e * std::pow(z[a], e - 1);
          for (int b = 0; b < dim; ++b)
            if (b != a) g *= std::pow(z[b], ex[i * dim + b]);
        }
        grad[i * dim + a] = g;
      }
    }
  }
}

// Coefficients C (lower triangular, row i = basis function i) of the
// reference orthonormal basis in monomials of xi - centroid: inverse Cholesky
// factor of the reference Gram matrix (exact quadrature).
static std::vector<double> ref_coeffs(int dim, int p) {
  std::vector<int> ex = graded_exponents(dim, p);
  int N = (int)ex.size() / dim;
  std::vector<double> pts, w;
  simplex_rule(dim, p + 1, pts, w);
  int nq = (int)w.size();
  std::vector<double> G(N * N, 0.0), m(N);
  double cen = 1.0 / (dim + 1);
  for (int q = 0; q < nq; ++q) {
    double z[3];
    for (int a = 0; a < dim; ++a) z[a] = pts[q * dim + a] - cen;
    monomials(dim, ex, z, m.data(), nullptr);
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) G[i * N + j] += w[q] * m[i] * m[j];
  }
  std::vector<double> L(N * N, 0.0);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = G[i * N + j];
      for (int k = 0; k < j; ++k) s -= L[i * N + k] * L[j * N + k];
      L[i * N + j] = (i == j) ? std::sqrt(s) : s / L[j * N + j];
    }
  std::vector<double> C(N * N, 0.0);  // C = L^{-1} by forward substitution
  for (int c = 0; c < N; ++c) {
    for (int i = 0; i < N; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) s -= L[i * N + k] * C[k * N + c];
      C[i * N + c] = s / L[i * N + i];
    }
  }
  return C;
}

void ref_basis_eval(int dim, int p, const std::vector<double>& pts, std::vector<double>* val,
                    std::vector<double>* grad) {
  std::vector<int> ex = graded_exponents(dim, p);
  int N = (int)ex.size() / dim;
  std::vector<double> C = ref_coeffs(dim, p);
  int np = (int)pts.size() / dim;
  if (val) val->assign(np * N, 0.0);
  if (grad) grad->assign(np * N * dim, 0.0);
  std::vector<double> m(N), g(N * dim);
  double cen = 1.0 / (dim + 1);
  for (int q = 0; q < np; ++q) {
    double z[3];
    for (int a = 0; a < dim; ++a) z[a] = pts[q * dim + a] - cen;
    monomials(dim, ex, z, m.data(), g.data());
    for (int i = 0; i < N; ++i)
      for (int a = 0; a <= i; ++a) {
        if (val) (*val)[q * N + i] += C[i * N + a] * m[a];
        if (grad)
          for (int d = 0; d < dim; ++d) (*grad)[(q * N + i) * dim + d] += C[i * N + a] * g[a * dim + d];
      }
  }
}

// ---------------------------------------------------------------- helpers
static int perm_index(int d, const int* pi) {
  // lexicographic index of a permutation of 0..d-1 (d = 2 or 3)
  int idx = 0;
  for (int i = 0; i < d; ++i) {
    int smaller = 0;
    for (int j = i + 1; j < d; ++j) smaller += pi[j] < pi[i];
    int f = 1;
    for (int k = 2; k <= d - 1 - i; ++k) f *= k;
    idx += smaller * f;
  }
  return idx;
}

static void perm_from_index(int d, int idx, int* pi) {
  std::vector<int> pool;
  for (int i = 0; i < d; ++i) pool.push_back(i);
  for (int i = 0; i < d; ++i) {
    int f = 1;
    for (int k = 2; k <= d - 1 - i; ++k) f *= k;
    int s = idx / f;
    idx %= f;
    pi[i] = pool[s];
    pool.erase(pool.begin() + s);
  }
}

struct Key {
  std::array<int64_t, 3> v;
  bool operator==(const Key& o) const { return v == o.v; }
};
struct KeyHash {
  size_t operator()(const Key& k) const {
    uint64_t h = 1469598103934665603ull;
    for (int64_t x : k.v) { h ^= (uint64_t)x + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2); }
    return (size_t)h;
  }
};

static void inv_det(int d, const double* A, double* Ainv, double* det) {
  if (d == 2) {
    double dt = A[0] * A[3] - A[1] * A[2];
    *det = dt;
    Ainv[0] = A[3] / dt; Ainv[1] = -A[1] / dt; Ainv[2] = -A[2] / dt; Ainv[3] = A[0] / dt;
  } else {
    double a = A[0], b = A[1], c = A[2], e = A[3], f = A[4], g = A[5], h = A[6], i = A[7], k = A[8];
    double dt = a * (f * k - g * i) - b * (e * k - g * h) + c * (e * i - f * h);
    *det = dt;
    Ainv[0] = (f * k - g * i) / dt; Ainv[1] = (c * i - b * k) / dt; Ainv[2] = (b * g - c * f) / dt;
    Ainv[3] = (g * h - e * k) / dt; Ainv[4] = (a * k - c * h) / dt; Ainv[5] = (c * e - a * g) / dt;
    Ainv[6] = (e * i - f * h) / dt; Ainv[7] = (b * h - a * i) / dt; Ainv[8] = (a * f - b * e) / dt;
  }
}

std::string build_setup(const MeshIn& m, int p, int tile, Setup& S) {
  const int d = m.dim;
  if (d != 2 && d != 3) return "arg: dim must be 2 or 3";
  if (p < 0 || (d == 2 && p > 3) || (d == 3 && p > 2)) return "unsupported: polynomial degree";
  if (m.n_elem <= 0 || m.n_vert <= 0 || !m.vert || !m.elem) return "arg: empty mesh";
  if (m.n_bface > 0 && (!m.bface || !m.bface_tag)) return "arg: boundary arrays missing";
  const int nf = d + 1;
  const int64_t nE = m.n_elem;
  S.dim = d; S.p = p; S.nv = d + 2; S.nb = n_basis(d, p); S.nf = nf;
  S.nori = d == 2 ? 2 : 6;
  S.nE = nE;
  S.Epad = ((nE + tile - 1) / tile) * tile;
  const int64_t Ep = S.Epad;
  auto canon = [&](int64_t v) -> int64_t { return m.vert_canon ? (int64_t)m.vert_canon[v] : v; };

  // ---- validate elements, geometry
  std::vector<double> A(nE * d * d), Ai(nE * d * d), det(nE), X0(nE * d), area(nE * nf);
  for (int64_t e = 0; e < nE; ++e) {
    int64_t c[4];
    for (int j = 0; j <= d; ++j) {
      int64_t v = m.elem[e * (d + 1) + j];
      if (v < 0 || v >= m.n_vert) return "mesh: vertex index out of range";
      if (m.vert_canon && (m.vert_canon[v] < 0 || m.vert_canon[v] >= m.n_vert))
        return "mesh: vert_canon out of range";
      c[j] = canon(v);
    }
    for (int j = 0; j <= d; ++j)
      for (int k = j + 1; k <= d; ++k)
        if (c[j] == c[k]) return "mesh: element touches its own periodic image";
    const double* P0 = m.vert + (int64_t)m.elem[e * (d + 1)] * d;
    for (int a = 0; a < d; ++a) X0[e * d + a] = P0[a];
    for (int j = 1; j <= d; ++j) {
      const double* Pj = m.vert + (int64_t)m.elem[e * (d + 1) + j] * d;
      for (int a = 0; a < d; ++a) A[e * d * d + a * d + (j - 1)] = Pj[a] - P0[a];
    }
    inv_det(d, &A[e * d * d], &Ai[e * d * d], &det[e]);
    if (!(det[e] > 0.0)) return "mesh: element with non-positive orientation";
  }

  // ---- faces
  std::unordered_map<Key, std::vector<int64_t>, KeyHash> faces;
  faces.reserve(nE * nf);
  auto local_face = [&](int f, int* lv) {
    int k = 0;
    for (int j = 0; j <= d; ++j)
      if (j != f) lv[k++] = j;
  };
  auto face_key = [&](int64_t e, int f) {
    int lv[3];
    local_face(f, lv);
    Key k{{-1, -1, -1}};
    for (int j = 0; j < d; ++j) k.v[j] = canon(m.elem[e * (d + 1) + lv[j]]);
    std::sort(k.v.begin(), k.v.begin() + d);
    return k;
  };
  for (int64_t e = 0; e < nE; ++e)
    for (int f = 0; f < nf; ++f) faces[face_key(e, f)].push_back(e * nf + f);
  std::unordered_map<Key, int, KeyHash> btag;
  for (int64_t b = 0; b < m.n_bface; ++b) {
    Key k{{-1, -1, -1}};
    for (int j = 0; j < d; ++j) {
      int64_t v = m.bface[b * d + j];
      if (v < 0 || v >= m.n_vert) return "mesh: boundary vertex index out of range";
      k.v[j] = canon(v);
    }
    std::sort(k.v.begin(), k.v.begin() + d);
    int t = m.bface_tag[b];
    if (t != 1 && t != 2) return "mesh: unknown boundary tag";
    btag[k] = t;
  }
  std::vector<int64_t> nbr_abi(nE * nf, -1);
  std::vector<int> nbr_face(nE * nf, -1), bc(nE * nf, 0);
  for (auto& kv : faces) {
    const auto& L = kv.second;
    if (L.size() == 2) {
      nbr_abi[L[0]] = L[1] / nf; nbr_face[L[0]] = (int)(L[1] % nf);
      nbr_abi[L[1]] = L[0] / nf; nbr_face[L[1]] = (int)(L[0] % nf);
    } else if (L.size() == 1) {
      auto it = btag.find(kv.first);
      if (it == btag.end()) return "mesh: unmatched face without boundary tag";
      bc[L[0]] = it->second;
    } else {
      return "mesh: face shared by more than two elements";
    }
  }

  // ---- orientation of each side relative to the owner's face parametrisation
  std::vector<int> own_ori(nE * nf, 0), nbr_ori(nE * nf, 0);
  for (int64_t e = 0; e < nE; ++e)
    for (int f = 0; f < nf; ++f) {
      int64_t id = e * nf + f;
      int64_t n = nbr_abi[id];
      if (n < 0) continue;
      int fn = nbr_face[id];
      int64_t ow = std::min(e, n);
      int ofc = (ow == e) ? f : fn;
      int lv[3];
      local_face(ofc, lv);
      int64_t cvec[3];
      for (int j = 0; j < d; ++j) cvec[j] = canon(m.elem[ow * (d + 1) + lv[j]]);
      auto ori_of = [&](int64_t el, int fl) {
        int l2[3], pi[3];
        local_face(fl, l2);
        for (int j = 0; j < d; ++j) {
          int64_t cid = canon(m.elem[el * (d + 1) + l2[j]]);
          pi[j] = -1;
          for (int t = 0; t < d; ++t)
            if (cvec[t] == cid) pi[j] = t;
        }
        return perm_index(d, pi);
      };
      own_ori[id] = ori_of(e, f);
      nbr_ori[id] = ori_of(n, fn);
    }

  // ---- reference quadrature and tables
  std::vector<double> pts, w, mu, wf;
  dg_rules(d, p, pts, w, mu, wf);
  S.nq = (int)w.size();
  S.ref_pts = pts;
  S.wq = w;
  ref_basis_eval(d, p, pts, &S.B, &S.Dg);
  S.nfq = (int)wf.size();
  S.wf = wf;
  S.nref.assign(nf * d, 0.0);
  double fact = (d == 2) ? 1.0 : 2.0;  // (d-1)!
  for (int a = 0; a < d; ++a) S.nref[0 * d + a] = 1.0 / fact;
  for (int f = 1; f < nf; ++f) S.nref[f * d + (f - 1)] = -1.0 / fact;
  S.Bf.assign((size_t)nf * S.nori * S.nfq * S.nb, 0.0);
  S.fpts.assign((size_t)nf * S.nori * S.nfq * d, 0.0);
  for (int f = 0; f < nf; ++f) {
    int lv[3];
    local_face(f, lv);
    for (int o = 0; o < S.nori; ++o) {
      int pi[3];
      perm_from_index(d, o, pi);
      std::vector<double> fp(S.nfq * d, 0.0);
      for (int r = 0; r < S.nfq; ++r)
        for (int j = 0; j < d; ++j) {
          double nu = mu[r * d + pi[j]];
          if (lv[j] > 0) fp[r * d + lv[j] - 1] += nu;  // reference vertex lv[j] = e_{lv[j]} (0 = origin)
        }
      std::copy(fp.begin(), fp.end(), S.fpts.begin() + ((size_t)(f * S.nori + o) * S.nfq) * d);
      std::vector<double> val;
      ref_basis_eval(d, p, fp, &val, nullptr);
      std::copy(val.begin(), val.end(), S.Bf.begin() + ((size_t)(f * S.nori + o) * S.nfq) * S.nb);
    }
  }
  {
    std::vector<double> cpt(d, 1.0 / (d + 1)), val;
    ref_basis_eval(d, p, cpt, &val, nullptr);
    S.Bc = val;
  }

  // ---- internal order (identity) and per-element arrays
  S.perm.resize(nE);
  for (int64_t e = 0; e < nE; ++e) S.perm[e] = (int32_t)e;
  S.ainv.assign((size_t)d * d * Ep, 0.0);
  S.amat.assign((size_t)d * d * Ep, 0.0);
  S.sdet.assign(Ep, 0.0);
  S.x0.assign((size_t)d * Ep, 0.0);
  S.hE.assign(Ep, 0.0);
  S.nbr.assign((size_t)nf * Ep, -1);
  S.finfo.assign((size_t)nf * Ep, 0);
  double fd = (d == 2) ? 2.0 : 6.0;  // d!
  S.volume_total = 0.0;
  for (int64_t e = 0; e < nE; ++e) {
    int64_t ie = S.perm[e];
    double surf = 0.0;
    for (int f = 0; f < nf; ++f) {
      // |f| n_f = det(A) A^{-T} nref_f
      double nl[3] = {0, 0, 0};
      for (int c = 0; c < d; ++c)
        for (int r = 0; r < d; ++r) nl[c] += Ai[e * d * d + r * d + c] * S.nref[f * d + r];
      double s2 = 0.0;
      for (int c = 0; c < d; ++c) s2 += nl[c] * nl[c];
      surf += det[e] * std::sqrt(s2);
      int64_t id = e * nf + f;
      int64_t n = nbr_abi[id];
      S.nbr[f * Ep + ie] = n >= 0 ? S.perm[n] : -1;
      int fn = n >= 0 ? nbr_face[id] : 0;
      S.finfo[f * Ep + ie] = (fn & 3) | ((nbr_ori[id] & 7) << 2) | ((own_ori[id] & 7) << 5) |
                             ((bc[id] & 3) << 8);
    }
    for (int k = 0; k < d * d; ++k) {
      S.ainv[k * Ep + ie] = Ai[e * d * d + k];
      S.amat[k * Ep + ie] = A[e * d * d + k];
    }
    for (int a = 0; a < d; ++a) S.x0[a * Ep + ie] = X0[e * d + a];
    S.sdet[ie] = std::sqrt(det[e]);
    double vol = det[e] / fd;
    S.hE[ie] = 2.0 * d * vol / surf;
    S.volume_total += vol;
  }

  // ---- Q_E: u_ref = Q_E u_paper (paper basis: Sec. 4.3, Alg. 1 read as MGS
  //      against the orthonormal psi_j, normalised after the inner loop)
  const int nb = S.nb, nq = S.nq;
  std::vector<int> ex = graded_exponents(d, p);
  S.Q.assign((size_t)nE * nb * nb, 0.0);
  auto work = [&](int64_t e_begin, int64_t e_end) {
    std::vector<double> chi(nq * nb), Wq(nq), Cm(nb * nb), G(nb * nb), c(nb);
    for (int64_t e = e_begin; e < e_end; ++e) {
      double X[4][3];
      for (int j = 0; j <= d; ++j)
        for (int a = 0; a < d; ++a) X[j][a] = m.vert[(int64_t)m.elem[e * (d + 1) + j] * d + a];
      double xc[3] = {0, 0, 0}, lo[3], hi[3];
      for (int a = 0; a < d; ++a) {
        lo[a] = hi[a] = X[0][a];
        for (int j = 0; j <= d; ++j) {
          xc[a] += X[j][a] / (d + 1);
          lo[a] = std::min(lo[a], X[j][a]);
          hi[a] = std::max(hi[a], X[j][a]);
        }
      }
      for (int qq = 0; qq < nq; ++qq) {
        double z[3];
        for (int a = 0; a < d; ++a) {
          double x = X[0][a];
          for (int j = 1; j <= d; ++j) x += (X[j][a] - X[0][a]) * pts[qq * d + j - 1];
          z[a] = (x - xc[a]) / (0.5 * (hi[a] - lo[a]));
        }
        monomials(d, ex, z, &chi[qq * nb], nullptr);
        Wq[qq] = w[qq] * det[e];
      }
      for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b) {
          double s = 0.0;
          for (int qq = 0; qq < nq; ++qq) s += Wq[qq] * chi[qq * nb + a] * chi[qq * nb + b];
          G[a * nb + b] = s;
        }
      std::fill(Cm.begin(), Cm.end(), 0.0);
      for (int i = 0; i < nb; ++i) {
        std::fill(c.begin(), c.end(), 0.0);
        c[i] = 1.0;
        for (int j = 0; j < i; ++j) {
          double wij = 0.0;
          for (int a = 0; a < nb; ++a)
            for (int b = 0; b < nb; ++b) wij += c[a] * G[a * nb + b] * Cm[j * nb + b];
          for (int a = 0; a < nb; ++a) c[a] -= wij * Cm[j * nb + a];
        }
        double nn = 0.0;
        for (int a = 0; a < nb; ++a)
          for (int b = 0; b < nb; ++b) nn += c[a] * G[a * nb + b] * c[b];
        nn = std::sqrt(nn);
        for (int a = 0; a < nb; ++a) Cm[i * nb + a] = c[a] / nn;
      }
      const double s = std::sqrt(det[e]);
      double* Qe = &S.Q[(size_t)e * nb * nb];
      for (int i = 0; i < nb; ++i)
        for (int j = 0; j < nb; ++j) {
          double acc = 0.0;
          for (int qq = 0; qq < nq; ++qq) {
            double psi = 0.0;
            for (int a = 0; a <= j; ++a) psi += Cm[j * nb + a] * chi[qq * nb + a];
            acc += w[qq] * S.B[qq * nb + i] * psi;
          }
          Qe[i * nb + j] = s * acc;
        }
    }
  };
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (nE < 4096) nt = 1;
  std::vector<std::thread> th;
  int64_t chunk = (nE + nt - 1) / nt;
  for (unsigned t = 0; t < nt; ++t) {
    int64_t a = t * chunk, b = std::min<int64_t>(nE, a + chunk);
    if (a < b) th.emplace_back(work, a, b);
  }
  for (auto& t : th) t.join();
  return "";
}

}  // namespace pcexp
