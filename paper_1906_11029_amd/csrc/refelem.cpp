// Reference-element tables for nodal DG on the d-simplex (section 3, DG on the tent
// patch): equispaced Lagrange basis (Silvester's product formula in barycentric
// coordinates), conical-product Gauss-Legendre quadrature, and the lambda_0-weighted
// operators of the mapped DG equation with the tent vertex numbered 0:
//   Mhat[b][a]  = int phi_b phi_a
//   D_l[b][a]   = int lambda_0 phi_a d_l phi_b           S_l = Mhat^{-1} D_l
//   E_j[b][s]   = int_{face j} lambda_0 l_s phi_b        L_j = Mhat^{-1} E_j
// (lambda_0 = delta / tent height restricted to one element).  Face j (1..d) is the face
// opposite vertex j, the coordinate face xhat_j = 0, measured in its own reference measure.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace mtp {

namespace {

// n-point Gauss-Legendre rule on [0,1] (Newton iteration on P_n).
void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = 0.5 * (1.0 - z);
    w[i] = 1.0 / ((1.0 - z * z) * dp * dp);  // 2/((1-z^2)P'^2) scaled by 1/2 for [0,1]
  }
}

// Conical-product rule on the reference k-simplex (k = 1, 2, 3), points (nq, k).
void simplex_rule(int k, int n, std::vector<double>& pts, std::vector<double>& wts) {
  std::vector<double> x, w;
  gauss_legendre01(n, x, w);
  pts.clear();
  wts.clear();
  if (k == 1) {
    for (int i = 0; i < n; ++i) { pts.push_back(x[i]); wts.push_back(w[i]); }
  } else if (k == 2) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double u = x[i], v = x[j];
        pts.push_back(u);
        pts.push_back((1 - u) * v);
        wts.push_back(w[i] * w[j] * (1 - u));
      }
  } else {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        for (int l = 0; l < n; ++l) {
          double u = x[i], v = x[j], s = x[l];
          pts.push_back(u);
          pts.push_back((1 - u) * v);
          pts.push_back((1 - u) * (1 - v) * s);
          wts.push_back(w[i] * w[j] * w[l] * (1 - u) * (1 - u) * (1 - v));
        }
  }
}

// Silvester's Lagrange basis at the equispaced nodes:
//   phi_a(lambda) = prod_m prod_{r < alpha_m} (p lambda_m - r) / (r + 1)
// Values and derivatives with respect to the reference coordinates xhat_l
// (lambda_l = xhat_l, lambda_0 = 1 - sum xhat, so d/dxhat_l = d/dlambda_l - d/dlambda_0).
struct Lagrange {
  int d, p, np;
  const std::vector<int>& mi;
  Lagrange(int d_, int p_, const std::vector<int>& mi_) : d(d_), p(p_), np((int)mi_.size() / (d_ + 1)), mi(mi_) {}

  static double factor(int a, int p, double lam, double* dval) {
    double val = 1.0, der = 0.0;
    for (int r = 0; r < a; ++r) {
      double f = (p * lam - r) / (r + 1.0);
      double df = p / (r + 1.0);
      der = der * f + val * df;
      val *= f;
    }
    if (dval) *dval = der;
    return val;
  }

  void eval(const double* xh, double* phi, double* grad /* np*d or null */) const {
    double lam[4];
    lam[0] = 1.0;
    for (int l = 0; l < d; ++l) { lam[l + 1] = xh[l]; lam[0] -= xh[l]; }
    for (int a = 0; a < np; ++a) {
      double f[4], df[4];
      for (int m = 0; m <= d; ++m) f[m] = factor(mi[a * (d + 1) + m], p, lam[m], &df[m]);
      double val = 1.0;
      for (int m = 0; m <= d; ++m) val *= f[m];
      phi[a] = val;
      if (grad) {
        double dl[4];
        for (int m = 0; m <= d; ++m) {
          double prod = df[m];
          for (int q = 0; q <= d; ++q)
            if (q != m) prod *= f[q];
          dl[m] = prod;
        }
        for (int l = 0; l < d; ++l) grad[a * d + l] = dl[l + 1] - dl[0];
      }
    }
  }
};

// Solve A X = B (A n x n symmetric positive definite, B n x k row-major) by Cholesky.
void spd_solve(int n, std::vector<double> A, std::vector<double>& B, int k) {
  for (int j = 0; j < n; ++j) {
    double s = A[j * n + j];
    for (int q = 0; q < j; ++q) s -= A[j * n + q] * A[j * n + q];
    if (!(s > 0)) throw Error(MTP_ERR_UNSUPPORTED, "reference mass matrix not positive definite");
    double r = std::sqrt(s);
    A[j * n + j] = r;
    for (int i = j + 1; i < n; ++i) {
      double t = A[i * n + j];
      for (int q = 0; q < j; ++q) t -= A[i * n + q] * A[j * n + q];
      A[i * n + j] = t / r;
    }
  }
  for (int c = 0; c < k; ++c) {
    for (int i = 0; i < n; ++i) {  // forward: L y = b
      double t = B[i * k + c];
      for (int q = 0; q < i; ++q) t -= A[i * n + q] * B[q * k + c];
      B[i * k + c] = t / A[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {  // backward: L^T x = y
      double t = B[i * k + c];
      for (int q = i + 1; q < n; ++q) t -= A[q * n + i] * B[q * k + c];
      B[i * k + c] = t / A[i * n + i];
    }
  }
}

int binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  int r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

}  // namespace

void vertex_order(int d, int k, int* order) {
  order[0] = k;
  int c = 1;
  for (int i = 0; i <= d; ++i)
    if (i != k) order[c++] = i;
}

RefElem build_refelem(int d, int p) {
  RefElem R;
  R.d = d;
  R.p = p;
  R.np = binom(p + d, d);
  R.nf = binom(p + d - 1, d - 1);
  const int np = R.np, nf = R.nf, nv = d + 1;
  // node multi-indices in the interchange order (i fastest, then j, then k)
  std::vector<int> index((size_t)std::pow(p + 1, d), -1);
  auto key = [&](const int* a) {  // a = (alpha_1..alpha_d)
    int k = 0;
    for (int l = d - 1; l >= 0; --l) k = k * (p + 1) + a[l];
    return k;
  };
  if (d == 2) {
    for (int j = 0; j <= p; ++j)
      for (int i = 0; i <= p - j; ++i) {
        int a[4] = {p - i - j, i, j, 0};
        R.mi.insert(R.mi.end(), a, a + 3);
      }
  } else {
    for (int kk = 0; kk <= p; ++kk)
      for (int j = 0; j <= p - kk; ++j)
        for (int i = 0; i <= p - j - kk; ++i) {
          int a[4] = {p - i - j - kk, i, j, kk};
          R.mi.insert(R.mi.end(), a, a + 4);
        }
  }
  for (int a = 0; a < np; ++a) index[key(&R.mi[a * nv + 1])] = a;
  auto node_of = [&](const int* alpha /* d+1 */) { return index[key(alpha + 1)]; };

  // permutations: vertex k moved to 0, the others in increasing order
  R.perm.assign(nv * np, 0);
  for (int k = 0; k <= d; ++k) {
    int order[4];
    vertex_order(d, k, order);
    for (int a = 0; a < np; ++a) {
      int old_alpha[4] = {0, 0, 0, 0};
      for (int i = 0; i <= d; ++i) old_alpha[order[i]] = R.mi[a * nv + i];
      R.perm[k * np + a] = node_of(old_alpha);
    }
  }

  // face node tables: face j (1..d), orientation o, face node s
  R.fnode.assign(d * 2 * nf, 0);
  for (int j = 1; j <= d; ++j) {
    int fv[2], c = 0;
    for (int i = 1; i <= d; ++i)
      if (i != j) fv[c++] = i;
    for (int o = 0; o < 2; ++o) {
      int f1 = fv[0], f2 = (d == 3) ? fv[1] : -1;
      if (o == 1 && d == 3) std::swap(f1, f2);
      int s = 0;
      if (d == 2) {
        for (int b1 = 0; b1 <= p; ++b1) {
          int alpha[4] = {0, 0, 0, 0};
          alpha[f1] = b1;
          alpha[0] = p - b1;
          R.fnode[((j - 1) * 2 + o) * nf + s++] = node_of(alpha);
        }
      } else {
        for (int b2 = 0; b2 <= p; ++b2)
          for (int b1 = 0; b1 <= p - b2; ++b1) {
            int alpha[4] = {0, 0, 0, 0};
            alpha[f1] = b1;
            alpha[f2] = b2;
            alpha[0] = p - b1 - b2;
            R.fnode[((j - 1) * 2 + o) * nf + s++] = node_of(alpha);
          }
      }
    }
  }

  // face node s <-> (beta_1, beta_2) in the order above; fswap[s] = index of (beta_2, beta_1)
  R.fswap.assign(nf, 0);
  if (d == 2) {
    for (int s = 0; s < nf; ++s) R.fswap[s] = s;
  } else {
    std::vector<int> idx((p + 1) * (p + 1), -1);
    int s = 0;
    for (int b2 = 0; b2 <= p; ++b2)
      for (int b1 = 0; b1 <= p - b2; ++b1) idx[b1 * (p + 1) + b2] = s++;
    for (int b2 = 0; b2 <= p; ++b2)
      for (int b1 = 0; b1 <= p - b2; ++b1) R.fswap[idx[b1 * (p + 1) + b2]] = idx[b2 * (p + 1) + b1];
  }

  Lagrange B(d, p, R.mi);
  // volume integrals
  std::vector<double> qp, qw;
  simplex_rule(d, p + 3, qp, qw);
  const int nq = (int)qw.size();
  std::vector<double> M(np * np, 0.0), D(d * np * np, 0.0);  // D[l][b][a]
  std::vector<double> phi(np), grad(np * d);
  for (int q = 0; q < nq; ++q) {
    B.eval(&qp[q * d], phi.data(), grad.data());
    double lam0 = 1.0;
    for (int l = 0; l < d; ++l) lam0 -= qp[q * d + l];
    for (int b = 0; b < np; ++b)
      for (int a = 0; a < np; ++a) {
        M[b * np + a] += qw[q] * phi[b] * phi[a];
        for (int l = 0; l < d; ++l) D[(l * np + b) * np + a] += qw[q] * lam0 * phi[a] * grad[b * d + l];
      }
  }
  R.Mhat = M;
  // S_l = M^{-1} D_l, stored [l][a][b]
  R.S.assign(d * np * np, 0.0);
  for (int l = 0; l < d; ++l) {
    std::vector<double> rhs(&D[l * np * np], &D[(l + 1) * np * np]);  // [b][a]
    spd_solve(np, M, rhs, np);
    for (int b = 0; b < np; ++b)
      for (int a = 0; a < np; ++a) R.S[(l * np + a) * np + b] = rhs[b * np + a];
  }
  // face integrals
  std::vector<double> fp, fw;
  simplex_rule(d - 1, p + 3, fp, fw);
  const int nfq = (int)fw.size();
  R.L.assign(d * nf * np, 0.0);
  for (int j = 1; j <= d; ++j) {
    std::vector<double> E(np * nf, 0.0);  // [b][s]
    for (int q = 0; q < nfq; ++q) {
      double xh[3] = {0, 0, 0};
      int c = 0;
      for (int l = 1; l <= d; ++l)
        if (l != j) xh[l - 1] = fp[q * (d - 1) + c++];
      B.eval(xh, phi.data(), nullptr);
      double lam0 = 1.0;
      for (int l = 0; l < d; ++l) lam0 -= xh[l];
      for (int s = 0; s < nf; ++s) {
        double ls = phi[R.fnode[((j - 1) * 2 + 0) * nf + s]];
        for (int b = 0; b < np; ++b) E[b * nf + s] += fw[q] * lam0 * ls * phi[b];
      }
    }
    spd_solve(np, M, E, nf);
    for (int s = 0; s < nf; ++s)
      for (int b = 0; b < np; ++b) R.L[((j - 1) * nf + s) * np + b] = E[b * nf + s];
  }
  return R;
}

}  // namespace mtp
