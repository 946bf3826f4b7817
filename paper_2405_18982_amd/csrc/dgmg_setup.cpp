// Host-side FP64 construction of the reference 1-D tables of the SIPG
// multigrid (Sec. 2.2, Sec. 3.2, Appendix A): Gauss-Lobatto nodes, Lagrange
// basis, cell mass/stiffness, the 1-D SIPG cell block, the embedding
// prolongation, and the fast-diagonalisation eigenpairs L S = M S Lambda of
// the two-cell patch restricted to the Dirichlet local space, on the whole
// patch (Full kernel) and on the clamped space, for each of the four 1-D
// patch types.  Everything is computed at h = 1, kappa = 1; the
// kernels scale by kappa h^(d-2).
#include "dgmg_setup.h"

#include <cmath>
#include <limits>

namespace dgmg {
namespace {

// Legendre P_m(x) and P_m'(x) by the three-term recurrence.
void legendre(int m, double x, double& p, double& dp) {
  double p0 = 1.0, p1 = x;
  if (m == 0) { p = 1.0; dp = 0.0; return; }
  for (int j = 2; j <= m; ++j) {
    const double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  // derivative from (1 - x^2) P_m' = m (P_{m-1} - x P_m), valid for |x| < 1
  dp = m * (p0 - x * p1) / (1.0 - x * x);
}

// m-point Gauss-Legendre rule on [0,1]: Newton on P_m from Chebyshev guesses.
void gauss01(int m, std::vector<double>& x, std::vector<double>& w) {
  x.assign(m, 0.0);
  w.assign(m, 0.0);
  for (int j = 0; j < m; ++j) {
    double t = -std::cos(M_PI * (j + 0.75) / (m + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(m, t, p, dp);
      const double dt = p / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    double p, dp;
    legendre(m, t, p, dp);
    x[j] = 0.5 * (t + 1.0);
    w[j] = 1.0 / ((1.0 - t * t) * dp * dp);  // 2/((1-t^2)P'^2) scaled by 1/2
  }
}

// Lagrange basis values and derivatives at y: V[j] = phi_j(y), Dv[j] = phi_j'(y).
void lagrange(const std::vector<double>& nd, double y, std::vector<double>& V,
              std::vector<double>& Dv) {
  const int n = (int)nd.size();
  V.assign(n, 0.0);
  Dv.assign(n, 0.0);
  for (int j = 0; j < n; ++j) {
    double den = 1.0;
    for (int m = 0; m < n; ++m)
      if (m != j) den *= nd[j] - nd[m];
    double num = 1.0;
    for (int m = 0; m < n; ++m)
      if (m != j) num *= y - nd[m];
    V[j] = num / den;
    double ds = 0.0;
    for (int l = 0; l < n; ++l) {
      if (l == j) continue;
      double pr = 1.0;
      for (int m = 0; m < n; ++m)
        if (m != j && m != l) pr *= y - nd[m];
      ds += pr;
    }
    Dv[j] = ds / den;
  }
}

// Cholesky A = C C^T of an SPD matrix (row-major, size m); false if not SPD.
bool cholesky(const std::vector<double>& A, int m, std::vector<double>& C) {
  C.assign(m * m, 0.0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = A[i * m + j];
      for (int l = 0; l < j; ++l) s -= C[i * m + l] * C[j * m + l];
      if (i == j) {
        if (!(s > 0.0)) return false;
        C[i * m + i] = std::sqrt(s);
      } else {
        C[i * m + j] = s / C[j * m + j];
      }
    }
  return true;
}

// Cyclic Jacobi eigen-decomposition of a symmetric matrix: A = Q diag(w) Q^T.
void jacobi_eigen(std::vector<double> A, int m, std::vector<double>& w, std::vector<double>& Q) {
  Q.assign(m * m, 0.0);
  for (int i = 0; i < m; ++i) Q[i * m + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        tot += A[i * m + j] * A[i * m + j];
        if (i != j) off += A[i * m + j] * A[i * m + j];
      }
    if (off <= 1e-32 * tot) break;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) {
        const double apq = A[p * m + q];
        if (apq == 0.0) continue;
        const double theta = (A[q * m + q] - A[p * m + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < m; ++k) {  // A <- A J (columns p, q)
          const double akp = A[k * m + p], akq = A[k * m + q];
          A[k * m + p] = c * akp - s * akq;
          A[k * m + q] = s * akp + c * akq;
        }
        for (int k = 0; k < m; ++k) {  // A <- J^T A (rows p, q)
          const double apk = A[p * m + k], aqk = A[q * m + k];
          A[p * m + k] = c * apk - s * aqk;
          A[q * m + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < m; ++k) {  // Q <- Q J
          const double qkp = Q[k * m + p], qkq = Q[k * m + q];
          Q[k * m + p] = c * qkp - s * qkq;
          Q[k * m + q] = s * qkp + c * qkq;
        }
      }
  }
  w.resize(m);
  for (int i = 0; i < m; ++i) w[i] = A[i * m + i];
}

// Generalised eigenpairs of the E x E patch matrices L, M on the subspace
// spanned by the m columns of Cb (row-major E x m): L_C S = M_C S Lambda with
// L_C = Cb^T L Cb, M_C = Cb^T M Cb, returned as Cb S padded to E x E
// (Sout[p*E + q], zero columns q >= m) and lam (+inf in unused slots).
// Via M_C = C C^T: C^{-1} L_C C^{-T} = Q Lambda Q^T, S = C^{-T} Q (S^T M_C S = I).
bool basis_eigenpairs(const std::vector<double>& L, const std::vector<double>& Mp, int E,
                      const std::vector<double>& Cb, int m, std::vector<double>& Sout,
                      std::vector<double>& lamout, const char** err) {
  std::vector<double> Lt(m * m, 0.0), Mt(m * m, 0.0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      double sl = 0.0, sm = 0.0;
      for (int p = 0; p < E; ++p)
        for (int q = 0; q < E; ++q) {
          const double w = Cb[p * m + i] * Cb[q * m + j];
          if (w == 0.0) continue;
          sl += w * L[p * E + q];
          sm += w * Mp[p * E + q];
        }
      Lt[i * m + j] = sl;
      Mt[i * m + j] = sm;
    }
  std::vector<double> C;
  if (!cholesky(Mt, m, C)) { *err = "patch mass matrix is not positive definite"; return false; }
  std::vector<double> Y(m * m), Bm(m * m);
  for (int col = 0; col < m; ++col)  // Y = C^{-1} L (forward substitution per column)
    for (int i = 0; i < m; ++i) {
      double s = Lt[i * m + col];
      for (int l = 0; l < i; ++l) s -= C[i * m + l] * Y[l * m + col];
      Y[i * m + col] = s / C[i * m + i];
    }
  for (int row = 0; row < m; ++row)  // B = Y C^{-T}: solve C B^T = Y^T row by row
    for (int i = 0; i < m; ++i) {
      double s = Y[row * m + i];
      for (int l = 0; l < i; ++l) s -= C[i * m + l] * Bm[row * m + l];
      Bm[row * m + i] = s / C[i * m + i];
    }
  for (int i = 0; i < m; ++i)  // symmetrise round-off
    for (int j = 0; j < i; ++j) {
      const double a = 0.5 * (Bm[i * m + j] + Bm[j * m + i]);
      Bm[i * m + j] = Bm[j * m + i] = a;
    }
  std::vector<double> w, Q;
  jacobi_eigen(Bm, m, w, Q);
  for (int i = 0; i < m; ++i)
    if (!(w[i] > 0.0)) { *err = "patch SIPG matrix is not positive definite (penalty too small)"; return false; }
  std::vector<double> S(m * m);  // S = C^{-T} Q: back substitution with C^T per column of Q
  for (int col = 0; col < m; ++col)
    for (int i = m - 1; i >= 0; --i) {
      double s = Q[i * m + col];
      for (int l = i + 1; l < m; ++l) s -= C[l * m + i] * S[l * m + col];
      S[i * m + col] = s / C[i * m + i];
    }
  Sout.assign(E * E, 0.0);
  lamout.assign(E, std::numeric_limits<double>::infinity());
  for (int q = 0; q < m; ++q) {
    lamout[q] = w[q];
    for (int p = 0; p < E; ++p) {
      double s = 0.0;
      for (int i = 0; i < m; ++i) s += Cb[p * m + i] * S[i * m + q];
      Sout[p * E + q] = s;
    }
  }
  return true;
}

// The same on the coordinate subspace of the nodes in keep.
bool patch_eigenpairs(const std::vector<double>& L, const std::vector<double>& Mp, int E,
                      const std::vector<int>& keep, std::vector<double>& Sout,
                      std::vector<double>& lamout, const char** err) {
  const int m = (int)keep.size();
  std::vector<double> Cb(E * m, 0.0);
  for (int i = 0; i < m; ++i) Cb[keep[i] * m + i] = 1.0;
  return basis_eigenpairs(L, Mp, E, Cb, m, Sout, lamout, err);
}

// Basis (row-major E x m) of the clamped space of a 1-D patch type: value and
// derivative vanish at every end on an interior face.  With Gauss-Lobatto
// nodes the value at an end is the end node; the derivative condition fixes
// the neighbouring node: left end v_1 = -sum_{a>=2} d0_a v_a / d0_1, right end
// v_{k-1} = -sum_{a<=k-2} d1_a v_a / d1_{k-1} (right cell).  Needs k >= 2.
std::vector<double> clamped_basis(int k, int t, const std::vector<double>& d0,
                                  const std::vector<double>& d1, int& m) {
  const int n = k + 1, E = 2 * n;
  const bool cl = !(t & 1), cr = !(t & 2);
  std::vector<std::vector<double>> cols;
  for (int a = 0; a < n; ++a) {  // left cell
    if (cl && a < 2) continue;
    std::vector<double> c(E, 0.0);
    c[a] = 1.0;
    if (cl) c[1] = -d0[a] / d0[1];
    cols.push_back(c);
  }
  for (int a = 0; a < n; ++a) {  // right cell
    if (cr && a > k - 2) continue;
    std::vector<double> c(E, 0.0);
    c[n + a] = 1.0;
    if (cr) c[n + k - 1] = -d1[a] / d1[k - 1];
    cols.push_back(c);
  }
  m = (int)cols.size();
  std::vector<double> Cb(E * m);
  for (int p = 0; p < E; ++p)
    for (int i = 0; i < m; ++i) Cb[p * m + i] = cols[i][p];
  return Cb;
}

}  // namespace

std::vector<double> gll_nodes01(int k) {
  std::vector<double> x(k + 1);
  x[0] = 0.0;
  x[k] = 1.0;
  // interior points: roots of P_k', Newton on P_k' with P_k'' from the
  // Legendre equation (1-t^2) P'' = 2 t P' - k(k+1) P
  for (int j = 1; j < k; ++j) {
    double t = -std::cos(M_PI * j / k);
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(k, t, p, dp);
      const double d2p = (2.0 * t * dp - k * (k + 1.0) * p) / (1.0 - t * t);
      const double dt = dp / d2p;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    x[j] = 0.5 * (t + 1.0);
  }
  return x;
}

bool build_host_tables(int k, double sigma, HostTables& T, const char** err) {
  const int n = k + 1, E = 2 * n;
  T.k = k;
  T.n = n;
  T.E = E;
  T.sigma = sigma;
  T.nodes = gll_nodes01(k);
  std::vector<double> xq, wq, V, Dv;
  gauss01(n, xq, wq);  // exact for degree 2k+1
  T.M.assign(n * n, 0.0);
  T.K.assign(n * n, 0.0);
  for (int q = 0; q < n; ++q) {
    lagrange(T.nodes, xq[q], V, Dv);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        T.M[i * n + j] += wq[q] * V[i] * V[j];
        T.K[i * n + j] += wq[q] * Dv[i] * Dv[j];
      }
  }
  lagrange(T.nodes, 0.0, V, T.d0);
  lagrange(T.nodes, 1.0, V, T.d1);
  // 1-D SIPG cell block with interior faces at both ends (h = 1):
  // K + sigma(e0 e0^T + e1 e1^T) + (e0 d0^T + d0 e0^T)/2 - (e1 d1^T + d1 e1^T)/2
  T.Lc = T.K;
  T.Lc[0] += sigma;
  T.Lc[k * n + k] += sigma;
  for (int j = 0; j < n; ++j) {
    T.Lc[0 * n + j] += 0.5 * T.d0[j];
    T.Lc[j * n + 0] += 0.5 * T.d0[j];
    T.Lc[k * n + j] -= 0.5 * T.d1[j];
    T.Lc[j * n + k] -= 0.5 * T.d1[j];
  }
  // stacked prolongation P[(o n + mu) n + nu] = phi_nu((xi_mu + o)/2)
  T.P.assign(E * n, 0.0);
  for (int o = 0; o < 2; ++o)
    for (int mu = 0; mu < n; ++mu) {
      lagrange(T.nodes, 0.5 * (T.nodes[mu] + o), V, Dv);
      for (int nu = 0; nu < n; ++nu) T.P[(o * n + mu) * n + nu] = V[nu];
    }
  // two-cell patch 1-D matrices: cell blocks Lc, the coupling across the
  // middle face, and the Nitsche corrections of the boundary types
  std::vector<double> Lp(E * E, 0.0), Mp(E * E, 0.0);
  for (int c = 0; c < 2; ++c)
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        Lp[(c * n + i) * E + c * n + j] = T.Lc[i * n + j];
        Mp[(c * n + i) * E + c * n + j] = T.M[i * n + j];
      }
  // rows of the left cell, columns of the right cell:
  // -sigma e1 e0^T - e1 d0^T / 2 + d1 e0^T / 2 (and its transpose)
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double v = 0.0;
      if (i == k && j == 0) v -= sigma;
      if (i == k) v -= 0.5 * T.d0[j];
      if (j == 0) v += 0.5 * T.d1[i];
      Lp[i * E + n + j] = v;
      Lp[(n + j) * E + i] = v;
    }
  for (int t = 0; t < 4; ++t) {
    std::vector<double> L = Lp;
    if (t & 1)  // left cell on x = 0: Nitsche adds (e0 d0^T + d0 e0^T)/2
      for (int j = 0; j < n; ++j) {
        L[0 * E + j] += 0.5 * T.d0[j];
        L[j * E + 0] += 0.5 * T.d0[j];
      }
    if (t & 2)  // right cell on x = 1: Nitsche adds -(e1 d1^T + d1 e1^T)/2
      for (int j = 0; j < n; ++j) {
        L[(E - 1) * E + n + j] -= 0.5 * T.d1[j];
        L[(n + j) * E + E - 1] -= 0.5 * T.d1[j];
      }
    std::vector<int> keep;
    for (int p = 0; p < E; ++p) {
      const bool drop = (p == 0 && !(t & 1)) || (p == E - 1 && !(t & 2));
      if (!drop) keep.push_back(p);
    }
    if (!patch_eigenpairs(L, Mp, E, keep, T.S[t], T.lam[t], err)) return false;
    // Full kernel: every node of the two cells
    std::vector<int> all(E);
    for (int p = 0; p < E; ++p) all[p] = p;
    if (!patch_eigenpairs(L, Mp, E, all, T.Sf[t], T.lamf[t], err)) return false;
    // clamped kernel (k >= 2; the library uses it for k >= 3)
    if (k >= 2) {
      int m = 0;
      const std::vector<double> Cb = clamped_basis(k, t, T.d0, T.d1, m);
      if (!basis_eigenpairs(L, Mp, E, Cb, m, T.Sc[t], T.lamc[t], err)) return false;
    } else {
      T.Sc[t].assign(E * E, 0.0);
      T.lamc[t].assign(E, std::numeric_limits<double>::infinity());
    }
  }
  return true;
}

}  // namespace dgmg
