// Host-side FP64 construction of the reference 1-D tables of the SIPG
// multigrid (Sec. 2.2, Sec. 3.2, Appendix A): the basis data of Q_k (the
// compile-time tables of dgmg_ref1d.h: Gauss-Lobatto nodes, mass, stiffness,
// end derivatives, prolongation), the 1-D SIPG cell block with the penalty,
// and the fast-diagonalisation eigenpairs L S = M S Lambda of
// the two-cell patch restricted to the Dirichlet local space, on the whole
// patch (Full kernel) and on the clamped space, for each of the four 1-D
// patch types.  Everything is computed at h = 1, kappa = 1; the
// kernels scale by kappa h^(d-2).
#include "dgmg_setup.h"

#include "dgmg_ref1d.h"

#include <cmath>
#include <limits>

namespace dgmg {
namespace {

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

template <int K>
void copy_ref(HostTables& T) {
  constexpr ref1d::Ref<K> R = ref1d::make_ref<K>();
  constexpr int n = K + 1;
  T.nodes.assign(R.nodes, R.nodes + n);
  T.M.assign(R.M, R.M + n * n);
  T.K.assign(R.Ks, R.Ks + n * n);
  T.d0.assign(R.d0, R.d0 + n);
  T.d1.assign(R.d1, R.d1 + n);
  T.Lc.assign(R.Lcons, R.Lcons + n * n);
  T.P.assign(R.P, R.P + 2 * n * n);
}

std::vector<double> gll_nodes01(int k) {
  HostTables T;
  switch (k) {
    case 1: copy_ref<1>(T); break;
    case 2: copy_ref<2>(T); break;
    case 3: copy_ref<3>(T); break;
    case 4: copy_ref<4>(T); break;
    case 5: copy_ref<5>(T); break;
    case 6: copy_ref<6>(T); break;
    default: copy_ref<7>(T); break;
  }
  return T.nodes;
}

bool build_host_tables(int k, double sigma, HostTables& T, const char** err) {
  const int n = k + 1, E = 2 * n;
  T.k = k;
  T.n = n;
  T.E = E;
  T.sigma = sigma;
  switch (k) {  // basis data of Q_k (compile-time tables shared with the kernels)
    case 1: copy_ref<1>(T); break;
    case 2: copy_ref<2>(T); break;
    case 3: copy_ref<3>(T); break;
    case 4: copy_ref<4>(T); break;
    case 5: copy_ref<5>(T); break;
    case 6: copy_ref<6>(T); break;
    case 7: copy_ref<7>(T); break;
    default: *err = "degree out of range"; return false;
  }
  // 1-D SIPG cell block with interior faces at both ends (h = 1): the
  // consistency part plus the penalty sigma (e0 e0^T + e1 e1^T)
  T.Lc[0] += sigma;
  T.Lc[k * n + k] += sigma;
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
    if (t == 0) {
      // interior patch: the Dirichlet space (nodes 1 .. E-2) and both 1-D
      // matrices are symmetric under the reflection p -> E-1-p, so the
      // eigenvectors split into even and odd ones.  They are computed on the
      // even and the odd subspace separately, which makes the symmetry exact:
      // columns q < h even, h <= q < 2h odd (h = n - 1), as the kernels'
      // even-odd contractions assume.
      const int h = n - 1;
      std::vector<double> Cp(E * h, 0.0), Cm(E * h, 0.0), Sp, lp, Sm, lm;
      for (int j = 0; j < h; ++j) {
        Cp[(1 + j) * h + j] = 1.0;
        Cp[(E - 2 - j) * h + j] = 1.0;
        Cm[(1 + j) * h + j] = 1.0;
        Cm[(E - 2 - j) * h + j] = -1.0;
      }
      if (!basis_eigenpairs(L, Mp, E, Cp, h, Sp, lp, err)) return false;
      if (!basis_eigenpairs(L, Mp, E, Cm, h, Sm, lm, err)) return false;
      T.S[t].assign(E * E, 0.0);
      T.lam[t].assign(E, std::numeric_limits<double>::infinity());
      for (int q = 0; q < h; ++q) {
        T.lam[t][q] = lp[q];
        T.lam[t][h + q] = lm[q];
        for (int p = 0; p < E; ++p) {
          T.S[t][p * E + q] = Sp[p * E + q];
          T.S[t][p * E + h + q] = Sm[p * E + q];
        }
      }
    } else {
      std::vector<int> keep;
      for (int p = 0; p < E; ++p) {
        const bool drop = (p == 0 && !(t & 1)) || (p == E - 1 && !(t & 2));
        if (!drop) keep.push_back(p);
      }
      if (!patch_eigenpairs(L, Mp, E, keep, T.S[t], T.lam[t], err)) return false;
    }
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
