// Reference 1-D data of Q_K on [0,1] (Appendix A: Lagrange basis on the K+1
// Gauss-Lobatto points), evaluated at compile time.  The kernels use these as
// instruction immediates (no table loads on the critical path of a patch);
// the host setup uses the same values for the tables that depend on the
// penalty (cell block, patch eigenpairs).
//   nodes : Gauss-Lobatto points in [0,1]
//   M     : int phi_i phi_j                         (exact, K+1 Gauss points)
//   Ks    : int phi_i' phi_j'
//   d0,d1 : phi_i'(0), phi_i'(1)
//   Lcons : Ks + (e0 d0^T + d0 e0^T)/2 - (e1 d1^T + d1 e1^T)/2, the cell block
//           of the 1-D SIPG operator with interior faces on both sides minus
//           its penalty part sigma (e0 e0^T + e1 e1^T)
//   P     : P[(o n + mu) n + nu] = phi_nu((xi_mu + o)/2), embedding of a
//           coarse cell into its child o
#pragma once

namespace dgmg {
namespace ref1d {

constexpr double kPi = 3.14159265358979323846;

constexpr double cabs(double x) { return x < 0 ? -x : x; }

// cos on [0, pi] by symmetry and a Taylor series on [0, pi/2] (initial guesses
// of Newton iterations only)
constexpr double ccos(double x) {
  double sign = 1.0;
  if (x > kPi / 2) {
    x = kPi - x;
    sign = -1.0;
  }
  double term = 1.0, sum = 1.0;
  for (int i = 1; i < 30; ++i) {
    term *= -x * x / ((2.0 * i - 1.0) * (2.0 * i));
    sum += term;
  }
  return sign * sum;
}

// Legendre P_m(x) and P_m'(x) on [-1,1] by the three-term recurrence
struct PD {
  double p, dp;
};
constexpr PD legendre(int m, double x) {
  if (m == 0) return {1.0, 0.0};
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  for (int j = 2; j <= m; ++j) {
    const double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
    const double d2 = d0 + (2.0 * j - 1.0) * p1;  // P_j' = P_{j-2}' + (2j-1) P_{j-1}
    p0 = p1;
    p1 = p2;
    d0 = d1;
    d1 = d2;
  }
  return {p1, d1};
}

template <int K>
struct Ref {
  static constexpr int n = K + 1;
  double nodes[n];
  double M[n * n];
  double Ks[n * n];
  double d0[n];
  double d1[n];
  double Lcons[n * n];
  double P[2 * n * n];
};

// Lagrange basis on the nodes: value (deriv = false) or derivative of phi_j at y
template <int n>
constexpr double lagrange(const double (&nd)[n], int j, double y, bool deriv) {
  double den = 1.0;
  for (int m = 0; m < n; ++m)
    if (m != j) den *= nd[j] - nd[m];
  if (!deriv) {
    double num = 1.0;
    for (int m = 0; m < n; ++m)
      if (m != j) num *= y - nd[m];
    return num / den;
  }
  double ds = 0.0;
  for (int l = 0; l < n; ++l) {
    if (l == j) continue;
    double pr = 1.0;
    for (int m = 0; m < n; ++m)
      if (m != j && m != l) pr *= y - nd[m];
    ds += pr;
  }
  return ds / den;
}

template <int K>
constexpr Ref<K> make_ref() {
  constexpr int n = K + 1;
  Ref<K> r{};
  // Gauss-Lobatto points: the ends and the roots of P_K', Newton on P_K' with
  // P_K'' from the Legendre equation (1 - t^2) P'' = 2 t P' - K(K+1) P
  r.nodes[0] = 0.0;
  r.nodes[K] = 1.0;
  for (int j = 1; j < K; ++j) {
    double t = -ccos(kPi * j / K);
    for (int it = 0; it < 100; ++it) {
      const PD v = legendre(K, t);
      const double d2p = (2.0 * t * v.dp - K * (K + 1.0) * v.p) / (1.0 - t * t);
      const double dt = v.dp / d2p;
      t -= dt;
      if (cabs(dt) < 1e-16) break;
    }
    r.nodes[j] = 0.5 * (t + 1.0);
  }
  // n-point Gauss rule on [0,1] (exact for degree 2K+1)
  double xq[n] = {}, wq[n] = {};
  for (int j = 0; j < n; ++j) {
    double t = -ccos(kPi * (j + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      const PD v = legendre(n, t);
      const double dt = v.p / v.dp;
      t -= dt;
      if (cabs(dt) < 1e-16) break;
    }
    const PD v = legendre(n, t);
    xq[j] = 0.5 * (t + 1.0);
    wq[j] = 1.0 / ((1.0 - t * t) * v.dp * v.dp);
  }
  for (int i = 0; i < n * n; ++i) r.M[i] = r.Ks[i] = 0.0;
  for (int q = 0; q < n; ++q)
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        r.M[i * n + j] += wq[q] * lagrange(r.nodes, i, xq[q], false) * lagrange(r.nodes, j, xq[q], false);
        r.Ks[i * n + j] += wq[q] * lagrange(r.nodes, i, xq[q], true) * lagrange(r.nodes, j, xq[q], true);
      }
  for (int j = 0; j < n; ++j) {
    r.d0[j] = lagrange(r.nodes, j, 0.0, true);
    r.d1[j] = lagrange(r.nodes, j, 1.0, true);
  }
  for (int i = 0; i < n * n; ++i) r.Lcons[i] = r.Ks[i];
  for (int j = 0; j < n; ++j) {
    r.Lcons[0 * n + j] += 0.5 * r.d0[j];
    r.Lcons[j * n + 0] += 0.5 * r.d0[j];
    r.Lcons[K * n + j] -= 0.5 * r.d1[j];
    r.Lcons[j * n + K] -= 0.5 * r.d1[j];
  }
  for (int o = 0; o < 2; ++o)
    for (int mu = 0; mu < n; ++mu)
      for (int nu = 0; nu < n; ++nu)
        r.P[(o * n + mu) * n + nu] = lagrange(r.nodes, nu, 0.5 * (r.nodes[mu] + o), false);
  return r;
}

}  // namespace ref1d
}  // namespace dgmg
