// Reference-element operators (host, FP64). See refops.hpp.
//
// Node set: the warp-and-blend nodes cited in Sec. 2. Every face of an equilateral
// tetrahedron carries a two-dimensional warp that moves the equispaced lattice toward the
// Gauss-Lobatto-Legendre distribution along each edge; the face warps are blended into the
// volume and the result is mapped back to the reference coordinates (r, s, t).
// Basis: the orthonormal polynomials of the collapsed coordinates (a, b, c).
#include "refops.hpp"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace dgh {
namespace {

// Blending exponent alpha_opt(N) of the warp-and-blend construction (Warburton 2006).
constexpr double kAlphaOpt[15] = {0.0,    0.0,    0.0,     0.1002, 1.1332, 1.5608, 1.3413, 1.2577,
                                  1.1603, 1.10153, 0.6080, 0.4523, 0.8856, 0.8717, 0.9655};
constexpr double kTol = 1e-10;

// Classical Jacobi polynomial P_n^{(a,b)}(x) by the three-term recurrence in n.
double jacobi_classic(double x, double a, double b, int n) {
  if (n == 0) return 1.0;
  double p0 = 1.0, p1 = 0.5 * ((a + b + 2.0) * x + (a - b));
  for (int m = 2; m <= n; ++m) {
    double c = 2.0 * m + a + b;
    double num = (c - 1.0) * (c * (c - 2.0) * x + a * a - b * b) * p1 -
                 2.0 * (m + a - 1.0) * (m + b - 1.0) * c * p0;
    double p2 = num / (2.0 * m * (m + a + b) * (c - 2.0));
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

// Squared weighted L2 norm of P_n^{(a,b)} on [-1, 1].
double jacobi_norm2(double a, double b, int n) {
  double lg = std::lgamma(n + a + 1.0) + std::lgamma(n + b + 1.0) - std::lgamma(n + a + b + 1.0) -
              std::lgamma(n + 1.0);
  return std::pow(2.0, a + b + 1.0) / (2.0 * n + a + b + 1.0) * std::exp(lg);
}

double jac(double x, double a, double b, int n) {
  return jacobi_classic(x, a, b, n) / std::sqrt(jacobi_norm2(a, b, n));
}

// Derivative of the normalised polynomial: d/dx P_n = (n+a+b+1)/2 P_{n-1}^{(a+1,b+1)}.
double djac(double x, double a, double b, int n) {
  if (n == 0) return 0.0;
  return 0.5 * (n + a + b + 1.0) * jacobi_classic(x, a + 1.0, b + 1.0, n - 1) /
         std::sqrt(jacobi_norm2(a, b, n));
}

// Gauss-Lobatto-Legendre points: the end points and the zeros of P_N', found by Newton's
// method from the Chebyshev-Lobatto points.
std::vector<double> gll(int N) {
  std::vector<double> x(N + 1);
  for (int k = 0; k <= N; ++k) x[k] = -std::cos(M_PI * k / N);
  for (int k = 1; k < N; ++k) {
    double z = x[k];
    for (int it = 0; it < 100; ++it) {
      double pm = 1.0, p = z;  // Legendre P_0, P_1
      for (int m = 2; m <= N; ++m) {
        double pn = ((2.0 * m - 1.0) * z * p - (m - 1.0) * pm) / m;
        pm = p;
        p = pn;
      }
      double dp = N * (z * p - pm) / (z * z - 1.0);              // P_N'
      double d2p = (2.0 * z * dp - N * (N + 1.0) * p) / (1.0 - z * z);  // P_N''
      double dz = dp / d2p;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[k] = z;
  }
  x[0] = -1.0;
  x[N] = 1.0;
  return x;
}

// Edge warp divided by the edge bubble (1 - x^2), evaluated without a division by the
// bubble: sum over interior points i of (x_i^GLL - x_i^eq) times the interior-only Lagrange
// factor product, divided by (1 - (x_i^eq)^2).
struct Warp1D {
  int N;
  std::vector<double> xeq, shift;
  explicit Warp1D(int n) : N(n), xeq(n + 1), shift(n + 1) {
    std::vector<double> g = gll(n);
    for (int i = 0; i <= n; ++i) {
      xeq[i] = -1.0 + 2.0 * i / n;
      shift[i] = g[i] - xeq[i];
    }
  }
  double operator()(double x) const {
    double w = 0.0;
    for (int i = 1; i < N; ++i) {
      double li = 1.0;
      for (int j = 1; j < N; ++j)
        if (j != i) li *= (x - xeq[j]) / (xeq[i] - xeq[j]);
      w += shift[i] * li / (1.0 - xeq[i] * xeq[i]);
    }
    return w;
  }
};

// LU factorisation with partial pivoting, in place; returns false if singular.
bool lu(std::vector<double>& a, std::vector<int>& piv, int n) {
  piv.resize(n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::fabs(a[k * n + k]);
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(a[i * n + k]) > best) best = std::fabs(a[i * n + k]), p = i;
    if (best == 0.0) return false;
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(a[k * n + j], a[p * n + j]);
    for (int i = k + 1; i < n; ++i) {
      double f = a[i * n + k] / a[k * n + k];
      a[i * n + k] = f;
      for (int j = k + 1; j < n; ++j) a[i * n + j] -= f * a[k * n + j];
    }
  }
  return true;
}

std::vector<double> matmul(const std::vector<double>& a, const std::vector<double>& b, int n, int k,
                           int m) {
  std::vector<double> c(size_t(n) * m, 0.0);
  for (int i = 0; i < n; ++i)
    for (int l = 0; l < k; ++l) {
      double av = a[size_t(i) * k + l];
      if (av == 0.0) continue;
      for (int j = 0; j < m; ++j) c[size_t(i) * m + j] += av * b[size_t(l) * m + j];
    }
  return c;
}

std::vector<double> transpose(const std::vector<double>& a, int n, int m) {
  std::vector<double> t(size_t(n) * m);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < m; ++j) t[size_t(j) * n + i] = a[size_t(i) * m + j];
  return t;
}

double ipow(double x, int p) {
  if (p < 0) return 0.0;  // only reached with a zero coefficient
  double r = 1.0;
  for (int i = 0; i < p; ++i) r *= x;
  return r;
}

// Collapsed coordinates of a point of the reference tetrahedron.
void collapse(double r, double s, double t, double& a, double& b, double& c) {
  a = (std::fabs(s + t) > 1e-12) ? 2.0 * (1.0 + r) / (-s - t) - 1.0 : -1.0;
  b = (std::fabs(t - 1.0) > 1e-12) ? 2.0 * (1.0 + s) / (1.0 - t) - 1.0 : -1.0;
  c = t;
}

// Orthonormal basis function (i,j,k) and its reference gradient at one point.
void basis_point(double r, double s, double t, int i, int j, int k, double* val, double* gr,
                 double* gs, double* gt) {
  double a, b, c;
  collapse(r, s, t, a, b, c);
  const double C = 2.0 * std::sqrt(2.0);
  const double bj = 2.0 * i + 1.0, ck = 2.0 * (i + j) + 2.0;
  double fa = jac(a, 0, 0, i), dfa = djac(a, 0, 0, i);
  double gb = jac(b, bj, 0, j), dgb = djac(b, bj, 0, j);
  double hc = jac(c, ck, 0, k), dhc = djac(c, ck, 0, k);
  double omb = 1.0 - b, omc = 1.0 - c;
  if (val) *val = C * fa * gb * ipow(omb, i) * hc * ipow(omc, i + j);
  if (!gr) return;
  // psi = C f(a) g(b) (1-b)^i h(c) (1-c)^(i+j); da/dr = 4/((1-b)(1-c)),
  // da/ds = da/dt = 2(1+a)/((1-b)(1-c)), db/ds = 2/(1-c), db/dt = (1+b)/(1-c), dc/dt = 1.
  double A = dfa * gb * ipow(omb, i - 1) * hc * ipow(omc, i + j - 1);
  double B = fa * (dgb * ipow(omb, i) - i * gb * ipow(omb, i - 1)) * hc * ipow(omc, i + j - 1);
  double Cc = fa * gb * ipow(omb, i) * (dhc * ipow(omc, i + j) - (i + j) * hc * ipow(omc, i + j - 1));
  *gr = C * 4.0 * A;
  *gs = C * (2.0 * (1.0 + a) * A + 2.0 * B);
  *gt = C * (2.0 * (1.0 + a) * A + (1.0 + b) * B + Cc);
}

double basis2d_point(double r, double s, int i, int j) {
  double a = (std::fabs(1.0 - s) > 1e-12) ? 2.0 * (1.0 + r) / (1.0 - s) - 1.0 : -1.0;
  return std::sqrt(2.0) * jac(a, 0, 0, i) * jac(s, 2.0 * i + 1.0, 0, j) * ipow(1.0 - s, i);
}

// Warp-and-blend nodes via per-face orthonormal tangent frames.
void build_nodes(int N, RefOps& R) {
  const double alpha = (N <= 15) ? kAlphaOpt[N - 1] : 1.0;
  const double s3 = std::sqrt(3.0), s6 = std::sqrt(6.0);
  const double V[4][3] = {{-1.0, -1.0 / s3, -1.0 / s6},
                          {1.0, -1.0 / s3, -1.0 / s6},
                          {0.0, 2.0 / s3, -1.0 / s6},
                          {0.0, 0.0, 3.0 / s6}};
  Warp1D warp(N);
  // Tangent frame of each face with vertices (p0, p1, p2): t1 along p0->p1, t2 from the
  // midpoint of p0p1 toward p2. In this frame the face is the equilateral triangle with
  // p0 = (-1, -1/sqrt3), p1 = (1, -1/sqrt3), p2 = (0, 2/sqrt3).
  double t1[4][3], t2[4][3];
  for (int f = 0; f < 4; ++f) {
    const double* p0 = V[kFaceVerts[f][0]];
    const double* p1 = V[kFaceVerts[f][1]];
    const double* p2 = V[kFaceVerts[f][2]];
    double n1 = 0, n2 = 0;
    for (int d = 0; d < 3; ++d) {
      t1[f][d] = p1[d] - p0[d];
      t2[f][d] = p2[d] - 0.5 * (p0[d] + p1[d]);
      n1 += t1[f][d] * t1[f][d];
      n2 += t2[f][d] * t2[f][d];
    }
    for (int d = 0; d < 3; ++d) t1[f][d] /= std::sqrt(n1), t2[f][d] /= std::sqrt(n2);
  }
  const double c120 = std::cos(2.0 * M_PI / 3.0), s120 = std::sin(2.0 * M_PI / 3.0);
  const double c240 = std::cos(4.0 * M_PI / 3.0), s240 = std::sin(4.0 * M_PI / 3.0);

  R.r.clear(), R.s.clear(), R.t.clear(), R.bary.clear();
  for (int k = 0; k <= N; ++k)
    for (int j = 0; j <= N - k; ++j)
      for (int i = 0; i <= N - k - j; ++i) {
        R.bary.push_back({N - i - j - k, i, j, k});
        double L[4] = {double(N - i - j - k) / N, double(i) / N, double(j) / N, double(k) / N};
        double X[3], sh[3] = {0, 0, 0};
        for (int d = 0; d < 3; ++d) X[d] = L[0] * V[0][d] + L[1] * V[1][d] + L[2] * V[2][d] + L[3] * V[3][d];
        for (int f = 0; f < 4; ++f) {
          double La = L[kFaceOpposite[f]];
          double l0 = L[kFaceVerts[f][0]], l1 = L[kFaceVerts[f][1]], l2 = L[kFaceVerts[f][2]];
          // 2D warp in the face frame: edge p0-p1 along 0 deg, p1-p2 along 120, p2-p0 along 240.
          double w01 = 4.0 * l0 * l1 * warp(l1 - l0) * (1.0 + (alpha * l2) * (alpha * l2));
          double w12 = 4.0 * l1 * l2 * warp(l2 - l1) * (1.0 + (alpha * l0) * (alpha * l0));
          double w20 = 4.0 * l2 * l0 * warp(l0 - l2) * (1.0 + (alpha * l1) * (alpha * l1));
          double dx = w01 + c120 * w12 + c240 * w20;
          double dy = s120 * w12 + s240 * w20;
          double tri[3];
          for (int d = 0; d < 3; ++d) tri[d] = dx * t1[f][d] + dy * t2[f][d];
          double denom = (l0 + 0.5 * La) * (l1 + 0.5 * La) * (l2 + 0.5 * La);
          double blend = denom > kTol ? (1.0 + (alpha * La) * (alpha * La)) * l0 * l1 * l2 / denom : 0.0;
          for (int d = 0; d < 3; ++d) sh[d] += blend * tri[d];
          int npos = (l0 > kTol) + (l1 > kTol) + (l2 > kTol);
          if (La < kTol && npos < 3)
            for (int d = 0; d < 3; ++d) sh[d] = tri[d];
        }
        for (int d = 0; d < 3; ++d) X[d] += sh[d];
        // back to reference coordinates: solve X = V0 + sum_{m=1..3} L_m (V_m - V0)
        double A[9], rhs[3];
        for (int d = 0; d < 3; ++d) {
          for (int m = 0; m < 3; ++m) A[d * 3 + m] = V[m + 1][d] - V[0][d];
          rhs[d] = X[d] - V[0][d];
        }
        std::vector<double> Am(A, A + 9);
        std::vector<int> piv;
        if (!lu(Am, piv, 3)) throw std::runtime_error("node map singular");
        for (int q = 0; q < 3; ++q) std::swap(rhs[q], rhs[piv[q]]);
        for (int q = 0; q < 3; ++q)
          for (int p = 0; p < q; ++p) rhs[q] -= Am[q * 3 + p] * rhs[p];
        for (int q = 2; q >= 0; --q) {
          for (int p = q + 1; p < 3; ++p) rhs[q] -= Am[q * 3 + p] * rhs[p];
          rhs[q] /= Am[q * 3 + q];
        }
        R.r.push_back(-1.0 + 2.0 * rhs[0]);
        R.s.push_back(-1.0 + 2.0 * rhs[1]);
        R.t.push_back(-1.0 + 2.0 * rhs[2]);
      }
}

}  // namespace

bool invert(std::vector<double>& a, int n) {
  std::vector<int> piv;
  std::vector<double> lu_a = a;
  if (!lu(lu_a, piv, n)) return false;
  std::vector<double> inv(size_t(n) * n, 0.0);
  for (int col = 0; col < n; ++col) {
    std::vector<double> x(n, 0.0);
    x[col] = 1.0;
    for (int q = 0; q < n; ++q) std::swap(x[q], x[piv[q]]);
    for (int q = 0; q < n; ++q)
      for (int p = 0; p < q; ++p) x[q] -= lu_a[q * n + p] * x[p];
    for (int q = n - 1; q >= 0; --q) {
      for (int p = q + 1; p < n; ++p) x[q] -= lu_a[q * n + p] * x[p];
      x[q] /= lu_a[q * n + q];
    }
    for (int q = 0; q < n; ++q) inv[size_t(q) * n + col] = x[q];
  }
  a.swap(inv);
  return true;
}

RefOps build_ref_ops(int N) {
  if (N < 1 || N > 10) throw std::runtime_error("unsupported order");
  RefOps R;
  R.N = N;
  R.Np = (N + 1) * (N + 2) * (N + 3) / 6;
  R.Nfp = (N + 1) * (N + 2) / 2;
  const int Np = R.Np, Nfp = R.Nfp;
  build_nodes(N, R);

  // Vandermonde matrix and its reference derivatives.
  std::vector<std::array<int, 3>> modes;
  for (int i = 0; i <= N; ++i)
    for (int j = 0; j <= N - i; ++j)
      for (int k = 0; k <= N - i - j; ++k) modes.push_back({i, j, k});
  std::vector<double> V(size_t(Np) * Np), Vr(V.size()), Vs(V.size()), Vt(V.size());
  for (int p = 0; p < Np; ++p)
    for (int m = 0; m < Np; ++m) {
      size_t q = size_t(p) * Np + m;
      basis_point(R.r[p], R.s[p], R.t[p], modes[m][0], modes[m][1], modes[m][2], &V[q], &Vr[q],
                  &Vs[q], &Vt[q]);
    }
  std::vector<double> Vinv = V;
  if (!invert(Vinv, Np)) throw std::runtime_error("Vandermonde singular");
  R.Dr = matmul(Vr, Vinv, Np, Np, Np);
  R.Ds = matmul(Vs, Vinv, Np, Np, Np);
  R.Dt = matmul(Vt, Vinv, Np, Np, Np);
  std::vector<double> VVt = matmul(V, transpose(V, Np, Np), Np, Np, Np);
  R.M = VVt;
  if (!invert(R.M, Np)) throw std::runtime_error("mass singular");

  // Face node lists from the integer lattice.
  R.Fmask.assign(4 * Nfp, -1);
  for (int f = 0; f < 4; ++f) {
    int cnt = 0;
    for (int p = 0; p < Np; ++p)
      if (R.bary[p][kFaceOpposite[f]] == 0) {
        if (cnt >= Nfp) throw std::runtime_error("face node count");
        R.Fmask[f * Nfp + cnt++] = p;
      }
    if (cnt != Nfp) throw std::runtime_error("face node count");
  }

  // Face mass matrices in in-face coordinates (r,s) / (r,t) / (s,t) / (s,t), embedded.
  std::vector<double> E(size_t(Np) * 4 * Nfp, 0.0);
  for (int f = 0; f < 4; ++f) {
    std::vector<double> V2(size_t(Nfp) * Nfp);
    for (int q = 0; q < Nfp; ++q) {
      int p = R.Fmask[f * Nfp + q];
      double c1 = (f == 0 || f == 1) ? R.r[p] : R.s[p];
      double c2 = (f == 0) ? R.s[p] : R.t[p];
      int m = 0;
      for (int i = 0; i <= N; ++i)
        for (int j = 0; j <= N - i; ++j) V2[size_t(q) * Nfp + m++] = basis2d_point(c1, c2, i, j);
    }
    std::vector<double> Mf = matmul(V2, transpose(V2, Nfp, Nfp), Nfp, Nfp, Nfp);
    if (!invert(Mf, Nfp)) throw std::runtime_error("face mass singular");
    for (int a = 0; a < Nfp; ++a)
      for (int b = 0; b < Nfp; ++b)
        E[size_t(R.Fmask[f * Nfp + a]) * 4 * Nfp + f * Nfp + b] = Mf[size_t(a) * Nfp + b];
  }
  // LIFT = M^-1 E = V V^T E
  R.LIFT = matmul(V, matmul(transpose(V, Np, Np), E, Np, Np, 4 * Nfp), Np, Np, 4 * Nfp);

  // Neighbour node table: a face node is identified by its integer barycentrics on the three
  // face vertices; the neighbour sees the same vertices in another order.
  R.nbr_node.assign(size_t(4) * 4 * 6 * Nfp, -1);
  for (int f = 0; f < 4; ++f)
    for (int f2 = 0; f2 < 4; ++f2)
      for (int o = 0; o < 6; ++o)
        for (int j = 0; j < Nfp; ++j) {
          const auto& mine = R.bary[R.Fmask[f * Nfp + j]];
          int want[3];
          for (int a = 0; a < 3; ++a) want[kPerm3[o][a]] = mine[kFaceVerts[f][a]];
          int found = -1;
          for (int j2 = 0; j2 < Nfp; ++j2) {
            const auto& th = R.bary[R.Fmask[f2 * Nfp + j2]];
            if (th[kFaceVerts[f2][0]] == want[0] && th[kFaceVerts[f2][1]] == want[1] &&
                th[kFaceVerts[f2][2]] == want[2])
              found = R.Fmask[f2 * Nfp + j2];
          }
          if (found < 0) throw std::runtime_error("face node table");
          R.nbr_node[((size_t(f) * 4 + f2) * 6 + o) * Nfp + j] = found;
        }
  return R;
}

}  // namespace dgh
