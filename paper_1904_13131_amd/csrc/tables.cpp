// Host construction of the 1-D tables (Sec. 5 tensor-product bases) and of
// the 1-D transfer matrices between nested levels (Sec. 6).
#include "tables.hpp"

#include <cmath>
#include <stdexcept>

namespace mfh {

namespace {

// Legendre polynomial P_n and its derivative on [-1, 1] by the three-term
// recurrence (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}.
void legendre(int n, double x, double& P, double& dP) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    P = 1.0;
    dP = 0.0;
    return;
  }
  for (int k = 1; k < n; ++k) {
    const double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
    p0 = p1;
    p1 = p2;
  }
  P = p1;
  // P_n' from (x^2 - 1) P_n' = n (x P_n - P_{n-1})
  dP = n * (x * p1 - p0) / (x * x - 1.0);
}

}  // namespace

std::vector<double> gauss_points(int q, std::vector<double>& w) {
  std::vector<double> x(q);
  w.assign(q, 0.0);
  for (int i = 0; i < q; ++i) {
    double t = std::cos(M_PI * (i + 0.75) / (q + 0.5));
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(q, t, P, dP);
      const double dt = P / dP;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    double P, dP;
    legendre(q, t, P, dP);
    x[q - 1 - i] = 0.5 * (t + 1.0);
    w[q - 1 - i] = 0.5 * 2.0 / ((1.0 - t * t) * dP * dP);
  }
  return x;
}

std::vector<double> gll_points(int p) {
  std::vector<double> x(p + 1);
  x[0] = 0.0;
  x[p] = 1.0;
  // interior points: roots of P_p', Newton with P_p'' from Legendre's equation
  for (int j = 1; j < p; ++j) {
    double t = -std::cos(M_PI * j / p);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(p, t, P, dP);
      const double d2P = (2.0 * t * dP - p * (p + 1) * P) / (1.0 - t * t);
      const double dt = dP / d2P;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    x[j] = 0.5 * (t + 1.0);
  }
  return x;
}

void lagrange(const std::vector<double>& nodes, double x, double* V, double* D) {
  const int n = (int)nodes.size();
  for (int a = 0; a < n; ++a) {
    double v = 1.0;
    for (int b = 0; b < n; ++b)
      if (b != a) v *= (x - nodes[b]) / (nodes[a] - nodes[b]);
    V[a] = v;
    if (D) {
      double d = 0.0;
      for (int m = 0; m < n; ++m) {
        if (m == a) continue;
        double term = 1.0 / (nodes[a] - nodes[m]);
        for (int b = 0; b < n; ++b)
          if (b != a && b != m) term *= (x - nodes[b]) / (nodes[a] - nodes[b]);
        d += term;
      }
      D[a] = d;
    }
  }
}

Tables<double> make_tables(int p) {
  if (p < 1 || p > kMaxDeg) throw std::invalid_argument("degree out of range");
  Tables<double> t = {};
  std::vector<double> w;
  const std::vector<double> xg = gauss_points(p + 1, w);
  const std::vector<double> xi = gll_points(p);
  for (int q = 0; q <= p; ++q) {
    lagrange(xi, xg[q], t.S[q], t.D[q]);
    t.w[q] = w[q];
    t.xg[q] = xg[q];
  }
  const int n = p + 1, h = n / 2;
  for (int M = 0; M < 4; ++M) {
    auto m = [&](int r, int c) { return M == 0 ? t.S[r][c] : M == 1 ? t.D[r][c] : M == 2 ? t.S[c][r] : t.D[c][r]; };
    for (int r = 0; r <= h && r < n; ++r) {
      for (int c = 0; c < h; ++c) {
        t.eo[M][0][r][c] = 0.5 * (m(r, c) + m(r, n - 1 - c));
        t.eo[M][1][r][c] = 0.5 * (m(r, c) - m(r, n - 1 - c));
      }
      t.mid[M][r] = m(r, h);
    }
  }
  return t;
}

Tables<float> to_float(const Tables<double>& t) {
  Tables<float> f = {};
  for (int i = 0; i < kMaxN1; ++i) {
    for (int j = 0; j < kMaxN1; ++j) {
      f.S[i][j] = (float)t.S[i][j];
      f.D[i][j] = (float)t.D[i][j];
    }
    f.w[i] = (float)t.w[i];
    f.xg[i] = (float)t.xg[i];
  }
  for (int M = 0; M < 4; ++M)
    for (int r = 0; r < kMaxN1; ++r) {
      for (int c = 0; c < kMaxN1 / 2; ++c)
        for (int k = 0; k < 2; ++k) f.eo[M][k][r][c] = (float)t.eo[M][k][r][c];
      f.mid[M][r] = (float)t.mid[M][r];
    }
  return f;
}

std::vector<double> lattice_coords(int N, int p) {
  const std::vector<double> xi = gll_points(p);
  const int L = p * N + 1;
  std::vector<double> X(L);
  const double h = 1.0 / N;
  for (int I = 0; I < L; ++I) {
    int e = I / p;
    if (e > N - 1) e = N - 1;
    X[I] = h * (e + xi[I - p * e]);
  }
  return X;
}

std::vector<double> eval_global_1d(int N, int p, const std::vector<double>& X) {
  const std::vector<double> xi = gll_points(p);
  const int L = p * N + 1;
  const double h = 1.0 / N;
  std::vector<double> M(X.size() * L, 0.0);
  std::vector<double> V(p + 1);
  for (size_t k = 0; k < X.size(); ++k) {
    int e = (int)std::floor(X[k] / h);
    if (e > N - 1) e = N - 1;
    if (e < 0) e = 0;
    const double t = (X[k] - e * h) / h;
    lagrange(xi, t, V.data(), nullptr);
    for (int a = 0; a <= p; ++a) {
      const double v = std::fabs(V[a]) < 1e-15 ? 0.0 : V[a];
      M[k * L + p * e + a] = v;
    }
  }
  return M;
}

BandHost make_band(const std::vector<double>& M, int nout, int nin) {
  BandHost b;
  b.nout = nout;
  b.nin = nin;
  std::vector<int> first(nout), last(nout);
  int K = 1;
  for (int o = 0; o < nout; ++o) {
    int f = -1, l = -1;
    for (int i = 0; i < nin; ++i)
      if (M[(size_t)o * nin + i] != 0.0) {
        if (f < 0) f = i;
        l = i;
      }
    if (f < 0) f = l = 0;
    first[o] = f;
    last[o] = l;
    if (l - f + 1 > K) K = l - f + 1;
  }
  b.K = K;
  b.start.resize(nout);
  b.vals.assign((size_t)nout * K, 0.0);
  for (int o = 0; o < nout; ++o) {
    int s = first[o];
    if (s + K > nin) s = nin - K;
    b.start[o] = s;
    for (int k = 0; k < K; ++k) b.vals[(size_t)o * K + k] = M[(size_t)o * nin + s + k];
  }
  return b;
}

double tridiag_min_eig(const std::vector<double>& d, const std::vector<double>& e) {
  // Smallest eigenvalue: the largest of the negated matrix.
  std::vector<double> nd(d.size()), ne(e.size());
  for (size_t i = 0; i < d.size(); ++i) nd[i] = -d[i];
  for (size_t i = 0; i < e.size(); ++i) ne[i] = -e[i];
  return -tridiag_max_eig(nd, ne);
}

double tridiag_max_eig(const std::vector<double>& d, const std::vector<double>& e) {
  // Largest eigenvalue of the symmetric tridiagonal matrix (diagonal d,
  // off-diagonal e) by bisection on the Sturm count.
  const int m = (int)d.size();
  if (m == 0) return 0.0;
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(e[i]) : 0.0);
    lo = std::fmin(lo, d[i] - r);
    hi = std::fmax(hi, d[i] + r);
  }
  auto count_below = [&](double x) {   // eigenvalues < x
    int c = 0;
    double q = d[0] - x;
    if (q < 0) ++c;
    for (int i = 1; i < m; ++i) {
      if (q == 0.0) q = 1e-300;
      q = d[i] - x - e[i - 1] * e[i - 1] / q;
      if (q < 0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::fmax(1.0, std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count_below(mid) >= m)
      hi = mid;
    else
      lo = mid;
  }
  return 0.5 * (lo + hi);
}

}  // namespace mfh
