// Host-side planning of the Chebyshev propagator (see plan.hpp for the scheme).
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>

namespace rp {

SystemSpec make_spec(int N1, int N2, const int32_t *two_I, const double *a_mT, double J_mT,
                     double kS, double kT, double T, double gamma) {
  SystemSpec s;
  s.N1 = N1;
  s.N2 = N2;
  s.gamma = gamma;
  s.J = J_mT * gamma;
  s.kS = kS;
  s.kT = kT;
  s.T = T;
  s.Z = 1;
  for (int k = 0; k < N1 + N2; ++k) {
    s.two_I.push_back(two_I[k]);
    s.a.push_back(a_mT[k] * gamma);
    s.Z *= (two_I[k] + 1);
  }
  return s;
}

void bessel_j(double x, int nmax, double *out) {
  for (int n = 0; n <= nmax; ++n) out[n] = 0.0;
  if (x == 0.0) {
    out[0] = 1.0;
    return;
  }
  // Start well above both nmax and x, where J_m(x) is negligible, and recur downwards
  // J_{n-1} = (2n/x) J_n - J_{n+1}; the recurrence is stable in this direction.
  const double top = std::max<double>(nmax, x);
  int m = (int)(top + 40.0 + 10.0 * std::cbrt(top + 1.0));
  m += (m & 1);
  std::vector<double> j(m + 2, 0.0);
  double jp1 = 0.0, jn = 1e-300;
  j[m] = jn;
  for (int n = m; n >= 1; --n) {
    double jm1 = (2.0 * n / x) * jn - jp1;
    jp1 = jn;
    jn = jm1;
    j[n - 1] = jm1;
    if (std::fabs(jn) > 1e250) {  // rescale everything computed so far
      for (int q = n - 1; q <= m; ++q) j[q] *= 1e-250;
      jp1 *= 1e-250;
      jn *= 1e-250;
    }
  }
  double norm = j[0];
  for (int k = 2; k <= m; k += 2) norm += 2.0 * j[k];
  for (int n = 0; n <= nmax; ++n) out[n] = j[n] / norm;
}

double spectral_radius_bound(const SystemSpec &s, double omega) {
  double rho = std::fabs(omega) + 1.5 * std::fabs(s.J);
  for (int k = 0; k < s.N(); ++k) rho += std::fabs(s.a[k]) * (0.5 * s.two_I[k] + 1.0) * 0.5;
  return rho;
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on P_n).
static void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      // p1 = P_n(z), p0 = P_{n-1}(z)
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
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Pivoted Cholesky of a symmetric positive semidefinite n x n matrix (row-major);
// stops when the largest remaining diagonal falls below tol * max(diag).
// Returns L as n x rank (row-major), A ~= L L^T.
static std::vector<double> pivoted_cholesky(const std::vector<double> &A, int n, double tol, int &rank) {
  std::vector<double> d(n);
  double dmax = 0.0;
  for (int i = 0; i < n; ++i) {
    d[i] = A[(size_t)i * n + i];
    dmax = std::max(dmax, d[i]);
  }
  std::vector<std::vector<double>> cols;
  std::vector<char> used(n, 0);
  while ((int)cols.size() < n) {
    int p = -1;
    double best = -1.0;
    for (int i = 0; i < n; ++i)
      if (!used[i] && d[i] > best) {
        best = d[i];
        p = i;
      }
    if (p < 0 || best <= tol * dmax) break;
    std::vector<double> col(n);
    const double piv = std::sqrt(best);
    for (int i = 0; i < n; ++i) {
      double v = A[(size_t)i * n + p];
      for (const auto &c : cols) v -= c[i] * c[p];
      col[i] = v / piv;
    }
    used[p] = 1;
    for (int i = 0; i < n; ++i) d[i] = used[i] ? 0.0 : d[i] - col[i] * col[i];
    cols.push_back(std::move(col));
  }
  rank = (int)cols.size();
  std::vector<double> L((size_t)n * std::max(rank, 1), 0.0);
  for (int r = 0; r < rank; ++r)
    for (int i = 0; i < n; ++i) L[(size_t)i * rank + r] = cols[r][i];
  return L;
}

bool plan_field(const SystemSpec &s, double B_mT, double tol, double rdt, double r_scale,
                double chol_tol, FieldPlan &out, std::string &msg) {
  out = FieldPlan();
  out.B_mT = B_mT;
  out.omega = s.gamma * std::fabs(B_mT);
  const double dk = std::fabs(s.kS - s.kT);
  out.rho = spectral_radius_bound(s, out.omega) * r_scale;
  // r covers the real spectrum; keep it above dk/4 so the imaginary extent stays <= 1.
  out.r = std::max({out.rho, 0.25 * dk, 1e-9});
  out.c_re = 0.0;
  out.c_im = -0.25 * dk;
  out.n_steps = std::max<int64_t>(1, (int64_t)std::ceil(out.r * s.T / rdt - 1e-12));
  out.dt = s.T / (double)out.n_steps;
  out.x = out.r * out.dt;

  // Growth of T_n on the spectral rectangle [-rho/r, rho/r] x i[-eps, eps].
  const double x0 = std::min(1.0, out.rho / out.r), eps = 0.25 * dk / out.r;
  std::complex<double> z(x0, eps);
  std::complex<double> w = z + std::sqrt(z * z - 1.0);
  double growth = std::max(std::abs(w), 1.0 / std::abs(w));
  growth = std::max(growth, 1.0);

  const int nmax = (int)(out.x + 80.0 + 25.0 * std::cbrt(out.x + 1.0));
  std::vector<double> J(nmax + 1);
  bessel_j(out.x, nmax, J.data());
  int N = 1;
  double lg = std::log(growth);
  for (int n = nmax; n >= 1; --n) {
    double term = 2.0 * std::fabs(J[n]) * std::exp(n * lg);
    if (term > tol) {
      N = n;
      break;
    }
  }
  if (N >= nmax - 5) {
    msg = "Chebyshev series did not reach the tolerance; reduce rdt";
    return false;
  }
  out.n_terms = N + 1;
  // a_n = (2 - delta_n0) (-i)^n J_n(x) exp(-i c dt)
  const std::complex<double> ph = std::exp(std::complex<double>(out.c_im * out.dt, -out.c_re * out.dt));
  const std::complex<double> mi(0.0, -1.0);
  std::complex<double> pw(1.0, 0.0);
  out.coef.resize(out.n_terms);
  for (int n = 0; n < out.n_terms; ++n) {
    out.coef[n] = (n == 0 ? 1.0 : 2.0) * J[n] * pw * ph;
    pw *= mi;
  }

  // In-step quadrature matrix Kq_mn = int_0^dt J_m(r s) J_n(r s) exp(-kappa s) ds.
  const int nt = out.n_terms;
  const double kappa = 0.5 * (s.kS + s.kT);
  std::vector<double> gx, gw;
  gauss_legendre(20, gx, gw);
  const int panels = std::max(1, (int)std::ceil(out.x / 2.0));
  const double h = out.dt / panels;
  std::vector<double> Kq((size_t)nt * nt, 0.0), Jn(nt);
  for (int p = 0; p < panels; ++p) {
    for (int q = 0; q < (int)gx.size(); ++q) {
      const double sq = p * h + 0.5 * h * (gx[q] + 1.0);
      const double wq = 0.5 * h * gw[q] * std::exp(-kappa * sq);
      bessel_j(out.r * sq, nt - 1, Jn.data());
      for (int m = 0; m < nt; ++m) {
        const double a = wq * Jn[m];
        double *row = &Kq[(size_t)m * nt];
        for (int n = m; n < nt; ++n) row[n] += a * Jn[n];
      }
    }
  }
  for (int m = 0; m < nt; ++m)
    for (int n = 0; n < m; ++n) Kq[(size_t)m * nt + n] = Kq[(size_t)n * nt + m];
  int rank = 0;
  std::vector<double> L = pivoted_cholesky(Kq, nt, chol_tol, rank);
  if (rank < 1) {
    msg = "in-step quadrature matrix has rank 0";
    return false;
  }
  out.rank = rank;
  out.ell.resize((size_t)nt * rank);
  for (int n = 0; n < nt; ++n) {
    const double f = (n == 0 ? 1.0 : 2.0) * M_SQRT1_2;
    for (int r = 0; r < rank; ++r) out.ell[(size_t)n * rank + r] = f * L[(size_t)n * rank + r];
  }
  return true;
}

}  // namespace rp
