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
    s.rad.push_back(k < N1 ? 0 : 1);
    s.perm.push_back(k);
    s.Z *= (two_I[k] + 1);
  }
  return s;
}

SystemSpec tile_order(const SystemSpec &s, bool high_first) {
  std::vector<int> idx(s.N());
  for (int k = 0; k < s.N(); ++k) idx[k] = k;
  std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) {
    return high_first ? s.two_I[x] > s.two_I[y] : s.two_I[x] < s.two_I[y];
  });
  SystemSpec o = s;
  for (int k = 0; k < s.N(); ++k) {
    o.two_I[k] = s.two_I[idx[k]];
    o.a[k] = s.a[idx[k]];
    o.rad[k] = s.rad[idx[k]];
    o.perm[k] = s.perm[idx[k]];
  }
  return o;
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

// H_i = omega S_z + sum_{k in radical i} a_k I_k.S on one radical (electron fastest,
// then the radical's nuclei in mixed radix, first fastest): y = H_i x.
struct RadicalOp {
  int n = 0;
  int64_t dim = 2;
  std::vector<int64_t> stride;
  std::vector<int> d;
  std::vector<double> a, twoI;
  double omega = 0.0;
  void apply(const double *x, double *y) const {
    for (int64_t i = 0; i < dim; ++i) y[i] = 0.0;
    for (int64_t m = 0; m < dim / 2; ++m) {
      double h = omega;
      for (int k = 0; k < n; ++k) {
        const int dig = (int)((m / stride[k]) % d[k]);
        const double I = 0.5 * twoI[k], mk = I - dig;
        h += a[k] * mk;
        if (dig + 1 < d[k]) {   // |alpha, m_k-1> -> |beta, m_k> by (a/2) I+ S-, and back
          const double f = 0.5 * a[k] * std::sqrt(I * (I + 1.0) - mk * (mk - 1.0));
          const int64_t p = m + stride[k];
          y[2 * m + 1] += f * x[2 * p];
          y[2 * p] += f * x[2 * m + 1];
        }
      }
      y[2 * m] += 0.5 * h * x[2 * m];
      y[2 * m + 1] -= 0.5 * h * x[2 * m + 1];
    }
  }
};

// Number of eigenvalues of the symmetric tridiagonal (alpha, beta) below t (Sturm count).
static int sturm_count(const std::vector<double> &al, const std::vector<double> &be, double t) {
  int c = 0;
  double q = 1.0;
  for (size_t j = 0; j < al.size(); ++j) {
    const double b2 = j ? be[j - 1] * be[j - 1] : 0.0;
    q = al[j] - t - (j ? b2 / q : 0.0);
    if (q == 0.0) q = -1e-300;
    if (q < 0.0) ++c;
  }
  return c;
}

// Extreme eigenvalues of a radical Hamiltonian by Lanczos with full reorthogonalisation.
static bool radical_extremes(const RadicalOp &op, double &lo, double &hi) {
  const int64_t n = op.dim;
  const int mmax = (int)std::min<int64_t>(n, 90);
  std::vector<std::vector<double>> Q;
  std::vector<double> al, be, v(n), w(n);
  uint64_t st = 0x9E3779B97F4A7C15ull;
  double nr = 0.0;
  for (int64_t i = 0; i < n; ++i) {   // deterministic pseudo-random start vector
    st ^= st << 13;
    st ^= st >> 7;
    st ^= st << 17;
    v[i] = ((double)(st >> 11) * 0x1p-53) - 0.5;
    nr += v[i] * v[i];
  }
  nr = std::sqrt(nr);
  for (auto &x : v) x /= nr;
  double prev_hi = 0, prev_lo = 0;
  for (int j = 0; j < mmax; ++j) {
    Q.push_back(v);
    op.apply(v.data(), w.data());
    double a = 0.0;
    for (int64_t i = 0; i < n; ++i) a += w[i] * v[i];
    al.push_back(a);
    for (int pass = 0; pass < 2; ++pass)
      for (const auto &q : Q) {
        double c = 0.0;
        for (int64_t i = 0; i < n; ++i) c += w[i] * q[i];
        for (int64_t i = 0; i < n; ++i) w[i] -= c * q[i];
      }
    double b = 0.0;
    for (int64_t i = 0; i < n; ++i) b += w[i] * w[i];
    b = std::sqrt(b);
    // extreme Ritz values by bisection on the Sturm count
    double gl = 1e300, gh = -1e300;
    for (size_t q = 0; q < al.size(); ++q) {
      const double r = (q ? std::fabs(be[q - 1]) : 0.0) + (q < be.size() ? std::fabs(be[q]) : 0.0);
      gl = std::min(gl, al[q] - r);
      gh = std::max(gh, al[q] + r);
    }
    double a0 = gl, b0 = gh;
    for (int it = 0; it < 200 && b0 - a0 > 1e-13 * (std::fabs(gl) + std::fabs(gh) + 1e-300); ++it) {
      const double mid = 0.5 * (a0 + b0);
      if (sturm_count(al, be, mid) >= 1) b0 = mid; else a0 = mid;
    }
    lo = 0.5 * (a0 + b0);
    a0 = gl;
    b0 = gh;
    const int nn = (int)al.size();
    for (int it = 0; it < 200 && b0 - a0 > 1e-13 * (std::fabs(gl) + std::fabs(gh) + 1e-300); ++it) {
      const double mid = 0.5 * (a0 + b0);
      if (sturm_count(al, be, mid) >= nn) b0 = mid; else a0 = mid;
    }
    hi = 0.5 * (a0 + b0);
    const double range = std::max(hi - lo, 1e-300);
    if (b < 1e-12 * range || j + 1 == mmax) break;   // invariant subspace or step limit
    if (j >= 20 && std::fabs(hi - prev_hi) < 1e-10 * range && std::fabs(lo - prev_lo) < 1e-10 * range) break;
    prev_hi = hi;
    prev_lo = lo;
    be.push_back(b);
    for (int64_t i = 0; i < n; ++i) v[i] = w[i] / b;
  }
  return std::isfinite(lo) && std::isfinite(hi);
}

bool spectral_interval(const SystemSpec &s, double omega, double &Emin, double &Emax) {
  double lo_sum = 0.0, hi_sum = 0.0;
  for (int rad = 0; rad < 2; ++rad) {
    RadicalOp op;
    op.omega = omega;
    int64_t st = 1;
    for (int k = 0; k < s.N(); ++k) {
      if (s.rad[k] != rad) continue;
      op.stride.push_back(st);
      op.d.push_back(s.two_I[k] + 1);
      op.a.push_back(s.a[k]);
      op.twoI.push_back(s.two_I[k]);
      st *= s.two_I[k] + 1;
      ++op.n;
    }
    op.dim = 2 * st;
    double lo, hi;
    if (!radical_extremes(op, lo, hi)) return false;
    lo_sum += lo;
    hi_sum += hi;
  }
  // 2 J S1.S2 has eigenvalues J/2 (triplet) and -3J/2 (singlet): Weyl's inequality.
  Emax = hi_sum + std::max(0.5 * s.J, -1.5 * s.J);
  Emin = lo_sum + std::min(0.5 * s.J, -1.5 * s.J);
  return true;
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

static bool plan_field_once(const SystemSpec &s, double B_mT, double tol, double rdt, double r_scale,
                            double chol_tol, FieldPlan &out, std::string &msg, double &log_growth) {
  out = FieldPlan();
  out.B_mT = B_mT;
  out.omega = s.gamma * B_mT;   // signed: B < 0 reverses the field along z
  const double dk = std::fabs(s.kS - s.kT);
  // Spectrum of H: per-radical Lanczos extremes (with a relative safety margin), else the
  // triangle-inequality bound.
  double Emin = 0.0, Emax = 0.0, centre = 0.0, half = spectral_radius_bound(s, out.omega);
  if (spectral_interval(s, out.omega, Emin, Emax)) {
    const double hw = 0.5 * (Emax - Emin);
    const double margin = 0.01 * hw + 1e-9;
    if (hw + margin < half) {
      centre = 0.5 * (Emax + Emin);
      half = hw + margin;
    }
  }
  out.rho = half * r_scale;
  // r covers the real spectrum; keep it above dk/4 so the imaginary extent stays <= 1.
  out.r = std::max({out.rho, 0.25 * dk, 1e-9});
  out.c_re = centre;
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
  log_growth = lg;
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
  log_growth = lg * N;   // worst-case growth of |T_n| over the step, on the spectral rectangle
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

bool plan_field(const SystemSpec &s, double B_mT, double tol, double rdt, double r_scale, double chol_tol,
                double max_growth, FieldPlan &out, std::string &msg) {
  // Strong dissipation (|kS - kT| comparable to the spectral width) makes T_n(Gh) grow on the
  // imaginary extent of the spectrum; rounding errors grow with it.  Shorten the step until the
  // worst-case growth over one step is at most max_growth.
  double lg = 0.0;
  for (int tries = 0; tries < 40; ++tries) {
    if (!plan_field_once(s, B_mT, tol, rdt, r_scale, chol_tol, out, msg, lg)) return false;
    if (lg <= std::log(max_growth) || rdt < 2.0) return true;
    rdt *= 0.8;
  }
  return true;
}

}  // namespace rp
