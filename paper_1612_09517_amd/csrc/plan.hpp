// Host-side planning of the Chebyshev propagation of one radical pair at one field.
//
// The wavepacket of Eq. 13 evolves under G = H - iK.  Writing
// K = k_min/2 + (dk/2) P_x (P_x = P_S if kS >= kT, else P_T; dk = |kS - kT|)
// the scalar decay exp(-k_min t/2) is factored out and G' = H - i (dk/2) P_x is
// expanded in Chebyshev polynomials of  Gh = (G' - c)/r  (Tal-Ezer & Kosloff):
//   exp(-i G' dt) = exp(-i c dt) sum_n (2 - delta_n0) (-i)^n J_n(r dt) T_n(Gh).
// The spectrum of H lies in [-rho, rho]; the dissipative part shifts it into
// the strip -dk/2 <= Im <= 0, so c = -i dk/4 centres it.  Within one step the
// time integral of ||P_S psi(t_j + s)||^2 exp(-k_min s) is the quadratic form
//   y_j = sum_M  e(M)^dag Kq e(M),  e_n(M) = (2 - delta_n0) (-i)^n <S|phi_n(M)>,
//   Kq_mn = int_0^dt J_m(r s) J_n(r s) exp(-kappa s) ds,  kappa = (kS + kT)/2,
// whose matrix Kq is computed by composite Gauss-Legendre and factored as
// ell ell^T by pivoted Cholesky, so that y_j = sum_r sum_M |sum_n ell_nr e_n(M)|^2.
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

namespace rp {

struct SystemSpec {
  int N1 = 0, N2 = 0;
  std::vector<int> two_I;
  std::vector<double> a;       // rad/us
  std::vector<int> rad;        // radical (0 or 1) of each nucleus
  std::vector<int> perm;       // caller's index of each nucleus (identity unless reordered)
  double J = 0.0;              // rad/us (term 2 J S1.S2)
  double kS = 0.0, kT = 0.0;   // 1/us
  double T = 0.0;              // us
  double gamma = 0.0;          // rad/us/mT
  int64_t Z = 1;
  int N() const { return N1 + N2; }
};

struct FieldPlan {
  double B_mT = 0.0;
  double omega = 0.0;          // gamma * B, rad/us
  double rho = 0.0;            // bound on the spectral radius of H
  double r = 0.0;              // Chebyshev half-width
  double c_re = 0.0, c_im = 0.0;   // expansion centre c (G' - c)/r
  double dt = 0.0;
  double x = 0.0;              // r dt
  int64_t n_steps = 0;
  int n_terms = 0;             // N + 1 polynomials per step
  int rank = 0;                // columns of ell
  std::vector<std::complex<double>> coef;  // [n_terms] a_n of one step
  std::vector<double> ell;     // [n_terms][rank]
};

// Builds the spec from the C-ABI struct fields (validated by the caller).
SystemSpec make_spec(int N1, int N2, const int32_t *two_I, const double *a_mT, double J_mT,
                     double kS, double kT, double T, double gamma);

// The same system with its nuclei reordered for the tiled kernels: spin-1/2 nuclei first
// (power-of-two strides), then the others by increasing 2I; with high_first, by decreasing
// 2I instead (higher spins on the fastest axes, for the mixed-radix kernel).  Radical flags
// and the caller's indices travel with each nucleus; the physics does not depend on the order.
SystemSpec tile_order(const SystemSpec &s, bool high_first = false);

// J_0(x)..J_nmax(x), x >= 0, Miller backward recurrence with the normalisation
// J_0 + 2 sum_k J_2k = 1.
void bessel_j(double x, int nmax, double *out);

// Plans one field.  tol: truncation tolerance; rdt: target r dt (shortened while the worst-case
// growth of the Chebyshev polynomials over one step exceeds max_growth); r_scale multiplies rho.
// Returns false (with msg) on failure.
bool plan_field(const SystemSpec &s, double B_mT, double tol, double rdt, double r_scale,
                double chol_tol, double max_growth, FieldPlan &out, std::string &msg);

// Upper bound on the spectral radius of H at field omega:
// |omega| + sum_k |a_k| (I_k + 1)/2 + 3|J|/2 (triangle inequality over Eq. 1 terms,
// with ||I.S|| = (I+1)/2 for a spin-1/2 electron and ||S1.S2|| = 3/4).
double spectral_radius_bound(const SystemSpec &s, double omega);

// [Emin, Emax] containing the spectrum of H: with J = 0 the spectrum of H is the sum of
// the spectra of the two radical Hamiltonians (each found by Lanczos on its own 2 Z_i
// dimensional space); J shifts eigenvalues by at most its extreme values J/2, -3J/2.
bool spectral_interval(const SystemSpec &s, double omega, double &Emin, double &Emax);

}  // namespace rp
