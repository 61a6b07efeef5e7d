// Quadrature rule for the square-root integral
//     sqrt(lambda) = (2/pi) int_0^inf lambda / (lambda + z^2) dz      (paper: Sec. 1, eq. sqrt_rational)
// on a spectrum inside [lo, hi], by the conformal-map (Jacobi elliptic) substitution of Hale,
// Higham and Trefethen, SIAM J. Numer. Anal. 46 (2008), their third method for A^{1/2}:
//   k = sqrt(lo/hi), complementary parameter m' = 1 - k^2, K' = K(m') = pi / (2 AGM(1, k)),
//   z(v) = sqrt(lo) sc(v | m') for v in (0, K'), midpoint nodes v_j = (j - 1/2) K' / N,
//   shift_j = z_j^2,   weight_j = (2/pi) (K'/N) sqrt(lo) dn(v_j) / cn(v_j)^2.
// Jacobi functions come from the arithmetic-geometric mean with descending Landen steps
// (Abramowitz & Stegun 16.4).  For v past K'/2 the quarter-period shift cn(K'-w) = k sd(w),
// sn(K'-w) = cd(w), dn(K'-w) = k nd(w) keeps the small cn accurate to full relative precision.
#include <cmath>
#include <vector>

namespace rbcg {

// sn, cn, dn of u for parameter m' given through the complementary modulus kc = sqrt(1 - m').
static void jacobi_sncndn(double u, double kc, double* sn, double* cn, double* dn) {
  double a[40], c[40];
  a[0] = 1.0;
  double b = kc;
  c[0] = std::sqrt((1.0 - kc) * (1.0 + kc));
  int n = 0;
  while (n < 38 && std::fabs(c[n]) > 1e-17 * a[n]) {
    const double an = a[n];
    a[n + 1] = 0.5 * (an + b);
    c[n + 1] = 0.5 * (an - b);
    b = std::sqrt(an * b);
    ++n;
  }
  double phi = std::ldexp(a[n] * u, n);
  double phi_prev = phi;
  for (int i = n; i > 0; --i) {
    phi_prev = phi;
    phi = 0.5 * (phi + std::asin(c[i] * std::sin(phi) / a[i]));
  }
  *sn = std::sin(phi);
  *cn = std::cos(phi);
  *dn = (n > 0) ? *cn / std::cos(phi_prev - phi) : 1.0;
  if (n == 0) *dn = std::sqrt(1.0 - (1.0 - kc * kc) * (*sn) * (*sn));
}

static double agm(double a, double b) {
  for (int i = 0; i < 60 && std::fabs(a - b) > 1e-16 * a; ++i) {
    const double an = 0.5 * (a + b);
    b = std::sqrt(a * b);
    a = an;
  }
  return 0.5 * (a + b);
}

// Fills shifts[N], weights[N]; returns false on bad input.
bool sqrt_rule(double lo, double hi, int N, double* shifts, double* weights) {
  if (!(lo > 0.0) || !(hi >= lo) || N < 1) return false;
  if (hi == lo) hi = lo * (1.0 + 1e-12);
  const double k = std::sqrt(lo / hi);             // complementary modulus of m'
  const double Kp = M_PI / (2.0 * agm(1.0, k));    // K(m'), m' = 1 - k^2
  const double sl = std::sqrt(lo);
  for (int j = 0; j < N; ++j) {
    const double v = (j + 0.5) * Kp / N;
    double sc, dn_cn2;
    if (v <= 0.5 * Kp) {
      double sn, cn, dn;
      jacobi_sncndn(v, k, &sn, &cn, &dn);
      sc = sn / cn;
      dn_cn2 = dn / (cn * cn);
    } else {
      double sn, cn, dn;
      jacobi_sncndn(Kp - v, k, &sn, &cn, &dn);
      // sn(v) = cn(w)/dn(w), cn(v) = k sn(w)/dn(w), dn(v) = k / dn(w)
      sc = cn / (k * sn);
      dn_cn2 = dn / (k * sn * sn);
    }
    const double z = sl * sc;
    shifts[j] = z * z;
    weights[j] = (2.0 / M_PI) * (Kp / N) * sl * dn_cn2;
  }
  return true;
}

}  // namespace rbcg
