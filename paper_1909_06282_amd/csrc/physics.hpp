// Background, gravity model and growth-ODE right-hand side (FP64, host and device).
//
// Units: c = 1, lengths in Mpc/h, wavenumbers in h/Mpc, H0 = 1/2997.92458.
//
// * Background: flat matter + Lambda, E^2(a) = Om a^-3 + OL;
//   Omega_m(a) = Om a^-3 / E^2; 4 pi G rho_bar = 1.5 H0^2 Om a^-3.
// * Hu-Sawicki n = 1 (eq. mihusawicki): m^2 = M1/3 with
//   M1 = 1.5 (H0^2/|fR0|) X^3 / X0^2, M2 = 2.25 (H0^2/|fR0|^2) X^5 / X0^4,
//   X = Om a^-3 + 4 OL, X0 = Om + 4 OL.
// * mu(k,a) = 1 + (1/3) (k^2/a^2) / (k^2/a^2 + m^2) (below eq. first-displ-mg);
//   Pi(k,a) = k^2/a^2 + m^2.
// * Growth ODE in x = ln a (eq. d1, eq. full-d2 with the operator read as
//   a^2 H^2 T - 4 pi G rho mu and the source normalised by its GR limit):
//     D'' + (2 - 1.5 Omega_m(a)) D' - 1.5 Omega_m(a) mu D = RHS,
//     RHS(D1) = 0, RHS(D2) = -1.5 Omega_m(a) D1(k1) D1(k2) B / (1 - c^2),
//   B the braced factor of eq. full-d2 for the triangle (k, k1, k2, c).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace lpt2 {

constexpr double kH0 = 1.0 / 2997.92458;  // h/Mpc with c = 1
constexpr double kPi = 3.14159265358979323846264338327950288;

enum { GRAV_GR = 0, GRAV_FR = 1, GRAV_MUC = 2 };

struct Cosmo {
  double om, ol;        // Omega_m, Omega_L = 1 - Omega_m
  double h, ns;         // BBKS Gamma = om h; tilt
  int gravity;
  double fr0;           // |f_R0|
  double mu0;           // constant mu (test model)
};

__host__ __device__ inline double ainv3(double a) { return 1.0 / (a * a * a); }
__host__ __device__ inline double omega_m_a(const Cosmo& c, double a) {
  const double m = c.om * ainv3(a);
  return m / (m + c.ol);
}
__host__ __device__ inline double four_pi_g_rho(const Cosmo& c, double a) { return 1.5 * kH0 * kH0 * c.om * ainv3(a); }
__host__ __device__ inline double hs_m2(const Cosmo& c, double a) {
  const double x = c.om * ainv3(a) + 4.0 * c.ol, x0 = c.om + 4.0 * c.ol;
  return 0.5 * (kH0 * kH0 / c.fr0) * (x * x * x) / (x0 * x0);
}
__host__ __device__ inline double hs_M2(const Cosmo& c, double a) {
  const double x = c.om * ainv3(a) + 4.0 * c.ol, x0 = c.om + 4.0 * c.ol;
  const double x2 = x * x, x02 = x0 * x0;
  return 2.25 * (kH0 * kH0 / (c.fr0 * c.fr0)) * (x2 * x2 * x) / (x02 * x02);
}
// mu(k,a); m2 is hs_m2(c, a) (unused unless f(R)).
__host__ __device__ inline double mu_of(const Cosmo& c, double k, double a, double m2) {
  if (c.gravity == GRAV_GR) return 1.0;
  if (c.gravity == GRAV_MUC) return c.mu0;
  const double q = k * k / (a * a);
  return 1.0 + (1.0 / 3.0) * q / (q + m2);
}
__host__ __device__ inline double big_pi(double k, double a, double m2) { return k * k / (a * a) + m2; }

// Braced factor B of eq. full-d2.
__host__ __device__ inline double brace(const Cosmo& c, double k, double k1, double k2, double cs, double a) {
  const double c2 = cs * cs;
  const double m2 = (c.gravity == GRAV_FR) ? hs_m2(c, a) : 0.0;
  const double mk = mu_of(c, k, a, m2), m1 = mu_of(c, k1, a, m2), mm2 = mu_of(c, k2, a, m2);
  double b = mk - c2 * (m1 + mm2 - mk);
  if (c.gravity == GRAV_FR) {
    const double pk = big_pi(k, a, m2), p1 = big_pi(k1, a, m2), p2 = big_pi(k2, a, m2);
    const double dot = k1 * k2 * cs;
    const double br = 2.0 * c2 * (m1 + mm2 - 2.0) + dot / (k1 * k1) * (m1 - 1.0) + dot / (k2 * k2) * (mm2 - 1.0);
    b += m2 / pk * br;
    b -= (2.0 / 27.0) * four_pi_g_rho(c, a) * (k * k / (a * a)) * hs_M2(c, a) / (pk * p1 * p2);
  }
  return b;
}

// Triangle with |k1 + k2| = k, k1 = r k2, angle cos = cs between k1 and k2.
__host__ __device__ inline void triangle(double k, double r, double cs, double& k1, double& k2) {
  k2 = k / sqrt(1.0 + r * r + 2.0 * r * cs);
  k1 = r * k2;
}

struct GrowthTri {
  double k, k1, k2, cs, bgr;  // wavenumbers, cos(theta), 1 - cos^2
  int winther;                // D1(k)^2 in place of D1(k1) D1(k2)
  int with_d2;
};

// The factors of the growth ODEs that depend on the time x = ln a only.
struct GrowthAFac {
  double ia2;   // a^-2
  double fr;    // 2 - 1.5 Omega_m(a)
  double gg;    // 1.5 Omega_m(a)
  double ms;    // m^2(a) (f(R))
  double gm2;   // (2/27) 4 pi G rho(a) M2(a) (f(R))
};

// The right-hand side of the growth ODEs with everything that does not
// depend on a or on the state worked out once per node, and everything that
// depends on a alone in GrowthAFac (powers of a from one exponential, one
// division for Omega_m(a)); one reciprocal per distinct wavenumber for 1/Pi
// remains.  The printed forms of mu, the brace and the M_k are algebraically
// the same expressions (see brace(), mu_of(), hs_m2(), hs_M2()).
struct GrowthRhs {
  int gravity;                   // GRAV_*
  double om, ol, mu0;
  double m2c, M2c, Gc;           // m^2 = m2c X^3, M2 = M2c X^5 (X = om a^-3 + 4 ol), 4 pi G rho = Gc a^-3
  double q, q1, q2;              // k^2, k1^2, k2^2
  double c2, r12, r21, ibgr;     // cos^2, (k1.k2)/k1^2, (k1.k2)/k2^2, 1/(1 - cos^2)
  bool sym;                      // k1 == k2: D1(k1) = D1(k2) (one pair of states serves both)
  int winther, with_d2;

  __host__ __device__ void init(const Cosmo& c, const GrowthTri& g) {
    gravity = c.gravity;
    om = c.om;
    ol = c.ol;
    mu0 = c.mu0;
    const double x0 = c.om + 4.0 * c.ol, x02 = x0 * x0;
    m2c = (c.gravity == GRAV_FR) ? 0.5 * (kH0 * kH0 / c.fr0) / x02 : 0.0;
    M2c = (c.gravity == GRAV_FR) ? 2.25 * (kH0 * kH0 / (c.fr0 * c.fr0)) / (x02 * x02) : 0.0;
    Gc = 1.5 * kH0 * kH0 * c.om;
    q = g.k * g.k;
    q1 = g.k1 * g.k1;
    q2 = g.k2 * g.k2;
    c2 = g.cs * g.cs;
    r12 = g.k1 > 0.0 ? g.cs * g.k2 / g.k1 : 0.0;
    r21 = g.k2 > 0.0 ? g.cs * g.k1 / g.k2 : 0.0;
    ibgr = 1.0 / g.bgr;
    sym = g.k1 == g.k2;
    winther = g.winther;
    with_d2 = g.with_d2;
  }

  __host__ __device__ GrowthAFac afac(double x) const {
    GrowthAFac f;
    const double ia = exp(-x), ia2 = ia * ia, ia3 = ia2 * ia;
    const double m = om * ia3;
    const double oma = m / (m + ol);
    f.ia2 = ia2;
    f.fr = 2.0 - 1.5 * oma;
    f.gg = 1.5 * oma;
    const double X = m + 4.0 * ol, X2 = X * X;
    f.ms = m2c * X2 * X;
    f.gm2 = (2.0 / 27.0) * (Gc * ia3) * (M2c * X2 * X2 * X);
    return f;
  }

  // y = [D1(k), D1'(k), D1(k1), D1'(k1), D1(k2), D1'(k2), D2, D2'].  When
  // sym, the D1(k2) pair takes the same operations on the same values as the
  // D1(k1) pair and stays equal to it bit for bit.  rcp(p) returns 1/p.
  template <class Rcp>
  __host__ __device__ void eval_at(const GrowthAFac& af, const double* y, double* dy, Rcp rcp) const {
    const double fr = af.fr, gg = af.gg;
    double mk = 1.0, m1 = 1.0, mm2 = 1.0, b = 1.0;  // b: the brace over (1 - cos^2)
    if (gravity == GRAV_MUC) {
      mk = m1 = mm2 = mu0;
      b = mu0;
    } else if (gravity == GRAV_FR) {
      const double ms = af.ms;
      const double qa = q * af.ia2, ipk = rcp(qa + ms);
      mk = 1.0 + (1.0 / 3.0) * qa * ipk;
      if (with_d2) {
        const double qa1 = q1 * af.ia2, ip1 = rcp(qa1 + ms);
        m1 = 1.0 + (1.0 / 3.0) * qa1 * ip1;
        double ip2 = ip1;
        if (sym) {
          mm2 = m1;
        } else {
          const double qa2 = q2 * af.ia2;
          ip2 = rcp(qa2 + ms);
          mm2 = 1.0 + (1.0 / 3.0) * qa2 * ip2;
        }
        double br = mk - c2 * (m1 + mm2 - mk);
        br += ms * ipk * (2.0 * c2 * (m1 + mm2 - 2.0) + r12 * (m1 - 1.0) + r21 * (mm2 - 1.0));
        br -= af.gm2 * qa * ipk * ip1 * ip2;
        b = br * ibgr;
      }
    }
    // every row runs in every case (no branch, so the state stays in
    // registers): without D2 the rows past the first pair see the initial
    // coefficients, stay finite and are never read
    const double p00 = y[0] * y[0], p24 = y[2] * y[4];
    const double src = winther ? p00 : p24;
    dy[0] = y[1];
    dy[1] = -fr * y[1] + gg * mk * y[0];
    dy[2] = y[3];
    dy[3] = -fr * y[3] + gg * m1 * y[2];
    dy[4] = y[5];
    dy[5] = -fr * y[5] + gg * mm2 * y[4];
    dy[6] = y[7];
    dy[7] = -fr * y[7] + gg * mk * y[6] - gg * src * b;
  }

  __host__ __device__ void eval(double x, const double* y, double* dy) const {
    eval_at(afac(x), y, dy, [](double p) { return 1.0 / p; });
  }
};

// EdS growing-mode start of the state (power-law mode for the constant-mu model).
__host__ __device__ inline void growth_start(const Cosmo& c, double a_init, double* y) {
  double dd1, sd1, dd2, sd2;
  if (c.gravity == GRAV_MUC) {
    const double p = (-0.5 + sqrt(0.25 + 6.0 * c.mu0)) / 2.0;
    const double cc = -1.5 * c.mu0 / (4.0 * p * p + p - 1.5 * c.mu0);
    dd1 = pow(a_init, p);
    sd1 = p * dd1;
    dd2 = cc * pow(a_init, 2.0 * p);
    sd2 = 2.0 * p * dd2;
  } else {
    dd1 = a_init;
    sd1 = a_init;
    dd2 = -3.0 / 7.0 * a_init * a_init;
    sd2 = -6.0 / 7.0 * a_init * a_init;
  }
  y[0] = dd1; y[1] = sd1; y[2] = dd1; y[3] = sd1; y[4] = dd1; y[5] = sd1; y[6] = dd2; y[7] = sd2;
}

// Classical RK4 from ln(a_init) to ln(a) in `steps` equal steps from the
// growing-mode start.  Returns raw D1, D2.
__host__ __device__ inline void growth_solve(const Cosmo& c, const GrowthTri& g, double a_init, double a,
                                             int steps, double& d1, double& d2) {
  GrowthRhs f;
  f.init(c, g);
  double y[8], k1[8], k2[8], k3[8], k4[8], t[8];
  growth_start(c, a_init, y);
  const double x0 = log(a_init), x1 = log(a);
  const double h = (x1 - x0) / steps;
  for (int s = 0; s < steps; ++s) {
    const double x = x0 + s * h;
    f.eval(x, y, k1);
    for (int i = 0; i < 8; ++i) t[i] = y[i] + 0.5 * h * k1[i];
    f.eval(x + 0.5 * h, t, k2);
    for (int i = 0; i < 8; ++i) t[i] = y[i] + 0.5 * h * k2[i];
    f.eval(x + 0.5 * h, t, k3);
    for (int i = 0; i < 8; ++i) t[i] = y[i] + h * k3[i];
    f.eval(x + h, t, k4);
    for (int i = 0; i < 8; ++i) y[i] = y[i] + (h / 6.0) * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
  }
  d1 = y[0];
  d2 = y[6];
}

// Linear interpolation in ln k on nk log-spaced nodes [kmin, kmax], clamped.
__host__ __device__ inline double interp_lnk(const double* tab, int nk, double lkmin, double lkmax, double k) {
  if (!(k > 0.0)) return tab[0];
  double u = (log(k) - lkmin) / (lkmax - lkmin) * (nk - 1);
  if (u < 0.0) u = 0.0;
  if (u > nk - 1.0) u = nk - 1.0;
  int i = (int)floor(u);
  if (i > nk - 2) i = nk - 2;
  const double t = u - i;
  return tab[i] + t * (tab[i + 1] - tab[i]);
}

// BBKS transfer function, q = k / (Om h).
__host__ __device__ inline double bbks(const Cosmo& c, double k) {
  const double q = k / (c.om * c.h);
  if (!(q > 0.0)) return 1.0;
  const double x = 2.34 * q;
  const double a1 = 16.1 * q, a2 = 5.46 * q, a3 = 6.71 * q;
  const double poly = 1.0 + 3.89 * q + a1 * a1 + a2 * a2 * a2 + (a3 * a3) * (a3 * a3);
  return log1p(x) / x * pow(poly, -0.25);
}

}  // namespace lpt2
