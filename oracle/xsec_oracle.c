/*
 * xsec_oracle.c -- plain FP64 CPU reference for the line-list cross-section path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  It shares no code,
 * header, table or constant with the GPU library: every constant below is
 * declared here on its own, and the Faddeeva function is computed by a
 * different published method (modified trapezoidal rule) from the GPU's.
 *
 * What it computes (PyExoCross 2.0, arXiv 2609.17273):
 *   - partition functions: Eq. (pf) for LTE, Eq. (Q nlte 2T) for two temperatures,
 *     Eq. (Q nlte Nvib) for custom vibronic densities;
 *   - line intensities: Eqs. (abs intensity lte), (nlte ab 2T),
 *     (ems intensity lte), (nlte em 2T), (nlte ab pop density),
 *     (nlte em pop density), with E_rot = E - E_vib(v) from Eqs. (Enonlte)
 *     and (Erot nonlte);
 *   - cross sections: Eq. (xsec) with unit-area profiles, evaluated only at grid
 *     points with |nu - nu_fi| <= cutoff (section "Spectral synthesis"), lines
 *     with nu_fi <= 0 discarded;
 *   - profiles of Table (tab:profile): Doppler / Gaussian, Lorentzian, and the
 *     SciPy-convention Voigt (Re of the Faddeeva function), sampled at the
 *     grid points or averaged over the bins centred on them ("binned"), and
 *     the Thompson and Olivero pseudo-Voigts;
 *   - the cooling function, Eq. (cf);
 *   - per-line adjoint sums of sigma against a cotangent dL/dsigma.
 *
 * Everything is the plain definition: sigma_k = sum_i S_i f_i(nu_k - nu_i),
 * summed in FP64 with Neumaier compensation.  Build with
 *   gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC
 * so that nu_k = nu0 + k*dnu and dnu_ik = nu_k - nu_i are rounded exactly as
 * written (no FMA contraction).
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* CODATA 2018 exact SI values, in CGS units (the paper's symbol table gives
 * h, c, k_B and c2 = h c / k_B by symbol only). */
#define OR_H 6.62607015e-27      /* erg s */
#define OR_C 2.99792458e10       /* cm / s */
#define OR_KB 1.380649e-16       /* erg / K */
#define OR_AMU 1.66053906660e-24 /* g */
#define OR_PI 3.14159265358979323846
#define OR_LN2 0.69314718055994530942

enum { OR_DOPPLER = 0, OR_GAUSSIAN = 1, OR_LORENTZ = 2, OR_VOIGT = 3 };
/* Bin-integrated forms of the same four profiles (Table tab:profile, "binned"
 * methods): the mean of the profile over the bin [nu_k - dnu/2, nu_k + dnu/2]
 * centred on the grid point. */
enum { OR_BIN_DOPPLER = 4, OR_BIN_GAUSSIAN = 5, OR_BIN_LORENTZ = 6, OR_BIN_VOIGT = 7 };
/* Pseudo-Voigt approximations of the profile table, with the Voigt's widths. */
enum { OR_PV_THOMPSON = 8, OR_PV_OLIVERO = 9 };
static int or_base(int profile) {
  return profile < 4 ? profile : (profile < 8 ? profile - 4 : OR_VOIGT);
}
enum { OR_ABSORPTION = 0, OR_EMISSION = 1 };
enum { OR_LTE = 0, OR_NLTE_2T = 1, OR_NLTE_DENSITY = 2 };

double or_c2(void) { return OR_H * OR_C / OR_KB; }
int or_max_threads(void) { return omp_get_max_threads(); }
/* Thread count of later parallel regions (timing only; results do not depend on it). */
void or_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
void or_constants(double* out5) {
  out5[0] = OR_H; out5[1] = OR_C; out5[2] = OR_KB; out5[3] = OR_AMU; out5[4] = or_c2();
}

/* ---- Neumaier (improved Kahan-Babuska) summation ------------------------ */
typedef struct { double s, c; } or_sum;
static void or_add(or_sum* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
  else a->c += (x - t) + a->s;
  a->s = t;
}
static double or_total(const or_sum* a) { return a->s + a->c; }

/* ---- Partition function ------------------------------------------------- */
/* LTE, Eq. (pf): Q(T) = sum_n g_n exp(-c2 E_n / T), and its T-derivative
 * dQ/dT = sum_n g_n (c2 E_n / T^2) exp(-c2 E_n / T).
 * Two temperatures, Eq. (Q nlte 2T): Q = sum g exp(-c2 Evib(v)/Tv) exp(-c2 Erot/Tr)
 * with Erot = E - Evib(v) (Eq. Erot nonlte).
 * Custom vibronic densities, Eq. (Q nlte Nvib): Q = sum g n_vib(v) exp(-c2 Erot/Tr).
 * dQdT is not defined for the non-LTE forms (NaN). */
int or_partition(int64_t n, const double* E, const double* g, const int32_t* v,
                 const double* evib, const double* nvib, int pop, double T, double Tv,
                 double Tr, double* Q, double* dQdT) {
  const double c2 = or_c2();
  or_sum q = {0, 0}, dq = {0, 0};
  for (int64_t i = 0; i < n; ++i) {
    if (pop == OR_LTE) {
      double b = exp(-c2 * E[i] / T);
      or_add(&q, g[i] * b);
      or_add(&dq, g[i] * (c2 * E[i] / (T * T)) * b);
    } else if (pop == OR_NLTE_2T) {
      double ev = evib[v[i]];
      double er = E[i] - ev;
      or_add(&q, g[i] * exp(-c2 * ev / Tv) * exp(-c2 * er / Tr));
    } else {
      double er = E[i] - evib[v[i]];
      or_add(&q, g[i] * nvib[v[i]] * exp(-c2 * er / Tr));
    }
  }
  *Q = or_total(&q);
  if (dQdT) *dQdT = (pop == OR_LTE) ? or_total(&dq) : NAN;
  return 0;
}

/* ---- Line intensities --------------------------------------------------- */
/* nu_i = E_u - E_l.  Lines with nu_i <= 0 are discarded (S = 0, keep = 0).
 * Absorption, LTE (Eq. abs intensity lte):
 *   I = g_u A / (8 pi c nu^2) * exp(-c2 E_l / T) * (1 - exp(-c2 nu / T)) / Q(T)
 * Absorption, two temperatures (Eqs. nlte v, nlte ab 2T):
 *   I = g_u A / (8 pi c nu^2) * exp(-c2 E_l,vib/Tv) exp(-c2 E_l,rot/Tr)
 *       * (1 - exp(-c2 (nu_vib/Tv + nu_rot/Tr))) / Q(Tv, Tr)
 * Emission, LTE (Eq. ems intensity lte):
 *   eps = g_u h c A nu / (4 pi) * exp(-c2 E_u / T) / Q(T)
 * Emission, two temperatures (Eq. nlte em 2T):
 *   eps = h c / (4 pi) g_u A nu * exp(-c2 E_u,vib/Tv) exp(-c2 E_u,rot/Tr) / Q(Tv, Tr)
 * Absorption, custom vibronic densities (Eq. nlte ab pop density):
 *   I = g_u A / (8 pi c nu^2) * n_vib(v_l) exp(-c2 E_l,rot/Tr) (1 - exp(-c2 nu/Tr)) / Q(Tr)
 * Emission, custom vibronic densities (Eq. nlte em pop density):
 *   eps = h c / (4 pi) g_u A nu * n_vib(v_u) exp(-c2 E_u,rot/Tr) / Q(Tr)
 * (1 - exp(-x)) is formed as -expm1(-x).  An optional per-line log scale s_i
 * multiplies S_i by exp(s_i) (the per-line scales of the adjoint). */
int or_intensities(int64_t nl, const int32_t* up, const int32_t* lo, const float* A,
                   const float* lscale, const double* E, const double* g,
                   const int32_t* v, const double* evib, const double* nvib, int mode,
                   int pop, double T, double Tv, double Tr, double Q, double* nu_out,
                   double* S_out, int8_t* keep) {
  const double c2 = or_c2();
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nl; ++i) {
    int32_t u = up[i], l = lo[i];
    double nu = E[u] - E[l];
    nu_out[i] = nu;
    if (!(nu > 0.0)) { S_out[i] = 0.0; keep[i] = 0; continue; }
    keep[i] = 1;
    double a = (double)A[i];
    double S;
    if (mode == OR_ABSORPTION) {
      double pre = g[u] * a / (8.0 * OR_PI * OR_C * nu * nu);
      if (pop == OR_LTE) {
        S = pre * exp(-c2 * E[l] / T) * (-expm1(-c2 * nu / T)) / Q;
      } else if (pop == OR_NLTE_2T) {
        double evu = evib[v[u]], evl = evib[v[l]];
        double nuv = evu - evl, nur = (E[u] - evu) - (E[l] - evl);
        S = pre * exp(-c2 * evl / Tv) * exp(-c2 * (E[l] - evl) / Tr) *
            (-expm1(-c2 * (nuv / Tv + nur / Tr))) / Q;
      } else {
        double evl = evib[v[l]];
        S = pre * nvib[v[l]] * exp(-c2 * (E[l] - evl) / Tr) * (-expm1(-c2 * nu / Tr)) / Q;
      }
    } else {
      double pre = g[u] * OR_H * OR_C * a * nu / (4.0 * OR_PI);
      if (pop == OR_LTE) {
        S = pre * exp(-c2 * E[u] / T) / Q;
      } else if (pop == OR_NLTE_2T) {
        double evu = evib[v[u]];
        S = pre * exp(-c2 * evu / Tv) * exp(-c2 * (E[u] - evu) / Tr) / Q;
      } else {
        double evu = evib[v[u]];
        S = pre * nvib[v[u]] * exp(-c2 * (E[u] - evu) / Tr) / Q;
      }
    }
    if (lscale) S *= exp((double)lscale[i]);
    S_out[i] = S;
  }
  return 0;
}

/* d ln S / dT for LTE (adjoint of the intensity with respect to T):
 *   absorption: c2 E_l / T^2 - (c2 nu / T^2) / (exp(c2 nu / T) - 1) - Q'/Q
 *   emission:   c2 E_u / T^2 - Q'/Q */
int or_dlnS_dT(int64_t nl, const int32_t* up, const int32_t* lo, const double* E, int mode,
               double T, double Q, double dQdT, double* out) {
  const double c2 = or_c2();
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nl; ++i) {
    double nu = E[up[i]] - E[lo[i]];
    if (!(nu > 0.0)) { out[i] = 0.0; continue; }
    if (mode == OR_ABSORPTION)
      out[i] = c2 * E[lo[i]] / (T * T) - (c2 * nu / (T * T)) / expm1(c2 * nu / T) - dQdT / Q;
    else
      out[i] = c2 * E[up[i]] / (T * T) - dQdT / Q;
  }
  return 0;
}

/* ---- Cooling function --------------------------------------------------- */
/* Eq. (cf): W(T) = 1/(4 pi Q(T)) sum over transitions of A h c nu g_u exp(-c2 E_u / T),
 * with Q(T) of Eq. (pf), for each temperature of T[n_T] (erg s^-1 molecule^-1
 * sr^-1).  Transitions with nu <= 0 are discarded, as everywhere.  The sum runs
 * over the lines as they come (no grouping), in Neumaier summation; OpenMP over
 * temperatures. */
int or_cooling(int64_t nl, const int32_t* up, const int32_t* lo, const float* A, int64_t ns,
               const double* E, const double* g, int32_t n_T, const double* T, double* W,
               double* Q_out) {
  const double c2 = or_c2();
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t j = 0; j < n_T; ++j) {
    or_sum q = {0, 0}, w = {0, 0};
    for (int64_t n = 0; n < ns; ++n) or_add(&q, g[n] * exp(-c2 * E[n] / T[j]));
    for (int64_t i = 0; i < nl; ++i) {
      double nu = E[up[i]] - E[lo[i]];
      if (!(nu > 0.0)) continue;
      or_add(&w, (double)A[i] * OR_H * OR_C * nu * g[up[i]] * exp(-c2 * E[up[i]] / T[j]));
    }
    double Q = or_total(&q);
    W[j] = or_total(&w) / (4.0 * OR_PI * Q);
    if (Q_out) Q_out[j] = Q;
  }
  return 0;
}

/* ---- Line widths (half widths at half maximum) -------------------------- */
/* Doppler: alpha = (nu / c) sqrt(2 k_B T ln2 / (M amu)); fixed Gaussian: alpha = hwhm.
 * Lorentz (pressure): gamma = gamma_ref (T_ref / T)^n (P / P_ref).
 * In non-LTE runs T is the rotational (kinetic) temperature.
 * Predissociation (lifetime) broadening, section "Spectral synthesis": an
 * upper state of lifetime tau (s) has the natural Lorentzian HWHM
 * 1 / (4 pi c tau) in cm^-1 (energy width hbar / tau, FWHM 1/(2 pi c tau));
 * Lorentzians convolve by adding their widths, so it adds to gamma.  Only a
 * finite tau > 0 broadens (a stable state, tau = inf, adds nothing).  tau and
 * up may be NULL. */
int or_widths(int64_t nl, const double* nu, const float* gref, const float* nexp,
              double gref_scalar, double nexp_scalar, int profile, double T, double P,
              double mass_amu, double T_ref, double P_ref, double hwhm_fixed,
              const double* tau, const int32_t* up, double* alpha, double* gamma) {
  const double dfac = sqrt(2.0 * OR_KB * T * OR_LN2 / (mass_amu * OR_AMU));
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nl; ++i) {
    alpha[i] = (or_base(profile) == OR_GAUSSIAN) ? hwhm_fixed : (nu[i] / OR_C) * dfac;
    double gr = gref ? (double)gref[i] : gref_scalar;
    double ne = nexp ? (double)nexp[i] : nexp_scalar;
    gamma[i] = gr * pow(T_ref / T, ne) * (P / P_ref);
    if (tau && up) {
      double t = tau[up[i]];
      if (t > 0.0 && isfinite(t)) gamma[i] += 1.0 / (4.0 * OR_PI * OR_C * t);
    }
  }
  return 0;
}

/* ---- Faddeeva function w(z) = exp(-z^2) erfc(-i z), Im z >= 0 ------------ */
/* Modified trapezoidal rule with pole correction (Matta & Reichel 1971;
 * Hunter & Regan 1972; error analysis: Al Azah & Chandler-Wilde 2021).
 * From w(z) = (i/pi) int exp(-t^2) / (z - t) dt, the trapezoidal rule with
 * step h on nodes t_n = n h (or (n + 1/2) h) gives
 *   T(z) = (i h / pi) sum_n exp(-t_n^2) / (z - t_n),
 * and the pole of the integrand at t = z adds, for 0 <= Im z < pi / h,
 *   2 exp(-z^2) / (1 - exp(-2 pi i z / h))    (nodes n h)
 *   2 exp(-z^2) / (1 + exp(-2 pi i z / h))    (nodes (n + 1/2) h).
 * The remaining error is of order exp(-pi^2 / h^2) (~1e-27 at h = 0.4).  The
 * node set whose nodes lie farthest from Re z is used, so no term is near its
 * pole.  Real and imaginary parts of the sum are written out in real
 * arithmetic: Re = (h/pi) sum e^{-t^2} y / ((x-t)^2 + y^2) has positive terms,
 * which keeps Re w accurate where Re w << |w|.  Symmetry: w(-x+iy) = conj(w(x+iy)).
 * Also returned: w'(z) and G(z) = d(z w)/dz = w + z w', each the exact
 * derivative of the same approximation, so the adjoint needs no difference of
 * nearly equal terms. */
#define OR_MR_H 0.4
#define OR_MR_N 23 /* nodes |n| <= 23: exp(-t^2) < 1e-33 beyond */
static double or_mr_e0[2 * OR_MR_N + 1], or_mr_e1[2 * OR_MR_N + 2];
static int or_mr_ready = 0;
static void or_mr_init(void) {
  if (or_mr_ready) return;
#pragma omp critical(or_mr_init)
  {
    if (!or_mr_ready) {
      for (int n = -OR_MR_N; n <= OR_MR_N; ++n) {
        double t = n * OR_MR_H;
        or_mr_e0[n + OR_MR_N] = exp(-t * t);
      }
      for (int n = -OR_MR_N - 1; n <= OR_MR_N; ++n) {
        double t = (n + 0.5) * OR_MR_H;
        or_mr_e1[n + OR_MR_N + 1] = exp(-t * t);
      }
      __atomic_store_n(&or_mr_ready, 1, __ATOMIC_RELEASE);
    }
  }
}

/* want: bit 0 -> w, bit 1 -> w', bit 2 -> G = w + z w' */
static void or_faddeeva_full(double x, double y, int want, double complex* w,
                             double complex* wp, double complex* G) {
  const double h = OR_MR_H;
  const int neg = x < 0.0;
  const double ax = fabs(x);
  const double fr = ax / h - floor(ax / h);
  const int shifted = !(fr >= 0.25 && fr < 0.75);
  const int nlo = shifted ? -OR_MR_N - 1 : -OR_MR_N;
  const double* ew = shifted ? or_mr_e1 : or_mr_e0;
  double sre = 0.0, sim = 0.0;             /* sum e^{-t^2} / (z - t) */
  for (int n = nlo; n <= OR_MR_N; ++n) {
    double t = (shifted ? (n + 0.5) : (double)n) * h;
    double e = ew[n - nlo];
    double dx = ax - t;
    double den = dx * dx + y * y;
    /* 1/(z - t) = (dx - i y) / den */
    sre += e * dx / den;
    sim += -e * y / den;
  }
  /* Derivative sums, with the nodes +t and -t taken together (both node sets
   * are symmetric), so that no two terms cancel:
   *   1/(z-t)^2 + 1/(z+t)^2 = 2 (z^2 + t^2) / (z^2 - t^2)^2
   *   t/(z-t)^2 - t/(z+t)^2 = 4 z t^2 / (z^2 - t^2)^2                      */
  double complex sd = 0.0, sg = 0.0;       /* sum e/(z-t)^2, sum e t/(z-t)^2 */
  if (want & 6) {
    double complex z = ax + I * y, Z = z * z;
    if (!shifted) sd += or_mr_e0[OR_MR_N] / Z; /* t = 0 */
    for (int n = shifted ? 0 : 1; n <= OR_MR_N; ++n) {
      double t = (shifted ? (n + 0.5) : (double)n) * h;
      double e = ew[n - nlo];
      double complex q = Z - t * t;
      double complex q2 = q * q;
      sd += e * 2.0 * (Z + t * t) / q2;
      sg += e * 4.0 * z * (t * t) / q2;
    }
  }
  const double c = h / OR_PI;
  /* (i h / pi) * (sre + i sim) */
  double complex wv = c * (-sim) + I * (c * sre);
  double complex wpv = -I * c * sd;   /* d/dz of (i h/pi) sum e/(z-t) */
  double complex Gv = -I * c * sg;    /* d/dz of (i h/pi) sum e z/(z-t) */
  if (y < OR_PI / h) {
    double complex z = ax + I * y;
    double complex ez = cexp(-z * z);
    double complex E = cexp(-2.0 * OR_PI * I * z / h);
    double s = shifted ? -1.0 : 1.0;   /* denominator 1 - s E */
    double complex dn = 1.0 - s * E;
    double complex C = 2.0 * ez / dn;
    wv += C;
    if (want & 6) {
      double complex Cp = -2.0 * z * C - (2.0 * OR_PI * I / h) * 2.0 * ez * s * E / (dn * dn);
      wpv += Cp;
      Gv += C + z * Cp;
    }
  }
  if (neg) { /* w(-x+iy) = conj w(x+iy); w'(-x+iy) = -conj w'(x+iy); G likewise conj */
    wv = conj(wv);
    wpv = -conj(wpv);
    Gv = conj(Gv);
  }
  if (w) *w = wv;
  if (wp) *wp = wpv;
  if (G) *G = Gv;
}

void or_faddeeva(double x, double y, double* re, double* im) {
  or_mr_init();
  double complex w;
  or_faddeeva_full(x, y, 1, &w, NULL, NULL);
  *re = creal(w);
  *im = cimag(w);
}

/* w'(z) and G(z) = w + z w' as (re, im) pairs. */
void or_faddeeva_deriv(double x, double y, double* wp_re, double* wp_im, double* g_re,
                       double* g_im) {
  or_mr_init();
  double complex wp, G;
  or_faddeeva_full(x, y, 6, NULL, &wp, &G);
  *wp_re = creal(wp); *wp_im = cimag(wp);
  *g_re = creal(G); *g_im = cimag(G);
}

/* ---- Unit-area line profiles (Table tab:profile; normalisation of Eq. xsec) */
/* Gaussian with HWHM alpha: sqrt(ln2/pi)/alpha exp(-ln2 d^2/alpha^2).
 * Lorentzian with HWHM gamma: gamma / (pi (d^2 + gamma^2)).
 * Voigt (scipy.special.voigt_profile convention): Re w(z) / (sg sqrt(2 pi)),
 *   z = (d + i gamma) / (sg sqrt 2), sg = alpha / sqrt(2 ln 2). */
/* Pseudo-Voigt: eta L(d; f) + (1 - eta) G(d; f), a unit-area Lorentzian and
 * Gaussian of the same FWHM f, from the Gaussian and Lorentzian FWHM
 * fG = 2 alpha, fL = 2 gamma.
 *   Thompson, Cox & Hastings (1987): f^5 = fG^5 + 2.69269 fG^4 fL
 *     + 2.42843 fG^3 fL^2 + 4.47163 fG^2 fL^3 + 0.07842 fG fL^4 + fL^5;
 *   Olivero & Longbothum (1977): f = 0.5346 fL + sqrt(0.2166 fL^2 + fG^2);
 * both with eta = 1.36603 r - 0.47719 r^2 + 0.11116 r^3, r = fL / f. */
static double or_pseudo_voigt(int profile, double d, double alpha, double gamma) {
  const double fG = 2.0 * alpha, fL = 2.0 * gamma;
  double f;
  if (profile == OR_PV_THOMPSON) {
    double s = pow(fG, 5) + 2.69269 * pow(fG, 4) * fL + 2.42843 * pow(fG, 3) * fL * fL +
               4.47163 * fG * fG * pow(fL, 3) + 0.07842 * fG * pow(fL, 4) + pow(fL, 5);
    f = pow(s, 0.2);
  } else {
    f = 0.5346 * fL + sqrt(0.2166 * fL * fL + fG * fG);
  }
  const double r = fL / f;
  const double eta = 1.36603 * r - 0.47719 * r * r + 0.11116 * r * r * r;
  const double L = 2.0 / (OR_PI * f) / (1.0 + 4.0 * d * d / (f * f));
  const double G = 2.0 * sqrt(OR_LN2 / OR_PI) / f * exp(-4.0 * OR_LN2 * d * d / (f * f));
  return eta * L + (1.0 - eta) * G;
}

static double or_profile1(int profile, double d, double alpha, double gamma) {
  if (profile >= OR_PV_THOMPSON) return or_pseudo_voigt(profile, d, alpha, gamma);
  if (profile == OR_DOPPLER || profile == OR_GAUSSIAN)
    return sqrt(OR_LN2 / OR_PI) / alpha * exp(-OR_LN2 * d * d / (alpha * alpha));
  if (profile == OR_LORENTZ) return gamma / (OR_PI * (d * d + gamma * gamma));
  double sg = alpha / sqrt(2.0 * OR_LN2);
  double s2 = sg * sqrt(2.0);
  double complex w;
  or_faddeeva_full(d / s2, gamma / s2, 1, &w, NULL, NULL);
  return creal(w) / (sg * sqrt(2.0 * OR_PI));
}

double or_profile(int profile, double d, double alpha, double gamma) {
  or_mr_init();
  return or_profile1(profile, d, alpha, gamma);
}

/* ---- Bin-integrated profiles --------------------------------------------- */
/* fbar = (1/dnu) int_{d - dnu/2}^{d + dnu/2} f(s) ds, d = nu_k - nu_i.
 * Gaussian (HWHM alpha), with X = sqrt(ln 2) / alpha:
 *   fbar = (erf(X d_b) - erf(X d_a)) / (2 dnu),
 *   taken as erfc(X d_a) - erfc(X d_b) when both edges lie right of the line
 *   centre (and mirrored on the left), so the far wing is no difference of
 *   numbers near 1.
 * Lorentzian (HWHM gamma):
 *   fbar = (atan(d_b/gamma) - atan(d_a/gamma)) / (pi dnu)
 *        = atan2(gamma dnu, gamma^2 + d_a d_b) / (pi dnu),
 *   the difference of the two angles written as the argument of
 *   (gamma + i d_b)(gamma - i d_a), exact and free of cancellation.
 * Voigt: with z = (s + i gamma)/(sg sqrt 2), ds = sg sqrt 2 dx,
 *   fbar = (1 / (dnu sqrt pi)) int_{x_a}^{x_b} Re w(x + i y) dx,
 *   integrated by composite 16-point Gauss-Legendre over pieces no longer than
 *   a quarter of max(1, |z|) on the piece (w is entire; its scale of
 *   variation near a point z is about max(1, |z|)), so each piece's rule
 *   converges far below the FP64 rounding level. */
#define OR_GL_N 16
static double or_gl_x[OR_GL_N], or_gl_w[OR_GL_N];
static int or_gl_ready = 0;
/* Nodes and weights of the Gauss-Legendre rule on [-1, 1]: the roots of P_16
 * by Newton's method from the Chebyshev-like start cos(pi (i + 3/4)/(n + 1/2)),
 * P_n by the three-term recurrence (n P_n = (2n-1) x P_{n-1} - (n-1) P_{n-2}),
 * w_i = 2 / ((1 - x_i^2) P_n'(x_i)^2). */
static void or_gl_init(void) {
  if (or_gl_ready) return;
#pragma omp critical(or_gl_init)
  {
    if (!or_gl_ready) {
      const int n = OR_GL_N;
      for (int i = 0; i < n; ++i) {
        double x = cos(OR_PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
          double p0 = 1.0, p1 = x;
          for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
          }
          dp = n * (x * p1 - p0) / (x * x - 1.0);
          double dx = p1 / dp;
          x -= dx;
          if (fabs(dx) < 1e-17) break;
        }
        {
          double p0 = 1.0, p1 = x;
          for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
          }
          dp = n * (x * p1 - p0) / (x * x - 1.0);
        }
        or_gl_x[i] = x;
        or_gl_w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
      }
      __atomic_store_n(&or_gl_ready, 1, __ATOMIC_RELEASE);
    }
  }
}

void or_gl_rule(double* x, double* w) {
  or_gl_init();
  memcpy(x, or_gl_x, sizeof(or_gl_x));
  memcpy(w, or_gl_w, sizeof(or_gl_w));
}

/* int_a^b Re w(x + i y) dx, accumulated into acc piece by piece. */
static void or_re_w_integral(double a, double b, double y, or_sum* acc) {
  double xn = (a <= 0.0 && b >= 0.0) ? 0.0 : fmin(fabs(a), fabs(b));
  double scale = fmax(1.0, sqrt(xn * xn + y * y));
  if (b - a > 0.25 * scale) {
    double mid = (a < 0.0 && b > 0.0) ? 0.0 : 0.5 * (a + b);
    or_re_w_integral(a, mid, y, acc);
    or_re_w_integral(mid, b, y, acc);
    return;
  }
  double c = 0.5 * (a + b), h = 0.5 * (b - a);
  or_sum s = {0, 0};
  for (int i = 0; i < OR_GL_N; ++i) {
    double complex w;
    or_faddeeva_full(c + h * or_gl_x[i], y, 1, &w, NULL, NULL);
    or_add(&s, or_gl_w[i] * creal(w));
  }
  or_add(acc, h * or_total(&s));
}

static double or_binned1(int profile, double d, double dnu, double alpha, double gamma) {
  const double da = d - 0.5 * dnu, db = d + 0.5 * dnu;
  const int base = or_base(profile);
  if (base == OR_DOPPLER || base == OR_GAUSSIAN) {
    const double X = sqrt(OR_LN2) / alpha;
    const double xa = X * da, xb = X * db;
    double v;
    if (xa >= 0.0) v = erfc(xa) - erfc(xb);
    else if (xb <= 0.0) v = erfc(-xb) - erfc(-xa);
    else v = erf(xb) - erf(xa);
    return v / (2.0 * dnu);
  }
  if (base == OR_LORENTZ) return atan2(gamma * dnu, gamma * gamma + da * db) / (OR_PI * dnu);
  const double s2 = alpha / sqrt(2.0 * OR_LN2) * sqrt(2.0);
  or_sum acc = {0, 0};
  or_re_w_integral(da / s2, db / s2, gamma / s2, &acc);
  return or_total(&acc) / (dnu * sqrt(OR_PI));
}

double or_binned(int profile, double d, double dnu, double alpha, double gamma) {
  or_mr_init();
  or_gl_init();
  return or_binned1(profile, d, dnu, alpha, gamma);
}

/* Profile value and its derivatives with respect to the Gaussian standard
 * deviation sg = alpha / sqrt(2 ln 2) and to gamma:
 *   Gaussian: dG/dsg = G (d^2/sg^2 - 1) / sg;   dG/dgamma = 0
 *   Lorentz:  dL/dsg = 0;   dL/dgamma = (d^2 - gamma^2) / (pi (d^2 + gamma^2)^2)
 *   Voigt:    dV/dgamma = -Im w'(z) / (2 sqrt(pi) sg^2)
 *             dV/dsg    = -Re G(z) / (sg^2 sqrt(2 pi)),  G = w + z w' */
static void or_profile_grad(int profile, double d, double alpha, double gamma, double* f,
                            double* dsg, double* dgam) {
  double sg = alpha / sqrt(2.0 * OR_LN2);
  if (profile == OR_DOPPLER || profile == OR_GAUSSIAN) {
    double v = sqrt(OR_LN2 / OR_PI) / alpha * exp(-OR_LN2 * d * d / (alpha * alpha));
    *f = v;
    *dsg = v * (d * d / (sg * sg) - 1.0) / sg;
    *dgam = 0.0;
  } else if (profile == OR_LORENTZ) {
    double q = d * d + gamma * gamma;
    *f = gamma / (OR_PI * q);
    *dsg = 0.0;
    *dgam = (d * d - gamma * gamma) / (OR_PI * q * q);
  } else {
    double s2 = sg * sqrt(2.0);
    double complex w, wp, G;
    or_faddeeva_full(d / s2, gamma / s2, 7, &w, &wp, &G);
    *f = creal(w) / (sg * sqrt(2.0 * OR_PI));
    *dgam = -cimag(wp) / (2.0 * sqrt(OR_PI) * sg * sg);
    *dsg = -creal(G) / (sg * sg * sqrt(2.0 * OR_PI));
  }
}

/* ---- Grid and cut-off window -------------------------------------------- */
/* Grid points nu_k = nu0 + k dnu (k = 0..n_bins-1).  Bin k receives line i iff
 * |nu_k - nu_i| <= cut, with nu_k and the difference rounded as written. */
static double or_nu_k(double nu0, double dnu, int64_t k) { return nu0 + (double)k * dnu; }
static int or_in_window(double nuk, double nui, double cut) { return fabs(nuk - nui) <= cut; }

/* First and last bin index of line i's window clipped to the grid; returns 0
 * when the window misses the grid.  The closed-form bounds, widened by two
 * bins, are tightened with the exact predicate (the window is contiguous,
 * because nu_k and the rounded difference are monotone in k). */
static int or_window(double nui, double cut, double nu0, double dnu, int64_t nb, int64_t* klo,
                     int64_t* khi) {
  double lo = ceil((nui - cut - nu0) / dnu) - 2.0, hi = floor((nui + cut - nu0) / dnu) + 2.0;
  if (hi < 0.0 || lo > (double)(nb - 1)) return 0;
  int64_t a = lo < 0.0 ? 0 : (int64_t)lo;
  int64_t b = hi > (double)(nb - 1) ? nb - 1 : (int64_t)hi;
  while (a <= b && !or_in_window(or_nu_k(nu0, dnu, a), nui, cut)) ++a;
  while (b >= a && !or_in_window(or_nu_k(nu0, dnu, b), nui, cut)) --b;
  if (a > b) return 0;
  *klo = a;
  *khi = b;
  return 1;
}

/* Per-line window sizes on the grid (0 if the window misses it, or nu <= 0). */
int64_t or_window_counts(int64_t nl, const double* nu, double cut, double nu0, double dnu,
                         int64_t nb, int64_t* counts) {
  int64_t total = 0;
#pragma omp parallel for schedule(static) reduction(+ : total)
  for (int64_t i = 0; i < nl; ++i) {
    int64_t a, b, c = 0;
    if (nu[i] > 0.0 && or_window(nu[i], cut, nu0, dnu, nb, &a, &b)) c = b - a + 1;
    if (counts) counts[i] = c;
    total += c;
  }
  return total;
}

/* ---- Cross section ------------------------------------------------------ */
typedef struct { double nu; int64_t i; } or_key;
static int or_key_cmp(const void* a, const void* b) {
  const or_key* p = (const or_key*)a;
  const or_key* q = (const or_key*)b;
  if (p->nu < q->nu) return -1;
  if (p->nu > q->nu) return 1;
  return (p->i > q->i) - (p->i < q->i);
}

/* sigma_k = sum_i S_i f_i(nu_k - nu_i) over lines with nu_i > 0 and
 * |nu_k - nu_i| <= cut (Eq. xsec, cut-off rule), at the requested bins
 * (binned profiles: f_i is the bin mean, and the cut-off still tests the bin
 * centre nu_k)
 * (bins == NULL: all n_bins).  Lines are sorted by nu (library sort) so each
 * bin's candidates are found by binary search; each candidate is then tested
 * with the exact predicate.  Bins are independent: OpenMP over bins. */
int or_sigma(int64_t nl, const double* nu, const double* S, const double* alpha,
             const double* gamma, int profile, double nu0, double dnu, int64_t n_bins,
             double cut, int64_t n_out, const int64_t* bins, double* out) {
  or_mr_init();
  or_gl_init();
  or_key* keys = (or_key*)malloc(sizeof(or_key) * (size_t)(nl > 0 ? nl : 1));
  if (!keys) return -2;
  int64_t m = 0;
  for (int64_t i = 0; i < nl; ++i)
    if (nu[i] > 0.0) { keys[m].nu = nu[i]; keys[m].i = i; ++m; }
  qsort(keys, (size_t)m, sizeof(or_key), or_key_cmp);
  const int64_t nq = bins ? n_out : n_bins;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t q = 0; q < nq; ++q) {
    int64_t k = bins ? bins[q] : q;
    double nuk = or_nu_k(nu0, dnu, k);
    double slack = 1e-9 * (fabs(nuk) + cut + 1.0);
    /* first sorted line with nu >= nuk - cut - slack */
    int64_t lo = 0, hi = m;
    while (lo < hi) {
      int64_t mid = lo + (hi - lo) / 2;
      if (keys[mid].nu < nuk - cut - slack) lo = mid + 1; else hi = mid;
    }
    or_sum acc = {0, 0};
    for (int64_t j = lo; j < m && keys[j].nu <= nuk + cut + slack; ++j) {
      int64_t i = keys[j].i;
      if (!or_in_window(nuk, nu[i], cut)) continue;
      double d = nuk - nu[i];
      double f = (profile >= 4 && profile < 8) ? or_binned1(profile, d, dnu, alpha[i], gamma[i])
                                               : or_profile1(profile, d, alpha[i], gamma[i]);
      or_add(&acc, S[i] * f);
    }
    out[q] = or_total(&acc);
  }
  free(keys);
  return 0;
}

/* ---- Adjoint sums -------------------------------------------------------- */
/* For each line i, over its window W_i on the grid:
 *   A_i = sum_k g_k f_ik,  B_i = sum_k g_k df/dsg,  C_i = sum_k g_k df/dgamma
 * where g_k = dL/dsigma_k.  With these, for sigma_k = sum_i S_i f_ik:
 *   dL/dS_i = A_i, and the chain rule through sg_i(T) and gamma_i(T, P) gives
 *   the condition and per-line gradients (assembled by the caller). */
int or_adjoint_sums(int64_t nl, const double* nu, const double* alpha, const double* gamma,
                    int profile, double nu0, double dnu, int64_t n_bins, double cut,
                    const double* g, double* A, double* B, double* C) {
  or_mr_init();
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t i = 0; i < nl; ++i) {
    or_sum a = {0, 0}, b = {0, 0}, c = {0, 0};
    int64_t klo, khi;
    if (nu[i] > 0.0 && or_window(nu[i], cut, nu0, dnu, n_bins, &klo, &khi)) {
      for (int64_t k = klo; k <= khi; ++k) {
        double nuk = or_nu_k(nu0, dnu, k);
        double f, dsg, dgam;
        or_profile_grad(profile, nuk - nu[i], alpha[i], gamma[i], &f, &dsg, &dgam);
        or_add(&a, g[k] * f);
        or_add(&b, g[k] * dsg);
        or_add(&c, g[k] * dgam);
      }
    }
    A[i] = or_total(&a);
    B[i] = or_total(&b);
    C[i] = or_total(&c);
  }
  return 0;
}

/* The same window sums with every term taken in absolute value,
 *   A'_i = sum_k |g_k f_ik|,  B'_i = sum_k |g_k df/dsg|,  C'_i = sum_k |g_k df/dgamma|.
 * They bound what rounding in the terms can do to the signed sums above: a
 * relative error e in every term moves A_i by at most e A'_i (likewise B, C),
 * so |A_i| <= A'_i and A'_i / |A_i| is the condition number of the sum.  The
 * tests use them for the per-element error of the adjoint's per-line
 * gradients, whose signed sums (cotangents of either sign, derivatives that
 * change sign across a profile) can cancel to any degree. */
int or_adjoint_abs_sums(int64_t nl, const double* nu, const double* alpha, const double* gamma,
                        int profile, double nu0, double dnu, int64_t n_bins, double cut,
                        const double* g, double* A, double* B, double* C) {
  or_mr_init();
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t i = 0; i < nl; ++i) {
    or_sum a = {0, 0}, b = {0, 0}, c = {0, 0};
    int64_t klo, khi;
    if (nu[i] > 0.0 && or_window(nu[i], cut, nu0, dnu, n_bins, &klo, &khi)) {
      for (int64_t k = klo; k <= khi; ++k) {
        double nuk = or_nu_k(nu0, dnu, k);
        double f, dsg, dgam;
        or_profile_grad(profile, nuk - nu[i], alpha[i], gamma[i], &f, &dsg, &dgam);
        or_add(&a, fabs(g[k] * f));
        or_add(&b, fabs(g[k] * dsg));
        or_add(&c, fabs(g[k] * dgam));
      }
    }
    A[i] = or_total(&a);
    B[i] = or_total(&b);
    C[i] = or_total(&c);
  }
  return 0;
}
