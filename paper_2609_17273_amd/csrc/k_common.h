// Device helpers shared by the kernels: grid/window arithmetic, log-domain
// line intensities, and the Faddeeva function w(z) = exp(-z^2) erfc(-iz).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "faddeeva_table.h"
#include "xsec_internal.h"

namespace xs {

// ---------------------------------------------------------------------------
// Grid and cut-off window (section "Spectral synthesis"): grid point
// nu_k = nu0 + k dnu receives line i iff |nu_k - nu_i| <= cut.  Both roundings
// are done exactly as written (no FMA contraction), so every precision of the
// path includes the same bins.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double nu_of_bin(double nu0, double dnu, int64_t k) {
#pragma clang fp contract(off)
  return nu0 + (double)k * dnu;
}

__device__ __forceinline__ bool in_window(double nuk, double nui, double cut) {
#pragma clang fp contract(off)
  return fabs(nuk - nui) <= cut;
}

// First/last bin of the window clipped to [0, nb-1]; false if empty.  The
// closed-form bounds widened by two bins are tightened by the exact predicate
// (the window is contiguous because nu_k and the rounded difference are
// monotone in k).
__device__ inline bool line_window(double nui, double cut, double nu0, double dnu, int64_t nb,
                                   int64_t& klo, int64_t& khi) {
#pragma clang fp contract(off)
  double lo = ceil((nui - cut - nu0) / dnu) - 2.0;
  double hi = floor((nui + cut - nu0) / dnu) + 2.0;
  if (!(hi >= 0.0) || !(lo <= (double)(nb - 1))) return false;
  int64_t a = lo < 0.0 ? 0 : (int64_t)lo;
  int64_t b = hi > (double)(nb - 1) ? nb - 1 : (int64_t)hi;
  while (a <= b && !in_window(nu_of_bin(nu0, dnu, a), nui, cut)) ++a;
  while (b >= a && !in_window(nu_of_bin(nu0, dnu, b), nui, cut)) --b;
  klo = a;
  khi = b;
  return a <= b;
}

// Nearest grid index of nu (the line's home bin) and the residual
// delta = nu - nu_{k_c} in [-dnu/2, dnu/2] up to rounding.
__device__ __forceinline__ int64_t home_bin(double nui, double nu0, double dnu) {
  double t = rint((nui - nu0) / dnu);
  t = fmin(fmax(t, -4.0e18), 4.0e18);
  return (int64_t)t;
}

// ---------------------------------------------------------------------------
// Line intensity in log form, ln|S| and its sign (nu > 0 assumed):
//  absorption LTE  (Eq. abs intensity lte):
//     ln(g_u A / (8 pi c nu^2)) - c2 E_l / T + ln(1 - exp(-c2 nu / T)) - ln Q
//  absorption 2T   (Eqs. nlte v, nlte ab 2T):
//     ... - c2 E_l,vib/Tv - c2 E_l,rot/Tr + ln|1 - exp(-c2 (nu_vib/Tv + nu_rot/Tr))| - ln Q
//     (negative intensity under population inversion)
//  emission LTE    (Eq. ems intensity lte):  ln(g_u h c A nu / (4 pi)) - c2 E_u / T - ln Q
//  emission 2T     (Eq. nlte em 2T):         ... - c2 E_u,vib/Tv - c2 E_u,rot/Tr - ln Q
//  absorption, custom densities (Eq. nlte ab pop density):
//     ln(g_u A / (8 pi c nu^2)) + ln n_vib(v_l) - c2 E_l,rot/Tr + ln(1 - exp(-c2 nu/Tr)) - ln Q
//  emission, custom densities (Eq. nlte em pop density):
//     ln(g_u h c A nu / (4 pi)) + ln n_vib(v_u) - c2 E_u,rot/Tr - ln Q
//     (a weight that is not > 0 gives ln S = -inf: no intensity)
// (1 - exp(-x)) is formed as -expm1(-x); a per-line log scale s adds s.
// ---------------------------------------------------------------------------
// A line is usable only if its state indices (and, for two temperatures,
// their manifold indices) are inside the caller's tables.
__device__ __forceinline__ bool line_indices_ok(const StatesView& st, int32_t u, int32_t l, int pop) {
  if ((uint32_t)u >= (uint64_t)st.n || (uint32_t)l >= (uint64_t)st.n) return false;
  if (pop != XS_LTE &&
      ((uint32_t)st.v[u] >= (uint32_t)st.n_v || (uint32_t)st.v[l] >= (uint32_t)st.n_v))
    return false;
  return true;
}

struct LineState {
  double Eu, El, gu, evu, evl;
  double nvu, nvl;  // vibronic densities of the upper and lower manifolds
};

// The part of ln|S| that no temperature enters: ln(g_u A / (8 pi c nu^2))
// (absorption) or ln(g_u h c A nu / (4 pi)) (emission).
__device__ inline double ln_line(int mode, const LineState& ls, double A, double nu) {
  if (mode == XS_ABSORPTION) return log(ls.gu * A) - log(8.0 * kPI * kC) - 2.0 * log(nu);
  return log(ls.gu * kH * kC * A * nu / (4.0 * kPI));
}

// The population (and stimulated-emission) part of ln|S| for one slot's
// temperatures, and the sign of S.
__device__ inline double ln_pop(int mode, int pop, const LineState& ls, double nu, double T, double Tv,
                                double Tr, int& sign) {
  sign = 1;
  if (mode == XS_ABSORPTION) {
    if (pop == XS_LTE) return -kC2 * ls.El / T + log(-expm1(-kC2 * nu / T));
    if (pop == XS_NLTE_DENSITY)
      return (ls.nvl > 0.0 ? log(ls.nvl) : -INFINITY) - kC2 * (ls.El - ls.evl) / Tr +
             log(-expm1(-kC2 * nu / Tr));
    const double nuv = ls.evu - ls.evl;
    const double nur = (ls.Eu - ls.evu) - (ls.El - ls.evl);
    const double x = kC2 * (nuv / Tv + nur / Tr);
    const double st = -expm1(-x);
    if (st < 0.0) sign = -1;
    return -kC2 * ls.evl / Tv - kC2 * (ls.El - ls.evl) / Tr + log(fabs(st));
  }
  if (pop == XS_LTE) return -kC2 * ls.Eu / T;
  if (pop == XS_NLTE_DENSITY) return (ls.nvu > 0.0 ? log(ls.nvu) : -INFINITY) - kC2 * (ls.Eu - ls.evu) / Tr;
  return -kC2 * ls.evu / Tv - kC2 * (ls.Eu - ls.evu) / Tr;
}

// ln|S| = ln_line + ln_pop - ln Q + s (the loops over slots take ln_line
// once per line and ln Q once per slot).
__device__ inline double ln_intensity(int mode, int pop, const LineState& ls, double A,
                                      double nu, double T, double Tv, double Tr, double lnQ,
                                      double lscale, int& sign) {
  return (ln_line(mode, ls, A, nu) + ln_pop(mode, pop, ls, nu, T, Tv, Tr, sign)) - lnQ + lscale;
}

// Order-preserving map of doubles to unsigned keys (for an atomic max).
__device__ __forceinline__ unsigned long long dbl_key(double v) {
  unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double key_dbl(unsigned long long k) {
  unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  return __longlong_as_double((long long)b);
}

// ---------------------------------------------------------------------------
// Faddeeva function.  Far region: the Gauss-Hermite rule with 2P nodes
// applied to w(z) = (i/pi) int exp(-t^2)/(z - t) dt; each node pair +-t_j
// contributes (i/pi) W_j 2z/(z^2 - tau_j), tau_j = t_j^2, so with u = x^2 and
// z^2 = u - y^2 + 2ixy,
//   Re w = (2y/pi) sum_j W_j (u + y^2 + tau_j) / ((u - y^2 - tau_j)^2 + 4 y^2 u),
// a sum of positive terms (no cancellation where Re w << |w|).  Near region
// |z| < 8 (|z| < 6 in the FP32 form): Weideman's rational approximation.
// ---------------------------------------------------------------------------
struct GH {
  static constexpr double s2[1] = XS_GH2_T;
  static constexpr double s4[2] = XS_GH4_T;
  static constexpr double s6[3] = XS_GH6_T;
  static constexpr double s8[4] = XS_GH8_T;
  static constexpr double s12[6] = XS_GH12_T;
  static constexpr double t2[1] = XS_GH2_TAU;
  static constexpr double w2[1] = XS_GH2_W;
  static constexpr double t3[1] = XS_GH3_TAU;  // three points: +-t and 0
  static constexpr double w3[1] = XS_GH3_W;
  static constexpr double w3c = XS_GH3_W0;     // weight of the node t = 0
  static constexpr double t4[2] = XS_GH4_TAU;
  static constexpr double w4[2] = XS_GH4_W;
  static constexpr double t6[3] = XS_GH6_TAU;
  static constexpr double w6[3] = XS_GH6_W;
  static constexpr double t8[4] = XS_GH8_TAU;
  static constexpr double w8[4] = XS_GH8_W;
  static constexpr double t12[6] = XS_GH12_TAU;
  static constexpr double w12[6] = XS_GH12_W;
};

template <int NP>
__device__ __forceinline__ const double* gh_tau() {
  if constexpr (NP == 1) return GH::t2;
  else if constexpr (NP == 2) return GH::t4;
  else if constexpr (NP == 3) return GH::t6;
  else if constexpr (NP == 4) return GH::t8;
  else return GH::t12;
}
template <int NP>
__device__ __forceinline__ const double* gh_node() {
  if constexpr (NP == 1) return GH::s2;
  else if constexpr (NP == 2) return GH::s4;
  else if constexpr (NP == 3) return GH::s6;
  else if constexpr (NP == 4) return GH::s8;
  else return GH::s12;
}
template <int NP>
__device__ __forceinline__ const double* gh_w() {
  if constexpr (NP == 1) return GH::w2;
  else if constexpr (NP == 2) return GH::w4;
  else if constexpr (NP == 3) return GH::w6;
  else if constexpr (NP == 4) return GH::w8;
  else return GH::w12;
}

// 1/d by the hardware FP64 reciprocal (relative error below 5e-8 on gfx950)
// and one Newton step (below 3e-15).
__device__ __forceinline__ double rcp_nr(double d) {
  const double r = __builtin_amdgcn_rcp(d);
  return fma(r, fma(-d, r, 1.0), r);
}

// sum_j W_j n_j / d_j with n_j = u + y2 + tau_j, d_j = (u - y2 - tau_j)^2 + q u,
// q = 4 y^2 (the caller multiplies by 2y/pi).  One node pair, or two pairs in
// FP64: a single division of the combined fraction.  Otherwise one reciprocal
// per pair: lanes of a row near a narrow line reach u ~ 1e18, where the
// product of the d_j would overflow (FP32: u > ~1e9; FP64 with 6 pairs:
// u > ~1e25).
template <int NP, typename R>
__device__ __forceinline__ R gh_re_sum(R u, R y2, R q) {
  const double* tau = gh_tau<NP>();
  const double* W = gh_w<NP>();
  const R qu = q * u;
  if constexpr (NP == 1 || (NP == 2 && sizeof(R) == 8)) {
    R num = (R)0, den = (R)1;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const R p = y2 + (R)tau[j];
      const R a = u - p;
      const R d = fma(a, a, qu);
      num = fma(num, d, (R)W[j] * (u + p) * den);
      den = den * d;
    }
    if constexpr (sizeof(R) == 4)
      return num * __builtin_amdgcn_rcpf(den);
    else
      return num * rcp_nr(den);
  } else {
    R sum = (R)0;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const R p = y2 + (R)tau[j];
      const R a = u - p;
      const R d = fma(a, a, qu);
      R id;
      if constexpr (sizeof(R) == 4) id = __builtin_amdgcn_rcpf(d);
      else id = rcp_nr(d);
      sum = fma((R)W[j] * (u + p), id, sum);
    }
    return sum;
  }
}

// w(z), Im z >= 0, by Weideman's rational approximation with N terms:
//   w(z) ~ 2 p(Z) q^2 + q / sqrt(pi),  q = 1/(L - iz),  Z = (L + iz) q,
// p(Z) = sum_{n=1..N} a_n Z^(n-1).  No table and no branch, valid on the whole
// half-plane: relative error (of |w|) below 5e-10 for N = 24 and 3e-14 for
// N = 40.
template <int N>
struct WM;
template <>
struct WM<24> {
  static constexpr double L = XS_WM24_L;
  static constexpr double a[24] = XS_WM24_A;
  static constexpr double b[24] = XS_WM24_B;
};
template <>
struct WM<40> {
  static constexpr double L = XS_WM40_L;
  static constexpr double a[40] = XS_WM40_A;
  static constexpr double b[40] = XS_WM40_B;
};

// p(Z) = sum_{n<N} c_n Z^n with real c_n at a complex Z: Horner's rule for
// the real quadratic Z^2 - t Z + m (t = 2 Re Z, m = |Z|^2), which Z solves
// (Knuth, TAOCP vol. 2, sec. 4.6.4):  b_k = c_k + t b_(k+1) - m b_(k+2) for
// k = N-1 .. 1, then p = b_1 Z + c_0 - m b_2.  Two FMAs per degree instead of
// the four of complex Horner; for |Z| <= 1 (every z of the upper half-plane)
// and the Weideman coefficients its rounding matches complex Horner's (both
// 1.5e-15 of |w| over |z|^2 < 64 for N = 40, against 40-digit values).
template <int N>
__device__ __forceinline__ void poly_real_at(const double (&c)[N], double Zr, double Zi, double& pr, double& pi) {
  const double t = 2.0 * Zr, mm = -fma(Zr, Zr, Zi * Zi);
  double b1 = c[N - 1], b2 = 0.0;
#pragma unroll
  for (int k = N - 2; k >= 1; --k) {
    const double b = fma(t, b1, fma(mm, b2, c[k]));
    b2 = b1;
    b1 = b;
  }
  pr = fma(b1, Zr, fma(mm, b2, c[0]));
  pi = b1 * Zi;
}

template <int N>
__device__ __forceinline__ void w_weideman(double x, double y, double& wr, double& wi) {
  constexpr double L = WM<N>::L;
  // q = 1/((L + y) - i x) = ((L + y) + i x) / D
  const double lr = L + y;
  const double iD = rcp_nr(fma(lr, lr, x * x));
  const double qr = lr * iD, qi = x * iD;
  // Z = ((L - y) + i x) q
  const double ly = L - y;
  const double Zr = fma(ly, qr, -x * qi), Zi = fma(ly, qi, x * qr);
  double pr, pi;
  poly_real_at<N>(WM<N>::a, Zr, Zi, pr, pi);
  const double q2r = fma(qr, qr, -qi * qi), q2i = 2.0 * qr * qi;
  constexpr double rsp = 0.56418958354775628695;  // 1/sqrt(pi)
  wr = fma(2.0, fma(pr, q2r, -pi * q2i), rsp * qr);
  wi = fma(2.0, fma(pr, q2i, pi * q2r), rsp * qi);
}

// Re w(x + iy) by the rational approximation, out of line (rare core chunks).
template <int N>
__device__ __noinline__ double re_w_core(double x, double y) {
  double wr, wi;
  w_weideman<N>(x, y, wr, wi);
  return wr;
}

// FP64 Re w(x + iy), y >= 0, relative accuracy ~1e-14 (bands chosen per |z|).
__device__ __noinline__ double re_w_f64(double x, double y) {
  const double u = x * x, y2 = y * y, rho = u + y2, q = 4.0 * y2;
  const double cy = y * (2.0 / kPI);
  if (rho >= 9.0e6) return cy * gh_re_sum<1>(u, y2, q);
  if (rho >= 6400.0) return cy * gh_re_sum<2>(u, y2, q);
  if (rho >= 400.0) return cy * gh_re_sum<3>(u, y2, q);
  if (rho >= 144.0) return cy * gh_re_sum<4>(u, y2, q);
  if (rho >= 64.0) return cy * gh_re_sum<6>(u, y2, q);
  double wr, wi;
  w_weideman<40>(x, y, wr, wi);
  return wr;
}

// ---------------------------------------------------------------------------
// Pseudo-Voigt (Table tab:profile): eta L(d; f) + (1 - eta) G(d; f) with a
// common FWHM f from fG = 2 alpha and fL = 2 gamma (Thompson-Cox-Hastings
// width polynomial, or Olivero-Longbothum), eta from the Thompson-Cox-Hastings
// cubic in fL / f.  In x = 2 d / f:
//   L = (2 / (pi f)) / (1 + x^2),  G = (2 sqrt(ln 2 / pi) / f) 2^(-x^2).
// ---------------------------------------------------------------------------
struct PVConst {
  double inv, cL, cG;  // x = d inv; S L = cL / (1 + x^2); S G = cG 2^(-x^2)
};
__device__ inline PVConst pv_const(int prof, double alpha, double gamma, double S) {
  const double fG = 2.0 * alpha, fL = 2.0 * gamma;
  double f;
  if (prof == XS_PV_THOMPSON) {
    const double g2 = fG * fG, l2 = fL * fL;
    const double s = g2 * g2 * fG + 2.69269 * g2 * g2 * fL + 2.42843 * g2 * fG * l2 +
                     4.47163 * g2 * l2 * fL + 0.07842 * fG * l2 * l2 + l2 * l2 * fL;
    f = pow(s, 0.2);
  } else {
    f = 0.5346 * fL + sqrt(0.2166 * fL * fL + fG * fG);
  }
  const double r = fL / f;
  const double eta = r * fma(r, fma(r, 0.11116, -0.47719), 1.36603);
  PVConst c;
  c.inv = 2.0 / f;
  c.cL = S * eta * 2.0 / (kPI * f);
  c.cG = S * (1.0 - eta) * 2.0 * sqrt(kLN2 / kPI) / f;
  return c;
}

// ---------------------------------------------------------------------------
// Bin-integrated profiles (the binned methods of Table tab:profile).  In a
// profile's own unit x the bin of a grid point is [x - hh, x + hh], hh half
// the bin width h; the kernels scale the integrals below by S / dnu and the
// profile's normalisation.
// ---------------------------------------------------------------------------
// Reciprocal: FP32 hardware (1 ulp); FP64 hardware plus one Newton step.
template <typename R>
__device__ __forceinline__ R rcp_r(R d) {
  if constexpr (sizeof(R) == 4) {
    return __builtin_amdgcn_rcpf(d);
  } else {
    const double r = __builtin_amdgcn_rcp(d);
    return fma(r, fma(-d, r, 1.0), r);
  }
}

// Largest t for which the odd series of atan to t^7 is used: its relative
// error is below t^8/9 (1.1e-9 in FP32 at 0.1, 2.8e-15 in FP64 at 0.02).
template <typename R>
__device__ __forceinline__ constexpr R atan_series_max() { return sizeof(R) == 4 ? (R)0.1 : (R)0.02; }

template <typename R>
__device__ __forceinline__ R atan_series(R t) {
  const R t2 = t * t;
  return t * fma(t2, fma(t2, fma(t2, (R)(-1.0 / 7.0), (R)0.2), (R)(-1.0 / 3.0)), (R)1);
}

// atan2(n, d) for n > 0 (an angle in (0, pi)): the series where d > 0 and
// n/d is small, the library function otherwise.
template <typename R>
__device__ __forceinline__ R angle(R n, R d) {
  if (d > (R)0 && n <= atan_series_max<R>() * d) return atan_series(n * rcp_r(d));
  return atan2(n, d);
}

// Gaussian in x = d sqrt(ln 2)/alpha: erf(x + hh) - erf(x - hh).  By symmetry
// on |x|; where both edges lie on one side of the centre it is the difference
// of the two erfc (no difference of numbers near 1).  Relative error about
// u / min(1, 2 hh) in precision u.
template <typename R>
__device__ __forceinline__ R erf_bin(R x, R hh) {
  const R ax = fabs(x), a = ax - hh, b = ax + hh;
  return a >= (R)0 ? erfc(a) - erfc(b) : erf(b) + erf(-a);
}

// Lorentzian in x = d/gamma: atan(x + hh) - atan(x - hh), as the one angle
// atan2(h, 1 + (x - hh)(x + hh)), h = 2 hh.
template <typename R>
__device__ __forceinline__ R lor_bin(R x, R hh, R h) {
  return angle<R>(h, fma(x - hh, x + hh, (R)1));
}

// Voigt, far region: the Gauss-Hermite node pair +-s (weight W) of
// w = (i/pi) int exp(-t^2)/(z - t) dt integrates over the bin to
//   (W/pi) [atan2(y h, y^2 + (x_a - s)(x_b - s)) + atan2(y h, y^2 + (x_a + s)(x_b + s))],
// x_a, b = x -+ hh: Lorentzians of width y centred on the nodes, integrated
// exactly.  Sum over NP pairs; with SERIES the caller guarantees both
// arguments positive with ratio below atan_series_max.
template <int NP, bool SERIES, typename R>
__device__ __forceinline__ R vpairs_bin(R xa, R xb, R yh, R y2) {
  const double* s = gh_node<NP>();
  const double* W = gh_w<NP>();
  R sum = (R)0;
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    const R sj = (R)s[j];
    const R dm = fma(xa - sj, xb - sj, y2), dp = fma(xa + sj, xb + sj, y2);
    R t;
    if constexpr (SERIES) t = atan_series(yh * rcp_r(dm)) + atan_series(yh * rcp_r(dp));
    else t = angle<R>(yh, dm) + angle<R>(yh, dp);
    sum = fma((R)(W[j] / kPI), t, sum);
  }
  return sum;
}

// Voigt, near region: int_{x-hh}^{x+hh} Re w(t + iy) dt from the closed-form
// antiderivative of the rational approximation (see w_weideman):
//   d/dz [Z^n / n] = 2iL Z^(n-1) q^2, d/dz [i ln(L - iz)] = q, so
//   int w dz ~ -(i/L) sum_n b_n Z^n + (i/sqrt(pi)) ln(L - iz),  b_n = a_n / n,
// whose real part between the edges is
//   (Im P(Z_b) - Im P(Z_a)) / L + atan2(h (L + y), (L + y)^2 + x_a x_b) / sqrt(pi).
// Its error is at most h times that of the approximation (absolute), so it
// serves every bin that reaches the near region, however wide.
template <int N>
__device__ __forceinline__ double w_int_im(double x, double y) {
  constexpr double L = WM<N>::L;
  const double lr = L + y;
  const double iD = rcp_nr(fma(lr, lr, x * x));
  const double qr = lr * iD, qi = x * iD;
  const double ly = L - y;
  const double Zr = fma(ly, qr, -x * qi), Zi = fma(ly, qi, x * qr);
  double pr, pi;
  poly_real_at<N>(WM<N>::b, Zr, Zi, pr, pi);
  return fma(pr, Zi, pi * Zr);  // Im(Z p)
}

template <int N>
__device__ __noinline__ double voigt_bin_core(double x, double y, double hh) {
  constexpr double L = WM<N>::L;
  constexpr double rsp = 0.56418958354775628695;  // 1/sqrt(pi)
  const double xa = x - hh, xb = x + hh, ly = L + y;
  return (w_int_im<N>(xb, y) - w_int_im<N>(xa, y)) * (1.0 / L) +
         rsp * atan2(2.0 * hh * ly, fma(ly, ly, xa * xb));
}

// FP64 bin integral of Re w, bands by the nearest point of the bin
// (|z|^2 >= 9e6, 6400, 400, 144, 64: 1, 2, 3, 4, 6 node pairs; below: the
// rational approximation with N = 40).
__device__ __noinline__ double voigt_bin_f64(double x, double y, double hh) {
  const double xn = fmax(fabs(x) - hh, 0.0), y2 = y * y, rho = fma(xn, xn, y2);
  const double xa = x - hh, xb = x + hh, yh = 2.0 * hh * y;
  if (rho >= 9.0e6) return vpairs_bin<1, false, double>(xa, xb, yh, y2);
  if (rho >= 6400.0) return vpairs_bin<2, false, double>(xa, xb, yh, y2);
  if (rho >= 400.0) return vpairs_bin<3, false, double>(xa, xb, yh, y2);
  if (rho >= 144.0) return vpairs_bin<4, false, double>(xa, xb, yh, y2);
  if (rho >= 64.0) return vpairs_bin<6, false, double>(xa, xb, yh, y2);
  return voigt_bin_core<40>(x, y, hh);
}

}  // namespace xs
