// Adjoint of the profile pass.  For sigma_k = sum_i S_i f(nu_k - nu_i; sg_i, gamma_i)
// and a cotangent g_k = dL/dsigma_k, each line needs the window sums
//   A_i = sum_k g_k f_ik,  B_i = sum_k g_k df/dsg,  C_i = sum_k g_k df/dgamma,
// recomputed here from the line's parameters (no (line, bin) pairs stored).
// Then, per line and condition (LTE; sg ~ sqrt(T), gamma = gamma_ref
// (T_ref/T)^n P/P_ref, S from Eq. abs/ems intensity lte with Q'(T)):
//   dL/ds_i         += S A                      (per-line log scale)
//   dL/dgamma_ref,i += S C (T_ref/T)^n P/P_ref
//   dL/dn_i         += S C gamma ln(T_ref/T)
//   dL/dT_c         += S [A dlnS/dT + B sg/(2T) - C n gamma/T]
//   dL/dP_c         += S C gamma / P
// Lanes own lines (a per-line reduction over bins needs no cross-lane sums);
// FP32 partial sums are flushed to FP64.  Blocks own fixed line sets and the
// per-condition scalars are reduced in a fixed order, so results are
// deterministic.
#include "k_common.h"

namespace xs {

// Voigt far region with NP Gauss-Hermite pairs: returns Re w, and
//   R1 = Re sum_j W_j (Z + tau_j)/(Z - tau_j)^2       (Im w' = -(2/pi) R1)
//   RG = (4/pi) sum_j W_j tau_j Im[z/(Z - tau_j)^2] = Re G,  G = w + z w'
// (each pair's term 2z/(Z - tau) of w gives f + z f' = -4 z tau/(Z - tau)^2),
// written without differences of nearly equal terms:
//   Re (Z+tau)/(Z-tau)^2 = A/d + 2 tau (A^2 - Zi^2)/d^2,
//   Im z/(Z-tau)^2       = y (A^2 - Zi^2 - 4 x^2 A)/d^2,
// with A = u - y^2 - tau, Zi = 2xy, d = A^2 + Zi^2.
template <int NP, typename R>
__device__ __forceinline__ void gh_adj(R x, R y, R& rew, R& r1, R& rg) {
  const double* tau = gh_tau<NP>();
  const double* W = gh_w<NP>();
  const R u = x * x, y2 = y * y, zi = (R)2 * x * y, zi2 = zi * zi;
  R sw = 0, s1 = 0, sg = 0;
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    const R t = (R)tau[j], w = (R)W[j];
    const R A = u - y2 - t;
    const R A2 = A * A;
    const R d = A2 + zi2;
    R id;
    if constexpr (sizeof(R) == 4) id = __builtin_amdgcn_rcpf(d);
    else id = rcp_nr(d);  // hardware reciprocal and one Newton step (3e-15), not a division
    const R id2 = id * id;
    sw += w * (u + y2 + t) * id;
    s1 += w * (A * id + (R)2 * t * (A2 - zi2) * id2);
    sg += w * t * (A2 - zi2 - (R)4 * u * A) * id2;
  }
  rew = (R)(2.0 / kPI) * y * sw;
  r1 = s1;
  rg = (R)(4.0 / kPI) * y * sg;
}

// f, df/dsg, df/dgamma of the unit-area profile at x (its own scaling per
// profile, see below), for one lane.
template <typename R, int PROF>
__device__ __forceinline__ void prof_grad(R x, R y, double sgm, double gam, int band, R& f,
                                          R& fs, R& fg) {
  if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN) {
    // x = d / alpha; f = sqrt(ln2/pi)/alpha 2^{-x^2}; df/dsg = f (2 ln2 x^2 - 1)/sg
    const R e = (sizeof(R) == 4) ? (R)__builtin_amdgcn_exp2f(-(float)(x * x)) : (R)exp2(-(double)(x * x));
    f = e;
    fs = e * ((R)(2.0 * kLN2) * x * x - (R)1);
    fg = 0;
  } else if (PROF == XS_LORENTZ) {
    // x = d / gamma; f = 1/(pi gamma (1 + x^2)); df/dgamma = (x^2 - 1)/(pi gamma^2 (1+x^2)^2)
    const R q = (R)1 + x * x;
    R iq;
    if constexpr (sizeof(R) == 4) iq = __builtin_amdgcn_rcpf(q);
    else iq = rcp_nr(q);
    f = iq;
    fs = 0;
    fg = (x * x - (R)1) * iq * iq;
  } else {
    // x, y: z = (d + i gamma)/(sg sqrt 2).  Returned: Re w, Im w' and Re G
    // (scaled to df/dgamma, df/dsg by the caller).
    R rew, r1, rg;
    switch (band) {
      case 1: gh_adj<1, R>(x, y, rew, r1, rg); f = rew; fg = (R)(-2.0 / kPI) * r1; fs = rg; return;
      case 2: gh_adj<2, R>(x, y, rew, r1, rg); f = rew; fg = (R)(-2.0 / kPI) * r1; fs = rg; return;
      case 3: gh_adj<3, R>(x, y, rew, r1, rg); f = rew; fg = (R)(-2.0 / kPI) * r1; fs = rg; return;
      case 4: gh_adj<4, R>(x, y, rew, r1, rg); f = rew; fg = (R)(-2.0 / kPI) * r1; fs = rg; return;
      case 6: gh_adj<6, R>(x, y, rew, r1, rg); f = rew; fg = (R)(-2.0 / kPI) * r1; fs = rg; return;
      default: break;
    }
    const R rho = x * x + y * y;
    if (rho >= (R)64) {
      if constexpr (sizeof(R) == 4) gh_adj<2, R>(x, y, rew, r1, rg);
      else gh_adj<6, R>(x, y, rew, r1, rg);
      f = rew;
      fg = (R)(-2.0 / kPI) * r1;
      fs = rg;
      return;
    }
    // near region: w by the rational approximation, w' = -2 z w + 2i/sqrt(pi)
    double wr, wi;
    if constexpr (sizeof(R) == 4) w_weideman<24>((double)x, (double)y, wr, wi);
    else w_weideman<40>((double)x, (double)y, wr, wi);
    const double xd = (double)x, yd = (double)y;
    const double dr = -2.0 * (xd * wr - yd * wi);
    const double di = -2.0 * (xd * wi + yd * wr) + 2.0 / sqrt(kPI);
    f = (R)wr;
    fg = (R)di;                                           // Im w'
    fs = (R)(wr + ((double)x * dr - (double)y * di));     // Re G = Re w + Re(z w')
  }
}

struct AdjArgs {
  ModelDev m;
  const CondDev* cond;
  const double* Q;
  const double* dQ;
  const double* sb;
  const int32_t* off;
  const double* rnu;
  const float* rgref;
  const float* rnexp;
  const double* rgpre;
  const int32_t* ridx;
  const double* rEs;
  const void* rS;
  int64_t max_lines;
  const double* g;
  const unsigned long long* gmax;  // [n_cond] bits of max_k |g_k| per condition
  double* dgref;
  double* dnexp;
  double* dls;
  double* part;   // [n_cond][2][gridDim.x]
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ float arcp(float d) { return __builtin_amdgcn_rcpf(d); }
// The hardware FP64 reciprocal has a relative error below 5e-8 on gfx950
// (measured over 1e6 arguments spanning 1e-30..1e30); one Newton step
// squares it, to below 3e-15.
__device__ __forceinline__ double arcp(double d) {
  const double r = __builtin_amdgcn_rcp(d);
  return fma(r, fma(-d, r, 1.0), r);
}

// One Gauss-Hermite node pair (tau = t^2, weight W) of the far-region form
//   Re w = y sum_j K_j (u + p_j)/d_j,  d_j = u (u + q_j) + p_j^2,
//   p_j = y^2 + tau_j,  q_j = 2 y^2 - 2 tau_j,  K_j = 2 W_j / pi,  u = x^2,
// and its derivatives, with e = (u + p)/d:
//   dRe w/dy  = sum_j K_j [e + 2 y^2 / d - 4 y^2 e^2]
//   x dRe w/dx = 2 y sum_j K_j (u/d) [(p^2 - p q)/d - (u/d)(u + 2 p)]
//              = 2 y sum_j K_j (u/d) [4 tau_j (p - u)/d - 1]
// (the last form from d = u^2 + q u + p^2 and 2p - q = 4 tau).  The fast
// loops accumulate g e, g / d and g e^2 separately and form dRe w/dy from
// them once per block.  Every product is formed from ratios of size <= 1/u,
// so FP32 neither overflows nor underflows for |x|, y < 1e9.
template <typename R>
struct PairD {
  R q, p2, p, k1, k2, K;  // k1 = 4 tau p, k2 = -4 tau
};
template <typename R>
__device__ __forceinline__ PairD<R> pair_d(double y, double tau, double W) {
  const double y2 = y * y, p = y2 + tau, q = 2.0 * y2 - 2.0 * tau;
  PairD<R> r;
  r.q = (R)q;
  r.p2 = (R)(p * p);
  r.p = (R)p;
  r.k1 = (R)(4.0 * tau * p);
  r.k2 = (R)(-4.0 * tau);
  r.K = (R)(2.0 * W / kPI);
  return r;
}
template <typename R>
__device__ __forceinline__ void pair_adj(const PairD<R>& P, R u, R& e, R& rd, R& t) {
  const R d = fma(u, u + P.q, P.p2);
  rd = arcp(d);
  e = (u + P.p) * rd;
  t = (u * rd) * fma(rd, fma(u, P.k2, P.k1), (R)-1);
}

// Per-lane state of one line under one condition.
template <typename R>
struct AdjLine {
  R a, nb;            // x = r a + nb, r = k - k_c
  PairD<R> P[3];      // node pairs of the far-region levels (Voigt)
  double ad, bd, y;   // FP64 copies for the general path
  int kc, rlo, rhi;   // home bin; window in r
  bool share4;        // FP64: one reciprocal may serve four points (wave-uniform)
};

// Far-region levels of the Voigt adjoint, where rho = x^2 + y^2 >= rho[l];
// inside the last level the general per-lane path picks more pairs or the
// rational approximation.  FP32: one and two node pairs.  FP64: one pair, the
// three-point rule (one pair and the node at 0), two pairs, three pairs.  The
// node at 0 with weight W_0 is the pair formula with tau = 0 and weight
// W_0 / 2 (then d = (u + y^2)^2, e = 1/(u + y^2), t = -u/d).
template <typename R>
struct Levels;
template <>
struct Levels<float> {
  static constexpr int n = 2;
  static constexpr double rho[2] = {900.0, 64.0};
};
template <>
struct Levels<double> {
  static constexpr int n = 4;
  static constexpr double rho[4] = {9.0e6, 4.5e4, 4000.0, 400.0};
};

// Voigt values for the general path, out of line (rational core and up to six
// node pairs): Re w, Re G and Im w' at (x, y) with the given band.
template <typename R>
struct Grad3 {
  R f, fs, fg;
};
template <typename R>
__device__ __noinline__ Grad3<R> voigt_grad(R x, R y, int band) {
  Grad3<R> g;
  prof_grad<R, XS_VOIGT>(x, y, 0.0, 0.0, band, g.f, g.fs, g.fg);
  return g;
}

// General per-lane evaluation at r (masked by the window): old-convention
// values Re w / Re G / Im w' (Voigt), e / e (2 ln2 u - 1) (Gaussian),
// 1/(1+u) / (u-1)/(1+u)^2 (Lorentz), accumulated in FP64.
template <typename R, int PROF>
__device__ __forceinline__ void general_eval(const AdjLine<R>& L, bool wide, int r, double gk, double& sA,
                                             double& sB, double& sC) {
  if (PROF == XS_VOIGT) {
    double f, fs, fg;
    if (sizeof(R) == 4 && wide) {
      const Grad3<double> v = voigt_grad<double>((double)r * L.ad - L.bd, L.y, 0);
      f = v.f;
      fs = v.fs;
      fg = v.fg;
    } else {
      const R x = fma((R)r, L.a, L.nb);
      const R y = (R)L.y;
      const R rho = x * x + y * y;
      int band;
      if (sizeof(R) == 4) {
        band = rho >= (R)(900.0 * 1.001) ? 1 : rho >= (R)(64.0 * 1.001) ? 2 : rho >= (R)(36.0 * 1.001) ? 3 : 0;
        // when a lane of the wave needs the rational approximation, the lanes
        // of the three-pair band (rho < 64) take it too, so the wave does not
        // run both; there w and w' = -2zw + 2i/sqrt(pi) keep absolute errors
        // below 5e-9, as in the core (further out, the cancellation in w'
        // grows with |z|^2, so the two-pair band keeps its own formula)
        const bool core_in_wave = __ballot(band == 0) != 0;  // every active lane votes
        if (band == 3 && core_in_wave) band = 0;
      } else band = rho >= (R)(9.0e6 * 1.001) ? 1 : rho >= (R)(6400.0 * 1.001) ? 2 : rho >= (R)(400.0 * 1.001) ? 3
                : rho >= (R)(144.0 * 1.001) ? 4 : rho >= (R)(64.0 * 1.001) ? 6 : 0;
      const Grad3<R> v = voigt_grad<R>(x, y, band);
      f = (double)v.f;
      fs = (double)v.fs;
      fg = (double)v.fg;
    }
    sA = fma(gk, f, sA);
    sB = fma(gk, fs, sB);
    sC = fma(gk, fg, sC);
  } else {
    const R x = fma((R)r, L.a, L.nb);
    R f, fs, fg;
    prof_grad<R, PROF>(x, (R)0, 0.0, 0.0, 1, f, fs, fg);
    sA = fma(gk, (double)f, sA);
    sB = fma(gk, (double)fs, sB);
    sC = fma(gk, (double)fg, sC);
  }
}

// Fast loop over r in [r0, r1], every lane inside its window and (Voigt) in
// the far region of level NP-1.  FP32 partial sums are flushed to FP64 every
// kFlush steps.
constexpr int kFlush = 256;

// Where a lane reads its cotangent g_k: straight from memory, or -- when the
// wave's home bins lie within kFlush of each other -- from the wave's LDS
// slice, refilled with one coalesced pass per block of kFlush steps.
template <typename R>
struct GSrc {
  const double* gc;  // g of this condition
  double gs;         // power-of-two scale applied to g (FP32 form: max |g gs| in [1/2, 1))
  int64_t nb;        // grid points
  int kcmin;         // smallest home bin of the wave's active lanes
  bool lds;
  R* buf;            // [2 kFlush] LDS slice of the wave
};

// SY, the block-summed form of a level (every line of the wave with y^2 at
// most half the level's rho bound): in the shifted variable s = u + h,
// h = y^2 - tau, a node pair has d = s^2 + c, c = 4 y^2 tau, and
// u + p = s + m, m = 2 tau, p - u = 2 y^2 - s.  Every sum the block needs is
// then, pair by pair, a combination of four sums
//   S0 = sum g/d,  S1 = sum g s/d,  S2 = sum g/d^2,  S3 = sum g s/d^2
// (with s^2/d^2 = 1/d - c/d^2):
//   sum g e   = S1 + m S0,      sum g e^2 = (S0 - c S2) + 2 m S3 + m^2 S2,
//   sum g (u/d)[4 tau (p - u)/d - 1]
//             = 4 tau [-(S0 - c S2) + (2 y^2 + h) S3 - 2 y^2 h S2] - (S1 - h S0),
// formed once per block in FP64 and weighted by K; a point costs, per pair,
// s, d, 1/d, g/d, g/d^2 and four sums.  C0: the second pair is the node at 0
// (tau = 0: h = y^2, c = m = 0, s = u + y^2 = v and d = v^2), for which only
// S0 = sum g/v^2 and S1 = sum g/v enter: a point costs v, 1/v, g/v and two
// sums.  The only difference of like terms is
// S1 - h S0 = sum g u/d: in a level's region (rho >= R) y^2 <= R/2 gives
// u = rho - y^2 >= R/2 >= h, so it loses at most a factor 2.  Per point the
// other combinations are sums of positive terms (bar -c/d^2, with c/d below
// 0.09 for every level) or enter scaled by 4 tau/d against it.  For larger y
// (u may reach 0) the per-point form is kept.
//
// UF, the u-form of the one-pair level for waves with larger y (where the
// block-summed form's S1 - h S0 would cancel): four sums in u = x^2 taken
// directly, S0 = sum g/d, U1 = sum g u/d, U2 = sum g u/d^2, U3 = sum g u^2/d^2.
// With d = u^2 + q u + p^2 and 2p - q = 4 tau, e^2 = 1/d + 4 tau u/d^2, so
//   sum g e = U1 + p S0,  sum g e^2 = S0 + 4 tau U2,
//   sum g t = 4 tau (p U2 - U3) - U1,
// where only the last difference changes sign (at u = p) and so cancels as
// the sum's own terms do.  A point costs u, d, 1/d and four sums (12 VALU
// instructions against 16.5 for the per-point form).
template <typename R, int PROF, int NP, bool SY = false, bool C0 = false, bool UF = false>
__device__ __forceinline__ void fast_range(const AdjLine<R>& L, const GSrc<R>& G, int r0, int r1,
                                           double& sA, double& sB, double& sC) {
  static_assert(!C0 || (SY && NP == 2 && sizeof(R) == 8), "the node at 0 has its own form in FP64 block sums");
  static_assert(!UF || (!SY && NP == 1), "the u-form is the one-pair level's");
  // the lanes running this loop (the wave's active lines) share the refills
  const unsigned long long act = __ballot(1);
  const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(act >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)act, 0u));
  const int nact = __popcll(act);
  // x at r = rb + j4 + jj as fma(rb + j4, a, nb + jj a): one conversion per
  // four points (nb + jj a rounds once, relative 6e-8 of at most 3.5 a, so x
  // keeps a relative error below 5e-7 for every r != 0)
  R nbj[4];
#pragma unroll
  for (int jj = 0; jj < 4; ++jj) nbj[jj] = fma((R)jj, L.a, L.nb);
  // SY: per pair h = q/2 (exact) and c = 4 y^2 tau = -k2 y^2
  R hS[NP], cS[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    hS[q] = (R)0.5 * L.P[q].q;
    cS[q] = (R)(-(double)L.P[q].k2 * L.y * L.y);
  }
  for (int rb = r0; rb <= r1; rb += kFlush) {
    const int n = min(kFlush, r1 - rb + 1);
    R s1 = 0, s2 = 0, s3 = 0, s4 = 0;
    R B[SY ? NP : 1][4];  // SY: S0..S3 per pair
#pragma unroll
    for (int q = 0; q < (SY ? NP : 1); ++q) B[q][0] = B[q][1] = B[q][2] = B[q][3] = 0;
    auto body = [&](R x, R gk) {
      const R u = x * x;
      if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN) {
        R e;
        if constexpr (sizeof(R) == 4) e = __builtin_amdgcn_exp2f(-u);
        else e = exp2(-u);
        const R ge = gk * e;
        s1 += ge;
        s2 = fma(ge, u, s2);
      } else if (PROF == XS_LORENTZ) {
        const R iq = arcp(u + (R)1);
        const R gi = gk * iq;
        s1 += gi;
        s2 = fma(gi, iq, s2);
      } else if constexpr (SY) {
        R sx[NP], rd[NP];
#pragma unroll
        for (int q = 0; q < NP; ++q) sx[q] = fma(x, x, hS[q]);
        if constexpr (sizeof(R) == 8 && NP >= 2) {
          // FP64: one reciprocal (and Newton step) for the first two pairs,
          // 1/d0 = d1/(d0 d1) and 1/d1 = d0/(d0 d1); d0 d1 stays finite
          // (C0: rd[1] = 1/v, v = sx[1])
          const R d0 = fma(sx[0], sx[0], cS[0]), d1 = C0 ? sx[1] : fma(sx[1], sx[1], cS[1]);
          const R r = arcp(d0 * d1);
          rd[0] = d1 * r;
          rd[1] = d0 * r;
          if constexpr (NP == 3) rd[2] = arcp(fma(sx[2], sx[2], cS[2]));
        } else {
#pragma unroll
          for (int q = 0; q < NP; ++q) rd[q] = arcp(fma(sx[q], sx[q], cS[q]));
        }
#pragma unroll
        for (int q = 0; q < (C0 ? 1 : NP); ++q) {
          const R grd = gk * rd[q], v = grd * rd[q];
          B[q][0] += grd;
          B[q][1] = fma(grd, sx[q], B[q][1]);
          B[q][2] += v;
          B[q][3] = fma(v, sx[q], B[q][3]);
        }
        if constexpr (C0) {
          const R gv = gk * rd[1];
          B[1][0] = fma(gv, rd[1], B[1][0]);
          B[1][1] += gv;
        }
      } else if constexpr (UF) {
        // s1 = S0, s2 = U1, s3 = U2, s4 = U3
        const PairD<R>& P = L.P[0];
        const R rd = arcp(fma(u, u + P.q, P.p2));
        const R gr = gk * rd;
        s1 += gr;
        s2 = fma(gr, u, s2);
        const R v = (gr * rd) * u;
        s3 += v;
        s4 = fma(v, u, s4);
      } else if constexpr (NP == 1) {
        // s1 = sum g e, s2 = sum g t, s3 = sum g / d, s4 = sum g e^2
        R e, rd, t;
        pair_adj<R>(L.P[0], u, e, rd, t);
        const R ge = gk * e;
        s1 += ge;
        s2 = fma(gk, t, s2);
        s3 = fma(gk, rd, s3);
        s4 = fma(ge, e, s4);
      } else {
        R E = 0, RD = 0, E2 = 0, T = 0;
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          R e, rd, t;
          pair_adj<R>(L.P[q], u, e, rd, t);
          const R Ke = L.P[q].K * e;
          E += Ke;
          RD = fma(L.P[q].K, rd, RD);
          E2 = fma(Ke, e, E2);
          T = fma(L.P[q].K, t, T);
        }
        s1 = fma(gk, E, s1);
        s2 = fma(gk, T, s2);
        s3 = fma(gk, RD, s3);
        s4 = fma(gk, E2, s4);
      }
    };
    // FP64 block-summed one-pair, three-point and two-pair levels: the four
    // points of a step share one reciprocal (with its Newton step) of the
    // product of their denominators P_h (d_0, d_0 v or d_0 d_1):
    // r = 1/(P_0 P_1 P_2 P_3), 1/P_0 = P_1 (P_2 P_3 r) and so on (the
    // hardware FP64 reciprocal issues at a quarter of the FMA rate)
    auto body4 = [&](R rf, auto gsrc, int j) {
      if constexpr (sizeof(R) == 8 && SY && NP <= 2 && PROF == XS_VOIGT) {
        R sx[4][NP], d[4][NP], P[4], gk[4];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const R x = fma(rf, L.a, nbj[h]);
          gk[h] = gsrc(j + h);
#pragma unroll
          for (int q = 0; q < NP; ++q) {
            sx[h][q] = fma(x, x, hS[q]);
            d[h][q] = (C0 && q == 1) ? sx[h][q] : fma(sx[h][q], sx[h][q], cS[q]);
          }
          P[h] = NP == 2 ? d[h][0] * d[h][1] : d[h][0];
        }
        const R p01 = P[0] * P[1], p23 = P[2] * P[3];
        const R r = arcp(p01 * p23);
        const R r01 = p23 * r, r23 = p01 * r;
        const R iP[4] = {P[1] * r01, P[0] * r01, P[3] * r23, P[2] * r23};
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          R rd[NP];
          if constexpr (NP == 2) {
            rd[0] = d[h][1] * iP[h];
            rd[1] = d[h][0] * iP[h];
          } else {
            rd[0] = iP[h];
          }
#pragma unroll
          for (int q = 0; q < (C0 ? 1 : NP); ++q) {
            const R grd = gk[h] * rd[q], v = grd * rd[q];
            B[q][0] += grd;
            B[q][1] = fma(grd, sx[h][q], B[q][1]);
            B[q][2] += v;
            B[q][3] = fma(v, sx[h][q], B[q][3]);
          }
          if constexpr (C0) {
            const R gv = gk[h] * rd[1];
            B[1][0] = fma(gv, rd[1], B[1][0]);
            B[1][1] += gv;
          }
        }
      }
    };
    auto run = [&](auto gsrc) {
      int j = 0;
      if (sizeof(R) == 8 && SY && NP <= 2 && PROF == XS_VOIGT && L.share4) {
        for (; j + 4 <= n; j += 4) body4((R)(rb + j), gsrc, j);
      } else {
        for (; j + 4 <= n; j += 4) {
          const R rf = (R)(rb + j);
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) body(fma(rf, L.a, nbj[jj]), gsrc(j + jj));
        }
      }
      for (; j < n; ++j) body(fma((R)(rb + j), L.a, L.nb), gsrc(j));
    };
    if (G.lds) {
      // refill the wave's slice with g[kcmin + rb + t], t < 2 kFlush
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      const int64_t kb = (int64_t)G.kcmin + rb;
      for (int t = rank; t < 2 * kFlush; t += nact) {
        const int64_t k = kb + t;
        G.buf[t] = (k >= 0 && k < G.nb) ? (R)(G.gc[k] * G.gs) : (R)0;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const R* gl = G.buf + (L.kc - G.kcmin);
      run([&](int j) { return gl[j]; });
    } else {
      const double* gp = G.gc + (L.kc + rb);
      if constexpr (sizeof(R) == 4) run([&](int j) { return (R)(gp[j] * G.gs); });
      else run([&](int j) { return (R)gp[j]; });
    }
    // to the general-path convention
    if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN) {
      sA += (double)s1;
      sB += 2.0 * kLN2 * (double)s2 - (double)s1;
    } else if (PROF == XS_LORENTZ) {
      sA += (double)s1;
      sC += (double)s1 - 2.0 * (double)s2;
    } else {
      const double k = (NP == 1 && !SY && !UF) ? (double)L.P[0].K : 1.0;
      const double y2 = L.y * L.y;
      // sums of g e, g t, g/d, g e^2 (K-weighted over the pairs but for the
      // one-pair per-point form)
      double ge = (double)s1, gt = (double)s2, gd = (double)s3, ge2 = (double)s4;
      if constexpr (UF) {
        const double K = (double)L.P[0].K, t4 = -(double)L.P[0].k2, p = (double)L.P[0].p;
        const double S0 = (double)s1, U1 = (double)s2, U2 = (double)s3, U3 = (double)s4;
        ge = K * (U1 + p * S0);
        gd = K * S0;
        ge2 = K * (S0 + t4 * U2);
        gt = K * (t4 * (p * U2 - U3) - U1);
      } else if constexpr (SY) {
        ge = gt = gd = ge2 = 0.0;
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          const double K = (double)L.P[q].K, t4 = -(double)L.P[q].k2, m = 0.5 * t4;
          const double h = (double)hS[q], c = (double)cS[q];
          const double S0 = (double)B[q][0], S1 = (double)B[q][1], S2 = (double)B[q][2], S3 = (double)B[q][3];
          const double sq = S0 - c * S2;  // sum g s^2/d^2
          ge += K * (S1 + m * S0);
          gd += K * S0;
          ge2 += K * (sq + 2.0 * m * S3 + m * m * S2);
          gt += K * (t4 * ((2.0 * y2 + h) * S3 - sq - 2.0 * y2 * h * S2) - (S1 - h * S0));
        }
      }
      const double e = k * ge, t = k * gt;
      const double w = k * (ge + 2.0 * y2 * gd - 4.0 * y2 * ge2);  // dRe w/dy
      sA += L.y * e;                      // Re w
      sB += L.y * (e + 2.0 * t) + L.y * w; // Re w + x dRe w/dx + y dRe w/dy
      sC -= w;                            // Im w' = -dRe w/dy
    }
  }
}

// Level l of Levels<R> (the caller has put the level's pairs in L.P; the
// node at 0 of the FP64 three-point level is L.P[1]).
template <typename R, int PROF>
__device__ __forceinline__ void fast_level(int level, const AdjLine<R>& L, const GSrc<R>& G, int r0, int r1,
                                           double& sA, double& sB, double& sC, bool blocksum = false) {
  if (PROF == XS_VOIGT && blocksum) {
    if (level == 0) fast_range<R, PROF, 1, true>(L, G, r0, r1, sA, sB, sC);
    else if constexpr (sizeof(R) == 4) fast_range<R, PROF, 2, true>(L, G, r0, r1, sA, sB, sC);
    else if (level == 1) fast_range<R, PROF, 2, true, true>(L, G, r0, r1, sA, sB, sC);
    else if (level == 2) fast_range<R, PROF, 2, true>(L, G, r0, r1, sA, sB, sC);
    else fast_range<R, PROF, 3, true>(L, G, r0, r1, sA, sB, sC);
    return;
  }
  if (PROF == XS_VOIGT && level == 0) fast_range<R, PROF, 1, false, false, true>(L, G, r0, r1, sA, sB, sC);
  else if (PROF != XS_VOIGT || level == 0) fast_range<R, PROF, 1>(L, G, r0, r1, sA, sB, sC);
  else if (sizeof(R) == 4 || level <= 2) fast_range<R, PROF, 2>(L, G, r0, r1, sA, sB, sC);
  else if constexpr (sizeof(R) == 8) fast_range<R, PROF, 3>(L, G, r0, r1, sA, sB, sC);
}

// r-range of the bins where |x| < X (widened by one bin), clipped to
// [lo - 1, hi + 1]; empty ranges are lo > hi.
__device__ __forceinline__ void r_range(double X, double a, double b, int lo, int hi, int& rl, int& rh) {
  if (!(X > 0.0)) {
    rl = 0x7fffffff;
    rh = -0x7fffffff;
    return;
  }
  const double l = fmax(floor((b - X) / a) - 1.0, (double)lo - 1.0);
  const double h = fmin(ceil((b + X) / a) + 1.0, (double)hi + 1.0);
  if (l > h) {
    rl = 0x7fffffff;
    rh = -0x7fffffff;
  } else {
    rl = (int)l;
    rh = (int)h;
  }
}

// Window sums of the lane's line (general-path convention: Re w, Re G, Im w'
// for the Voigt profile).
struct Sums3 {
  double A, B, C;
};

template <typename R, int PROF>
__device__ __forceinline__ Sums3 window_sums(bool on, int64_t klo, int64_t khi, double nu, double inv, double y,
                                             const double* gc, double gs, double nu0, double dnu, int64_t nbins,
                                             R* gbuf) {
  const int64_t kc64 = home_bin(nu, nu0, dnu);
  const double delta = nu - nu_of_bin(nu0, dnu, kc64);
  AdjLine<R> L;
  L.kc = (int)kc64;
  L.rlo = on ? (int)(klo - kc64) : 0x7fffffff;
  L.rhi = on ? (int)(khi - kc64) : -0x7fffffff;
  L.ad = dnu * inv;
  L.bd = delta * inv;
  L.y = y;
  L.a = (R)L.ad;
  L.nb = (R)(-L.bd);
  bool wide = false;
  if (PROF == XS_VOIGT) {
    // the node pairs of a far level are set in L.P when a run of it starts
    if (sizeof(R) == 4 && on) {
      const double xmax = fmax(fabs((double)L.rlo * L.ad - L.bd), fabs((double)L.rhi * L.ad - L.bd));
      wide = xmax > 1.0e9 || y > 1.0e9;
    }
  }
  // FP64 far levels share one reciprocal among four points when the product
  // of their denominators (up to eight fourth-degree factors in x^2 + y^2)
  // stays finite: |x| and y of every line of the wave below 1e9
  L.share4 = false;
  if (sizeof(R) == 8 && PROF == XS_VOIGT) {
    const double xmax = on ? fmax(fabs((double)L.rlo * L.ad - L.bd), fabs((double)L.rhi * L.ad - L.bd)) : 0.0;
    L.share4 = __ballot(on && !(xmax <= 1.0e9 && y <= 1.0e9)) == 0;
  }
  // uniform runs along r
  const int Rmin = wave_min(L.rlo), Rmax = wave_max(L.rhi);
  const int Alo = wave_max(on ? L.rlo : -0x7fffffff), Ahi = wave_min(on ? L.rhi : 0x7fffffff);
  const bool any_wide = __ballot(wide) != 0;
  constexpr int NL = (PROF == XS_VOIGT) ? Levels<R>::n : 1;
  int Hlo[NL], Hhi[NL];
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    int rl = 0x7fffffff, rh = -0x7fffffff;
    if (on) {
      double X;
      if (PROF == XS_VOIGT) X = sqrt(fmax(Levels<R>::rho[l] * 1.001 - y * y, 0.0));
      else if (PROF == XS_LORENTZ) X = 0.0;  // one level, no inner region
      else X = (sizeof(R) == 4) ? sqrt(160.0) : sqrt(1100.0);  // Gaussian: nonzero range
      r_range(X, L.ad, L.bd, L.rlo, L.rhi, rl, rh);
    }
    Hlo[l] = wave_min(rl);
    Hhi[l] = wave_max(rh);
  }
  double sA = 0.0, sB = 0.0, sC = 0.0;
  GSrc<R> G;
  G.gc = gc;
  G.gs = gs;
  G.nb = nbins;
  G.kcmin = wave_min(on ? L.kc : 0x7fffffff);
  G.lds = (int64_t)wave_max(on ? L.kc : -0x7fffffff) - G.kcmin <= kFlush;
  G.buf = gbuf;
  // levels whose block-summed form every line of the wave allows (bit l:
  // y^2 at most half of level l's rho bound)
  int blk = 0;
#pragma unroll
  for (int q = 0; q < NL; ++q)
    if (__ballot(on && !(y * y <= 0.5 * Levels<R>::rho[q])) == 0) blk |= 1 << q;
  if (on) {
    int r = Rmin;
    while (r <= Rmax) {
      int end, mode;  // mode: -2 skip, -1 general, l >= 0 fast level l
      if (any_wide || r < Alo || r > Ahi) {
        mode = -1;
        end = (any_wide || r > Ahi) ? Rmax : Alo - 1;
      } else if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN) {
        // outside the nonzero hull every lane's Gaussian is exactly 0
        if (Hlo[0] > Hhi[0] || r > Hhi[0]) { mode = -2; end = Ahi; }
        else if (r < Hlo[0]) { mode = -2; end = Hlo[0] - 1; }
        else { mode = 0; end = min(Hhi[0], Ahi); }
      } else if (PROF == XS_LORENTZ) {
        mode = 0;
        end = Ahi;
      } else {
        // deepest level whose hull holds r
        int l = 0;
#pragma unroll
        for (int q = 0; q < NL; ++q)
          if (l == q && Hlo[q] <= r && r <= Hhi[q]) l = q + 1;
        if (l == NL) {
          mode = -1;
          end = min(Hhi[NL - 1], Ahi);
        } else {
          mode = l;
          if (Hlo[l] <= Hhi[l] && r < Hlo[l]) end = Hlo[l] - 1;   // up to the next inner hull
          else end = (l == 0) ? Ahi : Hhi[l - 1];                  // to the end of this hull
          end = min(end, Ahi);
        }
      }
      if (mode >= 0) {
        if (PROF == XS_VOIGT) {
          // the level's node pairs (FP64: one pair, the three-point rule,
          // two pairs, three pairs; FP32: one pair, two pairs)
          const bool two = sizeof(R) == 8 ? mode == 2 : mode == 1;
          if (mode == 0) {
            L.P[0] = pair_d<R>(y, GH::t2[0], GH::w2[0]);
          } else if (two) {
            L.P[0] = pair_d<R>(y, GH::t4[0], GH::w4[0]);
            L.P[1] = pair_d<R>(y, GH::t4[1], GH::w4[1]);
          } else if (mode == 1) {
            L.P[0] = pair_d<R>(y, GH::t3[0], GH::w3[0]);
            L.P[1] = pair_d<R>(y, 0.0, 0.5 * GH::w3c);
          } else {
            L.P[0] = pair_d<R>(y, GH::t6[0], GH::w6[0]);
            L.P[1] = pair_d<R>(y, GH::t6[1], GH::w6[1]);
            L.P[2] = pair_d<R>(y, GH::t6[2], GH::w6[2]);
          }
          fast_level<R, PROF>(mode, L, G, r, end, sA, sB, sC, (blk >> mode) & 1);
        } else {
          fast_level<R, PROF>(0, L, G, r, end, sA, sB, sC);
        }
      } else if (mode == -1) {
        for (int rr = r; rr <= end; ++rr) {
          if (rr >= L.rlo && rr <= L.rhi) {
            const double gk = gc[L.kc + rr] * gs;
            general_eval<R, PROF>(L, wide, rr, gk, sA, sB, sC);
          }
        }
      }
      r = end + 1;
    }
  }
  return Sums3{sA, sB, sC};
}

// One wave owns 64 consecutive sorted lines (one per lane) and walks all of
// their windows together in steps of r = k - k_c.  Lanes of a wave hold lines
// of nearly equal wavenumber and width, so at a given r they need the same
// formula: the r axis is cut into uniform runs (far-region levels, the
// general core, masked window ends) decided once per wave.
template <typename R, int PROF>
__global__ __launch_bounds__(256, sizeof(R) == 4 ? 4 : 3) void k_adjoint(AdjArgs a) {
  __shared__ double sdt[4][kMaxCond];
  __shared__ double sdp[4][kMaxCond];
  __shared__ R s_g[4][2 * kFlush];  // per-wave cotangent slices
  const ModelDev& m = a.m;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int c = threadIdx.x; c < kMaxCond; c += 256)
    for (int w = 0; w < 4; ++w) sdt[w][c] = sdp[w][c] = 0.0;
  __syncthreads();
  const int64_t nk = a.off[m.n_buckets];
  const int64_t nbatch = (nk + 63) >> 6;
  const double sqrt2ln2 = sqrt(2.0 * kLN2);
  for (int64_t bt = (int64_t)blockIdx.x * 4 + wave; bt < nbatch; bt += (int64_t)gridDim.x * 4) {
    const int64_t p = bt * 64 + lane;
    const bool have = p < nk;
    double nu = 0.0, gref = 0.0, nexp = 0.0, gpre = 0.0, Es = 0.0;
    int32_t i = 0;
    if (have) {
      nu = a.rnu[p];
      gref = (double)a.rgref[p];
      nexp = (double)a.rnexp[p];
      gpre = a.rgpre ? a.rgpre[p] : 0.0;
      i = a.ridx[p];
      Es = a.rEs[p];
    }
    double dls = 0.0, dgr = 0.0, dne = 0.0;
    for (int c = 0; c < m.n_cond; ++c) {
      const CondDev cd = a.cond[c];
      int64_t klo = 0, khi = -1;
      bool on = have && line_window(nu, cd.cut, m.nu0, m.dnu, m.n_bins, klo, khi);
      double S = 0.0;
      if (on) {
        S = (sizeof(R) == 4)
                ? (double)((const float*)a.rS)[(int64_t)cd.slot * a.max_lines + p] * exp(a.sb[cd.slot])
                : ((const double*)a.rS)[(int64_t)cd.slot * a.max_lines + p];
        on = S != 0.0;
      }
      if (__ballot(on) == 0) continue;
      const double alpha = (PROF == XS_GAUSSIAN) ? cd.hwhm : nu * cd.dop;
      const double sgm = alpha / sqrt2ln2;
      const double gpow = exp(nexp * cd.lnTr);
      // gam: the pressure width (all the chain rule acts on); gtot adds the
      // upper state's lifetime width and shapes the profile
      const double gam = gref * gpow * cd.pfac;
      const double gtot = gam + gpre;
      double inv, y = 0.0;
      if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN) inv = 1.0 / alpha;
      else if (PROF == XS_LORENTZ) inv = 1.0 / gtot;
      else {
        inv = sqrt(kLN2) / alpha;
        y = gtot * inv;
      }
      // FP32 form: the cotangent enters the window sums scaled by a power of
      // two, gs, that brings its largest magnitude over the condition's grid
      // into [1/2, 1), so the FP32 block sums of g/d and g/d^2 terms stay in
      // the normal range whatever the loss's magnitude; the sums are
      // unscaled exactly in FP64.  (FP64: gs = 1.)
      double gs = 1.0, igs = 1.0;
      if (sizeof(R) == 4) {
        const double gm = __longlong_as_double((long long)a.gmax[c]);
        if (gm > 0.0 && gm <= 1.7976931348623157e308) {
          int e;
          (void)frexp(gm, &e);
          e = max(e, -1000);
          gs = ldexp(1.0, -e);
          igs = ldexp(1.0, e);
        }
      }
      const Sums3 ws = window_sums<R, PROF>(on, klo, khi, nu, inv, y, a.g + (int64_t)c * m.n_bins, gs, m.nu0,
                                            m.dnu, m.n_bins, s_g[wave]);
      const double sA = ws.A * igs, sB = ws.B * igs, sC = ws.C * igs;
      // scale to the unit-area profile and its derivatives
      double A, B, C;
      if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN) {
        const double c0 = sqrt(kLN2 / kPI) / alpha;
        A = c0 * sA;
        B = c0 * sB / sgm;
        C = 0.0;
      } else if (PROF == XS_LORENTZ) {
        A = sA / (kPI * gtot);
        B = 0.0;
        C = sC / (kPI * gtot * gtot);
      } else {
        const double c0 = 1.0 / (sgm * sqrt(2.0 * kPI));
        A = c0 * sA;
        C = -sC / (2.0 * sqrt(kPI) * sgm * sgm);          // -Im w' / (2 sqrt(pi) sg^2)
        B = -sB / (sgm * sgm * sqrt(2.0 * kPI));          // -Re G / (sg^2 sqrt(2 pi))
      }
      double vt = 0.0, vp = 0.0;
      if (on) {
        const double T = cd.Tk;
        double dlnS;
        if (m.mode == XS_ABSORPTION)  // Es = E of the lower state
          dlnS = kC2 * Es / (T * T) - (kC2 * nu / (T * T)) / expm1(kC2 * nu / T) - a.dQ[cd.slot] / a.Q[cd.slot];
        else                          // Es = E of the upper state
          dlnS = kC2 * Es / (T * T) - a.dQ[cd.slot] / a.Q[cd.slot];
        const double dsg_dT = (PROF == XS_GAUSSIAN) ? 0.0 : sgm / (2.0 * T);
        dls += S * A;
        dgr += S * C * gpow * cd.pfac;
        dne += S * C * gam * cd.lnTr;
        vt = S * (A * dlnS + B * dsg_dT - C * nexp * gam / T);
        vp = (cd.P > 0.0) ? S * C * gam / cd.P : 0.0;
      }
      vt = wave_sum(vt);
      vp = wave_sum(vp);
      if (lane == 0) {
        sdt[wave][c] += vt;
        sdp[wave][c] += vp;
      }
    }
    if (have) {
      a.dls[i] = dls;
      if (a.dgref) a.dgref[i] = dgr;
      if (a.dnexp) a.dnexp[i] = dne;
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < m.n_cond; c += 256) {
    const double t = ((sdt[0][c] + sdt[1][c]) + sdt[2][c]) + sdt[3][c];
    const double q = ((sdp[0][c] + sdp[1][c]) + sdp[2][c]) + sdp[3][c];
    a.part[((int64_t)c * 2 + 0) * gridDim.x + blockIdx.x] = t;
    a.part[((int64_t)c * 2 + 1) * gridDim.x + blockIdx.x] = q;
  }
}

__global__ __launch_bounds__(256) void k_adj_final(const double* part, int n_cond, int nblk, double* dT,
                                                   double* dP) {
  __shared__ double sh[256];
  const int c = blockIdx.x;
  for (int which = 0; which < 2; ++which) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) v += part[((int64_t)c * 2 + which) * nblk + b];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) (which ? dP : dT)[c] = sh[0];
    __syncthreads();
  }
}

__global__ void k_zero3(double* a, double* b, double* c, int64_t n, unsigned long long* gmax, int n_cond) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (a) a[i] = 0.0;
    if (b) b[i] = 0.0;
    if (c) c[i] = 0.0;
  }
  if (blockIdx.x == 0)
    for (int q = threadIdx.x; q < n_cond; q += blockDim.x) gmax[q] = 0ull;
}

// Largest |g_k| of each condition's cotangent (FP32 form's scale).  The bit
// patterns of non-negative doubles order like the values (a NaN above
// infinity), so an unsigned integer max finds it.
__global__ __launch_bounds__(256) void k_gmax(const double* g, int64_t n_bins, unsigned long long* gmax) {
  const int c = blockIdx.y;
  const double* gc = g + (int64_t)c * n_bins;
  unsigned long long v = 0ull;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n_bins; k += (int64_t)gridDim.x * 256) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(fabs(gc[k]));
    v = b > v ? b : v;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long w = (unsigned long long)__shfl_xor((long long)v, o, 64);
    v = w > v ? w : v;
  }
  if ((threadIdx.x & 63) == 0 && v) atomicMax(gmax + c, v);
}

void launch_adjoint(const ModelDev& m, const Work& w, const StatesView& st, const LinesView& ln,
                    const double* g, double* dT, double* dP, double* dgref, double* dnexp,
                    double* dls, int64_t n_lines, int adj_blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_zero3, dim3(2048), dim3(256), 0, s, dgref, dnexp, dls, n_lines, w.gmax, m.n_cond);
  if (m.prec == XS_FP32) {
    const int64_t gb = std::min<int64_t>((m.n_bins + 1023) / 1024, 512);
    hipLaunchKernelGGL(k_gmax, dim3((unsigned)gb, m.n_cond), dim3(256), 0, s, g, m.n_bins, w.gmax);
  }
  AdjArgs a;
  a.m = m;
  a.cond = w.cond;
  a.Q = w.Q;
  a.dQ = w.dQ;
  a.sb = w.sb;
  a.off = w.off;
  a.rnu = w.rnu;
  a.rgref = w.rgref;
  a.rnexp = w.rnexp;
  a.rgpre = w.rgpre;
  a.ridx = w.ridx;
  a.rEs = w.rEs;
  a.rS = w.rS;
  a.max_lines = w.max_lines;
  a.g = g;
  a.gmax = w.gmax;
  a.dgref = dgref;
  a.dnexp = dnexp;
  a.dls = dls;
  a.part = w.adjpart;
#define XS_A(R, P)                                                                      \
  if (m.profile == P) {                                                                 \
    hipLaunchKernelGGL((k_adjoint<R, P>), dim3(adj_blocks), dim3(256), 0, s, a);         \
  }
  if (m.prec == XS_FP32) {
    XS_A(float, XS_DOPPLER) XS_A(float, XS_GAUSSIAN) XS_A(float, XS_LORENTZ) XS_A(float, XS_VOIGT)
  } else {
    XS_A(double, XS_DOPPLER) XS_A(double, XS_GAUSSIAN) XS_A(double, XS_LORENTZ) XS_A(double, XS_VOIGT)
  }
#undef XS_A
  hipLaunchKernelGGL(k_adj_final, dim3(m.n_cond), dim3(256), 0, s, w.adjpart, m.n_cond, adj_blocks, dT, dP);
}

}  // namespace xs
