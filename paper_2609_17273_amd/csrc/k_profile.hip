// Profile pass: sigma_k = sum_i S_i f_i(nu_k - nu_i) over each line's cut-off
// window (Eq. xsec with the cut-off rule of section "Spectral synthesis").
//
// k_gather: grid-tile-parallel.  A work item is one wave on (tile t of
//   tile_bins grid points, condition c, slice of the tile's candidate lines);
//   the candidates are the buckets within cut-off reach of the tile (lines
//   were sorted by home bin).  Each batch of up to 64 candidates is staged one
//   line per lane (exact window test against the tile, per-line constants,
//   class of the line for the tile), compacted into LDS grouped by class with
//   a ballot and mbcnt per class, and evaluated over the tile's bins, lane l
//   owning bins tlo + 64 j + l.  Lines whose formula is uniform over the tile
//   run in branch-free loops; the rest take per-chunk decisions.  FP32 partial
//   sums are flushed to FP64 after each batch.  Tiles split over several items
//   write FP64 partial rows that k_reduce adds in item order; a persistent
//   grid pulls items from a device counter.
// k_scatter: line-parallel comparison: one wave per (line, condition) walks
//   the window and adds each term into sigma with hardware FP64 atomics.
#include "k_common.h"

namespace xs {

// ---------------------------------------------------------------------------
// Per-(line, condition) constants.  The lane variable is
//   x = (nu_k - nu_i) * inv = (k - k_c) a - b,  a = dnu inv,  b = delta inv,
// with inv = 1/alpha (Gaussian: f = c0 2^{-x^2}), 1/gamma (Lorentzian:
// f = c0 / (1 + x^2)) or 1/(sg sqrt 2) = sqrt(ln 2)/alpha (Voigt:
// f = c0 Re w(x + i y)).  For the Voigt far region each Gauss-Hermite node
// pair j contributes, with u = x^2, p_j = y^2 + tau_j, q_j = 2 y^2 - 2 tau_j,
//   c0 (2y/pi) W_j (u + p_j) / ((u - p_j)^2 + 4 y^2 u)
//     = (cW_j u + cW_j p_j) / (u (u + q_j) + p_j^2),
// so a far-wing evaluation is 2 FMA, 1 add, 1 reciprocal and 1 FMA into the
// accumulator after x and u.
// ---------------------------------------------------------------------------
struct LineParams {
  double inv, y, c0;
};

template <int PROF>
__device__ __forceinline__ LineParams line_params(const ModelDev& m, const CondDev& cd, double nu,
                                                  double gref, double nexp, double gpre, double S) {
  LineParams lp;
  double alpha = (PROF == XS_GAUSSIAN) ? cd.hwhm : nu * cd.dop;
  double gamma = gref * exp(nexp * cd.lnTr) * cd.pfac + gpre;
  if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN) {
    lp.inv = 1.0 / alpha;
    lp.y = 0.0;
    lp.c0 = S * sqrt(kLN2 / kPI) / alpha;
  } else if (PROF == XS_LORENTZ) {
    lp.inv = 1.0 / gamma;
    lp.y = 0.0;
    lp.c0 = S / (kPI * gamma);
  } else {
    lp.inv = sqrt(kLN2) / alpha;
    lp.y = gamma * lp.inv;
    lp.c0 = S * sqrt(kLN2) / (alpha * sqrt(kPI));
  }
  return lp;
}

// Far-region constants of node pair (tau, W) in the shifted variable
// s = x^2 + h, h = y^2 - tau: the pair's term is cW (s + 2 tau)/(s^2 + c),
// c = 4 y^2 tau (the same fraction as cW (u + p)/(u^2 + q u + p^2) with
// u = x^2, p = y^2 + tau, q = 2 y^2 - 2 tau, one operation fewer).
template <typename R>
struct Pair {
  R cw, cwt, h, c;  // cW, cW 2 tau, y^2 - tau, 4 y^2 tau
};
template <typename R>
__device__ __forceinline__ Pair<R> make_pair(double c0, double y, double tau, double W) {
  const double y2 = y * y;
  const double cw = c0 * (y * (2.0 / kPI)) * W;
  Pair<R> r;
  r.cw = (R)cw;
  r.cwt = (R)(cw * (2.0 * tau));
  r.h = (R)(y2 - tau);
  r.c = (R)(4.0 * y2 * tau);
  return r;
}

// Bin ranges of a line inside which a cheaper formula is not valid:
// |x| < X  <=>  k - k_c in ((b - X)/a, (b + X)/a); widened by one bin so the
// float evaluation of x cannot leave a range through rounding.  Empty ranges
// use lo > hi sentinels that intersect nothing.
struct KRange {
  int lo, hi;
};
__device__ __forceinline__ KRange x_range(double X, double a, double b, int64_t kc, int64_t klo,
                                          int64_t khi) {
  KRange r;
  if (!(X > 0.0)) {
    r.lo = 0x7fffffff;
    r.hi = -0x7fffffff;
    return r;
  }
  double lo = floor((b - X) / a) - 1.0 + (double)kc;
  double hi = ceil((b + X) / a) + 1.0 + (double)kc;
  lo = fmax(lo, (double)klo - 1.0);
  hi = fmin(hi, (double)khi + 1.0);
  if (lo > hi) {
    r.lo = 0x7fffffff;
    r.hi = -0x7fffffff;
    return r;
  }
  r.lo = (int)lo;
  r.hi = (int)hi;
  return r;
}

// Class of a staged line for the tile: 0 = nothing to add (outside the
// window, or a Gaussian whose 2^{-x^2} vanishes on every bin of the tile);
// 1 = every bin of the tile takes the first uniform formula (Voigt: one node
// pair; Gaussian, Lorentzian: the profile itself); 3 = second uniform formula
// (Voigt: two node pairs); 4, 5 = as 1, 3 where a window end falls inside the
// tile (the same formula under a window mask); 2 = general per-chunk path
// (the core, the Gaussian's zero chunks, lines evaluated in FP64).
constexpr int kRowSkip = 0, kRowF1 = 1, kRowGeneral = 2, kRowF2 = 3, kRowF1M = 4, kRowF2M = 5;
// FP64 form only: third uniform formula (three node pairs), plain and masked;
// the three-point formula of the sampled Voigt between the first and second.
constexpr int kRowF3 = 6, kRowF3M = 7, kRowF15 = 8, kRowF15M = 9;

// FP32 far-region node pair in shifted form.  With h = y^2 - tau and
// s = u + h = |z|^2 - tau (positive wherever a node rule is used),
//   cW (u + p)/d = cW (s + 2 tau)/(s^2 + 4 y^2 tau),
// so a pair costs three FMAs and a reciprocal from x, with no separate
// u = x^2; every term is positive, so nothing cancels.
struct PairS {
  float cw, cwt, h, c;  // cW, cW 2 tau, y^2 - tau, 4 y^2 tau
};
__device__ __forceinline__ float pair_term_s(const PairS& P, float x) {
  const float s = fmaf(x, x, P.h);
  return fmaf(P.cw, s, P.cwt) * __builtin_amdgcn_rcpf(fmaf(s, s, P.c));
}

// FP32 form.  The first-formula fields come first (two 16-byte LDS reads);
// the second formula reads a, nb, jfb and B1, B2.
//   rB: bins that are not far-wing (one node pair) -- for the Gaussian, the
//       bins where 2^{-x^2} is not zero in FP32; rC, rD: bins with
//       |z|^2 < 64 and < 36 (outside rC two node pairs suffice, outside rD
//       three; a chunk that meets rD takes the rational approximation).
struct __attribute__((aligned(16))) RecF {
  float a, nb, jfb, c0;  // x = (jfb + offset of the bin in the tile) a + nb; jfb = tlo - k_c
  PairS A;               // one node pair
  PairS B1, B2;          // two node pairs
  int klo, khi, flag, kc;
  KRange rB, rC;
  KRange rD;
  float y;
  int pad0;
};
// FP64 two node pairs (tau_1, W_1), (tau_2, W_2) of the four-point rule as
// one fraction N(s)/D(s) in s = x^2 + y^2 - tau_1 = |z|^2 - tau_1.  With
// d = tau_1 - tau_2, c_j = 4 y^2 tau_j and cw_j = c0 (2 y/pi) W_j the pairs
// are cw_1 (s + e_1)/(s^2 + c_1) + cw_2 (s + e_2)/((s + d)^2 + c_2),
// e_1 = 2 tau_1, e_2 = tau_1 + tau_2, so
//   N = cw_1 (s + e_1)(s^2 + 2 d s + q) + cw_2 (s + e_2)(s^2 + c_1),
//   D = (s^2 + c_1)(s^2 + 2 d s + q),  q = d^2 + c_2,
// expanded into a cubic and a monic quartic.  Where the rule is used,
// s >= 4000 - tau_1 and c_j <= 4 tau_j (s + tau_1), so every lower term of
// either polynomial is below 3e-3 of the leading one: Horner's rule keeps the
// relative error at a few units of rounding, with one FMA per degree.
struct Poly2 {
  double h, n3, n2, n1, n0, d3, d2, d1, d0;  // h = y^2 - tau_1
};
__device__ __forceinline__ Poly2 make_poly2(double c0, double y) {
  const double t1 = GH::t4[0], t2 = GH::t4[1];
  const double y2 = y * y, k = c0 * (y * (2.0 / kPI));
  const double cw1 = k * GH::w4[0], cw2 = k * GH::w4[1];
  const double d = t1 - t2, c1 = 4.0 * y2 * t1, q = d * d + 4.0 * y2 * t2;
  const double e1 = 2.0 * t1, e2 = t1 + t2;
  Poly2 B;
  B.h = y2 - t1;
  B.n3 = cw1 + cw2;
  B.n2 = cw1 * (2.0 * d + e1) + cw2 * e2;
  B.n1 = cw1 * (q + 2.0 * d * e1) + cw2 * c1;
  B.n0 = cw1 * e1 * q + cw2 * e2 * c1;
  B.d3 = 2.0 * d;
  B.d2 = q + c1;
  B.d1 = 2.0 * d * c1;
  B.d0 = c1 * q;
  return B;
}
__device__ __forceinline__ void poly2_nd(const Poly2& B, double x, double& N, double& D) {
  const double s = fma(x, x, B.h);
  N = fma(fma(fma(B.n3, s, B.n2), s, B.n1), s, B.n0);
  D = fma(fma(fma(s + B.d3, s, B.d2), s, B.d1), s, B.d0);
}

// FP64 three-point rule (nodes 0 and +-t, tau = t^2 = 3/2) as one fraction
// in s = |z|^2 - tau.  The pair is cw (s + 2 tau)/(s^2 + c), c = 4 y^2 tau,
// cw = c0 (2 y/pi) W; the node at 0 adds e/(x^2 + y^2) = e/(s + tau) with
// e = c0 (y/pi) W_0.  Together
//   N = (cw + e) s^2 + 3 cw tau s + (2 cw tau^2 + e c),
//   D = (s^2 + c)(s + tau) = s^3 + tau s^2 + c s + c tau:
// two FMAs for N and an add and two FMAs for D, against three and four for
// the four-point fraction.  Where it is used, s >= 4.5e4 - tau, so the lower
// terms are below 1e-4 of the leading ones.
struct Poly3 {
  double h, tau, n2, n1, n0, c, ct;  // h = y^2 - tau; ct = c tau
};
__device__ __forceinline__ Poly3 make_poly3(double c0, double y) {
  const double tau = GH::t3[0];
  const double y2 = y * y, k = c0 * (y * (2.0 / kPI));
  const double cw = k * GH::w3[0], e = 0.5 * k * GH::w3c, c = 4.0 * y2 * tau;
  Poly3 C;
  C.h = y2 - tau;
  C.tau = tau;
  C.n2 = cw + e;
  C.n1 = 3.0 * cw * tau;
  C.n0 = 2.0 * cw * tau * tau + e * c;
  C.c = c;
  C.ct = c * tau;
  return C;
}
__device__ __forceinline__ void poly3_nd(const Poly3& C, double x, double& N, double& D) {
  const double s = fma(x, x, C.h);
  N = fma(fma(C.n2, s, C.n1), s, C.n0);
  D = fma(fma(s + C.tau, s, C.c), s, C.ct);
}

// FP64 form.  r[0..4]: bins with |z|^2 below 9e6, 4000, 400, 144, 64 (the
// thresholds of the 1, 2, 3, 4 and 6 node-pair bands of the sampled Voigt;
// the binned Voigt's second threshold is 6400); for the Gaussian, r[0] holds
// the bins where 2^{-x^2} is not zero in FP64.  The far-region rows of the
// Voigt take x = (offset of the point in the row) a + xb.  A line stores the
// one-pair constants A when its row takes the first formula, the three-point
// fraction C when the row lies wholly at |z|^2 >= 4.5e4 (sampled Voigt),
// else the two-pair fraction B.
struct __attribute__((aligned(16))) RecD {
  double nu, inv, c0, y;
  double a, xb;  // a = dnu / width; xb = x at the row's first point
  int klo, khi, flag, kc;
  KRange r[5];
  int pad0, pad1;
  union {
    Pair<double> A;
    Poly2 B;
    Poly3 C;
  };
};

// The kernels tell the two record types apart by size, and a wave's LDS
// holds 64 records (12 KB of FP64 records, three waves per SIMD).
static_assert(sizeof(RecF) != sizeof(RecD), "record types are told apart by size");
static_assert(sizeof(RecD) == 192, "FP64 record: 64 per wave in 12 KB of LDS");

// the staging precision of a record type
template <typename Rec>
using LReal = typename std::conditional<sizeof(Rec) == sizeof(RecF), float, double>::type;

struct GatherArgs {
  ModelDev m;
  const CondDev* cond;
  const double* sb;
  const int32_t* off;
  const double* rnu;
  const float* rgref;
  const float* rnexp;
  const double* rgpre;      // lifetime widths, or null when the states have no lifetimes
  const void* rS;
  const int32_t* rkc;       // home bin of every sorted line
  const float* rdel;        // nu - nu_{k_c}
  const int32_t* rwin;      // exact windows per cut-off class
  int64_t max_lines;
  int32_t* counter;         // [0]: work queue; [2..3]: candidate total; [4..5]: lines per item
  const int32_t* ib;        // [n_ct + 1] first work item of each (tile, condition); ib[n_ct] = items
  const int32_t* pb;        // [n_ct + 1] first partial row of each split (tile, condition)
  double* part;             // partial rows of split tiles
  double* sigma;
  int32_t accumulate;
  int32_t n_tiles;
  int32_t n_ct;             // n_tiles * n_cond; ct = t * n_cond + c
  int32_t tile_bins;
  int32_t persistent;
  int64_t chunk_cfg;        // requested lines per work item (0: automatic)
  int64_t item_target;      // work items aimed at when tiles are split
};

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ bool meets(int lo, int hi, const KRange& r) { return hi >= r.lo && lo <= r.hi; }

// Candidate lines of tile t under condition cd: the buckets within the
// cut-off reach of the tile.
__device__ __forceinline__ void tile_candidates(const GatherArgs& g, const CondDev& cd, int t, int64_t& tlo,
                                                int64_t& thi, int64_t& plo, int64_t& phi) {
  const ModelDev& m = g.m;
  tlo = (int64_t)t * g.tile_bins;
  thi = min(tlo + g.tile_bins, m.n_bins) - 1;
  const int64_t lo = tlo - cd.wbins;
  const int64_t blo = max<int64_t>(0, lo >= 0 ? lo / m.bucket_bins : -1);
  const int64_t bhi = min<int64_t>(m.n_buckets - 1, (thi + cd.wbins) / m.bucket_bins);
  plo = g.off[blo];
  phi = g.off[bhi + 1];
}

__device__ __forceinline__ float rcp32(float d) { return __builtin_amdgcn_rcpf(d); }

// Bin range where |x| < X, relative to k_c, in FP32 (the one-bin margin
// covers the rounding of a, b and of the quotient, whose reciprocal is the
// hardware's, within 1 ulp), clipped to the window.
__device__ __forceinline__ KRange x_range_f(float X, float a, float b, int kc, int klo, int khi) {
  KRange r;
  r.lo = 0x7fffffff;
  r.hi = -0x7fffffff;
  if (!(X > 0.0f)) return r;
  const float ra = rcp32(a);
  const float lo = fminf(fmaxf(floorf((b - X) * ra) - 1.0f, -1.0e9f), 1.0e9f);
  const float hi = fminf(fmaxf(ceilf((b + X) * ra) + 1.0f, -1.0e9f), 1.0e9f);
  const int l = max((int)lo + kc, klo - 1), h = min((int)hi + kc, khi + 1);
  if (l <= h) {
    r.lo = l;
    r.hi = h;
  }
  return r;
}

// Per-line inputs of the staging for one condition.  They are loaded in one
// round (the window test does not wait for its own load before the rest are
// issued), and for the narrow Gaussians one batch ahead of their use.
template <typename Real>
struct LineIn {
  int2 win;     // exact window of the line's cut-off class
  int kc;       // home bin
  float del;    // FP32 form: nu - nu_{k_c}
  double nu;
  Real S;       // intensity (FP32 form: scaled)
  float gref, nexp;
  double gpre;  // lifetime width, 0 without lifetimes
};
template <typename Real, int PROF>
__device__ __forceinline__ LineIn<Real> load_line(const GatherArgs& g, const CondDev& cd, int64_t p) {
  constexpr int B = base_profile(PROF);
  LineIn<Real> in;
  in.win = ((const int2*)g.rwin)[(int64_t)cd.cclass * g.max_lines + p];
  in.kc = g.rkc[p];
  in.nu = g.rnu[p];
  in.S = ((const Real*)g.rS)[(int64_t)cd.slot * g.max_lines + p];
  in.del = sizeof(Real) == 4 ? g.rdel[p] : 0.0f;
  if constexpr (B == XS_LORENTZ || B == XS_VOIGT) {
    in.gref = g.rgref[p];
    in.nexp = g.rnexp[p];
    in.gpre = g.rgpre ? g.rgpre[p] : 0.0;
  } else {
    in.gref = 0.0f;
    in.nexp = 0.0f;
    in.gpre = 0.0;
  }
  return in;
}

// Staging: does line p touch bins [tlo, thi] under condition cd?  Fills the
// record and returns its class for the tile row [tlo, tlo + rowb - 1].  The
// line's home bin and exact window come from the record pass; the FP32 form
// derives its constants in FP32 (relative error a few units of 1e-7, far
// inside its tolerance), the FP64 form in FP64.
template <typename Rec, int PROF>
__device__ int stage_line(const GatherArgs& g, const CondDev& cd, const LineIn<LReal<Rec>>& in, int64_t tlo,
                          int64_t thi, int rowb, Rec& r) {
  const ModelDev& m = g.m;
  const int2 win = in.win;
  if (win.x > win.y || win.y < tlo || win.x > thi) return kRowSkip;
  const int kc = in.kc;
  const int klo = max(win.x, (int)tlo), khi = min(win.y, (int)thi);
  r.klo = klo;
  r.khi = khi;
  r.flag = 0;
  r.kc = kc;
  const int lo = (int)tlo, hi = lo + rowb - 1;
  const bool inside = klo <= lo && khi >= hi;
  // Gaussian: the nonzero range nz; first formula when the row lies inside it.
  // Voigt: first formula when the row avoids n1, second when it avoids n2.
  KRange nz = KRange{klo, khi}, n1 = KRange{0x7fffffff, -0x7fffffff}, n2 = n1;
  bool can2 = false, gauss = false;
  if constexpr (sizeof(Rec) == sizeof(RecF)) {
    const float S = in.S;
    if (S == 0.0f) return kRowSkip;
    const float nu = (float)in.nu;
    float inv, y = 0.0f, c0;
    if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN) {
      const float alpha = PROF == XS_GAUSSIAN ? (float)cd.hwhm : nu * (float)cd.dop;
      inv = rcp32(alpha);
      c0 = S * (float)0.46971863934982566 * inv;           // sqrt(ln2/pi)/alpha
    } else {
      const float gamma = fmaf(in.gref * __builtin_amdgcn_exp2f(in.nexp * (float)(cd.lnTr / kLN2)),
                               (float)cd.pfac, (float)in.gpre);
      if (PROF == XS_LORENTZ) {
        inv = rcp32(gamma);
        c0 = S * (float)(1.0 / kPI) * inv;
      } else {
        inv = (float)0.83255461115769776 * rcp32(nu * (float)cd.dop);  // sqrt(ln2)/alpha
        y = gamma * inv;
        c0 = S * (float)0.56418958354775628 * inv;         // 1/(sg sqrt(2 pi))
      }
    }
    const float a = (float)m.dnu * inv, b = in.del * inv;
    r.a = a;
    r.nb = -b;
    r.jfb = (float)(lo - kc);  // integer, exact in FP32 within a window
    r.c0 = c0;
    r.y = y;
    const KRange none = KRange{0x7fffffff, -0x7fffffff};
    r.rB = none;
    r.rC = none;
    r.rD = none;
    if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN) {
      r.rB = x_range_f(12.649110640673518f, a, b, kc, klo, khi);  // 2^{-x^2} = 0 beyond sqrt(160)
      nz = r.rB;
      gauss = true;
    } else if (PROF == XS_VOIGT) {
      const float y2 = y * y;
      auto make = [&](double tau, double W) {
        const float cw = c0 * (float)(2.0 / kPI) * y * (float)W;
        return PairS{cw, cw * (float)(2.0 * tau), y2 - (float)tau, 4.0f * y2 * (float)tau};
      };
      r.A = make(GH::t2[0], GH::w2[0]);
      r.rB = x_range_f(sqrtf(fmaxf(900.9f - y2, 0.0f)), a, b, kc, klo, khi);
      // FP32 keeps s^2 + 4 y^2 tau finite for |x|, y < ~1e9; lines beyond that
      // (nu of a few 1e-3 cm^-1 or less) are evaluated in FP64.
      const float xmax = fmaxf(fabsf((float)(klo - kc) * a - b), fabsf((float)(khi - kc) * a - b));
      if (!(xmax <= 1.0e9f) || !(y <= 1.0e9f)) r.flag = 1;
      // a row in the one-pair region needs nothing more (lines are sorted by
      // home bin, so whole batches far from the tile stop here together)
      if (!r.flag && !meets(lo, hi, r.rB)) return inside ? kRowF1 : kRowF1M;
      r.B1 = make(GH::t4[0], GH::w4[0]);
      r.B2 = make(GH::t4[1], GH::w4[1]);
      r.rC = x_range_f(sqrtf(fmaxf(64.064f - y2, 0.0f)), a, b, kc, klo, khi);
      r.rD = x_range_f(sqrtf(fmaxf(36.036f - y2, 0.0f)), a, b, kc, klo, khi);
      n1 = r.rB;
      n2 = r.rC;
      can2 = true;
    }
  } else {
    const double S = in.S;
    if (S == 0.0) return kRowSkip;
    const double nu = in.nu;
    const double delta = nu - nu_of_bin(m.nu0, m.dnu, kc);
    const LineParams lp = line_params<PROF>(m, cd, nu, (double)in.gref, (double)in.nexp, in.gpre, S);
    const double a = m.dnu * lp.inv, b = delta * lp.inv;
    const double y2 = lp.y * lp.y;
    r.nu = nu;
    r.inv = lp.inv;
    r.y = lp.y;
    r.c0 = lp.c0;
    // the ranges only pick formulas; FP32 with the one-bin margin suffices
    const float af = (float)a, bf = (float)b, y2f = (float)y2;
    auto xr = [&](double rho) { return x_range_f(sqrtf(fmaxf((float)rho - y2f, 0.0f)), af, bf, kc, klo, khi); };
    if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN) {
      r.r[0] = x_range(sqrt(1100.0), a, b, kc, klo, khi);
      nz = r.r[0];
      gauss = true;
    } else if (PROF == XS_VOIGT) {
      r.a = a;
      r.xb = fma((double)(lo - kc), a, -b);
      // The first and second formulas share one reciprocal among four
      // points, a product of up to eight fourth-degree factors in x^2 + y^2:
      // lines reaching |x| or y beyond 1e9 (nu below about 1e-5 cm^-1) take
      // the general path, with a reciprocal per point.
      const double xmax = fmax(fabs((double)(klo - kc) * a - b), fabs((double)(khi - kc) * a - b));
      if (!(xmax <= 1.0e9) || !(lp.y <= 1.0e9)) r.flag = 1;
      r.r[0] = xr(9.0e6 * 1.001);
      if (!r.flag && !meets(lo, hi, r.r[0])) {  // one-pair row
        r.A = make_pair<double>(lp.c0, lp.y, GH::t2[0], GH::w2[0]);
        return inside ? kRowF1 : kRowF1M;
      }
      if (!r.flag && !meets(lo, hi, xr(4.5e4 * 1.001))) {  // three-point row
        r.C = make_poly3(lp.c0, lp.y);
        return inside ? kRowF15 : kRowF15M;
      }
      r.B = make_poly2(lp.c0, lp.y);
      r.r[1] = xr(4000.0 * 1.001);
      r.r[2] = xr(400.0 * 1.001);
      r.r[3] = xr(144.0 * 1.001);
      r.r[4] = xr(64.0 * 1.001);
      n1 = r.r[0];
      n2 = r.r[1];
      can2 = true;
    }
  }
  if (!meets(lo, hi, nz)) return kRowSkip;
  if (r.flag) return kRowGeneral;
  if (gauss) return (inside && nz.lo <= lo && nz.hi >= hi) ? kRowF1 : kRowGeneral;
  if (!meets(lo, hi, n1)) return inside ? kRowF1 : kRowF1M;
  if (can2 && !meets(lo, hi, n2)) return inside ? kRowF2 : kRowF2M;
  if constexpr (sizeof(Rec) == sizeof(RecD)) {
    if (PROF == XS_VOIGT && !meets(lo, hi, r.r[2])) return inside ? kRowF3 : kRowF3M;
  }
  return kRowGeneral;
}

// Staging for the binned profiles (as stage_line).  Record fields: a = h, the
// bin width in the profile's unit x; nb, jfb as above; c0 = S / dnu times the
// profile's normalisation (Gaussian 1/2, Lorentzian 1/pi, Voigt 1/sqrt(pi));
// y (Voigt).  Ranges, all by the bin's nearest point to the line centre:
//   Gaussian: rB / r[0] = bins whose mean is not zero in the precision;
//   Lorentzian: rB / r[0] = bins where the atan series does not hold;
//   Voigt: FP32 rB, rC, rD = |z|^2 below 900, 64, 36 (1, 2, 3 node pairs
//   outside them, the rational antiderivative inside rD); FP64 r[0..4] =
//   below 9e6, 6400, 400, 144, 64.
// A Voigt line takes a uniform class only where every node term's atan
// argument is positive and small enough for the series on every bin of that
// band: with the band's nearest |x| = sqrt(rho - y^2), the denominators
// y^2 + (x_a -+ s)(x_b -+ s) are at least dmin below.
template <typename Rec, int PROF>
__device__ int stage_line_bin(const GatherArgs& g, const CondDev& cd, const LineIn<LReal<Rec>>& in, int64_t tlo,
                              int64_t thi, int rowb, Rec& r) {
  constexpr int BASE = PROF - 4;
  const ModelDev& m = g.m;
  const int2 win = in.win;
  if (win.x > win.y || win.y < tlo || win.x > thi) return kRowSkip;
  const int kc = in.kc;
  const int klo = max(win.x, (int)tlo), khi = min(win.y, (int)thi);
  r.klo = klo;
  r.khi = khi;
  r.flag = 0;
  r.kc = kc;
  const int lo = (int)tlo, hi = lo + rowb - 1;
  const bool inside = klo <= lo && khi >= hi;
  const KRange none = KRange{0x7fffffff, -0x7fffffff}, all = KRange{klo, khi};
  KRange nz = all, n1 = none, n2 = none, n3 = all;
  bool can2 = false, gauss = false;
  // Largest atan argument of the row's bins (a bound; huge if the series
  // cannot apply): Voigt node terms y h / (y^2 + (x_a - s)(x_b - s)) with
  // nodes up to s, Lorentzian h / (1 + x_a x_b).  xr0, xr1: x at the row's
  // first and last bin.
  auto row_t = [&](double xr0, double xr1, double hh, double y, double s) {
    const double xn = xr0 > 0.0 ? xr0 : (xr1 < 0.0 ? -xr1 : 0.0);  // nearest bin centre
    const double en = fmax(xn - hh, 0.0);                              // its nearer edge
    double dmin;
    if (BASE == XS_LORENTZ) dmin = xn > hh ? 1.0 + en * (en + 2.0 * hh) : 1.0 - hh * hh;
    else dmin = en > s ? y * y + (en - s) * (en - s) : y * y - hh * hh;
    const double num = BASE == XS_LORENTZ ? 2.0 * hh : 2.0 * y * hh;
    return dmin > 0.0 ? num / dmin : 1.0e30;
  };
  // terms of the atan series for a bound t (relative error t^2/3, t^4/5,
  // t^8/9 for 1, 2, 4 terms); 0 if t is beyond the series
  auto terms = [](double t, bool f32) {
    if (f32) return t <= 3.0e-4 ? 1 : t <= 0.02 ? 2 : t <= 0.1 ? 4 : 0;
    return t <= 5.0e-8 ? 1 : t <= 2.5e-4 ? 2 : t <= 0.02 ? 4 : 0;
  };
  int nt1 = 0, nt2 = 0, nt3 = 0;
  if constexpr (sizeof(Rec) == sizeof(RecF)) {
    const float S = in.S;
    if (S == 0.0f) return kRowSkip;
    const float nu = (float)in.nu;
    float inv, y = 0.0f, c0;
    if (BASE == XS_DOPPLER || BASE == XS_GAUSSIAN) {
      const float alpha = BASE == XS_GAUSSIAN ? (float)cd.hwhm : nu * (float)cd.dop;
      inv = (float)0.83255461115769776 * rcp32(alpha);  // sqrt(ln2)/alpha
      c0 = S * (float)(0.5 / m.dnu);
    } else {
      const float gamma = fmaf(in.gref * __builtin_amdgcn_exp2f(in.nexp * (float)(cd.lnTr / kLN2)),
                               (float)cd.pfac, (float)in.gpre);
      if (BASE == XS_LORENTZ) {
        inv = rcp32(gamma);
        c0 = S * (float)(1.0 / (kPI * m.dnu));
      } else {
        inv = (float)0.83255461115769776 * rcp32(nu * (float)cd.dop);
        y = gamma * inv;
        c0 = S * (float)(0.56418958354775628 / m.dnu);  // 1/(sqrt(pi) dnu)
      }
    }
    const float a = (float)m.dnu * inv, b = in.del * inv, hh = 0.5f * a;
    r.a = a;
    r.nb = -b;
    r.jfb = (float)(lo - kc);
    r.c0 = c0;
    r.y = y;
    r.rB = none;
    r.rC = none;
    r.rD = none;
    if (BASE == XS_DOPPLER || BASE == XS_GAUSSIAN) {
      r.rB = x_range_f(10.1f + hh, a, b, kc, klo, khi);  // erfc(10.1) < 1e-45
      nz = r.rB;
      gauss = true;
    } else {
      const double xr0 = (double)(lo - kc) * a - b, xr1 = (double)(hi - kc) * a - b;
      if (BASE == XS_LORENTZ) {
        // series where 1 + x_a x_b >= h / 0.1, i.e. |x| >= sqrt(10 h - 1 + hh^2)
        r.rB = x_range_f(sqrtf(fmaxf(10.0f * a - 1.0f + hh * hh, 0.0f)) * 1.001f, a, b, kc, klo, khi);
        nt1 = terms(row_t(xr0, xr1, hh, y, 0.0), true);
        n1 = nt1 ? none : all;
      } else {
        const float y2 = y * y;
        auto X = [&](float rho) { return rho > y2 ? sqrtf(rho - y2) + hh : 0.0f; };
        r.rB = x_range_f(X(900.9f), a, b, kc, klo, khi);
        const float xmax = fmaxf(fabsf((float)(klo - kc) * a - b), fabsf((float)(khi - kc) * a - b)) + hh;
        if (!(xmax <= 1.0e9f) || !(y <= 1.0e9f)) r.flag = 1;
        nt1 = terms(row_t(xr0, xr1, hh, y, GH::s2[0]), true);
        if (!r.flag && nt1 && !meets(lo, hi, r.rB)) {  // a one-pair row: nothing more needed
          r.pad0 = nt1;
          return inside ? kRowF1 : kRowF1M;
        }
        r.rC = x_range_f(X(64.064f), a, b, kc, klo, khi);
        r.rD = x_range_f(X(36.036f), a, b, kc, klo, khi);
        nt2 = terms(row_t(xr0, xr1, hh, y, GH::s4[1]), true);
        n1 = nt1 ? r.rB : all;
        n2 = nt2 ? r.rC : all;
        can2 = true;
      }
    }
  } else {
    const double S = in.S;
    if (S == 0.0) return kRowSkip;
    const double nu = in.nu;
    const double delta = nu - nu_of_bin(m.nu0, m.dnu, kc);
    double inv, y = 0.0, c0;
    const double gamma = (BASE == XS_LORENTZ || BASE == XS_VOIGT)
                             ? (double)in.gref * exp((double)in.nexp * cd.lnTr) * cd.pfac + in.gpre
                             : 0.0;
    if (BASE == XS_DOPPLER || BASE == XS_GAUSSIAN) {
      const double alpha = BASE == XS_GAUSSIAN ? cd.hwhm : nu * cd.dop;
      inv = sqrt(kLN2) / alpha;
      c0 = S * 0.5 / m.dnu;
    } else if (BASE == XS_LORENTZ) {
      inv = 1.0 / gamma;
      c0 = S / (kPI * m.dnu);
    } else {
      inv = sqrt(kLN2) / (nu * cd.dop);
      y = gamma * inv;
      c0 = S / (sqrt(kPI) * m.dnu);
    }
    const double a = m.dnu * inv, b = delta * inv, hh = 0.5 * a;
    r.nu = nu;
    r.inv = inv;
    r.y = y;
    r.c0 = c0;
    const float af = (float)a, bf = (float)b;
    if (BASE == XS_DOPPLER || BASE == XS_GAUSSIAN) {
      r.r[0] = x_range(27.3 + hh, a, b, kc, klo, khi);  // erfc(27.3) underflows FP64
      nz = r.r[0];
      gauss = true;
    } else {
      const double xr0 = (double)(lo - kc) * a - b, xr1 = (double)(hi - kc) * a - b;
      if (BASE == XS_LORENTZ) {
        // series where 1 + x_a x_b >= h / 0.02
        r.r[0] = x_range(sqrt(fmax(50.0 * a - 1.0 + hh * hh, 0.0)) * 1.001, a, b, kc, klo, khi);
        nt1 = terms(row_t(xr0, xr1, hh, y, 0.0), false);
        n1 = nt1 ? none : all;
      } else {
        const double y2 = y * y;
        auto xr = [&](double rho) {
          return x_range_f(rho > y2 ? (float)(sqrt(rho - y2) + hh) : 0.0f, af, bf, kc, klo, khi);
        };
        r.r[0] = xr(9.0e6 * 1.001);
        r.r[1] = xr(6400.0 * 1.001);
        r.r[2] = xr(400.0 * 1.001);
        r.r[3] = xr(144.0 * 1.001);
        r.r[4] = xr(64.0 * 1.001);
        nt1 = terms(row_t(xr0, xr1, hh, y, GH::s2[0]), false);
        nt2 = terms(row_t(xr0, xr1, hh, y, GH::s4[1]), false);
        nt3 = terms(row_t(xr0, xr1, hh, y, GH::s6[2]), false);
        n1 = nt1 ? r.r[0] : all;
        n2 = nt2 ? r.r[1] : all;
        n3 = nt3 ? r.r[2] : all;
        can2 = true;
      }
    }
  }
  if (!meets(lo, hi, nz)) return kRowSkip;
  if (r.flag) return kRowGeneral;
  if (gauss) return (inside && nz.lo <= lo && nz.hi >= hi) ? kRowF1 : kRowGeneral;
  // the uniform classes carry their series length in pad0
  r.pad0 = nt1;
  if (!meets(lo, hi, n1)) return inside ? kRowF1 : kRowF1M;
  r.pad0 = nt2;
  if (can2 && !meets(lo, hi, n2)) return inside ? kRowF2 : kRowF2M;
  if constexpr (sizeof(Rec) == sizeof(RecD)) {
    r.pad0 = nt3;
    if (BASE == XS_VOIGT && !meets(lo, hi, n3)) return inside ? kRowF3 : kRowF3M;
  }
  return kRowGeneral;
}

// Staging for the pseudo-Voigts (as stage_line).  Record fields: the lane
// variable x = 2 d / f as for the Lorentzian (a, nb, jfb / nu, inv);
// c0 = S times the Lorentzian part's factor, y = S times the Gaussian part's;
// rB / r[0] = bins where the Gaussian part 2^{-x^2} is not zero in the
// precision.  First class: rows where only the Lorentzian part is left.
template <typename Rec, int PROF>
__device__ int stage_line_pv(const GatherArgs& g, const CondDev& cd, const LineIn<LReal<Rec>>& in, int64_t tlo,
                             int64_t thi, int rowb, Rec& r) {
  const ModelDev& m = g.m;
  const int2 win = in.win;
  if (win.x > win.y || win.y < tlo || win.x > thi) return kRowSkip;
  const int kc = in.kc;
  const int klo = max(win.x, (int)tlo), khi = min(win.y, (int)thi);
  r.klo = klo;
  r.khi = khi;
  r.flag = 0;
  r.kc = kc;
  const int lo = (int)tlo, hi = lo + rowb - 1;
  const bool inside = klo <= lo && khi >= hi;
  const double nu = in.nu;
  const double S = (double)in.S;
  if (S == 0.0) return kRowSkip;
  const double gamma = (double)in.gref * exp((double)in.nexp * cd.lnTr) * cd.pfac + in.gpre;
  const PVConst pc = pv_const(PROF, nu * cd.dop, gamma, S);
  const double delta = nu - nu_of_bin(m.nu0, m.dnu, kc);
  const double a = m.dnu * pc.inv, b = delta * pc.inv;
  KRange gz;
  if constexpr (sizeof(Rec) == sizeof(RecF)) {
    r.a = (float)a;
    r.nb = (float)(-b);
    r.jfb = (float)(lo - kc);
    r.c0 = (float)pc.cL;
    r.y = (float)pc.cG;
    r.rB = x_range_f(12.649110640673518f, (float)a, (float)b, kc, klo, khi);  // 2^{-x^2} = 0 beyond sqrt(160)
    gz = r.rB;
  } else {
    r.nu = nu;
    r.inv = pc.inv;
    r.c0 = pc.cL;
    r.y = pc.cG;
    r.r[0] = x_range(sqrt(1100.0), a, b, kc, klo, khi);
    gz = r.r[0];
  }
  if (!meets(lo, hi, gz)) return inside ? kRowF1 : kRowF1M;
  return kRowGeneral;
}

// ---- far-region evaluators ------------------------------------------------
// The hardware FP64 reciprocal has a relative error below 5e-8 on gfx950
// (measured over 1e6 arguments spanning 1e-30..1e30); one Newton step
// squares it, to below 3e-15.
__device__ __forceinline__ double rcp64(double d) {
  const double r = __builtin_amdgcn_rcp(d);
  return fma(r, fma(-d, r, 1.0), r);
}

template <typename R>
__device__ __forceinline__ R pair_term(const Pair<R>& P, R x) {
  const R s = fma(x, x, P.h);
  const R n = fma(P.cw, s, P.cwt);
  const R d = fma(s, s, P.c);
  if constexpr (sizeof(R) == 4) return n * rcp32(d);
  else return n * rcp64(d);
}
// two pairs as one fraction (FP64 only: the product of the d_j stays finite)
__device__ __forceinline__ double pair2_term(const Pair<double>& P, const Pair<double>& Q, double x) {
  const double s1 = fma(x, x, P.h), s2 = fma(x, x, Q.h);
  const double n1 = fma(P.cw, s1, P.cwt), d1 = fma(s1, s1, P.c);
  const double n2 = fma(Q.cw, s2, Q.cwt), d2 = fma(s2, s2, Q.c);
  return fma(n1, d2, n2 * d1) * rcp64(d1 * d2);
}
__device__ __forceinline__ double poly2_term(const Poly2& B, double x) {
  double N, D;
  poly2_nd(B, x, N, D);
  return N * rcp64(D);
}
// NP node pairs from y (near-core chunks of the FP64 form; out of line, rare)
template <int NP>
__device__ __noinline__ double gh_pairs_y(double c0, double y, double u) {
  const double* tau = gh_tau<NP>();
  const double* W = gh_w<NP>();
  const double y2 = y * y, cy = c0 * (y * (2.0 / kPI));
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    const double p = y2 + tau[j];
    s = fma(cy * W[j] * (u + p), rcp64(fma(u, u + (2.0 * y2 - 2.0 * tau[j]), p * p)), s);
  }
  return s;
}

// Three node pairs (|z|^2 >= 36, relative error below 2e-7) from c0 and y,
// FP32 form.
__device__ __forceinline__ float gh3_f32(float u, float y, float c0) {
  const float y2 = y * y;
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const float tau = (float)GH::t6[j];
    const float p = y2 + tau;
    s = fmaf((float)GH::w6[j] * (u + p), rcp32(fmaf(u, u + (2.0f * y2 - 2.0f * tau), p * p)), s);
  }
  return c0 * (float)(2.0 / kPI) * y * s;
}

// Work item = (tile, condition, slice of the tile's candidate lines); one
// wave per item.  Lane l owns the bins tlo + 64 j + l, j = 0..M-1, so each
// "chunk" j is 64 consecutive bins and every per-chunk decision (window,
// band, zero skip) is a scalar compare of the chunk's range with the line's
// precomputed ranges.  Each batch of up to 64 candidates is staged one line
// per lane, and the survivors are compacted into LDS grouped by class (a
// ballot and mbcnt per class), so the first- and second-formula lines run in
// tight loops with no per-line branch.  A tile split over several items
// writes FP64 partial rows that k_reduce adds in item order.
// (The FP64 forms ask for at least three waves per SIMD and the FP32 binned
// Voigt for four: 6-8% faster than their register use would otherwise allow,
// with a few spills outside the hot loops.)
template <typename Real, int PROF, int M>
__global__ __launch_bounds__(64, sizeof(Real) == 8 ? 3 : (PROF == XS_BIN_VOIGT ? 4 : 1)) void k_gather(GatherArgs g) {
  using Rec = typename std::conditional<sizeof(Real) == 4, RecF, RecD>::type;
  constexpr bool F32 = sizeof(Real) == 4;
  constexpr int ROWB = 64 * M;
  __shared__ Rec srec[64];
  // FP32 Voigt: the points of a core chunk with |z|^2 < 36 go to a queue and
  // are evaluated 64 at a time by the rational approximation, their values
  // added into a row buffer; the chunk's other lanes take three node pairs.
  // Only these points need the approximation, while a core chunk spans 64
  // points (about five times as many for the benchmark's lines).
  constexpr bool CQ = F32 && PROF == XS_VOIGT;
  constexpr int CQN = CQ ? 128 : 1;
  __shared__ float cq_x[CQN], cq_y[CQN], cq_c[CQN];
  __shared__ int cq_b[CQN];
  __shared__ float rowbuf[CQ ? ROWB : 1];
  // Gaussian lines narrower than the tile (the usual Doppler case: a few
  // tens of nonzero points) add their nonzero points into an LDS row instead
  // of testing every chunk of the row per line: one line per lane where it
  // has at most kLaneSpan such points, else 64 points per wave step.
  constexpr bool GBIN = PROF == XS_BIN_DOPPLER || PROF == XS_BIN_GAUSSIAN;
  constexpr bool GN = PROF == XS_DOPPLER || PROF == XS_GAUSSIAN || GBIN;
  constexpr int kLaneSpan = 96;
  // The row is FP64 in both forms.  With an FP32 row the lanes' LDS float
  // adds held the FP32 waves three quarters of the time (about 16 cycles per
  // LDS instruction, against 2.8 for the FP64 form's double adds; spreading
  // the lanes over four copies of the row did not help), and the pass took
  // 3.7 ms on a 1e7-line chunk of the two-temperature workload, 0.7 ms with
  // double adds.  An FP64 row also needs no per-batch fold.
  __shared__ double gbuf[GN ? ROWB : 1];

  const int lane = threadIdx.x;
  const ModelDev& m = g.m;
  const int n_items = uni(g.ib[g.n_ct]);
  const int64_t chunk = *(const int64_t*)(g.counter + 4);
  const float lane_off = (float)lane;
  float lane_j[M];  // lane + 64 j: a point's offset from the tile's first point
  double lane_d[M];
#pragma unroll
  for (int j = 0; j < M; ++j) {
    lane_j[j] = (float)(lane + 64 * j);
    lane_d[j] = (double)(lane + 64 * j);
  }
  int item = blockIdx.x;
  for (;;) {
    if (g.persistent) {
      int v = 0;
      if (lane == 0) v = atomicAdd(g.counter, 1);
      item = __shfl(v, 0, 64);
    }
    item = uni(item);
    if (item >= n_items) return;
    // (tile, condition) of the item: the last ct with ib[ct] <= item
    int lo = 0, hi = g.n_ct - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (g.ib[mid] <= item) lo = mid;
      else hi = mid - 1;
    }
    const int ct = uni(lo);
    const int jpart = item - g.ib[ct];
    const int nch = g.ib[ct + 1] - g.ib[ct];
    const int c = ct % m.n_cond, t = ct / m.n_cond;
    const CondDev cd = g.cond[c];
    int64_t tlo, thi, plo, phi;
    tile_candidates(g, cd, t, tlo, thi, plo, phi);
    const int64_t q0 = plo + (int64_t)jpart * chunk;
    const int64_t q1 = min(phi, q0 + chunk);
    const int row_lo = (int)tlo;
    const int my0 = row_lo + lane;  // bin of chunk 0 of this lane
    // a masked row skips its 64-point chunks that lie wholly outside the
    // window (a uniform branch): about 3 of a window's 80 chunks
    auto off_chunk = [&](auto masked, int j, int klo, int khi) {
      const int cl = row_lo + 64 * j;
      return masked && (cl + 63 < klo || cl > khi);
    };

    double acc64[M];
    float acc32[M];
    double nuk[M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
      acc64[j] = 0.0;
      acc32[j] = 0.0f;
      if (!F32) nuk[j] = nu_of_bin(m.nu0, m.dnu, my0 + 64 * j);
      if constexpr (CQ) rowbuf[lane + 64 * j] = 0.0f;
      if constexpr (GN) gbuf[lane + 64 * j] = 0.0;
    }
    // ring of queued core points: qn entries from qh (wave-uniform).  The
    // block is one wave, whose LDS accesses complete in issue order, so a
    // compiler-level wave barrier orders the lanes' pushes and pops.
    int qh = 0, qn = 0;
    // evaluate the n (<= 64) oldest entries into the row buffer
    auto cq_pop = [&](int n) {
      if constexpr (CQ) {
        __builtin_amdgcn_wave_barrier();
        if (lane < n) {
          const int e = (qh + lane) & (CQN - 1);
          double wr, wi;
          w_weideman<24>((double)cq_x[e], (double)cq_y[e], wr, wi);
          atomicAdd(&rowbuf[cq_b[e]], (float)((double)cq_c[e] * wr));
        }
        __builtin_amdgcn_wave_barrier();
        qh = (qh + n) & (CQN - 1);
        qn -= n;
      }
    };
    // value of a Gaussian line at point k of the row: the profile (sampled)
    // or the mean over the point's bin (binned), times the line's constant
    auto gval = [&](const Rec& rr, int k) -> double {
      if constexpr (GBIN) {
        if constexpr (F32) {
          const float x = fmaf(rr.jfb + (float)(k - row_lo), rr.a, rr.nb);
          return (double)(rr.c0 * erf_bin<float>(x, 0.5f * rr.a));
        } else {
          double x;
          {
#pragma clang fp contract(off)
            x = (nu_of_bin(m.nu0, m.dnu, k) - rr.nu) * rr.inv;
          }
          return rr.c0 * erf_bin<double>(x, 0.5 * (m.dnu * rr.inv));
        }
      } else if constexpr (F32) {
        const float x = fmaf(rr.jfb + (float)(k - row_lo), rr.a, rr.nb);
        return (double)(rr.c0 * __builtin_amdgcn_exp2f(-(x * x)));
      } else {
        double x;
        {
#pragma clang fp contract(off)
          x = (nu_of_bin(m.nu0, m.dnu, k) - rr.nu) * rr.inv;
        }
        return rr.c0 * exp2(-(x * x));
      }
    };
    // general-class Gaussian lines wider than kLaneSpan points: the points of
    // the row inside both the window and the range where 2^{-x^2} is not
    // zero, 64 at a time; every point outside that range would add an exact
    // zero.  Within one wave the LDS adds of successive lines complete in
    // issue order.
    auto gauss_rows = [&](int l0, int l1) {
      if constexpr (GN) {
        for (int l = l0; l < l1; ++l) {
          const Rec& rr = srec[l];
          int kl, kh;
          if constexpr (F32) {
            kl = max(uni(rr.klo), uni(rr.rB.lo));
            kh = min(uni(rr.khi), uni(rr.rB.hi));
          } else {
            kl = max(uni(rr.klo), uni(rr.r[0].lo));
            kh = min(uni(rr.khi), uni(rr.r[0].hi));
          }
          kl = max(kl, row_lo);
          kh = min(kh, row_lo + ROWB - 1);
          for (int k0 = kl; k0 <= kh; k0 += 64) {
            const int k = k0 + lane;
            if (k <= kh) atomicAdd(&gbuf[k - row_lo], gval(rr, k));
          }
        }
      }
    };

    for (int64_t p0 = q0; p0 < q1; p0 += 64) {
      // ---- stage: exact window test and class, compaction into LDS by class ----
      Rec r;
      int cls = kRowSkip;
      const int64_t p = p0 + lane;
      if (p < q1) {
        const LineIn<Real> in = load_line<Real, PROF>(g, cd, p);
        if constexpr (PROF >= XS_PV_THOMPSON) cls = stage_line_pv<Rec, PROF>(g, cd, in, tlo, thi, ROWB, r);
        else if constexpr (PROF >= XS_BIN_DOPPLER) cls = stage_line_bin<Rec, PROF>(g, cd, in, tlo, thi, ROWB, r);
        else cls = stage_line<Rec, PROF>(g, cd, in, tlo, thi, ROWB, r);
      }
      if constexpr (GN) {
        // A narrow Gaussian (at most kLaneSpan nonzero points in the row)
        // stays on its lane, which adds its points into the LDS row; each
        // lane starts at its own offset within its points so that lanes of
        // neighbouring lines rarely add to one point in the same step.
        // Wider ones take the wave-wide path below.
        int kl = 0, n = 0;
        if (cls == kRowGeneral) {
          KRange R;
          if constexpr (F32) R = r.rB;
          else R = r.r[0];
          kl = max(r.klo, R.lo);
          n = min(r.khi, R.hi) - kl + 1;
          if (n <= kLaneSpan) cls = kRowSkip;
          else n = 0;
        }
        if (__ballot(n > 0)) {
          int i = n > 0 ? lane % n : 0;
          for (int it = 0; it < n; ++it) {
            const int k = kl + i;
            atomicAdd(&gbuf[k - row_lo], gval(r, k));
            i = (i + 1 == n) ? 0 : i + 1;
          }
        }
      }
      // LDS order: F1 (FP32 Voigt: those taking x from the tile's first
      // point, then the others) | F1M | F15 | F15M (FP64 Voigt) | F2 | F2M |
      // F3 | F3M (FP64) | general
      bool xb_ok = false;
      if constexpr (F32 && PROF == XS_VOIGT) xb_ok = cls == kRowF1 && r.a <= 2.0f;
      constexpr bool TP = !F32 && PROF == XS_VOIGT;  // three-point rows exist
      const unsigned long long b1x = __ballot(xb_ok);
      const unsigned long long b1 = __ballot(cls == kRowF1 && !xb_ok);
      const unsigned long long b1m = __ballot(cls == kRowF1M);
      const unsigned long long b15 = TP ? __ballot(cls == kRowF15) : 0ull;
      const unsigned long long b15m = TP ? __ballot(cls == kRowF15M) : 0ull;
      const unsigned long long b2 = __ballot(cls == kRowF2);
      const unsigned long long b2m = __ballot(cls == kRowF2M);
      const unsigned long long b3 = F32 ? 0ull : __ballot(cls == kRowF3);
      const unsigned long long b3m = F32 ? 0ull : __ballot(cls == kRowF3M);
      const unsigned long long bg = __ballot(cls == kRowGeneral);
      const int e1x = __popcll(b1x), e1 = e1x + __popcll(b1), e1m = e1 + __popcll(b1m);
      const int e15 = e1m + __popcll(b15), e15m = e15 + __popcll(b15m), e2 = e15m + __popcll(b2);
      const int e2m = e2 + __popcll(b2m), e3 = e2m + __popcll(b3), e3m = e3 + __popcll(b3m);
      const int eg = e3m + __popcll(bg);
      if (eg == 0) continue;
      unsigned long long mine = bg;
      int base = e3m;
      if (xb_ok) { mine = b1x; base = 0; }
      else if (cls == kRowF1) { mine = b1; base = e1x; }
      else if (cls == kRowF1M) { mine = b1m; base = e1; }
      else if (TP && cls == kRowF15) { mine = b15; base = e1m; }
      else if (TP && cls == kRowF15M) { mine = b15m; base = e15; }
      else if (cls == kRowF2) { mine = b2; base = e15m; }
      else if (cls == kRowF2M) { mine = b2m; base = e2; }
      else if (cls == kRowF3) { mine = b3; base = e2m; }
      else if (cls == kRowF3M) { mine = b3m; base = e3; }
      const int slot = base + __builtin_amdgcn_mbcnt_hi((unsigned)(mine >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((unsigned)mine, 0u));
      __syncthreads();
      if (cls != kRowSkip) srec[slot] = r;
      __syncthreads();

      if constexpr (PROF >= XS_PV_THOMPSON) {
        // ---- pseudo-Voigts: cL/(1 + x^2) + cG 2^{-x^2} ----
        auto xv = [&](const Rec& rr, int j) -> Real {
          if constexpr (F32) {
            return fmaf(rr.jfb + lane_off + (float)(64 * j), rr.a, rr.nb);
          } else {
#pragma clang fp contract(off)
            return (nuk[j] - rr.nu) * rr.inv;
          }
        };
        auto addv = [&](int j, Real v) {
          if constexpr (F32) acc32[j] += v;
          else acc64[j] += v;
        };
        // rows where the Gaussian part is zero: the Lorentzian part alone
        auto lor_rows = [&](int l0, int l1, auto masked) {
          for (int l = l0; l < l1; ++l) {
            const Rec& rr = srec[l];
            const Real c0 = rr.c0;
            int klo = 0, khi = 0;
            if (masked) {
              klo = uni(rr.klo);
              khi = uni(rr.khi);
            }
#pragma unroll
            for (int j = 0; j < M; ++j) {
              if (off_chunk(masked, j, klo, khi)) continue;
              const Real x = xv(rr, j);
              const Real t = c0 * rcp_r<Real>(fma(x, x, (Real)1));
              const int k = my0 + 64 * j;
              addv(j, (!masked || (k >= klo && k <= khi)) ? t : (Real)0);
            }
          }
        };
        lor_rows(0, e1, std::false_type());
        lor_rows(e1, e1m, std::true_type());
        for (int l = e3m; l < eg; ++l) {
          const Rec& rr = srec[l];
          const int klo = uni(rr.klo), khi = uni(rr.khi);
          KRange R0;
          if constexpr (F32) R0 = KRange{uni(rr.rB.lo), uni(rr.rB.hi)};
          else R0 = KRange{uni(rr.r[0].lo), uni(rr.r[0].hi)};
#pragma unroll
          for (int j = 0; j < M; ++j) {
            const int cl = row_lo + 64 * j, ch = cl + 63;
            if (ch < klo || cl > khi) continue;
            const bool full = cl >= klo && ch <= khi;
            const int k = my0 + 64 * j;
            const Real x = xv(rr, j);
            Real v = rr.c0 * rcp_r<Real>(fma(x, x, (Real)1));
            if (meets(cl, ch, R0)) {
              if constexpr (F32) v = fmaf(rr.y, __builtin_amdgcn_exp2f(-(x * x)), v);
              else v = fma(rr.y, exp2(-(x * x)), v);
            }
            addv(j, (full || (k >= klo && k <= khi)) ? v : (Real)0);
          }
        }
        if constexpr (F32) {
#pragma unroll
          for (int j = 0; j < M; ++j) {
            acc64[j] += (double)acc32[j];
            acc32[j] = 0.0f;
          }
        }
      } else if constexpr (PROF >= XS_BIN_DOPPLER) {
        // ---- binned profiles: bin means from the closed-form bin integrals ----
        constexpr int BASE = PROF - 4;
        constexpr bool GAU = BASE == XS_DOPPLER || BASE == XS_GAUSSIAN;
        // x of chunk j, and the bin width h, in the profile's unit
        auto xof = [&](const Rec& rr, int j) -> Real {
          if constexpr (F32) {
            return fmaf(rr.jfb + lane_off + (float)(64 * j), rr.a, rr.nb);
          } else {
#pragma clang fp contract(off)
            return (nuk[j] - rr.nu) * rr.inv;
          }
        };
        auto hof = [&](const Rec& rr) -> Real {
          if constexpr (F32) return rr.a;
          else return m.dnu * rr.inv;
        };
        auto add = [&](int j, Real v) {
          if constexpr (F32) acc32[j] += v;
          else acc64[j] += v;
        };
        // Uniform classes.  With 1 or 2 terms of the atan series, a Voigt
        // node pair +-s takes one reciprocal: den-+ = P -+ 2 s x with
        // P = x^2 + (y^2 + s^2 - hh^2), so t+ + t- = 2 y h P / D and
        // t+ t- = (y h)^2 / D, D = den- den+ = P^2 - 4 s^2 x^2; the series
        // atan(t+) + atan(t-) = (t+ + t-)(1 - (t+ + t-)^2/3 + t+ t-) + O(t^5).
        // The Lorentzian likewise: t = h / (x^2 + 1 - hh^2).
        auto uniform_bin = [&](int l0, int l1, auto masked, auto npairs) {
          constexpr int NP = decltype(npairs)::value;
          const double* tau = gh_tau<NP>();
          for (int l = l0; l < l1; ++l) {
            const Rec& rr = srec[l];
            const Real h = hof(rr), hh = (Real)0.5 * h, c0 = rr.c0, y = rr.y, y2 = y * y, yh = y * h;
            int klo = 0, khi = 0;
            if (masked) {
              klo = uni(rr.klo);
              khi = uni(rr.khi);
            }
            const int nt = GAU ? 4 : uni(rr.pad0);
            auto run = [&](auto nterms) {
              constexpr int NT = decltype(nterms)::value;
              if constexpr (BASE == XS_VOIGT && NP == 1 && NT == 1) {
                // one node pair, first series term: c0 2 y h (W/pi) P/D with
                // P = x^2 + y^2 + tau - hh^2 and D = P^2 - 4 tau x^2, in the
                // shifted variable s = x^2 + (y^2 - tau - hh^2):
                // P = s + 2 tau, D = s^2 + 4 tau (y^2 - hh^2) (the same
                // fraction; the per-point work of the sampled far form)
                const double t0 = tau[0];
                const Real sh = y2 - (Real)t0 - hh * hh, cc = (Real)(4.0 * t0) * (y2 - hh * hh);
                const Real K = c0 * (Real)2 * yh * (Real)(gh_w<1>()[0] / kPI), K2 = K * (Real)(2.0 * t0);
#pragma unroll
                for (int j = 0; j < M; ++j) {
                  if (off_chunk(masked, j, klo, khi)) continue;
                  const Real x = xof(rr, j);
                  const Real sv = fma(x, x, sh);
                  const Real v = fma(K, sv, K2) * rcp_r<Real>(fma(sv, sv, cc));
                  const int k = my0 + 64 * j;
                  add(j, (!masked || (k >= klo && k <= khi)) ? v : (Real)0);
                }
                return;
              }
              Real cp[NP];
#pragma unroll
              for (int q = 0; q < NP; ++q) cp[q] = (BASE == XS_LORENTZ) ? fma(-hh, hh, (Real)1) : y2 + ((Real)tau[q] - hh * hh);
#pragma unroll
              for (int j = 0; j < M; ++j) {
                if (off_chunk(masked, j, klo, khi)) continue;
                const Real x = xof(rr, j);
                Real t;
                if constexpr (GAU) {
                  t = erf_bin<Real>(x, hh);
                } else if constexpr (BASE == XS_LORENTZ) {
                  const Real tl = h * rcp_r<Real>(fma(x, x, cp[0]));
                  if constexpr (NT == 1) t = tl;
                  else if constexpr (NT == 2) t = tl * fma(tl * tl, (Real)(-1.0 / 3.0), (Real)1);
                  else t = atan_series<Real>(tl);
                } else if constexpr (NT == 4) {
                  t = vpairs_bin<NP, true, Real>(x - hh, x + hh, yh, y2);
                } else {
                  const Real u = x * x;
                  t = (Real)0;
#pragma unroll
                  for (int q = 0; q < NP; ++q) {
                    const Real P = u + cp[q];
                    const Real iD = rcp_r<Real>(fma(P, P, u * (Real)(-4.0 * tau[q])));
                    Real e;
                    if constexpr (NT == 1) {
                      e = P * iD;
                    } else {
                      const Real A = yh * iD, e1 = (Real)2 * P * A;
                      e = P * iD * fma(e1 * e1, (Real)(-1.0 / 3.0), (Real)1 + yh * A);
                    }
                    t = fma((Real)(gh_w<NP>()[q] / kPI), e, t);
                  }
                  t *= (Real)2 * yh;
                }
                const int k = my0 + 64 * j;
                add(j, (!masked || (k >= klo && k <= khi)) ? c0 * t : (Real)0);
              }
            };
            if (nt == 1) run(std::integral_constant<int, 1>());
            else if (nt == 2) run(std::integral_constant<int, 2>());
            else run(std::integral_constant<int, 4>());
          }
        };
        using P1 = std::integral_constant<int, 1>;
        using P2 = std::integral_constant<int, 2>;
        using P3 = std::integral_constant<int, 3>;
        uniform_bin(0, e1, std::false_type(), P1());
        uniform_bin(e1, e1m, std::true_type(), P1());
        if constexpr (BASE == XS_VOIGT) {
          uniform_bin(e1m, e2, std::false_type(), P2());
          uniform_bin(e2, e2m, std::true_type(), P2());
          if constexpr (!F32) {
            uniform_bin(e2m, e3, std::false_type(), P3());
            uniform_bin(e3, e3m, std::true_type(), P3());
          }
        }
        // general path: band per chunk (nearest point of each bin), the exact
        // angle where the series does not hold
        if constexpr (GBIN) gauss_rows(e3m, eg);
        else for (int l = e3m; l < eg; ++l) {
          const Rec& rr = srec[l];
          const Real h = hof(rr), hh = (Real)0.5 * h, c0 = rr.c0, y = rr.y, y2 = y * y, yh = y * h;
          const int klo = uni(rr.klo), khi = uni(rr.khi);
          KRange R0, R1, R2, R3, R4;
          if constexpr (F32) {
            R0 = KRange{uni(rr.rB.lo), uni(rr.rB.hi)};
            R1 = KRange{uni(rr.rC.lo), uni(rr.rC.hi)};
            R2 = KRange{uni(rr.rD.lo), uni(rr.rD.hi)};
            R3 = R2;
            R4 = R2;
          } else {
            R0 = KRange{uni(rr.r[0].lo), uni(rr.r[0].hi)};
            R1 = KRange{uni(rr.r[1].lo), uni(rr.r[1].hi)};
            R2 = KRange{uni(rr.r[2].lo), uni(rr.r[2].hi)};
            R3 = KRange{uni(rr.r[3].lo), uni(rr.r[3].hi)};
            R4 = KRange{uni(rr.r[4].lo), uni(rr.r[4].hi)};
          }
          const bool flag = F32 && BASE == XS_VOIGT && uni(rr.flag);
#pragma unroll
          for (int j = 0; j < M; ++j) {
            const int cl = row_lo + 64 * j, ch = cl + 63;
            if (ch < klo || cl > khi) continue;
            const bool full = cl >= klo && ch <= khi;
            const int k = my0 + 64 * j;
            const Real x = xof(rr, j);
            Real v;
            if constexpr (GAU) {
              if (!meets(cl, ch, R0)) continue;  // every bin mean of the chunk is 0
              v = erf_bin<Real>(x, hh);
            } else if constexpr (BASE == XS_LORENTZ) {
              v = !meets(cl, ch, R0) ? atan_series<Real>(h * rcp_r<Real>(fma(x - hh, x + hh, (Real)1)))
                                     : lor_bin<Real>(x, hh, h);
            } else {
              bool wide = false;
              if constexpr (F32) {
                if (flag) {
                  // |x| or y beyond FP32's safe range: the FP64 evaluator
                  const double xd = (double)(k - rr.kc) * (double)rr.a + (double)rr.nb;
                  v = (full || (k >= klo && k <= khi)) ? (Real)voigt_bin_f64(xd, (double)y, 0.5 * (double)h)
                                                       : (Real)0;
                  wide = true;
                }
              }
              if (wide) {
              } else if (!meets(cl, ch, R0)) {
                v = vpairs_bin<1, false, Real>(x - hh, x + hh, yh, y2);
              } else if (!meets(cl, ch, R1)) {
                v = vpairs_bin<2, false, Real>(x - hh, x + hh, yh, y2);
              } else if (!meets(cl, ch, R2)) {
                v = vpairs_bin<3, false, Real>(x - hh, x + hh, yh, y2);
              } else if constexpr (F32) {
                // a chunk that reaches |z|^2 < 36: the rational antiderivative
                // on every lane (valid everywhere, so no divergence)
                v = (Real)voigt_bin_core<24>((double)x, (double)y, 0.5 * (double)h);
              } else {
                const double xn = fmax(fabs(x) - hh, 0.0);
                if (!meets(cl, ch, R3)) v = vpairs_bin<4, false, Real>(x - hh, x + hh, yh, y2);
                else if (!meets(cl, ch, R4) || fma(xn, xn, y2) >= 64.0)
                  v = vpairs_bin<6, false, Real>(x - hh, x + hh, yh, y2);
                else v = voigt_bin_core<40>(x, y, hh);
              }
            }
            add(j, (full || (k >= klo && k <= khi)) ? c0 * v : (Real)0);
          }
        }
        if constexpr (F32) {
#pragma unroll
          for (int j = 0; j < M; ++j) {
            acc64[j] += (double)acc32[j];
            acc32[j] = 0.0f;
          }
        }
      } else if constexpr (F32) {
        // x = (k - k_c) a - b, with k - k_c = (tlo - k_c) + (offset in tile):
        // integers, exact in FP32 within a window
        // ---- first formula; then the same under the window mask ----
        auto first = [&](int l0, int l1, auto masked, auto from_xb) {
          for (int l = l0; l < l1; ++l) {
            const RecF& rr = srec[l];
            const float a = rr.a, nb = rr.nb, jf0 = rr.jfb + lane_off;
            int klo = 0, khi = 0;
            if (masked) {
              klo = uni(rr.klo);
              khi = uni(rr.khi);
            }
            if (PROF == XS_LORENTZ) {
              const float c0 = rr.c0;
#pragma unroll
              for (int j = 0; j < M; ++j) {
                if (off_chunk(masked, j, klo, khi)) continue;
                const float x = fmaf(jf0 + (float)(64 * j), a, nb);
                if (!masked) {
                  acc32[j] = fmaf(c0, rcp32(fmaf(x, x, 1.0f)), acc32[j]);
                } else {
                  const int k = my0 + 64 * j;
                  const float t = c0 * rcp32(fmaf(x, x, 1.0f));
                  acc32[j] += (k >= klo && k <= khi) ? t : 0.0f;
                }
              }
            } else if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN) {
              const float c0 = rr.c0;
#pragma unroll
              for (int j = 0; j < M; ++j) {
                const float x = fmaf(jf0 + (float)(64 * j), a, nb);
                acc32[j] = fmaf(c0, __builtin_amdgcn_exp2f(-(x * x)), acc32[j]);
              }
            } else {
              const PairS A = rr.A;
              // x from the tile's first point xb = x(tlo) (rows sorted first
              // by the compaction): one operation per line instead of one per
              // chunk.  Rounding xb costs an absolute error eps |xb| <=
              // eps (|x| + 255 a) in x; in the one-pair region
              // (s = x^2 + h >= 899.5) that moves s by a relative
              // 2 eps (1 + 255 a/30) at most, below 2.2e-6 for a <= 2.  Wider
              // steps (a > 2: lines narrower than half a bin) keep the exact
              // fma over the integer offset.
              auto run = [&](auto xof) {
#pragma unroll
                for (int j = 0; j < M; ++j) {
                  if (off_chunk(masked, j, klo, khi)) continue;
                  const float x = xof(j);
                  const float s = fmaf(x, x, A.h);
                  if (!masked) {
                    acc32[j] = fmaf(fmaf(A.cw, s, A.cwt), rcp32(fmaf(s, s, A.c)), acc32[j]);
                  } else {
                    const int k = my0 + 64 * j;
                    const float t = fmaf(A.cw, s, A.cwt) * rcp32(fmaf(s, s, A.c));
                    acc32[j] += (k >= klo && k <= khi) ? t : 0.0f;
                  }
                }
              };
              if constexpr (decltype(from_xb)::value) {
                const float xb = fmaf(rr.jfb, a, nb);
                run([&](int j) { return fmaf(lane_j[j], a, xb); });
              } else {
                run([&](int j) { return fmaf(jf0 + (float)(64 * j), a, nb); });
              }
            }
          }
        };
        first(0, e1x, std::false_type(), std::true_type());
        first(e1x, e1, std::false_type(), std::false_type());
        first(e1, e1m, std::true_type(), std::false_type());
        // ---- second formula (Voigt: two node pairs), unmasked then masked ----
        if (PROF == XS_VOIGT) {
          auto second = [&](int l0, int l1, auto masked) {
            for (int l = l0; l < l1; ++l) {
              const RecF& rr = srec[l];
              const float a = rr.a, nb = rr.nb, jf0 = rr.jfb + lane_off;
              const PairS B1 = rr.B1, B2 = rr.B2;
              int klo = 0, khi = 0;
              if (masked) {
                klo = uni(rr.klo);
                khi = uni(rr.khi);
              }
#pragma unroll
              for (int j = 0; j < M; ++j) {
                if (off_chunk(masked, j, klo, khi)) continue;
                const float x = fmaf(jf0 + (float)(64 * j), a, nb);
                const float t = pair_term_s(B1, x) + pair_term_s(B2, x);
                const int k = my0 + 64 * j;
                acc32[j] += (!masked || (k >= klo && k <= khi)) ? t : 0.0f;
              }
            }
          };
          second(e1m, e2, std::false_type());
          second(e2, e2m, std::true_type());
        }
        // ---- general path: per-chunk decisions ----
        if constexpr (GN) gauss_rows(e3m, eg);
        else for (int l = e3m; l < eg; ++l) {
          const RecF& rr = srec[l];
          const float a = rr.a, nb = rr.nb, jf0 = rr.jfb + lane_off;
          const int klo = uni(rr.klo), khi = uni(rr.khi);
          const KRange rB = {uni(rr.rB.lo), uni(rr.rB.hi)};
          const KRange rC = {uni(rr.rC.lo), uni(rr.rC.hi)};
          const KRange rD = {uni(rr.rD.lo), uni(rr.rD.hi)};
          const bool flag = PROF == XS_VOIGT && uni(rr.flag);
#pragma unroll
          for (int j = 0; j < M; ++j) {
            const int cl = row_lo + 64 * j, ch = cl + 63;
            if (ch < klo || cl > khi) continue;
            const bool full = cl >= klo && ch <= khi;
            const int k = my0 + 64 * j;
            const float x = fmaf(jf0 + (float)(64 * j), a, nb);
            float v;
            if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN) {
              if (!meets(cl, ch, rB)) continue;  // 2^{-x^2} is 0 in FP32 on this chunk
              v = rr.c0 * __builtin_amdgcn_exp2f(-(x * x));
            } else if (PROF == XS_LORENTZ) {
              v = rr.c0 * rcp32(fmaf(x, x, 1.0f));
            } else if (flag) {
              const double xd = (double)(k - rr.kc) * (double)a + (double)nb;
              v = (full || (k >= klo && k <= khi)) ? (float)((double)rr.c0 * re_w_f64(xd, (double)rr.y)) : 0.0f;
            } else if (!meets(cl, ch, rB)) {
              v = pair_term_s(rr.A, x);
            } else if (!meets(cl, ch, rC)) {
              v = pair_term_s(rr.B1, x) + pair_term_s(rr.B2, x);
            } else if (!meets(cl, ch, rD)) {
              v = gh3_f32(x * x, rr.y, rr.c0);
            } else if constexpr (CQ) {
              // a chunk that reaches |z| < 6: three node pairs where
              // |z|^2 >= 36, the others queued for the rational approximation
              const float u = x * x, y = rr.y;
              const bool core = fmaf(y, y, u) < 36.0f;
              const bool inwin = full || (k >= klo && k <= khi);
              v = core ? 0.0f : gh3_f32(u, y, rr.c0);
              const unsigned long long bal = __ballot(core && inwin);
              if (bal) {
                const int slot = (qh + qn + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32),
                                  __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u))) & (CQN - 1);
                if (core && inwin) {
                  cq_x[slot] = x;
                  cq_y[slot] = y;
                  cq_c[slot] = rr.c0;
                  cq_b[slot] = k - row_lo;
                }
                qn += __popcll(bal);
                if (qn >= 64) cq_pop(64);
              }
            } else {
              // a chunk that reaches |z| < 6: every lane takes the rational
              // approximation (valid everywhere, so no divergence)
              double wr, wi;
              w_weideman<24>((double)x, (double)rr.y, wr, wi);
              v = (float)((double)rr.c0 * wr);
            }
            acc32[j] += (full || (k >= klo && k <= khi)) ? v : 0.0f;
          }
        }
#pragma unroll
        for (int j = 0; j < M; ++j) {
          acc64[j] += (double)acc32[j];
          acc32[j] = 0.0f;
        }
      } else {
        // FP64 form: x from the exact difference (nu_k - nu_i) inv, with the
        // grid point nu_k rounded as the oracle rounds it.  (Stepping x from
        // the row's first point skips that rounding: up to an ulp of nu_k,
        // which moves the values of narrow lines near their core by ~1e-12.)
        // NN: nodes of the Gauss-Hermite rule of the rows (2, 3, 4 or 6)
        auto uniform = [&](int l0, int l1, auto masked, auto nodes) {
          constexpr int NN = decltype(nodes)::value;
          for (int l = l0; l < l1; ++l) {
            const RecD& rr = srec[l];
            const double nu = rr.nu, inv = rr.inv;
            int klo = 0, khi = 0;
            if (masked) {
              klo = uni(rr.klo);
              khi = uni(rr.khi);
            }
            double xs[M];
#pragma unroll
            for (int j = 0; j < M; ++j) {
#pragma clang fp contract(off)
              xs[j] = (nuk[j] - nu) * inv;
            }
            Pair<double> C[3];
            KRange R1 = KRange{0x7fffffff, -0x7fffffff};
            if (PROF == XS_VOIGT && NN == 6) {
#pragma unroll
              for (int q = 0; q < 3; ++q) C[q] = make_pair<double>(rr.c0, rr.y, GH::t6[q], GH::w6[q]);
              R1 = KRange{uni(rr.r[1].lo), uni(rr.r[1].hi)};
            }
            double t[M];
            if (PROF == XS_VOIGT && NN <= 4) {
              // The far region (one node pair, or the three- or four-point
              // rule as one fraction N/D), x from the row's first point:
              // x = (lane + 64 j) a + xb.  (It differs from (nu_k - nu) inv by
              // the rounding of nu_k, ~1e-10 absolute at most, which moves a
              // value at |x| >= 63 by a relative 3.2e-12 at most.)  One
              // reciprocal, with its Newton
              // step, serves the four points j..j+3 of the lane:
              // r = 1/(D_0 D_1 D_2 D_3), 1/D_0 = D_1 (D_2 D_3 r) and so on;
              // the product stays finite for |x|, y <= 1e9 (staging sends
              // wider lines to the general path).
              const double a = rr.a, xb = rr.xb;
#pragma unroll
              for (int j = 0; j < M; j += 4) {
                double N[4], D[4];
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                  const double x = fma(lane_d[j + h], a, xb);
                  if constexpr (NN == 2) {
                    const double sv = fma(x, x, rr.A.h);
                    N[h] = fma(rr.A.cw, sv, rr.A.cwt);
                    D[h] = fma(sv, sv, rr.A.c);
                  } else if constexpr (NN == 3) {
                    poly3_nd(rr.C, x, N[h], D[h]);
                  } else {
                    poly2_nd(rr.B, x, N[h], D[h]);
                  }
                }
                const double p01 = D[0] * D[1], p23 = D[2] * D[3];
                const double r = rcp64(p01 * p23);
                const double r01 = p23 * r, r23 = p01 * r;
                t[j] = N[0] * (D[1] * r01);
                t[j + 1] = N[1] * (D[0] * r01);
                t[j + 2] = N[2] * (D[3] * r23);
                t[j + 3] = N[3] * (D[2] * r23);
              }
            } else {
#pragma unroll
              for (int j = 0; j < M; ++j) {
                const double u = xs[j] * xs[j];
                if (PROF == XS_LORENTZ) t[j] = rr.c0 * rcp64(fma(xs[j], xs[j], 1.0));
                else if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN) t[j] = rr.c0 * exp2(-u);
                else if (NN == 2) t[j] = pair_term<double>(rr.A, xs[j]);
                else {
                  // three-pair row: chunks wholly at |z|^2 >= 4000 take two pairs
                  const int cl = row_lo + 64 * j;
                  if (!meets(cl, cl + 63, R1)) t[j] = poly2_term(rr.B, xs[j]);
                  else t[j] = pair_term<double>(C[0], xs[j]) + pair2_term(C[1], C[2], xs[j]);
                }
              }
            }
#pragma unroll
            for (int j = 0; j < M; ++j) {
              const int k = my0 + 64 * j;
              if (!masked || (k >= klo && k <= khi)) acc64[j] += t[j];
            }
          }
        };
        using N2 = std::integral_constant<int, 2>;
        using N3 = std::integral_constant<int, 3>;
        using N4 = std::integral_constant<int, 4>;
        using N6 = std::integral_constant<int, 6>;
        uniform(0, e1, std::false_type(), N2());
        uniform(e1, e1m, std::true_type(), N2());
        if (PROF == XS_VOIGT) {
          uniform(e1m, e15, std::false_type(), N3());
          uniform(e15, e15m, std::true_type(), N3());
          uniform(e15m, e2, std::false_type(), N4());
          uniform(e2, e2m, std::true_type(), N4());
          uniform(e2m, e3, std::false_type(), N6());
          uniform(e3, e3m, std::true_type(), N6());
        }
        if constexpr (GN) gauss_rows(e3m, eg);
        else for (int l = e3m; l < eg; ++l) {
          const RecD& rr = srec[l];
          const double nu = rr.nu, inv = rr.inv, c0 = rr.c0, y = rr.y;
          const int klo = uni(rr.klo), khi = uni(rr.khi);
          // the band ranges of the line, read from LDS once (per-chunk reads
          // would put an LDS round trip before every band decision)
          KRange R[5];
#pragma unroll
          for (int q = 0; q < 5; ++q) R[q] = KRange{uni(rr.r[q].lo), uni(rr.r[q].hi)};
          const bool core_all = uni((int)(y >= 1.0e-3 && rr.a <= 1.0)) != 0;
#pragma unroll
          for (int j = 0; j < M; ++j) {
            const int cl = row_lo + 64 * j, ch = cl + 63;
            if (ch < klo || cl > khi) continue;
            const bool full = cl >= klo && ch <= khi;
            const int k = my0 + 64 * j;
            double x;
            {
#pragma clang fp contract(off)
              x = (nuk[j] - nu) * inv;
            }
            double v;
            if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN) {
              if (!meets(cl, ch, R[0])) continue;
              v = c0 * exp2(-(x * x));
            } else if (PROF == XS_LORENTZ) {
              v = c0 * rcp64(fma(x, x, 1.0));
            } else {
              const double u = x * x;
              if (!meets(cl, ch, R[0])) {
                v = pair_term<double>(make_pair<double>(c0, y, GH::t2[0], GH::w2[0]), x);
              } else if (!meets(cl, ch, R[1])) {
                v = poly2_term(rr.B, x);
              } else if (!meets(cl, ch, R[2])) {
                v = pair_term<double>(make_pair<double>(c0, y, GH::t6[0], GH::w6[0]), x) +
                    pair2_term(make_pair<double>(c0, y, GH::t6[1], GH::w6[1]),
                               make_pair<double>(c0, y, GH::t6[2], GH::w6[2]), x);
              } else if (!meets(cl, ch, R[3])) {
                v = gh_pairs_y<4>(c0, y, u);
              } else if (!meets(cl, ch, R[4])) {
                v = gh_pairs_y<6>(c0, y, u);
              } else if (core_all) {
                // a chunk that reaches |z|^2 < 64 of a line with y >= 1e-3
                // and a <= 1: the rational approximation on every lane.  Its
                // points have |x| <= 8 + 64 a <= 72, where it keeps Re w
                // within 4e-12 relative for y >= 1e-3 (its absolute error,
                // 1.5e-15 of |w|, against Re w >= ~y |w| / |z|), so the lanes
                // need not split between it and six node pairs.
                v = c0 * re_w_core<40>(x, y);
              } else if (u + y * y >= 64.0) {
                v = gh_pairs_y<6>(c0, y, u);
              } else {
                v = c0 * re_w_core<40>(x, y);
              }
            }
            if (full || (k >= klo && k <= khi)) acc64[j] += v;
          }
        }
      }
    }

    if constexpr (GN) {
      __syncthreads();
#pragma unroll
      for (int j = 0; j < M; ++j) acc64[j] += gbuf[lane + 64 * j];
      __syncthreads();
    }
    if constexpr (CQ) {
      // the queue's remaining points, then the row buffer into the sums
      if (qn > 0) cq_pop(qn);
      __syncthreads();
#pragma unroll
      for (int j = 0; j < M; ++j) acc64[j] += (double)rowbuf[lane + 64 * j];
      __syncthreads();
    }
    // ---- write the tile, or this item's partial row ----
    if (nch == 1) {
      const double scale = F32 ? exp(g.sb[cd.slot]) : 1.0;
      double* out = g.sigma + (int64_t)c * m.n_bins;
#pragma unroll
      for (int j = 0; j < M; ++j) {
        const int64_t k = my0 + 64 * j;
        if (k <= thi) {
          const double v = scale * acc64[j];
          out[k] = g.accumulate ? out[k] + v : v;
        }
      }
    } else {
      double* row = g.part + (int64_t)(g.pb[ct] + jpart) * ROWB;
#pragma unroll
      for (int j = 0; j < M; ++j) row[lane + 64 * j] = acc64[j];
    }
    if (!g.persistent) return;
  }
}

// Candidate count of every (tile, condition) and their total.
__global__ __launch_bounds__(256) void k_items_count(GatherArgs g, int32_t* cnt) {
  unsigned long long local = 0;
  for (int64_t ct = (int64_t)blockIdx.x * 256 + threadIdx.x; ct < g.n_ct; ct += (int64_t)gridDim.x * 256) {
    const int c = (int)(ct % g.m.n_cond), t = (int)(ct / g.m.n_cond);
    int64_t tlo, thi, plo, phi;
    tile_candidates(g, g.cond[c], t, tlo, thi, plo, phi);
    cnt[ct] = (int32_t)(phi - plo);
    local += (unsigned long long)(phi - plo);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) local += __shfl_xor(local, o, 64);
  if ((threadIdx.x & 63) == 0 && local) atomicAdd((unsigned long long*)(g.counter + 2), local);
}

// Lines per work item (at least the requested number, and large enough that
// the items stay near the target count) and the items of every (tile,
// condition); split tiles also get partial rows.
__global__ __launch_bounds__(256) void k_items_split(GatherArgs g, const int32_t* cnt, int32_t* ib,
                                                     int32_t* pb) {
  const unsigned long long total = *(const unsigned long long*)(g.counter + 2);
  int64_t chunk = (int64_t)((total + g.item_target - 1) / g.item_target);
  chunk = max(chunk, g.chunk_cfg);
  chunk = max<int64_t>(64, (chunk + 63) / 64 * 64);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *(int64_t*)(g.counter + 4) = chunk;
    ib[g.n_ct] = 0;
    pb[g.n_ct] = 0;
  }
  for (int64_t ct = (int64_t)blockIdx.x * 256 + threadIdx.x; ct < g.n_ct; ct += (int64_t)gridDim.x * 256) {
    const int64_t n = cnt[ct];
    const int nch = n == 0 ? 1 : (int)((n + chunk - 1) / chunk);
    ib[ct] = nch;
    pb[ct] = nch > 1 ? nch : 0;
  }
}

// Sum of the partial rows of split tiles, in item order.
__global__ __launch_bounds__(256) void k_reduce(GatherArgs g) {
  for (int64_t ct = blockIdx.x; ct < g.n_ct; ct += gridDim.x) {
    const int nch = g.ib[ct + 1] - g.ib[ct];
    if (nch <= 1) continue;
    const int c = (int)(ct % g.m.n_cond), t = (int)(ct / g.m.n_cond);
    const double scale = g.m.prec == XS_FP32 ? exp(g.sb[g.cond[c].slot]) : 1.0;
    const double* rows = g.part + (int64_t)g.pb[ct] * g.tile_bins;
    double* out = g.sigma + (int64_t)c * g.m.n_bins;
    for (int o = threadIdx.x; o < g.tile_bins; o += 256) {
      const int64_t k = (int64_t)t * g.tile_bins + o;
      if (k >= g.m.n_bins) break;
      double s = 0.0;
      for (int j = 0; j < nch; ++j) s += rows[(int64_t)j * g.tile_bins + o];
      const double v = scale * s;
      out[k] = g.accumulate ? out[k] + v : v;
    }
  }
}

template <typename Real, int PROF>
static void gather_dispatch(const GatherArgs& a, int M, int blocks, hipStream_t s) {
#define XS_G(MM)                                                                      \
  if (M == MM) {                                                                      \
    hipLaunchKernelGGL((k_gather<Real, PROF, MM>), dim3(blocks), dim3(64), 0, s, a); \
    return;                                                                           \
  }
  XS_G(4) XS_G(8) XS_G(16)
#undef XS_G
}

void launch_gather(const ModelDev& m, const Work& w, const Tiling& t, double* sigma,
                   int accumulate, hipStream_t s) {
  GatherArgs a;
  a.m = m;
  a.cond = w.cond;
  a.sb = w.sb;
  a.off = w.off;
  a.rnu = w.rnu;
  a.rgref = w.rgref;
  a.rnexp = w.rnexp;
  a.rgpre = w.rgpre;
  a.rS = w.rS;
  a.rkc = w.rkc;
  a.rdel = w.rdel;
  a.rwin = w.rwin;
  a.max_lines = w.max_lines;
  a.counter = w.counter;
  a.ib = w.item_base;
  a.pb = w.part_base;
  a.part = w.part;
  a.sigma = sigma;
  a.accumulate = accumulate;
  a.tile_bins = t.tile_bins;
  a.n_tiles = (int)((m.n_bins + t.tile_bins - 1) / t.tile_bins);
  a.n_ct = a.n_tiles * m.n_cond;
  a.persistent = t.persistent;
  a.chunk_cfg = t.chunk_lines;
  a.item_target = w.item_target;
  // plan the work items
  launch_reset_queue(w, s);
  const int cb = (int)std::min<int64_t>(1024, (a.n_ct + 255) / 256);
  hipLaunchKernelGGL(k_items_count, dim3(cb), dim3(256), 0, s, a, w.item_cnt);
  hipLaunchKernelGGL(k_items_split, dim3(cb), dim3(256), 0, s, a, (const int32_t*)w.item_cnt,
                     w.item_base, w.part_base);
  launch_scan_i32(w.item_base, (int64_t)a.n_ct + 1, w.item_sums, s);
  launch_scan_i32(w.part_base, (int64_t)a.n_ct + 1, w.item_sums, s);
  // every item fits the bound n_ct + item_target (one per unsplit tile plus
  // at most total / chunk extra)
  const int blocks = t.persistent ? t.grid_blocks : (int)(a.n_ct + w.item_target);
  const int M = t.tile_bins / 64;
#define XS_P(R, P)                                   \
  if (m.profile == P) gather_dispatch<R, P>(a, M, blocks, s);
  if (m.prec == XS_FP32) {
    XS_P(float, XS_DOPPLER) XS_P(float, XS_GAUSSIAN) XS_P(float, XS_LORENTZ) XS_P(float, XS_VOIGT)
    XS_P(float, XS_BIN_DOPPLER) XS_P(float, XS_BIN_GAUSSIAN) XS_P(float, XS_BIN_LORENTZ) XS_P(float, XS_BIN_VOIGT)
    XS_P(float, XS_PV_THOMPSON) XS_P(float, XS_PV_OLIVERO)
  } else {
    XS_P(double, XS_DOPPLER) XS_P(double, XS_GAUSSIAN) XS_P(double, XS_LORENTZ) XS_P(double, XS_VOIGT)
    XS_P(double, XS_BIN_DOPPLER) XS_P(double, XS_BIN_GAUSSIAN) XS_P(double, XS_BIN_LORENTZ) XS_P(double, XS_BIN_VOIGT)
    XS_P(double, XS_PV_THOMPSON) XS_P(double, XS_PV_OLIVERO)
  }
#undef XS_P
  const int rb = (int)std::min<int64_t>(65536, a.n_ct);
  hipLaunchKernelGGL(k_reduce, dim3(rb), dim3(256), 0, s, a);
}

// Evaluators of the scatter (one lane per bin, band per lane).
struct ScatF {
  float a, b, y, y2, q, c0, cy;
};
struct ScatD {
  double nu, inv, y, y2, q, c0, cy;
};

template <int PROF>
__device__ __forceinline__ float eval_f32(const ScatF& r, float x) {
  if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN) {
    return r.c0 * __builtin_amdgcn_exp2f(-x * x);
  } else if (PROF == XS_LORENTZ) {
    return r.c0 * __builtin_amdgcn_rcpf(fmaf(x, x, 1.0f));
  } else {
    const float u = x * x;
    if (u + r.y2 >= 900.0f) return r.cy * gh_re_sum<1, float>(u, r.y2, r.q);
    if (u + r.y2 >= 64.0f) return r.cy * gh_re_sum<2, float>(u, r.y2, r.q);
    return r.c0 * (float)re_w_core<24>((double)x, (double)r.y);
  }
}

template <int PROF>
__device__ __forceinline__ double eval_f64(const ScatD& r, double x) {
  if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN) {
    return r.c0 * exp2(-x * x);
  } else if (PROF == XS_LORENTZ) {
    return r.c0 / fma(x, x, 1.0);
  } else {
    return r.c0 * re_w_f64(x, r.y);
  }
}

// ---------------------------------------------------------------------------
// Line-parallel scatter with atomics (comparison algorithm).
// ---------------------------------------------------------------------------
struct ScatterArgs {
  ModelDev m;
  const CondDev* cond;
  const double* sb;
  const int32_t* off;
  const double* rnu;
  const float* rgref;
  const float* rnexp;
  const double* rgpre;      // lifetime widths, or null when the states have no lifetimes
  const void* rS;
  int64_t max_lines;
  double* sigma;
};

template <typename Real, int PROF>
__global__ __launch_bounds__(256) void k_scatter(ScatterArgs g) {
  const ModelDev& m = g.m;
  const int lane = threadIdx.x & 63;
  const int64_t nkept = g.off[m.n_buckets];
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int64_t total = nkept * m.n_cond;
  for (int64_t wi = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); wi < total;
       wi += nwaves) {
    const int64_t p = wi / m.n_cond;
    const int c = (int)(wi % m.n_cond);
    const CondDev cd = g.cond[c];
    const double nu = g.rnu[p];
    int64_t klo, khi;
    if (!line_window(nu, cd.cut, m.nu0, m.dnu, m.n_bins, klo, khi)) continue;
    double S = sizeof(Real) == 4 ? (double)((const float*)g.rS)[(int64_t)cd.slot * g.max_lines + p]
                                 : ((const double*)g.rS)[(int64_t)cd.slot * g.max_lines + p];
    if (S == 0.0) continue;
    const double scale = sizeof(Real) == 4 ? exp(g.sb[cd.slot]) : 1.0;
    LineParams lp = line_params<PROF>(m, cd, nu, (double)g.rgref[p], (double)g.rnexp[p], g.rgpre ? g.rgpre[p] : 0.0, S);
    double* out = g.sigma + (int64_t)c * m.n_bins;
    if constexpr (sizeof(Real) == 4) {
      ScatF r;
      const int64_t kc = home_bin(nu, m.nu0, m.dnu);
      const double delta = nu - nu_of_bin(m.nu0, m.dnu, kc);
      r.a = (float)(m.dnu * lp.inv);
      r.b = (float)(delta * lp.inv);
      r.y = (float)lp.y;
      r.y2 = (float)(lp.y * lp.y);
      r.q = (float)(4.0 * lp.y * lp.y);
      r.c0 = (float)lp.c0;
      r.cy = (float)(lp.c0 * 2.0 * lp.y / kPI);
      const bool wide = PROF == XS_VOIGT &&
                        (fmax(fabs((double)(klo - kc) * r.a), fabs((double)(khi - kc) * r.a)) > 1.0e9 ||
                         lp.y > 1.0e9);
      for (int64_t k = klo + lane; k <= khi; k += 64) {
        const float x = fmaf((float)(k - kc), r.a, -r.b);
        float v;
        if (wide)
          v = (float)(lp.c0 * re_w_f64((double)(k - kc) * (double)r.a - (double)r.b, lp.y));
        else if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN)
          v = (x * x > 160.0f) ? 0.0f : eval_f32<PROF>(r, x);
        else
          v = eval_f32<PROF>(r, x);
        if (v != 0.0f) unsafeAtomicAdd(out + k, scale * (double)v);
      }
    } else {
      ScatD r;
      r.nu = nu;
      r.inv = lp.inv;
      r.y = lp.y;
      r.y2 = lp.y * lp.y;
      r.q = 4.0 * lp.y * lp.y;
      r.c0 = lp.c0;
      r.cy = lp.c0 * 2.0 * lp.y / kPI;
      for (int64_t k = klo + lane; k <= khi; k += 64) {
        double x;
        {
#pragma clang fp contract(off)
          x = (nu_of_bin(m.nu0, m.dnu, k) - nu) * r.inv;
        }
        double v;
        if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN)
          v = (x * x > 1100.0) ? 0.0 : eval_f64<PROF>(r, x);
        else
          v = eval_f64<PROF>(r, x);
        if (v != 0.0) unsafeAtomicAdd(out + k, v);
      }
    }
  }
}

// Line-parallel scatter of the binned profiles: one wave per (line,
// condition), the band chosen per lane by the bin's nearest point.
template <typename Real, int PROF>
__global__ __launch_bounds__(256) void k_scatter_bin(ScatterArgs g) {
  constexpr int BASE = PROF - 4;
  const ModelDev& m = g.m;
  const int lane = threadIdx.x & 63;
  const int64_t nkept = g.off[m.n_buckets];
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int64_t total = nkept * m.n_cond;
  for (int64_t wi = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); wi < total;
       wi += nwaves) {
    const int64_t p = wi / m.n_cond;
    const int c = (int)(wi % m.n_cond);
    const CondDev cd = g.cond[c];
    const double nu = g.rnu[p];
    int64_t klo, khi;
    if (!line_window(nu, cd.cut, m.nu0, m.dnu, m.n_bins, klo, khi)) continue;
    const double S = sizeof(Real) == 4 ? (double)((const float*)g.rS)[(int64_t)cd.slot * g.max_lines + p]
                                       : ((const double*)g.rS)[(int64_t)cd.slot * g.max_lines + p];
    if (S == 0.0) continue;
    const double scale = sizeof(Real) == 4 ? exp(g.sb[cd.slot]) : 1.0;
    double inv, y = 0.0, c0;
    if (BASE == XS_DOPPLER || BASE == XS_GAUSSIAN) {
      inv = sqrt(kLN2) / (BASE == XS_GAUSSIAN ? cd.hwhm : nu * cd.dop);
      c0 = S * 0.5 / m.dnu;
    } else {
      const double gamma = (double)g.rgref[p] * exp((double)g.rnexp[p] * cd.lnTr) * cd.pfac + (g.rgpre ? g.rgpre[p] : 0.0);
      if (BASE == XS_LORENTZ) {
        inv = 1.0 / gamma;
        c0 = S / (kPI * m.dnu);
      } else {
        inv = sqrt(kLN2) / (nu * cd.dop);
        y = gamma * inv;
        c0 = S / (sqrt(kPI) * m.dnu);
      }
    }
    const double h = m.dnu * inv, hh = 0.5 * h;
    double* out = g.sigma + (int64_t)c * m.n_bins;
    if constexpr (sizeof(Real) == 4) {
      const int64_t kc = home_bin(nu, m.nu0, m.dnu);
      const double delta = nu - nu_of_bin(m.nu0, m.dnu, kc);
      const float a = (float)h, b = (float)(delta * inv), hf = 0.5f * a, yf = (float)y, y2 = yf * yf;
      const float yh = yf * a, c0f = (float)c0;
      const bool wide = BASE == XS_VOIGT &&
                        (fmax(fabs((double)(klo - kc) * a), fabs((double)(khi - kc) * a)) + hh > 1.0e9 ||
                         y > 1.0e9);
      for (int64_t k = klo + lane; k <= khi; k += 64) {
        const float x = fmaf((float)(k - kc), a, -b);
        float v;
        if (BASE == XS_DOPPLER || BASE == XS_GAUSSIAN) {
          v = (fabsf(x) - hf > 10.1f) ? 0.0f : erf_bin<float>(x, hf);
        } else if (BASE == XS_LORENTZ) {
          v = lor_bin<float>(x, hf, a);
        } else if (wide) {
          v = (float)voigt_bin_f64((double)(k - kc) * (double)a - (double)b, y, (double)hf);
        } else {
          const float xn = fmaxf(fabsf(x) - hf, 0.0f), rho = fmaf(xn, xn, y2);
          if (rho >= 900.0f) v = vpairs_bin<1, false, float>(x - hf, x + hf, yh, y2);
          else if (rho >= 64.0f) v = vpairs_bin<2, false, float>(x - hf, x + hf, yh, y2);
          else if (rho >= 36.0f) v = vpairs_bin<3, false, float>(x - hf, x + hf, yh, y2);
          else v = (float)voigt_bin_core<24>((double)x, y, (double)hf);
        }
        v *= c0f;
        if (v != 0.0f) unsafeAtomicAdd(out + k, scale * (double)v);
      }
    } else {
      for (int64_t k = klo + lane; k <= khi; k += 64) {
        double x;
        {
#pragma clang fp contract(off)
          x = (nu_of_bin(m.nu0, m.dnu, k) - nu) * inv;
        }
        double v;
        if (BASE == XS_DOPPLER || BASE == XS_GAUSSIAN) v = (fabs(x) - hh > 27.3) ? 0.0 : erf_bin<double>(x, hh);
        else if (BASE == XS_LORENTZ) v = lor_bin<double>(x, hh, h);
        else v = voigt_bin_f64(x, y, hh);
        v *= c0;
        if (v != 0.0) unsafeAtomicAdd(out + k, v);
      }
    }
  }
}

// Line-parallel scatter of the pseudo-Voigts.
template <typename Real, int PROF>
__global__ __launch_bounds__(256) void k_scatter_pv(ScatterArgs g) {
  const ModelDev& m = g.m;
  const int lane = threadIdx.x & 63;
  const int64_t nkept = g.off[m.n_buckets];
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int64_t total = nkept * m.n_cond;
  for (int64_t wi = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); wi < total;
       wi += nwaves) {
    const int64_t p = wi / m.n_cond;
    const int c = (int)(wi % m.n_cond);
    const CondDev cd = g.cond[c];
    const double nu = g.rnu[p];
    int64_t klo, khi;
    if (!line_window(nu, cd.cut, m.nu0, m.dnu, m.n_bins, klo, khi)) continue;
    const double S = sizeof(Real) == 4 ? (double)((const float*)g.rS)[(int64_t)cd.slot * g.max_lines + p]
                                       : ((const double*)g.rS)[(int64_t)cd.slot * g.max_lines + p];
    if (S == 0.0) continue;
    const double scale = sizeof(Real) == 4 ? exp(g.sb[cd.slot]) : 1.0;
    const double gamma = (double)g.rgref[p] * exp((double)g.rnexp[p] * cd.lnTr) * cd.pfac + (g.rgpre ? g.rgpre[p] : 0.0);
    const PVConst pc = pv_const(PROF, nu * cd.dop, gamma, S);
    double* out = g.sigma + (int64_t)c * m.n_bins;
    if constexpr (sizeof(Real) == 4) {
      const int64_t kc = home_bin(nu, m.nu0, m.dnu);
      const double delta = nu - nu_of_bin(m.nu0, m.dnu, kc);
      const float a = (float)(m.dnu * pc.inv), b = (float)(delta * pc.inv);
      const float cL = (float)pc.cL, cG = (float)pc.cG;
      for (int64_t k = klo + lane; k <= khi; k += 64) {
        const float x = fmaf((float)(k - kc), a, -b);
        float v = cL * __builtin_amdgcn_rcpf(fmaf(x, x, 1.0f));
        if (x * x < 160.0f) v = fmaf(cG, __builtin_amdgcn_exp2f(-(x * x)), v);
        unsafeAtomicAdd(out + k, scale * (double)v);
      }
    } else {
      for (int64_t k = klo + lane; k <= khi; k += 64) {
        double x;
        {
#pragma clang fp contract(off)
          x = (nu_of_bin(m.nu0, m.dnu, k) - nu) * pc.inv;
        }
        double v = pc.cL / fma(x, x, 1.0);
        if (x * x < 1100.0) v = fma(pc.cG, exp2(-(x * x)), v);
        unsafeAtomicAdd(out + k, v);
      }
    }
  }
}

__global__ void k_fill(double* p, int64_t n, int accumulate) {
  if (accumulate) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

void launch_scatter(const ModelDev& m, const Work& w, double* sigma, int accumulate,
                    int64_t n_lines, hipStream_t s) {
  (void)n_lines;
  const int64_t nb = m.n_bins * m.n_cond;
  hipLaunchKernelGGL(k_fill, dim3(2048), dim3(256), 0, s, sigma, nb, accumulate);
  ScatterArgs a;
  a.m = m;
  a.cond = w.cond;
  a.sb = w.sb;
  a.off = w.off;
  a.rnu = w.rnu;
  a.rgref = w.rgref;
  a.rnexp = w.rnexp;
  a.rgpre = w.rgpre;
  a.rS = w.rS;
  a.max_lines = w.max_lines;
  a.sigma = sigma;
  const int blocks = 256 * 16;
#define XS_S(R, P)                                                                 \
  if (m.profile == P) {                                                            \
    hipLaunchKernelGGL((k_scatter<R, P>), dim3(blocks), dim3(256), 0, s, a);       \
    return;                                                                        \
  }
  if (m.prec == XS_FP32) {
    XS_S(float, XS_DOPPLER) XS_S(float, XS_GAUSSIAN) XS_S(float, XS_LORENTZ) XS_S(float, XS_VOIGT)
  } else {
    XS_S(double, XS_DOPPLER) XS_S(double, XS_GAUSSIAN) XS_S(double, XS_LORENTZ) XS_S(double, XS_VOIGT)
  }
#undef XS_S
#define XS_SB(R, P)                                                                \
  if (m.profile == P) {                                                            \
    hipLaunchKernelGGL((k_scatter_bin<R, P>), dim3(blocks), dim3(256), 0, s, a);   \
    return;                                                                        \
  }
  if (m.prec == XS_FP32) {
    XS_SB(float, XS_BIN_DOPPLER) XS_SB(float, XS_BIN_GAUSSIAN) XS_SB(float, XS_BIN_LORENTZ) XS_SB(float, XS_BIN_VOIGT)
  } else {
    XS_SB(double, XS_BIN_DOPPLER) XS_SB(double, XS_BIN_GAUSSIAN) XS_SB(double, XS_BIN_LORENTZ) XS_SB(double, XS_BIN_VOIGT)
  }
#undef XS_SB
#define XS_SPV(R, P)                                                               \
  if (m.profile == P) {                                                            \
    hipLaunchKernelGGL((k_scatter_pv<R, P>), dim3(blocks), dim3(256), 0, s, a);    \
    return;                                                                        \
  }
  if (m.prec == XS_FP32) {
    XS_SPV(float, XS_PV_THOMPSON) XS_SPV(float, XS_PV_OLIVERO)
  } else {
    XS_SPV(double, XS_PV_THOMPSON) XS_SPV(double, XS_PV_OLIVERO)
  }
#undef XS_SPV
}

}  // namespace xs
