// Profile pass: sigma_k = sum_i S_i f_i(nu_k - nu_i) over each line's cut-off
// window (Eq. xsec with the cut-off rule of section "Spectral synthesis").
//
// k_gather: grid-tile-parallel.  A work item is (condition c, tile t of
//   tile_bins grid points).  Its candidate lines are the buckets within the
//   cut-off reach of the tile (lines were counting-sorted by home bin).  Each
//   pass stages up to 256 candidates: every thread tests one line's exact
//   window against the tile, the survivors are compacted into LDS with a
//   wave-level prefix (ballot + mbcnt) and a 4-entry cross-wave scan, and then
//   every wave evaluates every staged line over its own 64*M consecutive bins
//   (M consecutive bins per lane), reading the line from LDS as a broadcast.
//   Accumulation: FP64, or FP32 partial sums flushed to FP64 after each pass.
//   Persistent mode: a fixed grid pulls items from a device counter.
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
                                                  double gref, double nexp, double S) {
  LineParams lp;
  double alpha = (PROF == XS_GAUSSIAN) ? cd.hwhm : nu * cd.dop;
  double gamma = gref * exp(nexp * cd.lnTr) * cd.pfac;
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

// Far-region pair constants (cW, cW p, q, p^2) for node pair (tau, W).
template <typename R>
struct Pair {
  R cw, cwp, q, p2;
};
template <typename R>
__device__ __forceinline__ Pair<R> make_pair(double c0, double y, double tau, double W) {
  const double y2 = y * y, p = y2 + tau;
  const double cw = c0 * (2.0 * y / kPI) * W;
  Pair<R> r;
  r.cw = (R)cw;
  r.cwp = (R)(cw * p);
  r.q = (R)(2.0 * y2 - 2.0 * tau);
  r.p2 = (R)(p * p);
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

// Row classes of a staged line, 2 bits per wave of the tile: 0 = the row
// gets nothing (outside the window, or a Gaussian row where 2^{-x^2}
// vanishes); 1 = the whole row is inside the window and takes the first
// uniform formula (FP32: one node pair / Gaussian / Lorentzian; FP64: one
// node pair / Gaussian / Lorentzian); 3 = inside the window, second uniform
// formula (FP32: two node pairs; FP64: two node pairs); 2 = general per-chunk
// path (window edges, the core, lines evaluated in FP64).
constexpr int kRowSkip = 0, kRowF1 = 1, kRowGeneral = 2, kRowF2 = 3;

// FP32 form.  The fast-path fields come first (two 16-byte LDS reads).
//   rB: bins that are not far-wing (one node pair) -- for the Gaussian, the
//       bins where 2^{-x^2} is not zero in FP32; rC: bins near the core that
//       need the per-lane choice (Taylor core or two node pairs).
struct RecF {
  int cls;
  float a, nb, jfb;  // x = (jfb + offset of the bin in the tile) a + nb; jfb = tlo - k_c
  Pair<float> A;
  int klo, khi, flag, kc;
  KRange rB, rC;
  float c0, y, pad0, pad1;
  Pair<float> B1, B2;
};
// FP64 form.  r[0..4]: bins with |z|^2 below 9e6, 6400, 400, 144, 64 (the
// thresholds of the 1, 2, 3, 4 and 6 node-pair bands); for the Gaussian,
// r[0] holds the bins where 2^{-x^2} is not zero in FP64.
struct RecD {
  int cls, klo, khi, flag;
  KRange r[5];
  int kc, pad2;
  double nu, inv, y, c0;
  Pair<double> A, B1, B2;
};

struct GatherArgs {
  ModelDev m;
  const CondDev* cond;
  const double* sb;
  const int32_t* off;
  const double* rnu;
  const float* rgref;
  const float* rnexp;
  const void* rS;
  int64_t max_lines;
  int32_t* counter;
  double* sigma;
  int32_t accumulate;
  int32_t n_tiles;
  int64_t n_items;
  int32_t tile_bins;
  int32_t persistent;
};

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ bool meets(int lo, int hi, const KRange& r) { return hi >= r.lo && lo <= r.hi; }

// Staging: does line p touch bins [tlo, thi] under condition cd?  Fills rec,
// including the class of each wave's row (rows of rowb bins from tlo).
template <typename Rec, int PROF, int WAVES>
__device__ bool stage_line(const GatherArgs& g, const CondDev& cd, int64_t p, int64_t tlo,
                           int64_t thi, int rowb, Rec& r) {
  const ModelDev& m = g.m;
  const double nu = g.rnu[p];
  int64_t klo, khi;
  if (!line_window(nu, cd.cut, m.nu0, m.dnu, m.n_bins, klo, khi)) return false;
  if (khi < tlo || klo > thi) return false;
  double S;
  if constexpr (sizeof(Rec) == sizeof(RecF))
    S = (double)((const float*)g.rS)[(int64_t)cd.slot * g.max_lines + p];
  else
    S = ((const double*)g.rS)[(int64_t)cd.slot * g.max_lines + p];
  if (S == 0.0) return false;
  const int64_t kc = home_bin(nu, m.nu0, m.dnu);
  const double delta = nu - nu_of_bin(m.nu0, m.dnu, kc);
  const LineParams lp = line_params<PROF>(m, cd, nu, (double)g.rgref[p], (double)g.rnexp[p], S);
  klo = klo > tlo ? klo : tlo;
  khi = khi < thi ? khi : thi;
  r.klo = (int)klo;
  r.khi = (int)khi;
  r.flag = 0;
  r.kc = (int)kc;
  const double a = m.dnu * lp.inv, b = delta * lp.inv;
  const double y2 = lp.y * lp.y;
  using R = decltype(r.A.cw);
  if (PROF == XS_VOIGT) {
    r.A = make_pair<R>(lp.c0, lp.y, GH::t2[0], GH::w2[0]);
    r.B1 = make_pair<R>(lp.c0, lp.y, GH::t4[0], GH::w4[0]);
    r.B2 = make_pair<R>(lp.c0, lp.y, GH::t4[1], GH::w4[1]);
  }
  auto xr = [&](double rho) { return x_range(sqrt(fmax(rho - y2, 0.0)), a, b, kc, klo, khi); };
  const KRange none = x_range(0.0, a, b, kc, klo, khi);
  // class of the row [lo, hi] given the ranges of the first and second uniform formula
  auto row_class = [&](int lo, int hi, KRange zero, KRange not1, KRange not2, bool can2) {
    if (hi < klo || lo > khi) return kRowSkip;
    if (!meets(lo, hi, zero)) return kRowSkip;
    const bool inside = klo <= lo && khi >= hi;
    if (!inside || r.flag) return kRowGeneral;
    if (!meets(lo, hi, not1)) return kRowF1;
    if (can2 && !meets(lo, hi, not2)) return kRowF2;
    return kRowGeneral;
  };
  KRange zero, not1, not2;
  bool can2;
  if constexpr (sizeof(Rec) == sizeof(RecF)) {
    r.a = (float)a;
    r.nb = (float)(-b);
    r.jfb = (float)(tlo - kc);  // integer, exact in FP32 within a window
    r.c0 = (float)lp.c0;
    r.y = (float)lp.y;
    if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN) {
      r.rB = x_range(sqrt(160.0), a, b, kc, klo, khi);
      r.rC = none;
      zero = r.rB;
      // a row inside the nonzero range takes the Gaussian directly
      not1 = KRange{-0x7fffffff, 0x7fffffff};
      if (r.rB.lo <= r.rB.hi) {
        not1 = KRange{(int)klo, r.rB.lo - 1};   // bins left of the nonzero range
      }
      not2 = KRange{r.rB.hi + 1, (int)khi};     // bins right of it
      can2 = false;
    } else if (PROF == XS_VOIGT) {
      r.rB = xr(900.0 * 1.001);
      r.rC = xr(64.0 * 1.001);
      // FP32 keeps u (u + q) + p^2 finite for |x|, y < ~1e9; lines beyond that
      // (nu of a few 1e-3 cm^-1 or less) are evaluated in FP64.
      const double xmax = fmax(fabs((double)(klo - kc) * a - b), fabs((double)(khi - kc) * a - b));
      if (xmax > 1.0e9 || lp.y > 1.0e9) r.flag = 1;
      zero = KRange{(int)klo, (int)khi};
      not1 = r.rB;
      not2 = r.rC;
      can2 = true;
    } else {
      r.rB = none;
      r.rC = none;
      zero = KRange{(int)klo, (int)khi};
      not1 = none;
      not2 = none;
      can2 = false;
    }
  } else {
    r.nu = nu;
    r.inv = lp.inv;
    r.y = lp.y;
    r.c0 = lp.c0;
    if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN) {
      r.r[0] = x_range(sqrt(1100.0), a, b, kc, klo, khi);
      zero = r.r[0];
      not1 = KRange{-0x7fffffff, 0x7fffffff};
      if (r.r[0].lo <= r.r[0].hi) not1 = KRange{(int)klo, r.r[0].lo - 1};
      not2 = KRange{r.r[0].hi + 1, (int)khi};
      can2 = false;
    } else if (PROF == XS_VOIGT) {
      r.r[0] = xr(9.0e6 * 1.001);
      r.r[1] = xr(6400.0 * 1.001);
      r.r[2] = xr(400.0 * 1.001);
      r.r[3] = xr(144.0 * 1.001);
      r.r[4] = xr(64.0 * 1.001);
      zero = KRange{(int)klo, (int)khi};
      not1 = r.r[0];
      not2 = r.r[1];
      can2 = true;
    } else {
      zero = KRange{(int)klo, (int)khi};
      not1 = none;
      not2 = none;
      can2 = false;
    }
  }
  // For the Gaussian the "first formula" test is: row inside the nonzero range.
  int cls = 0;
#pragma unroll
  for (int w = 0; w < WAVES; ++w) {
    const int lo = (int)tlo + w * rowb, hi = lo + rowb - 1;
    int c;
    if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN) {
      if (hi < klo || lo > khi || !meets(lo, hi, zero)) c = kRowSkip;
      else if (klo <= lo && khi >= hi && !meets(lo, hi, not1) && !meets(lo, hi, not2)) c = kRowF1;
      else c = kRowGeneral;
    } else {
      c = row_class(lo, hi, zero, not1, not2, can2);
    }
    cls |= c << (2 * w);
  }
  r.cls = cls;
  return cls != 0;
}

// ---- far-region evaluators ------------------------------------------------
__device__ __forceinline__ double rcp64(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float rcp32(float d) { return __builtin_amdgcn_rcpf(d); }

template <typename R>
__device__ __forceinline__ R pair_term(const Pair<R>& P, R u) {
  const R n = fma(P.cw, u, P.cwp);
  const R d = fma(u, u + P.q, P.p2);
  if constexpr (sizeof(R) == 4) return n * rcp32(d);
  else return n * rcp64(d);
}
// two pairs as one fraction (FP64 only: the product of the d_j stays finite)
__device__ __forceinline__ double pair2_term(const Pair<double>& P, const Pair<double>& Q, double u) {
  const double n1 = fma(P.cw, u, P.cwp), d1 = fma(u, u + P.q, P.p2);
  const double n2 = fma(Q.cw, u, Q.cwp), d2 = fma(u, u + Q.q, Q.p2);
  return fma(n1, d2, n2 * d1) * rcp64(d1 * d2);
}
// NP node pairs from y (near-core chunks of the FP64 form; out of line, rare)
template <int NP>
__device__ __noinline__ double gh_pairs_y(double c0, double y, double u) {
  const double* tau = gh_tau<NP>();
  const double* W = gh_w<NP>();
  const double y2 = y * y, cy = c0 * 2.0 * y / kPI;
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    const double p = y2 + tau[j];
    s = fma(cy * W[j] * (u + p), rcp64(fma(u, u + (2.0 * y2 - 2.0 * tau[j]), p * p)), s);
  }
  return s;
}

// Per-lane evaluation of a chunk that reaches |z| < 8 (FP32 form).
__device__ __noinline__ float voigt_near_f32(float x, float y, float c0, Pair<float> B1, Pair<float> B2) {
  const float u = x * x;
  if (u + y * y >= 64.0f) return pair_term<float>(B1, u) + pair_term<float>(B2, u);
  double wr, wi;
  w_core<16>((double)x, (double)y, wr, wi);
  return c0 * (float)wr;
}

// Tile layout: wave w owns the row [row_lo, row_lo + 64 M); lane l owns the
// bins row_lo + 64 j + l, j = 0..M-1, so each "chunk" j is 64 consecutive
// bins.  A line's narrow core region falls into one or two chunks, and every
// per-chunk decision (window, band, zero skip) is a scalar compare of the
// chunk's bin range with the line's precomputed ranges.
template <typename Real, int PROF, int M, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_gather(GatherArgs g) {
  using Rec = typename std::conditional<sizeof(Real) == 4, RecF, RecD>::type;
  constexpr bool F32 = sizeof(Real) == 4;
  constexpr int NT = 64 * WAVES;
  constexpr int ROWB = 64 * M;  // bins per wave row
  __shared__ Rec srec[NT];
  __shared__ int s_wcnt[WAVES];
  __shared__ long long s_item;

  // wave index made explicitly uniform so row and chunk bounds live in SGPRs
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const ModelDev& m = g.m;
  long long item = blockIdx.x;
  for (;;) {
    if (g.persistent) {
      if (tid == 0) s_item = atomicAdd((unsigned long long*)g.counter, 1ull);
      __syncthreads();
      item = s_item;
      __syncthreads();
    }
    if (item >= g.n_items) return;
    const int c = (int)(item % m.n_cond);
    const int t = (int)(item / m.n_cond);
    const CondDev cd = g.cond[c];
    const int64_t tlo = (int64_t)t * g.tile_bins;
    const int64_t thi = min(tlo + g.tile_bins, m.n_bins) - 1;
    const int64_t blo = max<int64_t>(0, (tlo - cd.wbins) / m.bucket_bins - ((tlo - cd.wbins) < 0 ? 1 : 0));
    const int64_t bhi = min<int64_t>(m.n_buckets - 1, (thi + cd.wbins) / m.bucket_bins);
    const int64_t plo = g.off[blo], phi = g.off[bhi + 1];
    const int row_lo = (int)tlo + wave * ROWB;
    const int row_hi = row_lo + ROWB - 1;
    const int my0 = row_lo + lane;          // bin of chunk 0 of this lane
    const float lane_off = (float)(wave * ROWB + lane);  // offset of that bin in the tile

    double acc64[M];
    float acc32[M];
    double nuk[M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
      acc64[j] = 0.0;
      acc32[j] = 0.0f;
      if (!F32) nuk[j] = nu_of_bin(m.nu0, m.dnu, my0 + 64 * j);
    }

    for (int64_t p0 = plo; p0 < phi; p0 += NT) {
      // ---- stage: exact window test, compaction into LDS ----
      Rec r;
      bool keep = false;
      const int64_t p = p0 + tid;
      if (p < phi) keep = stage_line<Rec, PROF, WAVES>(g, cd, p, tlo, thi, ROWB, r);
      const unsigned long long bal = __ballot(keep);
      const int before = __builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
      if (lane == 0) s_wcnt[wave] = __popcll(bal);
      __syncthreads();
      int base = 0, total = 0;
#pragma unroll
      for (int w2 = 0; w2 < WAVES; ++w2) {
        int cnum = s_wcnt[w2];
        base += (w2 < wave) ? cnum : 0;
        total += cnum;
      }
      if (keep) srec[base + before] = r;
      __syncthreads();

      // ---- evaluate every staged line over this wave's row ----
      for (int l = 0; l < total; ++l) {
        const Rec& rr = srec[l];
        const int cls = (uni(rr.cls) >> (2 * wave)) & 3;
        if (cls == kRowSkip) continue;
        if constexpr (F32) {
          // x = (k - k_c) a - b, with k - k_c = (tlo - k_c) + (offset in tile): integers,
          // exact in FP32 within a window
          const float a = rr.a, nb = rr.nb;
          const float jf0 = rr.jfb + lane_off;
          if (cls != kRowGeneral) {
            if (PROF == XS_LORENTZ) {
              const float c0 = rr.c0;
#pragma unroll
              for (int j = 0; j < M; ++j) {
                const float x = fmaf(jf0 + (float)(64 * j), a, nb);
                acc32[j] = fmaf(c0, rcp32(fmaf(x, x, 1.0f)), acc32[j]);
              }
            } else if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN) {
              const float c0 = rr.c0;
#pragma unroll
              for (int j = 0; j < M; ++j) {
                const float x = fmaf(jf0 + (float)(64 * j), a, nb);
                acc32[j] = fmaf(c0, __builtin_amdgcn_exp2f(-(x * x)), acc32[j]);
              }
            } else if (cls == kRowF1) {
              const float cw = rr.A.cw, cwp = rr.A.cwp, q = rr.A.q, p2 = rr.A.p2;
#pragma unroll
              for (int j = 0; j < M; ++j) {
                const float x = fmaf(jf0 + (float)(64 * j), a, nb);
                const float u = x * x;
                acc32[j] = fmaf(fmaf(cw, u, cwp), rcp32(fmaf(u, u + q, p2)), acc32[j]);
              }
            } else {
              const Pair<float> B1 = rr.B1, B2 = rr.B2;
#pragma unroll
              for (int j = 0; j < M; ++j) {
                const float x = fmaf(jf0 + (float)(64 * j), a, nb);
                const float u = x * x;
                acc32[j] += pair_term<float>(B1, u) + pair_term<float>(B2, u);
              }
            }
            continue;
          }
          // general path: per-chunk decisions
          const int klo = uni(rr.klo), khi = uni(rr.khi);
          const KRange rB = {uni(rr.rB.lo), uni(rr.rB.hi)};
          const KRange rC = {uni(rr.rC.lo), uni(rr.rC.hi)};
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
              const float u = x * x;
              const Pair<float> A = rr.A;
              v = fmaf(A.cw, u, A.cwp) * rcp32(fmaf(u, u + A.q, A.p2));
            } else if (!meets(cl, ch, rC)) {
              const float u = x * x;
              v = pair_term<float>(rr.B1, u) + pair_term<float>(rr.B2, u);
            } else {
              v = voigt_near_f32(x, rr.y, rr.c0, rr.B1, rr.B2);
            }
            acc32[j] += (full || (k >= klo && k <= khi)) ? v : 0.0f;
          }
        } else {
          // FP64 form: x from the exact difference nu_k - nu_i
          const double nu = rr.nu, inv = rr.inv;
          double xs[M];
#pragma unroll
          for (int j = 0; j < M; ++j) {
#pragma clang fp contract(off)
            xs[j] = (nuk[j] - nu) * inv;
          }
          if (cls != kRowGeneral) {
            if (PROF == XS_LORENTZ) {
              const double c0 = rr.c0;
#pragma unroll
              for (int j = 0; j < M; ++j) acc64[j] = fma(c0, rcp64(fma(xs[j], xs[j], 1.0)), acc64[j]);
            } else if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN) {
              const double c0 = rr.c0;
#pragma unroll
              for (int j = 0; j < M; ++j) acc64[j] = fma(c0, exp2(-(xs[j] * xs[j])), acc64[j]);
            } else if (cls == kRowF1) {
              const Pair<double> A = rr.A;
#pragma unroll
              for (int j = 0; j < M; ++j) acc64[j] += pair_term<double>(A, xs[j] * xs[j]);
            } else {
              const Pair<double> B1 = rr.B1, B2 = rr.B2;
#pragma unroll
              for (int j = 0; j < M; ++j) acc64[j] += pair2_term(B1, B2, xs[j] * xs[j]);
            }
            continue;
          }
          const int klo = uni(rr.klo), khi = uni(rr.khi);
#pragma unroll
          for (int j = 0; j < M; ++j) {
            const int cl = row_lo + 64 * j, ch = cl + 63;
            if (ch < klo || cl > khi) continue;
            const bool full = cl >= klo && ch <= khi;
            const int k = my0 + 64 * j;
            const double x = xs[j];
            double v;
            if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN) {
              if (!meets(cl, ch, KRange{uni(rr.r[0].lo), uni(rr.r[0].hi)})) continue;
              v = rr.c0 * exp2(-(x * x));
            } else if (PROF == XS_LORENTZ) {
              v = rr.c0 * rcp64(fma(x, x, 1.0));
            } else {
              const double u = x * x;
              if (!meets(cl, ch, KRange{uni(rr.r[0].lo), uni(rr.r[0].hi)})) {
                v = pair_term<double>(rr.A, u);
              } else if (!meets(cl, ch, KRange{uni(rr.r[1].lo), uni(rr.r[1].hi)})) {
                v = pair2_term(rr.B1, rr.B2, u);
              } else if (!meets(cl, ch, KRange{uni(rr.r[2].lo), uni(rr.r[2].hi)})) {
                v = gh_pairs_y<3>(rr.c0, rr.y, u);
              } else if (!meets(cl, ch, KRange{uni(rr.r[3].lo), uni(rr.r[3].hi)})) {
                v = gh_pairs_y<4>(rr.c0, rr.y, u);
              } else if (!meets(cl, ch, KRange{uni(rr.r[4].lo), uni(rr.r[4].hi)}) || u + rr.y * rr.y >= 64.0) {
                v = gh_pairs_y<6>(rr.c0, rr.y, u);
              } else {
                double wr, wi;
                w_core<22>(x, rr.y, wr, wi);
                v = rr.c0 * wr;
              }
            }
            if (full || (k >= klo && k <= khi)) acc64[j] += v;
          }
        }
      }
      if constexpr (F32) {
#pragma unroll
        for (int j = 0; j < M; ++j) {
          acc64[j] += (double)acc32[j];
          acc32[j] = 0.0f;
        }
      }
      __syncthreads();
    }

    // ---- write the tile ----
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
    if (!g.persistent) return;
  }
}

template <typename Real, int PROF>
static void gather_dispatch(const GatherArgs& a, const Tiling& t, int blocks, hipStream_t s) {
  const int w = t.waves, M = t.per_lane;
#define XS_G(MM, WW)                                                                       \
  if (M == MM && w == WW) {                                                                \
    hipLaunchKernelGGL((k_gather<Real, PROF, MM, WW>), dim3(blocks), dim3(64 * WW), 0, s, a); \
    return;                                                                                \
  }
  XS_G(4, 1) XS_G(8, 1) XS_G(4, 2) XS_G(8, 2) XS_G(2, 4) XS_G(4, 4) XS_G(8, 4)
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
  a.rS = w.rS;
  a.max_lines = w.max_lines;
  a.counter = w.counter;
  a.sigma = sigma;
  a.accumulate = accumulate;
  a.tile_bins = t.tile_bins;
  a.n_tiles = (int)((m.n_bins + t.tile_bins - 1) / t.tile_bins);
  a.n_items = (int64_t)a.n_tiles * m.n_cond;
  a.persistent = t.persistent;
  const int blocks = t.persistent ? t.grid_blocks : (int)a.n_items;
#define XS_P(R, P)                                   \
  if (m.profile == P) {                              \
    gather_dispatch<R, P>(a, t, blocks, s);          \
    return;                                          \
  }
  if (m.prec == XS_FP32) {
    XS_P(float, XS_DOPPLER) XS_P(float, XS_GAUSSIAN) XS_P(float, XS_LORENTZ) XS_P(float, XS_VOIGT)
  } else {
    XS_P(double, XS_DOPPLER) XS_P(double, XS_GAUSSIAN) XS_P(double, XS_LORENTZ) XS_P(double, XS_VOIGT)
  }
#undef XS_P
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
    double wr, wi;
    w_core<16>((double)x, (double)r.y, wr, wi);
    return r.c0 * (float)wr;
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
    LineParams lp = line_params<PROF>(m, cd, nu, (double)g.rgref[p], (double)g.rnexp[p], S);
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
}

}  // namespace xs
