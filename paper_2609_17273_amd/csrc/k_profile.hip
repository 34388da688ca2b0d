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

// Per-(line, condition) record staged in LDS.
struct RecF {
  int kc, klo, khi, flag;
  float a, b, y, y2, q, c0, cy, pad;
};
struct RecD {
  int kc, klo, khi, flag;
  float af, bf, y2f, pad;
  double nu, inv, y, y2, q, c0, cy, pad2;
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
__device__ __forceinline__ float uni(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double uni(double v) {
  long long b = __double_as_longlong(v);
  int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffff));
  int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Per-(line, condition) parameters.  For every profile the lane variable is
// x = (k - k_c) a - b = (nu_k - nu_i) * inv, with inv = 1/alpha (Gaussian, so
// f = c0 2^{-x^2}), 1/gamma (Lorentzian, f = c0 / (1 + x^2)) or
// 1/(sg sqrt 2) = sqrt(ln 2)/alpha (Voigt, f = c0 Re w(x + i y)).
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

// Staging: does line p touch bins [tlo, thi] under condition cd?  Fills rec.
template <typename Rec, int PROF>
__device__ bool stage_line(const GatherArgs& g, const CondDev& cd, int64_t p, int64_t tlo,
                           int64_t thi, Rec& r) {
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
  LineParams lp = line_params<PROF>(m, cd, nu, (double)g.rgref[p], (double)g.rnexp[p], S);
  r.kc = (int)kc;
  r.klo = (int)(klo > tlo ? klo : tlo);
  r.khi = (int)(khi < thi ? khi : thi);
  r.flag = 0;
  const double a = m.dnu * lp.inv, b = delta * lp.inv;
  if constexpr (sizeof(Rec) == sizeof(RecF)) {
    r.a = (float)a;
    r.b = (float)b;
    r.y = (float)lp.y;
    r.y2 = (float)(lp.y * lp.y);
    r.q = (float)(4.0 * lp.y * lp.y);
    r.c0 = (float)lp.c0;
    r.cy = (float)(lp.c0 * 2.0 * lp.y / kPI);
    // FP32 keeps (x^2 + y^2)^2 finite for |x|, y < ~1e9; beyond that
    // (lines with nu of a few 1e-3 cm^-1 or less) evaluate in FP64.
    double xmax = fmax(fabs((double)(r.klo - r.kc) * a - b), fabs((double)(r.khi - r.kc) * a - b));
    if (PROF == XS_VOIGT && (xmax > 1.0e9 || lp.y > 1.0e9)) r.flag = 1;
  } else {
    r.af = (float)a;
    r.bf = (float)b;
    r.y2f = (float)(lp.y * lp.y);
    r.nu = nu;
    r.inv = lp.inv;
    r.y = lp.y;
    r.y2 = lp.y * lp.y;
    r.q = 4.0 * lp.y * lp.y;
    r.c0 = lp.c0;
    r.cy = lp.c0 * 2.0 * lp.y / kPI;
  }
  return true;
}

// Contribution of one line to one bin given x (profile value times c0),
// FP32 form.  band: 1 = one Gauss-Hermite pair, 2 = two pairs, 0 = per lane.
template <int PROF>
__device__ __forceinline__ float eval_f32(const RecF& r, float x, int band) {
  if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN) {
    return r.c0 * __builtin_amdgcn_exp2f(-x * x);
  } else if (PROF == XS_LORENTZ) {
    return r.c0 * __builtin_amdgcn_rcpf(fmaf(x, x, 1.0f));
  } else {
    const float u = x * x;
    if (band == 1) return r.cy * gh_re_sum<1, float>(u, r.y2, r.q);
    if (band == 2 || u + r.y2 >= 64.0f) return r.cy * gh_re_sum<2, float>(u, r.y2, r.q);
    double wr, wi;
    w_core<16>((double)x, (double)r.y, wr, wi);
    return r.c0 * (float)wr;
  }
}

// FP64 form: x from the exact difference nu_k - nu_i.
template <int PROF>
__device__ __forceinline__ double eval_f64(const RecD& r, double x, int band) {
  if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN) {
    return r.c0 * exp2(-x * x);
  } else if (PROF == XS_LORENTZ) {
    return r.c0 / fma(x, x, 1.0);
  } else {
    const double u = x * x;
    switch (band) {
      case 1: return r.cy * gh_re_sum<1, double>(u, r.y2, r.q);
      case 2: return r.cy * gh_re_sum<2, double>(u, r.y2, r.q);
      case 3: return r.cy * gh_re_sum<3, double>(u, r.y2, r.q);
      case 4: return r.cy * gh_re_sum<4, double>(u, r.y2, r.q);
      case 6: return r.cy * gh_re_sum<6, double>(u, r.y2, r.q);
      default: break;
    }
    if (u + r.y2 >= 64.0) return r.cy * gh_re_sum<6, double>(u, r.y2, r.q);
    double wr, wi;
    w_core<22>(x, r.y, wr, wi);
    return r.c0 * wr;
  }
}

// Smallest |x| over the row [row_lo, row_lo + nb - 1] from its end bins.
__device__ __forceinline__ float row_min_abs_x(int row_lo, int nb, int kc, float a, float b) {
  float x0 = fmaf((float)(row_lo - kc), a, -b);
  float x1 = fmaf((float)(row_lo + nb - 1 - kc), a, -b);
  if (x0 <= 0.0f && x1 >= 0.0f) return 0.0f;
  return fminf(fabsf(x0), fabsf(x1));
}

// Band of a row (every lane uses at least as many Gauss-Hermite nodes as its
// own |z| requires, so rows do not diverge); 0: some lane may be in the core.
template <int PROF>
__device__ __forceinline__ int row_band_f32(float xmin, float y2) {
  if (PROF != XS_VOIGT) return 1;
  float rho = xmin * xmin + y2;
  if (rho >= 900.0f * 1.001f) return 1;
  if (rho >= 64.0f * 1.001f) return 2;
  return 0;
}
template <int PROF>
__device__ __forceinline__ int row_band_f64(float xmin, float y2) {
  if (PROF != XS_VOIGT) return 1;
  float rho = xmin * xmin + y2;
  if (rho >= 9.0e6f * 1.001f) return 1;
  if (rho >= 6400.0f * 1.001f) return 2;
  if (rho >= 400.0f * 1.001f) return 3;
  if (rho >= 144.0f * 1.001f) return 4;
  if (rho >= 64.0f * 1.001f) return 6;
  return 0;
}

// A Gaussian row whose smallest |x| makes 2^{-x^2} vanish in the working
// precision contributes exactly zero and is skipped.
template <int PROF>
__device__ __forceinline__ bool row_zero(float xmin, bool f32) {
  if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN) return xmin * xmin > (f32 ? 160.0f : 1100.0f);
  return false;
}

template <typename Real, int PROF, int M, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_gather(GatherArgs g) {
  using Rec = typename std::conditional<sizeof(Real) == 4, RecF, RecD>::type;
  constexpr bool F32 = sizeof(Real) == 4;
  constexpr int NT = 64 * WAVES;
  constexpr int ROWB = 64 * M;  // bins per wave row
  __shared__ Rec srec[NT];
  __shared__ int s_wcnt[WAVES];
  __shared__ long long s_item;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
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
    const int my_lo = row_lo + lane * M;

    double acc64[M];
    float acc32[M];
    double nuk[M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
      acc64[j] = 0.0;
      acc32[j] = 0.0f;
      if (!F32) nuk[j] = nu_of_bin(m.nu0, m.dnu, my_lo + j);
    }

    for (int64_t p0 = plo; p0 < phi; p0 += NT) {
      // ---- stage: exact window test, compaction into LDS ----
      Rec r;
      bool keep = false;
      const int64_t p = p0 + tid;
      if (p < phi) keep = stage_line<Rec, PROF>(g, cd, p, tlo, thi, r);
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
        const int kc = uni(srec[l].kc), klo = uni(srec[l].klo), khi = uni(srec[l].khi);
        if (khi < row_lo || klo > row_lo + ROWB - 1) continue;
        const bool full = klo <= row_lo && khi >= row_lo + ROWB - 1;
        if constexpr (F32) {
          const RecF rr = srec[l];
          const float a = uni(rr.a), b = uni(rr.b);
          const float xmin = row_min_abs_x(row_lo, ROWB, kc, a, b);
          if (row_zero<PROF>(xmin, true)) continue;
          if (PROF == XS_VOIGT && uni(rr.flag)) {
#pragma unroll
            for (int j = 0; j < M; ++j) {
              const int k = my_lo + j;
              if (k >= klo && k <= khi) {
                double x = (double)(k - kc) * (double)a - (double)b;
                acc32[j] += (float)((double)rr.c0 * re_w_f64(x, (double)rr.y));
              }
            }
            continue;
          }
          const int band = row_band_f32<PROF>(xmin, uni(rr.y2));
          RecF ru = rr;
          ru.y2 = uni(rr.y2);
          ru.q = uni(rr.q);
          ru.c0 = uni(rr.c0);
          ru.cy = uni(rr.cy);
          ru.y = uni(rr.y);
          if (full) {
#pragma unroll
            for (int j = 0; j < M; ++j) {
              const float x = fmaf((float)(my_lo + j - kc), a, -b);
              acc32[j] += eval_f32<PROF>(ru, x, band);
            }
          } else {
#pragma unroll
            for (int j = 0; j < M; ++j) {
              const int k = my_lo + j;
              const float x = fmaf((float)(k - kc), a, -b);
              const float v = eval_f32<PROF>(ru, x, band);
              acc32[j] += (k >= klo && k <= khi) ? v : 0.0f;
            }
          }
        } else {
          const RecD rr = srec[l];
          const float xmin = row_min_abs_x(row_lo, ROWB, kc, uni(rr.af), uni(rr.bf));
          if (row_zero<PROF>(xmin, false)) continue;
          const int band = row_band_f64<PROF>(xmin, uni(rr.y2f));
          RecD ru = rr;
          ru.nu = uni(rr.nu);
          ru.inv = uni(rr.inv);
          ru.y = uni(rr.y);
          ru.y2 = uni(rr.y2);
          ru.q = uni(rr.q);
          ru.c0 = uni(rr.c0);
          ru.cy = uni(rr.cy);
#pragma unroll
          for (int j = 0; j < M; ++j) {
            const int k = my_lo + j;
            double x;
            {
#pragma clang fp contract(off)
              x = (nuk[j] - ru.nu) * ru.inv;
            }
            const double v = eval_f64<PROF>(ru, x, band);
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
      const int64_t k = my_lo + j;
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
  XS_G(2, 4) XS_G(4, 4) XS_G(8, 4) XS_G(4, 8) XS_G(2, 8)
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
      RecF r;
      const int64_t kc = home_bin(nu, m.nu0, m.dnu);
      const double delta = nu - nu_of_bin(m.nu0, m.dnu, kc);
      r.kc = (int)kc;
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
          v = (x * x > 160.0f) ? 0.0f : eval_f32<PROF>(r, x, 1);
        else
          v = eval_f32<PROF>(r, x, 0);
        if (v != 0.0f) unsafeAtomicAdd(out + k, scale * (double)v);
      }
    } else {
      RecD r;
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
          v = (x * x > 1100.0) ? 0.0 : eval_f64<PROF>(r, x, 1);
        else
          v = eval_f64<PROF>(r, x, 0);
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
