// Host runtime of the cross-section library: the C-ABI of include/xsec.h.
//
// A plan holds the model, grid and conditions, the kernel configuration and
// the caller-bound device workspace.  Each call validates every argument on
// the host first (no HIP call before validation succeeds), then enqueues the
// path on the plan's stream:
//   partition functions -> intensity pass 1 (keys, ln S max) -> stable radix
//   sort by bucket -> bucket offsets + sorted records -> profile pass
//   (gather or scatter) [-> adjoint].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "xsec_internal.h"

using namespace xs;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

bool finite(double v) { return std::isfinite(v); }

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return XS_EDEVICE;
  }
  return XS_OK;
}

}  // namespace

struct xs_plan {
  xs_model model;
  xs_grid grid;
  std::vector<xs_condition> conds;
  int64_t max_lines;
  hipStream_t stream;
  int device;
  int n_cu;
  std::string arch;
  // derived
  ModelDev md;
  std::vector<CondDev> cdev;
  std::vector<SlotDev> sdev;
  std::vector<double> cut_class;
  std::vector<int32_t> cut_mult;
  Tiling tiling;
  int32_t bucket_bins;
  // workspace
  void* ws = nullptr;
  size_t ws_bytes = 0;
  Work w;
  // graph
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int64_t last_lines_in = 0;
  bool prepared = false;     // records of an xs_prepare are in the workspace
  std::vector<double> cf_T;  // temperatures of the last cooling-function call (upload source)
  bool has_tau = false;      // the last xs_prepare had state lifetimes (records hold their widths)
};

namespace {

int validate_model(const xs_model* m) {
  if (!m) return fail(XS_EINVAL, "model is NULL");
  if (m->profile < XS_DOPPLER || m->profile > XS_PV_OLIVERO) return fail(XS_EINVAL, "model.profile out of range");
  const int base = base_profile(m->profile);
  if (m->mode < XS_ABSORPTION || m->mode > XS_EMISSION) return fail(XS_EINVAL, "model.mode out of range");
  if (m->population < XS_LTE || m->population > XS_NLTE_DENSITY)
    return fail(XS_EINVAL, "model.population out of range");
  if (m->precision < XS_FP64 || m->precision > XS_FP32) return fail(XS_EINVAL, "model.precision out of range");
  if (m->algo < XS_GATHER || m->algo > XS_SCATTER) return fail(XS_EINVAL, "model.algo out of range");
  if ((base == XS_DOPPLER || base == XS_VOIGT) && !(m->mass_amu > 0.0 && finite(m->mass_amu)))
    return fail(XS_EINVAL, "model.mass_amu must be > 0");
  if (!(m->T_ref > 0.0 && finite(m->T_ref))) return fail(XS_EINVAL, "model.T_ref must be > 0");
  if (!(m->P_ref > 0.0 && finite(m->P_ref))) return fail(XS_EINVAL, "model.P_ref must be > 0");
  if (base == XS_GAUSSIAN && !(m->hwhm_fixed > 0.0 && finite(m->hwhm_fixed)))
    return fail(XS_EINVAL, "model.hwhm_fixed must be > 0 for XS_GAUSSIAN / XS_BIN_GAUSSIAN");
  return XS_OK;
}

int validate_grid(const xs_grid* g) {
  if (!g) return fail(XS_EINVAL, "grid is NULL");
  if (!finite(g->nu0)) return fail(XS_EINVAL, "grid.nu0 not finite");
  if (!(g->dnu > 0.0 && finite(g->dnu))) return fail(XS_EINVAL, "grid.dnu must be > 0");
  if (g->n_bins < 1 || g->n_bins > (int64_t(1) << 30)) return fail(XS_EINVAL, "grid.n_bins must be in [1, 2^30]");
  return XS_OK;
}

int validate_conds(const xs_model* m, const xs_grid* g, int32_t n, const xs_condition* c) {
  if (n < 1 || n > kMaxCond) return fail(XS_EINVAL, "n_cond must be in [1, 256]");
  if (!c) return fail(XS_EINVAL, "conditions are NULL");
  for (int i = 0; i < n; ++i) {
    const xs_condition& q = c[i];
    std::string id = "condition " + std::to_string(i) + ": ";
    if (!(q.cutoff > 0.0 && finite(q.cutoff))) return fail(XS_EINVAL, id + "cutoff must be > 0");
    if (q.cutoff / g->dnu > double(1 << 28)) return fail(XS_EINVAL, id + "cutoff / dnu too large");
    if (!(q.P >= 0.0 && finite(q.P))) return fail(XS_EINVAL, id + "P must be >= 0");
    if (base_profile(m->profile) == XS_LORENTZ && !(q.P > 0.0))
      return fail(XS_EINVAL, id + "P must be > 0 for XS_LORENTZ / XS_BIN_LORENTZ");
    if (m->population == XS_LTE) {
      if (!(q.T > 0.0 && finite(q.T))) return fail(XS_EINVAL, id + "T must be > 0");
    } else {
      if (m->population == XS_NLTE_2T && !(q.T_vib > 0.0 && finite(q.T_vib)))
        return fail(XS_EINVAL, id + "T_vib must be > 0");
      if (!(q.T_rot > 0.0 && finite(q.T_rot))) return fail(XS_EINVAL, id + "T_rot must be > 0");
    }
  }
  return XS_OK;
}

int validate_states(const xs_plan* p, const xs_states* s) {
  if (!s) return fail(XS_EINVAL, "states is NULL");
  if (s->n < 1 || s->n > (int64_t(1) << 31) - 1) return fail(XS_EINVAL, "states.n must be in [1, 2^31-1]");
  if (!s->energy || !s->g_tot) return fail(XS_EINVAL, "states.energy / states.g_tot is NULL");
  if (p->model.population != XS_LTE) {
    if (!s->v || !s->e_vib) return fail(XS_EINVAL, "non-LTE runs need states.v and states.e_vib");
    if (s->n_v < 1) return fail(XS_EINVAL, "states.n_v must be >= 1");
    if (p->model.population == XS_NLTE_DENSITY && !s->n_vib)
      return fail(XS_EINVAL, "custom-density runs need states.n_vib");
  }
  return XS_OK;
}

int validate_lines(const xs_plan* p, const xs_lines* l) {
  if (!l) return fail(XS_EINVAL, "lines is NULL");
  if (l->n < 0 || l->n > p->max_lines) return fail(XS_EINVAL, "lines.n must be in [0, max_lines]");
  if (l->n > 0 && (!l->upper || !l->lower || !l->einstein_a))
    return fail(XS_EINVAL, "lines.upper / lower / einstein_a is NULL");
  const int prof = base_profile(p->model.profile);
  if ((prof == XS_LORENTZ || prof == XS_VOIGT)) {
    if (!l->gamma_ref && !(l->gamma_ref_scalar >= 0.0 && finite(l->gamma_ref_scalar)))
      return fail(XS_EINVAL, "lines.gamma_ref_scalar must be >= 0");
    if (!l->n_exp && !finite(l->n_exp_scalar)) return fail(XS_EINVAL, "lines.n_exp_scalar not finite");
  }
  return XS_OK;
}

int validate_config(const xs_config* c) {
  if (!c) return fail(XS_EINVAL, "config is NULL");
  if (c->tile_bins != 256 && c->tile_bins != 512 && c->tile_bins != 1024)
    return fail(XS_EINVAL, "config.tile_bins must be 256, 512 or 1024");
  if (c->chunk_lines < 0 || c->chunk_lines > (1 << 30) || c->chunk_lines % 64)
    return fail(XS_EINVAL, "config.chunk_lines must be 0 or a multiple of 64 up to 2^30");
  const int b = c->bucket_bins;
  if (b < 64 || b > 4096 || (b & (b - 1))) return fail(XS_EINVAL, "config.bucket_bins must be a power of two in [64, 4096]");
  if (c->persistent != 0 && c->persistent != 1) return fail(XS_EINVAL, "config.persistent must be 0 or 1");
  if (c->waves_per_cu < 4 || c->waves_per_cu > 64) return fail(XS_EINVAL, "config.waves_per_cu must be in [4, 64]");
  if (c->adj_blocks != 0 && (c->adj_blocks < 256 || c->adj_blocks > kAdjBlocksMax || c->adj_blocks % 256))
    return fail(XS_EINVAL, "config.adj_blocks must be 0 or a multiple of 256 in [256, 32768]");
  return XS_OK;
}

StatesView view(const xs_states* s) {
  StatesView v;
  v.n = s->n;
  v.E = s->energy;
  v.g = s->g_tot;
  v.v = s->v;
  v.ev = s->e_vib;
  v.n_v = s->n_v;
  v.nv = s->n_vib;
  v.tau = s->lifetime;
  return v;
}

LinesView view(const xs_lines* l) {
  LinesView v;
  v.n = l->n;
  v.up = l->upper;
  v.lo = l->lower;
  v.A = l->einstein_a;
  v.gref = l->gamma_ref;
  v.nexp = l->n_exp;
  v.lscale = l->log_scale;
  v.gref_scalar = l->gamma_ref_scalar;
  v.nexp_scalar = l->n_exp_scalar;
  return v;
}

// Tile shape (64 lanes x tile_bins / 64 bins), launch mode and lines per work item.
void tiling_for(xs_plan* p, int tile_bins, int persistent, int waves_per_cu, int chunk_lines,
                int adj_blocks) {
  Tiling t;
  t.tile_bins = tile_bins;
  t.persistent = persistent;
  t.grid_blocks = std::max(1, p->n_cu * waves_per_cu);
  t.chunk_lines = chunk_lines;
  t.adj_blocks = adj_blocks > 0 ? adj_blocks : kAdjBlocks;
  p->tiling = t;
}

void derive(xs_plan* p) {
  const xs_model& m = p->model;
  ModelDev& d = p->md;
  d.profile = m.profile;
  d.mode = m.mode;
  d.pop = m.population;
  d.prec = m.precision;
  d.nu0 = p->grid.nu0;
  d.dnu = p->grid.dnu;
  d.n_bins = p->grid.n_bins;
  d.T_ref = m.T_ref;
  d.P_ref = m.P_ref;
  d.hwhm_fixed = m.hwhm_fixed;
  d.mass_amu = m.mass_amu;
  d.n_cond = (int32_t)p->conds.size();
  d.bucket_bins = p->bucket_bins;
  d.n_buckets = (int32_t)((p->grid.n_bins + p->bucket_bins - 1) / p->bucket_bins);
  d.n_fine = (int32_t)((p->grid.n_bins + kFineBins - 1) / kFineBins);
  d.fine_per_bucket = p->bucket_bins / kFineBins;
  // intensity slots: distinct population temperatures
  p->sdev.clear();
  p->cdev.clear();
  p->cut_class.clear();
  p->cut_mult.clear();
  double maxcut = 0.0;
  for (const xs_condition& c : p->conds) {
    SlotDev s;
    if (m.population == XS_LTE) {
      s.T = c.T;
      s.Tv = c.T;
      s.Tr = c.T;
    } else {
      s.T = c.T_rot;
      s.Tv = (m.population == XS_NLTE_2T) ? c.T_vib : 0.0;  // unused with densities
      s.Tr = c.T_rot;
    }
    int slot = -1;
    for (size_t q = 0; q < p->sdev.size(); ++q)
      if (p->sdev[q].Tv == s.Tv && p->sdev[q].Tr == s.Tr) slot = (int)q;
    if (slot < 0) {
      slot = (int)p->sdev.size();
      p->sdev.push_back(s);
    }
    CondDev cd;
    cd.T = c.T;
    cd.P = c.P;
    cd.Tv = c.T_vib;
    cd.Tr = c.T_rot;
    cd.cut = c.cutoff;
    cd.Tk = (m.population == XS_LTE) ? c.T : c.T_rot;
    cd.dop = (base_profile(m.profile) == XS_GAUSSIAN || base_profile(m.profile) == XS_LORENTZ)
                 ? 0.0
                 : std::sqrt(2.0 * kKB * cd.Tk * kLN2 / (m.mass_amu * kAMU)) / kC;
    cd.hwhm = m.hwhm_fixed;
    cd.lnTr = std::log(m.T_ref / cd.Tk);
    cd.pfac = c.P / m.P_ref;
    cd.slot = slot;
    cd.wbins = (int32_t)std::ceil(c.cutoff / p->grid.dnu) + 2;
    if (base_profile(m.profile) == XS_DOPPLER || base_profile(m.profile) == XS_GAUSSIAN) {
      // 2^{-(d/alpha)^2} is exactly zero in the working precision once
      // (d/alpha)^2 exceeds 160 (FP32) or 1100 (FP64), and a bin mean once
      // its nearer edge lies beyond 10.1 (FP32) or 27.3 (FP64) in units of
      // alpha/sqrt(ln2); a kept line has nu <= grid end + cut-off, so no line
      // reaches a tile from farther than that: the gather need not stage it.
      const bool binned = m.profile >= XS_BIN_DOPPLER;
      const bool f32 = m.precision == XS_FP32;
      const double nu_end = p->grid.nu0 + (double)(p->grid.n_bins - 1) * p->grid.dnu;
      const double amax = (base_profile(m.profile) == XS_GAUSSIAN) ? m.hwhm_fixed : (nu_end + c.cutoff) * cd.dop;
      const double dmax = binned ? (f32 ? 10.1 : 27.3) / std::sqrt(kLN2) * amax + 0.5 * p->grid.dnu
                                 : (f32 ? std::sqrt(160.0) : std::sqrt(1100.0)) * amax;
      const double reach = std::ceil(dmax / p->grid.dnu) + 2.0;
      if (std::isfinite(reach) && reach < (double)cd.wbins) cd.wbins = (int32_t)reach;
    }
    maxcut = std::max(maxcut, c.cutoff);
    int cc = -1;
    for (size_t q = 0; q < p->cut_class.size(); ++q)
      if (p->cut_class[q] == c.cutoff) cc = (int)q;
    if (cc < 0) {
      cc = (int)p->cut_class.size();
      p->cut_class.push_back(c.cutoff);
      p->cut_mult.push_back(1);
    } else {
      p->cut_mult[cc] += 1;
    }
    cd.cclass = cc;
    cd.pad = 0;
    p->cdev.push_back(cd);
  }
  d.n_slots = (int32_t)p->sdev.size();
  d.n_cut_classes = (int32_t)p->cut_class.size();
  d.max_cut = maxcut;
}

// item_target: gather work items aimed at when tiles are split (sizes the
// partial-row buffer, 2 item_target rows); 0 = kItemsPerCU per compute unit.
// with_adjoint: carve the adjoint's per-block partial sums (the
// allocation-free forward path leaves them out).
size_t layout(xs_plan* p, char* base, Work* w, int64_t item_target = 0, bool with_adjoint = true) {
  const ModelDev& d = p->md;
  const int64_t L = p->max_lines;
  const int nsb = (int)((L + kSortBlock - 1) / kSortBlock);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + std::max<size_t>(bytes, 1));
    return base ? (void*)(base + at) : nullptr;
  };
  Work x;
  x.cond = (CondDev*)take(sizeof(CondDev) * d.n_cond);
  x.slot = (SlotDev*)take(sizeof(SlotDev) * d.n_slots);
  x.model = (ModelDev*)take(sizeof(ModelDev));
  x.qpart = (double*)take(sizeof(double) * d.n_slots * 2 * kQBlocks);
  x.Q = (double*)take(sizeof(double) * d.n_slots);
  x.dQ = (double*)take(sizeof(double) * d.n_slots);
  x.smax = (unsigned long long*)take(8 * d.n_slots);
  x.sb = (double*)take(8 * d.n_slots);
  x.key = (int32_t*)take(4 * L);
  x.keyA = (int32_t*)take(4 * L);
  x.valA = (int32_t*)take(4 * L);
  // keyB and valB adjacent: before the sort's last pass they hold the first
  // line pass's packed state table
  x.keyB = (int32_t*)take(4 * L);
  x.valB = (int32_t*)take(4 * L);
  x.hist = (int32_t*)take(4 * (size_t)256 * nsb);
  x.hsum = (int32_t*)take(4 * ((size_t)256 * nsb / 1024 + 2));
  // sized for the finest bucket (64 points), so a change of bucket size never
  // needs a larger workspace
  x.off = (int32_t*)take(4 * (size_t)((p->grid.n_bins + 63) / 64 + 2));
  x.rnu = (double*)take(8 * L);
  x.rgref = (float*)take(4 * L);
  x.rnexp = (float*)take(4 * L);
  x.rgpre = (double*)take(8 * L);
  x.ridx = (int32_t*)take(4 * L);
  x.rEs = (double*)take(8 * L);
  x.lpack = (LinePack*)take(sizeof(LinePack) * L);
  x.rkc = (int32_t*)take(4 * L);
  x.rdel = (float*)take(4 * L);
  x.rwin = (int32_t*)take(8 * (size_t)d.n_cut_classes * L);
  x.rS = take((size_t)(d.prec == XS_FP32 ? 4 : 8) * d.n_slots * L);
  x.counter = (int32_t*)take(4 * kCounterInts);
  {
    // work items of the gather: sized for the smallest tile (256 bins)
    const int64_t n_ct = (int64_t)d.n_cond * ((p->grid.n_bins + 255) / 256);
    x.item_cnt = (int32_t*)take(4 * (size_t)n_ct);
    x.item_base = (int32_t*)take(4 * (size_t)(n_ct + 1));
    x.part_base = (int32_t*)take(4 * (size_t)(n_ct + 1));
    x.item_sums = (int32_t*)take(4 * (size_t)((n_ct + 1) / 1024 + 2));
    x.item_target = item_target > 0 ? item_target : kItemsPerCU * (int64_t)std::max(1, p->n_cu);
    x.part = (double*)take(sizeof(double) * 2 * (size_t)x.item_target * 1024);
  }
  x.stats = (unsigned long long*)take(8 * 8);
  x.adjpart = with_adjoint ? (double*)take(sizeof(double) * d.n_cond * 2 * kAdjBlocksMax) : nullptr;
  x.gmax = (unsigned long long*)take(sizeof(unsigned long long) * d.n_cond);
  x.cut_class = (double*)take(sizeof(double) * d.n_cut_classes);
  x.cut_mult = (int32_t*)take(sizeof(int32_t) * d.n_cut_classes);
  x.max_lines = L;
  x.n_sort_blocks = nsb;
  if (w) *w = x;
  return o;
}

int upload(xs_plan* p) {
  const ModelDev& d = p->md;
  int rc;
  if ((rc = hip_check(hipMemcpyAsync(p->w.cond, p->cdev.data(), sizeof(CondDev) * d.n_cond,
                                     hipMemcpyHostToDevice, p->stream), "upload conditions")))
    return rc;
  if ((rc = hip_check(hipMemcpyAsync(p->w.slot, p->sdev.data(), sizeof(SlotDev) * d.n_slots,
                                     hipMemcpyHostToDevice, p->stream), "upload slots")))
    return rc;
  if ((rc = hip_check(hipMemcpyAsync(p->w.model, &p->md, sizeof(ModelDev), hipMemcpyHostToDevice,
                                     p->stream), "upload model")))
    return rc;
  if ((rc = hip_check(hipMemcpyAsync(p->w.cut_class, p->cut_class.data(),
                                     sizeof(double) * d.n_cut_classes, hipMemcpyHostToDevice,
                                     p->stream), "upload cut-offs")))
    return rc;
  if ((rc = hip_check(hipMemcpyAsync(p->w.cut_mult, p->cut_mult.data(),
                                     sizeof(int32_t) * d.n_cut_classes, hipMemcpyHostToDevice,
                                     p->stream), "upload cut-off counts")))
    return rc;
  return hip_check(hipStreamSynchronize(p->stream), "upload sync");
}

// The workspace as the kernels see it: without state lifetimes the records'
// lifetime widths are neither written nor read.
Work kernel_work(const xs_plan* p) {
  Work w = p->w;
  if (!p->has_tau) w.rgpre = nullptr;
  return w;
}

// Everything up to the sorted records; returns XS_OK once enqueued.
int preprocess(xs_plan* p, const xs_states* st, const xs_lines* ln) {
  const StatesView sv = view(st);
  const LinesView lv = view(ln);
  launch_reset(p->w, p->stream);
  launch_partition(p->md, p->w, sv, p->stream);
  launch_lines_pass1(p->md, p->w, sv, lv, p->stream);
  int32_t *sk = nullptr, *svv = nullptr;
  launch_radix_sort(p->md, p->w, lv.n, p->md.n_fine, p->stream, &sk, &svv);
  p->has_tau = st->lifetime != nullptr;
  launch_offsets_records(p->md, kernel_work(p), sv, lv, sk ? sk : p->w.keyA, svv ? svv : p->w.valA, lv.n,
                         p->stream);
  p->last_lines_in = lv.n;
  p->prepared = true;
  return hip_check(hipGetLastError(), "preprocess launch");
}

int profile_pass(xs_plan* p, double* sigma, int accumulate) {
  if (p->model.algo == XS_SCATTER)
    launch_scatter(p->md, kernel_work(p), sigma, accumulate, 0, p->stream);
  else
    launch_gather(p->md, kernel_work(p), p->tiling, sigma, accumulate, p->stream);
  return hip_check(hipGetLastError(), "profile launch");
}

int check_call(xs_plan* p, const xs_states* st, const xs_lines* ln) {
  if (!p) return fail(XS_EINVAL, "plan is NULL");
  if (!p->ws) return fail(XS_EWORKSPACE, "no workspace bound (xs_plan_set_workspace)");
  int rc;
  if ((rc = validate_states(p, st))) return rc;
  if (ln && (rc = validate_lines(p, ln))) return rc;
  return XS_OK;
}

}  // namespace

extern "C" {

const char* xs_last_error(void) { return g_err.c_str(); }

const char* xs_version(void) { return "xsec 0.1 (gfx950)"; }

int xs_plan_create(xs_plan** out, const xs_model* model, const xs_grid* grid, int32_t n_cond,
                   const xs_condition* conds, int64_t max_lines, void* stream) {
  if (!out) return fail(XS_EINVAL, "out is NULL");
  *out = nullptr;
  int rc;
  if ((rc = validate_model(model))) return rc;
  if ((rc = validate_grid(grid))) return rc;
  if ((rc = validate_conds(model, grid, n_cond, conds))) return rc;
  if (max_lines < 1 || max_lines > (int64_t(1) << 31) - 1)
    return fail(XS_EINVAL, "max_lines must be in [1, 2^31-1]");
  xs_plan* p = new (std::nothrow) xs_plan();
  if (!p) return fail(XS_ENOMEM, "plan allocation failed");
  p->model = *model;
  p->grid = *grid;
  p->conds.assign(conds, conds + n_cond);
  p->max_lines = max_lines;
  p->stream = (hipStream_t)stream;
  // narrow Gaussians reach few buckets beyond their tile, so finer buckets
  // stage fewer lines per tile; the other profiles reach a whole cut-off
  p->bucket_bins = (base_profile(model->profile) == XS_DOPPLER || base_profile(model->profile) == XS_GAUSSIAN) ? 64 : 256;
  if ((rc = hip_check(hipGetDevice(&p->device), "hipGetDevice"))) {
    delete p;
    return rc;
  }
  hipDeviceProp_t prop;
  if ((rc = hip_check(hipGetDeviceProperties(&prop, p->device), "hipGetDeviceProperties"))) {
    delete p;
    return rc;
  }
  p->n_cu = prop.multiProcessorCount;
  p->arch = prop.gcnArchName;
  derive(p);
  tiling_for(p, 256, 1, 16, 0, kAdjBlocks);  // the autotuner's usual pick for every profile measured
  std::memset(&p->w, 0, sizeof(p->w));
  *out = p;
  g_err.clear();
  return XS_OK;
}

int xs_plan_set_conditions(xs_plan* p, int32_t n_cond, const xs_condition* conds) {
  if (!p) return fail(XS_EINVAL, "plan is NULL");
  if (n_cond != (int32_t)p->conds.size()) return fail(XS_EINVAL, "n_cond differs from the plan's");
  int rc;
  if ((rc = validate_conds(&p->model, &p->grid, n_cond, conds))) return rc;
  p->conds.assign(conds, conds + n_cond);
  p->prepared = false;
  const int32_t old_slots = p->md.n_slots, old_cc = p->md.n_cut_classes;
  derive(p);
  if (p->md.n_slots > old_slots || p->md.n_cut_classes > old_cc) {
    // more intensity slots or cut-off classes than the workspace was carved for
    if (p->ws && p->ws_bytes < layout(p, nullptr, nullptr)) {
      p->ws = nullptr;
      return fail(XS_EWORKSPACE, "workspace too small for the new conditions; rebind it");
    }
  }
  if (p->gexec) {
    (void)hipGraphExecDestroy(p->gexec);
    p->gexec = nullptr;
  }
  if (p->graph) {
    (void)hipGraphDestroy(p->graph);
    p->graph = nullptr;
  }
  if (p->ws) {
    layout(p, (char*)p->ws, &p->w);
    return upload(p);
  }
  return XS_OK;
}

void xs_plan_destroy(xs_plan* p) {
  if (!p) return;
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  delete p;
}

int xs_plan_workspace_bytes(const xs_plan* p, size_t* bytes) {
  if (!p || !bytes) return fail(XS_EINVAL, "plan or bytes is NULL");
  *bytes = layout(const_cast<xs_plan*>(p), nullptr, nullptr);
  return XS_OK;
}

int xs_plan_set_workspace(xs_plan* p, void* dptr, size_t bytes) {
  if (!p) return fail(XS_EINVAL, "plan is NULL");
  if (!dptr || ((uintptr_t)dptr & 255)) return fail(XS_EINVAL, "workspace must be non-NULL and 256-byte aligned");
  size_t need = layout(p, nullptr, nullptr);
  if (bytes < need) return fail(XS_EWORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  p->ws = dptr;
  p->ws_bytes = bytes;
  p->prepared = false;
  layout(p, (char*)dptr, &p->w);
  return upload(p);
}

int xs_plan_set_config(xs_plan* p, const xs_config* c) {
  if (!p) return fail(XS_EINVAL, "plan is NULL");
  int rc;
  if ((rc = validate_config(c))) return rc;
  if (c->bucket_bins != p->bucket_bins) {
    p->bucket_bins = c->bucket_bins;
    p->prepared = false;
    derive(p);
    if (p->ws) {  // the bucket table size changed: re-carve and re-upload
      size_t need = layout(p, nullptr, nullptr);
      if (p->ws_bytes < need) {
        p->ws = nullptr;
        return fail(XS_EWORKSPACE, "workspace too small for the new bucket size; rebind it");
      }
      layout(p, (char*)p->ws, &p->w);
      if ((rc = upload(p))) return rc;
    }
  }
  tiling_for(p, c->tile_bins, c->persistent, c->waves_per_cu, c->chunk_lines, c->adj_blocks);
  return XS_OK;
}

int xs_plan_get_config(const xs_plan* p, xs_config* c) {
  if (!p || !c) return fail(XS_EINVAL, "plan or config is NULL");
  c->tile_bins = p->tiling.tile_bins;
  c->bucket_bins = p->bucket_bins;
  c->persistent = p->tiling.persistent;
  c->waves_per_cu = p->tiling.grid_blocks / std::max(1, p->n_cu);
  c->chunk_lines = (int32_t)p->tiling.chunk_lines;
  c->adj_blocks = p->tiling.adj_blocks;
  return XS_OK;
}

int xs_partition_function(xs_plan* p, const xs_states* st, double* Q, double* dQdT) {
  int rc;
  if ((rc = check_call(p, st, nullptr))) return rc;
  if (!Q) return fail(XS_EINVAL, "Q is NULL");
  launch_partition(p->md, p->w, view(st), p->stream);
  launch_q_out(p->md, p->w, Q, dQdT, p->stream);
  return hip_check(hipGetLastError(), "partition launch");
}

int xs_line_intensities(xs_plan* p, const xs_states* st, const xs_lines* ln, void* S,
                        double* log_scale) {
  int rc;
  if ((rc = check_call(p, st, ln))) return rc;
  if (!S && ln->n > 0) return fail(XS_EINVAL, "S is NULL");
  if (p->model.precision == XS_FP32 && !log_scale) return fail(XS_EINVAL, "log_scale is NULL (FP32 form)");
  const StatesView sv = view(st);
  const LinesView lv = view(ln);
  launch_reset(p->w, p->stream);
  launch_partition(p->md, p->w, sv, p->stream);
  launch_lines_pass1(p->md, p->w, sv, lv, p->stream);
  if (ln->n > 0) launch_intensity_out(p->md, p->w, sv, lv, S, log_scale, p->stream);
  return hip_check(hipGetLastError(), "intensity launch");
}

int xs_cross_section(xs_plan* p, const xs_states* st, const xs_lines* ln, double* sigma,
                     int32_t accumulate) {
  int rc;
  if ((rc = check_call(p, st, ln))) return rc;
  if (!sigma) return fail(XS_EINVAL, "sigma is NULL");
  if (accumulate != 0 && accumulate != 1) return fail(XS_EINVAL, "accumulate must be 0 or 1");
  if ((rc = preprocess(p, st, ln))) return rc;
  return profile_pass(p, sigma, accumulate);
}

int xs_prepare(xs_plan* p, const xs_states* st, const xs_lines* ln) {
  int rc;
  if ((rc = check_call(p, st, ln))) return rc;
  return preprocess(p, st, ln);
}

int xs_profile_pass(xs_plan* p, double* sigma, int32_t accumulate) {
  if (!p) return fail(XS_EINVAL, "plan is NULL");
  if (!p->ws) return fail(XS_EWORKSPACE, "no workspace bound (xs_plan_set_workspace)");
  if (!p->prepared) return fail(XS_EINVAL, "xs_profile_pass before xs_prepare");
  if (!sigma) return fail(XS_EINVAL, "sigma is NULL");
  if (accumulate != 0 && accumulate != 1) return fail(XS_EINVAL, "accumulate must be 0 or 1");
  launch_reset_queue(p->w, p->stream);
  return profile_pass(p, sigma, accumulate);
}

int xs_profile_adjoint(xs_plan* p, const xs_states* st, const xs_lines* ln, const double* g,
                       double* dT, double* dP, double* dgref, double* dnexp, double* dls) {
  int rc;
  if ((rc = check_call(p, st, ln))) return rc;
  if (!p->prepared) return fail(XS_EINVAL, "xs_profile_adjoint before xs_prepare");
  if (p->model.population != XS_LTE)
    return fail(XS_EUNSUPPORTED, "adjoint: two-temperature populations are not supported");
  if (p->model.profile >= XS_BIN_DOPPLER)
    return fail(XS_EUNSUPPORTED, "adjoint: binned and pseudo-Voigt profiles are not supported");
  if (!g || !dT || !dP || !dls) return fail(XS_EINVAL, "adjoint: dL_dsigma, dL_dT, dL_dP and dL_dlog_scale are required");
  if (ln->n != p->last_lines_in) return fail(XS_EINVAL, "adjoint: lines differ from the prepared ones");
  launch_adjoint(p->md, kernel_work(p), view(st), view(ln), g, dT, dP, dgref, dnexp, dls, ln->n,
                 p->tiling.adj_blocks, p->stream);
  return hip_check(hipGetLastError(), "adjoint launch");
}

int xs_cross_section_adjoint(xs_plan* p, const xs_states* st, const xs_lines* ln,
                             const double* g, double* dT, double* dP, double* dgref, double* dnexp,
                             double* dls) {
  int rc;
  if ((rc = check_call(p, st, ln))) return rc;
  if (p->model.population != XS_LTE)
    return fail(XS_EUNSUPPORTED, "adjoint: two-temperature populations are not supported");
  if (p->model.profile >= XS_BIN_DOPPLER)
    return fail(XS_EUNSUPPORTED, "adjoint: binned and pseudo-Voigt profiles are not supported");
  if (!g || !dT || !dP || !dls) return fail(XS_EINVAL, "adjoint: dL_dsigma, dL_dT, dL_dP and dL_dlog_scale are required");
  if ((rc = preprocess(p, st, ln))) return rc;
  launch_adjoint(p->md, kernel_work(p), view(st), view(ln), g, dT, dP, dgref, dnexp, dls, ln->n,
                 p->tiling.adj_blocks, p->stream);
  return hip_check(hipGetLastError(), "adjoint launch");
}

int xs_cooling_function(xs_plan* p, const xs_states* st, const xs_lines* ln, int32_t n_T,
                        const double* T, double* W, double* Q) {
  int rc;
  if ((rc = check_call(p, st, ln))) return rc;
  if (p->model.population != XS_LTE)
    return fail(XS_EUNSUPPORTED, "cooling function: LTE populations only (Eq. cf)");
  if (n_T < 1 || n_T > (1 << 20)) return fail(XS_EINVAL, "n_T must be in [1, 2^20]");
  if (!T || !W) return fail(XS_EINVAL, "cooling function: T and W are required");
  for (int32_t j = 0; j < n_T; ++j)
    if (!(T[j] > 0.0 && std::isfinite(T[j]))) return fail(XS_EINVAL, "cooling function: temperatures must be > 0");
  // temperatures and the per-(chunk, temperature) partial sums live in the
  // gather's partial-row buffer
  const int64_t need = ((int64_t)n_T + 31) / 32 * 32 + 2 * (int64_t)cooling_chunks(n_T) * n_T;
  if (need > 2 * p->w.item_target * 1024)
    return fail(XS_EINVAL, "cooling function: n_T too large for this plan's workspace");
  p->cf_T.assign(T, T + n_T);
  if ((rc = hip_check(hipMemcpyAsync(p->w.part, p->cf_T.data(), sizeof(double) * n_T,
                                     hipMemcpyHostToDevice, p->stream), "cooling temperatures")))
    return rc;
  if ((rc = hip_check(hipStreamSynchronize(p->stream), "cooling temperatures sync"))) return rc;
  launch_cooling(p->md, p->w, view(st), view(ln), p->w.part, n_T, W, Q, p->stream);
  p->prepared = false;  // the records area now holds the cooling function's runs
  p->last_lines_in = ln->n;
  return hip_check(hipGetLastError(), "cooling launch");
}

int xs_plan_capture(xs_plan* p, const xs_states* st, const xs_lines* ln, double* sigma,
                    int32_t accumulate) {
  int rc;
  if ((rc = check_call(p, st, ln))) return rc;
  if (!sigma) return fail(XS_EINVAL, "sigma is NULL");
  if (accumulate != 0 && accumulate != 1) return fail(XS_EINVAL, "accumulate must be 0 or 1");
  if (!p->cap_stream &&
      (rc = hip_check(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking), "capture stream")))
    return rc;
  if (p->gexec) {
    (void)hipGraphExecDestroy(p->gexec);
    p->gexec = nullptr;
  }
  if (p->graph) {
    (void)hipGraphDestroy(p->graph);
    p->graph = nullptr;
  }
  // capture on the library stream, replay on the plan's stream
  hipStream_t keep = p->stream;
  p->stream = p->cap_stream;
  if ((rc = hip_check(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture"))) {
    p->stream = keep;
    return rc;
  }
  int rc1 = preprocess(p, st, ln);
  int rc2 = rc1 ? rc1 : profile_pass(p, sigma, accumulate);
  hipGraph_t g = nullptr;
  int rc3 = hip_check(hipStreamEndCapture(p->cap_stream, &g), "end capture");
  p->stream = keep;
  if (rc2 || rc3) {
    if (g) (void)hipGraphDestroy(g);
    return rc2 ? rc2 : rc3;
  }
  p->graph = g;
  return hip_check(hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0), "graph instantiate");
}

int xs_plan_replay(xs_plan* p) {
  if (!p) return fail(XS_EINVAL, "plan is NULL");
  if (!p->gexec) return fail(XS_EINVAL, "no captured graph (xs_plan_capture)");
  return hip_check(hipGraphLaunch(p->gexec, p->stream), "graph launch");
}

int xs_plan_get_stats(xs_plan* p, xs_stats* s) {
  if (!p || !s) return fail(XS_EINVAL, "plan or stats is NULL");
  if (!p->ws) return fail(XS_EWORKSPACE, "no workspace bound");
  unsigned long long h[8] = {0};
  int rc;
  if ((rc = hip_check(hipMemcpyAsync(h, p->w.stats, sizeof(h), hipMemcpyDeviceToHost, p->stream), "stats copy")))
    return rc;
  if ((rc = hip_check(hipStreamSynchronize(p->stream), "stats sync"))) return rc;
  s->lines_in = p->last_lines_in;
  s->lines_kept = (int64_t)h[1];
  s->window_pairs = (int64_t)h[2];
  const int64_t nt = (p->grid.n_bins + p->tiling.tile_bins - 1) / p->tiling.tile_bins;
  s->work_items = nt * (int64_t)p->conds.size();
  s->lines_invalid = (int64_t)h[3];
  return XS_OK;
}

int xs_plan_sync(xs_plan* p) {
  if (!p) return fail(XS_EINVAL, "plan is NULL");
  return hip_check(hipStreamSynchronize(p->stream), "stream sync");
}

// ---- allocation-free cross section ---------------------------------------
// For callers that cannot allocate device memory, xs_cross_section_noalloc
// runs the xs_cross_section path with its workspace carved from this array
// instead of a caller-bound buffer.  Each GPU that runs the library holds its
// own copy until the process ends.  Host code never uses the array's name as
// an address: the device address comes from hipGetSymbolAddress, taken once
// per device with that device current.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kNoallocItemsPerCU = 2;  // partial-row buffer: 2 x 2 rows of 8 KiB per compute unit
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch (dev must be the current device).
int scratch_base(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(XS_EDEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    int rc;
    if ((rc = hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)")))
      return rc;
    if (!ptr || ((uintptr_t)ptr & 255)) return fail(XS_EDEVICE, "scratch address is not 256-byte aligned");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return XS_OK;
}
}  // namespace

int xs_cross_section_noalloc(xs_plan* p, const xs_states* st, const xs_lines* ln,
                             double* sigma, int32_t accumulate) {
  if (!p) return fail(XS_EINVAL, "plan is NULL");
  int rc;
  if ((rc = validate_states(p, st))) return rc;
  if ((rc = validate_lines(p, ln))) return rc;
  if (!sigma) return fail(XS_EINVAL, "sigma is NULL");
  if (accumulate != 0 && accumulate != 1) return fail(XS_EINVAL, "accumulate must be 0 or 1");
  const int64_t items = (int64_t)kNoallocItemsPerCU * std::max(1, p->n_cu);
  const size_t need = layout(p, nullptr, nullptr, items, false);
  if (need > kScratchBytes)
    return fail(XS_EWORKSPACE, "the plan needs " + std::to_string(need) + " bytes of scratch, more than the " +
                                   std::to_string(kScratchBytes) +
                                   " of the allocation-free path (fewer max_lines, grid points or conditions)");
  int dev = -1;
  if ((rc = hip_check(hipGetDevice(&dev), "hipGetDevice"))) return rc;
  if (dev != p->device) return fail(XS_EINVAL, "the plan's GPU is not the current device");
  void* base = nullptr;
  if ((rc = scratch_base(dev, &base))) return rc;
  // run on the scratch; the plan's own workspace and the state of its last
  // xs_prepare are left as they were
  const Work keep_w = p->w;
  void* const keep_ws = p->ws;
  const size_t keep_bytes = p->ws_bytes;
  const bool keep_prepared = p->prepared, keep_tau = p->has_tau;
  const int64_t keep_last = p->last_lines_in;
  layout(p, (char*)base, &p->w, items, false);
  p->ws = base;
  p->ws_bytes = kScratchBytes;
  rc = upload(p);
  if (!rc) rc = preprocess(p, st, ln);
  if (!rc) rc = profile_pass(p, sigma, accumulate);
  p->w = keep_w;
  p->ws = keep_ws;
  p->ws_bytes = keep_bytes;
  p->prepared = keep_prepared;
  p->has_tau = keep_tau;
  p->last_lines_in = keep_last;
  return rc;
}

// ---- autotuner ----------------------------------------------------------
static std::string tune_key(const xs_plan* p, int64_t n_lines) {
  double maxcut = 0.0;
  for (auto& c : p->conds) maxcut = std::max(maxcut, c.cutoff);
  const int64_t wb = (int64_t)std::ceil(maxcut / p->grid.dnu);
  int lb = 0;
  while ((int64_t(1) << (lb + 1)) <= std::max<int64_t>(n_lines, 1)) ++lb;
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s|p%d|f%d|w%lld|n2^%d|c%d", p->arch.c_str(), p->model.profile,
                p->model.precision, (long long)wb, lb, (int)p->conds.size());
  return buf;
}

static bool cache_lookup(const char* path, const std::string& key, xs_config* c) {
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof(line), f)) {
    char k[256];
    int t, b, per, wv, cl, ab;
    if (std::sscanf(line, " {\"key\": \"%255[^\"]\", \"tile_bins\": %d, \"bucket_bins\": %d, \"persistent\": %d, \"waves_per_cu\": %d, \"chunk_lines\": %d, \"adj_blocks\": %d",
                    k, &t, &b, &per, &wv, &cl, &ab) == 7 && key == k) {
      c->tile_bins = t;
      c->bucket_bins = b;
      c->persistent = per;
      c->waves_per_cu = wv;
      c->chunk_lines = cl;
      c->adj_blocks = ab;
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

static void cache_store(const char* path, const std::string& key, const xs_config& c, double ms,
                        double adj_ms) {
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "{\"key\": \"%s\", \"tile_bins\": %d, \"bucket_bins\": %d, \"persistent\": %d, \"waves_per_cu\": %d, \"chunk_lines\": %d, \"adj_blocks\": %d, \"ms\": %.4f, \"adj_ms\": %.4f}\n",
               key.c_str(), c.tile_bins, c.bucket_bins, c.persistent, c.waves_per_cu, c.chunk_lines,
               c.adj_blocks, ms, adj_ms);
  std::fclose(f);
}

int xs_plan_autotune(xs_plan* p, const xs_states* st, const xs_lines* ln, double* sigma,
                     const char* cache_path) {
  int rc;
  if ((rc = check_call(p, st, ln))) return rc;
  if (!sigma) return fail(XS_EINVAL, "sigma is NULL");
  const std::string key = tune_key(p, ln->n);
  xs_config best;
  if (cache_lookup(cache_path, key, &best)) return xs_plan_set_config(p, &best);
  if (p->model.algo != XS_GATHER) return XS_OK;
  if ((rc = preprocess(p, st, ln))) return rc;
  hipEvent_t e0, e1;
  if ((rc = hip_check(hipEventCreate(&e0), "event"))) return rc;
  if ((rc = hip_check(hipEventCreate(&e1), "event"))) {
    (void)hipEventDestroy(e0);
    return rc;
  }
  // best of two timed runs after one untimed
  auto time3 = [&](auto run, float& ms_best) {
    ms_best = 1e30f;
    for (int rep = 0; rep < 3 && !rc; ++rep) {
      (void)hipEventRecord(e0, p->stream);
      rc = run();
      (void)hipEventRecord(e1, p->stream);
      if (!rc) rc = hip_check(hipEventSynchronize(e1), "autotune sync");
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0) ms_best = std::min(ms_best, ms);
    }
  };
  // profile pass: bucket size (the plan's own first) x tile width x launch
  // mode (persistent queue with two grid sizes, or one block per item)
  const int buckets[2] = {p->bucket_bins, p->bucket_bins == 64 ? 256 : 64};
  const int tiles[3] = {256, 512, 1024};
  const int modes[3][2] = {{0, 16}, {1, 16}, {1, 32}};
  double best_ms = 1e300;
  xs_config cur;
  cur.chunk_lines = 0;
  cur.adj_blocks = p->tiling.adj_blocks;
  for (int bi = 0; bi < 2 && !rc; ++bi) {
    if (buckets[bi] != p->bucket_bins) {
      // re-bucket the lines (the workspace holds any bucket size)
      p->bucket_bins = buckets[bi];
      p->prepared = false;
      derive(p);
      layout(p, (char*)p->ws, &p->w);
      if ((rc = upload(p))) break;
      if ((rc = preprocess(p, st, ln))) break;
    }
    cur.bucket_bins = p->bucket_bins;
    for (int si = 0; si < 3 && !rc; ++si) {
      for (int mi = 0; mi < 3 && !rc; ++mi) {
        cur.tile_bins = tiles[si];
        cur.persistent = modes[mi][0];
        cur.waves_per_cu = modes[mi][1];
        tiling_for(p, cur.tile_bins, cur.persistent, cur.waves_per_cu, cur.chunk_lines, cur.adj_blocks);
        float ms_best;
        time3([&]() {
          launch_reset_queue(p->w, p->stream);
          return profile_pass(p, sigma, 0);
        }, ms_best);
        if (!rc && ms_best < best_ms) {
          best_ms = ms_best;
          best = cur;
        }
      }
    }
  }
  // adjoint grid size (LTE, sampled profiles): the records of the chosen
  // bucket size, the last profile pass's sigma as the cotangent, and outputs
  // in scratch the adjoint does not read (the line pack and partial rows)
  double adj_ms = 0.0;
  if (!rc && p->model.population == XS_LTE && p->model.profile < XS_BIN_DOPPLER) {
    if ((rc = xs_plan_set_config(p, &best)) == XS_OK && !p->prepared) rc = preprocess(p, st, ln);
    const int cand[4] = {4096, 8192, 16384, 32768};
    double* outs = (double*)p->w.lpack;  // 64 B per line: room for three gradients
    double* dTP = p->w.part;             // dL/dT, dL/dP
    float adj_best = 1e30f;
    for (int ci = 0; ci < 4 && !rc; ++ci) {
      float ms_best;
      time3([&]() {
        launch_adjoint(p->md, kernel_work(p), view(st), view(ln), sigma, dTP, dTP + p->conds.size(), outs,
                       outs + ln->n, outs + 2 * ln->n, ln->n, cand[ci], p->stream);
        return hip_check(hipGetLastError(), "adjoint launch");
      }, ms_best);
      if (!rc && ms_best < adj_best) {
        adj_best = ms_best;
        best.adj_blocks = cand[ci];
      }
    }
    adj_ms = adj_best;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  // the best bucket size (re-bucketed on the next prepare when it is not
  // the last one tried) and tiling
  if ((rc = xs_plan_set_config(p, &best))) return rc;
  cache_store(cache_path, key, best, best_ms, adj_ms);
  return XS_OK;
}

}  // extern "C"
