// Line-side kernels: partition functions, the intensity pass, bucketing of
// lines by home bin (stable LSD radix sort) and the sorted line records.
#include <algorithm>

#include "k_common.h"

namespace xs {

// ---------------------------------------------------------------------------
// Partition functions, Eq. (pf): Q(T) = sum_n g_n exp(-c2 E_n / T) and
// dQ/dT = sum_n g_n (c2 E_n / T^2) exp(-c2 E_n / T); two temperatures,
// Eq. (Q nlte 2T), with E_rot = E - E_vib(v).  FP64, deterministic two-stage
// tree reduction (per-block partials, then one block per slot).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum256(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void k_partition(ModelDev m, const SlotDev* slots,
                                                   StatesView st, double* qpart) {
  __shared__ double sh[256];
  const int slot = blockIdx.y;
  const SlotDev sd = slots[slot];
  double q = 0.0, dq = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < st.n; i += (int64_t)gridDim.x * 256) {
    const double E = st.E[i];
    if (m.pop == XS_LTE) {
      const double b = st.g[i] * exp(-kC2 * E / sd.T);
      q += b;
      dq += b * (kC2 * E / (sd.T * sd.T));
    } else {
      const int32_t vi = st.v[i];
      if ((uint32_t)vi < (uint32_t)st.n_v) {  // states with an invalid manifold index are skipped
        const double ev = st.ev[vi];
        if (m.pop == XS_NLTE_2T) {
          q += st.g[i] * exp(-kC2 * ev / sd.Tv - kC2 * (E - ev) / sd.Tr);
        } else {  // custom vibronic densities, Eq. (Q nlte Nvib)
          const double w = st.nv[vi];
          if (w > 0.0) q += st.g[i] * w * exp(-kC2 * (E - ev) / sd.Tr);
        }
      }
    }
  }
  q = block_sum256(q, sh);
  dq = block_sum256(dq, sh);
  if (threadIdx.x == 0) {
    qpart[(slot * 2 + 0) * kQBlocks + blockIdx.x] = q;
    qpart[(slot * 2 + 1) * kQBlocks + blockIdx.x] = dq;
  }
}

__global__ __launch_bounds__(256) void k_partition_final(ModelDev m, const double* qpart,
                                                         double* Q, double* dQ,
                                                         unsigned long long* smax) {
  __shared__ double sh[256];
  const int slot = blockIdx.x;
  double q = block_sum256(qpart[(slot * 2 + 0) * kQBlocks + threadIdx.x], sh);
  double dq = block_sum256(qpart[(slot * 2 + 1) * kQBlocks + threadIdx.x], sh);
  if (threadIdx.x == 0) {
    Q[slot] = q;
    dQ[slot] = (m.pop == XS_LTE) ? dq : __longlong_as_double(0x7ff8000000000000ll);
    smax[slot] = 0ull;  // reset the running max of ln|S| for the intensity pass
  }
}

void launch_partition(const ModelDev& m, const Work& w, const StatesView& st, hipStream_t s) {
  hipLaunchKernelGGL(k_partition, dim3(kQBlocks, m.n_slots), dim3(256), 0, s, m, w.slot, st,
                     w.qpart);
  hipLaunchKernelGGL(k_partition_final, dim3(m.n_slots), dim3(256), 0, s, m, w.qpart, w.Q, w.dQ,
                     w.smax);
}

__global__ void k_q_out(ModelDev m, const CondDev* cond, const double* Q, const double* dQ,
                        double* Qo, double* dQo) {
  const int c = threadIdx.x;
  if (c < m.n_cond) {
    Qo[c] = Q[cond[c].slot];
    if (dQo) dQo[c] = dQ[cond[c].slot];
  }
}

void launch_q_out(const ModelDev& m, const Work& w, double* Q, double* dQ, hipStream_t s) {
  hipLaunchKernelGGL(k_q_out, dim3(1), dim3(256), 0, s, m, w.cond, w.Q, w.dQ, Q, dQ);
}

// ---------------------------------------------------------------------------
// Intensity pass 1: nu_i = E_u - E_l; keep lines with nu > 0 whose window
// (widest cut-off) reaches the grid; key = k_c / kFineBins for the home bin
// k_c = rint((nu - nu0)/dnu), clamped to the grid (lines past either end
// keep their wings, section "Spectral synthesis"); dropped lines get key
// n_fine.  FP32 form: running max of ln|S| per slot.  Counters:
// kept lines and window pairs (exact windows per distinct cut-off).
// ---------------------------------------------------------------------------
__device__ __forceinline__ LineState line_state(const StatesView& st, int32_t u, int32_t l,
                                                int pop) {
  LineState s;
  s.Eu = st.E[u];
  s.El = st.E[l];
  s.gu = st.g[u];
  if (pop != XS_LTE) {
    s.evu = st.ev[st.v[u]];
    s.evl = st.ev[st.v[l]];
  } else {
    s.evu = s.evl = 0.0;
  }
  if (pop == XS_NLTE_DENSITY) {
    s.nvu = st.nv[st.v[u]];
    s.nvl = st.nv[st.v[l]];
  } else {
    s.nvu = s.nvl = 1.0;
  }
  return s;
}

// As line_state, with the energies, degeneracy and manifold energies from
// the line's pack (the state tables are read only for the custom densities).
__device__ __forceinline__ LineState line_state(const StatesView& st, const LinePack& lp, int pop) {
  LineState s;
  s.Eu = lp.Eu;
  s.El = lp.El;
  s.gu = lp.gu;
  s.evu = lp.evu;
  s.evl = lp.evl;
  if (pop == XS_NLTE_DENSITY) {
    s.nvu = st.nv[st.v[lp.u]];
    s.nvl = st.nv[st.v[lp.l]];
  } else {
    s.nvu = s.nvl = 1.0;
  }
  return s;
}

// Per-state record for the first line pass: one random load per state of a
// line instead of one per table (energies, degeneracies, manifold index and
// energy).  Built once per prepare into the sort's second ping-pong buffers,
// which are free until the sort's last pass; lists with more states than that
// space holds read the tables directly.
struct __attribute__((aligned(16))) StatePackLTE {
  double E, g;
};
struct __attribute__((aligned(32))) StatePackNLTE {
  double E, g, ev;  // ev: E_vib of the state's manifold
  int64_t vi;       // manifold index, or -1 when outside the table
};

__global__ __launch_bounds__(256) void k_state_pack(ModelDev m, StatesView st, void* pack) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < st.n; i += (int64_t)gridDim.x * 256) {
    if (m.pop == XS_LTE) {
      StatePackLTE r;
      r.E = st.E[i];
      r.g = st.g[i];
      ((StatePackLTE*)pack)[i] = r;
    } else {
      StatePackNLTE r;
      r.E = st.E[i];
      r.g = st.g[i];
      const int32_t vi = st.v[i];
      const bool ok = (uint32_t)vi < (uint32_t)st.n_v;
      r.ev = ok ? st.ev[vi] : 0.0;
      r.vi = ok ? (int64_t)vi : -1;
      ((StatePackNLTE*)pack)[i] = r;
    }
  }
}

// The states of one line, read once: from the packed table, or from the
// caller's tables.  ok: both indices (and, non-LTE, both manifolds) inside
// the tables.
template <int MODE>
__device__ __forceinline__ bool gather_line_states(const ModelDev& m, const StatesView& st, const void* pack,
                                                   int32_t u, int32_t l, LineState& ls, int32_t& vu, int32_t& vl) {
  if ((uint32_t)u >= (uint64_t)st.n || (uint32_t)l >= (uint64_t)st.n) return false;
  if (m.pop == XS_LTE) {
    if (MODE) {
      const StatePackLTE a = ((const StatePackLTE*)pack)[u], b = ((const StatePackLTE*)pack)[l];
      ls.Eu = a.E;
      ls.gu = a.g;
      ls.El = b.E;
    } else {
      ls.Eu = st.E[u];
      ls.gu = st.g[u];
      ls.El = st.E[l];
    }
    ls.evu = ls.evl = 0.0;
    vu = vl = 0;
  } else {
    if (MODE) {
      const StatePackNLTE a = ((const StatePackNLTE*)pack)[u], b = ((const StatePackNLTE*)pack)[l];
      if (a.vi < 0 || b.vi < 0) return false;
      ls.Eu = a.E;
      ls.gu = a.g;
      ls.evu = a.ev;
      ls.El = b.E;
      ls.evl = b.ev;
      vu = (int32_t)a.vi;
      vl = (int32_t)b.vi;
    } else {
      vu = st.v[u];
      vl = st.v[l];
      if ((uint32_t)vu >= (uint32_t)st.n_v || (uint32_t)vl >= (uint32_t)st.n_v) return false;
      ls.Eu = st.E[u];
      ls.gu = st.g[u];
      ls.El = st.E[l];
      ls.evu = st.ev[vu];
      ls.evl = st.ev[vl];
    }
  }
  if (m.pop == XS_NLTE_DENSITY) {
    ls.nvu = st.nv[vu];
    ls.nvl = st.nv[vl];
  } else {
    ls.nvu = ls.nvl = 1.0;
  }
  return true;
}

// MODE 1: states from the packed table; 0: from the caller's tables.  The
// running maximum of ln|S| of each slot (FP32 form) is kept per thread in LDS
// rather than in registers, so the pass holds few registers and many waves
// keep its random state loads in flight.
constexpr int kPass1Slots = 8;  // slots whose maximum is kept per thread; more use atomics
template <int MODE>
__global__ __launch_bounds__(256) void k_lines_pass1(ModelDev m, const SlotDev* slots,
                                                     const double* Q, const double* cutc,
                                                     const int32_t* cutm, StatesView st, const void* spack,
                                                     LinesView ln, int32_t* key,
                                                     LinePack* lpack,
                                                     unsigned long long* smax,
                                                     unsigned long long* stats) {
  __shared__ double lmax[kPass1Slots][256];
  __shared__ double lnq[kPass1Slots];
  __shared__ unsigned long long scnt[3];
  const int tid = threadIdx.x;
  const bool f32 = m.prec == XS_FP32;
  const int ns = min(m.n_slots, kPass1Slots);
  if (tid < 3) scnt[tid] = 0;
  if (tid < ns && f32) lnq[tid] = log(Q[tid]);
  for (int q = 0; q < ns; ++q) lmax[q][tid] = -INFINITY;
  __syncthreads();
  unsigned long long kept = 0, pairs = 0, bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + tid; i < ln.n; i += (int64_t)gridDim.x * 256) {
    const int32_t u = ln.up[i], l = ln.lo[i];
    int32_t kk = m.n_fine;
    LineState ls;
    int32_t vu, vl;
    if (!gather_line_states<MODE>(m, st, spack, u, l, ls, vu, vl)) {
      ++bad;
      key[i] = kk;
      continue;
    }
    const double nu = ls.Eu - ls.El;
    int64_t a, b;
    if (nu > 0.0 && line_window(nu, m.max_cut, m.nu0, m.dnu, m.n_bins, a, b)) {
      int64_t kc = home_bin(nu, m.nu0, m.dnu);
      int64_t fk = kc < 0 ? 0 : kc / kFineBins;
      kk = (int32_t)(fk < m.n_fine - 1 ? fk : m.n_fine - 1);
      ++kept;
      LinePack lp;
      lp.Eu = ls.Eu;
      lp.El = ls.El;
      lp.gu = ls.gu;
      lp.u = u;
      lp.l = l;
      const float Af = ln.A[i];
      const float lsf = ln.lscale ? ln.lscale[i] : 0.0f;
      lp.A = Af;
      lp.gref = ln.gref ? ln.gref[i] : (float)ln.gref_scalar;
      lp.nexp = ln.nexp ? ln.nexp[i] : (float)ln.nexp_scalar;
      lp.lscale = lsf;
      lp.evu = ls.evu;
      lp.evl = ls.evl;
      lpack[i] = lp;
      if (m.n_cut_classes == 1 && cutc[0] == m.max_cut) {
        pairs += (unsigned long long)(b - a + 1) * (unsigned long long)cutm[0];
      } else {
#pragma unroll 1
        for (int q = 0; q < m.n_cut_classes; ++q) {
          if (line_window(nu, cutc[q], m.nu0, m.dnu, m.n_bins, a, b))
            pairs += (unsigned long long)(b - a + 1) * (unsigned long long)cutm[q];
        }
      }
      if (f32) {
        const double sc = (double)lsf;
        const double base = ln_line(m.mode, ls, (double)Af, nu);
#pragma unroll 1
        for (int q = 0; q < m.n_slots; ++q) {
          const SlotDev sd = slots[q];
          int sg;
          const double lS = base + ln_pop(m.mode, m.pop, ls, nu, sd.T, sd.Tv, sd.Tr, sg) + sc;
          if (q < kPass1Slots) {
            lmax[q][tid] = fmax(lmax[q][tid], lS - lnq[q]);
          } else if (lS - log(Q[q]) > -INFINITY) {  // rare: more than kPass1Slots temperatures
            atomicMax(smax + q, dbl_key(lS - log(Q[q])));
          }
        }
      }
    }
    key[i] = kk;
  }
  atomicAdd(&scnt[0], kept);
  atomicAdd(&scnt[1], pairs);
  atomicAdd(&scnt[2], bad);
  if (f32) {
    for (int q = 0; q < ns; ++q) {
      __syncthreads();
      for (int s2 = 128; s2 > 0; s2 >>= 1) {
        if (tid < s2) lmax[q][tid] = fmax(lmax[q][tid], lmax[q][tid + s2]);
        __syncthreads();
      }
      if (tid == 0 && lmax[q][0] > -INFINITY) atomicMax(smax + q, dbl_key(lmax[q][0]));
    }
  }
  __syncthreads();
  if (tid == 0) {
    atomicAdd(stats + 1, scnt[0]);
    atomicAdd(stats + 2, scnt[1]);
    atomicAdd(stats + 3, scnt[2]);
  }
}

__global__ void k_scale_final(ModelDev m, const unsigned long long* smax, double* sb) {
  const int q = threadIdx.x;
  if (q < m.n_slots) sb[q] = smax[q] ? key_dbl(smax[q]) : 0.0;
}

void launch_lines_pass1(const ModelDev& m, const Work& w, const StatesView& st,
                        const LinesView& ln, hipStream_t s) {
  int64_t blocks = (ln.n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  // the packed state table goes into the sort's second ping-pong buffers
  // (keyB, valB: adjacent), when it fits there
  const size_t rec = (m.pop == XS_LTE) ? sizeof(StatePackLTE) : sizeof(StatePackNLTE);
  const size_t room = (size_t)((const char*)w.valB - (const char*)w.keyB) + 4 * (size_t)w.max_lines;
  const bool packed = (size_t)st.n * rec <= room && ((uintptr_t)w.keyB % 32) == 0;
  if (packed) {
    const int64_t sb = std::min<int64_t>((st.n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_state_pack, dim3((unsigned)sb), dim3(256), 0, s, m, st, (void*)w.keyB);
    hipLaunchKernelGGL(k_lines_pass1<1>, dim3((unsigned)blocks), dim3(256), 0, s, m, w.slot, w.Q,
                       w.cut_class, w.cut_mult, st, (const void*)w.keyB, ln, w.key, w.lpack, w.smax, w.stats);
  } else {
    hipLaunchKernelGGL(k_lines_pass1<0>, dim3((unsigned)blocks), dim3(256), 0, s, m, w.slot, w.Q,
                       w.cut_class, w.cut_mult, st, (const void*)nullptr, ln, w.key, w.lpack, w.smax,
                       w.stats);
  }
  hipLaunchKernelGGL(k_scale_final, dim3(1), dim3(256), 0, s, m, w.smax, w.sb);
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of the bucket keys, 8 bits per pass.  Each block owns
// kSortBlock consecutive keys.  Pass: (1) per-block digit histogram;
// (2) exclusive scan of the digit-major [256][blocks] table; (3) stable
// scatter: the rank of a key among equal digits of its block is the running
// count from earlier steps + the counts of earlier waves in this step + the
// number of earlier lanes of its wave with the same digit (8 ballots).
// Stability makes the sorted order, and so every later summation order,
// deterministic.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sort_hist(const int32_t* keys, int64_t n, int shift,
                                                   int32_t* hist, int nblk) {
  __shared__ int h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortBlock;
  for (int s = 0; s < kSortItems; ++s) {
    const int64_t i = base + s * 256 + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255], 1);
  }
  __syncthreads();
  hist[threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of int32 arrays: per-block scan of 1024 elements, block sums
// scanned by one block, then added back.
__device__ __forceinline__ int block_excl_scan256(int v, int* sh, int& total) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    int t = tid >= o ? sh[tid - o] : 0;
    __syncthreads();
    sh[tid] += t;
    __syncthreads();
  }
  int incl = sh[tid];
  total = sh[255];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(256) void k_scan_blocks(int32_t* a, int64_t n, int32_t* sums) {
  __shared__ int sh[256];
  const int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x * 4;
  int v[4], s = 0;
  for (int j = 0; j < 4; ++j) {
    v[j] = (base + j < n) ? a[base + j] : 0;
    s += v[j];
  }
  int total;
  int ex = block_excl_scan256(s, sh, total);
  for (int j = 0; j < 4; ++j) {
    if (base + j < n) a[base + j] = ex;
    ex += v[j];
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void k_scan_sums(int32_t* sums, int64_t n) {
  __shared__ int sh[256];
  int carry = 0;
  for (int64_t b0 = 0; b0 < n; b0 += 256) {
    const int64_t i = b0 + threadIdx.x;
    int v = i < n ? sums[i] : 0;
    int total;
    int ex = block_excl_scan256(v, sh, total);
    if (i < n) sums[i] = ex + carry;
    carry += total;
  }
}

__global__ __launch_bounds__(256) void k_scan_add(int32_t* a, int64_t n, const int32_t* sums) {
  const int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x * 4;
  const int add = sums[blockIdx.x];
  for (int j = 0; j < 4; ++j)
    if (base + j < n) a[base + j] += add;
}

// Stable scatter of one pass, staged through LDS: the block places its keys
// in digit order in LDS (the rank of a key among equal digits of its block is
// the running count from earlier steps + the counts of earlier waves in this
// step + the number of earlier lanes of its wave with the same digit, from 8
// ballots), then writes each digit's run to its global place, so neighbouring
// threads write neighbouring addresses.  offs: the exclusive scan of the
// digit-major [256][nblk] histogram; the block's count of digit d is the step
// from its entry to the next one (n after the last).
__global__ __launch_bounds__(256) void k_sort_scatter(const int32_t* keys, const int32_t* vals,
                                                      int64_t n, int shift, const int32_t* offs,
                                                      int nblk, int32_t* okeys, int32_t* ovals) {
  __shared__ int lstart[256];   // first LDS position of each digit
  __shared__ int goff[256];     // global position of the block's first key of each digit
  __shared__ int run[256];      // keys of each digit placed so far
  __shared__ int wc[4][256];
  __shared__ int sk[kSortBlock], sv[kSortBlock];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t base = (int64_t)blockIdx.x * kSortBlock;
  {
    const int64_t e = (int64_t)tid * nblk + blockIdx.x;
    const int64_t next = (e + 1 < (int64_t)256 * nblk) ? (int64_t)offs[e + 1] : n;
    const int c = (int)(next - offs[e]);
    goff[tid] = offs[e];
    // exclusive scan of the block's digit counts (Hillis-Steele in LDS)
    lstart[tid] = c;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
      const int t = tid >= o ? lstart[tid - o] : 0;
      __syncthreads();
      lstart[tid] += t;
      __syncthreads();
    }
    lstart[tid] -= c;
    run[tid] = 0;
    wc[0][tid] = wc[1][tid] = wc[2][tid] = wc[3][tid] = 0;
    __syncthreads();
  }
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int st = 0; st < kSortItems; ++st) {
    const int64_t i = base + st * 256 + tid;
    const bool act = i < n;
    const int k = act ? keys[i] : 0;
    const int d = (k >> shift) & 255;
    unsigned long long same = __ballot(act);
#pragma unroll
    for (int bt = 0; bt < 8; ++bt) {
      const unsigned long long bb = __ballot(act && ((d >> bt) & 1));
      same &= ((d >> bt) & 1) ? bb : ~bb;
    }
    const int rank = __popcll(same & lt);
    if (act && rank == 0) wc[wave][d] = __popcll(same);
    __syncthreads();
    if (act) {
      int pos = lstart[d] + run[d] + rank;
      for (int w2 = 0; w2 < wave; ++w2) pos += wc[w2][d];
      sk[pos] = k;
      sv[pos] = vals ? vals[i] : (int32_t)i;
    }
    __syncthreads();
    run[tid] += wc[0][tid] + wc[1][tid] + wc[2][tid] + wc[3][tid];
    wc[0][tid] = wc[1][tid] = wc[2][tid] = wc[3][tid] = 0;
    __syncthreads();
  }
  const int cnt = (int)min<int64_t>(kSortBlock, n - base);
  for (int p = tid; p < cnt; p += 256) {
    const int k = sk[p];
    const int d = (k >> shift) & 255;
    const int64_t g = (int64_t)goff[d] + (p - lstart[d]);
    okeys[g] = k;
    ovals[g] = sv[p];
  }
}

static void scan_excl(int32_t* a, int64_t n, int32_t* sums, hipStream_t s) {
  const int64_t nb = (n + 1023) / 1024;
  hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(256), 0, s, a, n, sums);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, s, sums, nb);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(256), 0, s, a, n, sums);
}

void launch_radix_sort(const ModelDev& m, const Work& w, int64_t n, int64_t max_key, hipStream_t s,
                       int32_t** sorted_keys, int32_t** sorted_vals) {
  (void)m;
  int bits = 1;
  while ((1ll << bits) <= (long long)max_key) ++bits;
  const int passes = (bits + 7) / 8;
  const int nblk = (int)((n + kSortBlock - 1) / kSortBlock);
  const int32_t* ik = w.key;
  const int32_t* iv = nullptr;
  int32_t* ok = w.keyA;
  int32_t* ov = w.valA;
  for (int p = 0; p < passes; ++p) {
    if (nblk > 0) {
      hipLaunchKernelGGL(k_sort_hist, dim3(nblk), dim3(256), 0, s, ik, n, 8 * p, w.hist, nblk);
      scan_excl(w.hist, (int64_t)256 * nblk, w.hsum, s);
      hipLaunchKernelGGL(k_sort_scatter, dim3(nblk), dim3(256), 0, s, ik, iv, n, 8 * p, w.hist,
                         nblk, ok, ov);
    }
    ik = ok;
    iv = ov;
    ok = (ok == w.keyA) ? w.keyB : w.keyA;
    ov = (ov == w.valA) ? w.valB : w.valA;
  }
  *sorted_keys = const_cast<int32_t*>(ik);
  *sorted_vals = const_cast<int32_t*>(iv);
}

// ---------------------------------------------------------------------------
// Bucket offsets from the sorted fine keys (bucket = key / fine_per_bucket,
// the dropped key n_fine is bucket n_buckets, and position n acts as bucket
// n_buckets + 1, so every bucket 0..n_buckets gets its start;
// off[n_buckets] = kept lines),
// and the sorted line records: nu, gamma_ref, n_exp, original index, and the
// intensity of every slot, S (FP64) or S~ = sign exp(ln|S| - s_b) (FP32).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_offsets(const int32_t* skeys, int64_t n, int nbk, int nfine, int fpb,
                                                 int32_t* off) {
  auto bucket = [&](int fk) { return fk >= nfine ? nbk : fk / fpb; };
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p <= n;
       p += (int64_t)gridDim.x * 256) {
    const int k = (p < n) ? bucket(skeys[p]) : nbk + 1;
    const int kp = (p > 0) ? bucket(skeys[p - 1]) : -1;
    for (int b = kp + 1; b <= k && b <= nbk; ++b) off[b] = (int32_t)p;
  }
}

__global__ __launch_bounds__(256) void k_records(ModelDev m, const SlotDev* slots, const double* Q,
                                                 const double* sb, StatesView st,
                                                 const LinePack* lpack,
                                                 const int32_t* svals, const int32_t* off,
                                                 int64_t max_lines, double* rnu, float* rgref,
                                                 float* rnexp, double* rgpre, int32_t* ridx, double* rEs,
                                                 void* rS,
                                                 const double* cut_class, int32_t* rkc, float* rdel,
                                                 int32_t* rwin) {
  __shared__ double lnQ[kMaxCond];  // ln Q of every slot, once per block
  for (int q = threadIdx.x; q < m.n_slots; q += 256) lnQ[q] = log(Q[q]);
  __syncthreads();
  const int64_t nk = off[m.n_buckets];
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < nk;
       p += (int64_t)gridDim.x * 256) {
    const int32_t i = svals[p];
    const LinePack lp = lpack[i];
    const int32_t u = lp.u, l = lp.l;
    const double nu = lp.Eu - lp.El;
    rnu[p] = nu;
    rgref[p] = lp.gref;
    rnexp[p] = lp.nexp;
    if (rgpre) {
      // natural width of a predissociating upper state: HWHM 1/(4 pi c tau)
      const double tau = st.tau[u];
      rgpre[p] = (tau > 0.0 && tau < INFINITY) ? 1.0 / (4.0 * kPI * kC * tau) : 0.0;
    }
    ridx[p] = i;
    rEs[p] = (m.mode == XS_ABSORPTION) ? lp.El : lp.Eu;
    // home bin, offset from it, and the exact window of every cut-off class
    const int64_t kc = home_bin(nu, m.nu0, m.dnu);
    rkc[p] = (int32_t)kc;
    rdel[p] = (float)(nu - nu_of_bin(m.nu0, m.dnu, kc));
    for (int q = 0; q < m.n_cut_classes; ++q) {
      int64_t klo, khi;
      if (!line_window(nu, cut_class[q], m.nu0, m.dnu, m.n_bins, klo, khi)) {
        klo = 1;
        khi = 0;
      }
      rwin[((int64_t)q * max_lines + p) * 2] = (int32_t)klo;
      rwin[((int64_t)q * max_lines + p) * 2 + 1] = (int32_t)khi;
    }
    const LineState ls = line_state(st, lp, m.pop);
    const double A = (double)lp.A;
    const double sc = (double)lp.lscale;
    const double base = ln_line(m.mode, ls, A, nu);
    for (int q = 0; q < m.n_slots; ++q) {
      const SlotDev sd = slots[q];
      int sg;
      const double lS = (base + ln_pop(m.mode, m.pop, ls, nu, sd.T, sd.Tv, sd.Tr, sg)) - lnQ[q] + sc;
      if (m.prec == XS_FP32)
        ((float*)rS)[(int64_t)q * max_lines + p] = (float)(sg * exp(lS - sb[q]));
      else
        ((double*)rS)[(int64_t)q * max_lines + p] = sg * exp(lS);
    }
  }
}

void launch_offsets_records(const ModelDev& m, const Work& w, const StatesView& st,
                            const LinesView& ln, const int32_t* skeys, const int32_t* svals,
                            int64_t n, hipStream_t s) {
  int64_t blocks = (n + 256) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_offsets, dim3((unsigned)blocks), dim3(256), 0, s, skeys, n, m.n_buckets, m.n_fine,
                     m.fine_per_bucket, w.off);
  hipLaunchKernelGGL(k_records, dim3((unsigned)blocks), dim3(256), 0, s, m, w.slot, w.Q, w.sb, st,
                     w.lpack, svals, w.off, w.max_lines, w.rnu, w.rgref, w.rnexp, w.rgpre, w.ridx, w.rEs, w.rS,
                     w.cut_class, w.rkc, w.rdel, w.rwin);
}

// ---------------------------------------------------------------------------
// Stick spectrum output: S of every line for every condition, original order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_intensity_out(ModelDev m, const CondDev* cond,
                                                       const SlotDev* slots, const double* Q,
                                                       const double* sb, StatesView st,
                                                       LinesView ln, void* S, double* lsc) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < ln.n;
       i += (int64_t)gridDim.x * 256) {
    const int32_t u = ln.up[i], l = ln.lo[i];
    const bool ok = line_indices_ok(st, u, l, m.pop);
    const double nu = ok ? st.E[u] - st.E[l] : 0.0;
    const LineState ls = ok ? line_state(st, u, l, m.pop) : LineState{0, 0, 0, 0, 0};
    const double A = (double)ln.A[i];
    const double sc = ln.lscale ? (double)ln.lscale[i] : 0.0;
    for (int c = 0; c < m.n_cond; ++c) {
      const int q = cond[c].slot;
      const SlotDev sd = slots[q];
      double v = 0.0;
      if (nu > 0.0) {
        int sg;
        const double lS = ln_intensity(m.mode, m.pop, ls, A, nu, sd.T, sd.Tv, sd.Tr, log(Q[q]), sc, sg);
        v = (m.prec == XS_FP32) ? sg * exp(lS - sb[q]) : sg * exp(lS);
      }
      if (m.prec == XS_FP32)
        ((float*)S)[(int64_t)c * ln.n + i] = (float)v;
      else
        ((double*)S)[(int64_t)c * ln.n + i] = v;
    }
  }
  if (lsc && blockIdx.x == 0 && threadIdx.x < m.n_cond) lsc[threadIdx.x] = sb[cond[threadIdx.x].slot];
}

void launch_intensity_out(const ModelDev& m, const Work& w, const StatesView& st,
                          const LinesView& ln, void* S, double* log_scale, hipStream_t s) {
  int64_t blocks = (ln.n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_intensity_out, dim3((unsigned)blocks), dim3(256), 0, s, m, w.cond, w.slot,
                     w.Q, w.sb, st, ln, S, log_scale);
}

// Clear the per-call counters and the work queue (a kernel, not a memset, so
// the step can be captured in a graph).
__global__ void k_reset(int32_t* counter, unsigned long long* stats) {
  const int t = threadIdx.x;
  for (int q = t; q < kCounterInts; q += 64) counter[q] = 0;
  if (t < 8) stats[t] = 0ull;
}

void launch_reset(const Work& w, hipStream_t s) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, w.counter, w.stats);
}

// Only the work queue (the counters of xs_prepare are kept).
__global__ void k_reset_queue(int32_t* counter) {
  for (int q = threadIdx.x; q < kCounterInts; q += 64) counter[q] = 0;
}

void launch_scan_i32(int32_t* a, int64_t n, int32_t* sums, hipStream_t s) { scan_excl(a, n, sums, s); }

void launch_reset_queue(const Work& w, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, s, w.counter);
}

}  // namespace xs
