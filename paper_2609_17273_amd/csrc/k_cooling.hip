// Cooling function, Eq. (cf):
//   W(T) = h c / (4 pi Q(T)) sum_u g_u exp(-c2 E_u / T) sum_{lines from u} A nu,
// with Q(T) of Eq. (pf).  The lines are grouped by upper state first (stable
// radix sort of the upper index, then one ordered sum of A nu per run of equal
// keys), so the temperature loop runs over the upper states that have lines,
// not over the lines.  Q and W are then the same reduction
//   sum_i w_i exp(-c2 E_i / T)
// over two lists (every state with w = g; every run with w = g_u sum A nu),
// evaluated per (chunk of items, temperature) and added in chunk order, so the
// result does not depend on scheduling.
#include "k_common.h"

namespace xs {

// Key of every line: its upper state if the line counts (valid indices,
// nu > 0), else n_states (sorts after every state).  Counters: kept lines
// (stats[1]) and lines with an index outside the states (stats[3]).
__global__ __launch_bounds__(256) void k_cf_keys(StatesView st, LinesView ln, int32_t* key,
                                                 unsigned long long* stats) {
  unsigned long long kept = 0, bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < ln.n; i += (int64_t)gridDim.x * 256) {
    const int32_t u = ln.up[i], l = ln.lo[i];
    int32_t k = (int32_t)st.n;
    if ((uint32_t)u < (uint64_t)st.n && (uint32_t)l < (uint64_t)st.n) {
      if (st.E[u] - st.E[l] > 0.0) {
        k = u;
        ++kept;
      }
    } else {
      ++bad;
    }
    key[i] = k;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    kept += __shfl_xor(kept, o, 64);
    bad += __shfl_xor(bad, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    if (kept) atomicAdd(stats + 1, kept);
    if (bad) atomicAdd(stats + 3, bad);
  }
}

__device__ __forceinline__ bool run_start(const int32_t* sk, int64_t p, int32_t nst) {
  return sk[p] < nst && (p == 0 || sk[p] != sk[p - 1]);
}

// 1 at the first sorted position of every upper state (scanned afterwards
// into run numbers).
__global__ __launch_bounds__(256) void k_cf_flags(const int32_t* sk, int64_t n, int32_t nst, int32_t* flag) {
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256)
    flag[p] = run_start(sk, p, nst) ? 1 : 0;
}

// One run per upper state: E_u and g_u sum A nu, the sum in sorted order (the
// lines' original order, the sort being stable).  n_runs goes to *nruns.
__global__ __launch_bounds__(256) void k_cf_runs(const int32_t* sk, const int32_t* sv, const int32_t* rank,
                                                 int64_t n, StatesView st, LinesView ln, double* runE,
                                                 double* runW, int32_t* nruns) {
  const int32_t nst = (int32_t)st.n;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256) {
    if (p == n - 1) *nruns = rank[p] + (run_start(sk, p, nst) ? 1 : 0);
    if (!run_start(sk, p, nst)) continue;
    const int32_t u = sk[p];
    const double Eu = st.E[u];
    double s = 0.0;
    for (int64_t q = p; q < n && sk[q] == u; ++q) {
      const int32_t i = sv[q];
      s += (double)ln.A[i] * (Eu - st.E[ln.lo[i]]);
    }
    runE[rank[p]] = Eu;
    runW[rank[p]] = st.g[u] * s;
  }
}

// part[c][j] = sum over chunk c of the items of w_i exp(-c2 E_i / T_j).  One
// thread per temperature; the block stages 256 items at a time in LDS
// (-c2 E_i and w_i, read by every lane at the same address).
__global__ __launch_bounds__(256) void k_cf_sum(const double* E, const double* wgt, int64_t n_static,
                                                const int32_t* n_dyn, const double* T, int32_t nT,
                                                double* part) {
  __shared__ double sE[256], sW[256];
  const int64_t n = n_dyn ? (int64_t)*n_dyn : n_static;
  const int chunks = gridDim.x, c = blockIdx.x;
  const int64_t per = (n + chunks - 1) / chunks;
  const int64_t i0 = min<int64_t>(n, (int64_t)c * per), i1 = min<int64_t>(n, i0 + per);
  const int j = blockIdx.y * 256 + threadIdx.x;
  const double invT = j < nT ? 1.0 / T[j] : 0.0;
  double acc = 0.0;
  for (int64_t b = i0; b < i1; b += 256) {
    const int64_t i = b + threadIdx.x;
    __syncthreads();
    sE[threadIdx.x] = i < i1 ? -kC2 * E[i] : 0.0;
    sW[threadIdx.x] = i < i1 ? wgt[i] : 0.0;
    __syncthreads();
    const int m = (int)min<int64_t>(256, i1 - b);
    for (int k = 0; k < m; ++k) acc = fma(sW[k], exp(sE[k] * invT), acc);
  }
  if (j < nT) part[(int64_t)c * nT + j] = acc;
}

__global__ __launch_bounds__(256) void k_cf_final(const double* partQ, const double* partW, int chunks,
                                                  int32_t nT, double* W, double* Q) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= nT) return;
  double q = 0.0, w = 0.0;
  for (int c = 0; c < chunks; ++c) {
    q += partQ[(int64_t)c * nT + j];
    w += partW[(int64_t)c * nT + j];
  }
  W[j] = (kH * kC / (4.0 * kPI)) * w / q;
  if (Q) Q[j] = q;
}

int cooling_chunks(int32_t nT) {
  const int tb = (nT + 255) / 256;
  return std::max(1, std::min(1024, (2048 + tb - 1) / tb));
}

void launch_cooling(const ModelDev& m, const Work& w, const StatesView& st, const LinesView& ln,
                    const double* T_dev, int32_t nT, double* W, double* Q, hipStream_t s) {
  const int64_t n = ln.n;
  const int bl = (int)std::max<int64_t>(1, std::min<int64_t>(8192, (n + 255) / 256));
  launch_reset(w, s);
  hipLaunchKernelGGL(k_cf_keys, dim3(bl), dim3(256), 0, s, st, ln, w.key, w.stats);
  int32_t *sk = w.key, *sv = nullptr;
  launch_radix_sort(m, w, n, st.n, s, &sk, &sv);
  // run numbers: the flags go to the free ping-pong buffer
  int32_t* rank = (sk == w.keyA) ? w.keyB : w.keyA;
  int32_t* nruns = w.counter + 8;
  double* runE = w.rnu;
  double* runW = reinterpret_cast<double*>(w.rwin);
  if (n > 0) {
    hipLaunchKernelGGL(k_cf_flags, dim3(bl), dim3(256), 0, s, sk, n, (int32_t)st.n, rank);
    launch_scan_i32(rank, n, w.hist, s);  // block sums: the sort's histogram space is free
    hipLaunchKernelGGL(k_cf_runs, dim3(bl), dim3(256), 0, s, sk, sv, rank, n, st, ln, runE, runW, nruns);
  }
  const int chunks = cooling_chunks(nT);
  const int64_t tpad = ((int64_t)nT + 31) / 32 * 32;
  double* partQ = w.part + tpad;
  double* partW = partQ + (int64_t)chunks * nT;
  const dim3 grid(chunks, (nT + 255) / 256);
  hipLaunchKernelGGL(k_cf_sum, grid, dim3(256), 0, s, st.E, st.g, st.n, (const int32_t*)nullptr, T_dev, nT,
                     partQ);
  hipLaunchKernelGGL(k_cf_sum, grid, dim3(256), 0, s, (const double*)runE, (const double*)runW, (int64_t)0,
                     n > 0 ? (const int32_t*)nruns : (const int32_t*)nullptr, T_dev, nT, partW);
  hipLaunchKernelGGL(k_cf_final, dim3((nT + 255) / 256), dim3(256), 0, s, (const double*)partQ,
                     (const double*)partW, chunks, nT, W, Q);
}

}  // namespace xs
