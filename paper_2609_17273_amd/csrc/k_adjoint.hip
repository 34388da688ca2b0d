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
// One wave owns one sorted line (all conditions), lanes stride the window;
// sums are FP64.  Blocks own fixed line sets and the per-condition scalars
// are reduced in a fixed order, so results are deterministic.
#include "k_common.h"

namespace xs {

// Voigt far region with NP Gauss-Hermite pairs: returns Re w, and
//   R1 = Re sum_j W_j (Z + tau_j)/(Z - tau_j)^2       (Im w' = -(2/pi) R1)
//   RG = (4y/pi) sum_j W_j tau_j Im[z/(Z - tau_j)^2] = Re G,  G = w + z w'
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
    else id = (R)1 / d;
    const R id2 = id * id;
    sw += w * (u + y2 + t) * id;
    s1 += w * (A * id + (R)2 * t * (A2 - zi2) * id2);
    sg += w * t * (A2 - zi2 - (R)4 * u * A) * id2;
  }
  rew = (R)(2.0 / kPI) * y * sw;
  r1 = s1;
  rg = (R)(4.0 / kPI) * y * y * sg;
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
    else iq = (R)1 / q;
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
    double wr, wi, dr, di;
    if constexpr (sizeof(R) == 4) w_core_d<16>((double)x, (double)y, wr, wi, dr, di);
    else w_core_d<22>((double)x, (double)y, wr, wi, dr, di);
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
  const int32_t* ridx;
  const void* rS;
  int64_t max_lines;
  StatesView st;
  LinesView ln;
  const double* g;
  double* dgref;
  double* dnexp;
  double* dls;
  double* part;   // [n_cond][2][kAdjBlocks]
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename R, int PROF>
__global__ __launch_bounds__(256) void k_adjoint(AdjArgs a) {
  __shared__ double sdt[4][kMaxCond];
  __shared__ double sdp[4][kMaxCond];
  const ModelDev& m = a.m;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c = threadIdx.x; c < kMaxCond; c += 256)
    for (int w = 0; w < 4; ++w) sdt[w][c] = sdp[w][c] = 0.0;
  __syncthreads();
  const int64_t nk = a.off[m.n_buckets];
  const double sqrt2ln2 = sqrt(2.0 * kLN2);
  for (int64_t p = (int64_t)blockIdx.x * 4 + wave; p < nk; p += (int64_t)gridDim.x * 4) {
    const double nu = a.rnu[p];
    const double gref = (double)a.rgref[p], nexp = (double)a.rnexp[p];
    const int32_t i = a.ridx[p];
    const double Eu = a.st.E[a.ln.up[i]], El = a.st.E[a.ln.lo[i]];
    double dls = 0.0, dgr = 0.0, dne = 0.0;
    for (int c = 0; c < m.n_cond; ++c) {
      const CondDev cd = a.cond[c];
      int64_t klo, khi;
      if (!line_window(nu, cd.cut, m.nu0, m.dnu, m.n_bins, klo, khi)) continue;
      double S = (sizeof(R) == 4)
                     ? (double)((const float*)a.rS)[(int64_t)cd.slot * a.max_lines + p] * exp(a.sb[cd.slot])
                     : ((const double*)a.rS)[(int64_t)cd.slot * a.max_lines + p];
      if (S == 0.0) continue;
      const double alpha = (PROF == XS_GAUSSIAN) ? cd.hwhm : nu * cd.dop;
      const double sgm = alpha / sqrt2ln2;
      const double gpow = exp(nexp * cd.lnTr);
      const double gam = gref * gpow * cd.pfac;
      double inv, y = 0.0;
      if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN) inv = 1.0 / alpha;
      else if (PROF == XS_LORENTZ) inv = 1.0 / gam;
      else {
        inv = sqrt(kLN2) / alpha;
        y = gam * inv;
      }
      const int64_t kc = home_bin(nu, m.nu0, m.dnu);
      const double delta = nu - nu_of_bin(m.nu0, m.dnu, kc);
      const R ra = (R)(m.dnu * inv), rb = (R)(delta * inv), ry = (R)y;
      double sA = 0.0, sB = 0.0, sC = 0.0;
      const double* gc = a.g + (int64_t)c * m.n_bins;
      for (int64_t k0 = klo; k0 <= khi; k0 += 64) {
        // row band from the end bins (uniform across the wave)
        int band = 1;
        if (PROF == XS_VOIGT) {
          const double k1 = (double)(k0 + 63 < khi ? k0 + 63 : khi);
          const double x0 = (double)(k0 - kc) * (double)ra - (double)rb;
          const double x1 = (k1 - (double)kc) * (double)ra - (double)rb;
          const double xm = (x0 <= 0.0 && x1 >= 0.0) ? 0.0 : fmin(fabs(x0), fabs(x1));
          const double rho = xm * xm + y * y;
          if (sizeof(R) == 4) band = rho >= 900.0 * 1.001 ? 1 : (rho >= 64.0 * 1.001 ? 2 : 0);
          else band = rho >= 9.0e6 * 1.001 ? 1 : rho >= 6400.0 * 1.001 ? 2 : rho >= 400.0 * 1.001 ? 3
                    : rho >= 144.0 * 1.001 ? 4 : rho >= 64.0 * 1.001 ? 6 : 0;
        }
        const int64_t k = k0 + lane;
        if (k <= khi) {
          R x;
          if constexpr (sizeof(R) == 4) {
            x = fmaf((float)(k - kc), ra, -rb);
          } else {
#pragma clang fp contract(off)
            x = (nu_of_bin(m.nu0, m.dnu, k) - nu) * inv;
          }
          R f, fs, fg;
          prof_grad<R, PROF>(x, ry, sgm, gam, band, f, fs, fg);
          const double gk = gc[k];
          sA += gk * (double)f;
          sB += gk * (double)fs;
          sC += gk * (double)fg;
        }
      }
      sA = wave_sum(sA);
      sB = wave_sum(sB);
      sC = wave_sum(sC);
      // scale to the unit-area profile and its derivatives
      double A, B, C;
      if (PROF == XS_DOPPLER || PROF == XS_GAUSSIAN) {
        const double c0 = sqrt(kLN2 / kPI) / alpha;
        A = c0 * sA;
        B = c0 * sB / sgm;
        C = 0.0;
      } else if (PROF == XS_LORENTZ) {
        A = sA / (kPI * gam);
        B = 0.0;
        C = sC / (kPI * gam * gam);
      } else {
        const double c0 = 1.0 / (sgm * sqrt(2.0 * kPI));
        A = c0 * sA;
        C = -sC / (2.0 * sqrt(kPI) * sgm * sgm);          // -Im w' / (2 sqrt(pi) sg^2)
        B = -sB / (sgm * sgm * sqrt(2.0 * kPI));          // -Re G / (sg^2 sqrt(2 pi))
      }
      const double T = cd.Tk;
      double dlnS;
      if (m.mode == XS_ABSORPTION)
        dlnS = kC2 * El / (T * T) - (kC2 * nu / (T * T)) / expm1(kC2 * nu / T) - a.dQ[cd.slot] / a.Q[cd.slot];
      else
        dlnS = kC2 * Eu / (T * T) - a.dQ[cd.slot] / a.Q[cd.slot];
      const double dsg_dT = (PROF == XS_GAUSSIAN) ? 0.0 : sgm / (2.0 * T);
      dls += S * A;
      dgr += S * C * gpow * cd.pfac;
      dne += S * C * gam * cd.lnTr;
      if (lane == 0) {
        sdt[wave][c] += S * (A * dlnS + B * dsg_dT - C * nexp * gam / T);
        sdp[wave][c] += (cd.P > 0.0) ? S * C * gam / cd.P : 0.0;
      }
    }
    if (lane == 0) {
      a.dls[i] = dls;
      if (a.dgref) a.dgref[i] = dgr;
      if (a.dnexp) a.dnexp[i] = dne;
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < m.n_cond; c += 256) {
    const double t = ((sdt[0][c] + sdt[1][c]) + sdt[2][c]) + sdt[3][c];
    const double q = ((sdp[0][c] + sdp[1][c]) + sdp[2][c]) + sdp[3][c];
    a.part[((int64_t)c * 2 + 0) * kAdjBlocks + blockIdx.x] = t;
    a.part[((int64_t)c * 2 + 1) * kAdjBlocks + blockIdx.x] = q;
  }
}

__global__ __launch_bounds__(256) void k_adj_final(const double* part, int n_cond, double* dT,
                                                   double* dP) {
  __shared__ double sh[256];
  const int c = blockIdx.x;
  for (int which = 0; which < 2; ++which) {
    double v = 0.0;
    for (int b = threadIdx.x; b < kAdjBlocks; b += 256) v += part[((int64_t)c * 2 + which) * kAdjBlocks + b];
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

__global__ void k_zero3(double* a, double* b, double* c, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (a) a[i] = 0.0;
    if (b) b[i] = 0.0;
    if (c) c[i] = 0.0;
  }
}

void launch_adjoint(const ModelDev& m, const Work& w, const StatesView& st, const LinesView& ln,
                    const double* g, double* dT, double* dP, double* dgref, double* dnexp,
                    double* dls, int64_t n_lines, hipStream_t s) {
  hipLaunchKernelGGL(k_zero3, dim3(2048), dim3(256), 0, s, dgref, dnexp, dls, n_lines);
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
  a.ridx = w.ridx;
  a.rS = w.rS;
  a.max_lines = w.max_lines;
  a.st = st;
  a.ln = ln;
  a.g = g;
  a.dgref = dgref;
  a.dnexp = dnexp;
  a.dls = dls;
  a.part = w.adjpart;
#define XS_A(R, P)                                                                      \
  if (m.profile == P) {                                                                 \
    hipLaunchKernelGGL((k_adjoint<R, P>), dim3(kAdjBlocks), dim3(256), 0, s, a);         \
  }
  if (m.prec == XS_FP32) {
    XS_A(float, XS_DOPPLER) XS_A(float, XS_GAUSSIAN) XS_A(float, XS_LORENTZ) XS_A(float, XS_VOIGT)
  } else {
    XS_A(double, XS_DOPPLER) XS_A(double, XS_GAUSSIAN) XS_A(double, XS_LORENTZ) XS_A(double, XS_VOIGT)
  }
#undef XS_A
  hipLaunchKernelGGL(k_adj_final, dim3(m.n_cond), dim3(256), 0, s, w.adjpart, m.n_cond, dT, dP);
}

}  // namespace xs
