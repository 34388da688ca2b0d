// Internal interface between the host runtime (xsec_api.cpp) and the HIP
// kernels (k_*.hip): device-side parameter blocks and launch wrappers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/xsec.h"

namespace xs {

// CODATA 2018 exact SI values in CGS; c2 = h c / k_B (second radiation
// constant, symbol table of the paper).
constexpr double kH = 6.62607015e-27;      // erg s
constexpr double kC = 2.99792458e10;       // cm / s
constexpr double kKB = 1.380649e-16;       // erg / K
constexpr double kAMU = 1.66053906660e-24; // g
constexpr double kC2 = kH * kC / kKB;      // cm K
constexpr double kPI = 3.14159265358979323846;
constexpr double kLN2 = 0.69314718055994530942;

constexpr int kMaxCond = 256;
// The kind whose widths a profile uses: XS_BIN_x -> XS_x; pseudo-Voigts -> XS_VOIGT.
constexpr int base_profile(int profile) {
  return profile < 4 ? profile : (profile < 8 ? profile - 4 : 3);
}
constexpr int kQBlocks = 256;     // partial sums per slot in the partition-function reduction
constexpr int kItemsPerCU = 256;  // gather work items aimed at per compute unit when tiles are split
constexpr int kAdjBlocks = 16384;    // blocks of the adjoint's grid in a new plan
constexpr int kAdjBlocksMax = 32768;  // the most the configuration allows (sizes the partial sums)
constexpr int kSortItems = 16;    // keys per thread in the radix sort (4096 per block)
// Device counters (int32): [0] gather work queue, [2..3] candidate total,
// [4..5] lines per item, [8] cooling-function runs.
constexpr int kCounterInts = 64;
constexpr int kSortBlock = 256 * kSortItems;
constexpr int kFineBins = 64;  // grid points per sort key (the smallest bucket size)

// Per-condition scalars, uploaded with the workspace.
struct CondDev {
  double T, P, Tv, Tr, cut;
  double Tk;      // kinetic temperature of the widths (T, or T_rot for two temperatures)
  double dop;     // Doppler HWHM per unit wavenumber: alpha = nu * dop (0 for fixed Gaussian)
  double hwhm;    // fixed Gaussian HWHM
  double lnTr;    // ln(T_ref / Tk)
  double pfac;    // P / P_ref
  int32_t slot;   // intensity slot (distinct T or (T_vib, T_rot))
  int32_t wbins;  // bound on |k - k_c| of a nonzero term: ceil(cut / dnu) + 2, less for a narrow Gaussian
  int32_t cclass; // cut-off class (index of the distinct cut-off)
  int32_t pad;
};

// Per intensity slot: the temperatures of the populations.
struct SlotDev {
  double T, Tv, Tr;
};

// Model and grid scalars shared by the kernels.
struct ModelDev {
  int32_t profile, mode, pop, prec;
  double nu0, dnu;
  int64_t n_bins;
  double T_ref, P_ref, hwhm_fixed, mass_amu;
  int32_t n_cond, n_slots;
  int32_t bucket_bins, n_buckets;  // lines bucketed by k_c / bucket_bins
  // Lines are sorted by the finer key k_c / kFineBins (key n_fine = dropped),
  // whatever the bucket size, so that neighbouring sorted lines have nearly
  // equal home bins; a bucket is fine_per_bucket consecutive fine keys.
  int32_t n_fine, fine_per_bucket;
  int32_t n_cut_classes;           // distinct cut-offs (window statistics)
  double max_cut;
};

// Views of the caller's inputs.
struct StatesView {
  int64_t n;
  const double* E;
  const double* g;
  const int32_t* v;
  const double* ev;
  int32_t n_v;
  const double* nv;  // vibronic densities (custom-density populations)
  const double* tau; // state lifetimes (s) for predissociation broadening, or null
};
struct LinesView {
  int64_t n;
  const int32_t* up;
  const int32_t* lo;
  const float* A;
  const float* gref;
  const float* nexp;
  const float* lscale;
  double gref_scalar, nexp_scalar;
};

// One line's inputs and the energies and degeneracy of its states, packed
// by the first line pass in input order, so that the record pass, which
// visits the lines in wavenumber order, fetches one 64-byte block per line
// instead of a cache line from each input array and state table.
struct __attribute__((aligned(64))) LinePack {
  double Eu, El, gu;
  float A, gref, nexp, lscale;
  int32_t u, l;
  double evu, evl;  // E_vib of the upper and lower manifolds (non-LTE; 0 for LTE)
};

// Workspace pointers (carved by the host runtime from the caller's buffer).
struct Work {
  CondDev* cond;            // [n_cond]
  SlotDev* slot;            // [n_slots]
  ModelDev* model;          // [1]
  double* qpart;            // [n_slots][2][kQBlocks]
  double* Q;                // [n_slots]
  double* dQ;               // [n_slots]
  unsigned long long* smax; // [n_slots] ordered keys of max ln|S|
  double* sb;               // [n_slots] log scale s_b (FP32 form)
  int32_t* key;             // [max_lines] bucket key per line
  int32_t* keyA;            // sort ping-pong
  int32_t* keyB;
  int32_t* valA;
  int32_t* valB;
  int32_t* hist;            // [256 * n_sort_blocks] (+ scan block sums)
  int32_t* hsum;            // scan block sums
  int32_t* off;             // [n_buckets + 2] bucket offsets into the sorted records
  double* rnu;              // sorted records: nu
  float* rgref;             //                 gamma_ref
  float* rnexp;             //                 n_exp
  double* rgpre;            //                 lifetime HWHM of the upper state, 1/(4 pi c tau) or 0
                            //                 (kernels get null when the states carry no lifetimes)
  int32_t* ridx;            //                 original line index
  double* rEs;              //                 energy of the state whose population enters S
                            //                 (lower: absorption, upper: emission; LTE adjoint)
  LinePack* lpack;          // [max_lines] line inputs in input order (first pass -> record pass)
  int32_t* rkc;             //                 home bin k_c = rint((nu - nu0)/dnu)
  float* rdel;              //                 nu - nu_{k_c}
  int32_t* rwin;            //                 [n_cut_classes][max_lines][2] window (klo, khi), klo > khi if empty
  void* rS;                 //                 S (f64) or S~ (f32), [n_slots][max_lines]
  int32_t* counter;         // [kCounterInts] work queues, candidate total, lines per item
  int32_t* item_cnt;        // [n_ct_max] candidate lines of each (tile, condition)
  int32_t* item_base;       // [n_ct_max + 1] work items of each (tile, condition), scanned
  int32_t* part_base;       // [n_ct_max + 1] partial rows of split tiles, scanned
  int32_t* item_sums;       // scan block sums
  double* part;             // [2 item_target][1024] partial rows
  int64_t item_target;      // work items aimed at when tiles are split
  unsigned long long* stats;// [8]
  double* adjpart;          // [n_cond][2][kAdjBlocksMax]
  unsigned long long* gmax; // [n_cond] max |dL/dsigma| per condition (bits; FP32 adjoint's scale)
  double* cut_class;        // [n_cut_classes] distinct cut-offs
  int32_t* cut_mult;        // [n_cut_classes] conditions sharing each cut-off
  int64_t max_lines;
  int32_t n_sort_blocks;
};

struct Tiling {
  int32_t tile_bins;   // bins per gather tile: 64 lanes x tile_bins / 64 bins each
  int32_t persistent;
  int32_t grid_blocks; // persistent grid size (one wave per block)
  int64_t chunk_lines; // requested candidate lines per work item (0: automatic)
  int32_t adj_blocks;  // persistent blocks of the adjoint
};

// ---- launch wrappers (k_lines.hip) ----
void launch_partition(const ModelDev& m, const Work& w, const StatesView& st, hipStream_t s);
void launch_lines_pass1(const ModelDev& m, const Work& w, const StatesView& st,
                        const LinesView& ln, hipStream_t s);
// Stable sort of the int32 keys w.key[0..n) (values 0..max_key) with their
// positions; returns the sorted keys and positions (ping-pong buffers).
void launch_radix_sort(const ModelDev& m, const Work& w, int64_t n, int64_t max_key, hipStream_t s,
                       int32_t** sorted_keys, int32_t** sorted_vals);
void launch_offsets_records(const ModelDev& m, const Work& w, const StatesView& st,
                            const LinesView& ln, const int32_t* skeys, const int32_t* svals,
                            int64_t n, hipStream_t s);
void launch_intensity_out(const ModelDev& m, const Work& w, const StatesView& st,
                          const LinesView& ln, void* S, double* log_scale, hipStream_t s);
void launch_q_out(const ModelDev& m, const Work& w, double* Q, double* dQ, hipStream_t s);
void launch_reset(const Work& w, hipStream_t s);
void launch_reset_queue(const Work& w, hipStream_t s);
void launch_scan_i32(int32_t* a, int64_t n, int32_t* sums, hipStream_t s);  // exclusive, in place

// ---- profile pass (k_profile.hip) ----
void launch_gather(const ModelDev& m, const Work& w, const Tiling& t, double* sigma,
                   int accumulate, hipStream_t s);
void launch_scatter(const ModelDev& m, const Work& w, double* sigma, int accumulate,
                    int64_t n_lines, hipStream_t s);

// ---- cooling function (k_cooling.hip) ----
int cooling_chunks(int32_t nT);
void launch_cooling(const ModelDev& m, const Work& w, const StatesView& st, const LinesView& ln,
                    const double* T_dev, int32_t nT, double* W, double* Q, hipStream_t s);

// ---- adjoint (k_adjoint.hip) ----
void launch_adjoint(const ModelDev& m, const Work& w, const StatesView& st, const LinesView& ln,
                    const double* g, double* dT, double* dP, double* dgref, double* dnexp,
                    double* dls, int64_t n_lines, int adj_blocks, hipStream_t s);

}  // namespace xs
