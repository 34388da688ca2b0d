/*
 * xsec.h -- C-ABI of the MI355X (gfx950) line-list cross-section library.
 *
 * The library computes, on one GPU, the line-list post-processing path of
 * PyExoCross 2.0 (arXiv 2609.17273):
 *   states (E, g) + transitions (u, l, A) + broadening (gamma_ref, n_exp)
 *   + conditions (T, P or T_vib, T_rot) + grid + cut-off + profile
 *   -> partition functions Q, line intensities S_i, cross sections sigma(nu).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Array arguments are DEVICE pointers (memory of the GPU the plan was made
 *    on), contiguous, structure-of-arrays, owned by the caller.  The library
 *    never frees them and never keeps them beyond the call, except inside a
 *    captured graph (xs_plan_capture), which keeps the pointers it was given
 *    until the plan is destroyed or recaptured.
 *  - Structs passed by pointer (xs_model, xs_grid, xs_condition arrays,
 *    xs_states, xs_lines) are HOST memory, read during the call only.
 *  - Calls enqueue work on the plan's HIP stream and return XS_OK once it is
 *    enqueued; results are ready when that stream is synchronised.  Faults in
 *    enqueued work surface as XS_EDEVICE from xs_plan_sync or a later call.
 *  - All arguments are validated on the host before any GPU work is enqueued;
 *    a rejected call returns a negative xs_status, enqueues nothing and sets
 *    the thread-local message returned by xs_last_error().  Nothing aborts and
 *    no C++ exception crosses the ABI.
 *  - Lines with nu = E_upper - E_lower <= 0 are discarded (not an error), as are
 *    lines whose cut-off window misses the grid (section "Spectral synthesis":
 *    lines outside the grid still count when their wings reach it).
 *  - One plan must not be used from two host threads at once; two plans on one
 *    GPU may run concurrently on different streams.
 */
#ifndef XSEC_H
#define XSEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  XS_OK = 0,
  XS_EINVAL = -1,       /* an argument is out of range or a required pointer is NULL */
  XS_ENOMEM = -2,       /* a host allocation failed */
  XS_EDEVICE = -3,      /* a HIP runtime call or an enqueued kernel failed */
  XS_EWORKSPACE = -4,   /* no workspace bound, or the bound one is too small */
  XS_EUNSUPPORTED = -5  /* a valid combination this library does not implement */
} xs_status;

/* Line profile (Table tab:profile): Doppler (width from T, nu, mass); Gaussian
 * with a user HWHM; Lorentzian (pressure); Voigt in the scipy.special
 * voigt_profile convention (Gaussian standard deviation sg = alpha/sqrt(2 ln2),
 * Lorentzian HWHM gamma), i.e. Re w(z)/(sg sqrt(2 pi)), z = (d + i gamma)/(sg sqrt 2).
 * XS_BIN_*: the binned (bin-integrated) methods of the same table: the mean of
 * the profile over the bin [nu_k - dnu/2, nu_k + dnu/2] centred on each grid
 * point, i.e. (F(d + dnu/2) - F(d - dnu/2)) / dnu with F the profile's
 * cumulative distribution; the cut-off still tests the bin centre.  Widths and
 * parameters as for the sampled kind (XS_BIN_x = XS_x + 4).
 * XS_PV_*: the pseudo-Voigt methods of the same table, with the Voigt's widths
 * (Doppler alpha, Lorentzian gamma): eta L(d; f) + (1 - eta) G(d; f), a
 * unit-area Lorentzian and Gaussian of one FWHM f from fG = 2 alpha and
 * fL = 2 gamma, by the Thompson-Cox-Hastings width polynomial (XS_PV_THOMPSON)
 * or the Olivero-Longbothum formula 0.5346 fL + sqrt(0.2166 fL^2 + fG^2)
 * (XS_PV_OLIVERO), with eta = 1.36603 r - 0.47719 r^2 + 0.11116 r^3,
 * r = fL / f.  Binned and pseudo-Voigt kinds are forward only: the adjoint
 * returns XS_EUNSUPPORTED for them. */
typedef enum {
  XS_DOPPLER = 0, XS_GAUSSIAN = 1, XS_LORENTZ = 2, XS_VOIGT = 3,
  XS_BIN_DOPPLER = 4, XS_BIN_GAUSSIAN = 5, XS_BIN_LORENTZ = 6, XS_BIN_VOIGT = 7,
  XS_PV_THOMPSON = 8, XS_PV_OLIVERO = 9
} xs_profile;
/* Absorption (Eq. abs intensity lte, Eq. nlte ab 2T) or emission
 * (Eq. ems intensity lte, Eq. nlte em 2T) intensities. */
typedef enum { XS_ABSORPTION = 0, XS_EMISSION = 1 } xs_mode;
/* LTE Boltzmann populations (Eq. F lte); the two-temperature populations of
 * Eq. (F nlte 2T) with E = E_vib(v) + E_rot (Eqs. Enonlte, Erot nonlte),
 * intensities by Eqs. (nlte ab 2T), (nlte em 2T); or custom vibronic
 * densities, Eq. (F nlte Nvib): a user weight n_vib(v) per manifold and
 * rotational levels at T_rot, Q(T_rot) by Eq. (Q nlte Nvib), intensities by
 * Eqs. (nlte ab pop density), (nlte em pop density). */
typedef enum { XS_LTE = 0, XS_NLTE_2T = 1, XS_NLTE_DENSITY = 2 } xs_population;
/* XS_FP64: every step in FP64.  XS_FP32: profile arithmetic in FP32 with
 * intensities stored as S~ = exp(ln S - s_b) in FP32 (s_b = max ln|S| over
 * the chunk, per temperature), FP64 partition functions, window bounds and
 * per-bin accumulation; sigma = exp(s_b) * acc in FP64. */
typedef enum { XS_FP64 = 0, XS_FP32 = 1 } xs_precision;
/* XS_GATHER: grid-tile-parallel gather over the wavenumber-bucketed line
 * stream.  XS_SCATTER: line-parallel evaluation with atomic adds into sigma. */
typedef enum { XS_GATHER = 0, XS_SCATTER = 1 } xs_algo;

typedef struct {
  int32_t profile;     /* xs_profile */
  int32_t mode;        /* xs_mode */
  int32_t population;  /* xs_population */
  int32_t precision;   /* xs_precision */
  int32_t algo;        /* xs_algo */
  double mass_amu;     /* molecular mass for the Doppler width (> 0 for Doppler/Voigt) */
  double T_ref;        /* reference temperature of gamma_ref, K (> 0; ExoMol: 296) */
  double P_ref;        /* reference pressure of gamma_ref, bar (> 0; 1) */
  double hwhm_fixed;   /* Gaussian HWHM in cm^-1 for XS_GAUSSIAN, XS_BIN_GAUSSIAN (> 0), else ignored */
} xs_model;

/* Grid points nu_k = nu0 + k * dnu, k = 0 .. n_bins-1 (cm^-1), the user
 * wavenumber grid of section "Spectral synthesis". */
typedef struct {
  double nu0;
  double dnu;      /* > 0 */
  int64_t n_bins;  /* >= 1 */
} xs_grid;

/* One thermodynamic condition.  LTE uses T (K); two-temperature runs use
 * T_vib and T_rot, custom-density runs T_rot only (T and T_vib ignored); both
 * non-LTE forms take T_rot as the kinetic temperature of the Doppler and
 * pressure widths (section on LTE/non-LTE comparison).  P in bar (>= 0;
 * > 0 for Lorentzian).  cutoff: line-wing cut-off in cm^-1 (> 0): grid point k
 * receives line i iff |nu_k - nu_i| <= cutoff, both sides rounded in FP64. */
typedef struct {
  double T, P, T_vib, T_rot, cutoff;
} xs_condition;

/* Predissociation (lifetime) broadening (section "Spectral synthesis"): with
 * states.lifetime given, a line whose upper state has a finite lifetime
 * tau > 0 gets the natural Lorentzian HWHM 1/(4 pi c tau) (cm^-1) added to its
 * pressure width gamma, for every profile with a Lorentzian part (Lorentzian,
 * Voigt and their binned forms); stable states (tau = inf) and tau <= 0 or
 * NaN add nothing.  The adjoint's gamma_ref, n_exp, T and P gradients act on
 * the pressure part only, which the lifetime width does not depend on.
 *
 * States (Table tab:exomolstates, compulsory part): term values E (cm^-1,
 * FP64) and total degeneracies g_tot (FP64), dense 0-based indices.  Non-LTE
 * runs also need v[n] (manifold index, 0 <= v < n_v) and the table e_vib[n_v]
 * of E_vib(v) (cm^-1); custom-density runs also the weights n_vib[n_v]
 * (relative populations of the manifolds, Eq. Nvib; only their ratios
 * matter, since Q carries the same weights; a weight that is not > 0 gives
 * its manifold's states no population).  All arrays are device memory. */
typedef struct {
  int64_t n;
  const double* energy;
  const double* g_tot;
  const int32_t* v;        /* NULL for LTE */
  const double* e_vib;     /* NULL for LTE */
  int32_t n_v;
  const double* n_vib;     /* XS_NLTE_DENSITY only, else ignored */
  const double* lifetime;  /* per-state lifetime tau in s, or NULL: predissociation broadening */
} xs_states;

/* Transitions (Table tab:exomoltrans) and broadening (Table tab:exomolbroad):
 * upper/lower 0-based state indices, Einstein A (s^-1), and per-line
 * gamma_ref (cm^-1/bar at T_ref, P_ref) and temperature exponent n_exp, or
 * NULL to use the scalars.  log_scale: optional per-line log-intensity scale
 * s_i (S_i -> S_i exp(s_i)); NULL means 0. */
typedef struct {
  int64_t n;
  const int32_t* upper;
  const int32_t* lower;
  const float* einstein_a;
  const float* gamma_ref;
  const float* n_exp;
  const float* log_scale;
  double gamma_ref_scalar;
  double n_exp_scalar;
} xs_lines;

/* Kernel configuration.  The gather cuts the grid into tiles of tile_bins
 * points (256, 512 or 1024, 256 in a new plan; one wave of 64 lanes, each lane
 * every 64th point).
 * A work item is one (tile, condition) and a slice of at most chunk_lines of
 * the tile's candidate lines; a tile split over several items is summed from
 * their partial rows in item order, so results do not depend on scheduling.
 * chunk_lines: 0 = automatic (about 256 items per compute unit when the
 * tiles alone are too few), else a multiple of 64 (the automatic size wins
 * when it is larger).  bucket_bins: grid points per line bucket (power of two,
 * 64..4096; a new plan starts at 64 for the Doppler and fixed-width Gaussian,
 * 256 otherwise); persistent: 1 = one persistent launch pulling items from a
 * device queue, 0 = one workgroup per item; waves_per_cu: size of the
 * persistent grid in waves per compute unit (4..64); adj_blocks: blocks of
 * 256 threads of the adjoint's grid, each wave taking every (4 adj_blocks)-th
 * batch of 64 sorted lines (0 = 16384, else a multiple of 256 in
 * 256..32768; its per-block partial sums of dL/dT, dL/dP are added in block
 * order, so each value is deterministic). */
typedef struct {
  int32_t tile_bins;
  int32_t bucket_bins;
  int32_t persistent;
  int32_t waves_per_cu;
  int32_t chunk_lines;
  int32_t adj_blocks;
} xs_config;

/* Counters of the last xs_cross_section / adjoint call (read after sync). */
typedef struct {
  int64_t lines_in;        /* lines given */
  int64_t lines_kept;      /* lines with nu > 0 whose window reaches the grid */
  int64_t window_pairs;    /* sum over conditions and kept lines of window bins on the grid */
  int64_t work_items;      /* gather work items (conditions x tiles) */
  int64_t lines_invalid;   /* lines dropped for a state (or manifold) index outside the tables */
} xs_stats;

typedef struct xs_plan xs_plan;

/* Create a plan for one grid, model and list of n_cond conditions (host
 * array), for line chunks of at most max_lines lines, on the GPU that is
 * current and the given stream (a hipStream_t; NULL = the default stream).
 * Conditions that share T (LTE) or (T_vib, T_rot) share one intensity vector
 * (the paper's combined stick-spectrum / cross-section reuse).  Errors:
 * XS_EINVAL for out-of-range values (listed in the types above), n_cond < 1,
 * max_lines < 1 or > 2^31 - 1, n_bins > 2^31 - 1; XS_ENOMEM; XS_EDEVICE if no
 * GPU is usable.  *out is NULL on error. */
int xs_plan_create(xs_plan** out, const xs_model* model, const xs_grid* grid, int32_t n_cond,
                   const xs_condition* conds, int64_t max_lines, void* stream);

/* Replace the plan's conditions (same count n_cond; validated as in
 * xs_plan_create) and re-upload them to the bound workspace.  A captured
 * graph is dropped (recapture before replaying).  Errors: XS_EINVAL. */
int xs_plan_set_conditions(xs_plan* plan, int32_t n_cond, const xs_condition* conds);

/* Release the plan, its captured graph and its internal events.  Does not
 * touch the caller's workspace or arrays.  NULL is ignored. */
void xs_plan_destroy(xs_plan* plan);

/* Device workspace the plan needs for chunks of max_lines lines (bytes). */
int xs_plan_workspace_bytes(const xs_plan* plan, size_t* bytes);

/* Bind caller-allocated device memory (256-byte aligned, >= the size above)
 * as the plan's workspace.  The plan uses it until rebound or destroyed.
 * Errors: XS_EINVAL (NULL/misaligned), XS_EWORKSPACE (too small). */
int xs_plan_set_workspace(xs_plan* plan, void* dptr, size_t bytes);

/* Override or read the kernel configuration (validated; XS_EINVAL otherwise). */
int xs_plan_set_config(xs_plan* plan, const xs_config* cfg);
int xs_plan_get_config(const xs_plan* plan, xs_config* cfg);

/* Partition functions, Eq. (pf) (LTE) or Eq. (Q nlte 2T), one per condition,
 * in FP64: Q[n_cond] and, for LTE, dQdT[n_cond] = sum g (c2 E / T^2)
 * exp(-c2 E/T) (may be NULL; NaN for two temperatures).  Device outputs. */
int xs_partition_function(xs_plan* plan, const xs_states* states, double* Q, double* dQdT);

/* Line intensities (stick spectrum) of every line for every condition,
 * S[c * n + i], by Eqs. (abs intensity lte), (nlte ab 2T), (ems intensity lte)
 * or (nlte em 2T); 0 for discarded lines.  XS_FP64: S is double[n_cond * n].
 * XS_FP32: S is float[n_cond * n] holding S~ = S exp(-s_c) and log_scale[c]
 * (double, device) holds s_c = max_i ln|S_ic|; S = exp(s_c) * S~.  Two-
 * temperature absorption can be negative (population inversion).  Requires
 * lines->n <= max_lines. */
int xs_line_intensities(xs_plan* plan, const xs_states* states, const xs_lines* lines,
                        void* S, double* log_scale);

/* Cross sections, Eq. (xsec) with unit-area profiles and the cut-off rule:
 * sigma[c * n_bins + k] = (accumulate ? sigma : 0) + sum_i S_ic f_ic(nu_k - nu_i)
 * over kept lines with |nu_k - nu_i| <= cutoff_c.  sigma is double
 * [n_cond][n_bins], device.  accumulate = 1 adds this chunk of lines to sigma
 * (streaming a line list in chunks of at most max_lines).  Requires a bound
 * workspace (XS_EWORKSPACE). */
int xs_cross_section(xs_plan* plan, const xs_states* states, const xs_lines* lines,
                     double* sigma, int32_t accumulate);

/* Adjoint of xs_cross_section (LTE, sampled profiles; XS_EUNSUPPORTED otherwise): given
 * dL_dsigma[n_cond][n_bins] (double, device), writes
 *   dL_dT[n_cond], dL_dP[n_cond]                              (double, device)
 *   dL_dgamma_ref[n], dL_dn_exp[n], dL_dlog_scale[n]           (double, device,
 *       original line order, summed over conditions; 0 for discarded lines)
 * through S_i(T) (Eq. abs/ems intensity lte, Q'(T)), the Doppler width
 * alpha ~ sqrt(T) and the pressure width gamma = gamma_ref (T_ref/T)^n P/P_ref.
 * The profile windows are recomputed; no (line, bin) pairs are stored.
 * dL_dgamma_ref and dL_dn_exp may be NULL.  With per-line gamma_ref/n_exp NULL
 * (scalars), their gradients are still returned per line.  The FP32 form sums
 * window blocks in FP32 with the cotangent of each condition scaled by the
 * power of two that brings its largest magnitude into [1/2, 1), and removes
 * the scale exactly in FP64, so its accuracy does not depend on the loss's
 * magnitude (cotangents of 1e-30 and 1e+10 behave alike); a non-finite
 * cotangent propagates into the results unscaled. */
int xs_cross_section_adjoint(xs_plan* plan, const xs_states* states, const xs_lines* lines,
                             const double* dL_dsigma, double* dL_dT, double* dL_dP,
                             double* dL_dgamma_ref, double* dL_dn_exp, double* dL_dlog_scale);

/* The two stages of xs_cross_section, for callers that reuse one line list
 * (the paper's combined stick-spectrum / cross-section mode) or time the
 * profile kernel on its own.
 * xs_prepare: partition functions, intensities, bucketing of the lines by
 *   home bin and the sorted line records, kept in the workspace.
 * xs_profile_pass: the profile pass (gather or scatter per model.algo) over the
 *   records of the last xs_prepare; same sigma contract as xs_cross_section.
 * xs_profile_adjoint: the adjoint over the records of the last xs_prepare;
 *   same contract as xs_cross_section_adjoint (states and lines must be the
 *   ones given to xs_prepare).
 * Calling xs_profile_pass / xs_profile_adjoint without a preceding xs_prepare on the same workspace
 * returns XS_EINVAL. */
int xs_prepare(xs_plan* plan, const xs_states* states, const xs_lines* lines);
int xs_profile_pass(xs_plan* plan, double* sigma, int32_t accumulate);
int xs_profile_adjoint(xs_plan* plan, const xs_states* states, const xs_lines* lines,
                       const double* dL_dsigma, double* dL_dT, double* dL_dP,
                       double* dL_dgamma_ref, double* dL_dn_exp, double* dL_dlog_scale);

/* Cooling function, Eq. (cf) (LTE; XS_EUNSUPPORTED otherwise):
 *   W(T_j) = 1/(4 pi Q(T_j)) sum over lines of A h c nu g_u exp(-c2 E_u / T_j)
 * in erg s^-1 molecule^-1 sr^-1, with Q(T_j) of Eq. (pf), for the n_T
 * temperatures T[n_T] (HOST array, K, each > 0 and finite; 1 <= n_T <= 2^20).
 * W[n_T] (double, device) receives W; Q[n_T] (double, device, may be NULL)
 * receives Q.  Lines with nu <= 0 or state indices outside the table add
 * nothing (counted in xs_stats as for xs_prepare).  FP64 throughout, whatever
 * model.precision; deterministic.  Uses the plan's workspace and stream and
 * returns once the temperatures are uploaded; it overwrites the records of
 * the last xs_prepare (xs_profile_pass / xs_profile_adjoint then need a new
 * xs_prepare).  Requires lines->n <= max_lines.  Errors: XS_EINVAL (bad
 * arguments, or n_T beyond what the workspace holds: 32 x 1024 x the GPU's
 * compute units x 2 doubles less the partial sums), XS_EWORKSPACE. */
int xs_cooling_function(xs_plan* plan, const xs_states* states, const xs_lines* lines,
                        int32_t n_T, const double* T, double* W, double* Q);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * xs_cross_section path with the same arguments and sigma contract, run with
 * its workspace carved from a static scratch array of 64 MiB that the library
 * holds on each GPU it runs on until the process ends, instead of the plan's
 * bound workspace (which need not exist, and is left untouched with the
 * records of its last xs_prepare).  Nothing is allocated: no hipMalloc,
 * hipFree or allocating library routine.  The gather aims at 2 work items per
 * compute unit here, so FP64 results agree with xs_cross_section to rounding
 * (the split of tiles into partial rows differs) rather than bitwise.  Every
 * call on one GPU shares that GPU's scratch and leaves its contents behind:
 * calls that overlap on one GPU (other threads, or plans on other streams
 * with work still running) race.  The call uploads the plan's conditions and
 * waits for the plan's stream to take them, then returns once the path is
 * enqueued.  xs_plan_get_stats keeps reporting the plan's own workspace.
 * Errors: as xs_cross_section, but no workspace is required; XS_EWORKSPACE
 * when the plan's layout (max_lines lines, n_bins points, n_cond conditions)
 * exceeds 64 MiB; XS_EINVAL when the plan's GPU is not the current device. */
int xs_cross_section_noalloc(xs_plan* plan, const xs_states* states, const xs_lines* lines,
                             double* sigma, int32_t accumulate);

/* Record one xs_cross_section call with these arguments into a HIP graph
 * (no kernel runs during capture); xs_plan_replay launches it on the plan's
 * stream.  The pointers are kept until destroy or the next capture. */
int xs_plan_capture(xs_plan* plan, const xs_states* states, const xs_lines* lines,
                    double* sigma, int32_t accumulate);
int xs_plan_replay(xs_plan* plan);

/* Time the candidate kernel configurations on these inputs (sigma is used as
 * scratch and overwritten): the plan's bucket size and the other of 64 and
 * 256 points (the lines are re-bucketed in the plan's workspace), each with
 * 256-, 512- and 1024-point tiles and three launch modes; then, for LTE
 * sampled profiles, the adjoint's grid of 4096, 8192, 16384 or 32768 blocks
 * (sigma serves as its cotangent).  Keeps the fastest and caches it under
 * cache_path (JSON, keyed by device, profile, precision, window size, line
 * count and number of conditions; NULL: no file).  A cached entry is reused
 * without timing.  When the chosen bucket size is not the last one tried,
 * the next xs_cross_section re-buckets the lines. */
int xs_plan_autotune(xs_plan* plan, const xs_states* states, const xs_lines* lines,
                     double* sigma, const char* cache_path);

/* Counters of the last call, read after synchronising (see xs_stats). */
int xs_plan_get_stats(xs_plan* plan, xs_stats* stats);

/* Wait for the plan's stream; XS_EDEVICE if enqueued work failed. */
int xs_plan_sync(xs_plan* plan);

/* Message of the last failed call on this thread ("" if none). */
const char* xs_last_error(void);

/* Library version string. */
const char* xs_version(void);

#ifdef __cplusplus
}
#endif
#endif /* XSEC_H */
