/*
 * fstat.h -- C-ABI of the MI355X (gfx950) F-statistic demodulation library.
 *
 * The library computes, for every template (sky direction n, frequency f,
 * spindown fdot) of a work unit, the F-statistic 2F from a set of SFTs (short
 * Fourier transforms of detector data).  This is the F-statistic loop nest of
 * the paper (Listing 1, Section 2): an independent loop over the frequencies
 * of a band, a sum over detectors and, inside it, a sum over the SFTs of each
 * detector followed by a normalisation.  The per-SFT body, which the paper
 * leaves undefined, is the Dirichlet-kernel demodulation:
 *
 *   tau    = (t_start + T/2 - t_ref) + r . n      r: SSB position, light-s
 *   Tdot   = 1 + v . n                            v: velocity, units of c
 *   P      = Tdot * T,   q = (fdot * tau) * P
 *   Dphi   = fma(f, P, q)                         (f + fdot tau) Tdot T: frequency in SFT bins
 *   k*     = floor(Dphi),   kappa = Dphi - k*
 *   phi    = tau * (f + (fdot/2) * tau)           phase in cycles
 *   z      = exp(-2 pi i frac(phi)) * sum_{m=-D}^{D-1} (-1)^(k*-m) x[k*-m] sinc(kappa+m)
 *   Fa     = sum a z,  Fb = sum b z               over all SFTs of all detectors
 *   2F     = 2 (B |Fa|^2 + A |Fb|^2 - 2 C Re(Fa conj Fb)) / (A B - C^2)
 *   A = sum a^2, B = sum b^2, C = sum a b,  sinc(x) = sin(pi x)/(pi x)
 *
 * Frequency templates are f_j = f0 + j*df, spindowns fdot_i = fdot0 + i*dfdot.
 * Dphi and k* are evaluated in IEEE binary64, round to nearest, in exactly the
 * order written above: t_mid = t_start + 0.5 * T, r . n = (r0 n0 + r1 n1) + r2 n2
 * (v . n likewise), tau, Tdot, P and q are each rounded operation by
 * operation, and Dphi is one fused multiply-add f * P + q with a single
 * rounding; nothing else is fused.  So k* and kappa are reproducible bit for
 * bit by any IEEE evaluation of the same sequence.  The window sums and Fa,
 * Fb are accumulated in FP32.  The data arrays follow the flat
 * layout the paper's GPU port adopted (Section 7): the SFTs of all detectors
 * are concatenated along one axis and every per-SFT array (t_start, pos,
 * vel, a, b) is indexed the same way, so detector blocks of any length need
 * no offset array here (the sum over detectors is coherent; a caller's
 * offsets only say which rows belong to which detector).
 *
 * Memory: every array pointer in fstat_wu / fstat_out is a DEVICE pointer on
 * the plan's device, owned by the caller, which must keep it alive until the
 * work queued on the stream has completed.  `stream` arguments are
 * hipStream_t values (NULL = the null stream).  Return values are FSTAT_OK (0)
 * or a negative FSTAT_E_* code; no call aborts or throws.  A plan may be used
 * by one host thread and one stream at a time; distinct plans are independent.
 */
#ifndef FSTAT_H
#define FSTAT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ codes --- */
#define FSTAT_OK 0
#define FSTAT_E_ARG (-1)          /* NULL pointer, bad size or parameter */
#define FSTAT_E_BAND (-2)         /* a Dirichlet window leaves the stored band */
#define FSTAT_E_SIZE (-3)         /* a size exceeds the plan's maxima */
#define FSTAT_E_NOMEM (-4)        /* device or pinned allocation failed */
#define FSTAT_E_DEVICE (-5)       /* HIP runtime error (see fstat_last_error) */
#define FSTAT_E_UNSUPPORTED (-6)  /* option not available on this device */

/* SFT storage: complex64 (float re, float im), or 16-bit pairs with a per-SFT
 * FP32 scale: x = scale[sft] * (re, im). */
#define FSTAT_STORAGE_C64 0
#define FSTAT_STORAGE_BF16 1
#define FSTAT_STORAGE_FP16 2

/* Phase arithmetic: frac(phi) in FP64, or in a double-FP32 (split) product.
 * Dphi and k* are always FP64. */
#define FSTAT_PHASE_FP64 0
#define FSTAT_PHASE_SPLIT_FP32 1

/* Window evaluation: the Dterms loop (DIRECT), or per-bin Chebyshev
 * coefficients of the window sum as a function of kappa (INTERP); AUTO picks. */
#define FSTAT_KERNEL_AUTO 0
#define FSTAT_KERNEL_DIRECT 1
#define FSTAT_KERNEL_INTERP 2

/* fstat_desc.flags */
#define FSTAT_FLAG_NO_GRAPH 1     /* batched: launch directly, no hipGraph */
/* Mixed-precision form of the interp kernel: the per-bin window polynomials
 * (see fstat_compute), written in kappa - 1/2, are stored as FP16 with a
 * per-SFT power-of-two scale and evaluated in packed FP16 arithmetic; the
 * phase rotation and the sums over SFTs stay FP32.  Half the coefficient
 * bytes and fewer vector instructions per (template, SFT) pair.  2F agrees
 * with the FP64 oracle to a relative error of 5e-3 instead of 1e-4.  Not
 * available with FSTAT_KERNEL_DIRECT (FSTAT_E_UNSUPPORTED at plan creation). */
#define FSTAT_FLAG_COEF16 2

/* --------------------------------------------------------- structures --- */

/* Plan descriptor: maxima over every work unit the plan will see. */
typedef struct fstat_desc {
  int64_t max_sft;     /* SFTs per work unit, all detectors together, >= 1 */
  int64_t max_bins;    /* bins per SFT band, >= 1 */
  int64_t max_sky;     /* sky points per work unit, >= 1 */
  int64_t max_fd;      /* spindown templates, >= 1 */
  int64_t max_f;       /* frequency templates, >= 1 */
  int32_t max_dterms;  /* largest Dterms D, 1 <= D <= 64 */
  int32_t storage;     /* FSTAT_STORAGE_* */
  int32_t phase_mode;  /* FSTAT_PHASE_* */
  int32_t kernel;      /* FSTAT_KERNEL_* */
  int32_t flags;       /* FSTAT_FLAG_* */
  int32_t device;      /* HIP device ordinal, or -1 for the current device */
  int64_t max_cands;   /* toplist: capacity of the per-work-unit buffer of templates above the
                          threshold, rounded up to a power of two (0: 65536; at most 2^24) */
} fstat_desc;

/* One work unit (all pointers are device pointers, caller-owned). */
typedef struct fstat_wu {
  int32_t n_det;              /* detectors, >= 1 */
  const int64_t* det_offset;  /* HOST array [n_det + 1] or NULL: the SFTs of detector d are rows
                                 [det_offset[d], det_offset[d+1]) (the flat data + offset arrays of
                                 Section 7); checked (0, non-decreasing, n_sft at the end), otherwise
                                 informational: the sum over detectors is coherent */
  int64_t n_sft;              /* SFTs of all detectors together */
  int64_t n_bins;             /* bins per SFT */
  int64_t k_first;            /* absolute bin index of column 0 (bin k <-> k / T Hz) */
  double t_sft;               /* SFT length T, seconds */
  const void* sft;            /* [n_sft][n_bins] complex: float2 (C64) or uint16 pairs (BF16/FP16) */
  const float* sft_scale;     /* [n_sft] dequantisation scale (16-bit storage), else NULL */
  const double* t_start;      /* [n_sft] GPS start times, seconds */
  const double* pos;          /* [n_sft][3] detector position at the SFT midpoint, light-s */
  const double* vel;          /* [n_sft][3] detector velocity at the SFT midpoint, units of c */
  int64_t n_sky;              /* sky points */
  const double* sky;          /* [n_sky][3] unit vectors towards the source */
  const float* a;             /* [n_sky][n_sft] antenna-pattern factor a (noise weights folded in) */
  const float* b;             /* [n_sky][n_sft] antenna-pattern factor b */
  double f0, df;              /* frequency grid */
  int64_t n_f;
  double fdot0, dfdot;        /* spindown grid, Hz/s */
  int64_t n_fd;
  double t_ref;               /* reference time of f and fdot, seconds */
  int32_t dterms;             /* D: 2D bins per SFT, 1 <= D <= max_dterms */
} fstat_wu;

/* One toplist entry: 2F and the template's sky, spindown and frequency
 * indices (all -1 past the last template that passed the threshold). */
typedef struct fstat_cand {
  float twoF;
  int32_t sky, fdot, f;
} fstat_cand;

/* Outputs, [n_sky][n_fd][n_f] with frequency fastest (device pointers).
 *
 * Toplist (the step after the demodulation, as the search client keeps only
 * the strongest candidates of a work unit for the next stage): with top_k > 0
 * the call also writes to `top` the top_k templates of largest 2F among
 * those with 2F >= threshold, by 2F descending (equal 2F: smaller linear
 * template index (sky * n_fd + fdot) * n_f + f first), and to *n_above the
 * number of templates with 2F >= threshold.  The 2F values are the ones the
 * full output would hold.  If *n_above exceeds the plan's max_cands, the
 * buffer overflowed and `top` holds the best of only max_cands of them: the
 * caller should raise the threshold or max_cands.  twoF may then be NULL, so
 * that the full 2F array is not written at all. */
typedef struct fstat_out {
  float* twoF;                /* [n_sky][n_fd][n_f]; required unless top_k > 0 */
  float* fa;                  /* optional complex (re, im) pairs, or NULL */
  float* fb;                  /* optional complex (re, im) pairs, or NULL */
  int32_t top_k;              /* toplist length, 0 for none; at most max_cands */
  float threshold;            /* toplist: 2F threshold */
  fstat_cand* top;            /* toplist: [top_k] */
  unsigned long long* n_above;/* toplist: one counter */
} fstat_out;

/* Detector site on a spherical Earth: latitude, east longitude, and the
 * azimuths of the two arms from local north towards east (radians). */
typedef struct fstat_site {
  double lat, lon, az_x, az_y;
} fstat_site;

/* Orbit and rotation model of fstat_detector_inputs: the Earth's centre on a
 * circle of radius orbit_radius (light-s) in the ecliptic, tilted by
 * `obliquity` from the equatorial axes, at phase orbit_phase + orbit_rate
 * (t - t0); the site at earth_radius (light-s; 0 drops the diurnal term) with
 * local sidereal angle lon + sidereal_phase + sidereal_rate (t - t0). */
typedef struct fstat_earth {
  double t0;
  double orbit_radius, orbit_rate, orbit_phase, obliquity;
  double earth_radius, sidereal_rate, sidereal_phase;
} fstat_earth;

#define FSTAT_MAX_SITES 8

typedef struct fstat_plan fstat_plan;

/* ------------------------------------------------------------- calls --- */

/* Create a plan for work units within the maxima of *d.  Allocates the plan's
 * device scratch lazily.  Returns FSTAT_E_ARG for an invalid descriptor,
 * FSTAT_E_DEVICE if the device cannot be used.  *out is NULL on failure. */
int fstat_plan_create(fstat_plan** out, const fstat_desc* d);

/* 2F (and optionally Fa, Fb) of every template of one work unit: the
 * frequency-band loop of the F-statistic (Listing 1) with the detector and
 * SFT sums inside.  Validates arguments on the host, then enqueues on
 * `stream`: (1) per (sky, SFT) geometry tau, Tdot and per-sky A, B, C with a
 * check that every window [k*-D+1, k*+D] of the grid lies in the band; the
 * call waits for this check and returns FSTAT_E_BAND (nothing else
 * launched) if it fails; (2) the demodulation kernel, which writes `out`
 * asynchronously.  Between the two, the interp kernel's host side copies the
 * sky vectors back (one more short wait) to pair neighbouring sky points
 * into tiles of two where the slice can hold both (fstat_last_tile reports
 * the shape that ran).  Returns after (2) is enqueued. */
int fstat_compute(fstat_plan* p, const fstat_wu* wu, const fstat_out* out, void* stream);

/* fstat_compute for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and results as fstat_compute on the same plan, with every
 * piece of device scratch (geometry, coefficients, status record, toplist
 * buffer) in one static device array of FSTAT_NOALLOC_SCRATCH_BYTES that
 * each GPU using the library holds until the process ends.  The call itself
 * allocates nothing, device or pinned; create the plan beforehand.  The work
 * unit must fit the array: about 16 B per (sky point, SFT) plus, for the
 * interp kernel, 64 B per (SFT, bin) (32 B with FSTAT_FLAG_COEF16) must stay
 * within FSTAT_NOALLOC_SCRATCH_BYTES less 2 MiB + 4 KiB (the tables, status
 * record and toplist buffer), and top_k within 65536;
 * otherwise FSTAT_E_SIZE with the sizes in fstat_last_error, before anything
 * is launched.  Every call on one GPU shares that GPU's array: calls that
 * overlap in time on one GPU (other threads, other streams, other plans) race
 * and give wrong results; serialise them.  Inputs, outputs, errors and the
 * wait for the band check are as for fstat_compute. */
#define FSTAT_NOALLOC_SCRATCH_BYTES (128u << 20)
int fstat_compute_noalloc(fstat_plan* p, const fstat_wu* wu, const fstat_out* out, void* stream);

/* 2F of many work units with uneven SFT counts, bands and template grids in
 * persistent launches shared by all of them (the "several clients per
 * system" idea of the Cell port, Section 5, done on one device).  Each
 * unit's spindowns are split into ranges run 16 (where its slice holds every
 * window), 8, 7, 6, 5 or 4 per thread (8 or 4 with FP16 coefficients), chosen
 * per unit to waste the fewest lanes weighted by the measured cost of each
 * size (5 spindowns run as one block of 5, 12 as 6 + 6, 32 as 16 + 16); the
 * blocks of at most 8 take tiles of two neighbouring sky points where the
 * unit's sky grid allows (FP32 coefficients; the host reads the sky vectors
 * back once per group to pair them).  Per block of SFTs (256 unless fstat_autotune chose
 * another) one persistent launch per spindown-block size runs over the units
 * with SFTs left; inside a launch the tiles are dealt to one queue per XCD in
 * chunks of consecutive tiles, so that tiles sharing coefficients are served
 * by one L2.  All
 * work units are validated and band-checked before anything is launched; on
 * failure the index of the first failing work unit is in fstat_last_error.
 * The launch sequence is captured once in a hipGraph per signature (table
 * address and shape, SFT blocks, kernel variants, toplist buffers) and
 * replayed; the work-unit table lives in device memory, so a replay may
 * change every pointer and size of the units.  Plan scratch per unit:
 * geometry (16 B per sky point and SFT), coefficients (64 B per SFT and bin,
 * 32 B with FP16 coefficients) and, for units of more SFTs than one block,
 * the carried Fa, Fb (16 B per template); units are processed in groups whose
 * scratch fits 64 GB (FSTAT_BATCH_SCRATCH_GB overrides).  outs[i] belongs to
 * wus[i]. */
int fstat_batch_compute(fstat_plan* p, const fstat_wu* wus, int32_t n_wu, const fstat_out* outs,
                        void* stream);

/* Semi-coherent combination (the search client's second stage combines
 * per-segment statistics incoherently, Section 2): the n_seg work units are
 * time segments of one observation that share the template grid (sky
 * points, f0, df, n_f, fdot0, dfdot, n_fd, t_ref; bands and SFT counts may
 * differ).  The call writes out->twoF = the sum over segments of each
 * segment's coherent 2F, accumulated in segment order (so the result is
 * reproducible bit for bit), and, if out->top_k > 0, the toplist of that sum
 * with the threshold applied to the sum.  out->twoF is required (it holds the
 * sum); Fa/Fb outputs are not available (must be NULL).  Every segment's
 * geometry and band check run first, with one wait for all of them: on
 * FSTAT_E_BAND (or a singular antenna-pattern matrix) nothing has been
 * demodulated and fstat_last_error names the first failing segment; then
 * the segments' demodulations are enqueued back to back.  Plan scratch: the
 * geometry of all segments at once (16 B per sky point and SFT over all
 * segments).  fstat_last_kernel_ms gives the sum over the segments'
 * demodulation launches. */
int fstat_semicoherent(fstat_plan* p, const fstat_wu* segs, int32_t n_seg, const fstat_out* out, void* stream);

/* Bin index, offset and phase of (template, SFT) pairs, computed by the same
 * device code the demodulation kernels use (step "bin index + phase").
 * Index arrays and outputs are device arrays of length n: sky, spindown,
 * frequency and SFT indices in; k* (int64), kappa and frac(phi) (FP64) out. */
int fstat_bins(fstat_plan* p, const fstat_wu* wu, int64_t n, const int32_t* i_sky, const int32_t* i_fd,
               const int32_t* i_f, const int32_t* i_sft, int64_t* kstar, double* kappa, double* phi_frac,
               void* stream);

/* Detector inputs of a work unit, computed on the device (the step before
 * the demodulation; the paper's Cell port notes that most of the data the
 * demodulation reads is produced while the client runs, Section 5):
 * for SFT al with midpoint t_mid[al] taken at site site_of_sft[al] (an index
 * into the host array sites[n_sites], n_sites <= FSTAT_MAX_SITES), the
 * detector position pos[al][3] (light-s) and velocity vel[al][3] (units of c)
 * in equatorial axes, and for each sky direction sky[s][3] the antenna-pattern
 * factors a[s][al], b[s][al]: the plus and cross projections of the detector
 * tensor (u u^T - w w^T)/2 of arm directions u, w on the wave frame
 * X = (sin al, -cos al, 0), Y = (-sin d cos al, -sin d sin al, cos d) of the
 * direction (right ascension al, declination d; al = 0 at the poles).  earth
 * and sites are host pointers; the arrays are device pointers, caller-owned.
 * FP64 arithmetic; a, b are rounded to FP32.  A site index outside
 * [0, n_sites) gives NaN outputs for that SFT. */
int fstat_detector_inputs(fstat_plan* p, const fstat_earth* earth, int32_t n_sites, const fstat_site* sites,
                          int64_t n_sft, const double* t_mid, const int32_t* site_of_sft, int64_t n_sky,
                          const double* sky, double* pos, double* vel, float* a, float* b, void* stream);

/* Measure the candidate tile shapes on this work unit (timed on `stream`,
 * outputs overwritten) and keep the fastest for work units of its class
 * (storage, Dterms, kernel), and, for the interp kernel, the fastest launch
 * shape of fstat_batch_compute for the plan's batch class (storage and
 * coefficient form), timed on this unit as a batch of one.  `cache_path` (may
 * be NULL) names a text file that stores results across processes; it is read
 * first and updated, and only what it lacks is measured.  One line per class:
 * "<class> <nf_reg> <chunk> <sblock> <threads>".  Single-unit classes
 * ("s<storage>_d<Dterms>_k<kernel>_c<coef16>"): spindowns or frequencies per
 * thread (interp 8: the unit's spindowns split into blocks as in
 * fstat_batch_compute, 16 and 4 to 8 per thread for the 256-thread tile with
 * four waves per SIMD and FP32 coefficients, else 8 and 4),
 * waves per SIMD (interp) or SFTs per LDS chunk (direct), SFTs per
 * launch with 0 = all, work-group size of the interp kernel.  Batch classes
 * ("batch_s<storage>_c<coef16>"): spindowns per thread (8: blocks of 16 and
 * 4 to 8 split per unit as fstat_batch_compute describes; 4: blocks of 4 only),
 * tiles per chunk of the per-XCD queues, SFTs per launch (0 = all), 256.
 * Lines naming a shape the library does not implement are ignored. */
int fstat_autotune(fstat_plan* p, const fstat_wu* wu, const fstat_out* out, void* stream,
                   const char* cache_path);

/* Width in bins of the coefficient slice the interp kernel stages in LDS per
 * SFT for a tile of `threads` (256 or 64) frequency templates x nfd
 * spindowns, for a work unit with frequency step df and spindown step dfdot
 * whose (sky, SFT) pairs have at most max_abs_tau = max |tau| (s) and
 * max_p = max Tdot T (s): the bins k* can move across such a tile
 * ((threads - 1) df + |dfdot| (nfd - 1) max_abs_tau) max_p, plus slack,
 * rounded down to a multiple of 4 and capped at the LDS row (296 bins, or 384
 * with coef16 != 0, for 256 threads).  *fits (may be NULL) is 1 when the cap
 * did not bind: then every window of every tile lies in its slice and the
 * kernel variant without a global-memory path runs.  Should that ever be
 * false for some tile and SFT, the tile's outputs are NaN and the next call
 * on the plan returns FSTAT_E_DEVICE saying how many tiles were affected.
 * A host function: no device, plan or allocation involved. */
int32_t fstat_interp_slice(double df, double dfdot, int32_t nfd, int32_t threads, int32_t coef16, double max_abs_tau,
                           double max_p, int32_t* fits);

/* The pairing of sky points into tiles of two that the interp kernels use
 * for ranges of at most 8 spindowns per thread (FP32 coefficients), for a
 * work unit with the given template grids whose geometry has at most
 * max_abs_tau = max |tau| (s), max_p = max Tdot T (s) over its (sky, SFT)
 * pairs, max_v = max |v| (units of c) and max_r = max |r| (light-s) over its
 * SFTs.  The bins of two sky points differ by at most |n0 - n1| (f_max T max_v
 * + |fdot|max (max_abs_tau T max_v + max_p max_r)), which widens the slice
 * of one sky point's tile (fstat_interp_slice at min(n_fd, 8) spindowns);
 * neighbouring points (bands of z, alternately rising and falling longitude)
 * pair while that width fits the LDS row.  sky: host array [n_sky][3] of
 * unit vectors.  Writes the tiles to `pairs` (host [2 n_sky]: tile t covers
 * sky points pairs[2t] and pairs[2t + 1], equal for a point without a
 * partner) and their count to *n_pairs, and returns the paired tiles' slice
 * width, or 0 when one sky point per tile is kept (fewer than half the
 * points pair, or n_sky < 4; *n_pairs is then 0).  Returns FSTAT_E_ARG for
 * NULL arrays or n_sky < 1.  A host function: no device, plan or allocation
 * involved. */
int32_t fstat_sky_pairs(int64_t n_sky, const double* sky, double f0, double df, int64_t n_f, double fdot0,
                        double dfdot, int64_t n_fd, double t_sft, double max_abs_tau, double max_p, double max_v,
                        double max_r, int32_t* pairs, int64_t* n_pairs);

/* The split of n_fd spindowns into blocks per thread that the interp kernels
 * run (fstat_compute with its default tile, fstat_batch_compute with its
 * default launch shape): out[0..5] = the spindowns run 16, 8, 7, 6, 5 and 4
 * per thread, as consecutive ranges in that order, each range's last block
 * possibly partial.  The split minimises the lanes computed weighted by the
 * measured time per lane of each block size.  allow16: blocks of 16 allowed
 * (the library allows them where their wider slice holds every window);
 * paired: the unit's sky points pair into tiles of two (which makes the
 * blocks of at most 8 cheaper); coef16: the FP16-coefficient form (blocks of
 * 8 and 4 only, never paired).  A host function: no device, plan or
 * allocation involved.  Returns FSTAT_OK, or FSTAT_E_ARG for n_fd < 1 or a
 * NULL `out`. */
int fstat_spindown_split(int64_t n_fd, int32_t coef16, int32_t allow16, int32_t paired, int64_t* out);

/* Duration in milliseconds of the last demodulation kernel of the last
 * fstat_compute / fstat_batch_compute call (after fstat_semicoherent: the
 * sum over its segments' demodulation kernels), measured with HIP events on
 * the stream it ran on (waits for it).  Returns a negative value if none. */
double fstat_last_kernel_ms(fstat_plan* p);

/* The launch shape of the plan's last single-unit demodulation (the last
 * fstat_compute or fstat_compute_noalloc call, the last segment of
 * fstat_semicoherent, the last unit of fstat_batch_compute with the direct
 * kernel, or the last shape fstat_autotune timed; the batched interp form
 * does not set it), for tuning and tests: out[0..4] = spindowns per thread (interp) or frequencies
 * per thread (direct), waves per SIMD or SFTs per LDS chunk, slice width,
 * SFTs per launch (0: all), work-group size; out[5] = slice width of the
 * tiles of two sky points (0: one sky point per tile); out[6] = number of
 * sky tiles (sky points, or pairs); out[7..12] = the spindowns run 16, 8, 7,
 * 6, 5 and 4 per thread (all 0: one range at out[0] per thread).  `out`
 * holds FSTAT_LAST_TILE_LEN entries.  Returns FSTAT_OK, or FSTAT_E_ARG for
 * NULL arguments or before any such call. */
#define FSTAT_LAST_TILE_LEN 13
int fstat_last_tile(const fstat_plan* p, int32_t* out);

/* Release the plan and everything it allocated (waits for its device work).
 * Safe on NULL and after any error. */
void fstat_plan_destroy(fstat_plan* p);

/* Static text for a return code. */
const char* fstat_strerror(int code);

/* Text of the plan's last error ("" if none); valid until the next call on p. */
const char* fstat_last_error(const fstat_plan* p);

#ifdef __cplusplus
}
#endif

#endif /* FSTAT_H */
