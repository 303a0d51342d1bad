// Internal declarations shared by the HIP kernels and the host plan code.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fstat {

// Device-side view of one work unit plus the plan scratch it uses.
struct WuDev {
  const void* sft;         // [n_sft][n_bins] float2 or packed 16-bit pairs
  const float* scale;      // [n_sft] (16-bit storage)
  const double* t_start;   // [n_sft]
  const double* pos;       // [n_sft][3]
  const double* vel;       // [n_sft][3]
  const double* sky;       // [n_sky][3]
  const float* a;          // [n_sky][n_sft]
  const float* b;          // [n_sky][n_sft]
  double2* geo;            // scratch [n_sky][n_sft]: (tau, Tdot T)
  double4* abcd;           // scratch [n_sky]: (A, B, C, AB - C^2)
  float* twoF;             // [n_sky][n_fd][n_f]
  float2* fa;              // optional, same shape
  float2* fb;              // optional
  float4* coef;            // interp kernel scratch: [n_sft][kCoefPairs][n_bins] coefficient pairs, or with
                           // coef16 [n_sft][2][n_bins] of four FP16 complex coefficients each
  int32_t* cexp;           // coef16: per-SFT exponent e, coefficients stored times 2^-e
  double csum;             // coef16: max_p sum_m |t[m][p]| of the table (bounds |c_p| / max|x|)
  int32_t coef16;
  const double* ctab;      // interp kernel: [2D][kCoef] polynomial coefficients of sinc(kappa+m), in
                           // kappa, or in kappa - 1/2 for the FP16 form
  float4* acc;             // interp kernel scratch: running (Fa, Fb) per template between SFT blocks
  // toplist: templates with 2F >= threshold are appended to cand (2F bits,
  // 0, linear index lo, hi) through the counter cand_count; NULL: no toplist
  uint4* cand;
  unsigned long long* cand_count;
  int64_t cand_cap;        // power of two
  float threshold;
  int32_t top_k;
  int4* top;               // [top_k] (2F bits, sky, fdot, f)
  unsigned long long* n_above;
  int32_t accumulate;      // 1: the epilogue adds 2F to twoF (semi-coherent sum) instead of storing it
  // interp tiles of two sky points: tile sky index p covers sky points
  // sky_pairs[p].x and .y (equal for a point without a partner: computed
  // twice, written once); NULL / 0: one sky point per tile
  const int2* sky_pairs;
  int64_t n_pairs;
  // interp kernels compiled without the global-memory path: tiles (per launch)
  // with an SFT whose windows were not all inside the LDS slice are counted
  // here, and their outputs set to NaN; NULL: not counted
  unsigned long long* dropped;
  int64_t n_sft, n_bins, k_first, n_sky, n_f, n_fd;
  double t_sft, f0, df, fdot0, dfdot, t_ref;
  int32_t dterms;
  int32_t storage;
  int32_t phase_mode;      // 0: frac(phi) in FP64; 1: in double-FP32 (split) products
};

// Spindown-block sizes of split interp launches, largest first: index i runs
// split_nfd(i) = 16, 8, 7, 6, 5, 4 spindowns per thread.
constexpr int kSplitSizes = 6;
__host__ __device__ constexpr int split_nfd(int i) { return i == 0 ? 16 : 9 - i; }

// Tile shape of the demodulation kernels.
struct Tile {
  int32_t nf_reg;   // direct: frequency templates per thread (1, 2 or 4); interp: spindowns per thread
  int32_t chunk;    // direct: SFTs staged in LDS per pass; interp: waves per SIMD the registers must allow (2 to 5)
  int32_t seg;      // interp: LDS segment width in bins (0: derived)
  int32_t sblock;   // interp: SFTs per launch (the SFT loop is split into launches of this many SFTs)
  int32_t threads;  // interp: work-group size, 64 or 256
  int32_t fast;     // interp: 1 if the slice holds every window of every SFT (no slice width was capped), so
                    // the kernel without the global-memory fallback may run
  int32_t pair_seg; // interp: > 0: the ranges of at most 8 spindowns per thread run tiles of two sky points
                    // (WuDev::sky_pairs) with this slice width
  // interp with nf_reg 8, filled by the host for the work unit: the
  // spindowns run as consecutive ranges of fd_split[i] spindowns,
  // split_nfd(i) per thread, slice width seg_split[i], largest blocks first;
  // all zero: one range of nf_reg per thread with slice width seg
  int32_t fd_split[kSplitSizes];
  int32_t seg_split[kSplitSizes];
};

enum Kernel : int32_t { KERNEL_DIRECT = 1, KERNEL_INTERP = 2 };

// Interp kernel: each window weight sinc(kappa + m), kappa in [0, 1), is
// replaced by a degree-7 polynomial in kappa (Chebyshev projection, max error
// 4.3e-7 over the interval, written in monomials of kappa), so the whole
// window sum of bin k is a degree-7 polynomial in kappa with kCoef complex
// coefficients per bin.
constexpr int kCoef = 8;
constexpr int kCoefPairs = kCoef / 2;
// Widest coefficient slice (bins) a work-group of NT threads stages per SFT:
// NT frequency templates plus NT/8 + 2 bins of Doppler and spindown spread
// (34 for 256 threads, 10 for 64) and the slack of 6.  Two buffers of it take
// 37 KB of LDS for 256 threads, so with the per-SFT values four work-groups
// fit a CU.
__host__ __device__ constexpr int seg_cap(int nt) { return nt + nt / 8 + 8; }
constexpr int kSegMax = seg_cap(256);
// FP16 coefficient form: one bin is 2 float4-sized rows (four complex FP16
// coefficients each); a row holds 3 NT / 2 bins (384 for 256 threads).
constexpr int kRows16 = 2;
__host__ __device__ constexpr int seg_cap16(int nt) { return 3 * nt / 2; }
constexpr int kSegMax16 = seg_cap16(256);

// One entry of a batched launch: a work unit's device view and, for the
// demodulation tables, its slice width, its spindowns per thread (4 to 8 or 16),
// the spindown range its tiles cover and the index of its first tile in the
// concatenated tile list.  A work unit has an entry in the table of each
// block size its spindowns are split into (e.g. 13 spindowns: [0, 8) at 8
// per thread and [8, 13) at 5).
struct BatchEntry {
  WuDev w;
  int32_t seg;
  int32_t nfd;
  int32_t fd_begin, fd_end;
  int32_t fast;         // the slice holds every window (see Tile::fast)
  int32_t pad;
  int64_t tile_begin;   // first tile in the concatenated tile list
  int64_t n_tiles;
  int64_t coef_begin;   // first block of the batched coefficient pass
  int64_t sft_begin;    // first SFT in the concatenated SFT list (coef16 exponent pass)
};

// Geometry pass results read back by the host, and the demodulation's count
// of tiles that met a slice too narrow for an SFT's windows (reset once per
// call, not by each geometry pass).
struct GeoStatus {
  int flags;                  // bit 1: window outside the band; bit 2: AB - C^2 <= 0
  int pad;
  unsigned long long max_abs_tau_bits;   // max |tau| over (sky, SFT), as FP64 bits
  unsigned long long max_p_bits;         // max Tdot T over (sky, SFT), as FP64 bits
  unsigned long long max_v_bits;         // max |v| over SFTs (units of c), as FP64 bits
  unsigned long long max_r_bits;         // max |r| over SFTs (light-seconds), as FP64 bits
  unsigned long long dropped;            // demodulation: tiles with an SFT outside the slice
};
// The geometry pass resets the first kGeoResetInts ints (not `dropped`).
constexpr int kGeoResetInts = 10;

// Static scratch of the no-allocation entry point: one array of this many
// bytes per device, laid out as the polynomial tables of every Dterms in both
// bases (kStaticTabBytes), the status record and toplist counter, the
// toplist buffer (kStaticCands entries) and the work region.
constexpr size_t kStaticScratchBytes = (size_t)128 << 20;
constexpr size_t kStaticTabBytes = (size_t)1 << 20;
constexpr size_t kStaticStatusOff = kStaticTabBytes;            // GeoStatus
constexpr size_t kStaticCountOff = kStaticTabBytes + 256;       // toplist counter (2 x u64)
constexpr int64_t kStaticCands = 65536;
constexpr size_t kStaticCandOff = kStaticTabBytes + 4096;       // kStaticCands x 16 B
constexpr size_t kStaticWorkOff = kStaticCandOff + (size_t)kStaticCands * 16;
// Address of this device's static scratch (the current device must be the one asked for).
hipError_t static_scratch_address(void** ptr);

constexpr int kThreads = 256;          // work-group size of the demodulation kernels
// XCDs of the device: the persistent batch kernel keeps one tile queue per XCD
// (kXcds counters of 8 bytes per launch).
constexpr int kXcds = 8;
constexpr int kMaxDterms = 64;

// Width in bins of the LDS segment staged per SFT for a tile of `nf` frequency
// templates: the window span 2D, the templates' spread (nf bins times the
// Doppler factor, below nf + 1 for |v| < 1e-3 c), a one-bin slack on each
// side and rounding to a multiple of 4.
__host__ __device__ inline int seg_width(int nf, int dterms) { return ((nf + 2 * dterms + 4) + 3) & ~3; }

hipError_t launch_fill_int(int* p, int v, int n, hipStream_t s);
hipError_t launch_geometry(const WuDev& w, GeoStatus* status, hipStream_t s);
hipError_t launch_coef(const WuDev& w, hipStream_t s);
hipError_t launch_demod(const WuDev& w, const Tile& t, int kernel, hipStream_t s);
int interp_launches(const WuDev& w, const Tile& t);
// Tiles of spindowns [fd0, fd1) at nfd per thread and nsky sky points per tile.
int64_t interp_tiles(const WuDev& w, int nfd, int64_t fd0, int64_t fd1, int nsky);
int64_t coef_blocks(const WuDev& w);
hipError_t launch_coef_batch(const BatchEntry* ents_dev, int n_ent, int64_t total_blocks, bool c16, hipStream_t s);
// SFTs [al0, al1) of the first n_ent entries (each clipped to its unit's
// SFT count; every one of them must have more than al0 SFTs).
// Tiles are dealt to kXcds queues (counters[0, kXcds)) in chunks of `chunk`.
// The batched kernel exists for split_nfd(i) spindowns per thread, i <
// kSplitSizes (with FP16 coefficients for 8 and 4 only), with one sky point
// per tile, and for 4 to 8 (FP32 coefficients) with tiles of two
// (nsky = 2, the entries' WuDev::sky_pairs); other shapes are refused with
// hipErrorInvalidValue.
hipError_t launch_interp_batch(const BatchEntry* ents_dev, int n_ent, int64_t total_tiles,
                               unsigned long long* counters, int64_t chunk, int grid, bool c16, int nfd, bool fast,
                               int nsky, int64_t al0, int64_t al1, hipStream_t s);
int interp_batch_grid(bool c16, int nfd, bool fast, int nsky);
hipError_t launch_bins(const WuDev& w, int64_t n, const int32_t* i_sky, const int32_t* i_fd, const int32_t* i_f,
                       const int32_t* i_sft, int64_t* kstar, double* kappa, double* phi_frac, hipStream_t s);
int interp_max_seg(int threads, bool c16);
hipError_t launch_cexp(const WuDev& w, hipStream_t s);
// Detector inputs (fstat_detector_inputs): per-SFT position, velocity and
// detector tensor (6 unique components into dten), then a, b per (sky, SFT).
struct SiteModel {
  double lat, lon, az_x, az_y;
};
struct EarthModel {
  double t0, orbit_radius, orbit_rate, orbit_phase, obliquity, earth_radius, sidereal_rate, sidereal_phase;
  int32_t n_sites;
  SiteModel sites[8];
};
hipError_t launch_detector_inputs(const EarthModel& m, int64_t n_sft, const double* t_mid, const int32_t* site_of_sft,
                                  int64_t n_sky, const double* sky, double* pos, double* vel, double* dten, float* a,
                                  float* b, hipStream_t s);
// Toplist selection after the demodulation: sort each work unit's candidate
// segment (cap entries, cap a power of two) and write top and n_above.
hipError_t launch_top_select(const WuDev& w, hipStream_t s);
// Candidates of an existing 2F array (the semi-coherent sum) for the toplist.
hipError_t launch_cand_scan(const WuDev& w, hipStream_t s);
hipError_t launch_top_select_batch(const BatchEntry* ents_dev, int n_ent, uint4* cand, int64_t cap, int max_top_k,
                                   hipStream_t s);
hipError_t launch_cexp_batch(const BatchEntry* ents_dev, int n_ent, int64_t total_sfts, hipStream_t s);

}  // namespace fstat
