// Host side of the F-statistic library: plan, argument validation, scratch
// management, launch sequencing, autotuning and the C-ABI entry points
// declared in include/fstat.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fstat.h"
#include "fstat_internal.h"

using fstat::Tile;
using fstat::WuDev;

struct fstat_plan {
  fstat_desc d{};
  int device = 0;
  int cu_count = 0;
  char err[512] = "";
  // scratch (device)
  void* geo = nullptr;
  size_t geo_bytes = 0;
  void* abcd = nullptr;
  size_t abcd_bytes = 0;
  fstat::GeoStatus* status_d = nullptr;
  fstat::GeoStatus* status_h = nullptr;  // pinned
  double max_abs_tau = 0.0;               // from the last geometry pass
  double max_p = 0.0;                     // max Tdot T, from the last geometry pass
  // interp kernel: coefficient scratch and per-Dterms polynomial tables
  void* coef = nullptr;
  size_t coef_bytes = 0;
  void* acc = nullptr;
  size_t acc_bytes = 0;
  std::map<int, double*> ctab;
  std::map<int, double> csum;              // per Dterms: max_p sum_m |t[m][p]|
  void* cexp = nullptr;                    // FP16 coefficient form: per-SFT exponents
  size_t cexp_bytes = 0;
  // toplist: candidate capacity per work unit (power of two), the single-unit
  // buffer and counter, and the batched ones (one segment per work unit)
  int64_t cand_cap = 0;
  void* cand = nullptr;
  size_t cand_bytes = 0;
  void* cand_count = nullptr;
  size_t cand_count_bytes = 0;
  void* bcand = nullptr;
  size_t bcand_bytes = 0;
  void* bcount = nullptr;
  size_t bcount_bytes = 0;
  // detector inputs: per-SFT detector tensors
  void* dten = nullptr;
  size_t dten_bytes = 0;
  // timing
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipStream_t ev_stream = nullptr;
  bool timed = false;
  double ms_prev = 0.0;                    // semi-coherent: demodulation time of the earlier segments
  // tile choices per class key
  std::map<std::string, Tile> tiles;
  // batched form: scratch arena, per-work-unit statuses, work-unit tables,
  // tile counter, capture stream and instantiated graphs
  void* arena = nullptr;
  size_t arena_bytes = 0;
  fstat::GeoStatus* bstat_d = nullptr;
  fstat::GeoStatus* bstat_h = nullptr;
  size_t bstat_cap = 0;
  fstat::BatchEntry* ents_d = nullptr;
  fstat::BatchEntry* ents_h = nullptr;
  size_t ents_cap = 0;
  unsigned long long* counter = nullptr;
  // launch shape of the last single-unit demodulation (fstat_last_tile)
  bool have_last = false;
  Tile last_tile{};
  int64_t last_sky_tiles = 0;
  // tiles of two sky points (single-unit interp): the sky vectors on the
  // host and the pair table
  double* sky_h = nullptr;              // pinned
  size_t sky_h_cap = 0;
  int2* pairs_d = nullptr;
  int2* pairs_h = nullptr;              // pinned
  size_t pairs_cap = 0;
  // semi-coherent calls: the geometry and A, B, C of every segment, and an
  // event pair per segment around its demodulation launches (seg_timed
  // pairs recorded by the last call)
  void* seg_arena = nullptr;
  size_t seg_arena_bytes = 0;
  std::vector<hipEvent_t> seg_ev;
  int seg_timed = 0;
  // the sky array whose host copy the geometry pass's wait brought into
  // sky_h (stage_sky), for the pairing that follows it in the same call
  const void* sky_staged = nullptr;
  // the band order of the last sky grid paired, kept while the sky vectors
  // stay the same (time segments, repeated calls on one grid)
  std::vector<double> ord_sky;
  std::vector<int64_t> ord_idx;
  hipStream_t cap_stream = nullptr;
  // persistent grids of the batch kernels with split_nfd(c % kSplitSizes)
  // spindowns and 1 + c / kSplitSizes sky points per tile, with [c][1] and
  // without [c][0] the global-memory fallback
  int batch_grid[2 * fstat::kSplitSizes][2] = {};
  std::map<std::vector<int64_t>, hipGraphExec_t> graphs;
  // fault injection (host-side forcing of error paths); force_seg > 0 runs the
  // interp kernels without the global-memory path at that slice width
  long fail_malloc_at = -1, fail_launch_at = -1;
  long n_malloc = 0, n_launch = 0;
  int force_seg = 0;
  // the demodulation's count of tiles that met an SFT outside their slice, copied to status_h
  // (single unit) or bstat_h[0, drop_units) (batched) after each call and
  // checked when the next call starts
  hipEvent_t ev_drop = nullptr;
  bool drop_pending = false;
  int drop_units = 0;
};

namespace {

int set_err(fstat_plan* p, int code, const char* fmt, ...) {
  if (p) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(p->err, sizeof p->err, fmt, ap);
    va_end(ap);
  }
  return code;
}

int hip_err(fstat_plan* p, hipError_t e, const char* what) {
  return set_err(p, FSTAT_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// The Nth allocation / launch fails when FSTAT_FAULT="malloc:N" / "launch:N".
void read_fault_env(fstat_plan* p) {
  const char* e = getenv("FSTAT_FAULT");
  if (!e) return;
  long n = 0;
  if (sscanf(e, "malloc:%ld", &n) == 1) p->fail_malloc_at = n;
  if (sscanf(e, "launch:%ld", &n) == 1) p->fail_launch_at = n;
  if (sscanf(e, "narrow:%ld", &n) == 1 && n >= 8 && n <= 4096) p->force_seg = (int)(n & ~3L);
}


int dev_alloc(fstat_plan* p, void** ptr, size_t* have, size_t need, const char* what) {
  if (*have >= need && *ptr) return FSTAT_OK;
  if (++p->n_malloc == p->fail_malloc_at) return set_err(p, FSTAT_E_NOMEM, "%s: injected allocation failure", what);
  if (*ptr) {
    (void)hipDeviceSynchronize();
    (void)hipFree(*ptr);
    *ptr = nullptr;
    *have = 0;
  }
  hipError_t e = hipMalloc(ptr, need);
  if (e != hipSuccess) {
    *ptr = nullptr;
    (void)hipGetLastError();
    return set_err(p, FSTAT_E_NOMEM, "%s: hipMalloc(%zu) failed: %s", what, need, hipGetErrorString(e));
  }
  *have = need;
  return FSTAT_OK;
}

int check_launch(fstat_plan* p, hipError_t e, const char* what) {
  if (++p->n_launch == p->fail_launch_at) return set_err(p, FSTAT_E_DEVICE, "%s: injected launch failure", what);
  if (e != hipSuccess) return hip_err(p, e, what);
  return FSTAT_OK;
}

// The previous call's tiles that met an SFT outside their slice, once the copy has landed:
// an error naming them (their templates' outputs are NaN), else FSTAT_OK.
int check_prev_drops(fstat_plan* p) {
  if (!p->drop_pending) return FSTAT_OK;
  p->drop_pending = false;
  if (hipEventSynchronize(p->ev_drop) != hipSuccess) return set_err(p, FSTAT_E_DEVICE, "previous call did not complete");
  unsigned long long n = 0;
  int unit = -1;
  if (p->drop_units == 0) {
    n = p->status_h->dropped;
  } else {
    for (int k = 0; k < p->drop_units; ++k)
      if (p->bstat_h[k].dropped) {
        n += p->bstat_h[k].dropped;
        if (unit < 0) unit = k;
      }
  }
  if (n == 0) return FSTAT_OK;
  if (unit >= 0)
    return set_err(p, FSTAT_E_DEVICE,
                   "the previous call met %llu tiles with an SFT whose windows were outside the LDS slice, first in "
                   "work unit %d; the outputs of those tiles are NaN",
                   n, unit);
  return set_err(p, FSTAT_E_DEVICE,
                 "the previous call met %llu tiles with an SFT whose windows were outside the LDS slice; the "
                 "outputs of those tiles are NaN",
                 n);
}

// Copies the drop count(s) of this call's demodulation to the host, to be
// checked when the next call starts.
void queue_drop_check(fstat_plan* p, fstat::GeoStatus* src_d, fstat::GeoStatus* dst_h, int n_units, hipStream_t st) {
  const size_t n = n_units > 0 ? (size_t)n_units : 1;
  if (hipMemcpyAsync(dst_h, src_d, n * sizeof(fstat::GeoStatus), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipEventRecord(p->ev_drop, st) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  p->drop_pending = true;
  p->drop_units = n_units;
}

// Resets the drop counter of a single-unit call.
int reset_drops(fstat_plan* p, fstat::GeoStatus* status_d, hipStream_t st) {
  return check_launch(p, fstat::launch_fill_int((int*)&status_d->dropped, 0, 2, st), "status reset");
}

bool finite(double x) { return std::isfinite(x); }

int validate_wu(fstat_plan* p, const fstat_wu* w, const fstat_out* o, int idx) {
  const fstat_desc& d = p->d;
  char tag[32] = "";
  if (idx >= 0) snprintf(tag, sizeof tag, "work unit %d: ", idx);
  if (!w || !o) return set_err(p, FSTAT_E_ARG, "%snull work unit or output", tag);
  if (!w->sft || !w->t_start || !w->pos || !w->vel || !w->sky || !w->a || !w->b)
    return set_err(p, FSTAT_E_ARG, "%snull input array", tag);
  if (d.storage != FSTAT_STORAGE_C64 && !w->sft_scale)
    return set_err(p, FSTAT_E_ARG, "%s16-bit storage needs sft_scale", tag);
  if (o->top_k < 0) return set_err(p, FSTAT_E_ARG, "%snegative top_k", tag);
  if (!o->twoF && o->top_k == 0) return set_err(p, FSTAT_E_ARG, "%snull twoF output and no toplist", tag);
  if (o->top_k > 0 && (!o->top || !o->n_above)) return set_err(p, FSTAT_E_ARG, "%stoplist needs top and n_above", tag);
  if (o->top_k > p->cand_cap)
    return set_err(p, FSTAT_E_SIZE, "%stop_k %d exceeds the candidate capacity %lld", tag, o->top_k,
                   (long long)p->cand_cap);
  if (o->top_k > 0 && !std::isfinite(o->threshold))
    return set_err(p, FSTAT_E_ARG, "%snon-finite toplist threshold", tag);
  if (w->n_det < 1) return set_err(p, FSTAT_E_ARG, "%sn_det < 1", tag);
  if (w->det_offset) {               // detector blocks of the flat SFT array
    if (w->det_offset[0] != 0 || w->det_offset[w->n_det] != w->n_sft)
      return set_err(p, FSTAT_E_ARG, "%sdet_offset must run from 0 to n_sft", tag);
    for (int d = 0; d < w->n_det; ++d)
      if (w->det_offset[d + 1] < w->det_offset[d])
        return set_err(p, FSTAT_E_ARG, "%sdet_offset decreases at detector %d", tag, d);
  }
  if (w->dterms < 1 || w->dterms > d.max_dterms) return set_err(p, FSTAT_E_ARG, "%sdterms %d outside [1, %d]", tag, w->dterms, d.max_dterms);
  if (w->n_sft < 1 || w->n_bins < 1 || w->n_sky < 1 || w->n_f < 1 || w->n_fd < 1)
    return set_err(p, FSTAT_E_ARG, "%ssizes must be >= 1", tag);
  if (w->n_sft > d.max_sft || w->n_bins > d.max_bins || w->n_sky > d.max_sky || w->n_f > d.max_f || w->n_fd > d.max_fd)
    return set_err(p, FSTAT_E_SIZE, "%ssize exceeds the plan maxima", tag);
  if (w->n_bins < 2 * (int64_t)w->dterms) return set_err(p, FSTAT_E_BAND, "%sband narrower than the 2D-bin window", tag);
  if (!(w->t_sft > 0) || !finite(w->t_sft) || !(w->df > 0) || !finite(w->df) || !(w->f0 > 0) || !finite(w->f0) ||
      !finite(w->fdot0) || !finite(w->dfdot) || !finite(w->t_ref))
    return set_err(p, FSTAT_E_ARG, "%snon-finite or non-positive grid parameter", tag);
  if (w->k_first < 0 || w->k_first + w->n_bins > 0x7fffffffLL)
    return set_err(p, FSTAT_E_BAND, "%sband outside [0, 2^31)", tag);
  if (w->n_sky * w->n_fd * w->n_f > ((int64_t)1 << 40)) return set_err(p, FSTAT_E_SIZE, "%stoo many templates", tag);
  // the interp kernel addresses one SFT's coefficients with 32-bit offsets
  if (w->n_bins > ((int64_t)1 << 25)) return set_err(p, FSTAT_E_SIZE, "%sband wider than 2^25 bins", tag);
  return FSTAT_OK;
}

WuDev make_dev(const fstat_plan* p, const fstat_wu* w, const fstat_out* o) {
  WuDev v{};
  v.sft = w->sft;
  v.scale = w->sft_scale;
  v.t_start = w->t_start;
  v.pos = w->pos;
  v.vel = w->vel;
  v.sky = w->sky;
  v.a = w->a;
  v.b = w->b;
  v.geo = (double2*)p->geo;
  v.abcd = (double4*)p->abcd;
  v.twoF = o ? o->twoF : nullptr;
  v.fa = o ? (float2*)o->fa : nullptr;
  v.fb = o ? (float2*)o->fb : nullptr;
  v.coef = (float4*)p->coef;
  v.acc = (float4*)p->acc;
  auto it = p->ctab.find(w->dterms);
  v.ctab = it != p->ctab.end() ? it->second : nullptr;
  auto is = p->csum.find(w->dterms);
  v.csum = is != p->csum.end() ? is->second : 0.0;
  v.coef16 = (p->d.flags & FSTAT_FLAG_COEF16) ? 1 : 0;
  v.cexp = (int32_t*)p->cexp;
  v.dropped = p->status_d ? &p->status_d->dropped : nullptr;
  v.cand = nullptr;
  v.cand_count = nullptr;
  v.cand_cap = p->cand_cap;
  v.top_k = 0;
  v.top = nullptr;
  v.n_above = nullptr;
  v.threshold = 0.f;
  if (o && o->top_k > 0) {
    v.cand = (uint4*)p->cand;
    v.cand_count = (unsigned long long*)p->cand_count;
    v.top_k = o->top_k;
    v.top = (int4*)o->top;
    v.n_above = o->n_above;
    v.threshold = o->threshold;
  }
  v.n_sft = w->n_sft;
  v.n_bins = w->n_bins;
  v.k_first = w->k_first;
  v.n_sky = w->n_sky;
  v.n_f = w->n_f;
  v.n_fd = w->n_fd;
  v.t_sft = w->t_sft;
  v.f0 = w->f0;
  v.df = w->df;
  v.fdot0 = w->fdot0;
  v.dfdot = w->dfdot;
  v.t_ref = w->t_ref;
  v.dterms = w->dterms;
  v.storage = p->d.storage;
  v.phase_mode = p->d.phase_mode;
  return v;
}

// Coefficient scratch of one work unit: [n_sft][rows][n_bins] 16-byte
// elements (4 rows of FP32 pairs, or 2 rows of FP16 quadruples), plus one
// slice row of padding that the staging of the last SFT may read (into
// columns it never uses).
bool coef16(const fstat_plan* p) { return (p->d.flags & FSTAT_FLAG_COEF16) != 0; }

size_t coef_bytes(const fstat_plan* p, const fstat_wu* w) {
  const size_t rows = coef16(p) ? fstat::kRows16 : fstat::kCoefPairs;
  const size_t pad = fstat::kSegMax > fstat::kSegMax16 ? fstat::kSegMax : fstat::kSegMax16;
  return ((size_t)w->n_sft * w->n_bins * rows + pad) * sizeof(float4);
}

int resolved_kernel(const fstat_plan* p) {
  return p->d.kernel == FSTAT_KERNEL_DIRECT ? fstat::KERNEL_DIRECT : fstat::KERNEL_INTERP;
}

double host_sinc(double x) { return x == 0.0 ? 1.0 : sin(M_PI * x) / (M_PI * x); }

// Monomial coefficients in kappa of the degree-(kCoef-1) Chebyshev
// projection of sinc(kappa + m) on kappa in [0, 1], for m = -D .. D-1:
// Chebyshev coefficients from 64 Chebyshev nodes (discrete cosine sums), the
// three-term recurrence T_{j+1} = 2u T_j - T_{j-1} to monomials of
// u = 2 kappa - 1, then the binomial expansion of (2 kappa - 1)^q, or, for
// the FP16 form (centred), monomials of v = kappa - 1/2 = u / 2: its
// polynomials are evaluated in FP16, where |v| <= 1/2 rounds to half the
// absolute error of kappa and the centred basis has the smaller coefficient
// sums.
std::vector<double> sinc_poly_table(int D, bool centred) {
  const int N = 64, P = fstat::kCoef;
  std::vector<double> tab((size_t)2 * D * P, 0.0);
  std::vector<std::vector<double>> Tm(P, std::vector<double>(P, 0.0));
  Tm[0][0] = 1.0;
  if (P > 1) Tm[1][1] = 1.0;
  for (int j = 1; j + 1 < P; ++j)
    for (int q = 0; q < P; ++q) Tm[j + 1][q] = (q > 0 ? 2.0 * Tm[j][q - 1] : 0.0) - Tm[j - 1][q];
  for (int m = -D; m < D; ++m) {
    std::vector<double> a(P, 0.0);
    for (int j = 0; j < P; ++j) {
      double acc = 0.0;
      for (int k = 0; k < N; ++k) {
        const double th = M_PI * (k + 0.5) / N;
        const double kap = 0.5 * (cos(th) + 1.0);
        acc += host_sinc(kap + m) * cos(j * th);
      }
      a[j] = (j == 0 ? 1.0 : 2.0) * acc / N;
    }
    std::vector<double> cu(P, 0.0);
    for (int j = 0; j < P; ++j)
      for (int q = 0; q < P; ++q) cu[q] += a[j] * Tm[j][q];
    double* row = &tab[(size_t)(m + D) * P];
    if (centred) {                    // cu[q] u^q = cu[q] 2^q v^q
      for (int q = 0; q < P; ++q) row[q] = cu[q] * ldexp(1.0, q);
      continue;
    }
    for (int q = 0; q < P; ++q) {     // cu[q] (2 kappa - 1)^q = cu[q] sum_r C(q,r) 2^r kappa^r (-1)^(q-r)
      double binom = 1.0;
      for (int r = 0; r <= q; ++r) {
        row[r] += cu[q] * binom * ldexp(1.0, r) * (((q - r) & 1) ? -1.0 : 1.0);
        binom = binom * (q - r) / (r + 1);
      }
    }
  }
  return tab;
}

int ensure_ctab(fstat_plan* p, int D) {
  if (p->ctab.count(D)) return FSTAT_OK;
  std::vector<double> tab = sinc_poly_table(D, coef16(p));
  void* d = nullptr;
  size_t have = 0;
  int rc = dev_alloc(p, &d, &have, tab.size() * sizeof(double), "polynomial table");
  if (rc) return rc;
  hipError_t e = hipMemcpy(d, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return hip_err(p, e, "polynomial table upload");
  }
  p->ctab[D] = (double*)d;
  double mx = 0.0;                       // bound on |c_p| / max|x| for the FP16 form's scale
  for (int q = 0; q < fstat::kCoef; ++q) {
    double sum = 0.0;
    for (int m = 0; m < 2 * D; ++m) sum += fabs(tab[(size_t)m * fstat::kCoef + q]);
    mx = sum > mx ? sum : mx;
  }
  p->csum[D] = mx;
  return FSTAT_OK;
}

// ------------------------------------------------ static scratch (no alloc)
// fstat_compute_noalloc keeps all its device memory in one static device
// array per GPU (fstat_kernels.hip).  Once per device, with that device
// current, the array's device address is taken (the host-side name of the
// array is not a device address and is never used) and the polynomial
// tables of every Dterms, in both bases, are copied to its start.
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
char* g_static_base[kMaxDevices] = {};
int g_static_state[kMaxDevices] = {};                    // 0: not set up, 1: ready, -1: failed
size_t g_tab_off[2][fstat::kMaxDterms + 1] = {};         // byte offset of the table of [centred][D]
double g_tab_csum[2][fstat::kMaxDterms + 1] = {};        // its max_p sum_m |t[m][p]|

void static_setup(int dev) {
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (dev < 0 || dev >= kMaxDevices || g_static_state[dev] != 0) return;
  g_static_state[dev] = -1;
  void* base = nullptr;
  if (fstat::static_scratch_address(&base) != hipSuccess || !base) {
    (void)hipGetLastError();
    return;
  }
  std::vector<double> all;
  for (int c = 0; c < 2; ++c)
    for (int D = 1; D <= fstat::kMaxDterms; ++D) {
      const std::vector<double> tab = sinc_poly_table(D, c == 1);
      g_tab_off[c][D] = all.size() * sizeof(double);
      double mx = 0.0;
      for (int q = 0; q < fstat::kCoef; ++q) {
        double sum = 0.0;
        for (int m = 0; m < 2 * D; ++m) sum += fabs(tab[(size_t)m * fstat::kCoef + q]);
        mx = sum > mx ? sum : mx;
      }
      g_tab_csum[c][D] = mx;
      all.insert(all.end(), tab.begin(), tab.end());
    }
  static_assert(2 * 16 * (64 * 65 / 2) * sizeof(double) <= fstat::kStaticTabBytes, "tables fit their region");
  if (hipMemcpy(base, all.data(), all.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  g_static_base[dev] = (char*)base;
  g_static_state[dev] = 1;
}

std::string class_key(const fstat_plan* p, const fstat_wu* w) {
  char b[64];
  snprintf(b, sizeof b, "s%d_d%d_k%d_c%d", p->d.storage, w->dterms, p->d.kernel, coef16(p) ? 1 : 0);
  return b;
}

// LDS slice width (bins) of the interp kernel: the NT frequency templates of
// a work-group span (NT-1) df T Tdot bins, the spindowns of a block shift k*
// by up to |dfdot| (NFD-1) max|tau| T Tdot more; plus slack, rounded to 4.
// Lanes whose window falls outside the slice read their coefficients from
// global memory instead, so a narrower slice costs speed, not correctness;
// the slice is capped at the LDS row length: NT + NT / 8 + 8 bins (296 for
// 256 threads: 37 KB of LDS, double-buffered) or 3 NT / 2 bins with FP16
// coefficients (384: 24 KB).
//
// With max_p = max Tdot T of the geometry pass, D-hat-phi varies over a tile
// by at most `spread` bins, so k* by at most spread + 1; the slice starts one
// bin below the tile's lowest k* and every window lies in it when
// W >= spread + 3.  W >= spread + 4 here whenever the cap did not bind, and
// *fits reports that: the kernel without the global-memory fallback may run.
int interp_seg_tau(const fstat_wu* w, int nfd, int threads, bool c16, double max_abs_tau, double max_p,
                   bool* fits) {
  const double nt = threads;
  const double spread = ((nt - 1.0) * w->df + fabs(w->dfdot) * (nfd - 1) * max_abs_tau) * max_p;
  const double width = nt + 6.0 + ceil(spread - (nt - 1.0) > 0 ? spread - (nt - 1.0) : 0.0);
  const int cap = fstat::interp_max_seg(threads, c16);
  if (fits) *fits = std::isfinite(width) && width <= cap;
  int W = !(width <= cap) ? cap : (int)width;
  return W & ~3;
}

int interp_seg(const fstat_plan* p, const fstat_wu* w, int nfd, int threads, bool* fits) {
  return interp_seg_tau(w, nfd, threads, coef16(p), p->max_abs_tau, p->max_p, fits);
}

Tile default_tile(const fstat_plan* p, const fstat_wu* w) {
  if (resolved_kernel(p) == fstat::KERNEL_INTERP) {
    // 3 or more spindowns: tiles of 8 per thread, which complete_tile splits
    // into blocks of 16 and 4 to 8 (split_spindowns; 3 or 4 spindowns: one
    // block of 4, which may take tiles of two sky points)
    const int nfd = w->n_fd >= 3 ? 8 : (w->n_fd >= 2 ? 2 : 1);
    // measured on the work-unit-shaped case: 8 spindowns per thread with room
    // for 4 waves per SIMD (5 with FP16 coefficients, whose slices and packed
    // FP16 polynomials take fewer registers and less LDS) is fastest.  Splitting the SFT loop into launches
    // keeps the resident work-groups on nearby SFTs, so their slices stay in
    // L2: with FP32 coefficients launches of 512 SFTs took the case from 125.1
    // to 122.7 ms (L2 hit rate 0.62 -> 0.91); with fewer spindowns per thread
    // the staged slices are reused less and shorter launches pay more
    // (with tiles of two sky points, which use each staged slice for twice the
    // pairs, one launch over all SFTs is fastest: 114.7 against 115.6 ms on
    // that case; prepare_pairs sets it)
    const int minw = nfd == 8 ? (coef16(p) ? 5 : 4) : 3;
    const int sb = nfd < 4 ? 256 : (nfd == 8 && !coef16(p) && w->n_sft > 1024 ? 512 : 0);
    return Tile{nfd, minw, 0, sb, fstat::kThreads};
  }
  return Tile{4, 4, 0, 0, 0};   // fastest direct tile on the work-unit-shaped case
}

// The spindowns of one unit (single or batched) as blocks of b per thread,
// b from the allowed sizes (bit b of `sizes`, b = 16 or 4 <= b <= 8): n[i]
// spindowns run split_nfd(i) per thread, as consecutive ranges (largest
// blocks first), each range's last block possibly partial.  The split
// minimises the lanes computed weighted by the time per lane of each block
// size (more spindowns per thread use each staged slice and each thread's
// per-SFT work for more pairs).  Measured on the work-unit-shaped case,
// relative to 8 per thread with one sky point per tile: with one sky point,
// on the batched kernel with 840 (832 for 16) spindowns, every size dividing
// it, identical outputs: 16: 0.890, 8: 1, 7: 1.072, 6: 1.136, 5: 1.259, 4:
// 1.415; with tiles of two sky points (`paired`, the ranges of at most 8),
// single-unit calls of 2000 sky points with that many spindowns: 8: 0.967,
// 7: 0.996, 6: 1.034, 5: 1.093, 4: 1.102.  So without pairs 5 spindowns run
// as one block of 5 rather than a partial 8, 12 as 6 + 6 rather than 8 + 4,
// 32 as 16 + 16 and 13 as one partial block of 16; with pairs 13 runs as
// 7 + 6.  All but the last two to three blocks' worth run in blocks of the
// largest allowed size (the cheapest per lane); the tail is split exactly by
// dynamic programming.
struct FdSplit {
  int64_t n[fstat::kSplitSizes] = {};
};

int split_index(int b) { return b == 16 ? 0 : 9 - b; }

FdSplit split_spindowns(int64_t nf, unsigned sizes, bool paired = false) {
  static const double kOne[17] = {0.0, 0.0, 0.0, 0.0, 1.415, 1.259, 1.136, 1.072, 1.0,
                                  0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.890};
  static const double kPaired[17] = {0.0, 0.0, 0.0, 0.0, 1.102, 1.093, 1.034, 0.996, 0.967,
                                     0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.890};
  const double* kLaneCost = paired ? kPaired : kOne;
  static const int kSizes[] = {16, 8, 7, 6, 5, 4};   // larger blocks first: ties take fewer tiles
  constexpr int kTail = 48;
  FdSplit r;
  int bmax = 0;
  for (int b : kSizes) {
    if ((sizes >> b) & 1u) {
      bmax = b;
      break;
    }
  }
  if (nf <= 0 || !bmax) return r;
  const int64_t head = nf > 3 * bmax ? ((nf - 2 * bmax) / bmax) * bmax : 0;
  const int t = (int)(nf - head);                 // at most 3 bmax <= kTail
  double best[kTail + 1];
  int pick[kTail + 1];
  best[0] = 0.0;
  pick[0] = 0;
  for (int x = 1; x <= t; ++x) {
    best[x] = HUGE_VAL;
    pick[x] = bmax;
    for (int b : kSizes) {
      if (!((sizes >> b) & 1u)) continue;
      const double c = best[x > b ? x - b : 0] + b * kLaneCost[b];
      if (c < best[x]) {
        best[x] = c;
        pick[x] = b;
      }
    }
  }
  r.n[split_index(bmax)] = head;
  for (int x = t; x > 0;) {
    const int b = pick[x], take = x > b ? b : x;
    r.n[split_index(b)] += take;
    x -= take;
  }
  return r;
}

// Block sizes (bit b: b spindowns per thread) with kernels for every
// block size of the split: 16 and 4 to 8.
constexpr unsigned kAllSplitSizes = (1u << 16) | 0x1F0u;

// Block sizes a single-unit tile of 8 spindowns per thread may split a unit's
// spindowns into: 16 and 4 to 8 for the 256-thread FP32-coefficient tile
// with four waves per SIMD (the sizes with kernels of that shape), else 8
// and 4; 0 for other tiles (one range).
unsigned single_sizes(const fstat_plan* p, const Tile& t) {
  if (t.nf_reg != 8) return 0u;
  if (!coef16(p) && t.threads == fstat::kThreads && t.chunk >= 4) return kAllSplitSizes;
  return (1u << 8) | (1u << 4);
}

// Slice widths of a tile for this work unit, its spindown split
// (split_spindowns, when it is anything but one range of nf_reg per thread,
// with the costs of paired tiles if `paired`) and whether the variant
// without the global-memory path may run.
Tile complete_tile(const fstat_plan* p, const fstat_wu* w, Tile t, bool paired = false) {
  if (resolved_kernel(p) == fstat::KERNEL_INTERP) {
    bool fits = false;
    t.seg = interp_seg(p, w, t.nf_reg, t.threads, &fits);
    t.fast = fits;
    for (int i = 0; i < fstat::kSplitSizes; ++i) t.fd_split[i] = t.seg_split[i] = 0;
    unsigned sizes = single_sizes(p, t);
    if ((sizes >> 16) & 1u) {         // 16 per thread only where its wider slice holds every window
      bool f16 = false;
      (void)interp_seg(p, w, 16, t.threads, &f16);
      if (!f16) sizes &= ~(1u << 16);
    }
    const FdSplit sp = split_spindowns(w->n_fd, sizes, paired);
    if (sizes && sp.n[split_index(8)] != w->n_fd) {
      t.fast = 1;
      for (int i = 0; i < fstat::kSplitSizes; ++i) {
        if (sp.n[i] <= 0) continue;
        bool f = false;
        t.fd_split[i] = (int32_t)sp.n[i];
        t.seg_split[i] = interp_seg(p, w, fstat::split_nfd(i), t.threads, &f);
        t.fast = t.fast && f;
      }
    }
    if (p->force_seg > 0) {          // fault injection: a slice narrower than the windows need
      t.seg = p->force_seg;
      for (int i = 0; i < fstat::kSplitSizes; ++i) t.seg_split[i] = t.fd_split[i] > 0 ? p->force_seg : 0;
      t.fast = 1;
    }
  }
  return t;
}

Tile pick_tile(const fstat_plan* p, const fstat_wu* w, bool* is_default = nullptr) {
  auto it = p->tiles.find(class_key(p, w));
  if (is_default) *is_default = it == p->tiles.end();
  return complete_tile(p, w, it != p->tiles.end() ? it->second : default_tile(p, w));
}

int ensure_toplist(fstat_plan* p, const fstat_out* o) {
  if (!o || o->top_k <= 0) return FSTAT_OK;
  int rc = dev_alloc(p, &p->cand, &p->cand_bytes, (size_t)p->cand_cap * sizeof(uint4), "toplist candidates");
  if (rc) return rc;
  return dev_alloc(p, &p->cand_count, &p->cand_count_bytes, 64, "toplist counter");
}

int ensure_scratch(fstat_plan* p, const fstat_wu* w) {
  int rc = dev_alloc(p, &p->geo, &p->geo_bytes, (size_t)w->n_sky * w->n_sft * sizeof(double2), "geometry scratch");
  if (rc) return rc;
  rc = dev_alloc(p, &p->abcd, &p->abcd_bytes, (size_t)w->n_sky * sizeof(double4), "A,B,C scratch");
  if (rc) return rc;
  if (resolved_kernel(p) == fstat::KERNEL_INTERP) {
    rc = dev_alloc(p, &p->coef, &p->coef_bytes, coef_bytes(p, w), "coefficient scratch");
    if (rc) return rc;
    if (coef16(p)) {
      rc = dev_alloc(p, &p->cexp, &p->cexp_bytes, (size_t)w->n_sft * sizeof(int32_t), "coefficient exponents");
      if (rc) return rc;
    }
    rc = dev_alloc(p, &p->acc, &p->acc_bytes, (size_t)w->n_sky * w->n_fd * w->n_f * sizeof(float4),
                   "accumulator scratch");
    if (rc) return rc;
    rc = ensure_ctab(p, w->dterms);
  }
  return rc;
}

int stage_sky(fstat_plan* p, const fstat_wu* wu, hipStream_t st);

// Geometry + band check into the status record status_d; waits for the
// check.  With `stage` (a unit whose sky points may be paired) the host copy
// of its sky vectors rides on the same wait.  Returns FSTAT_OK or an error.
int run_geometry_at(fstat_plan* p, const WuDev& v, fstat::GeoStatus* status_d, hipStream_t st, int idx,
                    const fstat_wu* stage = nullptr) {
  p->sky_staged = nullptr;
  int rc = check_launch(p, fstat::launch_fill_int((int*)status_d, 0, fstat::kGeoResetInts, st), "status reset");
  if (rc) return rc;
  rc = check_launch(p, fstat::launch_geometry(v, status_d, st), "geometry kernel");
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(p->status_h, status_d, sizeof(fstat::GeoStatus), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return hip_err(p, e, "status copy");
  if (stage) {
    rc = stage_sky(p, stage, st);
    if (rc) return rc;
  }
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_err(p, e, "geometry kernel");
  const int st_bits = p->status_h->flags;
  unsigned long long tb = p->status_h->max_abs_tau_bits;
  memcpy(&p->max_abs_tau, &tb, sizeof tb);
  tb = p->status_h->max_p_bits;
  memcpy(&p->max_p, &tb, sizeof tb);
  char tag[32] = "";
  if (idx >= 0) snprintf(tag, sizeof tag, "work unit %d: ", idx);
  if (st_bits & 1) return set_err(p, FSTAT_E_BAND, "%sa Dirichlet window [k*-D+1, k*+D] leaves the stored band", tag);
  if (st_bits & 2) return set_err(p, FSTAT_E_ARG, "%santenna-pattern matrix is singular (A B - C^2 <= 0)", tag);
  return FSTAT_OK;
}

int run_geometry(fstat_plan* p, const WuDev& v, hipStream_t st, int idx, const fstat_wu* stage = nullptr) {
  return run_geometry_at(p, v, p->status_d, st, idx, stage);
}

// `e0`, `e1`: the events around the demodulation launches (default: the
// plan's ev0, ev1, which fstat_last_kernel_ms reads).
int run_demod(fstat_plan* p, const WuDev& v, const Tile& t, hipStream_t st, hipEvent_t e0 = nullptr,
              hipEvent_t e1 = nullptr) {
  const int kernel = resolved_kernel(p);
  p->have_last = true;
  p->last_tile = t;
  p->last_sky_tiles = v.n_pairs > 0 && t.pair_seg > 0 ? v.n_pairs : v.n_sky;
  if (kernel == fstat::KERNEL_INTERP) {
    if (v.coef16) {
      int rc = check_launch(p, fstat::launch_cexp(v, st), "coefficient exponent kernel");
      if (rc) return rc;
    }
    int rc = check_launch(p, fstat::launch_coef(v, st), "coefficient kernel");
    if (rc) return rc;
  }
  if (v.cand) {
    int rc = check_launch(p, fstat::launch_fill_int((int*)v.cand_count, 0, 2, st), "toplist counter reset");
    if (rc) return rc;
  }
  const bool own = e0 == nullptr;
  (void)hipEventRecord(own ? p->ev0 : e0, st);
  int rc = check_launch(p, fstat::launch_demod(v, t, kernel, st), "demodulation kernel");
  (void)hipEventRecord(own ? p->ev1 : e1, st);
  p->ev_stream = st;
  if (own) p->timed = (rc == FSTAT_OK);
  if (rc == FSTAT_OK && v.cand) rc = check_launch(p, fstat::launch_top_select(v, st), "toplist selection");
  return rc;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct WuScratch {
  size_t geo, abcd, coef, cexp, acc, total;
};

// Batched form: geometry, A,B,C,D, coefficients, FP16 exponents and, for a
// unit of more than one SFT block of `sblock` SFTs, Fa, Fb between the
// blocks' launches.
WuScratch wu_scratch(const fstat_plan* p, const fstat_wu* w, int64_t sblock) {
  WuScratch r;
  r.geo = align256((size_t)w->n_sky * w->n_sft * sizeof(double2));
  r.abcd = align256((size_t)w->n_sky * sizeof(double4));
  r.coef = align256(coef_bytes(p, w));
  r.cexp = coef16(p) ? align256((size_t)w->n_sft * sizeof(int32_t)) : 0;
  r.acc = w->n_sft > sblock ? align256((size_t)w->n_sky * w->n_fd * w->n_f * sizeof(float4)) : 0;
  r.total = r.geo + r.abcd + r.coef + r.cexp + r.acc;
  return r;
}

template <class T>
int ensure_pinned_pair(fstat_plan* p, T** dev, T** host, size_t* cap, size_t need, const char* what) {
  if (*cap >= need) return FSTAT_OK;
  (void)hipDeviceSynchronize();                    // earlier batches may still read the old table
  for (auto& kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
  p->graphs.clear();
  if (*dev) (void)hipFree(*dev);
  if (*host) (void)hipHostFree(*host);
  *dev = nullptr;
  *host = nullptr;
  *cap = 0;
  if (++p->n_malloc == p->fail_malloc_at) return set_err(p, FSTAT_E_NOMEM, "%s: injected allocation failure", what);
  if (hipMalloc((void**)dev, need * sizeof(T)) != hipSuccess ||
      hipHostMalloc((void**)host, need * sizeof(T), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return set_err(p, FSTAT_E_NOMEM, "%s: allocation of %zu entries failed", what, need);
  }
  *cap = need;
  return FSTAT_OK;
}

// Geometry and band check of work units [k0, k1) into their status slots,
// with the geometry written to `geo_base` (one work unit at a time).
int batch_check(fstat_plan* p, const fstat_wu* wus, const fstat_out* outs, int k0, int k1, char* geo_base,
                const std::vector<size_t>& offs, hipStream_t st) {
  for (int k = k0; k < k1; ++k) {
    WuDev v = make_dev(p, &wus[k], &outs[k]);
    const WuScratch sc = wu_scratch(p, &wus[k], 0);   // geometry and A,B,C,D come first either way
    v.geo = (double2*)(geo_base + offs[k]);
    v.abcd = (double4*)(geo_base + offs[k] + sc.geo);
    int rc = check_launch(p, fstat::launch_fill_int((int*)(p->bstat_d + k), 0, sizeof(fstat::GeoStatus) / sizeof(int), st),
                          "status reset");
    if (rc) return rc;
    rc = check_launch(p, fstat::launch_geometry(v, p->bstat_d + k, st), "geometry kernel");
    if (rc) return rc;
  }
  hipError_t e = hipMemcpyAsync(p->bstat_h + k0, p->bstat_d + k0, (size_t)(k1 - k0) * sizeof(fstat::GeoStatus),
                                hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return hip_err(p, e, "status copy");
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_err(p, e, "geometry kernel");
  for (int k = k0; k < k1; ++k) {
    const int f = p->bstat_h[k].flags;
    if (f & 1) return set_err(p, FSTAT_E_BAND, "work unit %d: a Dirichlet window [k*-D+1, k*+D] leaves the stored band", k);
    if (f & 2) return set_err(p, FSTAT_E_ARG, "work unit %d: antenna-pattern matrix is singular (A B - C^2 <= 0)", k);
  }
  return FSTAT_OK;
}

double status_tau(const fstat::GeoStatus& g) {
  double t;
  memcpy(&t, &g.max_abs_tau_bits, sizeof t);
  return t;
}

double status_p(const fstat::GeoStatus& g) {
  double t;
  memcpy(&t, &g.max_p_bits, sizeof t);
  return t;
}

double status_bits(unsigned long long b) {
  double t;
  memcpy(&t, &b, sizeof t);
  return t;
}

// Sky point indices in the order the pairing walks them: bands of z of the
// grid's spacing, alternately by increasing and decreasing longitude (ties by
// index).
void band_order(const double* sk, int64_t n, std::vector<int64_t>* ord) {
  const double h = sqrt(4.0 * M_PI / (double)n);           // grid spacing
  const int64_t n_band = std::max<int64_t>(1, (int64_t)ceil(2.0 / h));
  std::vector<std::pair<std::pair<int64_t, double>, int64_t>> key((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    const double z = sk[3 * i + 2], ph = atan2(sk[3 * i + 1], sk[3 * i]);
    int64_t b = (int64_t)floor((z + 1.0) / 2.0 * (double)n_band);
    b = b < 0 ? 0 : (b >= n_band ? n_band - 1 : b);
    key[(size_t)i] = {{b, (b & 1) ? -ph : ph}, i};
  }
  std::sort(key.begin(), key.end());
  ord->resize((size_t)n);
  for (int64_t i = 0; i < n; ++i) (*ord)[(size_t)i] = key[(size_t)i].second;
}

// Tiles of two sky points for the interp kernels' ranges of at most 8
// spindowns per thread: a tile evaluates (sky point, spindown) slots of both
// points per thread and SFT from one staged slice, which halves the slice
// loads per pair (and with them the L2 traffic that holds the clock down)
// and shares each thread's per-SFT work.  The slice must then hold the
// windows of both sky points: their bins differ by at most
//   |n0 - n1| (f_max T |v|max + |fdot|max (|tau|max T |v|max + P_max |r|max))
// (P = Tdot T = (1 + v.n) T and tau = t - t_ref + r.n, so P0 - P1 = T v.(n0 -
// n1) and tau0 - tau1 = r.(n0 - n1)), which is added to the spread of one
// sky point over min(n_fd, 8) spindowns (the widest such range).  Sky points
// are ordered in bands of z of the grid's spacing, alternately by
// increasing and decreasing longitude, and consecutive points are paired
// when the pair's slice still fits the LDS capacity.  The points this leaves
// alone (mostly at the ends of bands) are then paired among themselves: each
// with the nearest of the next 16 unpaired ones in the same order that fits.
// A point still without a partner forms a tile of its own sky point twice
// (computed twice, written once).  Tiles are written in the band order of
// their first point, so that consecutive tiles stay neighbours on the sky.
// Writes the n_pairs tiles to `out` (room for n_sky) and returns the slice
// width, or 0 when pairing does not apply (fewer than half the points find a
// partner, or no width fits).  `order` is the band_order of these sky
// vectors when the caller has it (else it is computed here).
int make_pairs(const fstat_wu* wu, const fstat::GeoStatus& g, const double* sk, int2* out, int64_t* n_pairs,
               const std::vector<int64_t>* order = nullptr) {
  *n_pairs = 0;
  const int64_t n = wu->n_sky;
  const int nt = fstat::kThreads, cap = fstat::interp_max_seg(nt, false);
  const double vmax = status_bits(g.max_v_bits), rmax = status_bits(g.max_r_bits);
  const double max_tau = status_bits(g.max_abs_tau_bits), max_p = status_bits(g.max_p_bits);
  const double f_max = std::max(fabs(wu->f0), fabs(wu->f0 + (double)(wu->n_f - 1) * wu->df));
  const double fd_max = std::max(fabs(wu->fdot0), fabs(wu->fdot0 + (double)(wu->n_fd - 1) * wu->dfdot));
  const double T = wu->t_sft;
  // bins per unit of |n0 - n1|
  const double C = f_max * T * vmax + fd_max * (max_tau * T * vmax + max_p * rmax);
  // the widest range of at most 8 spindowns per thread spans min(n_fd, 8) of them
  const double fd_span = (double)(std::min<int64_t>(wu->n_fd, 8) - 1);
  const double spread1 = ((nt - 1.0) * wu->df + fabs(wu->dfdot) * fd_span * max_tau) * max_p;
  const double over1 = spread1 - (nt - 1.0) > 0 ? spread1 - (nt - 1.0) : 0.0;
  // extra bins the pair may add with the width nt + 6 + ceil(over1 + extra) <= cap
  const double budget = (double)(cap - nt - 6) - over1 - 1.0;
  // (pair tables hold 32-bit sky indices)
  if (n < 4 || n > INT32_MAX || !std::isfinite(C) || !std::isfinite(budget) || budget < 1.0) return 0;
  const double d_max = C > 0.0 ? budget / C : 4.0;
  std::vector<int64_t> own;
  if (!order || (int64_t)order->size() != n) {
    band_order(sk, n, &own);
    order = &own;
  }
  const std::vector<int64_t>& key = *order;
  auto dist = [&](int64_t a, int64_t b) {
    const double dx = sk[3 * a] - sk[3 * b], dy = sk[3 * a + 1] - sk[3 * b + 1], dz = sk[3 * a + 2] - sk[3 * b + 2];
    return sqrt((dx * dx + dy * dy) + dz * dz);
  };
  int64_t np = 0, paired = 0;
  double worst = 0.0;
  std::vector<int64_t> partner((size_t)n, -1), left;
  for (int64_t q = 0; q < n;) {
    const int64_t a = key[(size_t)q];
    if (q + 1 < n) {
      const int64_t b = key[(size_t)q + 1];
      const double d = dist(a, b);
      if (d <= d_max) {
        partner[(size_t)a] = b;
        partner[(size_t)b] = a;
        worst = std::max(worst, d);
        paired += 2;
        q += 2;
        continue;
      }
    }
    left.push_back(a);
    ++q;
  }
  for (size_t i = 0; i < left.size(); ++i) {
    const int64_t a = left[i];
    if (partner[(size_t)a] >= 0) continue;
    int64_t best = -1;
    double bd = 0.0;
    for (size_t j = i + 1; j < left.size() && j <= i + 16; ++j) {
      const int64_t b = left[j];
      if (partner[(size_t)b] >= 0) continue;
      const double d = dist(a, b);
      if (d <= d_max && (best < 0 || d < bd)) {
        best = b;
        bd = d;
      }
    }
    if (best >= 0) {
      partner[(size_t)a] = best;
      partner[(size_t)best] = a;
      worst = std::max(worst, bd);
      paired += 2;
    }
  }
  std::vector<char> done((size_t)n, 0);
  for (int64_t q = 0; q < n; ++q) {
    const int64_t a = key[(size_t)q];
    if (done[(size_t)a]) continue;
    const int64_t b = partner[(size_t)a] >= 0 ? partner[(size_t)a] : a;
    done[(size_t)a] = done[(size_t)b] = 1;
    out[np++] = make_int2((int)a, (int)b);
  }
  const double width = nt + 6.0 + ceil(over1 + worst * C);
  if (2 * paired < n || !(width <= cap)) return 0;
  *n_pairs = np;
  return (int)width & ~3;
}

// Enqueues the host copy of the unit's sky vectors into sky_h (pinned, grown
// as needed) on st; sky_staged names the array once the stream has been
// waited for.
int stage_sky(fstat_plan* p, const fstat_wu* wu, hipStream_t st) {
  const int64_t n = wu->n_sky;
  p->sky_staged = nullptr;
  if (p->sky_h_cap < (size_t)(3 * n)) {
    if (p->sky_h) (void)hipHostFree(p->sky_h);
    p->sky_h = nullptr;
    p->sky_h_cap = 0;
    if (hipHostMalloc((void**)&p->sky_h, (size_t)(3 * n) * sizeof(double), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return set_err(p, FSTAT_E_NOMEM, "sky vectors: allocation of %lld entries failed", (long long)n);
    }
    p->sky_h_cap = (size_t)(3 * n);
  }
  const hipError_t e = hipMemcpyAsync(p->sky_h, wu->sky, (size_t)(3 * n) * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return hip_err(p, e, "sky vector copy");
  p->sky_staged = wu->sky;
  return FSTAT_OK;
}

// Whether a single-unit call on this plan may pair the unit's sky points
// (prepare_pairs decides once the tile is known).
bool may_pair(const fstat_plan* p, const fstat_wu* wu) {
  return resolved_kernel(p) == fstat::KERNEL_INTERP && !coef16(p) && wu->n_sky >= 4 && p->force_seg <= 0;
}

// Whether the tile's ranges of at most 8 spindowns may take tiles of two sky
// points: FP32 coefficients, 256 threads, four waves, 8 per thread.
bool pairs_apply(const fstat_plan* p, const fstat_wu* wu, const Tile& t) {
  return resolved_kernel(p) == fstat::KERNEL_INTERP && !coef16(p) && t.nf_reg == 8 && t.threads == fstat::kThreads &&
         t.chunk >= 4 && wu->n_sky >= 4 && p->force_seg <= 0;
}

// The pairing itself, from a host copy of the sky vectors and the unit's
// geometry status; the table goes to pairs_h and is uploaded to pairs_d
// (room for n_sky entries each).
int pair_sky(fstat_plan* p, const fstat_wu* wu, WuDev& v, Tile& t, hipStream_t st, bool default_tile_used,
             const fstat::GeoStatus& g, const double* sky, int2* pairs_h, int2* pairs_d) {
  const int64_t n = wu->n_sky;
  int64_t np = 0;
  if (n <= INT32_MAX &&
      (p->ord_sky.size() != (size_t)(3 * n) || memcmp(p->ord_sky.data(), sky, (size_t)(3 * n) * sizeof(double)))) {
    p->ord_sky.assign(sky, sky + 3 * n);
    band_order(sky, n, &p->ord_idx);
  }
  const int width = make_pairs(wu, g, sky, pairs_h, &np, &p->ord_idx);
  if (!width) return FSTAT_OK;
  // the split with the costs of paired tiles; pairs serve its ranges of at most 8
  const Tile tp = complete_tile(p, wu, t, true);
  bool small = std::all_of(tp.fd_split, tp.fd_split + fstat::kSplitSizes, [](int32_t x) { return x == 0; });
  for (int i = 0; i < fstat::kSplitSizes; ++i) small = small || (fstat::split_nfd(i) <= 8 && tp.fd_split[i] > 0);
  if (!small) return FSTAT_OK;
  const hipError_t e = hipMemcpyAsync(pairs_d, pairs_h, (size_t)np * sizeof(int2), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_err(p, e, "sky pair upload");
  v.sky_pairs = pairs_d;
  v.n_pairs = np;
  t = tp;
  t.pair_seg = width;
  if (default_tile_used) t.sblock = 0;   // the default tile: one launch over all SFTs with pairs
  return FSTAT_OK;
}

// Sky points of a single-unit tile of 8 spindowns per thread with ranges of
// at most 8 per thread (FP32 coefficients, 256 threads, four waves), paired
// by make_pairs after this unit's geometry pass; sets v.sky_pairs, v.n_pairs
// and t.pair_seg, or leaves one sky point per tile; with the default tile
// (`default_tile_used`) the SFT loop then runs in one launch.  Uses the sky
// vectors the geometry pass's wait brought (stage_sky), else copies them and
// waits for the stream (idle after the band check).
int prepare_pairs(fstat_plan* p, const fstat_wu* wu, WuDev& v, Tile& t, hipStream_t st, bool default_tile_used) {
  v.sky_pairs = nullptr;
  v.n_pairs = 0;
  t.pair_seg = 0;
  if (!pairs_apply(p, wu, t)) return FSTAT_OK;
  int rc = ensure_pinned_pair(p, &p->pairs_d, &p->pairs_h, &p->pairs_cap, (size_t)wu->n_sky, "sky pairs");
  if (rc) return rc;
  if (p->sky_staged != wu->sky) {          // not brought by this call's geometry wait
    rc = stage_sky(p, wu, st);
    if (rc) return rc;
    const hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_err(p, e, "sky vector copy");
  }
  p->sky_staged = nullptr;
  return pair_sky(p, wu, v, t, st, default_tile_used, *p->status_h, p->sky_h, p->pairs_h, p->pairs_d);
}

// Launch shape of the batched form (a Tile under the plan's batch class):
// nf_reg 8 runs each unit's spindowns in blocks of 4 to 8 per thread (8 or 4
// with FP16 coefficients) chosen by split_spindowns, nf_reg 4 runs all of
// them in blocks of 4; chunk = tiles per chunk of the per-XCD queues;
// sblock = SFTs per launch (0: all).
std::string batch_key(const fstat_plan* p) {
  char b[64];
  snprintf(b, sizeof b, "batch_s%d_c%d", p->d.storage, coef16(p) ? 1 : 0);
  return b;
}

bool valid_batch_tile(const Tile& t) {
  return (t.nf_reg == 8 || t.nf_reg == 4) && t.chunk >= 1 && t.chunk <= (1 << 20) && t.sblock >= 0 &&
         t.sblock <= (1 << 24) && t.threads == fstat::kThreads;
}

// Measured on 64 units of the 256-unit case: blocks of 8 spindowns, chunks of
// 256 tiles (L2 hit rate 0.88 against 0.62 for chunks of one tile, a third of
// the bytes fetched, 4 % faster), launches of 256 SFTs (1.5 % faster than 512).
Tile default_batch_tile() { return Tile{8, 256, 0, 256, fstat::kThreads, 0, 0}; }

Tile batch_tile(const fstat_plan* p) {
  auto it = p->tiles.find(batch_key(p));
  return it != p->tiles.end() ? it->second : default_batch_tile();
}

// Block sizes the batched form may use with this plan and launch shape.
unsigned batch_sizes(const fstat_plan* p, const Tile& bt) {
  if (bt.nf_reg == 4) return 1u << 4;
  return coef16(p) ? (1u << 8) | (1u << 4) : kAllSplitSizes;      // {8, 4} or 16, 4..8
}

// Per unit of a batched group (in launch order): its sky pairs (make_pairs,
// where `pairing` allows; width 0 = one sky point per tile, pair table at the
// unit's offset sky_off[k] of the plan's pair buffer, uploaded on `st`) and
// its spindown split with the costs of its tiles.  The sky vectors are read
// back in one wait for the group.
struct UnitShape {
  int pair_width = 0;
  int64_t n_pairs = 0;
  FdSplit split;
};

int batch_unit_shapes(fstat_plan* p, const fstat_wu* wus, const std::vector<int>& order, unsigned sizes, bool pairing,
                      const std::vector<int64_t>& sky_off, hipStream_t st, std::vector<UnitShape>* out) {
  const int m = (int)order.size();
  std::vector<UnitShape>& us = *out;
  us.assign(m, UnitShape{});
  if (pairing) {
    std::vector<int> cand;
    for (int q = 0; q < m; ++q) {
      const int k = order[q];
      if (wus[k].n_sky < 4) continue;
      hipError_t e = hipMemcpyAsync(p->sky_h + 3 * sky_off[k], wus[k].sky, (size_t)(3 * wus[k].n_sky) * sizeof(double),
                                    hipMemcpyDeviceToHost, st);
      if (e != hipSuccess) return hip_err(p, e, "sky vector copy");
      cand.push_back(q);
    }
    if (!cand.empty()) {
      hipError_t e = hipStreamSynchronize(st);
      if (e != hipSuccess) return hip_err(p, e, "sky vector copy");
      for (int q : cand) {
        const int k = order[q];
        us[q].pair_width =
            make_pairs(&wus[k], p->bstat_h[k], p->sky_h + 3 * sky_off[k], p->pairs_h + sky_off[k], &us[q].n_pairs);
        if (!us[q].pair_width) continue;
        e = hipMemcpyAsync(p->pairs_d + sky_off[k], p->pairs_h + sky_off[k], (size_t)us[q].n_pairs * sizeof(int2),
                           hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_err(p, e, "sky pair upload");
      }
    }
  }
  for (int q = 0; q < m; ++q) {
    const int k = order[q];
    unsigned sz = sizes;
    if ((sz >> 16) & 1u) {          // 16 per thread only where its wider slice holds every window
      bool f16 = false;
      (void)interp_seg_tau(&wus[k], 16, fstat::kThreads, coef16(p), status_tau(p->bstat_h[k]), status_p(p->bstat_h[k]),
                           &f16);
      if (!f16) sz &= ~(1u << 16);
    }
    us[q].split = split_spindowns(wus[k].n_fd, sz, us[q].pair_width > 0);
  }
  return FSTAT_OK;
}

// The demodulation tables of a batched group: table c = i + kSplitSizes
// (nsky - 1) holds the ranges run split_nfd(i) spindowns per thread with
// nsky sky points per tile, one entry per unit that has such a range (units
// most SFTs first), written to eh[m ...) after the group's m unit entries
// (whose device views they copy).  Per table: entries, first entry, tiles
// and whether every entry's slice holds its windows.  Returns the number of
// entries written in all (m included).
constexpr int kBatchTables = 2 * fstat::kSplitSizes;
struct BatchTables {
  int mc[kBatchTables] = {}, off[kBatchTables] = {};
  int64_t tiles[kBatchTables] = {};
  bool fast[kBatchTables] = {};
};

int batch_tables(const fstat_plan* p, const fstat_wu* wus, const std::vector<int>& order,
                 const std::vector<UnitShape>& us, const std::vector<int64_t>& sky_off, fstat::BatchEntry* eh,
                 BatchTables* tb) {
  constexpr int NS = fstat::kSplitSizes;
  const int m = (int)order.size();
  int ne = m;
  for (int c = 0; c < kBatchTables; ++c) {
    const int i = c % NS, nsky = 1 + c / NS, nfd = fstat::split_nfd(i);
    tb->off[c] = ne;
    tb->fast[c] = true;
    for (int q = 0; q < m; ++q) {
      const int k = order[q];
      const bool paired = us[q].pair_width > 0 && nfd <= 8;
      if ((nsky == 2) != paired) continue;
      int64_t lo = 0;
      for (int j = 0; j < i; ++j) lo += us[q].split.n[j];
      const int64_t hi = lo + us[q].split.n[i];
      if (hi <= lo) continue;
      fstat::BatchEntry& e = eh[ne++];
      e = eh[q];
      e.nfd = nfd;
      e.fd_begin = (int32_t)lo;
      e.fd_end = (int32_t)hi;
      bool fits = false;
      if (paired) {                    // the pair's width holds both points' windows by construction
        e.w.sky_pairs = p->pairs_d + sky_off[k];
        e.w.n_pairs = us[q].n_pairs;
        e.seg = us[q].pair_width;
        fits = true;
      } else {
        e.seg = interp_seg_tau(&wus[k], nfd, fstat::kThreads, coef16(p), status_tau(p->bstat_h[k]),
                               status_p(p->bstat_h[k]), &fits);
      }
      if (p->force_seg > 0) {          // fault injection: a slice narrower than the windows need
        e.seg = p->force_seg;
        fits = true;
      }
      e.fast = fits ? 1 : 0;
      tb->fast[c] = tb->fast[c] && fits;
      e.n_tiles = fstat::interp_tiles(e.w, nfd, lo, hi, nsky);
      e.tile_begin = tb->tiles[c];
      tb->tiles[c] += e.n_tiles;
      ++tb->mc[c];
    }
  }
  return ne;
}

// Batched interp path: work units are grouped so that one group's scratch
// (geometry, A,B,C, coefficients) fits the budget; per group the geometry is
// computed and checked, the work-unit table is uploaded, and the coefficient
// pass plus the persistent demodulation kernel run as one captured graph.
int batch_interp(fstat_plan* p, const fstat_wu* wus, int n, const fstat_out* outs, hipStream_t st) {
  const Tile bt = batch_tile(p);
  int64_t max_sft = 1;
  for (int k = 0; k < n; ++k) max_sft = wus[k].n_sft > max_sft ? wus[k].n_sft : max_sft;
  const int64_t B = bt.sblock > 0 ? bt.sblock : max_sft;    // SFTs per launch
  std::vector<size_t> offs(n);
  std::vector<std::pair<int, int>> groups;
  double budget_gb = 64.0;
  if (const char* e = getenv("FSTAT_BATCH_SCRATCH_GB")) budget_gb = atof(e) > 0 ? atof(e) : budget_gb;
  const size_t budget = (size_t)(budget_gb * 1073741824.0);
  size_t cur = 0, biggest = 0;
  int g0 = 0;
  for (int k = 0; k < n; ++k) {
    const size_t need = wu_scratch(p, &wus[k], B).total;
    if (cur > 0 && cur + need > budget) {
      groups.push_back({g0, k});
      g0 = k;
      cur = 0;
    }
    offs[k] = cur;
    cur += need;
    biggest = cur > biggest ? cur : biggest;
  }
  groups.push_back({g0, n});
  int rc = dev_alloc(p, &p->arena, &p->arena_bytes, biggest, "batch scratch");
  if (rc) return rc;
  rc = ensure_pinned_pair(p, &p->bstat_d, &p->bstat_h, &p->bstat_cap, (size_t)n, "batch status");
  if (rc) return rc;
  // per group: one entry per unit and up to one demodulation entry per unit
  // and table (block size, one or two sky points per tile)
  constexpr int NS = fstat::kSplitSizes, NC = kBatchTables;
  constexpr int kEnts = 1 + NC;
  rc = ensure_pinned_pair(p, &p->ents_d, &p->ents_h, &p->ents_cap, kEnts * (size_t)n, "work-unit table");
  if (rc) return rc;
  for (int k = 0; k < n; ++k) {
    rc = ensure_ctab(p, wus[k].dterms);
    if (rc) return rc;
  }
  if (!p->counter) {               // the per-XCD tile queues of the launch of each block size
    size_t have = 0;
    rc = dev_alloc(p, (void**)&p->counter, &have, NC * fstat::kXcds * sizeof(unsigned long long), "tile counters");
    if (rc) return rc;
  }
  bool any_top = false;
  for (int k = 0; k < n; ++k) any_top = any_top || outs[k].top_k > 0;
  if (any_top) {   // one candidate segment and counter per work unit
    const size_t cand_need = (size_t)n * p->cand_cap * sizeof(uint4);
    const size_t count_need = align256((size_t)n * sizeof(unsigned long long));
    if (p->bcand_bytes < cand_need || p->bcount_bytes < count_need) {
      // the captured graphs hold these buffers' addresses
      (void)hipDeviceSynchronize();
      for (auto& kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
      p->graphs.clear();
    }
    rc = dev_alloc(p, &p->bcand, &p->bcand_bytes, cand_need, "toplist candidates");
    if (rc) return rc;
    rc = dev_alloc(p, &p->bcount, &p->bcount_bytes, count_need, "toplist counters");
    if (rc) return rc;
  }
  const unsigned sizes = batch_sizes(p, bt);
  // tiles of two sky points: FP32 coefficients, ranges of at most 8 per thread
  const bool pairing = !coef16(p) && p->force_seg <= 0;
  for (int c = 0; c < NC; ++c) {
    const int nfd = fstat::split_nfd(c % NS), nsky = 1 + c / NS;
    if (!((sizes >> nfd) & 1u) || (nsky == 2 && (!pairing || nfd > 8)) || p->batch_grid[c][0]) continue;
    for (int sf = 0; sf < 2; ++sf) p->batch_grid[c][sf] = fstat::interp_batch_grid(coef16(p), nfd, sf == 0, nsky);
  }
  // sky vectors and pair tables, at each unit's offset in the batch
  std::vector<int64_t> sky_off(n + 1, 0);
  for (int k = 0; k < n; ++k) sky_off[k + 1] = sky_off[k] + wus[k].n_sky;
  if (pairing) {
    p->sky_staged = nullptr;                 // sky_h now holds the batch's sky vectors
    if (p->sky_h_cap < (size_t)(3 * sky_off[n])) {
      if (p->sky_h) (void)hipHostFree(p->sky_h);
      p->sky_h = nullptr;
      p->sky_h_cap = 0;
      if (hipHostMalloc((void**)&p->sky_h, (size_t)(3 * sky_off[n]) * sizeof(double), hipHostMallocDefault) !=
          hipSuccess) {
        (void)hipGetLastError();
        return set_err(p, FSTAT_E_NOMEM, "sky vectors: allocation of %lld entries failed", (long long)sky_off[n]);
      }
      p->sky_h_cap = (size_t)(3 * sky_off[n]);
    }
    rc = ensure_pinned_pair(p, &p->pairs_d, &p->pairs_h, &p->pairs_cap, (size_t)sky_off[n], "sky pairs");
    if (rc) return rc;
  }
  // every work unit is checked before anything is demodulated
  if (groups.size() > 1) {
    for (auto& g : groups) {
      for (int k = g.first; k < g.second; ++k) {
        rc = batch_check(p, wus, outs, k, k + 1, (char*)p->arena, std::vector<size_t>(n, 0), st);
        if (rc) return rc;
      }
    }
  }
  bool first = true;
  for (auto& g : groups) {
    rc = batch_check(p, wus, outs, g.first, g.second, (char*)p->arena, offs, st);
    if (rc) return rc;
    // table of the group: one entry per work unit (coefficient passes and
    // toplists), most SFTs first; then one demodulation table per block size
    // (8 down to 4 spindowns per thread): each unit's spindowns split by
    // split_spindowns into consecutive ranges, one per block size; one
    // persistent launch per table, most SFTs first within each
    std::vector<int> order;
    for (int k = g.first; k < g.second; ++k) order.push_back(k);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return wus[x].n_sft > wus[y].n_sft; });
    const int m = (int)order.size();
    fstat::BatchEntry* eh = p->ents_h + kEnts * (size_t)g.first;
    int64_t blocks = 0, sfts = 0;
    int max_top_k = 0;
    uint4* gcand = any_top ? (uint4*)p->bcand + (size_t)g.first * p->cand_cap : nullptr;
    unsigned long long* gcount = any_top ? (unsigned long long*)p->bcount + g.first : nullptr;
    for (int q = 0; q < m; ++q) {
      const int k = order[q];
      fstat::BatchEntry& e = eh[q];
      e = fstat::BatchEntry{};
      WuDev v = make_dev(p, &wus[k], &outs[k]);
      const WuScratch sc = wu_scratch(p, &wus[k], B);
      char* base = (char*)p->arena + offs[k];
      v.geo = (double2*)base;
      v.abcd = (double4*)(base + sc.geo);
      v.coef = (float4*)(base + sc.geo + sc.abcd);
      v.cexp = sc.cexp ? (int32_t*)(base + sc.geo + sc.abcd + sc.coef) : nullptr;
      v.acc = sc.acc ? (float4*)(base + sc.geo + sc.abcd + sc.coef + sc.cexp) : nullptr;
      if (outs[k].top_k > 0) {                         // segment q of the group's candidates
        v.cand = gcand + (size_t)q * p->cand_cap;
        v.cand_count = gcount + q;
        max_top_k = outs[k].top_k > max_top_k ? outs[k].top_k : max_top_k;
      } else {
        v.cand = nullptr;
        v.cand_count = nullptr;
      }
      v.dropped = &p->bstat_d[k].dropped;
      e.w = v;
      e.coef_begin = blocks;
      e.sft_begin = sfts;
      blocks += fstat::coef_blocks(v);
      sfts += wus[k].n_sft;
    }
    std::vector<UnitShape> shapes;
    rc = batch_unit_shapes(p, wus, order, sizes, pairing, sky_off, st, &shapes);
    if (rc) return rc;
    BatchTables tb;
    const int ne = batch_tables(p, wus, order, shapes, sky_off, eh, &tb);
    const int* mc = tb.mc;
    const int* off = tb.off;
    const int64_t* tiles = tb.tiles;
    const bool* fast = tb.fast;
    fstat::BatchEntry* ed = p->ents_d + kEnts * (size_t)g.first;
    hipError_t e = hipMemcpyAsync(ed, eh, (size_t)ne * sizeof(fstat::BatchEntry), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_err(p, e, "work-unit table upload");
    if (first) {
      (void)hipEventRecord(p->ev0, st);
      first = false;
    }
    const bool c16 = coef16(p);
    // The SFT loop in blocks of B SFTs: block b runs the entries with
    // more than b blocks' SFTs, a prefix of each table (most SFTs first),
    // whose tiles are the first tile_begin of the first entry left out.
    const int64_t n_blocks = (wus[order[0]].n_sft + B - 1) / B;
    std::vector<int64_t> bplan;             // per block and table: entries and tiles
    for (int64_t b = 0; b < n_blocks; ++b) {
      for (int c = 0; c < NC; ++c) {
        int x = 0;
        while (x < mc[c] && eh[off[c] + x].w.n_sft > b * B) ++x;
        bplan.insert(bplan.end(), {x, x < mc[c] ? eh[off[c] + x].tile_begin : tiles[c]});
      }
    }
    auto launch_demod_blocks = [&](hipStream_t s, bool counted) -> int {
      for (int64_t b = 0; b < n_blocks; ++b) {
        for (int c = 0; c < NC; ++c) {
          const int64_t* q = &bplan[2 * (NC * b + c)];
          if (q[0] == 0) continue;
          hipError_t ek = fstat::launch_interp_batch(ed + off[c], (int)q[0], q[1], p->counter + c * fstat::kXcds,
                                                     bt.chunk, p->batch_grid[c][fast[c] ? 0 : 1], c16,
                                                     fstat::split_nfd(c % NS), fast[c], 1 + c / NS,
                                                     b * B, (b + 1) * B, s);
          const int r = counted ? check_launch(p, ek, "batch kernel")
                                : (ek == hipSuccess ? FSTAT_OK : hip_err(p, ek, "graph capture"));
          if (r) return r;
        }
      }
      return FSTAT_OK;
    };
    if (p->d.flags & FSTAT_FLAG_NO_GRAPH) {
      if (max_top_k > 0) {
        rc = check_launch(p, fstat::launch_fill_int((int*)gcount, 0, 2 * m, st), "toplist counter reset");
        if (rc) return rc;
      }
      if (c16) {
        rc = check_launch(p, fstat::launch_cexp_batch(ed, m, sfts, st), "coefficient exponent kernel");
        if (rc) return rc;
      }
      rc = check_launch(p, fstat::launch_coef_batch(ed, m, blocks, c16, st), "coefficient kernel");
      if (rc) return rc;
      rc = launch_demod_blocks(st, true);
      if (rc) return rc;
      rc = check_launch(p, fstat::launch_top_select_batch(ed, m, gcand, p->cand_cap, max_top_k, st),
                        "toplist selection");
      if (rc) return rc;
      continue;
    }
    // everything a captured graph holds by value: addresses, counts, kernel variants
    std::vector<int64_t> sig = {(int64_t)(intptr_t)ed, (int64_t)(intptr_t)gcand, (int64_t)(intptr_t)gcount,
                                m, blocks, sfts, max_top_k, n_blocks, B, bt.chunk};
    for (int c = 0; c < NC; ++c) sig.insert(sig.end(), {mc[c], off[c], tiles[c], fast[c] ? 1 : 0});
    sig.insert(sig.end(), bplan.begin(), bplan.end());
    auto it = p->graphs.find(sig);
    if (it == p->graphs.end()) {
      if (!p->cap_stream) {
        if (hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess)
          return set_err(p, FSTAT_E_DEVICE, "capture stream creation failed");
      }
      e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return hip_err(p, e, "graph capture");
      hipError_t e0 = max_top_k > 0 ? fstat::launch_fill_int((int*)gcount, 0, 2 * m, p->cap_stream) : hipSuccess;
      if (e0 == hipSuccess && c16) e0 = fstat::launch_cexp_batch(ed, m, sfts, p->cap_stream);
      hipError_t e1 = e0 != hipSuccess ? e0 : fstat::launch_coef_batch(ed, m, blocks, c16, p->cap_stream);
      const int rd = e1 == hipSuccess ? launch_demod_blocks(p->cap_stream, false) : FSTAT_OK;
      hipError_t e2 = hipSuccess;
      if (e1 == hipSuccess && rd == FSTAT_OK)
        e2 = fstat::launch_top_select_batch(ed, m, gcand, p->cand_cap, max_top_k, p->cap_stream);
      hipGraph_t graph = nullptr;
      e = hipStreamEndCapture(p->cap_stream, &graph);
      if (e1 != hipSuccess || rd != FSTAT_OK || e2 != hipSuccess || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        if (rd != FSTAT_OK) return rd;
        return hip_err(p, e1 != hipSuccess ? e1 : (e2 != hipSuccess ? e2 : e), "graph capture");
      }
      hipGraphExec_t exec = nullptr;
      e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) return hip_err(p, e, "graph instantiation");
      it = p->graphs.emplace(sig, exec).first;
    }
    if (++p->n_launch == p->fail_launch_at) return set_err(p, FSTAT_E_DEVICE, "graph launch: injected launch failure");
    e = hipGraphLaunch(it->second, st);
    if (e != hipSuccess) return hip_err(p, e, "graph launch");
  }
  (void)hipEventRecord(p->ev1, st);
  p->timed = true;
  queue_drop_check(p, p->bstat_d, p->bstat_h, n, st);
  return FSTAT_OK;
}

}  // namespace

extern "C" {

int fstat_plan_create(fstat_plan** out, const fstat_desc* d) {
  if (!out) return FSTAT_E_ARG;
  *out = nullptr;
  if (!d) return FSTAT_E_ARG;
  if (d->max_sft < 1 || d->max_bins < 1 || d->max_sky < 1 || d->max_fd < 1 || d->max_f < 1) return FSTAT_E_ARG;
  if (d->max_dterms < 1 || d->max_dterms > fstat::kMaxDterms) return FSTAT_E_ARG;
  if (d->storage < 0 || d->storage > 2) return FSTAT_E_ARG;
  if (d->phase_mode < 0 || d->phase_mode > 1) return FSTAT_E_ARG;
  if (d->kernel < 0 || d->kernel > 2) return FSTAT_E_ARG;
  if (d->flags & ~(FSTAT_FLAG_NO_GRAPH | FSTAT_FLAG_COEF16)) return FSTAT_E_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return FSTAT_E_DEVICE;
  }
  int dev = d->device;
  if (dev < 0) {
    if (hipGetDevice(&dev) != hipSuccess) return FSTAT_E_DEVICE;
  }
  if (dev >= ndev) return FSTAT_E_ARG;
  if (hipSetDevice(dev) != hipSuccess) return FSTAT_E_DEVICE;
  fstat_plan* p = new (std::nothrow) fstat_plan();
  if (!p) return FSTAT_E_NOMEM;
  p->d = *d;
  p->device = dev;
  read_fault_env(p);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    delete p;
    return FSTAT_E_DEVICE;
  }
  p->cu_count = prop.multiProcessorCount;
  static_setup(dev);
  if (d->max_cands < 0 || d->max_cands > ((int64_t)1 << 24)) {
    delete p;
    return FSTAT_E_ARG;
  }
  p->cand_cap = 1;
  while (p->cand_cap < (d->max_cands > 0 ? d->max_cands : 65536)) p->cand_cap <<= 1;
  if ((p->d.phase_mode == FSTAT_PHASE_SPLIT_FP32 || (p->d.flags & FSTAT_FLAG_COEF16)) &&
      p->d.kernel == FSTAT_KERNEL_DIRECT) {
    // the split phase form and the FP16 coefficients belong to the interpolated kernel only
    delete p;
    return FSTAT_E_UNSUPPORTED;
  }
  if (hipMalloc((void**)&p->status_d, sizeof(fstat::GeoStatus)) != hipSuccess ||
      hipHostMalloc((void**)&p->status_h, sizeof(fstat::GeoStatus), hipHostMallocDefault) != hipSuccess ||
      hipEventCreate(&p->ev0) != hipSuccess || hipEventCreate(&p->ev1) != hipSuccess ||
      hipEventCreateWithFlags(&p->ev_drop, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    fstat_plan_destroy(p);
    return FSTAT_E_NOMEM;
  }
  *out = p;
  return FSTAT_OK;
}

void fstat_plan_destroy(fstat_plan* p) {
  if (!p) return;
  (void)hipSetDevice(p->device);
  (void)hipDeviceSynchronize();
  if (p->geo) (void)hipFree(p->geo);
  if (p->abcd) (void)hipFree(p->abcd);
  for (auto& kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->arena) (void)hipFree(p->arena);
  if (p->bstat_d) (void)hipFree(p->bstat_d);
  if (p->bstat_h) (void)hipHostFree(p->bstat_h);
  if (p->ents_d) (void)hipFree(p->ents_d);
  if (p->ents_h) (void)hipHostFree(p->ents_h);
  if (p->counter) (void)hipFree(p->counter);
  if (p->sky_h) (void)hipHostFree(p->sky_h);
  if (p->pairs_d) (void)hipFree(p->pairs_d);
  if (p->pairs_h) (void)hipHostFree(p->pairs_h);
  if (p->coef) (void)hipFree(p->coef);
  if (p->acc) (void)hipFree(p->acc);
  if (p->cexp) (void)hipFree(p->cexp);
  if (p->cand) (void)hipFree(p->cand);
  if (p->cand_count) (void)hipFree(p->cand_count);
  if (p->bcand) (void)hipFree(p->bcand);
  if (p->bcount) (void)hipFree(p->bcount);
  if (p->dten) (void)hipFree(p->dten);
  for (auto& kv : p->ctab) (void)hipFree(kv.second);
  if (p->status_d) (void)hipFree(p->status_d);
  if (p->status_h) (void)hipHostFree(p->status_h);
  if (p->ev0) (void)hipEventDestroy(p->ev0);
  if (p->ev1) (void)hipEventDestroy(p->ev1);
  if (p->ev_drop) (void)hipEventDestroy(p->ev_drop);
  if (p->seg_arena) (void)hipFree(p->seg_arena);
  for (hipEvent_t e : p->seg_ev) (void)hipEventDestroy(e);
  (void)hipGetLastError();
  delete p;
}

int fstat_compute(fstat_plan* p, const fstat_wu* wu, const fstat_out* out, void* stream) {
  if (!p) return FSTAT_E_ARG;
  p->err[0] = 0;
  p->timed = false;
  p->ms_prev = 0.0;
  p->seg_timed = 0;
  int rc = check_prev_drops(p);
  if (rc) return rc;
  rc = validate_wu(p, wu, out, -1);
  if (rc) return rc;
  if (hipSetDevice(p->device) != hipSuccess) return set_err(p, FSTAT_E_DEVICE, "hipSetDevice failed");
  hipStream_t st = (hipStream_t)stream;
  rc = ensure_scratch(p, wu);
  if (rc) return rc;
  rc = ensure_toplist(p, out);
  if (rc) return rc;
  rc = reset_drops(p, p->status_d, st);
  if (rc) return rc;
  WuDev v = make_dev(p, wu, out);
  rc = run_geometry(p, v, st, -1, may_pair(p, wu) ? wu : nullptr);
  if (rc) return rc;
  bool dflt = false;
  Tile t = pick_tile(p, wu, &dflt);
  rc = prepare_pairs(p, wu, v, t, st, dflt);
  if (rc) return rc;
  rc = run_demod(p, v, t, st);
  if (rc == FSTAT_OK) queue_drop_check(p, p->status_d, p->status_h, 0, st);
  return rc;
}

int fstat_compute_noalloc(fstat_plan* p, const fstat_wu* wu, const fstat_out* out, void* stream) {
  if (!p) return FSTAT_E_ARG;
  p->err[0] = 0;
  p->timed = false;
  p->ms_prev = 0.0;
  p->seg_timed = 0;
  int rc = check_prev_drops(p);
  if (rc) return rc;
  rc = validate_wu(p, wu, out, -1);
  if (rc) return rc;
  if (hipSetDevice(p->device) != hipSuccess) return set_err(p, FSTAT_E_DEVICE, "hipSetDevice failed");
  char* base = p->device < kMaxDevices && g_static_state[p->device] == 1 ? g_static_base[p->device] : nullptr;
  if (!base) return set_err(p, FSTAT_E_DEVICE, "the static scratch of device %d is not available", p->device);
  // work region: geometry, A,B,C,D and, for the interp kernel, the
  // coefficients (with their padding) and the FP16 form's exponents
  const bool interp = resolved_kernel(p) == fstat::KERNEL_INTERP;
  const size_t geo = align256((size_t)wu->n_sky * wu->n_sft * sizeof(double2));
  const size_t abcd = align256((size_t)wu->n_sky * sizeof(double4));
  const size_t coef = interp ? align256(coef_bytes(p, wu)) : 0;
  const size_t cexp = interp && coef16(p) ? align256((size_t)wu->n_sft * sizeof(int32_t)) : 0;
  const size_t need = geo + abcd + coef + cexp, have = fstat::kStaticScratchBytes - fstat::kStaticWorkOff;
  if (need > have)
    return set_err(p, FSTAT_E_SIZE, "fstat_compute_noalloc: the work unit needs %zu bytes of scratch, the static array "
                   "has %zu", need, have);
  const int64_t cap = p->cand_cap < fstat::kStaticCands ? p->cand_cap : fstat::kStaticCands;
  if (out->top_k > cap)
    return set_err(p, FSTAT_E_SIZE, "fstat_compute_noalloc: top_k %d exceeds the static toplist capacity %lld",
                   out->top_k, (long long)cap);
  hipStream_t st = (hipStream_t)stream;
  fstat::GeoStatus* status = (fstat::GeoStatus*)(base + fstat::kStaticStatusOff);
  rc = reset_drops(p, status, st);
  if (rc) return rc;
  WuDev v = make_dev(p, wu, out);
  char* work = base + fstat::kStaticWorkOff;
  v.geo = (double2*)work;
  v.abcd = (double4*)(work + geo);
  v.coef = interp ? (float4*)(work + geo + abcd) : nullptr;
  v.cexp = cexp ? (int32_t*)(work + geo + abcd + coef) : nullptr;
  v.acc = nullptr;
  const int c = coef16(p) ? 1 : 0;
  v.ctab = interp ? (const double*)(base + g_tab_off[c][wu->dterms]) : nullptr;
  v.csum = g_tab_csum[c][wu->dterms];
  v.dropped = &status->dropped;
  v.cand_cap = cap;
  if (out->top_k > 0) {
    v.cand = (uint4*)(base + fstat::kStaticCandOff);
    v.cand_count = (unsigned long long*)(base + fstat::kStaticCountOff);
  }
  rc = run_geometry_at(p, v, status, st, -1);
  if (rc) return rc;
  Tile t = pick_tile(p, wu);
  t.sblock = 0;                      // one launch over all SFTs: no carried Fa, Fb
  rc = run_demod(p, v, t, st);
  if (rc == FSTAT_OK) queue_drop_check(p, status, p->status_h, 0, st);
  return rc;
}

int fstat_batch_compute(fstat_plan* p, const fstat_wu* wus, int32_t n_wu, const fstat_out* outs, void* stream) {
  if (!p) return FSTAT_E_ARG;
  p->err[0] = 0;
  p->timed = false;
  p->ms_prev = 0.0;
  p->seg_timed = 0;
  int rc0 = check_prev_drops(p);
  if (rc0) return rc0;
  if (n_wu < 0 || (n_wu > 0 && (!wus || !outs))) return set_err(p, FSTAT_E_ARG, "bad work-unit list");
  for (int k = 0; k < n_wu; ++k) {
    int rc = validate_wu(p, &wus[k], &outs[k], k);
    if (rc) return rc;
  }
  if (hipSetDevice(p->device) != hipSuccess) return set_err(p, FSTAT_E_DEVICE, "hipSetDevice failed");
  hipStream_t st = (hipStream_t)stream;
  if (n_wu == 0) return FSTAT_OK;
  if (resolved_kernel(p) == fstat::KERNEL_INTERP) return batch_interp(p, wus, n_wu, outs, st);
  // direct kernel: one work unit after the other
  int rc = reset_drops(p, p->status_d, st);
  if (rc) return rc;
  for (int k = 0; k < n_wu; ++k) {
    rc = ensure_scratch(p, &wus[k]);
    if (rc) return rc;
    rc = ensure_toplist(p, &outs[k]);
    if (rc) return rc;
    WuDev v = make_dev(p, &wus[k], &outs[k]);
    rc = run_geometry(p, v, st, k);
    if (rc) return rc;
    rc = run_demod(p, v, pick_tile(p, &wus[k]), st);
    if (rc) return rc;
  }
  queue_drop_check(p, p->status_d, p->status_h, 0, st);
  return FSTAT_OK;
}

int fstat_semicoherent(fstat_plan* p, const fstat_wu* segs, int32_t n_seg, const fstat_out* out, void* stream) {
  if (!p) return FSTAT_E_ARG;
  p->err[0] = 0;
  p->timed = false;
  p->ms_prev = 0.0;
  p->seg_timed = 0;
  int rc0 = check_prev_drops(p);
  if (rc0) return rc0;
  if (n_seg < 1 || !segs || !out) return set_err(p, FSTAT_E_ARG, "semi-coherent: need n_seg >= 1 segments and an output");
  if (!out->twoF) return set_err(p, FSTAT_E_ARG, "semi-coherent: the twoF output holds the sum and is required");
  if (out->fa || out->fb) return set_err(p, FSTAT_E_UNSUPPORTED, "semi-coherent: no Fa/Fb outputs");
  const fstat_wu& g = segs[0];
  for (int k = 0; k < n_seg; ++k) {
    int rc = validate_wu(p, &segs[k], out, k);
    if (rc) return rc;
    const fstat_wu& w = segs[k];
    if (w.n_sky != g.n_sky || w.n_f != g.n_f || w.n_fd != g.n_fd || w.f0 != g.f0 || w.df != g.df ||
        w.fdot0 != g.fdot0 || w.dfdot != g.dfdot || w.t_ref != g.t_ref)
      return set_err(p, FSTAT_E_ARG, "segment %d: template grid or reference time differs from segment 0", k);
  }
  if (hipSetDevice(p->device) != hipSuccess) return set_err(p, FSTAT_E_DEVICE, "hipSetDevice failed");
  hipStream_t st = (hipStream_t)stream;
  int rc = ensure_toplist(p, out);
  if (rc) return rc;
  rc = reset_drops(p, p->status_d, st);
  if (rc) return rc;
  fstat_out o = *out;
  o.top_k = 0;                       // the toplist is taken of the sum, after the last segment
  // Every segment's geometry, A, B, C and band check first, with one wait for
  // all of them (which also brings the sky vectors for the pairing), then the
  // segments' coefficient passes and demodulations back to back on the
  // stream: nothing is demodulated unless every segment passed its check,
  // and the device does not wait for the host between segments.
  const int64_t n = g.n_sky;
  for (int k = 0; k < n_seg; ++k) {  // buffers reach their largest size before any pointer is taken
    rc = ensure_scratch(p, &segs[k]);
    if (rc) return rc;
  }
  std::vector<size_t> goff((size_t)n_seg + 1, 0);
  for (int k = 0; k < n_seg; ++k)
    goff[k + 1] = goff[k] + align256((size_t)n * segs[k].n_sft * sizeof(double2)) + align256((size_t)n * sizeof(double4));
  rc = dev_alloc(p, &p->seg_arena, &p->seg_arena_bytes, goff[n_seg], "segment geometry");
  if (rc) return rc;
  rc = ensure_pinned_pair(p, &p->bstat_d, &p->bstat_h, &p->bstat_cap, (size_t)n_seg, "segment status");
  if (rc) return rc;
  const bool pair = may_pair(p, &g);
  p->sky_staged = nullptr;
  if (pair) {
    const size_t need = (size_t)n_seg * 3 * (size_t)n;
    if (p->sky_h_cap < need) {
      if (p->sky_h) (void)hipHostFree(p->sky_h);
      p->sky_h = nullptr;
      p->sky_h_cap = 0;
      if (hipHostMalloc((void**)&p->sky_h, need * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return set_err(p, FSTAT_E_NOMEM, "sky vectors: allocation of %lld entries failed", (long long)(n * n_seg));
      }
      p->sky_h_cap = need;
    }
    rc = ensure_pinned_pair(p, &p->pairs_d, &p->pairs_h, &p->pairs_cap, (size_t)n_seg * (size_t)n, "sky pairs");
    if (rc) return rc;
  }
  while (p->seg_ev.size() < 2 * (size_t)n_seg) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return set_err(p, FSTAT_E_DEVICE, "semi-coherent: event creation failed");
    p->seg_ev.push_back(e);
  }
  std::vector<WuDev> vs((size_t)n_seg);
  for (int k = 0; k < n_seg; ++k) {
    WuDev v = make_dev(p, &segs[k], &o);
    char* base = (char*)p->seg_arena + goff[k];
    v.geo = (double2*)base;
    v.abcd = (double4*)(base + align256((size_t)n * segs[k].n_sft * sizeof(double2)));
    v.accumulate = k > 0;
    rc = check_launch(p, fstat::launch_fill_int((int*)(p->bstat_d + k), 0, fstat::kGeoResetInts, st), "status reset");
    if (rc) return rc;
    rc = check_launch(p, fstat::launch_geometry(v, p->bstat_d + k, st), "geometry kernel");
    if (rc) return rc;
    if (pair) {
      const hipError_t e = hipMemcpyAsync(p->sky_h + 3 * (size_t)n * k, segs[k].sky, (size_t)(3 * n) * sizeof(double),
                                          hipMemcpyDeviceToHost, st);
      if (e != hipSuccess) return hip_err(p, e, "sky vector copy");
    }
    vs[(size_t)k] = v;
  }
  hipError_t e = hipMemcpyAsync(p->bstat_h, p->bstat_d, (size_t)n_seg * sizeof(fstat::GeoStatus),
                                hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_err(p, e, "geometry kernel");
  for (int k = 0; k < n_seg; ++k) {
    const int bits = p->bstat_h[k].flags;
    if (bits & 1) return set_err(p, FSTAT_E_BAND, "segment %d: a Dirichlet window [k*-D+1, k*+D] leaves the stored band", k);
    if (bits & 2) return set_err(p, FSTAT_E_ARG, "segment %d: antenna-pattern matrix is singular (A B - C^2 <= 0)", k);
  }
  for (int k = 0; k < n_seg; ++k) {
    WuDev v = vs[(size_t)k];
    p->max_abs_tau = status_tau(p->bstat_h[k]);       // the slice widths of this segment's tile
    p->max_p = status_p(p->bstat_h[k]);
    bool dflt = false;
    Tile t = pick_tile(p, &segs[k], &dflt);
    t.pair_seg = 0;
    if (pair && pairs_apply(p, &segs[k], t)) {
      rc = pair_sky(p, &segs[k], v, t, st, dflt, p->bstat_h[k], p->sky_h + 3 * (size_t)n * k,
                    p->pairs_h + (size_t)n * k, p->pairs_d + (size_t)n * k);
      if (rc) return rc;
    }
    rc = run_demod(p, v, t, st, p->seg_ev[2 * (size_t)k], p->seg_ev[2 * (size_t)k + 1]);
    if (rc) return rc;
  }
  p->seg_timed = n_seg;
  if (out->top_k > 0) {
    WuDev v = make_dev(p, &g, out);
    rc = check_launch(p, fstat::launch_fill_int((int*)v.cand_count, 0, 2, st), "toplist counter reset");
    if (rc) return rc;
    rc = check_launch(p, fstat::launch_cand_scan(v, st), "semi-coherent candidate scan");
    if (rc) return rc;
    rc = check_launch(p, fstat::launch_top_select(v, st), "toplist selection");
  }
  if (rc == FSTAT_OK) queue_drop_check(p, p->status_d, p->status_h, 0, st);
  return rc;
}

int fstat_bins(fstat_plan* p, const fstat_wu* wu, int64_t n, const int32_t* i_sky, const int32_t* i_fd,
               const int32_t* i_f, const int32_t* i_sft, int64_t* kstar, double* kappa, double* phi_frac,
               void* stream) {
  if (!p) return FSTAT_E_ARG;
  p->err[0] = 0;
  if (!wu || !wu->t_start || !wu->pos || !wu->vel || !wu->sky) return set_err(p, FSTAT_E_ARG, "null geometry input");
  if (n < 0) return set_err(p, FSTAT_E_ARG, "n < 0");
  if (wu->n_sft < 1 || wu->n_sky < 1 || wu->n_f < 1 || wu->n_fd < 1 || !(wu->t_sft > 0))
    return set_err(p, FSTAT_E_ARG, "bad work-unit sizes");
  if (n > 0 && (!i_sky || !i_fd || !i_f || !i_sft || !kstar || !kappa || !phi_frac))
    return set_err(p, FSTAT_E_ARG, "null index or output array");
  if (hipSetDevice(p->device) != hipSuccess) return set_err(p, FSTAT_E_DEVICE, "hipSetDevice failed");
  WuDev v = make_dev(p, wu, nullptr);
  return check_launch(p, fstat::launch_bins(v, n, i_sky, i_fd, i_f, i_sft, kstar, kappa, phi_frac, (hipStream_t)stream),
                      "bins kernel");
}

// A tile the launchers implement (cache entries are checked against it).
static_assert(FSTAT_NOALLOC_SCRATCH_BYTES == fstat::kStaticScratchBytes, "one size of the static scratch");

static bool valid_tile(const fstat_plan* p, const Tile& t) {
  if (t.sblock < 0) return false;
  if (resolved_kernel(p) == fstat::KERNEL_INTERP) {
    const bool nf_ok = t.nf_reg == 8 || t.nf_reg == 4 || t.nf_reg == 2 || t.nf_reg == 1;
    // 4 (FP16 coefficients: 4 or 5) waves per SIMD: 256-thread tiles with 8 spindowns per thread
    const bool wide = t.nf_reg == 8 && t.threads == 256 && (t.chunk == 4 || (t.chunk == 5 && coef16(p)));
    const bool w_ok = t.chunk == 2 || t.chunk == 3 || wide;
    if (coef16(p))   // 256-thread tiles
      return nf_ok && w_ok && t.threads == 256;
    return nf_ok && w_ok && (t.threads == 256 || (t.threads == 64 && t.nf_reg >= 4));
  }
  return (t.nf_reg == 1 && (t.chunk == 16 || t.chunk == 8)) || (t.nf_reg == 2 && (t.chunk == 8 || t.chunk == 4)) ||
         (t.nf_reg == 4 && t.chunk == 4);
}

int fstat_detector_inputs(fstat_plan* p, const fstat_earth* earth, int32_t n_sites, const fstat_site* sites,
                          int64_t n_sft, const double* t_mid, const int32_t* site_of_sft, int64_t n_sky,
                          const double* sky, double* pos, double* vel, float* a, float* b, void* stream) {
  if (!p) return FSTAT_E_ARG;
  p->err[0] = 0;
  if (!earth || !sites) return set_err(p, FSTAT_E_ARG, "null earth model or site list");
  if (n_sites < 1 || n_sites > FSTAT_MAX_SITES) return set_err(p, FSTAT_E_ARG, "n_sites %d outside [1, 8]", n_sites);
  if (n_sft < 1 || n_sky < 1) return set_err(p, FSTAT_E_ARG, "sizes must be >= 1");
  if (!t_mid || !site_of_sft || !sky || !pos || !vel || !a || !b) return set_err(p, FSTAT_E_ARG, "null array");
  if (n_sft > ((int64_t)1 << 40) / n_sky) return set_err(p, FSTAT_E_SIZE, "too many (sky, SFT) pairs");
  const double vals[8] = {earth->t0, earth->orbit_radius, earth->orbit_rate, earth->orbit_phase, earth->obliquity,
                          earth->earth_radius, earth->sidereal_rate, earth->sidereal_phase};
  for (double x : vals)
    if (!std::isfinite(x)) return set_err(p, FSTAT_E_ARG, "non-finite earth model parameter");
  fstat::EarthModel m{};
  m.t0 = earth->t0;
  m.orbit_radius = earth->orbit_radius;
  m.orbit_rate = earth->orbit_rate;
  m.orbit_phase = earth->orbit_phase;
  m.obliquity = earth->obliquity;
  m.earth_radius = earth->earth_radius;
  m.sidereal_rate = earth->sidereal_rate;
  m.sidereal_phase = earth->sidereal_phase;
  m.n_sites = n_sites;
  for (int k = 0; k < n_sites; ++k) {
    const fstat_site& s = sites[k];
    if (!std::isfinite(s.lat) || !std::isfinite(s.lon) || !std::isfinite(s.az_x) || !std::isfinite(s.az_y))
      return set_err(p, FSTAT_E_ARG, "non-finite site %d", k);
    m.sites[k] = fstat::SiteModel{s.lat, s.lon, s.az_x, s.az_y};
  }
  if (hipSetDevice(p->device) != hipSuccess) return set_err(p, FSTAT_E_DEVICE, "hipSetDevice failed");
  int rc = dev_alloc(p, &p->dten, &p->dten_bytes, (size_t)n_sft * 6 * sizeof(double), "detector tensors");
  if (rc) return rc;
  return check_launch(p,
                      fstat::launch_detector_inputs(m, n_sft, t_mid, site_of_sft, n_sky, sky, pos, vel,
                                                    (double*)p->dten, a, b, (hipStream_t)stream),
                      "detector input kernels");
}

int fstat_autotune(fstat_plan* p, const fstat_wu* wu, const fstat_out* out, void* stream, const char* cache_path) {
  if (!p) return FSTAT_E_ARG;
  p->err[0] = 0;
  int rc = check_prev_drops(p);
  if (rc) return rc;
  rc = validate_wu(p, wu, out, -1);
  if (rc) return rc;
  const bool interp = resolved_kernel(p) == fstat::KERNEL_INTERP;
  const std::string key = class_key(p, wu), bkey = batch_key(p);
  bool have = false, have_b = !interp;            // the batched form of the direct kernel has no shape
  if (cache_path) {
    if (FILE* f = fopen(cache_path, "r")) {
      char k[64];
      int nf, ch, sb, nt;
      while (fscanf(f, "%63s %d %d %d %d", k, &nf, &ch, &sb, &nt) == 5) {
        const Tile t{nf, ch, 0, sb, nt};
        if (key == k && valid_tile(p, t)) {
          p->tiles[key] = t;
          have = true;
        }
        if (interp && bkey == k && valid_batch_tile(t)) {
          p->tiles[bkey] = t;
          have_b = true;
        }
      }
      fclose(f);
      if (have && have_b) return FSTAT_OK;
    }
  }
  if (hipSetDevice(p->device) != hipSuccess) return set_err(p, FSTAT_E_DEVICE, "hipSetDevice failed");
  hipStream_t st = (hipStream_t)stream;
  const bool verbose = getenv("FSTAT_TUNE_VERBOSE") != nullptr;
  auto append = [&](const std::string& k, const Tile& t) {
    if (!cache_path) return;
    if (FILE* f = fopen(cache_path, "a")) {
      fprintf(f, "%s %d %d %d %d\n", k.c_str(), t.nf_reg, t.chunk, t.sblock, t.threads);
      fclose(f);
    }
  };
  if (!have) {
    // single-unit tiles: spindowns or frequencies per thread, waves per SIMD
    // (interp) or SFTs per LDS chunk (direct), SFTs per launch, work-group size
    rc = ensure_scratch(p, wu);
    if (rc) return rc;
    rc = ensure_toplist(p, out);
    if (rc) return rc;
    rc = reset_drops(p, p->status_d, st);
    if (rc) return rc;
    WuDev v = make_dev(p, wu, out);
    rc = run_geometry(p, v, st, -1);
    if (rc) return rc;
    std::vector<Tile> cands;
    if (interp) {
      for (int nt : {256, 64})
        for (int nfd : {8, 4, 2, 1})
          for (int minw : {2, 3, 4, 5})
            for (int sb : {64, 256, 512, 0}) {
              const Tile t{nfd, minw, 0, sb, nt};
              if ((nfd <= 2 * wu->n_fd || nfd == 1) && (nfd == 8 || minw == 3) && valid_tile(p, t)) cands.push_back(t);
            }
    } else {
      cands = {Tile{1, 16, 0, 0, 0}, Tile{1, 8, 0, 0, 0}, Tile{2, 8, 0, 0, 0}, Tile{2, 4, 0, 0, 0}, Tile{4, 4, 0, 0, 0}};
    }
    float best = 1e30f;
    Tile best_t = default_tile(p, wu);
    for (Tile t0 : cands) {
      Tile t = complete_tile(p, wu, t0);            // as pick_tile and fstat_compute run it
      WuDev vt = v;
      rc = prepare_pairs(p, wu, vt, t, st, false);
      if (rc) return rc;
      float ms = 0.f;
      for (int rep = 0; rep < 2; ++rep) {
        rc = run_demod(p, vt, t, st);
        if (rc) return rc;
        hipError_t e = hipEventSynchronize(p->ev1);
        if (e != hipSuccess) return hip_err(p, e, "autotune");
        (void)hipEventElapsedTime(&ms, p->ev0, p->ev1);
      }
      if (verbose)
        fprintf(stderr, "[fstat autotune] %s tile nf_reg=%d chunk=%d seg=%d sblock=%d threads=%d: %.3f ms\n",
                key.c_str(), t.nf_reg, t.chunk, t.seg, t.sblock, t.threads, ms);
      if (ms < best) {
        best = ms;
        best_t = t0;
      }
    }
    p->tiles[key] = best_t;
    queue_drop_check(p, p->status_d, p->status_h, 0, st);
    append(key, best_t);
  }
  if (!have_b) {
    // the batched launch shape, timed on this unit as a batch of one: the
    // spindown blocking, tiles per chunk of the per-XCD queues, SFTs per launch
    rc = check_prev_drops(p);
    if (rc) return rc;
    float best = 1e30f;
    Tile best_t = default_batch_tile();
    for (int nfd : {8, 4})
      for (int chunk : {64, 256, 1024})
        for (int sb : {256, 512, 1024, 0}) {
          const Tile t{nfd, chunk, 0, sb, fstat::kThreads, 0, 0};
          p->tiles[bkey] = t;
          float ms = 0.f;
          for (int rep = 0; rep < 2; ++rep) {       // the first call also captures the graph
            rc = batch_interp(p, wu, 1, out, st);
            if (rc) return rc;
            hipError_t e = hipEventSynchronize(p->ev1);
            if (e != hipSuccess) return hip_err(p, e, "autotune");
            (void)hipEventElapsedTime(&ms, p->ev0, p->ev1);
          }
          rc = check_prev_drops(p);
          if (rc) return rc;
          if (verbose)
            fprintf(stderr, "[fstat autotune] %s nfd=%d chunk=%d sblock=%d: %.3f ms\n", bkey.c_str(), nfd, chunk, sb,
                    ms);
          if (ms < best) {
            best = ms;
            best_t = t;
          }
        }
    p->tiles[bkey] = best_t;
    append(bkey, best_t);
  }
  return FSTAT_OK;
}

int32_t fstat_interp_slice(double df, double dfdot, int32_t nfd, int32_t threads, int32_t coef16, double max_abs_tau,
                           double max_p, int32_t* fits) {
  fstat_wu w{};
  w.df = df;
  w.dfdot = dfdot;
  bool f = false;
  const int W = interp_seg_tau(&w, nfd, threads == 64 ? 64 : fstat::kThreads, coef16 != 0, max_abs_tau, max_p, &f);
  if (fits) *fits = f ? 1 : 0;
  return W;
}

int32_t fstat_sky_pairs(int64_t n_sky, const double* sky, double f0, double df, int64_t n_f, double fdot0,
                        double dfdot, int64_t n_fd, double t_sft, double max_abs_tau, double max_p, double max_v,
                        double max_r, int32_t* pairs, int64_t* n_pairs) {
  if (n_sky < 1 || !sky || !pairs || !n_pairs || n_f < 1 || n_fd < 1) return FSTAT_E_ARG;
  fstat_wu w{};
  w.n_sky = n_sky;
  w.f0 = f0;
  w.df = df;
  w.n_f = n_f;
  w.fdot0 = fdot0;
  w.dfdot = dfdot;
  w.n_fd = n_fd;
  w.t_sft = t_sft;
  fstat::GeoStatus g{};
  memcpy(&g.max_abs_tau_bits, &max_abs_tau, sizeof(double));
  memcpy(&g.max_p_bits, &max_p, sizeof(double));
  memcpy(&g.max_v_bits, &max_v, sizeof(double));
  memcpy(&g.max_r_bits, &max_r, sizeof(double));
  int64_t np = 0;
  const int width = make_pairs(&w, g, sky, reinterpret_cast<int2*>(pairs), &np);
  *n_pairs = width ? np : 0;
  return width;
}

int fstat_spindown_split(int64_t n_fd, int32_t coef16, int32_t allow16, int32_t paired, int64_t* out) {
  if (n_fd < 1 || !out) return FSTAT_E_ARG;
  unsigned sizes = coef16 ? (1u << 8) | (1u << 4) : kAllSplitSizes;
  if (!allow16) sizes &= ~(1u << 16);
  const FdSplit sp = split_spindowns(n_fd, sizes, paired && !coef16);
  for (int i = 0; i < fstat::kSplitSizes; ++i) out[i] = sp.n[i];
  return FSTAT_OK;
}

int fstat_last_tile(const fstat_plan* p, int32_t* out) {
  if (!p || !out || !p->have_last) return FSTAT_E_ARG;
  const Tile& t = p->last_tile;
  const int32_t head[7] = {t.nf_reg, t.chunk, t.seg, t.sblock, t.threads, t.pair_seg, (int32_t)p->last_sky_tiles};
  for (int i = 0; i < 7; ++i) out[i] = head[i];
  for (int i = 0; i < fstat::kSplitSizes; ++i) out[7 + i] = t.fd_split[i];
  return FSTAT_OK;
}

double fstat_last_kernel_ms(fstat_plan* p) {
  if (p && p->seg_timed > 0) {           // semi-coherent: the sum over the segments' launches
    if (hipEventSynchronize(p->seg_ev[2 * (size_t)p->seg_timed - 1]) != hipSuccess) return -1.0;
    double total = 0.0;
    for (int k = 0; k < p->seg_timed; ++k) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, p->seg_ev[2 * (size_t)k], p->seg_ev[2 * (size_t)k + 1]) != hipSuccess) return -1.0;
      total += ms;
    }
    return total;
  }
  if (!p || !p->timed) return -1.0;
  if (hipEventSynchronize(p->ev1) != hipSuccess) return -1.0;
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, p->ev0, p->ev1) != hipSuccess) return -1.0;
  return p->ms_prev + ms;
}

const char* fstat_strerror(int code) {
  switch (code) {
    case FSTAT_OK: return "ok";
    case FSTAT_E_ARG: return "invalid argument";
    case FSTAT_E_BAND: return "Dirichlet window outside the stored band";
    case FSTAT_E_SIZE: return "size exceeds the plan maxima";
    case FSTAT_E_NOMEM: return "out of memory";
    case FSTAT_E_DEVICE: return "HIP device error";
    case FSTAT_E_UNSUPPORTED: return "unsupported option";
    default: return "unknown error";
  }
}

const char* fstat_last_error(const fstat_plan* p) { return p ? p->err : ""; }

}  // extern "C"
