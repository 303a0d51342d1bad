// HIP kernels (gfx950, wave64) of the F-statistic demodulation.
//
// Steps, in the order of the per-SFT body of the F-statistic loop nest
// (Listing 1, Section 2) read as the Dirichlet demodulation:
//   geometry   per (sky, SFT): tau, Tdot T; per sky: A, B, C; band check
//   demod      per (template, SFT): FP64 bin index k*, offset kappa, phase;
//              2D-bin window gathered from an LDS-staged slice of the SFT;
//              FP32 Dirichlet sum; phase rotation; a/b weighting; the sum over
//              SFTs runs in registers; the 2F normalisation is fused at the end.
// The file is compiled with -ffp-contract=off: every FP64 expression below is
// rounded operation by operation in the order written, which makes k* and
// kappa identical bit for bit to any other IEEE binary64 evaluation of the
// same formula.  FP32 fused multiply-adds are written explicitly.
#include <type_traits>

#include "fstat_internal.h"

namespace fstat {

// ------------------------------------------------------------ FP64 helpers
__device__ __forceinline__ void sft_geometry(const WuDev& w, int64_t s, int64_t al, double& tau, double& tdot) {
  const double* r = w.pos + 3 * al;
  const double* v = w.vel + 3 * al;
  const double* n = w.sky + 3 * s;
  const double t_mid = w.t_start[al] + 0.5 * w.t_sft;
  const double rn = (r[0] * n[0] + r[1] * n[1]) + r[2] * n[2];
  const double vn = (v[0] * n[0] + v[1] * n[1]) + v[2] * n[2];
  tau = (t_mid - w.t_ref) + rn;
  tdot = 1.0 + vn;
}

__device__ __forceinline__ double template_f(const WuDev& w, int64_t j) { return w.f0 + (double)j * w.df; }
__device__ __forceinline__ double template_fd(const WuDev& w, int64_t i) { return w.fdot0 + (double)i * w.dfdot; }

// Instantaneous frequency in SFT bins, (f + fdot tau) Tdot T, evaluated as
// f P + q with one rounding (fused multiply-add), where P = Tdot T and
// q = (fdot tau) P are rounded products formed once per SFT (and spindown).
__device__ __forceinline__ double bin_scale(double tdot, double t_sft) { return tdot * t_sft; }
__device__ __forceinline__ double bin_offset(double fd, double tau, double p) { return (fd * tau) * p; }
__device__ __forceinline__ double bin_position(double f, double q, double p) { return __builtin_fma(f, p, q); }

__device__ __forceinline__ double fract64(double x) { return __builtin_amdgcn_fract(x); }

// FP64 value as an unevaluated sum hi + lo of two FP32 (48 significant bits).
__device__ __forceinline__ float2 split64(double x) {
  const float hi = (float)x;
  return make_float2(hi, (float)(x - (double)hi));
}

__device__ __forceinline__ float frac32(float x) { return x - floorf(x); }

// frac(a * b) for a = a.x + a.y, b = b.x + b.y in FP32 arithmetic only: each
// partial product is split into its rounded value and its exact rounding
// error (Dekker's product with a fused multiply-add), the fractional part of
// every term is taken exactly, and only the small remainders are summed.
// Resolution: that of the 48-bit operands (about 5e-5 cycles for a
// 1.2e7 s baseline at 1.5 kHz) plus a few FP32 roundings of values below 4.
__device__ __forceinline__ float frac_split_product(float2 a, float2 b) {
  const float p = a.x * b.x, pe = __builtin_fmaf(a.x, b.x, -p);
  const float q = a.x * b.y, qe = __builtin_fmaf(a.x, b.y, -q);
  const float r = a.y * b.x, re = __builtin_fmaf(a.y, b.x, -r);
  const float t = a.y * b.y;
  float acc = frac32(p) + frac32(pe);
  acc += frac32(q) + frac32(r);
  acc += (qe + re) + t;
  return frac32(acc);
}

// sin(2 pi x) and cos(2 pi x) for x in revolutions (hardware transcendental
// units; |x| < 256).
__device__ __forceinline__ float sin_rev(float x) { return __builtin_amdgcn_sinf(x); }
__device__ __forceinline__ float cos_rev(float x) { return __builtin_amdgcn_cosf(x); }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// ------------------------------------------------------- SFT bin loading
__device__ __forceinline__ float2 load_bin(const WuDev& w, int64_t al, int64_t col) {
  const int64_t e = al * w.n_bins + col;
  if (w.storage == 0) return reinterpret_cast<const float2*>(w.sft)[e];
  const uint32_t u = reinterpret_cast<const uint32_t*>(w.sft)[e];
  const float sc = w.scale[al];
  float re, im;
  if (w.storage == 1) {  // bfloat16: the 16 bits are the top of an FP32
    re = __uint_as_float(u << 16);
    im = __uint_as_float(u & 0xffff0000u);
  } else {               // IEEE half
    re = (float)__builtin_bit_cast(_Float16, (uint16_t)(u & 0xffffu));
    im = (float)__builtin_bit_cast(_Float16, (uint16_t)(u >> 16));
  }
  return make_float2(re * sc, im * sc);
}

// ------------------------------------------------------------- geometry
// ------------------------------------------------------ toplist append
// Templates with 2F >= threshold are appended to the work unit's candidate
// buffer by the epilogue: one atomic per wave reserves the slots of its
// qualifying lanes.  Slots beyond the capacity are dropped (the counter keeps
// counting, which the caller sees as n_above > capacity).
__device__ __forceinline__ void cand_push(const WuDev& w, float tf, int64_t o) {
  const bool q = tf >= w.threshold;                      // NaN never qualifies
  const unsigned long long mask = __ballot(q);
  if (mask == 0ull) return;
  const int lane = (int)__lane_id();
  const int leader = __ffsll((long long)mask) - 1;
  unsigned long long base = 0ull;
  if (lane == leader) base = atomicAdd(w.cand_count, (unsigned long long)__popcll(mask));
  base = __shfl(base, leader, 64);
  if (q) {
    const unsigned long long c = base + (unsigned long long)__popcll(mask & ((1ull << lane) - 1ull));
    if (c < (unsigned long long)w.cand_cap)
      w.cand[c] = make_uint4(__float_as_uint(tf), 0u, (uint32_t)o, (uint32_t)((uint64_t)o >> 32));
  }
}

__device__ __forceinline__ double warp_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Raises the maximum stored as FP64 bits at *m to x >= 0.
__device__ __forceinline__ void raise_max(unsigned long long* m, double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  if (__hip_atomic_load(m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < b) atomicMax(m, b);
}

// One block per sky point (grid-stride).  Writes (tau, Tdot) of every SFT and
// (A, B, C, AB - C^2), and sets status bit 1 if some window of the template
// grid leaves the band, bit 2 if AB - C^2 <= 0.  k* is monotone in f and in
// fdot (every rounding step is monotone), so the grid corners bound it.  The
// status also receives max |tau|, max Tdot T and (from sky point 0's block)
// max |v| and max |r| over the SFTs, which bound slice widths on the host.
__global__ __launch_bounds__(256) void geometry_kernel(WuDev w, GeoStatus* status) {
  __shared__ double red[7][4];
  const double T = w.t_sft;
  const double f_lo = template_f(w, 0), f_hi = template_f(w, w.n_f - 1);
  const double fd_a = template_fd(w, 0), fd_b = template_fd(w, w.n_fd - 1);
  const double band_lo = (double)w.k_first, band_hi = (double)(w.k_first + w.n_bins - 1);
  const int D = w.dterms;
  for (int64_t s = blockIdx.x; s < w.n_sky; s += gridDim.x) {
    double A = 0.0, B = 0.0, C = 0.0, tmax = 0.0, pmax = 0.0, vmax = 0.0, rmax = 0.0;
    int bad = 0;
    for (int64_t al = threadIdx.x; al < w.n_sft; al += blockDim.x) {
      double tau, tdot;
      sft_geometry(w, s, al, tau, tdot);
      if (s == 0) {
        const double* r = w.pos + 3 * al;
        const double* v = w.vel + 3 * al;
        vmax = fmax(vmax, sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]));
        rmax = fmax(rmax, sqrt((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]));
      }
      tmax = fmax(tmax, fabs(tau));
      const double P = bin_scale(tdot, T);
      pmax = fmax(pmax, P);
      w.geo[s * w.n_sft + al] = make_double2(tau, P);
      const double a = w.a[s * w.n_sft + al], b = w.b[s * w.n_sft + al];
      A += a * a;
      B += b * b;
      C += a * b;
      const double q_a = bin_offset(fd_a, tau, P), q_b = bin_offset(fd_b, tau, P);
      const double d1 = bin_position(f_lo, q_a, P), d2 = bin_position(f_lo, q_b, P);
      const double d3 = bin_position(f_hi, q_a, P), d4 = bin_position(f_hi, q_b, P);
      const double kmin = floor(d1 < d2 ? (d1 < d3 ? (d1 < d4 ? d1 : d4) : (d3 < d4 ? d3 : d4))
                                        : (d2 < d3 ? (d2 < d4 ? d2 : d4) : (d3 < d4 ? d3 : d4)));
      const double kmax = floor(d1 > d2 ? (d1 > d3 ? (d1 > d4 ? d1 : d4) : (d3 > d4 ? d3 : d4))
                                        : (d2 > d3 ? (d2 > d4 ? d2 : d4) : (d3 > d4 ? d3 : d4)));
      // NaN fails both comparisons
      if (!(kmin - (double)(D - 1) >= band_lo && kmax + (double)D <= band_hi)) bad = 1;
    }
    A = warp_sum(A);
    B = warp_sum(B);
    C = warp_sum(C);
    for (int o = 32; o > 0; o >>= 1) tmax = fmax(tmax, __shfl_xor(tmax, o, 64));
    for (int o = 32; o > 0; o >>= 1) pmax = fmax(pmax, __shfl_xor(pmax, o, 64));
    for (int o = 32; o > 0; o >>= 1) vmax = fmax(vmax, __shfl_xor(vmax, o, 64));
    for (int o = 32; o > 0; o >>= 1) rmax = fmax(rmax, __shfl_xor(rmax, o, 64));
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    if (ln == 0) {
      red[0][wv] = A; red[1][wv] = B; red[2][wv] = C; red[3][wv] = tmax; red[4][wv] = pmax;
      red[5][wv] = vmax; red[6][wv] = rmax;
    }
    const int any_bad = __syncthreads_or(bad);
    if (threadIdx.x == 0) {
      A = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
      B = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
      C = (red[2][0] + red[2][1]) + (red[2][2] + red[2][3]);
      const double Dd = A * B - C * C;
      w.abcd[s] = make_double4(A, B, C, Dd);
      int flags = any_bad ? 1 : 0;
      if (!(Dd > 0.0)) flags |= 2;
      if (flags) atomicOr(&status->flags, flags);
      // the maxima are non-negative, so their bits order as the values; a
      // block whose value does not exceed the one already stored skips the
      // atomic (the stored value only grows), which keeps thousands of blocks
      // from queueing on one address
      const double tm = fmax(fmax(red[3][0], red[3][1]), fmax(red[3][2], red[3][3]));
      raise_max(&status->max_abs_tau_bits, tm);
      const double pm = fmax(fmax(red[4][0], red[4][1]), fmax(red[4][2], red[4][3]));
      raise_max(&status->max_p_bits, pm);
      if (s == 0) {
        const double vm = fmax(fmax(red[5][0], red[5][1]), fmax(red[5][2], red[5][3]));
        const double rm = fmax(fmax(red[6][0], red[6][1]), fmax(red[6][2], red[6][3]));
        raise_max(&status->max_v_bits, vm);
        raise_max(&status->max_r_bits, rm);
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------ Dirichlet window
// Window sum of one (template, SFT) pair before the sign (-1)^k* and the phase
// rotation:
//   S = sum_{m=-D}^{D-1} x[k*-m] sin(pi kappa) / (pi (kappa + m))
// with x(b) = x[k* - D + 1 + b], b = 0 .. 2D-1 (m = D - 1 - b).  The two
// terms next to the instantaneous frequency (m = 0, -1) use the bounded
// weights sinc(kappa) and -sinc(1 - kappa), with s = sin(pi min(kappa, 1-kappa))
// so that kappa -> 0 and kappa -> 1 lose no accuracy.  The remaining 2D - 2
// terms are summed as running fractions n / p (one reciprocal per 16 terms
// instead of one per term), separately for kappa + m > 0 and < 0.
template <int DT, class Load>
__device__ __forceinline__ float2 dirichlet_sum(const Load& x, int Drt, float kap, float om) {
  const int D = DT > 0 ? DT : Drt;
  const float s = sin_rev(0.5f * fminf(kap, om));           // sin(pi min(kappa, 1 - kappa))
  constexpr float kInvPi = 0.318309886183790672f;
  float gr = 0.f, gi = 0.f;                                 // sum of the far terms, times (kappa + m)^-1
  {
    float nr = 0.f, ni = 0.f, p = 1.f;
    int cnt = 0;
#pragma unroll
    for (int b = 0; b < (DT > 0 ? DT - 1 : 1); ++b) {
      if (DT == 0) break;
      const float q = kap + (float)(D - 1 - b);             // m = D-1 .. 1
      const float2 v = x(b);
      nr = __builtin_fmaf(v.x, p, nr * q);
      ni = __builtin_fmaf(v.y, p, ni * q);
      p *= q;
      if (++cnt == 16) { const float r = rcp(p); gr = __builtin_fmaf(nr, r, gr); gi = __builtin_fmaf(ni, r, gi); nr = ni = 0.f; p = 1.f; cnt = 0; }
    }
    if (DT == 0) {
      for (int b = 0; b < D - 1; ++b) {
        const float q = kap + (float)(D - 1 - b);
        const float2 v = x(b);
        nr = __builtin_fmaf(v.x, p, nr * q);
        ni = __builtin_fmaf(v.y, p, ni * q);
        p *= q;
        if (++cnt == 16) { const float r = rcp(p); gr = __builtin_fmaf(nr, r, gr); gi = __builtin_fmaf(ni, r, gi); nr = ni = 0.f; p = 1.f; cnt = 0; }
      }
    }
    const float r = rcp(p);
    gr = __builtin_fmaf(nr, r, gr);
    gi = __builtin_fmaf(ni, r, gi);
  }
  {
    float nr = 0.f, ni = 0.f, p = 1.f;
    int cnt = 0;
#pragma unroll
    for (int b = (DT > 0 ? DT + 1 : 0); b < (DT > 0 ? 2 * DT : 0); ++b) {
      const float q = kap + (float)(D - 1 - b);             // m = -2 .. -D
      const float2 v = x(b);
      nr = __builtin_fmaf(v.x, p, nr * q);
      ni = __builtin_fmaf(v.y, p, ni * q);
      p *= q;
      if (++cnt == 16) { const float r = rcp(p); gr = __builtin_fmaf(nr, r, gr); gi = __builtin_fmaf(ni, r, gi); nr = ni = 0.f; p = 1.f; cnt = 0; }
    }
    if (DT == 0) {
      for (int b = D + 1; b < 2 * D; ++b) {
        const float q = kap + (float)(D - 1 - b);
        const float2 v = x(b);
        nr = __builtin_fmaf(v.x, p, nr * q);
        ni = __builtin_fmaf(v.y, p, ni * q);
        p *= q;
        if (++cnt == 16) { const float r = rcp(p); gr = __builtin_fmaf(nr, r, gr); gi = __builtin_fmaf(ni, r, gi); nr = ni = 0.f; p = 1.f; cnt = 0; }
      }
    }
    const float r = rcp(p);
    gr = __builtin_fmaf(nr, r, gr);
    gi = __builtin_fmaf(ni, r, gi);
  }
  const float sp = s * kInvPi;
  const float w0 = kap > 0.f ? sp * rcp(kap) : 1.f;         // sinc(kappa)
  const float w1 = sp * rcp(om);                            // sinc(1 - kappa); om > 0 always
  const float2 x0 = x(D - 1), x1 = x(D);                    // bins k*, k*+1
  float sr = __builtin_fmaf(w0, x0.x, -w1 * x1.x);
  float si = __builtin_fmaf(w0, x0.y, -w1 * x1.y);
  sr = __builtin_fmaf(sp, gr, sr);
  si = __builtin_fmaf(sp, gi, si);
  return make_float2(sr, si);
}

struct LdsWindow {
  const float2* p;
  __device__ __forceinline__ float2 operator()(int b) const { return p[b]; }
};

struct GlobalWindow {
  const WuDev* w;
  int64_t al, col0;
  __device__ __forceinline__ float2 operator()(int b) const { return load_bin(*w, al, col0 + b); }
};

// Window sum read straight from global memory, for a lane whose window is
// outside the LDS slice (the asm statement keeps its loads from being merged
// with the LDS path into generic loads).
template <int DT>
__device__ __forceinline__ float2 dirichlet_sum_global(const WuDev& w, int64_t al, int64_t col, int D, float kap,
                                                       float om) {
  col = col < 0 ? 0 : col;                          // memory safety only: the band
  if (col > w.n_bins - 2 * D) col = w.n_bins - 2 * D;   // check rules this out
  const float2 r = dirichlet_sum<DT>(GlobalWindow{&w, al, col}, D, kap, om);
  __asm__ volatile("" ::: "memory");
  return r;
}

// --------------------------------------------------------- demodulation
// One work-group per tile of (sky s, spindown i, kThreads * NF frequencies);
// thread t owns frequencies j0 + t + kThreads * r, r < NF.  SFTs are taken
// CH at a time: their band slices are staged in LDS as float2 (16-bit
// storage is dequantised on the way), then every thread demodulates its NF
// templates against each staged SFT.  Fa, Fb stay in registers across all
// SFTs, so the sum over SFTs and detectors needs no reduction; 2F is formed
// at the end from A, B, C of the sky point.
template <int DT, int NF, int CH>
__global__ __launch_bounds__(kThreads) void demod_direct_kernel(WuDev w) {
  extern __shared__ float2 seg[];                 // [CH][W]
  __shared__ int64_t lo_col[CH];
  const int D = DT > 0 ? DT : w.dterms;
  const int W = seg_width(kThreads * NF, D);
  // Sky point fastest: work-groups resident at the same time share a
  // frequency tile, so their SFT slices (offset only by the Doppler shift of
  // each sky point) overlap and stay in L2.
  int64_t bid = blockIdx.x;
  const int64_t s = bid % w.n_sky;
  bid /= w.n_sky;
  const int64_t i = bid % w.n_fd;
  const int64_t ft = bid / w.n_fd;
  const int tid = threadIdx.x;
  const int64_t j0 = ft * (kThreads * NF);
  const double fd = template_fd(w, i);
  const double hfd = 0.5 * fd;
  const double f_first = template_f(w, j0);
  double f[NF];
#pragma unroll
  for (int r = 0; r < NF; ++r) {
    int64_t j = j0 + tid + (int64_t)kThreads * r;
    if (j > w.n_f - 1) j = w.n_f - 1;             // idle lanes recompute the last template
    f[r] = template_f(w, j);
  }
  float far[NF], fai[NF], fbr[NF], fbi[NF];
#pragma unroll
  for (int r = 0; r < NF; ++r) far[r] = fai[r] = fbr[r] = fbi[r] = 0.f;

  const double2* geo = w.geo + s * w.n_sft;
  const float* arow = w.a + s * w.n_sft;
  const float* brow = w.b + s * w.n_sft;
  const int64_t max_lo = w.n_bins > W ? w.n_bins - W : 0;

  for (int64_t al0 = 0; al0 < w.n_sft; al0 += CH) {
    const int nc = (int)(w.n_sft - al0 < CH ? w.n_sft - al0 : CH);
    __syncthreads();                                // previous chunk consumed
    if (tid < nc) {
      const double2 g = geo[al0 + tid];
      const double d = bin_position(f_first, bin_offset(fd, g.x, g.y), g.y);
      int64_t lo = (int64_t)floor(d) - (D - 1) - w.k_first - 1;   // one bin of slack
      lo = lo < 0 ? 0 : (lo > max_lo ? max_lo : lo);
      lo_col[tid] = lo;
    }
    __syncthreads();
    for (int c = 0; c < nc; ++c) {
      const int64_t lo = lo_col[c];
      const int64_t al = al0 + c;
      for (int e = tid; e < W; e += kThreads) {
        const int64_t col = lo + e;
        seg[c * W + e] = col < w.n_bins ? load_bin(w, al, col) : make_float2(0.f, 0.f);
      }
    }
    __syncthreads();
    for (int c = 0; c < nc; ++c) {
      const int64_t al = al0 + c;
      const double2 g = geo[al];
      const float a = arow[al], b = brow[al];
      const double gf = bin_offset(fd, g.x, g.y);   // (fdot tau) Tdot T
      const double gh = hfd * g.x;                  // (fdot / 2) * tau
      const int base = (int)(w.k_first + lo_col[c]);   // absolute bin of slice column 0
#pragma unroll
      for (int r = 0; r < NF; ++r) {
        const double dphi = bin_position(f[r], gf, g.y);
        const int kst = (int)dphi;                  // floor: dphi > 0
        const double kap64 = fract64(dphi);         // dphi - k*, exact
        const float kap = (float)kap64;
        const float om = (float)(1.0 - kap64);
        const double phi = g.x * (f[r] + gh);
        const float ph = (float)fract64(phi);
        const int off = kst - (D - 1) - base;     // first window bin within the LDS slice
        float2 S;
        if (off >= 0 && off + 2 * D <= W) {
          S = dirichlet_sum<DT>(LdsWindow{seg + c * W + off}, D, kap, om);
        } else {
          S = dirichlet_sum_global<DT>(w, al, (int64_t)kst - (D - 1) - w.k_first, D, kap, om);
        }
        const uint32_t sg = (uint32_t)kst << 31;   // (-1)^k*
        S.x = __uint_as_float(__float_as_uint(S.x) ^ sg);
        S.y = __uint_as_float(__float_as_uint(S.y) ^ sg);
        const float cs = cos_rev(ph), sn = sin_rev(ph);
        const float zr = __builtin_fmaf(S.x, cs, S.y * sn);       // S * exp(-2 pi i phi)
        const float zi = __builtin_fmaf(S.y, cs, -S.x * sn);
        far[r] = __builtin_fmaf(a, zr, far[r]);
        fai[r] = __builtin_fmaf(a, zi, fai[r]);
        fbr[r] = __builtin_fmaf(b, zr, fbr[r]);
        fbi[r] = __builtin_fmaf(b, zi, fbi[r]);
      }
    }
  }
  const double4 abcd = w.abcd[s];
#pragma unroll
  for (int r = 0; r < NF; ++r) {
    const int64_t j = j0 + tid + (int64_t)kThreads * r;
    if (j >= w.n_f) continue;
    const double ar = far[r], ai = fai[r], br = fbr[r], bi = fbi[r];
    const double fa2 = ar * ar + ai * ai, fb2 = br * br + bi * bi, re = ar * br + ai * bi;
    const double two_f = 2.0 * (abcd.y * fa2 + abcd.x * fb2 - 2.0 * abcd.z * re) / abcd.w;
    const int64_t o = (s * w.n_fd + i) * w.n_f + j;
    if (w.twoF) w.twoF[o] = w.accumulate ? w.twoF[o] + (float)two_f : (float)two_f;
    if (w.cand) cand_push(w, (float)two_f, o);
    if (w.fa) w.fa[o] = make_float2(far[r], fai[r]);
    if (w.fb) w.fb[o] = make_float2(fbr[r], fbi[r]);
  }
}


// ------------------------------------------- interpolated window (INTERP)
// The window sum of bin k as a function of kappa,
//   G_k(kappa) = sum_{m=-D}^{D-1} (-1)^(k-m) x[k-m] sinc(kappa + m),
// is an entire function of kappa; on [0, 1) it is replaced by the polynomial
// sum_p c[k][p] kappa^p, whose coefficients
//   c[k][p] = sum_m (-1)^(k-m) x[k-m] t[m][p]
// follow from the per-term polynomials t[m][.] of sinc(kappa + m).  This pass
// computes c for every bin of every SFT (in FP64, stored as FP32 pairs
// (c_p, c_p+1) per float4); the demodulation kernel then evaluates one
// polynomial per (template, SFT) pair instead of 2D weighted terms.  Bins
// whose window would leave the band get zeros (no valid k* selects them).
typedef _Float16 h2v __attribute__((ext_vector_type(2)));
typedef _Float16 h8v __attribute__((ext_vector_type(8)));

// Two FP64 values rounded to FP16 and packed into the bits of one float.
__device__ __forceinline__ float pack_h2(double re, double im) {
  const h2v h = {(_Float16)(float)re, (_Float16)(float)im};
  return __builtin_bit_cast(float, h);
}

template <bool C16>
__device__ __forceinline__ void coef_block(const WuDev& w, int64_t block, float2* xs, double* tab) {
  const int D = w.dterms;
  const int64_t n_cc = (w.n_bins + 255) / 256;
  const int64_t al = block / n_cc;
  const int64_t c0 = (block % n_cc) * 256;
  const int tid = threadIdx.x;
  for (int e = tid; e < 2 * D * kCoef; e += 256) tab[e] = w.ctab[e];
  for (int e = tid; e < 256 + 2 * D; e += 256) {
    const int64_t n = c0 - D + e;
    float2 v = make_float2(0.f, 0.f);
    if (n >= 0 && n < w.n_bins) {
      v = load_bin(w, al, n);
      if ((w.k_first + n) & 1) { v.x = -v.x; v.y = -v.y; }   // (-1)^(absolute bin)
    }
    xs[e] = v;
  }
  __syncthreads();
  const int64_t c = c0 + tid;
  if (c >= w.n_bins) return;
  double cr[kCoef], ci[kCoef];
#pragma unroll
  for (int p = 0; p < kCoef; ++p) cr[p] = ci[p] = 0.0;
  if (c >= D - 1 && c <= w.n_bins - 1 - D) {
    for (int m = -D; m < D; ++m) {
      const float2 x = xs[tid + D - m];                         // bin k - m
      const double* t = tab + (m + D) * kCoef;
#pragma unroll
      for (int p = 0; p < kCoef; ++p) {
        cr[p] = __builtin_fma((double)x.x, t[p], cr[p]);
        ci[p] = __builtin_fma((double)x.y, t[p], ci[p]);
      }
    }
  }
  if constexpr (C16) {          // four complex coefficients per row, times 2^-e of the SFT
    const double sc = ldexp(1.0, -w.cexp[al]);
    float4* dst = w.coef + (al * kRows16) * w.n_bins + c;
#pragma unroll
    for (int q = 0; q < kRows16; ++q)
      dst[q * w.n_bins] = make_float4(pack_h2(cr[4 * q] * sc, ci[4 * q] * sc),
                                      pack_h2(cr[4 * q + 1] * sc, ci[4 * q + 1] * sc),
                                      pack_h2(cr[4 * q + 2] * sc, ci[4 * q + 2] * sc),
                                      pack_h2(cr[4 * q + 3] * sc, ci[4 * q + 3] * sc));
  } else {
    float4* dst = w.coef + (al * kCoefPairs) * w.n_bins + c;
#pragma unroll
    for (int q = 0; q < kCoefPairs; ++q)
      dst[q * w.n_bins] = make_float4((float)cr[2 * q], (float)ci[2 * q], (float)cr[2 * q + 1], (float)ci[2 * q + 1]);
  }
}

template <bool C16>
__global__ __launch_bounds__(256) void coef_kernel(WuDev w) {
  __shared__ float2 xs[256 + 2 * kMaxDterms];
  __shared__ double tab[2 * kMaxDterms * kCoef];
  coef_block<C16>(w, blockIdx.x, xs, tab);
}

// The coefficient pass of many work units in one launch; block b belongs to
// the last entry whose coef_begin <= b.
template <bool C16>
__global__ __launch_bounds__(256) void coef_batch_kernel(const BatchEntry* __restrict__ ents, int n_ent) {
  __shared__ float2 xs[256 + 2 * kMaxDterms];
  __shared__ double tab[2 * kMaxDterms * kCoef];
  const int64_t b = blockIdx.x;
  int lo = 0, hi = n_ent - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ents[mid].coef_begin <= b) lo = mid; else hi = mid - 1;
  }
  const WuDev w = ents[lo].w;
  coef_block<C16>(w, b - ents[lo].coef_begin, xs, tab);
}

// Per-SFT exponent of the FP16 coefficient form: e = (binary exponent of
// max|x| csum) - 12, max over the SFT's bins of max(|re|, |im|), so that every
// stored coefficient |c 2^-e| <= 2^12 and the Horner partial sums of a bin's
// eight coefficients stay below 2^15 < 65504 (the FP16 range).  An all-zero
// SFT gets 0; e is clamped to [-120, 120].
__device__ __forceinline__ void cexp_sft(const WuDev& w, int64_t al, float* red) {
  float mx = 0.f;
  for (int64_t n = threadIdx.x; n < w.n_bins; n += 256) {
    const float2 v = load_bin(w, al, n);
    mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y)));
  }
  for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double m = (double)fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3])) * w.csum;
    int e = 0;
    if (m > 0.0) {
      int ex = 121;
      if (m < 1e300) (void)frexp(m, &ex);
      e = ex - 12;
      e = e < -120 ? -120 : (e > 120 ? 120 : e);
    }
    w.cexp[al] = e;
  }
  __syncthreads();                                 // red is reused by the next SFT
}

__global__ __launch_bounds__(256) void cexp_kernel(WuDev w) {
  __shared__ float red[4];
  for (int64_t al = blockIdx.x; al < w.n_sft; al += gridDim.x) cexp_sft(w, al, red);
}

// The exponent pass of many work units: block b takes SFT b of the
// concatenated SFT list (the last entry whose sft_begin <= b).
__global__ __launch_bounds__(256) void cexp_batch_kernel(const BatchEntry* __restrict__ ents, int n_ent) {
  __shared__ float red[4];
  const int64_t b = blockIdx.x;
  int lo = 0, hi = n_ent - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ents[mid].sft_begin <= b) lo = mid; else hi = mid - 1;
  }
  const WuDev w = ents[lo].w;
  cexp_sft(w, b - ents[lo].sft_begin, red);
}

struct CoefSet {
  float4 c[kCoefPairs];
};

typedef float v4f __attribute__((ext_vector_type(4)));   // native vector: stays in registers

struct CoefSet16 {
  v4f c[kRows16];
};

// Coefficients of one bin read straight from global memory, for a lane whose
// bin is outside the LDS slice.  The empty asm statement after the loads
// keeps the compiler from sinking them into the join with the LDS reads,
// where both would become generic (flat) loads.
__device__ __forceinline__ CoefSet load_coef_global(const WuDev& w, int64_t al, int64_t col) {
  col = col < 0 ? 0 : (col >= w.n_bins ? w.n_bins - 1 : col);   // memory safety only
  const float4* src = w.coef + al * kCoefPairs * w.n_bins + col;
  CoefSet r;
#pragma unroll
  for (int q = 0; q < kCoefPairs; ++q) r.c[q] = src[q * w.n_bins];
  __asm__ volatile("" ::: "memory");
  return r;
}

__device__ __forceinline__ CoefSet16 load_coef16_global(const WuDev& w, int64_t al, int64_t col) {
  col = col < 0 ? 0 : (col >= w.n_bins ? w.n_bins - 1 : col);   // memory safety only
  const v4f* src = reinterpret_cast<const v4f*>(w.coef) + al * kRows16 * w.n_bins + col;
  CoefSet16 r;
#pragma unroll
  for (int q = 0; q < kRows16; ++q) r.c[q] = src[q * w.n_bins];
  __asm__ volatile("" ::: "memory");
  return r;
}

// Values shared by the work-group for a group of S consecutive SFTs: for each
// SFT the first column of its coefficient slice and whether every window of
// the tile falls inside the slice, and per (SFT, spindown) the FP64 product
// fdot * tau and the phase factor exp(-2 pi i frac(tau (fdot/2) tau)).
template <int NFD, int S, int NSKY = 1>
struct GroupMeta {
  double2 geo[S][NSKY];     // (tau, Tdot T) of the tile's sky points
  float2 tsplit[S][NSKY];   // tau as hi + lo FP32 (split phase mode)
  float a[S][NSKY], b[S][NSKY];
  int lo[S];
  int fast[S];
  double g[S][NSKY][NFD];
  float2 e[S][NSKY][NFD];
};

// Fills the meta of SFTs [al0, al0 + n) with all threads of the work-group.
// k* is monotone in f and in fdot, so the tile's corners bound the bins of
// every (template, SFT) pair of the tile: [kmin, kmax] in slice columns, over
// the tile's NSKY sky points (rows geo[u], arow[u], brow[u]).
template <int NFD, int S, int NT, int NSKY>
__device__ __forceinline__ void group_meta(const WuDev& w, const double2* const* geo, const float* const* arow,
                                           const float* const* brow, int64_t al0, int n, int64_t i0, int64_t i_last,
                                           double f_first, double f_last, int W, GroupMeta<NFD, S, NSKY>& m) {
  const int tid = threadIdx.x;
  // NSKY S threads before the last S copy tau, Tdot T, a, b
  const int t3 = tid - (NT - (NSKY + 1) * S);
  if (t3 >= 0 && t3 < NSKY * S && t3 % S < n) {
    const int u = t3 / S, c = t3 % S;
    m.geo[c][u] = geo[u][al0 + c];
    m.tsplit[c][u] = split64(geo[u][al0 + c].x);
    // the FP16 coefficient form stores c 2^-e: the weights carry 2^e
    const float sa = w.coef16 ? ldexpf(1.f, w.cexp[al0 + c]) : 1.f;
    m.a[c][u] = arow[u][al0 + c] * sa;
    m.b[c][u] = brow[u][al0 + c] * sa;
  }
  for (int e = tid; e < n * NSKY * NFD; e += NT) {
    const int c = e / (NSKY * NFD), u = (e / NFD) % NSKY, r = e % NFD;
    const double2 g = geo[u][al0 + c];
    const int64_t i = (i0 + r < w.n_fd) ? i0 + r : w.n_fd - 1;
    const double fd = template_fd(w, i);
    m.g[c][u][r] = bin_offset(fd, g.x, g.y);
    const double h = (0.5 * fd) * g.x;                 // (fdot / 2) tau
    const float q = w.phase_mode ? frac_split_product(split64(g.x), split64(h)) : (float)fract64(g.x * h);
    m.e[c][u][r] = make_float2(cos_rev(q), -sin_rev(q));
  }
  const int t2 = tid - (NT - S);                 // the last S threads do the slice bounds
  if (t2 >= 0 && t2 < n) {
    double lo_d = 0.0, hi_d = 0.0;
#pragma unroll
    for (int u = 0; u < NSKY; ++u) {
      const double2 g = geo[u][al0 + t2];
      const double ga = bin_offset(template_fd(w, i0), g.x, g.y), gb = bin_offset(template_fd(w, i_last), g.x, g.y);
      const double d1 = bin_position(f_first, ga, g.y), d2 = bin_position(f_first, gb, g.y);
      const double d3 = bin_position(f_last, ga, g.y), d4 = bin_position(f_last, gb, g.y);
      const double mn = d1 < d2 ? d1 : d2, mx = d3 > d4 ? d3 : d4;
      lo_d = (u == 0 || mn < lo_d) ? mn : lo_d;
      hi_d = (u == 0 || mx > hi_d) ? mx : hi_d;
    }
    // column offsets of the extreme bins; the band is below 2^31 bins
    const int kmin = (int)(floor(lo_d) - (double)w.k_first);
    const int kmax = (int)(floor(hi_d) - (double)w.k_first);
    const int nb = (int)w.n_bins;
    const int max_lo = nb > W ? nb - W : 0;
    int lo = (kmin > 1 ? kmin : 1) - 1;           // one bin of slack
    lo = lo > max_lo ? max_lo : lo;
    m.lo[t2] = lo;
    m.fast[t2] = (kmin >= lo && kmax <= lo + W - 1 && kmax < nb) ? 1 : 0;
  }
}

// LDS (address space 3) pointers as 32-bit byte addresses.
typedef const __attribute__((address_space(3))) v4f* LdsPtr;
__device__ __forceinline__ uint32_t lds_address(const float4* p) {
  return (uint32_t)(uintptr_t)(LdsPtr)(const v4f*)p;
}
__device__ __forceinline__ LdsPtr lds_pointer(uint32_t a) { return (LdsPtr)(uintptr_t)a; }
__device__ __forceinline__ float4 lds_load(LdsPtr p, int i) {
  const v4f v = p[i];
  return make_float4(v.x, v.y, v.z, v.w);
}

// Slice geometry of each coefficient form: float4 rows per bin and bins per
// LDS row.  For staging, each row is cut into blocks of 64 columns (the last
// one partial unless cap is a multiple of 64), and the NT / 64 waves of a
// work-group take `runs` blocks each.
template <int NT, bool C16>
struct SliceForm {
  static constexpr int rows = C16 ? kRows16 : kCoefPairs;
  static constexpr int cap = C16 ? seg_cap16(NT) : seg_cap(NT);
  static constexpr int waves = NT / 64;
  static constexpr int blocks_per_row = (cap + 63) / 64;
  static constexpr int runs = rows * blocks_per_row / waves;
  static_assert(rows * blocks_per_row == runs * waves, "the waves must share the slice blocks evenly");
};

// Staging of one SFT's coefficient slice: rows x cap float4 starting at band
// column lo (columns W .. cap-1 are padding), loaded from global memory
// straight into `buf` while the other buffer is evaluated, so the loads hold
// no registers.  Wave q moves blocks q, q + NT/64, ...; block b is row
// b / blocks_per_row, columns 64 (b % blocks_per_row) + lane.  Each load is
// one buffer instruction: a resource over the SFT's coefficients from
// column lo (bounds-checked: reads beyond it return 0), a scalar offset per
// block and the lane's byte offset.  Reads past the band's last column land
// in the next row, or, for the last SFT, in the padding the coefficient
// buffer carries (at least cap float4), and fill only padding columns.
// Completion is awaited with lds_dma_wait before the barrier that publishes
// the buffer.
template <int NT, bool C16>
__device__ __forceinline__ void slice_load_lds(const WuDev& w, int64_t al, int lo, float4* buf, uint32_t lane16) {
  using F = SliceForm<NT, C16>;
  const int lo_u = __builtin_amdgcn_readfirstlane(lo);
  const int q = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  // the base address through readfirstlane, so that the resource is known
  // to be uniform (otherwise the compiler may loop over lanes to build it)
  const uint64_t a = reinterpret_cast<uint64_t>(w.coef + (al * F::rows * w.n_bins + lo_u));
  const uint64_t au = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(a >> 32)) << 32) |
                      (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)a);
  const int nb = __builtin_amdgcn_readfirstlane((int)w.n_bins);
  // raw buffer: stride 0, size in bytes (offsets at or past it read 0), and
  // the descriptor's last word with a 32-bit data format (0x00020000), as
  // the buffer instructions of this architecture expect for untyped loads
  const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
      reinterpret_cast<void*>(au), (short)0, (int)(((F::rows - 1) * nb + F::cap) * (int)sizeof(float4)), 0x00020000);
#pragma unroll
  for (int i = 0; i < F::runs; ++i) {
    const int b = i * F::waves + q;                // wave-uniform
    const int row = b / F::blocks_per_row, c0 = 64 * (b % F::blocks_per_row);
    float4* dst = buf + row * F::cap + c0;
    const uint32_t soff = __builtin_amdgcn_readfirstlane((row * nb + c0) * (int)sizeof(float4));
    if (c0 + 64 <= F::cap || lane16 < 16u * (uint32_t)(F::cap - c0))
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (__attribute__((address_space(3))) void*)dst, 16, lane16, soff,
                                               0, 0);
  }
}

// 16 x the lane index, kept in a register for the staging addresses (opaque,
// so that it is not recomputed for every load).
__device__ __forceinline__ uint32_t lane_bytes16() {
  uint32_t v = (threadIdx.x & 63u) << 4;
  __asm__ volatile("" : "+v"(v));
  return v;
}

// Waits for this wave's outstanding global loads, the LDS-direct ones included.
__device__ __forceinline__ void lds_dma_wait() { __builtin_amdgcn_s_waitcnt(0x0F70); }   // vmcnt(0)

// Degree-7 complex polynomial in u = kappa (Horner) times exp(-2 pi i phi),
// added to Fa, Fb with the weights a, b.
__device__ __forceinline__ void interp_accumulate(float4 c01, float4 c23, float4 c45, float4 c67, float u, float cf,
                                                  float sf, float2 eq, float a, float b, float& far, float& fai,
                                                  float& fbr, float& fbi) {
  float gr = __builtin_fmaf(c67.z, u, c67.x), gi = __builtin_fmaf(c67.w, u, c67.y);
  gr = __builtin_fmaf(gr, u, c45.z); gi = __builtin_fmaf(gi, u, c45.w);
  gr = __builtin_fmaf(gr, u, c45.x); gi = __builtin_fmaf(gi, u, c45.y);
  gr = __builtin_fmaf(gr, u, c23.z); gi = __builtin_fmaf(gi, u, c23.w);
  gr = __builtin_fmaf(gr, u, c23.x); gi = __builtin_fmaf(gi, u, c23.y);
  gr = __builtin_fmaf(gr, u, c01.z); gi = __builtin_fmaf(gi, u, c01.w);
  gr = __builtin_fmaf(gr, u, c01.x); gi = __builtin_fmaf(gi, u, c01.y);
  // exp(-2 pi i phi) = exp(-2 pi i frac(tau f)) * exp(-2 pi i frac(tau (fdot/2) tau))
  const float er = __builtin_fmaf(cf, eq.x, sf * eq.y);
  const float ei = __builtin_fmaf(cf, eq.y, -sf * eq.x);
  const float zr = __builtin_fmaf(gr, er, -gi * ei);
  const float zi = __builtin_fmaf(gr, ei, gi * er);
  far = __builtin_fmaf(a, zr, far);
  fai = __builtin_fmaf(a, zi, fai);
  fbr = __builtin_fmaf(b, zr, fbr);
  fbi = __builtin_fmaf(b, zi, fbi);
}

// The same with the FP16 coefficient form: two float4-sized rows hold c0..c3
// and c4..c7 as FP16 (re, im) pairs of the polynomial in v = kappa - 1/2.
// The Horner steps run in packed FP16 (one v_pk_fma_f16 per step for the
// real and imaginary parts, v rounded to FP16); the rotation reads the FP16
// result directly in mixed FP32 fused multiply-adds, and Fa, Fb accumulate in
// FP32.  The per-SFT scale 2^-e keeps every partial sum of the Horner scheme
// below 2^15 (no FP16 overflow).
__device__ __forceinline__ void interp_accumulate16(v4f r0, v4f r1, float u, float cf, float sf, float2 eq, float a,
                                                    float b, float& far, float& fai, float& fbr, float& fbi) {
  // whole rows are reinterpreted (bit-casting single vector elements is not
  // reliable): lo[2p], lo[2p+1] = re, im of c_p, hi likewise for c_{p+4}
  const h8v lo = __builtin_bit_cast(h8v, r0), hi = __builtin_bit_cast(h8v, r1);
  const _Float16 k16 = (_Float16)(u - 0.5f);
  const h2v k = {k16, k16};
  h2v g = {hi[6], hi[7]};
  g = __builtin_elementwise_fma(g, k, (h2v){hi[4], hi[5]});
  g = __builtin_elementwise_fma(g, k, (h2v){hi[2], hi[3]});
  g = __builtin_elementwise_fma(g, k, (h2v){hi[0], hi[1]});
  g = __builtin_elementwise_fma(g, k, (h2v){lo[6], lo[7]});
  g = __builtin_elementwise_fma(g, k, (h2v){lo[4], lo[5]});
  g = __builtin_elementwise_fma(g, k, (h2v){lo[2], lo[3]});
  g = __builtin_elementwise_fma(g, k, (h2v){lo[0], lo[1]});
  const float gr = (float)g.x, gi = (float)g.y;
  const float er = __builtin_fmaf(cf, eq.x, sf * eq.y);
  const float ei = __builtin_fmaf(cf, eq.y, -sf * eq.x);
  // written as fused multiply-adds so that the FP16 operands stay unconverted
  const float zr = __builtin_fmaf(gr, er, __builtin_fmaf(gi, -ei, 0.0f));
  const float zi = __builtin_fmaf(gr, ei, __builtin_fmaf(gi, er, 0.0f));
  far = __builtin_fmaf(a, zr, far);
  fai = __builtin_fmaf(a, zi, fai);
  fbr = __builtin_fmaf(b, zr, fbr);
  fbi = __builtin_fmaf(b, zi, fbi);
}

__device__ __forceinline__ v4f lds_load_v(LdsPtr p, int i) { return p[i]; }

// Demodulation over SFTs [al_begin, al_end) for tiles of (sky s, NFD
// spindowns, NT frequencies), sky point fastest, one tile per work-group.
// The host may split the SFT loop into launches of a few hundred SFTs: the
// work-groups resident at once then stay on nearby SFTs and share their
// coefficient slices (the same frequency tile, offset by each sky point's
// Doppler shift) in L2; Fa, Fb carry over between launches in `acc`.  Within
// a launch the slices (one SFT each) are double-buffered in LDS: the loads of
// SFT k+1 go straight to the idle buffer while SFT k is evaluated, with one
// barrier per SFT.  The per-SFT values shared by the
// work-group are prepared S SFTs at a time by all threads, one group ahead.
// Each thread owns one frequency at NFD spindowns: per SFT it forms
// exp(-2 pi i frac(tau f)) once and, per spindown, the canonical FP64 Dphi,
// k*, kappa, the degree-7 polynomial in kappa, the rotation and the
// a/b accumulation in registers.  An SFT whose windows are not all inside
// the slice (only possible for slices narrower than the tile's spread) takes
// the same arithmetic with coefficients read from global memory; with SAFE
// false (the host has shown that the slice holds every window) that path is
// not compiled.
//
// The tile covers spindowns [fd0, fd1) of the work unit in blocks of NFD
// (the last block of a range may be partial: its missing spindowns repeat
// the range's last one and are not written).
template <int NFD, int S, int G, int NT, bool C16, bool SAFE, int NSKY = 1>
__device__ __forceinline__ void interp_tile(const WuDev& w, int W, int64_t tile, int64_t al_begin, int64_t al_end,
                                            float4* cbuf0, float4* cbuf1, GroupMeta<NFD, S, NSKY>* meta, int64_t fd0,
                                            int64_t fd1) {
  const int tid = threadIdx.x;
  const int64_t n_fdb = (fd1 - fd0 + NFD - 1) / NFD;
  using F = SliceForm<NT, C16>;
  constexpr int Wp = F::cap;                       // LDS row stride
  int64_t t = tile;
  const int64_t n_st = NSKY == 2 ? w.n_pairs : w.n_sky;    // sky tiles
  const int64_t st_idx = t % n_st;
  t /= n_st;
  int64_t su[NSKY];                                // the tile's sky points
  if constexpr (NSKY == 2) {
    const int2 pr = w.sky_pairs[st_idx];
    su[0] = pr.x;
    su[1] = pr.y;
  } else {
    su[0] = st_idx;
  }
  const int64_t ib = t % n_fdb;
  const int64_t ft = t / n_fdb;
  const int64_t j0 = ft * NT;
  int64_t j = j0 + tid;
  const bool jvalid = j < w.n_f;
  if (!jvalid) j = w.n_f - 1;
  const int64_t j_last = (j0 + NT - 1 < w.n_f - 1) ? j0 + NT - 1 : w.n_f - 1;
  const int64_t i0 = fd0 + ib * NFD;
  const int64_t i_last = (i0 + NFD - 1 < fd1 - 1) ? i0 + NFD - 1 : fd1 - 1;
  const double f = template_f(w, j);
  const float2 fsplit = split64(f);
  const bool split_phase = w.phase_mode != 0;
  const double f_first = template_f(w, j0), f_last = template_f(w, j_last);
  const double2* geo[NSKY];
  const float* arow[NSKY];
  const float* brow[NSKY];
#pragma unroll
  for (int u = 0; u < NSKY; ++u) {
    geo[u] = w.geo + su[u] * w.n_sft;
    arow[u] = w.a + su[u] * w.n_sft;
    brow[u] = w.b + su[u] * w.n_sft;
  }
  const int n = (int)(al_end - al_begin);
  const int k_first = (int)w.k_first;

  // accumulators of (sky point u, spindown r) at slot u NFD + r
  constexpr int NSL = NSKY * NFD;
  float far[NSL], fai[NSL], fbr[NSL], fbi[NSL];
#pragma unroll
  for (int x = 0; x < NSL; ++x) {
    const int u = x / NFD, r = x % NFD;
    const int64_t i = (i0 + r < fd1) ? i0 + r : fd1 - 1;
    if (al_begin > 0) {
      const float4 v = w.acc[(su[u] * w.n_fd + i) * w.n_f + j];
      far[x] = v.x; fai[x] = v.y; fbr[x] = v.z; fbi[x] = v.w;
    } else {
      far[x] = fai[x] = fbr[x] = fbi[x] = 0.f;
    }
  }

  // waves whose frequencies all lie beyond the band's last template only
  // help stage slices
  const bool wave_live = __builtin_amdgcn_readfirstlane((int)(j0 + (tid & ~63) < w.n_f));
  bool dropped_any = false;                        // (not SAFE) an SFT left its slice: outputs become NaN
  group_meta<NFD, S, NT, NSKY>(w, geo, arow, brow, al_begin, n < S ? n : S, i0, i_last, f_first, f_last, W, meta[0]);
  __syncthreads();
  const uint32_t lane16 = lane_bytes16();
  slice_load_lds<NT, C16>(w, al_begin, meta[0].lo[0], cbuf0, lane16);
  lds_dma_wait();
  __syncthreads();
  // One SFT per step; the step is written twice (even SFTs read cbuf0 and
  // fill cbuf1, odd SFTs the reverse) so that every LDS access has a fixed
  // buffer.
  // A wave whose frequencies are all beyond the last template runs the same
  // steps without the evaluation; the loop is written once per case so that
  // the accumulators are not merged across the two at every SFT.
  auto step = [&](int k, const float4* seg, float4* next, auto live) __attribute__((always_inline)) {
    const int kk = k % S, gq = (k / S) & 1;
    if (kk == 0 && k + S < n) {                    // values of the next group, read after >= 1 barrier
      const int n1 = n - (k + S) < S ? n - (k + S) : S;
      group_meta<NFD, S, NT, NSKY>(w, geo, arow, brow, al_begin + k + S, n1, i0, i_last, f_first, f_last, W,
                                   meta[gq ^ 1]);
    }
    const bool more = k + 1 < n;
    // unconditional (the last step reloads its own SFT and discards it), so
    // that the registers carry no branch-merged values the compiler must wait
    // for
    // the other buffer was consumed before the last barrier
    const int k1 = more ? k + 1 : k;
    slice_load_lds<NT, C16>(w, al_begin + k1, meta[(k1 / S) & 1].lo[k1 % S], next, lane16);
    const GroupMeta<NFD, S, NSKY>& m = meta[gq];
    const int64_t al = al_begin + k;
    if constexpr (decltype(live)::value) {
    // per sky point: Tdot T, the weights and exp(-2 pi i frac(tau f))
    double pu[NSKY];
    float au[NSKY], bu[NSKY], cf[NSKY], sf[NSKY];
#pragma unroll
    for (int u = 0; u < NSKY; ++u) {
      const double2 g = m.geo[kk][u];
      pu[u] = g.y;
      au[u] = m.a[kk][u];
      bu[u] = m.b[kk][u];
      const float pf = split_phase ? frac_split_product(m.tsplit[kk][u], fsplit)   // frac(tau f)
                                   : (float)fract64(g.x * f);
      cf[u] = cos_rev(pf);
      sf[u] = sin_rev(pf);
    }
    // LDS byte address of bin k in row 0 of the slice: 16 k + (seg - 16 (k_first + lo)),
    // in 32-bit modular arithmetic
    // (uniform; kept opaque in a scalar register so that the compiler forms one
    // shift-and-add per pair rather than folding the sign into a subtraction)
    uint32_t boff = __builtin_amdgcn_readfirstlane(lds_address(seg) - 16u * (uint32_t)(k_first + m.lo[kk]));
    __asm__ volatile("" : "+s"(boff));
    // SAFE: an SFT whose windows are not all in the slice reads its
    // coefficients from global memory.  Otherwise the host has shown that
    // the slice holds every window (the flag is always set), and without a
    // second arithmetic path the accumulators keep their registers through
    // the loop (with one, the compiler copies them at every other SFT).  The
    // flag stays a run-time branch: with the test folded away the compiler
    // schedules across SFTs and spills.
    if (__builtin_amdgcn_readfirstlane(m.fast[kk])) {
#pragma unroll
      for (int x = 0; x < NSL; ++x) {
        const int u = x / NFD, r = x % NFD;
        const double dphi = bin_position(f, m.g[kk][u][r], pu[u]);
        const LdsPtr c = lds_pointer(((uint32_t)(int)dphi << 4) + boff);
        const float kap = (float)fract64(dphi);
        if constexpr (C16)
          interp_accumulate16(lds_load_v(c, 0), lds_load_v(c, Wp), kap, cf[u], sf[u], m.e[kk][u][r], au[u], bu[u],
                              far[x], fai[x], fbr[x], fbi[x]);
        else
          interp_accumulate(lds_load(c, 0), lds_load(c, Wp), lds_load(c, 2 * Wp), lds_load(c, 3 * Wp), kap, cf[u],
                            sf[u], m.e[kk][u][r], au[u], bu[u], far[x], fai[x], fbr[x], fbi[x]);
        if (x % G == G - 1) __builtin_amdgcn_sched_barrier(0);   // bounds the coefficient registers in flight
      }
    } else if constexpr (SAFE) {
#pragma unroll
      for (int x = 0; x < NSL; ++x) {
        const int u = x / NFD, r = x % NFD;
        const double dphi = bin_position(f, m.g[kk][u][r], pu[u]);
        const float kap = (float)fract64(dphi);
        if constexpr (C16) {
          const CoefSet16 cs = load_coef16_global(w, al, (int64_t)(int)dphi - w.k_first);
          interp_accumulate16(cs.c[0], cs.c[1], kap, cf[u], sf[u], m.e[kk][u][r], au[u], bu[u], far[x], fai[x],
                              fbr[x], fbi[x]);
        } else {
          const CoefSet cs = load_coef_global(w, al, (int64_t)(int)dphi - w.k_first);
          interp_accumulate(cs.c[0], cs.c[1], cs.c[2], cs.c[3], kap, cf[u], sf[u], m.e[kk][u][r], au[u], bu[u],
                            far[x], fai[x], fbr[x], fbi[x]);
        }
      }
    } else {
      // no global-memory path: an SFT whose windows leave the slice cannot be
      // evaluated; the tile is counted and its outputs set to NaN (below)
      dropped_any = true;
    }
    }
    lds_dma_wait();
    __syncthreads();
  };
  if (wave_live) {
    for (int k = 0; k < n; k += 2) {
      step(k, cbuf0, cbuf1, std::true_type{});
      if (k + 1 < n) step(k + 1, cbuf1, cbuf0, std::true_type{});
    }
  } else {
    for (int k = 0; k < n; k += 2) {
      step(k, cbuf0, cbuf1, std::false_type{});
      if (k + 1 < n) step(k + 1, cbuf1, cbuf0, std::false_type{});
    }
  }
  if (!jvalid) return;
  if (!SAFE && dropped_any) {
    if (tid == 0 && w.dropped) atomicAdd(w.dropped, 1ull);
    const float nan = __builtin_nanf("");
#pragma unroll
    for (int x = 0; x < NSL; ++x) far[x] = fai[x] = fbr[x] = fbi[x] = nan;
  }
  const bool last = al_end == w.n_sft;
#pragma unroll
  for (int x = 0; x < NSL; ++x) {
    const int u = x / NFD, r = x % NFD;
    if (u > 0 && su[u] == su[0]) continue;         // a sky point without a partner is written once
    const int64_t s = su[u];
    const int64_t i = i0 + r;
    if (i >= fd1) continue;
    const int64_t o = (s * w.n_fd + i) * w.n_f + j;
    if (!last) {
      w.acc[o] = make_float4(far[x], fai[x], fbr[x], fbi[x]);
      continue;
    }
    const double4 abcd = w.abcd[s];
    const double ar = far[x], ai = fai[x], br = fbr[x], bi = fbi[x];
    const double fa2 = ar * ar + ai * ai, fb2 = br * br + bi * bi, re = ar * br + ai * bi;
    const double two_f = 2.0 * (abcd.y * fa2 + abcd.x * fb2 - 2.0 * abcd.z * re) / abcd.w;
    if (w.twoF) w.twoF[o] = w.accumulate ? w.twoF[o] + (float)two_f : (float)two_f;
    if (w.cand) cand_push(w, (float)two_f, o);
    if (w.fa) w.fa[o] = make_float2(far[x], fai[x]);
    if (w.fb) w.fb[o] = make_float2(fbr[x], fbi[x]);
  }
}

// One tile per work-group (see interp_tile) over spindowns [fd0, fd1).
template <int NFD, int S, int MINW, int G, int NT, bool C16, bool SAFE, int NSKY = 1>
__global__ __launch_bounds__(NT, MINW) void demod_interp_kernel(WuDev w, int W, int64_t al_begin, int64_t al_end,
                                                                 int64_t fd0, int64_t fd1) {
  using F = SliceForm<NT, C16>;
  __shared__ GroupMeta<NFD, S, NSKY> meta[2];
  __shared__ float4 cbuf0[F::rows * F::cap];
  __shared__ float4 cbuf1[F::rows * F::cap];
  interp_tile<NFD, S, G, NT, C16, SAFE, NSKY>(w, W, blockIdx.x, al_begin, al_end, cbuf0, cbuf1, meta, fd0, fd1);
}

// Many work units in one persistent launch: the grid holds as many
// work-groups as fit on the device at once; each takes tiles of the
// concatenated tile list from device counters until none is left (every
// work-group reaches that exit).  Entries are ordered by cost (SFT count)
// descending, so the long tiles start first and the tail is short.  Tiles of
// one work unit are sky point fastest, as in the single-unit kernel, so
// consecutive tiles share coefficient slices.  The list is cut into chunks of
// `chunk` consecutive tiles dealt in turn to kXcds queues, one per XCD (the
// hardware places work-group b of a launch on XCD b mod kXcds): the
// work-groups of one XCD take the tiles of its chunks in order, so a slice is
// read by the work-groups of one L2 rather than of all eight.  A work-group
// whose queue is drained takes tiles from the next queue, so every tile runs
// once whatever the placement.  Dterms may differ between work units: the
// window is folded into the coefficients.
// One launch serves the work units of one spindown block size (16 or 4 to 8
// per thread; 8 or 4 with FP16 coefficients; four waves per SIMD, five for 8
// with FP16 coefficients, three for 16, whose 64 accumulators per thread
// take the registers of a fourth but which uses each staged slice for twice
// the pairs; with tiles of two sky points three, and four for 4 per thread,
// whose 128 registers spill 28 bytes of per-tile state but which ran the 64
// uneven units 1.4 % faster than at three), and SFTs [al0, al1) of each: the
// host runs the SFT loop as a sequence of such launches (Fa, Fb carried in
// `acc`), because over thousands of SFTs the work-groups sharing a slice
// drift apart and L2 no longer holds it for all of them.
// Waves per SIMD the registers of a batched specialisation leave room for.
__host__ __device__ constexpr int batch_minw(int nfd, bool c16, int nsky) {
  return nfd == 16 ? 3 : nsky == 2 ? (nfd <= 4 ? 4 : 3) : nfd == 8 ? (c16 ? 5 : 4) : (nfd >= 5 ? 4 : 3);
}

template <int NFD, bool C16, bool SAFE, int NSKY = 1>
__global__ __launch_bounds__(kThreads, batch_minw(NFD, C16, NSKY)) void demod_interp_batch_kernel(
    const BatchEntry* __restrict__ ents, int n_ent, int64_t total_tiles, unsigned long long* counters, int64_t chunk,
    int64_t al0, int64_t al1) {
  using F = SliceForm<kThreads, C16>;
  // per-SFT values per group: four work-groups' LDS fits a CU
  constexpr int S = C16 ? 16 : (NSKY == 2 && NFD <= 4 ? 4 : 8);
  __shared__ GroupMeta<NFD, S, NSKY> meta[2];
  __shared__ float4 cbuf0[F::rows * F::cap];
  __shared__ float4 cbuf1[F::rows * F::cap];
  __shared__ long long next;
  __shared__ int queue[2];                         // thread 0's queue and count of drained queues
  if (threadIdx.x == 0) {
    queue[0] = (int)(blockIdx.x % kXcds);          // this XCD's queue first
    queue[1] = 0;
  }
  for (;;) {
    if (threadIdx.x == 0) {
      long long t = -1;
      int q = queue[0], drained = queue[1];
      while (drained < kXcds) {
        // queue q hands out chunks q, q + kXcds, ... in order; past the end
        // of the list it stays past it, so it is drained once seen so
        const unsigned long long n = atomicAdd(counters + q, 1ull);
        const long long c = (long long)q + (long long)kXcds * (long long)(n / (unsigned long long)chunk);
        const long long u = c * chunk + (long long)(n % (unsigned long long)chunk);
        if (u < total_tiles) {
          t = u;
          break;
        }
        q = q + 1 == kXcds ? 0 : q + 1;
        ++drained;
      }
      queue[0] = q;
      queue[1] = drained;
      next = t;
    }
    __syncthreads();
    const int64_t tile = (int64_t)next;
    __syncthreads();                                 // all have read `next` before it is replaced
    if (tile < 0) break;
    int lo = 0, hi = n_ent - 1;                      // last entry with tile_begin <= tile
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (ents[mid].tile_begin <= tile) lo = mid; else hi = mid - 1;
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    const WuDev& w = ents[lo].w;                  // fields read from the table as needed, not copied
    const int W = ents[lo].seg;
    const int64_t local = tile - ents[lo].tile_begin;
    const int64_t al_end = w.n_sft < al1 ? w.n_sft : al1;
    // tiles of two sky points keep two slots' coefficients in flight (four
    // with one): the queue loop's registers on top of 2 NFD accumulator sets
    interp_tile<NFD, S, NSKY == 2 ? 2 : 4, kThreads, C16, SAFE, NSKY>(w, W, local, al0, al_end, cbuf0, cbuf1, meta,
                                                                     ents[lo].fd_begin, ents[lo].fd_end);
    __syncthreads();                                 // LDS free for the next tile
  }
}

// ------------------------------------------------------------ toplist
// Candidates of a 2F array already in memory (the semi-coherent sum): one
// thread per template.
__global__ __launch_bounds__(256) void cand_scan_kernel(WuDev w, int64_t n) {
  const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (o >= n) return;
  cand_push(w, w.twoF[o], o);
}

// Ranking of candidates: larger 2F first, then smaller linear template index.
__device__ __forceinline__ bool cand_better(uint4 x, uint4 y) {
  const float fx = __uint_as_float(x.x), fy = __uint_as_float(y.x);
  if (fx != fy) return fx > fy;
  return (((uint64_t)x.w << 32) | x.z) < (((uint64_t)y.w << 32) | y.z);
}

// Segment q of the candidate arena belongs to work unit q: its counter and
// output pointers, read from the work-unit table (batched) or the one device
// view (single unit).
struct SingleSeg {
  WuDev w;
  __device__ const WuDev& unit(int) const { return w; }
};
struct BatchSeg {
  const BatchEntry* ents;
  __device__ const WuDev& unit(int q) const { return ents[q].w; }
};

// Slots past a segment's count become sentinels that rank last.
template <class Seg>
__global__ __launch_bounds__(256) void cand_pad_kernel(Seg seg, uint4* cand, int64_t cap, int64_t total) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  const int q = (int)(i / cap);
  const WuDev& w = seg.unit(q);
  const unsigned long long cnt = w.cand_count ? *w.cand_count : 0ull;
  const int64_t n = cnt < (unsigned long long)cap ? (int64_t)cnt : cap;
  if ((i & (cap - 1)) >= n) cand[i] = make_uint4(__float_as_uint(-__builtin_huge_valf()), 0u, ~0u, ~0u);
}

// One compare-exchange pass of a bitonic sort of every cap-long segment
// (pass (k, j), j < k <= cap): best-ranked first when k reaches cap.
__global__ __launch_bounds__(256) void cand_sort_pass_kernel(uint4* cand, int64_t total, int64_t cap, int64_t k,
                                                             int64_t j) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  const int64_t p = i ^ j;
  if (p <= i) return;
  const bool first_best = ((i & (cap - 1)) & k) == 0;
  const uint4 a = cand[i], b = cand[p];
  if (first_best ? cand_better(b, a) : cand_better(a, b)) {
    cand[i] = b;
    cand[p] = a;
  }
}

// The first top_k entries of each sorted segment, decoded to (2F, sky, fdot,
// f); entries past the count get indices -1.  Also publishes n_above.
template <class Seg>
__global__ __launch_bounds__(256) void top_write_kernel(Seg seg, const uint4* cand, int64_t cap) {
  const int q = blockIdx.y;
  const WuDev& w = seg.unit(q);
  if (!w.cand || w.top_k <= 0) return;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const unsigned long long cnt = *w.cand_count;
  if (t == 0) *w.n_above = cnt;
  if (t >= w.top_k) return;
  const int64_t n = cnt < (unsigned long long)cap ? (int64_t)cnt : cap;
  if (t >= n) {
    w.top[t] = make_int4(0, -1, -1, -1);
    return;
  }
  const uint4 c = cand[(int64_t)q * cap + t];
  const int64_t o = (int64_t)(((uint64_t)c.w << 32) | c.z);
  const int64_t per_sky = w.n_fd * w.n_f;
  const int64_t s = o / per_sky, r = o - s * per_sky;
  w.top[t] = make_int4((int)c.x, (int)s, (int)(r / w.n_f), (int)(r % w.n_f));
}

// ------------------------------------------------------------ bin probe
__global__ void bins_kernel(WuDev w, int64_t n, const int32_t* i_sky, const int32_t* i_fd, const int32_t* i_f,
                            const int32_t* i_sft, int64_t* kstar, double* kappa, double* phi_frac) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int64_t s = i_sky[t], i = i_fd[t], j = i_f[t], al = i_sft[t];
  if (s < 0 || s >= w.n_sky || i < 0 || i >= w.n_fd || j < 0 || j >= w.n_f || al < 0 || al >= w.n_sft) {
    kstar[t] = -1;                                   // index outside the work unit
    kappa[t] = phi_frac[t] = __builtin_nan("");
    return;
  }
  double tau, tdot;
  sft_geometry(w, s, al, tau, tdot);
  const double fd = template_fd(w, i);
  const double f = template_f(w, j);
  const double P = bin_scale(tdot, w.t_sft);
  const double dphi = bin_position(f, bin_offset(fd, tau, P), P);
  kstar[t] = (int64_t)dphi;
  kappa[t] = fract64(dphi);
  if (w.phase_mode) {       // the demodulation kernel's split form: frac(tau f) + frac(tau (fdot/2) tau)
    const float a = frac_split_product(split64(tau), split64(f));
    const float b = frac_split_product(split64(tau), split64((0.5 * fd) * tau));
    phi_frac[t] = (double)frac32(a + b);
  } else {
    phi_frac[t] = fract64(tau * (f + (0.5 * fd) * tau));
  }
}

// ---------------------------------------------- static scratch (no alloc)
// Device memory of fstat_compute_noalloc, for callers that cannot allocate:
// every device that loads the library holds one copy of this array until the
// process ends.  Host code never passes the array's name to a kernel or a
// copy: it asks for the device address once per device (below) and uses that.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

hipError_t static_scratch_address(void** ptr) { return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch)); }

// Small fill kernel used instead of hipMemsetAsync, so that the same code is
// safe inside captured graphs.
__global__ void fill_int_kernel(int* p, int v, int n) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = v;
}

// ----------------------------------------------------------- launchers
hipError_t launch_fill_int(int* p, int v, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_int_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

hipError_t launch_geometry(const WuDev& w, GeoStatus* status, hipStream_t st) {
  const int64_t blocks = w.n_sky < 65536 ? w.n_sky : 65536;
  hipLaunchKernelGGL(geometry_kernel, dim3((unsigned)blocks), dim3(256), 0, st, w, status);
  return hipGetLastError();
}

int64_t coef_blocks(const WuDev& w) { return ((w.n_bins + 255) / 256) * w.n_sft; }

hipError_t launch_coef(const WuDev& w, hipStream_t st) {
  const int64_t blocks = coef_blocks(w);
  if (blocks <= 0 || blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  if (w.coef16)
    hipLaunchKernelGGL(coef_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, st, w);
  else
    hipLaunchKernelGGL(coef_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, st, w);
  return hipGetLastError();
}

hipError_t launch_cexp(const WuDev& w, hipStream_t st) {
  const int64_t blocks = w.n_sft < 65536 ? w.n_sft : 65536;
  if (blocks <= 0) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(cexp_kernel, dim3((unsigned)blocks), dim3(256), 0, st, w);
  return hipGetLastError();
}

hipError_t launch_cexp_batch(const BatchEntry* ents_dev, int n_ent, int64_t total_sfts, hipStream_t st) {
  if (n_ent <= 0 || total_sfts <= 0) return hipSuccess;
  if (total_sfts > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(cexp_batch_kernel, dim3((unsigned)total_sfts), dim3(256), 0, st, ents_dev, n_ent);
  return hipGetLastError();
}

hipError_t launch_coef_batch(const BatchEntry* ents_dev, int n_ent, int64_t total_blocks, bool c16, hipStream_t st) {
  if (n_ent <= 0 || total_blocks <= 0) return hipSuccess;
  if (total_blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  if (c16)
    hipLaunchKernelGGL(coef_batch_kernel<true>, dim3((unsigned)total_blocks), dim3(256), 0, st, ents_dev, n_ent);
  else
    hipLaunchKernelGGL(coef_batch_kernel<false>, dim3((unsigned)total_blocks), dim3(256), 0, st, ents_dev, n_ent);
  return hipGetLastError();
}

int64_t interp_tiles(const WuDev& w, int nfd, int64_t fd0, int64_t fd1, int nsky) {
  return ((w.n_f + kThreads - 1) / kThreads) * ((fd1 - fd0 + nfd - 1) / nfd) * (nsky == 2 ? w.n_pairs : w.n_sky);
}

template <int NFD, bool C16, bool SAFE, int NSKY = 1>
static int batch_grid_t(int cus) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, demod_interp_batch_kernel<NFD, C16, SAFE, NSKY>,
                                                   kThreads, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return per_cu * cus;
}

int interp_batch_grid(bool c16, int nfd, bool fast, int nsky) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  if (nsky == 2 && !c16) {
    switch (nfd) {
      case 8: return fast ? batch_grid_t<8, false, false, 2>(cus) : batch_grid_t<8, false, true, 2>(cus);
      case 7: return fast ? batch_grid_t<7, false, false, 2>(cus) : batch_grid_t<7, false, true, 2>(cus);
      case 6: return fast ? batch_grid_t<6, false, false, 2>(cus) : batch_grid_t<6, false, true, 2>(cus);
      case 5: return fast ? batch_grid_t<5, false, false, 2>(cus) : batch_grid_t<5, false, true, 2>(cus);
      default: return fast ? batch_grid_t<4, false, false, 2>(cus) : batch_grid_t<4, false, true, 2>(cus);
    }
  }
  if (c16) {
    if (nfd == 8) return fast ? batch_grid_t<8, true, false>(cus) : batch_grid_t<8, true, true>(cus);
    return fast ? batch_grid_t<4, true, false>(cus) : batch_grid_t<4, true, true>(cus);
  }
  switch (nfd) {
    case 16: return fast ? batch_grid_t<16, false, false>(cus) : batch_grid_t<16, false, true>(cus);
    case 8: return fast ? batch_grid_t<8, false, false>(cus) : batch_grid_t<8, false, true>(cus);
    case 7: return fast ? batch_grid_t<7, false, false>(cus) : batch_grid_t<7, false, true>(cus);
    case 6: return fast ? batch_grid_t<6, false, false>(cus) : batch_grid_t<6, false, true>(cus);
    case 5: return fast ? batch_grid_t<5, false, false>(cus) : batch_grid_t<5, false, true>(cus);
    default: return fast ? batch_grid_t<4, false, false>(cus) : batch_grid_t<4, false, true>(cus);
  }
}

hipError_t launch_interp_batch(const BatchEntry* ents_dev, int n_ent, int64_t total_tiles,
                               unsigned long long* counters, int64_t chunk, int grid, bool c16, int nfd, bool fast,
                               int nsky, int64_t al0, int64_t al1, hipStream_t st) {
  if (n_ent <= 0 || total_tiles <= 0) return hipSuccess;
  if (al0 < 0 || al1 <= al0 || chunk < 1) return hipErrorInvalidValue;
  if (c16 ? (nfd != 8 && nfd != 4) : ((nfd < 4 || nfd > 8) && nfd != 16)) return hipErrorInvalidValue;
  if (nsky != 1 && (nsky != 2 || c16 || nfd > 8)) return hipErrorInvalidValue;
  // kernel, not memset: safe under capture
  hipError_t e = launch_fill_int((int*)counters, 0, 2 * kXcds, st);
  if (e != hipSuccess) return e;
  const dim3 g((unsigned)grid), b(kThreads);
#define FSTAT_BATCH_LAUNCH(N, C, SF) \
  hipLaunchKernelGGL((demod_interp_batch_kernel<N, C, SF>), g, b, 0, st, ents_dev, n_ent, total_tiles, counters, \
                     chunk, al0, al1)
#define FSTAT_BATCH_LAUNCH2(N, C) \
  do { if (fast) FSTAT_BATCH_LAUNCH(N, C, false); else FSTAT_BATCH_LAUNCH(N, C, true); } while (0)
#define FSTAT_BATCH_LAUNCH_P(N) \
  do { \
    if (fast) hipLaunchKernelGGL((demod_interp_batch_kernel<N, false, false, 2>), g, b, 0, st, ents_dev, n_ent, \
                                 total_tiles, counters, chunk, al0, al1); \
    else hipLaunchKernelGGL((demod_interp_batch_kernel<N, false, true, 2>), g, b, 0, st, ents_dev, n_ent, \
                            total_tiles, counters, chunk, al0, al1); \
  } while (0)
  if (nsky == 2) {
    switch (nfd) {
      case 8: FSTAT_BATCH_LAUNCH_P(8); break;
      case 7: FSTAT_BATCH_LAUNCH_P(7); break;
      case 6: FSTAT_BATCH_LAUNCH_P(6); break;
      case 5: FSTAT_BATCH_LAUNCH_P(5); break;
      default: FSTAT_BATCH_LAUNCH_P(4); break;
    }
  } else if (c16) {
    if (nfd == 8) FSTAT_BATCH_LAUNCH2(8, true);
    else FSTAT_BATCH_LAUNCH2(4, true);
  } else {
    switch (nfd) {
      case 16: FSTAT_BATCH_LAUNCH2(16, false); break;
      case 8: FSTAT_BATCH_LAUNCH2(8, false); break;
      case 7: FSTAT_BATCH_LAUNCH2(7, false); break;
      case 6: FSTAT_BATCH_LAUNCH2(6, false); break;
      case 5: FSTAT_BATCH_LAUNCH2(5, false); break;
      default: FSTAT_BATCH_LAUNCH2(4, false); break;
    }
  }
#undef FSTAT_BATCH_LAUNCH_P
#undef FSTAT_BATCH_LAUNCH2
#undef FSTAT_BATCH_LAUNCH
  return hipGetLastError();
}

int interp_launches(const WuDev& w, const Tile& t) {
  const int64_t sb = t.sblock > 0 ? t.sblock : w.n_sft;
  return (int)((w.n_sft + sb - 1) / sb);
}

template <int NFD, int S, int MINW, int G, int NT, bool C16, bool SAFE = true, int NSKY = 1>
static hipError_t launch_interp_t(const WuDev& w, const Tile& t, hipStream_t st, int64_t fd0, int64_t fd1) {
  const int W = t.seg;
  const int64_t n_ft = (w.n_f + NT - 1) / NT;
  if (NSKY == 2 && (!w.sky_pairs || w.n_pairs <= 0)) return hipErrorInvalidValue;
  const int64_t n_tiles = n_ft * ((fd1 - fd0 + NFD - 1) / NFD) * (NSKY == 2 ? w.n_pairs : w.n_sky);
  if (n_tiles <= 0 || n_tiles > 0x7fffffffLL || W < 8 || W > SliceForm<NT, C16>::cap)
    return hipErrorInvalidConfiguration;
  const int64_t sb = t.sblock > 0 ? t.sblock : w.n_sft;
  if (sb < w.n_sft && !w.acc) return hipErrorInvalidValue;
  for (int64_t al = 0; al < w.n_sft; al += sb) {
    const int64_t end = al + sb < w.n_sft ? al + sb : w.n_sft;
    hipLaunchKernelGGL((demod_interp_kernel<NFD, S, MINW, G, NT, C16, SAFE, NSKY>), dim3((unsigned)n_tiles), dim3(NT),
                       0, st, w, W, al, end, fd0, fd1);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int interp_max_seg(int threads, bool c16) {
  const int nt = threads == 64 ? 64 : kThreads;
  return c16 ? seg_cap16(nt) : seg_cap(nt);
}

// Tile: nf_reg = spindowns per thread, chunk = minimum waves per SIMD the
// compiler must leave room for (2 to 5), threads = work-group size (64: one
// wave per work-group, no barrier between waves; 256: four waves share one
// staged slice; the FP16 coefficient form has 256-thread tiles only),
// fast = the variant without the global-memory path may run (the default
// shapes have one).
static hipError_t launch_interp_range(const WuDev& w, const Tile& t, hipStream_t st, int64_t fd0, int64_t fd1) {
  const bool w3 = t.chunk >= 3;
  if (w.coef16) {
    if (t.threads == 64) return hipErrorInvalidValue;
    switch (t.nf_reg) {
      case 8: return t.chunk >= 5 ? (t.fast ? launch_interp_t<8, 16, 5, 4, kThreads, true, false>(w, t, st, fd0, fd1)
                                            : launch_interp_t<8, 16, 5, 4, kThreads, true>(w, t, st, fd0, fd1))
                   : t.chunk >= 4 ? launch_interp_t<8, 16, 4, 4, kThreads, true>(w, t, st, fd0, fd1)
                     : w3         ? launch_interp_t<8, 16, 3, 4, kThreads, true>(w, t, st, fd0, fd1)
                                  : launch_interp_t<8, 16, 2, 4, kThreads, true>(w, t, st, fd0, fd1);
      case 4: return w3 ? (t.fast ? launch_interp_t<4, 16, 3, 4, kThreads, true, false>(w, t, st, fd0, fd1)
                                  : launch_interp_t<4, 16, 3, 4, kThreads, true>(w, t, st, fd0, fd1))
                        : launch_interp_t<4, 16, 2, 4, kThreads, true>(w, t, st, fd0, fd1);
      case 2: return launch_interp_t<2, 16, 3, 4, kThreads, true>(w, t, st, fd0, fd1);
      case 1: return launch_interp_t<1, 16, 3, 4, kThreads, true>(w, t, st, fd0, fd1);
      default: return hipErrorInvalidValue;
    }
  }
  if (t.threads == 64) {
    switch (t.nf_reg) {
      case 8: return w3 ? launch_interp_t<8, 16, 3, 4, 64, false>(w, t, st, fd0, fd1)
                        : launch_interp_t<8, 16, 2, 4, 64, false>(w, t, st, fd0, fd1);
      case 4: return launch_interp_t<4, 16, 3, 4, 64, false>(w, t, st, fd0, fd1);
      case 2: return launch_interp_t<2, 16, 3, 4, 64, false>(w, t, st, fd0, fd1);
      case 1: return launch_interp_t<1, 16, 3, 4, 64, false>(w, t, st, fd0, fd1);
      default: return hipErrorInvalidValue;
    }
  }
  switch (t.nf_reg) {
    // 4 waves per SIMD: per-SFT values for 8 SFTs at a time, so that four
    // work-groups' LDS fits a CU
    // tiles of two sky points (t.pair_seg > 0): 16 accumulator slots per
    // thread, three waves per SIMD
    case 8: if (t.pair_seg > 0)
              return t.fast ? launch_interp_t<8, 8, 3, 4, kThreads, false, false, 2>(w, t, st, fd0, fd1)
                            : launch_interp_t<8, 8, 3, 4, kThreads, false, true, 2>(w, t, st, fd0, fd1);
            return t.chunk >= 4 ? (t.fast ? launch_interp_t<8, 8, 4, 4, kThreads, false, false>(w, t, st, fd0, fd1)
                                          : launch_interp_t<8, 8, 4, 4, kThreads, false>(w, t, st, fd0, fd1))
                   : w3         ? launch_interp_t<8, 16, 3, 4, kThreads, false>(w, t, st, fd0, fd1)
                                : launch_interp_t<8, 16, 2, 4, kThreads, false>(w, t, st, fd0, fd1);
    // 16 and 7 to 5: ranges of a split 8-spindown tile (three waves per SIMD
    // for 16, four for the others); ranges of 4 to 7 with tiles of two sky
    // points (t.pair_seg > 0) have their own specialisations
    case 16: return t.fast ? launch_interp_t<16, 8, 3, 4, kThreads, false, false>(w, t, st, fd0, fd1)
                           : launch_interp_t<16, 8, 3, 4, kThreads, false>(w, t, st, fd0, fd1);
    case 7: if (t.pair_seg > 0)
              return t.fast ? launch_interp_t<7, 8, 3, 4, kThreads, false, false, 2>(w, t, st, fd0, fd1)
                            : launch_interp_t<7, 8, 3, 4, kThreads, false, true, 2>(w, t, st, fd0, fd1);
            return t.fast ? launch_interp_t<7, 8, 4, 4, kThreads, false, false>(w, t, st, fd0, fd1)
                          : launch_interp_t<7, 8, 4, 4, kThreads, false>(w, t, st, fd0, fd1);
    case 6: if (t.pair_seg > 0)
              return t.fast ? launch_interp_t<6, 8, 3, 4, kThreads, false, false, 2>(w, t, st, fd0, fd1)
                            : launch_interp_t<6, 8, 3, 4, kThreads, false, true, 2>(w, t, st, fd0, fd1);
            return t.fast ? launch_interp_t<6, 8, 4, 4, kThreads, false, false>(w, t, st, fd0, fd1)
                          : launch_interp_t<6, 8, 4, 4, kThreads, false>(w, t, st, fd0, fd1);
    case 5: if (t.pair_seg > 0)
              return t.fast ? launch_interp_t<5, 8, 3, 4, kThreads, false, false, 2>(w, t, st, fd0, fd1)
                            : launch_interp_t<5, 8, 3, 4, kThreads, false, true, 2>(w, t, st, fd0, fd1);
            return t.fast ? launch_interp_t<5, 8, 4, 4, kThreads, false, false>(w, t, st, fd0, fd1)
                          : launch_interp_t<5, 8, 4, 4, kThreads, false>(w, t, st, fd0, fd1);
    case 4: if (t.pair_seg > 0)        // 4 groups of per-SFT values: four work-groups' LDS fits a CU
              return t.fast ? launch_interp_t<4, 4, 4, 4, kThreads, false, false, 2>(w, t, st, fd0, fd1)
                            : launch_interp_t<4, 4, 4, 4, kThreads, false, true, 2>(w, t, st, fd0, fd1);
            return w3 ? (t.fast ? launch_interp_t<4, 16, 3, 4, kThreads, false, false>(w, t, st, fd0, fd1)
                                : launch_interp_t<4, 16, 3, 4, kThreads, false>(w, t, st, fd0, fd1))
                      : launch_interp_t<4, 16, 2, 4, kThreads, false>(w, t, st, fd0, fd1);
    case 2: return launch_interp_t<2, 16, 3, 4, kThreads, false>(w, t, st, fd0, fd1);
    case 1: return launch_interp_t<1, 16, 3, 4, kThreads, false>(w, t, st, fd0, fd1);
    default: return hipErrorInvalidValue;
  }
}

// The spindowns in blocks of nf_reg, or, with a split (Tile::fd_split), as
// consecutive ranges with 16, 8, 7, ..., 4 per thread, one launch sequence
// per range (t.fast covers every range's slice); ranges of at most 8 per
// thread run tiles of two sky points when the host paired them.
static hipError_t launch_interp(const WuDev& w, const Tile& t, hipStream_t st) {
  // ranges of at most 8 spindowns per thread may run tiles of two sky points (t.pair_seg)
  const bool pairs = t.pair_seg > 0 && w.sky_pairs && w.n_pairs > 0 && !w.coef16 && t.threads == kThreads;
  int64_t total = 0;
  for (int i = 0; i < kSplitSizes; ++i) total += t.fd_split[i] > 0 ? t.fd_split[i] : 0;
  if (total == 0) {
    Tile t1 = t;
    const bool pr = pairs && t.nf_reg == 8;
    t1.seg = pr ? t.pair_seg : t.seg;
    t1.pair_seg = pr ? t.pair_seg : 0;
    return launch_interp_range(w, t1, st, 0, w.n_fd);
  }
  if (total != w.n_fd) return hipErrorInvalidValue;
  int64_t lo = 0;
  for (int i = 0; i < kSplitSizes; ++i) {
    if (t.fd_split[i] <= 0) continue;
    Tile ti = t;
    ti.nf_reg = split_nfd(i);
    const bool pr = pairs && ti.nf_reg <= 8;
    ti.seg = pr ? t.pair_seg : t.seg_split[i];
    ti.pair_seg = pr ? t.pair_seg : 0;
    if (ti.nf_reg == 4 || ti.nf_reg == 16) ti.chunk = t.chunk > 3 ? 3 : t.chunk;
    else if (ti.nf_reg < 8) ti.chunk = 4;
    const hipError_t e = launch_interp_range(w, ti, st, lo, lo + t.fd_split[i]);
    if (e != hipSuccess) return e;
    lo += t.fd_split[i];
  }
  return hipSuccess;
}

template <class Seg>
static hipError_t top_select(const Seg& seg, int n_seg, uint4* cand, int64_t cap, int max_top_k, hipStream_t st) {
  const int64_t total = (int64_t)n_seg * cap;
  if (n_seg <= 0 || cap <= 0 || (cap & (cap - 1)) != 0 || total / 256 + 1 > 0x7fffffffLL)
    return hipErrorInvalidConfiguration;
  const dim3 grid((unsigned)((total + 255) / 256)), block(256);
  hipLaunchKernelGGL(cand_pad_kernel<Seg>, grid, block, 0, st, seg, cand, cap, total);
  hipError_t e = hipGetLastError();
  for (int64_t k = 2; k <= cap && e == hipSuccess; k <<= 1)
    for (int64_t j = k >> 1; j > 0 && e == hipSuccess; j >>= 1) {
      hipLaunchKernelGGL(cand_sort_pass_kernel, grid, block, 0, st, cand, total, cap, k, j);
      e = hipGetLastError();
    }
  if (e != hipSuccess) return e;
  if (max_top_k <= 0) return hipSuccess;
  hipLaunchKernelGGL(top_write_kernel<Seg>, dim3((unsigned)((max_top_k + 255) / 256), (unsigned)n_seg), block, 0, st,
                     seg, (const uint4*)cand, cap);
  return hipGetLastError();
}

hipError_t launch_cand_scan(const WuDev& w, hipStream_t st) {
  const int64_t n = w.n_sky * w.n_fd * w.n_f;
  const int64_t blocks = (n + 255) / 256;
  if (!w.cand || !w.twoF || blocks <= 0 || blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(cand_scan_kernel, dim3((unsigned)blocks), dim3(256), 0, st, w, n);
  return hipGetLastError();
}

hipError_t launch_top_select(const WuDev& w, hipStream_t st) {
  if (!w.cand || w.top_k <= 0) return hipSuccess;
  return top_select(SingleSeg{w}, 1, w.cand, w.cand_cap, w.top_k, st);
}

hipError_t launch_top_select_batch(const BatchEntry* ents_dev, int n_ent, uint4* cand, int64_t cap, int max_top_k,
                                   hipStream_t st) {
  if (max_top_k <= 0) return hipSuccess;
  return top_select(BatchSeg{ents_dev}, n_ent, cand, cap, max_top_k, st);
}

template <int DT, int NF, int CH>
static hipError_t launch_direct_t(const WuDev& w, hipStream_t st) {
  const int64_t n_ft = (w.n_f + kThreads * NF - 1) / (kThreads * NF);
  const int64_t blocks = n_ft * w.n_fd * w.n_sky;
  if (blocks <= 0 || blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  const size_t lds = (size_t)CH * seg_width(kThreads * NF, DT > 0 ? DT : w.dterms) * sizeof(float2);
  hipLaunchKernelGGL((demod_direct_kernel<DT, NF, CH>), dim3((unsigned)blocks), dim3(kThreads), lds, st, w);
  return hipGetLastError();
}

template <int DT>
static hipError_t launch_direct_d(const WuDev& w, const Tile& t, hipStream_t st) {
  if (t.nf_reg == 1 && t.chunk == 16) return launch_direct_t<DT, 1, 16>(w, st);
  if (t.nf_reg == 1 && t.chunk == 8) return launch_direct_t<DT, 1, 8>(w, st);
  if (t.nf_reg == 2 && t.chunk == 8) return launch_direct_t<DT, 2, 8>(w, st);
  if (t.nf_reg == 2 && t.chunk == 4) return launch_direct_t<DT, 2, 4>(w, st);
  if (t.nf_reg == 4 && t.chunk == 4) return launch_direct_t<DT, 4, 4>(w, st);
  return hipErrorInvalidValue;
}

hipError_t launch_demod(const WuDev& w, const Tile& t, int kernel, hipStream_t st) {
  if (kernel == KERNEL_INTERP) return launch_interp(w, t, st);
  switch (w.dterms) {
    case 8: return launch_direct_d<8>(w, t, st);
    case 16: return launch_direct_d<16>(w, t, st);
    default: return launch_direct_d<0>(w, t, st);
  }
}

hipError_t launch_bins(const WuDev& w, int64_t n, const int32_t* i_sky, const int32_t* i_fd, const int32_t* i_f,
                       const int32_t* i_sft, int64_t* kstar, double* kappa, double* phi_frac, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(bins_kernel, dim3((unsigned)blocks), dim3(256), 0, st, w, n, i_sky, i_fd, i_f, i_sft, kstar,
                     kappa, phi_frac);
  return hipGetLastError();
}

}  // namespace fstat
