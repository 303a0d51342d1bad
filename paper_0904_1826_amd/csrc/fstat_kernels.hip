// HIP kernels (gfx950, wave64) of the F-statistic demodulation.
//
// Steps, in the order of the per-SFT body of the F-statistic loop nest
// (Listing 1, Section 2) read as the Dirichlet demodulation:
//   geometry   per (sky, SFT): tau, Tdot; per sky: A, B, C; band check
//   demod      per (template, SFT): FP64 bin index k*, offset kappa, phase;
//              2D-bin window gathered from an LDS-staged slice of the SFT;
//              FP32 Dirichlet sum; phase rotation; a/b weighting; the sum over
//              SFTs runs in registers; the 2F normalisation is fused at the end.
// The file is compiled with -ffp-contract=off: every FP64 expression below is
// rounded operation by operation in the order written, which makes k* and
// kappa identical bit for bit to any other IEEE binary64 evaluation of the
// same formula.  FP32 fused multiply-adds are written explicitly.
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

// Instantaneous frequency in SFT bins, given g = fdot * tau.
__device__ __forceinline__ double bin_position(double f, double g, double tdot, double t_sft) {
  return ((f + g) * tdot) * t_sft;
}

__device__ __forceinline__ double fract64(double x) { return __builtin_amdgcn_fract(x); }

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
__device__ __forceinline__ double warp_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One block per sky point (grid-stride).  Writes (tau, Tdot) of every SFT and
// (A, B, C, AB - C^2), and sets status bit 1 if some window of the template
// grid leaves the band, bit 2 if AB - C^2 <= 0.  k* is monotone in f and in
// fdot (every rounding step is monotone), so the grid corners bound it.
__global__ __launch_bounds__(256) void geometry_kernel(WuDev w, int* status) {
  __shared__ double red[3][4];
  const double T = w.t_sft;
  const double f_lo = template_f(w, 0), f_hi = template_f(w, w.n_f - 1);
  const double fd_a = template_fd(w, 0), fd_b = template_fd(w, w.n_fd - 1);
  const double band_lo = (double)w.k_first, band_hi = (double)(w.k_first + w.n_bins - 1);
  const int D = w.dterms;
  for (int64_t s = blockIdx.x; s < w.n_sky; s += gridDim.x) {
    double A = 0.0, B = 0.0, C = 0.0;
    int bad = 0;
    for (int64_t al = threadIdx.x; al < w.n_sft; al += blockDim.x) {
      double tau, tdot;
      sft_geometry(w, s, al, tau, tdot);
      w.geo[s * w.n_sft + al] = make_double2(tau, tdot);
      const double a = w.a[s * w.n_sft + al], b = w.b[s * w.n_sft + al];
      A += a * a;
      B += b * b;
      C += a * b;
      const double g_a = fd_a * tau, g_b = fd_b * tau;
      const double d1 = bin_position(f_lo, g_a, tdot, T), d2 = bin_position(f_lo, g_b, tdot, T);
      const double d3 = bin_position(f_hi, g_a, tdot, T), d4 = bin_position(f_hi, g_b, tdot, T);
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
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    if (ln == 0) { red[0][wv] = A; red[1][wv] = B; red[2][wv] = C; }
    const int any_bad = __syncthreads_or(bad);
    if (threadIdx.x == 0) {
      A = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
      B = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
      C = (red[2][0] + red[2][1]) + (red[2][2] + red[2][3]);
      const double Dd = A * B - C * C;
      w.abcd[s] = make_double4(A, B, C, Dd);
      int flags = any_bad ? 1 : 0;
      if (!(Dd > 0.0)) flags |= 2;
      if (flags) atomicOr(status, flags);
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
  const int64_t n_ft = (w.n_f + kThreads * NF - 1) / (kThreads * NF);
  int64_t bid = blockIdx.x;
  const int64_t ft = bid % n_ft;
  bid /= n_ft;
  const int64_t i = bid % w.n_fd;
  const int64_t s = bid / w.n_fd;
  const int tid = threadIdx.x;
  const int64_t j0 = ft * (kThreads * NF);
  const double T = w.t_sft;
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
      const double d = bin_position(f_first, fd * g.x, g.y, T);
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
      const double gf = fd * g.x;                   // fdot * tau
      const double gh = hfd * g.x;                  // (fdot / 2) * tau
      const int64_t lo = lo_col[c];
#pragma unroll
      for (int r = 0; r < NF; ++r) {
        const double dphi = bin_position(f[r], gf, g.y, T);
        const int kst = (int)dphi;                  // floor: dphi > 0
        const double kap64 = fract64(dphi);         // dphi - k*, exact
        const float kap = (float)kap64;
        const float om = (float)(1.0 - kap64);
        const double phi = g.x * (f[r] + gh);
        const float ph = (float)fract64(phi);
        const int64_t col = (int64_t)kst - (D - 1) - w.k_first;
        const int64_t off = col - lo;
        float2 S;
        if (off >= 0 && off + 2 * D <= W) {
          S = dirichlet_sum<DT>(LdsWindow{seg + c * W + off}, D, kap, om);
        } else {
          int64_t cc = col < 0 ? 0 : col;           // memory safety only: the band
          if (cc > w.n_bins - 2 * D) cc = w.n_bins - 2 * D;   // check rules this out
          S = dirichlet_sum<DT>(GlobalWindow{&w, al, cc}, D, kap, om);
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
    w.twoF[o] = (float)two_f;
    if (w.fa) w.fa[o] = make_float2(far[r], fai[r]);
    if (w.fb) w.fb[o] = make_float2(fbr[r], fbi[r]);
  }
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
  const double dphi = bin_position(f, fd * tau, tdot, w.t_sft);
  kstar[t] = (int64_t)dphi;
  kappa[t] = fract64(dphi);
  phi_frac[t] = fract64(tau * (f + (0.5 * fd) * tau));
}

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

hipError_t launch_geometry(const WuDev& w, int* status, hipStream_t st) {
  const int64_t blocks = w.n_sky < 65536 ? w.n_sky : 65536;
  hipLaunchKernelGGL(geometry_kernel, dim3((unsigned)blocks), dim3(256), 0, st, w, status);
  return hipGetLastError();
}

size_t demod_lds_bytes(const WuDev& w, const Tile& t, int kernel) {
  (void)kernel;
  return (size_t)t.chunk * seg_width(kThreads * t.nf_reg, w.dterms) * sizeof(float2);
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
  (void)kernel;
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
