// HIP kernels (gfx950) of the detector inputs of the demodulation: detector
// position and velocity per SFT from a circular-orbit and rotating-Earth
// model, and the antenna-pattern factors a, b per (sky, SFT) as the plus and
// cross projections of the detector tensor on the wave frame.  All FP64
// (hardware sin/cos of arguments below 1e4 rad), a and b stored as FP32.
#include "fstat_internal.h"

namespace fstat {

// One thread per SFT: r, v (sum of the orbital and the diurnal parts) and
// the six unique components of D = (u u^T - w w^T) / 2 in the order
// xx, yy, zz, xy, xz, yz.
__global__ __launch_bounds__(256) void detector_sft_kernel(EarthModel m, int64_t n_sft, const double* t_mid,
                                                           const int32_t* site_of_sft, double* pos, double* vel,
                                                           double* dten) {
  const int64_t al = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (al >= n_sft) return;
  const int si = site_of_sft[al];
  if (si < 0 || si >= m.n_sites) {
    const double nan = __builtin_nan("");
    for (int c = 0; c < 3; ++c) pos[3 * al + c] = vel[3 * al + c] = nan;
    for (int c = 0; c < 6; ++c) dten[6 * al + c] = nan;
    return;
  }
  const SiteModel st = m.sites[si];
  const double dt = t_mid[al] - m.t0;
  double sp, cp, se, ce, sth, cth, sla, cla;
  sincos(m.orbit_phase + m.orbit_rate * dt, &sp, &cp);
  sincos(m.obliquity, &se, &ce);
  sincos(st.lon + m.sidereal_phase + m.sidereal_rate * dt, &sth, &cth);
  sincos(st.lat, &sla, &cla);
  const double R = m.orbit_radius, RW = m.orbit_radius * m.orbit_rate;
  const double Re = m.earth_radius, ReW = m.earth_radius * m.sidereal_rate;
  pos[3 * al + 0] = R * cp + Re * cla * cth;
  pos[3 * al + 1] = R * sp * ce + Re * cla * sth;
  pos[3 * al + 2] = R * sp * se + Re * sla;
  vel[3 * al + 0] = -RW * sp - ReW * cla * sth;
  vel[3 * al + 1] = RW * cp * ce + ReW * cla * cth;
  vel[3 * al + 2] = RW * cp * se;
  // local east and north, then the arms
  const double e[3] = {-sth, cth, 0.0};
  const double nn[3] = {-sla * cth, -sla * sth, cla};
  double sx, cx, sy, cy;
  sincos(st.az_x, &sx, &cx);
  sincos(st.az_y, &sy, &cy);
  double u[3], w[3];
  for (int c = 0; c < 3; ++c) {
    u[c] = cx * nn[c] + sx * e[c];
    w[c] = cy * nn[c] + sy * e[c];
  }
  double* d = dten + 6 * al;
  d[0] = 0.5 * (u[0] * u[0] - w[0] * w[0]);
  d[1] = 0.5 * (u[1] * u[1] - w[1] * w[1]);
  d[2] = 0.5 * (u[2] * u[2] - w[2] * w[2]);
  d[3] = 0.5 * (u[0] * u[1] - w[0] * w[1]);
  d[4] = 0.5 * (u[0] * u[2] - w[0] * w[2]);
  d[5] = 0.5 * (u[1] * u[2] - w[1] * w[2]);
}

// x^T D y for the symmetric D stored as (xx, yy, zz, xy, xz, yz).
__device__ __forceinline__ double tensor_form(const double* d, const double* x, const double* y) {
  return d[0] * x[0] * y[0] + d[1] * x[1] * y[1] + d[2] * x[2] * y[2] + d[3] * (x[0] * y[1] + x[1] * y[0]) +
         d[4] * (x[0] * y[2] + x[2] * y[0]) + d[5] * (x[1] * y[2] + x[2] * y[1]);
}

// One thread per (sky, SFT), SFT fastest (coalesced a, b rows).  The wave
// frame of n = (cos d cos al, cos d sin al, sin d) is formed from the
// components directly: with rho = sqrt(nx^2 + ny^2), X = (ny, -nx, 0) / rho,
// Y = (-nz nx / rho, -nz ny / rho, rho); at the poles (rho = 0) al = 0.
__global__ __launch_bounds__(256) void antenna_kernel(int64_t n_sft, int64_t n_sky, const double* sky,
                                                      const double* dten, float* a, float* b) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n_sft * n_sky) return;
  const int64_t s = t / n_sft, al = t - s * n_sft;
  const double nx = sky[3 * s], ny = sky[3 * s + 1], nzr = sky[3 * s + 2];
  const double nz = nzr > 1.0 ? 1.0 : (nzr < -1.0 ? -1.0 : nzr);
  const double rho = sqrt(nx * nx + ny * ny);
  double X[3], Y[3];
  if (rho > 0.0) {
    const double ca = nx / rho, sa = ny / rho;
    const double cd = sqrt(1.0 - nz * nz);     // cos of the declination from sin d = nz
    X[0] = sa; X[1] = -ca; X[2] = 0.0;
    Y[0] = -nz * ca; Y[1] = -nz * sa; Y[2] = cd;
  } else {
    X[0] = 0.0; X[1] = -1.0; X[2] = 0.0;
    Y[0] = -nz; Y[1] = 0.0; Y[2] = 0.0;
  }
  const double* d = dten + 6 * al;
  a[t] = (float)(tensor_form(d, X, X) - tensor_form(d, Y, Y));
  b[t] = (float)(2.0 * tensor_form(d, X, Y));
}

hipError_t launch_detector_inputs(const EarthModel& m, int64_t n_sft, const double* t_mid, const int32_t* site_of_sft,
                                  int64_t n_sky, const double* sky, double* pos, double* vel, double* dten, float* a,
                                  float* b, hipStream_t st) {
  if (n_sft <= 0 || n_sky <= 0) return hipErrorInvalidValue;
  const int64_t b1 = (n_sft + 255) / 256, b2 = (n_sft * n_sky + 255) / 256;
  if (b1 > 0x7fffffffLL || b2 > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(detector_sft_kernel, dim3((unsigned)b1), dim3(256), 0, st, m, n_sft, t_mid, site_of_sft, pos, vel,
                     dten);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(antenna_kernel, dim3((unsigned)b2), dim3(256), 0, st, n_sft, n_sky, sky, dten, a, b);
  return hipGetLastError();
}

}  // namespace fstat
