/*
 * FP64 CPU oracle for the F-statistic demodulation (test infrastructure).
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg use
 * this file.  It shares no code with the GPU library: it is written from the
 * mathematics of the SFT-domain F-statistic, in plain loops, in IEEE binary64
 * with round-to-nearest; the one fused multiply-add is the explicit fma() in
 * Dphi, nothing else may be contracted (build with -ffp-contract=off and
 * without -ffast-math).
 *
 * What it computes follows the F-statistic loop nest of the paper (Listing 1,
 * Section 2): an independent loop over the frequencies of a band, a sum over
 * detectors, and inside it a sum over the SFTs of each detector followed by a
 * normalisation.  The per-SFT body, which the paper leaves undefined, is the
 * Dirichlet-kernel demodulation of one SFT:
 *
 *   tau_a   = (t_a + T/2 - t_ref) + r_a . n          (arrival-time offset)
 *   Tdot_a  = 1 + v_a . n                            (Doppler factor)
 *   P_a     = Tdot_a * T,  q_a = (fdot * tau_a) * P_a
 *   Dphi_a  = fma(f, P_a, q_a)                       (instantaneous frequency in bins,
 *                                                     (f + fdot tau_a) Tdot_a T)
 *   k*_a    = floor(Dphi_a),  kappa_a = Dphi_a - k*_a
 *   phi_a   = tau_a * (f + (fdot/2) * tau_a)         (phase at the SFT midpoint, cycles)
 *   z_a     = exp(-2 pi i frac(phi_a)) *
 *             sum_{m=-D}^{D-1} (-1)^(k*-m) x_a[k*-m] sinc(kappa_a + m)
 *   Fa      = sum_a a_a z_a,   Fb = sum_a b_a z_a      (over all SFTs of all detectors)
 *   2F      = 2 (B |Fa|^2 + A |Fb|^2 - 2 C Re(Fa conj Fb)) / (A B - C^2)
 *   A = sum a^2, B = sum b^2, C = sum a b
 *
 * with sinc(x) = sin(pi x) / (pi x) and sinc(0) = 1.  z_a is the integral over
 * the SFT of the data times exp(-2 pi i Phi(t)) for a phase that is linear
 * across the SFT; sinc is the continuous Dirichlet kernel, truncated to the
 * 2D bins nearest the instantaneous frequency.  A window that leaves the
 * stored band is an error (no clamping, no padding).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_E_ARG -1
#define ORACLE_E_BAND -2

typedef struct oracle_wu {
  int n_sft, n_bins;
  int64_t k_first;
  double t_sft;
  const double* sft;      /* [n_sft][n_bins][2] (re, im), already dequantised */
  const double* t_start;  /* [n_sft] */
  const double* pos;      /* [n_sft][3] light-s */
  const double* vel;      /* [n_sft][3] units of c */
  int n_sky;
  const double* sky;      /* [n_sky][3] unit vectors */
  const double* a;        /* [n_sky][n_sft] */
  const double* b;        /* [n_sky][n_sft] */
  double f0, df;
  int n_f;
  double fdot0, dfdot;
  int n_fd;
  double t_ref;
  int dterms;
} oracle_wu;

/* Normalised sinc with its removable singularity filled in. */
double oracle_sinc(double x) {
  if (x == 0.0) return 1.0;
  return sin(M_PI * x) / (M_PI * x);
}

/* Dirichlet window weights for offset kappa: w[m + D] = sinc(kappa + m),
 * m = -D .. D-1.  Written as (-1)^m sin(pi kappa) / (pi (kappa + m)), which
 * is the same number because sin(pi (kappa + m)) = (-1)^m sin(pi kappa); it
 * keeps full relative accuracy of every weight when kappa is tiny.  For
 * kappa > 1/2 the sine is taken of pi (1 - kappa), which is exact in FP64,
 * so the weights keep their accuracy as kappa approaches 1 as well. */
void oracle_window_weights(double kappa, int dterms, double* w) {
  double s = (kappa <= 0.5) ? sin(M_PI * kappa) : sin(M_PI * (1.0 - kappa));
  for (int m = -dterms; m < dterms; ++m) {
    double x = kappa + (double)m;
    double v;
    if (x == 0.0)
      v = 1.0;
    else
      v = ((m & 1) ? -s : s) / (M_PI * x);
    w[m + dterms] = v;
  }
}

/* Per-SFT geometry for one sky direction (the canonical operation order). */
static void sft_geometry(const oracle_wu* w, int s, int al, double* tau, double* tdot) {
  const double* r = w->pos + 3 * al;
  const double* v = w->vel + 3 * al;
  const double* n = w->sky + 3 * s;
  double t_mid = w->t_start[al] + 0.5 * w->t_sft;
  double rn = (r[0] * n[0] + r[1] * n[1]) + r[2] * n[2];
  double vn = (v[0] * n[0] + v[1] * n[1]) + v[2] * n[2];
  *tau = (t_mid - w->t_ref) + rn;
  *tdot = 1.0 + vn;
}

/* Bin index, fractional offset and phase of one (template, SFT) pair. */
static void bin_and_phase(const oracle_wu* w, int s, int ifd, int jf, int al, int64_t* kstar,
                          double* kappa, double* phi_frac, double* dphi_out) {
  double f = w->f0 + (double)jf * w->df;
  double fd = w->fdot0 + (double)ifd * w->dfdot;
  double tau, tdot;
  sft_geometry(w, s, al, &tau, &tdot);
  double P = tdot * w->t_sft;
  double q = (fd * tau) * P;
  double dphi = fma(f, P, q);     /* f P + q, rounded once */
  double k = floor(dphi);
  *kstar = (int64_t)k;
  *kappa = dphi - k;
  double phi = tau * (f + (0.5 * fd) * tau);
  *phi_frac = phi - floor(phi);
  if (dphi_out) *dphi_out = dphi;
}

/* A, B, C and D = AB - C^2 of one sky point, summed over all SFTs. */
void oracle_abc(const oracle_wu* w, int s, double* A, double* B, double* C, double* D) {
  double sa = 0, sb = 0, sc = 0;
  for (int al = 0; al < w->n_sft; ++al) {
    double a = w->a[(size_t)s * w->n_sft + al], b = w->b[(size_t)s * w->n_sft + al];
    sa += a * a;
    sb += b * b;
    sc += a * b;
  }
  *A = sa; *B = sb; *C = sc; *D = sa * sb - sc * sc;
}

/* Exported for the bin-selection and phase pins: k*, kappa, frac(phi) and
 * Dphi of every (template, SFT) pair, [n_tmpl][n_sft]. */
int oracle_bins(const oracle_wu* w, int n_tmpl, const int* tsky, const int* tfd, const int* tf,
                int64_t* kstar, double* kappa, double* phi_frac, double* dphi) {
  for (int t = 0; t < n_tmpl; ++t)
    for (int al = 0; al < w->n_sft; ++al) {
      size_t o = (size_t)t * w->n_sft + al;
      bin_and_phase(w, tsky[t], tfd[t], tf[t], al, kstar + o, kappa + o, phi_frac + o, dphi ? dphi + o : 0);
    }
  return ORACLE_OK;
}

/* Demodulated SFT value z for one (template, SFT) pair; returns 0 or
 * ORACLE_E_BAND when the window is not inside the stored band. */
static int demod_one(const oracle_wu* w, int s, int ifd, int jf, int al, double* wbuf, double* zr, double* zi) {
  int64_t kstar;
  double kappa, phi_frac;
  bin_and_phase(w, s, ifd, jf, al, &kstar, &kappa, &phi_frac, 0);
  int D = w->dterms;
  int64_t lo = kstar - D + 1 - w->k_first, hi = kstar + D - w->k_first;
  if (lo < 0 || hi > (int64_t)w->n_bins - 1) return ORACLE_E_BAND;
  oracle_window_weights(kappa, D, wbuf);
  double sr = 0.0, si = 0.0;
  const double* x = w->sft + (size_t)al * w->n_bins * 2;
  for (int m = -D; m < D; ++m) {           /* ascending m */
    int64_t k = kstar - m;
    double sign = (k & 1) ? -1.0 : 1.0;     /* (-1)^(k* - m) */
    int64_t col = k - w->k_first;
    double wt = sign * wbuf[m + D];
    sr += x[2 * col] * wt;
    si += x[2 * col + 1] * wt;
  }
  double c = cos(2.0 * M_PI * phi_frac), sn = sin(2.0 * M_PI * phi_frac);
  /* (sr + i si) * (c - i sn) */
  *zr = sr * c + si * sn;
  *zi = si * c - sr * sn;
  return ORACLE_OK;
}

/* 2F, Fa, Fb for a list of templates (sky, spindown, frequency indices).
 * fa, fb are [n_tmpl][2] or NULL.  On a band error, *bad receives the first
 * failing template (or -1) and ORACLE_E_BAND is returned. */
int oracle_fstat(const oracle_wu* w, int n_tmpl, const int* tsky, const int* tfd, const int* tf,
                 double* twoF, double* fa, double* fb, int nthreads, int* bad) {
  if (!w || w->dterms < 1 || w->n_sft < 1 || w->n_bins < 1) return ORACLE_E_ARG;
  int err_t = -1;
  (void)nthreads;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
  {
    double* wbuf = (double*)malloc(sizeof(double) * 2 * (size_t)w->dterms);
#pragma omp for schedule(dynamic, 16)
    for (int t = 0; t < n_tmpl; ++t) {
      int s = tsky[t];
      double far = 0, fai = 0, fbr = 0, fbi = 0;
      int bad_here = 0;
      for (int al = 0; al < w->n_sft; ++al) {
        double zr, zi;
        if (demod_one(w, s, tfd[t], tf[t], al, wbuf, &zr, &zi) != ORACLE_OK) { bad_here = 1; break; }
        double a = w->a[(size_t)s * w->n_sft + al], b = w->b[(size_t)s * w->n_sft + al];
        far += a * zr; fai += a * zi;
        fbr += b * zr; fbi += b * zi;
      }
      if (bad_here) {
#pragma omp critical
        { if (err_t < 0 || t < err_t) err_t = t; }
        twoF[t] = NAN;
        continue;
      }
      double A, B, C, D;
      oracle_abc(w, s, &A, &B, &C, &D);
      double fa2 = far * far + fai * fai, fb2 = fbr * fbr + fbi * fbi;
      double re_ab = far * fbr + fai * fbi;   /* Re(Fa conj(Fb)) */
      twoF[t] = 2.0 * (B * fa2 + A * fb2 - 2.0 * C * re_ab) / D;
      if (fa) { fa[2 * t] = far; fa[2 * t + 1] = fai; }
      if (fb) { fb[2 * t] = fbr; fb[2 * t + 1] = fbi; }
    }
    free(wbuf);
  }
  if (bad) *bad = err_t;
  return err_t >= 0 ? ORACLE_E_BAND : ORACLE_OK;
}

/*
 * Detector inputs of the demodulation (the step before it; the paper's Cell
 * port notes that most of the data the demodulation reads is produced while
 * the client runs rather than read from the work unit, Section 5): for each SFT
 * the detector position r and velocity v in the solar-system frame
 * (equatorial axes, light-seconds and units of c) and, for each sky direction
 * n, the antenna-pattern factors a, b at the SFT midpoint.
 *
 * Model (plain definitions, one formula per line below):
 *   orbit phase   phi_o = phi_o0 + W_o (t - t0); Earth centre on a circle of
 *                 radius R_o in the ecliptic, tilted by the obliquity eps:
 *                 r_o = R_o (cos phi_o, sin phi_o cos eps, sin phi_o sin eps)
 *   local sidereal angle  th = lon + th0 + W_s (t - t0)
 *   site on a sphere of radius R_e: r_s = R_e (cos lat cos th, cos lat sin th, sin lat)
 *   r = r_o + r_s, v = dr/dt
 *   local east  e = (-sin th, cos th, 0), north  N = (-sin lat cos th, -sin lat sin th, cos lat)
 *   arm directions  u = cos az_x N + sin az_x e,  w = cos az_y N + sin az_y e
 *   detector tensor D = (u u^T - w w^T) / 2
 *   wave frame of n = (cos d cos al, cos d sin al, sin d):
 *     X = (sin al, -cos al, 0),  Y = (-sin d cos al, -sin d sin al, cos d)
 *     (at the poles al = 0)
 *   a = X^T D X - Y^T D Y,  b = 2 X^T D Y   (plus and cross responses)
 */
typedef struct oracle_earth {
  double t0, orbit_radius, orbit_rate, orbit_phase, obliquity, earth_radius, sidereal_rate, sidereal_phase;
} oracle_earth;

typedef struct oracle_site {
  double lat, lon, az_x, az_y;
} oracle_site;

static void quad_form(const double D[3][3], const double* x, const double* y, double* out) {
  double s = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) s += x[i] * D[i][j] * y[j];
  *out = s;
}

int oracle_detector_inputs(const oracle_earth* e, int n_sites, const oracle_site* sites, int n_sft,
                           const double* t_mid, const int* site_of_sft, int n_sky, const double* sky,
                           double* pos, double* vel, double* a, double* b) {
  for (int al = 0; al < n_sft; ++al) {
    const int si = site_of_sft[al];
    if (si < 0 || si >= n_sites) return ORACLE_E_ARG;
    const oracle_site* st = &sites[si];
    const double dt = t_mid[al] - e->t0;
    const double po = e->orbit_phase + e->orbit_rate * dt;
    const double ce = cos(e->obliquity), se = sin(e->obliquity);
    const double th = st->lon + e->sidereal_phase + e->sidereal_rate * dt;
    const double cl = cos(st->lat), sl = sin(st->lat);
    double r[3], v[3];
    r[0] = e->orbit_radius * cos(po);
    r[1] = e->orbit_radius * sin(po) * ce;
    r[2] = e->orbit_radius * sin(po) * se;
    v[0] = -e->orbit_radius * e->orbit_rate * sin(po);
    v[1] = e->orbit_radius * e->orbit_rate * cos(po) * ce;
    v[2] = e->orbit_radius * e->orbit_rate * cos(po) * se;
    r[0] += e->earth_radius * cl * cos(th);
    r[1] += e->earth_radius * cl * sin(th);
    r[2] += e->earth_radius * sl;
    v[0] += -e->earth_radius * e->sidereal_rate * cl * sin(th);
    v[1] += e->earth_radius * e->sidereal_rate * cl * cos(th);
    for (int c = 0; c < 3; ++c) {
      pos[3 * al + c] = r[c];
      vel[3 * al + c] = v[c];
    }
    const double east[3] = {-sin(th), cos(th), 0.0};
    const double north[3] = {-sl * cos(th), -sl * sin(th), cl};
    double u[3], w[3], D[3][3];
    for (int c = 0; c < 3; ++c) {
      u[c] = cos(st->az_x) * north[c] + sin(st->az_x) * east[c];
      w[c] = cos(st->az_y) * north[c] + sin(st->az_y) * east[c];
    }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) D[i][j] = 0.5 * (u[i] * u[j] - w[i] * w[j]);
    for (int s = 0; s < n_sky; ++s) {
      const double* n = sky + 3 * s;
      const double dl = asin(n[2] > 1.0 ? 1.0 : (n[2] < -1.0 ? -1.0 : n[2]));
      const double rho = sqrt(n[0] * n[0] + n[1] * n[1]);
      const double alpha = rho > 0.0 ? atan2(n[1], n[0]) : 0.0;
      const double X[3] = {sin(alpha), -cos(alpha), 0.0};
      const double Y[3] = {-sin(dl) * cos(alpha), -sin(dl) * sin(alpha), cos(dl)};
      double xx, yy, xy;
      quad_form(D, X, X, &xx);
      quad_form(D, Y, Y, &yy);
      quad_form(D, X, Y, &xy);
      a[(size_t)s * n_sft + al] = xx - yy;
      b[(size_t)s * n_sft + al] = 2.0 * xy;
    }
  }
  return ORACLE_OK;
}
