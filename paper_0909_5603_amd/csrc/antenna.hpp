// Laser antenna on the device (Sec. 2, second paragraph): the pulse enters
// the box through a plane that is at rest in the laboratory and therefore
// moves at -beta_b in the boosted frame.
//
// The lab plane z = Z_a sits at z'_a(t') = Z_a / gamma_b - beta_b t'.  The
// grid is made to carry H (E_i, B_i), the boosted incident wave above the
// plane (H = 1 where z' > z'_a, at each point's own staggered z and time)
// and nothing below.  The sources are what the discrete leapfrog needs for
// that:
//   J^{n+1/2} = curl_h (H B_i)^{n+1/2} - ((H E_i)^{n+1} - (H E_i)^n) / dt,
//   M^n = -curl_h (H E_i)^n - ((H B_i)^{n+1/2} - (H B_i)^{n-1/2}) / dt,
// with the Yee differences of the field update, kept only at points whose
// update involves both sides of the plane; E^{n+1} -= dt J^{n+1/2} and
// B^{n+1/2} -= dt M^n.  Integer-time B (the gather's, the diagnostics' and
// the read-back's) stays B^{n-1/2} - dt/2 curl E^n.
//
// The incident wave is the lab pulse (flat phase fronts, Gaussian transverse
// profile and envelope, B = z x E) at the lab event of the point, boosted:
// a forward wave, so its boosted amplitude is D- times the lab one.  The
// plane positions and the H comparisons are evaluated without fused
// multiply-adds, so every launch that recomputes them agrees.
#pragma once

#include "pic_dev.hpp"

namespace pic {

__device__ __forceinline__ double ant_z(RunC& rd, double t) {
#pragma clang fp contract(off)
  return rd.ant_z_lab / rd.gamma_b - rd.beta_b * t;
}

// the antenna acts at level n while its plane is two cells inside the box
__device__ __forceinline__ bool ant_on(RunC& rd, long long n) {
#pragma clang fp contract(off)
  if (!rd.antenna) return false;
  const double za = ant_z(rd, (double)n * rd.dt);
  return za >= 2.0 * rd.dz && za < (rd.nz - 2) * rd.dz;
}

// H times the incident boosted field, component c (0..5) at its point
// (k, i, j) and boosted time t; lo / hi collect the H values seen
__device__ __forceinline__ double ant_hinc(RunC& rd, int c, int k, int i, int j, double t, int& lo, int& hi) {
#pragma clang fp contract(off)
  const double z = (k + 0.5 * stag(c, 0)) * rd.dz;
  const int h = z > ant_z(rd, t) ? 1 : 0;
  lo = h < lo ? h : lo;
  hi = h > hi ? h : hi;
  const int pc = rd.pol_axis - 1;                   // polarised E component
  const int bc = rd.pol_axis == 1 ? 4 : 3;          // its B partner (By or Bx)
  if (!h || (c != pc && c != bc)) return 0.0;
  i = wrapi(i, rd.nx);
  j = rd.dims == 3 ? wrapi(j, rd.ny) : 0;
  const double x = (i + 0.5 * stag(c, 1)) * rd.dx - 0.5 * rd.nx * rd.dx;
  double r2 = x * x;
  if (rd.dims == 3) {
    const double y = (j + 0.5 * stag(c, 2)) * rd.dy - 0.5 * rd.ny * rd.dy;
    r2 += y * y;
  }
  const double g = rd.gamma_b, b = rd.beta_b;
  const double zl = g * (z + b * t), tl = g * (t + b * z);
  const double zeta = zl - rd.ant_z_lab - (tl - rd.ant_t_peak);
  const double amp = rd.E0_lab * exp(-r2 / (rd.waist * rd.waist)) *
                     exp(-zeta * zeta / (rd.L_lab * rd.L_lab)) * cos(rd.k0_lab * zeta);
  // boosted forward wave: E' = D- E along the polarisation, B' = z x E'
  const double e = rd.dminus * amp;
  return (c == bc && rd.pol_axis == 2) ? -e : e;
}

// J^{n+1/2} (c = 0..2) or M^n (c = 3..5) at (k, i, j); *straddle tells
// whether the point's update involves both sides of the plane
__device__ __forceinline__ double ant_source(RunC& rd, int c, long long n, int k, int i, int j,
                                             bool* straddle) {
#pragma clang fp contract(off)
  *straddle = false;
  if (!ant_on(rd, n)) return 0.0;
  const double dt = rd.dt;
  const double z = (k + 0.5 * stag(c, 0)) * rd.dz;
  if (fabs(z - ant_z(rd, (double)n * dt)) > 3.0 * rd.dz) return 0.0;
  const double idz = 1.0 / rd.dz, idx = 1.0 / rd.dx, idy = rd.dims == 3 ? 1.0 / rd.dy : 0.0;
  int lo = 1, hi = 0;
  double r;
  if (c < 3) {
    const double th = ((double)n + 0.5) * dt, t0 = (double)n * dt, t1 = (double)(n + 1) * dt;
    double curl;
    if (c == 0)
      curl = (ant_hinc(rd, 5, k, i, j, th, lo, hi) - ant_hinc(rd, 5, k, i, j - 1, th, lo, hi)) * idy -
             (ant_hinc(rd, 4, k, i, j, th, lo, hi) - ant_hinc(rd, 4, k - 1, i, j, th, lo, hi)) * idz;
    else if (c == 1)
      curl = (ant_hinc(rd, 3, k, i, j, th, lo, hi) - ant_hinc(rd, 3, k - 1, i, j, th, lo, hi)) * idz -
             (ant_hinc(rd, 5, k, i, j, th, lo, hi) - ant_hinc(rd, 5, k, i - 1, j, th, lo, hi)) * idx;
    else
      curl = (ant_hinc(rd, 4, k, i, j, th, lo, hi) - ant_hinc(rd, 4, k, i - 1, j, th, lo, hi)) * idx -
             (ant_hinc(rd, 3, k, i, j, th, lo, hi) - ant_hinc(rd, 3, k, i, j - 1, th, lo, hi)) * idy;
    const double e1 = ant_hinc(rd, c, k, i, j, t1, lo, hi), e0 = ant_hinc(rd, c, k, i, j, t0, lo, hi);
    r = curl - (e1 - e0) / dt;
  } else {
    const double t0 = (double)n * dt, tm = ((double)n - 0.5) * dt, tq = ((double)n + 0.5) * dt;
    double curl;
    if (c == 3)
      curl = (ant_hinc(rd, 2, k, i, j + 1, t0, lo, hi) - ant_hinc(rd, 2, k, i, j, t0, lo, hi)) * idy -
             (ant_hinc(rd, 1, k + 1, i, j, t0, lo, hi) - ant_hinc(rd, 1, k, i, j, t0, lo, hi)) * idz;
    else if (c == 4)
      curl = (ant_hinc(rd, 0, k + 1, i, j, t0, lo, hi) - ant_hinc(rd, 0, k, i, j, t0, lo, hi)) * idz -
             (ant_hinc(rd, 2, k, i + 1, j, t0, lo, hi) - ant_hinc(rd, 2, k, i, j, t0, lo, hi)) * idx;
    else
      curl = (ant_hinc(rd, 1, k, i + 1, j, t0, lo, hi) - ant_hinc(rd, 1, k, i, j, t0, lo, hi)) * idx -
             (ant_hinc(rd, 0, k, i, j + 1, t0, lo, hi) - ant_hinc(rd, 0, k, i, j, t0, lo, hi)) * idy;
    const double b1 = ant_hinc(rd, c, k, i, j, tq, lo, hi), b0 = ant_hinc(rd, c, k, i, j, tm, lo, hi);
    r = -curl - (b1 - b0) / dt;
  }
  *straddle = lo != hi;
  return lo != hi ? r : 0.0;
}

}  // namespace pic
