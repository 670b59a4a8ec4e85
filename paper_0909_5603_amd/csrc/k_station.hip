// Laboratory-frame stations (Sec. 2: the boosted-frame run is diagnosed at
// stations immobile in the laboratory, sampled at a succession of lab times,
// with interpolation because lab events do not fall on the boosted grid).
//
// Station q is the plane z_lab = Z_q.  At boosted time t' = n dt it sits at
// z' = Z_q / gamma_b - beta_b t' (z_lab = gamma_b (z' + beta_b t')), and the
// event it samples has lab time t_lab = gamma_b (t' + beta_b z') =
// t' / gamma_b + beta_b Z_q.  On every step whose z' lies in [0, nz dz) the
// station takes E^n and B^n at z' on its transverse sample points: each
// component linearly interpolated in z between its own staggered points, B
// advanced from the stored B^{n-1/2} by half a step on the fly
// (B^n = B^{n-1/2} - dt/2 curl E^n), then transformed back to the
// laboratory with the boost of velocity -beta_b.
//
// Two launches per step, before the step advance flips the field buffers:
// k_station writes sample number st_count[q] of every station in range,
// k_station_count then increments the counts.  The work is a few loads per
// sample point, negligible next to the particle kernel; it is enumerated as
// one flat range per run, visited run by run, with the arithmetic in FP64
// for both precisions.
#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "pic_dev.hpp"

namespace pic {
namespace {

// boosted-frame position of station q at step n, and whether it is inside
// (unfused multiply-adds: both launches of a step take the same decision)
__device__ __forceinline__ bool station_z(RunC& rd, int q, long long n, double& zp, double& tp,
                                          double& Z) {
#pragma clang fp contract(off)
  tp = (double)n * rd.dt;
  Z = rd.st_z0 + q * rd.st_dz;
  zp = Z / rd.gamma_b - rd.beta_b * tp;
  return zp >= 0.0 && zp < rd.nz * rd.dz;
}

__device__ __forceinline__ double lab_time(double tp, double g, double b, double Z) {
#pragma clang fp contract(off)
  return tp / g + b * Z;
}

// B^n of component c (0..2) at z index k and transverse node (i, j): zero
// outside the component's range on an open z axis
template <typename R>
__device__ __forceinline__ double b_int(RunC& rd, R* const* E, R* const* B, int c, int k, int i, int j) {
  if (rd.open) {
    if (k < 0 || k >= zcount(rd, 3 + c)) return 0.0;
  } else {
    k = wrapi(k, rd.nz);
  }
  return (double)B[c][gidx(rd, k, i, j)] - 0.5 * rd.dt * curl_e(rd, E, c, k, i, j);
}

template <typename R>
__global__ __launch_bounds__(256) void k_station(const BatchTable* __restrict__ bt) {
  for (int r = 0; r < bt->n; ++r) {
    RunC& rd = *bt->run[r];
    if (rd.n_stations <= 0) continue;
    const long long n = rd.ctr->step;
    const int fb = rd.ctr->fbuf;
    R* const* E = reinterpret_cast<R* const*>(rd.E[fb]);
    R* const* B = reinterpret_cast<R* const*>(rd.B[fb]);
    const int nxs = rd.st_nxs, per = nxs * rd.st_nys;
    const long long items = (long long)rd.n_stations * per;
    const long long cap = rd.st_cap;
    for (long long w = (long long)blockIdx.x * 256 + threadIdx.x; w < items;
         w += (long long)gridDim.x * 256) {
      const int q = (int)(w / per);
      const int rem = (int)(w - (long long)q * per);
      const int js = rem / nxs, is = rem - js * nxs;
      double zp, tp, Z;
      if (!station_z(rd, q, n, zp, tp, Z)) continue;
      const long long t = rd.st_count[q];
      if (t >= cap) continue;
      const int i = is * rd.st_stride, j = js * rd.st_stride;
      double f[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const double u = zp / rd.dz - 0.5 * stag(c, 0);
        const int k = (int)floor(u);
        const double a = u - k;
        const double v0 = c < 3 ? ev(rd, E, c, k, i, j) : b_int(rd, E, B, c - 3, k, i, j);
        const double v1 = c < 3 ? ev(rd, E, c, k + 1, i, j) : b_int(rd, E, B, c - 3, k + 1, i, j);
        f[c] = (1.0 - a) * v0 + a * v1;
      }
      // back to the laboratory: boost of velocity -beta_b along z
      const double g = rd.gamma_b, b = rd.beta_b;
      const double lab[6] = {g * (f[0] + b * f[4]), g * (f[1] - b * f[3]), f[2],
                             g * (f[3] - b * f[1]), g * (f[4] + b * f[0]), f[5]};
      PIC_G double* out = rd.st_data + ((long long)q * cap + t) * 6 * per + rem;
#pragma unroll
      for (int c = 0; c < 6; ++c) out[(long long)c * per] = lab[c];
      if (rem == 0) rd.st_time[(long long)q * cap + t] = lab_time(tp, g, b, Z);
    }
  }
}

__global__ __launch_bounds__(256) void k_station_count(const BatchTable* __restrict__ bt) {
  for (int r = 0; r < bt->n; ++r) {
    RunC& rd = *bt->run[r];
    if (rd.n_stations <= 0) continue;
    const long long n = rd.ctr->step;
    for (int q = blockIdx.x * 256 + threadIdx.x; q < rd.n_stations; q += gridDim.x * 256) {
      double zp, tp, Z;
      if (station_z(rd, q, n, zp, tp, Z)) rd.st_count[q] += 1;
    }
  }
}

}  // namespace

void launch_stations(int prec, const BatchTable* bt, long long max_items, int grid, hipStream_t s) {
  long long g = (max_items + 255) / 256;
  g = g < 1 ? 1 : (g > grid ? grid : g);
  if (prec) hipLaunchKernelGGL(k_station<double>, dim3((unsigned)g), dim3(256), 0, s, bt);
  else hipLaunchKernelGGL(k_station<float>, dim3((unsigned)g), dim3(256), 0, s, bt);
  hipLaunchKernelGGL(k_station_count, dim3(1), dim3(256), 0, s, bt);
}

}  // namespace pic
