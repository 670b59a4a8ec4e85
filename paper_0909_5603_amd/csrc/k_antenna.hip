// Laser antenna sources in the field update (Sec. 2, second paragraph): the
// pulse enters through a laboratory-fixed plane, which moves at -beta_b in
// the boosted frame.
//
// Two launches per step, for the runs of the table whose antenna is on:
//   phase 0, after the B pass:  B^{n+1/2} -= dt M^n;
//   phase 1, after the E pass and before the Mur ends:  E^{n+1} -= dt J^{n+1/2}.
// The plane moves less than a cell per step (|beta_b dt| < dz), so every
// point whose update straddles it lies within three cells of z'_a(n dt):
// each launch visits that band of 7 z planes times the transverse points
// and the three components, and touches only the straddling points.
#include <hip/hip_runtime.h>

#include "antenna.hpp"
#include "launch.hpp"
#include "pic_dev.hpp"

namespace pic {
namespace {

constexpr int ANT_BAND = 7;

template <typename R>
__global__ __launch_bounds__(256) void k_antenna(const BatchTable* __restrict__ bt, int phase) {
  for (int r = 0; r < bt->n; ++r) {
    RunC& rd = *bt->run[r];
    const long long n = rd.ctr->step;
    if (!ant_on(rd, n)) continue;
    const int fb = rd.ctr->fbuf;
    const int ka = (int)floor(ant_z(rd, (double)n * rd.dt) / rd.dz);
    const long long plane = rd.nperp;
    const long long items = 3LL * ANT_BAND * plane;
    for (long long w = (long long)blockIdx.x * 256 + threadIdx.x; w < items;
         w += (long long)gridDim.x * 256) {
      const int c = (int)(w / (ANT_BAND * plane));
      const long long rem = w - (long long)c * ANT_BAND * plane;
      const int k = ka - 3 + (int)(rem / plane);
      const long long t = rem - (long long)(k - ka + 3) * plane;
      const int i = (int)(t % rd.nx), j = (int)(t / rd.nx);
      const int comp = phase == 0 ? 3 + c : c;
      if (k < 0 || k >= zcount(rd, comp)) continue;
      bool st;
      const double src = ant_source(rd, comp, n, k, i, j, &st);
      if (!st) continue;
      const long long q = gidx(rd, k, i, j);
      PIC_G R* f = phase == 0 ? fptr<R>(rd.B[fb ^ 1][c]) : fptr<R>(rd.E[fb ^ 1][c]);
      f[q] = R((double)f[q] - rd.dt * src);
    }
  }
}

}  // namespace

void launch_antenna(int prec, const BatchTable* bt, long long max_plane, int phase, int grid, hipStream_t s) {
  long long g = (3LL * ANT_BAND * max_plane + 255) / 256;
  g = g < 1 ? 1 : (g > grid ? grid : g);
  if (prec) hipLaunchKernelGGL(k_antenna<double>, dim3((unsigned)g), dim3(256), 0, s, bt, phase);
  else hipLaunchKernelGGL(k_antenna<float>, dim3((unsigned)g), dim3(256), 0, s, bt, phase);
}

}  // namespace pic
