// Initial boosted-frame fields and the diagnostics kernels.
//
// Laser (Sec. 2, second paragraph: laser parameters are given in the
// laboratory and the waves are Doppler shifted in the boosted frame): every
// Yee point (z', x, y) of the boosted grid at t' = 0 corresponds to the
// laboratory event z = gamma_b z', t = gamma_b beta_b z'.  The laboratory
// pulse (flat phase fronts, Gaussian transverse profile and envelope, B =
// z x E) is evaluated there in FP64 and the fields are boosted with the
// Lorentz field transformation, then stored in the run's precision.  B is
// then moved back half a step to B^{-1/2}, the leapfrog state.
//
// Diagnostics run outside the step loop and accumulate in FP64.
#include <hip/hip_runtime.h>

#include "antenna.hpp"
#include "launch.hpp"
#include "pic_dev.hpp"

namespace pic {

// ------------------------------------------------------------------ laser
template <typename R>
__global__ void k_laser(const RunDev* __restrict__ rdp) {
  RunC& rd = *(RunC*)rdp;
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= rd.npts) return;
  const int k = (int)(q % rd.nzf);
  const long long t = q / rd.nzf;
  const int i = (int)(t % rd.nx), j = (int)(t / rd.nx);
  const double gb = rd.gamma_b, bb = rd.beta_b;
  const double Lx = rd.nx * rd.dx, Ly = rd.ny * rd.dy;
  for (int c = 0; c < 6; ++c) {
    const int kmax = rd.open ? (stag(c, 0) ? rd.nz : rd.nz + 1) : rd.nz;
    R val = R(0);
    if (k < kmax) {
      const double zp = (k + 0.5 * stag(c, 0)) * rd.dz;
      const double x = (i + 0.5 * stag(c, 1)) * rd.dx;
      const double y = rd.dims == 3 ? (j + 0.5 * stag(c, 2)) * rd.dy : 0.0;
      // laboratory event of the boosted point at t' = 0
      const double zl = gb * zp, tl = gb * bb * zp;
      const double zeta = zl - rd.dminus * rd.zc_boost - tl;
      double r2 = (x - 0.5 * Lx) * (x - 0.5 * Lx);
      if (rd.dims == 3) r2 += (y - 0.5 * Ly) * (y - 0.5 * Ly);
      const double amp = rd.E0_lab * exp(-r2 / (rd.waist * rd.waist)) *
                         exp(-zeta * zeta / (rd.L_lab * rd.L_lab)) * cos(rd.k0_lab * zeta);
      double E[3] = {0, 0, 0}, B[3] = {0, 0, 0};
      if (rd.pol_axis == 1) {
        E[0] = amp;
        B[1] = amp;
      } else {
        E[1] = amp;
        B[0] = -amp;
      }
      // field boost along +z
      double v;
      switch (c) {
        case 0: v = gb * (E[0] - bb * B[1]); break;
        case 1: v = gb * (E[1] + bb * B[0]); break;
        case 2: v = E[2]; break;
        case 3: v = gb * (B[0] + bb * E[1]); break;
        case 4: v = gb * (B[1] - bb * E[0]); break;
        default: v = B[2]; break;
      }
      if (rd.antenna) {
        // antenna: the incident wave above the plane only; a B point whose
        // first update straddles the plane starts at (H B_i)^{-1/2} - dt/2
        // curl_h (H E_i)^0 (the mean of H B_i at t' = -dt/2 and dt/2 plus
        // dt/2 M^0), so that B^{-1/2} = B^0 + dt/2 curl E^0 is H B_i there
        int lo = 1, hi = 0;
        bool st = false;
        double m0 = 0.0;
        if (c >= 3) m0 = ant_source(rd, c, 0, k, i, j, &st);
        if (st) {
          const double h = 0.5 * rd.dt;
          v = 0.5 * (ant_hinc(rd, c, k, i, j, -h, lo, hi) + ant_hinc(rd, c, k, i, j, h, lo, hi)) + h * m0;
        } else {
          v = ant_hinc(rd, c, k, i, j, 0.0, lo, hi);
        }
      }
      val = R(v);
    }
    if (c < 3)
      fptr<R>(rd.E[0][c])[q] = val;
    else
      fptr<R>(rd.B[0][c - 3])[q] = val;
  }
}

// B^{n+s dt} from B at the stored time: out = B + coef * curl E (valid points)
template <typename R>
__global__ void k_bshift(const RunDev* __restrict__ rdp, int src, int dst, double coef) {
  RunC& rd = *(RunC*)rdp;
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= rd.npts) return;
  const int k = (int)(q % rd.nzf);
  const long long t = q / rd.nzf;
  const int i = (int)(t % rd.nx), j = (int)(t / rd.nx);
  const int fb = rd.ctr->fbuf;
  R* const* E = reinterpret_cast<R* const*>(rd.E[fb]);
  const int bs = src < 0 ? fb : src, bd = dst < 0 ? (fb ^ 1) : dst;
  for (int c = 0; c < 3; ++c) {
    const bool valid = !rd.open || k < zcount(rd, 3 + c);
    double v = 0.0;
    if (valid) v = (double)fptr<R>(rd.B[bs][c])[q] + coef * curl_e(rd, E, c, k, i, j);
    fptr<R>(rd.B[bd][c])[q] = R(v);
  }
}

void launch_init_fields(int dims, int prec, const RunDev* rd, long long npts, hipStream_t s) {
  (void)dims;
  const int B = 256;
  const unsigned G = (unsigned)((npts + B - 1) / B);
  if (prec) {
    hipLaunchKernelGGL(k_laser<double>, dim3(G), dim3(B), 0, s, rd);
  } else {
    hipLaunchKernelGGL(k_laser<float>, dim3(G), dim3(B), 0, s, rd);
  }
}

// ------------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m));
  return v;
}
// block (256 threads) reductions; result valid in thread 0
__device__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return r;
}
__device__ double block_max(double v, double* sh) {
  v = wave_max(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
  __syncthreads();
  return r;
}

__device__ __forceinline__ bool interior(RunC& rd, int comp, int k) {
  if (!rd.open) return true;
  const int hi = stag(comp, 0) ? rd.nz - 3 : rd.nz - 2;
  return k >= 2 && k <= hi;
}

__global__ void k_fill(double* p, long long n, double v) {
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (long long)gridDim.x * blockDim.x)
    p[q] = v;
}

// ------------------------------------------------------------------ charge
// electron charge density on nodes (linear shape), FP64 atomics.  With
// use_snap, liveness is taken from the snapshot of the cells before the
// step, so particles removed during the step still count at their new
// position.
template <int DIM, typename R>
__global__ void k_rho(const RunDev* __restrict__ rdp, double* rho, int use_snap) {
  RunC& rd = *(RunC*)rdp;
  const PIC_G Counters& c = *rd.ctr;
  const int pb = c.pbuf;
  const double qw = -rd.weight;
  double dv = rd.dz * rd.dx * (DIM == 3 ? rd.dy : 1.0);
  const double s = qw / dv;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < c.n_slots;
       q += (long long)gridDim.x * blockDim.x) {
    const int cc = rd.cell[pb][q];
    const bool live = use_snap ? (rd.cell_snap[q] >= 0) : (cc >= 0);
    if (!live) continue;
    const int cu = cc & 0x7fffffff;
    const int k = cell_k(cu), i = cell_i(cu), j = DIM == 3 ? cell_j(cu) : 0;
    const double oz = (double)fptr<R>(rd.off[pb][0])[q];
    const double ox = (double)fptr<R>(rd.off[pb][1])[q];
    const double oy = DIM == 3 ? (double)fptr<R>(rd.off[pb][2])[q] : 0.0;
    const double wz[2] = {1.0 - oz, oz}, wx[2] = {1.0 - ox, ox}, wy[2] = {1.0 - oy, oy};
    for (int cy = 0; cy < (DIM == 3 ? 2 : 1); ++cy)
      for (int cx = 0; cx < 2; ++cx)
        for (int cz = 0; cz < 2; ++cz) {
          int kk = k + cz;
          const int ii = wrapi(i + cx, rd.nx), jj = DIM == 3 ? wrapi(j + cy, rd.ny) : 0;
          if (rd.open) {
            if (kk < 0 || kk > rd.nz) continue;
          } else {
            kk = wrapi(kk, rd.nz);
          }
          const double wgt = wz[cz] * wx[cx] * (DIM == 3 ? wy[cy] : 1.0);
          g_add((PIC_G double*)rho + gidx(rd, kk, ii, jj), s * wgt);
        }
  }
}

__global__ void k_snap(const RunDev* __restrict__ rdp) {
  RunC& rd = *(RunC*)rdp;
  const PIC_G Counters& c = *rd.ctr;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < c.n_slots;
       q += (long long)gridDim.x * blockDim.x)
    rd.cell_snap[q] = rd.cell[c.pbuf][q];
}

// divergence at node (k,i,j) of a field staggered like E
template <typename R>
__device__ __forceinline__ double div_e(RunC& rd, R* const* F, int k, int i, int j) {
  const double idz = 1.0 / rd.dz, idx = 1.0 / rd.dx, idy = rd.dims == 3 ? 1.0 / rd.dy : 0.0;
  return (ev(rd, F, 0, k, i, j) - ev(rd, F, 0, k, i - 1, j)) * idx +
         (ev(rd, F, 1, k, i, j) - ev(rd, F, 1, k, i, j - 1)) * idy +
         (ev(rd, F, 2, k, i, j) - ev(rd, F, 2, k - 1, i, j)) * idz;
}

// divergence of the fixed-point current at node (k,i,j), in units of 1/jscale
__device__ __forceinline__ double jv(RunC& rd, const long long* const* J, int c, int k, int i, int j) {
  i = wrapi(i, rd.nx);
  j = rd.dims == 3 ? wrapi(j, rd.ny) : 0;
  if (rd.open) {
    if (k < 0 || k >= zcount(rd, c)) return 0.0;
  } else {
    k = wrapi(k, rd.nz);
  }
  return (double)J[c][gidx(rd, k, i, j)];
}
__device__ __forceinline__ double div_j(RunC& rd, const long long* const* J, int k, int i, int j) {
  const double idz = 1.0 / rd.dz, idx = 1.0 / rd.dx, idy = rd.dims == 3 ? 1.0 / rd.dy : 0.0;
  return (jv(rd, J, 0, k, i, j) - jv(rd, J, 0, k, i - 1, j)) * idx +
         (jv(rd, J, 1, k, i, j) - jv(rd, J, 1, k, i, j - 1)) * idy +
         (jv(rd, J, 2, k, i, j) - jv(rd, J, 2, k - 1, i, j)) * idz;
}

// continuity residual |rho_b - rho_a + dt div J| and |rho_a| maxima (interior nodes)
template <typename R>
__global__ __launch_bounds__(256) void k_cont(const RunDev* __restrict__ rdp) {
  __shared__ double sh[4];
  RunC& rd = *(RunC*)rdp;
  const long long* const* J = reinterpret_cast<const long long* const*>(rd.J[rd.ctr->fbuf]);
  double res = 0.0, rmax = 0.0;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < rd.npts;
       q += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(q % rd.nzf);
    const long long t = q / rd.nzf;
    const int i = (int)(t % rd.nx), j = (int)(t / rd.nx);
    if (rd.open && k > rd.nz) continue;
    if (!interior(rd, 0, k)) continue;
    const double d = rd.rho_b[q] - rd.rho_a[q] + rd.dt * rd.jinv * div_j(rd, J, k, i, j);
    res = fmax(res, fabs(d));
    rmax = fmax(rmax, fabs(rd.rho_a[q]));
  }
  res = block_max(res, sh);
  rmax = block_max(rmax, sh);
  if (threadIdx.x == 0) {
    atomic_max_pos(&rd.ctr->cont_res_bits, res);
    atomic_max_pos(&rd.ctr->cont_rho_bits, rmax);
  }
}

__global__ void k_cont_fin(const RunDev* __restrict__ rdp) {
  PIC_G Counters* c = rdp->ctr;
  const double res = __longlong_as_double((long long)c->cont_res_bits);
  const double rho = __longlong_as_double((long long)c->cont_rho_bits);
  const double rel = rho > 0 ? res / rho : res;
  if (rel > c->cont_max) c->cont_max = rel;
  c->cont_res_bits = 0;
  c->cont_rho_bits = 0;
}

template <typename R>
__global__ void k_jlast(const RunDev* __restrict__ rdp) {
  RunC& rd = *(RunC*)rdp;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < rd.npts;
       q += (long long)gridDim.x * blockDim.x)
    for (int c = 0; c < 3; ++c)
      rd.jlast[c][q] = (double)reinterpret_cast<const long long*>(rd.J[rd.ctr->fbuf][c])[q] * rd.jinv;
}

// ------------------------------------------------------------------ filter
// One stage of the current filter applied to a node scalar (the electron
// density of the filtered Gauss diagnostic): the same passes, weights and
// open-end rule as the current's, with the z range of a node-type component.
template <int DIM>
__global__ __launch_bounds__(256) void k_filter_nodes(const RunDev* __restrict__ rdp, const double* src,
                                                      double* dst, int stage) {
  RunC& rd = *(RunC*)rdp;
  constexpr int NAX = DIM == 3 ? 3 : 2;
  const int axis = stage % NAX;
  const bool cpass = stage >= rd.filter_passes * NAX;
  const double ws = cpass ? -0.25 * rd.filter_passes : 0.25;
  const double wm = cpass ? 1.0 + 0.5 * rd.filter_passes : 0.5;
  const int zc = rd.open ? rd.nz + 1 : rd.nz;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < rd.npts;
       q += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(q % rd.nzf);
    const long long t = q / rd.nzf;
    const int i = (int)(t % rd.nx), j = (int)(t / rd.nx);
    if (k >= zc) {
      dst[q] = 0.0;
      continue;
    }
    double lo, hi;
    if (axis == 0) {
      if (rd.open) {
        lo = k > 0 ? src[q - 1] : src[q];  // beyond an end: the end value
        hi = k + 1 < zc ? src[q + 1] : src[q];
      } else {
        lo = src[gidx(rd, wrapi(k - 1, rd.nz), i, j)];
        hi = src[gidx(rd, wrapi(k + 1, rd.nz), i, j)];
      }
    } else if (axis == 1) {
      lo = src[gidx(rd, k, wrapi(i - 1, rd.nx), j)];
      hi = src[gidx(rd, k, wrapi(i + 1, rd.nx), j)];
    } else {
      lo = src[gidx(rd, k, i, wrapi(j - 1, rd.ny))];
      hi = src[gidx(rd, k, i, wrapi(j + 1, rd.ny))];
    }
    dst[q] = wm * src[q] + ws * (lo + hi);
  }
}

// ------------------------------------------------------------------ Gauss
// mode 0: store G0 = div E - rhoG - rho_ion and max|rho_e| (interior);
// mode 1: max |G - G0| over interior nodes into amax[1].  rhoG is the
// electron density, filtered like the current when the filter is on.
template <typename R>
__global__ __launch_bounds__(256) void k_gauss(const RunDev* __restrict__ rdp, int mode, const double* rhoG) {
  __shared__ double sh[4];
  RunC& rd = *(RunC*)rdp;
  R* const* E = reinterpret_cast<R* const*>(rd.E[rd.ctr->fbuf]);
  double m = 0.0;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < rd.npts;
       q += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(q % rd.nzf);
    const long long t = q / rd.nzf;
    const int i = (int)(t % rd.nx), j = (int)(t / rd.nx);
    if (rd.open && k > rd.nz) continue;
    const double G = div_e(rd, E, k, i, j) - rhoG[q] - rd.rho_ion;
    if (mode == 0) {
      rd.gauss0[q] = G;
      if (interior(rd, 0, k)) m = fmax(m, fabs(rd.rho_a[q]));
    } else if (interior(rd, 0, k)) {
      m = fmax(m, fabs(G - rd.gauss0[q]));
    }
  }
  m = block_max(m, sh);
  if (threadIdx.x == 0) {
    if (mode == 0)
      atomic_max_pos((PIC_G unsigned long long*)&rd.ctr->rho0_max, m);
    else
      atomic_max_pos(&rd.ctr->amax[1], m);
  }
}

// ------------------------------------------------------------------ energies
template <typename R>
__global__ __launch_bounds__(256) void k_diag_fields(const RunDev* __restrict__ rdp) {
  __shared__ double sh[4];
  RunC& rd = *(RunC*)rdp;
  const int fb = rd.ctr->fbuf;
  R* const* E = reinterpret_cast<R* const*>(rd.E[fb]);
  double ue = 0.0, ub = 0.0, ezm = 0.0;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < rd.npts;
       q += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(q % rd.nzf);
    const long long t = q / rd.nzf;
    const int i = (int)(t % rd.nx), j = (int)(t / rd.nx);
    for (int c = 0; c < 3; ++c) {
      if (rd.open && k >= zcount(rd, c)) continue;
      if (!interior(rd, c, k)) continue;
      const double e = (double)E[c][q];
      ue += e * e;
      if (c == 2) ezm = fmax(ezm, fabs(e));
    }
    for (int c = 0; c < 3; ++c) {
      if (rd.open && k >= zcount(rd, 3 + c)) continue;
      if (!interior(rd, 3 + c, k)) continue;
      const double b = (double)fptr<R>(rd.B[fb][c])[q] - 0.5 * rd.dt * curl_e(rd, E, c, k, i, j);
      ub += b * b;
    }
  }
  ue = block_sum(ue, sh);
  ub = block_sum(ub, sh);
  ezm = block_max(ezm, sh);
  if (threadIdx.x == 0) {
    const double dv = rd.dz * rd.dx * (rd.dims == 3 ? rd.dy : 1.0);
    g_add(&rd.ctr->acc[0], 0.5 * ue * dv);
    g_add(&rd.ctr->acc[1], 0.5 * ub * dv);
    atomic_max_pos(&rd.ctr->amax[0], ezm);
  }
}

template <int DIM, typename R>
__global__ __launch_bounds__(256) void k_diag_particles(const RunDev* __restrict__ rdp) {
  __shared__ double sh[4];
  RunC& rd = *(RunC*)rdp;
  const PIC_G Counters& c = *rd.ctr;
  const int pb = c.pbuf;
  double ke = 0.0, cnt = 0.0;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < c.n_slots;
       q += (long long)gridDim.x * blockDim.x) {
    const int cc = rd.cell[pb][q];
    if (cc < 0) continue;
    const int k = cell_k(cc);
    const double z = k + (double)fptr<R>(rd.off[pb][0])[q];
    const bool inbox = !rd.open || (z >= 0.0 && z < rd.nz);
    const bool inner = !rd.open || (z >= 2.0 && z < rd.nz - 2);
    if (inbox) cnt += 1.0;
    if (inner) {
      const double ux = (double)fptr<R>(rd.u[pb][0])[q], uy = (double)fptr<R>(rd.u[pb][1])[q];
      const double uz = (double)fptr<R>(rd.u[pb][2])[q];
      ke += rd.weight * (sqrt(1.0 + ux * ux + uy * uy + uz * uz) - 1.0);
    }
  }
  ke = block_sum(ke, sh);
  cnt = block_sum(cnt, sh);
  if (threadIdx.x == 0) {
    g_add(&rd.ctr->acc[2], ke);
    g_add(&rd.ctr->acc[3], cnt);
  }
}

// ------------------------------------------------------------------ launches
static unsigned gridfor(long long n, int B, unsigned cap = 65536) {
  long long g = (n + B - 1) / B;
  if (g < 1) g = 1;
  return (unsigned)(g > cap ? cap : g);
}

void launch_cont_pre(int dims, int prec, const RunDev* rd, long long npts, long long cap, hipStream_t s) {
  (void)dims;
  (void)prec;
  hipLaunchKernelGGL(k_snap, dim3(gridfor(cap, 256)), dim3(256), 0, s, rd);
}

// the rho arrays are passed by the host (their device addresses)
void launch_rho(int dims, int prec, const RunDev* rd, double* rho, long long npts, long long cap,
                int use_snap, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(gridfor(npts, 256)), dim3(256), 0, s, rho, npts, 0.0);
  const unsigned g = gridfor(cap, 256);
  if (dims == 3) {
    if (prec) hipLaunchKernelGGL((k_rho<3, double>), dim3(g), dim3(256), 0, s, rd, rho, use_snap);
    else hipLaunchKernelGGL((k_rho<3, float>), dim3(g), dim3(256), 0, s, rd, rho, use_snap);
  } else {
    if (prec) hipLaunchKernelGGL((k_rho<2, double>), dim3(g), dim3(256), 0, s, rd, rho, use_snap);
    else hipLaunchKernelGGL((k_rho<2, float>), dim3(g), dim3(256), 0, s, rd, rho, use_snap);
  }
}

void launch_cont_post(int dims, int prec, const RunDev* rd, long long npts, long long cap, hipStream_t s) {
  (void)dims;
  (void)cap;
  const unsigned g = gridfor(npts, 256, 4096);
  if (prec) {
    hipLaunchKernelGGL(k_cont<double>, dim3(g), dim3(256), 0, s, rd);
    hipLaunchKernelGGL(k_jlast<double>, dim3(gridfor(npts, 256)), dim3(256), 0, s, rd);
  } else {
    hipLaunchKernelGGL(k_cont<float>, dim3(g), dim3(256), 0, s, rd);
    hipLaunchKernelGGL(k_jlast<float>, dim3(gridfor(npts, 256)), dim3(256), 0, s, rd);
  }
  hipLaunchKernelGGL(k_cont_fin, dim3(1), dim3(1), 0, s, rd);
}

void launch_gauss(int prec, const RunDev* rd, long long npts, int mode, const double* rhoG, hipStream_t s) {
  const unsigned g = gridfor(npts, 256, 4096);
  if (prec) hipLaunchKernelGGL(k_gauss<double>, dim3(g), dim3(256), 0, s, rd, mode, rhoG);
  else hipLaunchKernelGGL(k_gauss<float>, dim3(g), dim3(256), 0, s, rd, mode, rhoG);
}

const double* launch_filter_nodes(int dims, const RunDev* rd, long long npts, int stages, const double* rho,
                                  double* t0, double* t1, hipStream_t s) {
  const unsigned g = gridfor(npts, 256, 4096);
  const double* src = rho;
  for (int st = 0; st < stages; ++st) {
    double* dst = (st & 1) ? t1 : t0;
    if (dims == 3) hipLaunchKernelGGL(k_filter_nodes<3>, dim3(g), dim3(256), 0, s, rd, src, dst, st);
    else hipLaunchKernelGGL(k_filter_nodes<2>, dim3(g), dim3(256), 0, s, rd, src, dst, st);
    src = dst;
  }
  return src;
}

void launch_diag(int dims, int prec, const RunDev* rd, long long npts, long long cap, unsigned what,
                 hipStream_t s) {
  if (what & 1u) {
    const unsigned g = gridfor(npts, 256, 4096);
    if (prec) hipLaunchKernelGGL(k_diag_fields<double>, dim3(g), dim3(256), 0, s, rd);
    else hipLaunchKernelGGL(k_diag_fields<float>, dim3(g), dim3(256), 0, s, rd);
  }
  if (what & 2u) {
    const unsigned g = gridfor(cap, 256, 4096);
    if (dims == 3) {
      if (prec) hipLaunchKernelGGL((k_diag_particles<3, double>), dim3(g), dim3(256), 0, s, rd);
      else hipLaunchKernelGGL((k_diag_particles<3, float>), dim3(g), dim3(256), 0, s, rd);
    } else {
      if (prec) hipLaunchKernelGGL((k_diag_particles<2, double>), dim3(g), dim3(256), 0, s, rd);
      else hipLaunchKernelGGL((k_diag_particles<2, float>), dim3(g), dim3(256), 0, s, rd);
    }
  }
}

void launch_bshift(int prec, const RunDev* rd, long long npts, int src, int dst, double coef,
                   hipStream_t s) {
  const unsigned g = gridfor(npts, 256, 1u << 30);
  if (prec) hipLaunchKernelGGL(k_bshift<double>, dim3(g), dim3(256), 0, s, rd, src, dst, coef);
  else hipLaunchKernelGGL(k_bshift<float>, dim3(g), dim3(256), 0, s, rd, src, dst, coef);
}

}  // namespace pic
