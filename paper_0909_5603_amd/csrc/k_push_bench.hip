// Pusher microbenchmark: n particles, each in its own uniform field, one
// step per launch.  Sec. 2 (first paragraph): the modified Lorentz-force
// pusher cancels E by v x B exactly where the Boris pusher does not.
// Positions are an int32 cell plus an offset in [0,1) on a unit grid.
#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "pusher.hpp"

namespace pic {

template <typename R, int PUSHER>
__global__ __launch_bounds__(256) void k_push_bench(long long n, R dt, R bx, R by, R bz,
                                                    const R* __restrict__ Ex, R* __restrict__ u,
                                                    int* __restrict__ cell, R* __restrict__ off) {
  const R eps = R(-0.5) * dt;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (long long)gridDim.x * blockDim.x) {
    R ux = u[p], uy = u[n + p], uz = u[2 * n + p];
    const R ex = Ex[p];
    if (PUSHER == 1)
      push_boris<R>(ux, uy, uz, ex, R(0), R(0), bx, by, bz, eps);
    else
      push_vay<R>(ux, uy, uz, ex, R(0), R(0), bx, by, bz, eps);
    const R ig = frsq(R(1) + ux * ux + uy * uy + uz * uz);
    const R v[3] = {ux * ig, uy * ig, uz * ig};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      R o = off[d * n + p] + dt * v[d];
      int c = 0;
      if (o < R(0)) {
        o += R(1);
        c = -1;
        if (o >= R(1)) {
          o = R(0);
          c = 0;
        }
      } else if (o >= R(1)) {
        o -= R(1);
        c = 1;
      }
      off[d * n + p] = o;
      if (c) cell[d * n + p] += c;
    }
    u[p] = ux;
    u[n + p] = uy;
    u[2 * n + p] = uz;
  }
}

void launch_push_bench(int prec, int pusher, long long n, double dt, const double B[3], void* Ex,
                       void* u, int* cell, void* off, hipStream_t s) {
  long long g = (n + 255) / 256;
  if (g > 256 * 64) g = 256 * 64;
  if (g < 1) g = 1;
  if (prec) {
    auto k = pusher ? k_push_bench<double, 1> : k_push_bench<double, 0>;
    hipLaunchKernelGGL(k, dim3((unsigned)g), dim3(256), 0, s, n, dt, B[0], B[1], B[2],
                       (const double*)Ex, (double*)u, cell, (double*)off);
  } else {
    auto k = pusher ? k_push_bench<float, 1> : k_push_bench<float, 0>;
    hipLaunchKernelGGL(k, dim3((unsigned)g), dim3(256), 0, s, n, (float)dt, (float)B[0], (float)B[1],
                       (float)B[2], (const float*)Ex, (float*)u, cell, (float*)off);
  }
}

// Plain streaming copy of n 16-byte words (read n*16 bytes, write n*16
// bytes): the reference kernel of known traffic against which the memory
// counters of the other kernels are calibrated.
__global__ __launch_bounds__(256) void k_copy_bench(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                    long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// Tuned streaming kernels that establish the HBM bandwidth a kernel can reach
// on the device: every thread moves U 16-byte words per iteration, all loads
// issued before the stores, with non-temporal hints (the data is used once).
//   mode 0: copy (read and write each byte once)
//   mode 1: read only (the words are folded into one value, stored only if it
//           equals a sentinel, so the loads cannot be dropped)
//   mode 2: write only
typedef unsigned v4u __attribute__((ext_vector_type(4)));
template <int MODE, int U>
__global__ __launch_bounds__(256) void k_stream_bench(const v4u* __restrict__ src, v4u* __restrict__ dst,
                                                      long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x * U;
  unsigned acc = 0;
  for (long long b = (long long)blockIdx.x * blockDim.x * U + threadIdx.x; b < n; b += stride) {
    v4u v[U];
    if (MODE != 2) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const long long i = b + (long long)u * blockDim.x;
        v[u] = i < n ? __builtin_nontemporal_load(src + i) : v4u{0u, 0u, 0u, 0u};
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long i = b + (long long)u * blockDim.x;
      if (MODE == 1) {
        acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
      } else if (i < n) {
        const v4u w = MODE == 0 ? v[u] : v4u{(unsigned)i, 1u, 2u, 3u};
        __builtin_nontemporal_store(w, dst + i);
      }
    }
  }
  if (MODE == 1 && acc == 0x9e3779b9u) dst[0].x = acc;
}

void launch_stream_bench(int mode, const void* src, void* dst, long long n16, hipStream_t s) {
  constexpr int U = 8;
  long long g = (n16 + 256LL * U - 1) / (256LL * U);
  if (g > 16384) g = 16384;
  if (g < 1) g = 1;
  const v4u* a = (const v4u*)src;
  v4u* b = (v4u*)dst;
  if (mode == 0) hipLaunchKernelGGL((k_stream_bench<0, U>), dim3((unsigned)g), dim3(256), 0, s, a, b, n16);
  else if (mode == 1) hipLaunchKernelGGL((k_stream_bench<1, U>), dim3((unsigned)g), dim3(256), 0, s, a, b, n16);
  else hipLaunchKernelGGL((k_stream_bench<2, U>), dim3((unsigned)g), dim3(256), 0, s, a, b, n16);
}

void launch_copy_bench(const void* src, void* dst, long long n16, hipStream_t s) {
  long long g = (n16 + 255) / 256;
  if (g > 256 * 64) g = 256 * 64;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_copy_bench, dim3((unsigned)g), dim3(256), 0, s, (const uint4*)src, (uint4*)dst, n16);
}

}  // namespace pic
