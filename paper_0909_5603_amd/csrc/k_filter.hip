// Low-pass digital filtering of the current (Sec. 2, third paragraph, names
// it among the means that keep the boosted-frame run stable without giving
// the filter): binomial passes per axis with an optional compensating pass,
// between the deposit and the E update.
#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "pic_dev.hpp"

namespace pic {

// All the passes along one axis per launch.  The binomial passes (1/4, 1/2, 1/4) and
// the optional compensating pass (-N/4, 1 + N/2, -N/4) along different axes
// commute, so the filter runs as z, then x, then y.  Both kernels stage a
// slab of one component in LDS, and a thread then takes FILTER_RUN
// consecutive points of one row with HALO neighbours on each side into
// registers and applies the passes there in order, with no barrier between
// passes: after pass p the values from index p to W-1-p of its W registers
// are exact, which covers its outputs for every number of passes up to HALO.
//   k_filter_z: a work item is a block of consecutive transverse columns of
//     one component.  Each staged column carries ghost points beyond its z
//     range: along a periodic z axis the wrapped values; along an open axis
//     the range mirrored about its end faces (the value at -1-m is the one
//     at m).  A pass maps mirrored data to mirrored data, and at the end
//     point it computes exactly what the end rule (a neighbour beyond the
//     range repeats the end value, so a current streaming uniformly out
//     through an end passes unchanged) gives, so the mirror realises that
//     rule for all passes at once.  Points outside the range are 0.  Reads
//     the fixed-point deposit (times its scale), writes jf[0].
//   k_filter_xy: along the periodic x (axis 1, jf[0] -> jf[1]) and y (axis 2,
//     jf[1] -> jf[0]) axes.  A work item is a chunk of zc consecutive z
//     points (up to 64: one 256-byte run in HBM in FP32) of every point
//     along the axis; the next item's loads are issued before the current
//     one is filtered, so they are in flight meanwhile (at 512x256x256 the
//     64-point chunks run at 3.1-3.4 TB/s against 2.6-3.1 for 32 points).
// HBM is read and written once per axis.  The E update reads the last
// axis's output.
constexpr int FILTER_ZMAX = 2048;  // z points of a column (the cell packing keeps nzf below)
constexpr int FILTER_HMAX = 17;    // N <= 16 passes plus compensation
constexpr int FILTER_RUN = 16;     // outputs of a thread along the filtered axis
constexpr int FILTER_Z_BLOCK = 256;
#ifndef PIC_FXY_BLOCK
#define PIC_FXY_BLOCK 1024
#endif
#ifndef PIC_FXY_LDS
#define PIC_FXY_LDS 65536
#endif
#ifndef PIC_FXY_LZC
#define PIC_FXY_LZC 6
#endif
constexpr int FILTER_XY_BLOCK = PIC_FXY_BLOCK;
constexpr int FILTER_XY_LDS = PIC_FXY_LDS;  // bytes of the staged slab
constexpr int FILTER_XY_LZC = PIC_FXY_LZC;  // log2 of the largest z chunk

// per-run prefix of work items in LDS (thread 0 scans; every thread calls)
template <class F>
__device__ __forceinline__ long long filter_items(const BatchTable* __restrict__ bt, long long* pre, F&& count) {
  const int n = bt->n;
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
    RunC& rd = *bt->run[r];
    pre[r + 1] = rd.filter_stages > 0 ? count(rd) : 0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    long long acc = 0;
    pre[0] = 0;
    for (int r = 0; r < n; ++r) {
      acc += pre[r + 1];
      pre[r + 1] = acc;
    }
  }
  __syncthreads();
  return pre[n];
}

// npass passes over the W registers: np binomial ones, then the
// compensating one when npass > np
template <typename R, int W>
__device__ __forceinline__ void filter_passes(R (&v)[W], int npass, int np) {
  for (int p = 0; p < npass; ++p) {
    const bool cpass = p >= np;
    const R ws = cpass ? R(-0.25) * R(np) : R(0.25);
    const R wm = cpass ? R(1) + R(0.5) * R(np) : R(0.5);
    R prev = v[0];
#pragma unroll
    for (int j = 1; j < W - 1; ++j) {
      const R a = v[j];
      v[j] = wm * a + ws * (prev + v[j + 1]);
      prev = a;
    }
  }
}

// index of the staged value that stands at z index k of a column (range
// 0..zc-1): the wrapped index (periodic) or the mirrored one (open)
__device__ __forceinline__ int filter_zsrc(int k, int zc, bool open) {
  if (!open) return ((k % zc) + zc) % zc;
  while (k < 0 || k >= zc) k = k < 0 ? -1 - k : 2 * zc - 1 - k;
  return k;
}

// LDS position of staged index e of a column: one pad word after every 16,
// so that lanes reading runs of FILTER_RUN = 16 consecutive values start 17
// words apart and hit distinct banks
__device__ __forceinline__ int filter_zpos(int e) { return e + (e >> 4); }

template <int DIM, typename R, int HALO>
__global__ __launch_bounds__(FILTER_Z_BLOCK) void k_filter_z(const BatchTable* __restrict__ bt) {
  constexpr int P = FILTER_RUN, W = P + 2 * HALO;
  static_assert(P == 16, "filter_zpos pads after every 16 values");
  // staged columns: 16 KiB in FP32, 24 KiB in FP64 (a column of FILTER_ZMAX
  // points with its ghosts must fit)
  constexpr int CAP = (sizeof(R) == 4 ? 16384 : 24576) / (int)sizeof(R);
  constexpr int LPT = (CAP + FILTER_Z_BLOCK - 1) / FILTER_Z_BLOCK;  // loads per thread
  static_assert((FILTER_ZMAX + P + 2 * FILTER_HMAX) * 17 / 16 + 1 <= CAP, "a column must fit");
  static_assert(FILTER_ZMAX / P <= FILTER_Z_BLOCK, "a column's groups must fit the block");
  __shared__ R col[CAP];
  __shared__ long long pre[MAX_BATCH + 1];
  // a staged column holds nzf + P + 2 HALO values plus the pads
  auto span = [](int nzf) { return filter_zpos(nzf + P + 2 * HALO - 1) + 1; };
  // columns of an item: as many as fit the buffer, at most 8, and few enough
  // that every group of FILTER_RUN points has a thread of its own
  auto ncols = [&](RunC& rd) {
    const int ngr = (rd.nzf + P - 1) / P;
    return max(1, min(min(8, FILTER_Z_BLOCK / ngr), CAP / span(rd.nzf)));
  };
  const long long items = filter_items(bt, pre, [&](RunC& rd) {
    const int B = ncols(rd);
    return 3 * ((rd.nperp + B - 1) / B);
  });
  const int n = bt->n;
  for (long long w = blockIdx.x; w < items; w += gridDim.x) {
    const int r = __builtin_amdgcn_readfirstlane(locate(pre, n, w));
    RunC& rd = *bt->run[r];
    const int nzf = rd.nzf, nz = rd.nz;
    const int npass = rd.filter_stages / (DIM == 3 ? 3 : 2), np = rd.filter_passes;
    if (nzf > FILTER_ZMAX || npass > HALO) {  // excluded by the parameter checks; never filtered
      if (threadIdx.x == 0) g_or(&rd.ctr->err, (unsigned)PIC_ERR_TILE);
      continue;
    }
    const bool open = rd.open != 0;
    const int B = ncols(rd), S = span(nzf), ns = nzf + P + 2 * HALO;
    const unsigned it = (unsigned)(w - pre[r]);
    const int c = (int)(it % 3u);
    const long long col0 = (long long)(it / 3u) * B;
    const int nb = (int)min((long long)B, rd.nperp - col0);  // columns of this item
    const int zc = (c == 2 && open) ? nz : nzf;               // z range of the component
    // the item's columns are consecutive in HBM: nb * nzf values from col0 * nzf
    PIC_G long long* __restrict__ J = (PIC_G long long*)rd.J[rd.ctr->fbuf][c] + col0 * nzf;
    PIC_G R* __restrict__ dst = (PIC_G R*)rd.jf[0][c] + col0 * nzf;
    const double jinv = rd.jinv;
    const int nflat = nb * nzf;
    const unsigned mz = 0xffffffffu / (unsigned)nzf + 1u;  // f / nzf = umulhi(f, mz) for f < 2^32 / nzf
    // all loads first (indices clamped into the item, so none waits on a
    // branch), then the conversions
    long long raw[LPT];
#pragma unroll
    for (int u = 0; u < LPT; ++u)
      raw[u] = at32(J, 8u * (unsigned)min((int)threadIdx.x + u * FILTER_Z_BLOCK, nflat - 1));
    __syncthreads();  // the previous item's columns are done with
#pragma unroll
    for (int u = 0; u < LPT; ++u) {
      const int f = threadIdx.x + u * FILTER_Z_BLOCK;
      if (f < nflat) {
        const int b = (int)__umulhi((unsigned)f, mz), k = f - b * nzf;
        col[b * S + filter_zpos(HALO + k)] = R((double)raw[u] * jinv);
      }
    }
    __syncthreads();
    // ghosts: staged indices below HALO and from HALO + zc on (this also
    // replaces the point outside the range), copied from the wrapped or
    // mirrored points of the range
    const int ng = ns - zc;
    for (int t = threadIdx.x; t < nb * ng; t += FILTER_Z_BLOCK) {
      const int b = t / ng, g = t - b * ng;
      const int e = g < HALO ? g : zc + g;
      col[b * S + filter_zpos(e)] = col[b * S + filter_zpos(HALO + filter_zsrc(e - HALO, zc, open))];
    }
    __syncthreads();
    // each thread filters at most one group of P points (nb * ngr is at most
    // the block size: FILTER_ZMAX / P <= FILTER_Z_BLOCK), keeps it in registers across the barrier
    // and writes it back over the staged range; the item is then stored
    // with the coalesced flat indexing of the loads
    const int ngr = (nzf + P - 1) / P;  // groups of a column
    const int t = threadIdx.x;
    const bool active = t < nb * ngr;
    const int b = active ? t / ngr : 0, k0 = active ? (t - b * ngr) * P : 0;
    R v[W];
    if (active) {
      const R* cs = col + b * S;
#pragma unroll
      for (int j = 0; j < W; ++j) v[j] = cs[filter_zpos(k0 + j)];  // staged index of z = k0 - HALO + j
      filter_passes<R, W>(v, npass, np);
    }
    __syncthreads();
    if (active) {
      R* cs = col + b * S;
#pragma unroll
      for (int q = 0; q < P; ++q)
        if (k0 + q < nzf) cs[filter_zpos(HALO + k0 + q)] = k0 + q < zc ? v[HALO + q] : R(0);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < LPT; ++u) {
      const int f = threadIdx.x + u * FILTER_Z_BLOCK;
      if (f < nflat) {
        const int bb = (int)__umulhi((unsigned)f, mz), k = f - bb * nzf;
        at32(dst, (unsigned)sizeof(R) * (unsigned)f) = col[bb * S + filter_zpos(HALO + k)];
      }
    }
  }
}

template <int DIM, typename R, int HALO>
__global__ __launch_bounds__(FILTER_XY_BLOCK) void k_filter_xy(const BatchTable* __restrict__ bt, int axis) {
  constexpr int CAP = FILTER_XY_LDS / (int)sizeof(R);
  constexpr int LPT = CAP / FILTER_XY_BLOCK;  // staged values per thread
  constexpr int P = FILTER_RUN, W = P + 2 * HALO;
  __shared__ R row[CAP];
  __shared__ long long pre[MAX_BATCH + 1];
  // chunk of zc = 2^lzc z points: the largest power of two up to
  // 2^FILTER_XY_LZC whose slab (zc x the axis length) fits the staging buffer
  auto chunk = [axis](RunC& rd) {
    const int na = axis == 1 ? rd.nx : rd.ny;
    int l = FILTER_XY_LZC;
    while (l > 0 && (na << l) > CAP) --l;
    return l;
  };
  const long long items = filter_items(bt, pre, [&](RunC& rd) {
    const int lzc = chunk(rd);
    const long long nch = (rd.nzf + (1 << lzc) - 1) >> lzc;
    const long long other = axis == 1 ? (DIM == 3 ? rd.ny : 1) : rd.nx;
    return 3 * nch * other;
  });
  struct Item {
    const PIC_G R* src;
    PIC_G R* dst;
    long long stride;
    int na, lzc, kend, kmax, npass, np;
  };
  const int n = bt->n;
  auto decode = [&](long long w, Item& g) {
    const int r = __builtin_amdgcn_readfirstlane(locate(pre, n, w));
    RunC& rd = *bt->run[r];
    const int nzf = rd.nzf, nx = rd.nx;
    g.na = axis == 1 ? nx : rd.ny;
    g.lzc = chunk(rd);
    const int zc = 1 << g.lzc;
    const unsigned nch = (unsigned)((nzf + zc - 1) >> g.lzc);
    const unsigned it = (unsigned)(w - pre[r]);
    const int c = (int)(it % 3u);
    const unsigned t3 = it / 3u;
    const int k0 = (int)(t3 % nch) << g.lzc;
    const long long o = t3 / nch;  // index across the axis (y for axis 1, x for axis 2)
    g.kend = min(zc, nzf - k0);                                         // points of this chunk
    g.kmax = (c == 2 && rd.open) ? min(zc, rd.nz - k0) : g.kend;        // Jz has no point at k = nz
    g.stride = axis == 1 ? (long long)nzf : (long long)nx * nzf;
    const long long base = (axis == 1 ? o * nx * (long long)nzf : o * nzf) + k0;
    g.src = (const PIC_G R*)rd.jf[(axis - 1) & 1][c] + base;
    g.dst = (PIC_G R*)rd.jf[axis & 1][c] + base;
    g.npass = rd.filter_stages / (DIM == 3 ? 3 : 2);  // passes + compensation
    g.np = rd.filter_passes;
    if (g.npass > HALO) {  // excluded by the choice of HALO; never filtered
      if (threadIdx.x == 0) g_or(&rd.ctr->err, (unsigned)PIC_ERR_TILE);
      g.npass = 0;
      g.kmax = 0;
    }
  };
  // the loads of an item's slab into registers (nothing waits for them here)
  auto issue = [&](const Item& g, R (&ld)[LPT]) {
    const int zc = 1 << g.lzc, npt = g.na << g.lzc;
#pragma unroll
    for (int u = 0; u < LPT; ++u) {
      const int t = threadIdx.x + u * FILTER_XY_BLOCK;
      const int kk = t & (zc - 1), ia = t >> g.lzc;
      ld[u] = (t < npt && kk < g.kmax) ? g.src[ia * g.stride + kk] : R(0);
    }
  };
  long long w = blockIdx.x;
  Item g;
  R ld[LPT];
  if (w < items) {
    decode(w, g);
    issue(g, ld);
  }
  for (; w < items; w += gridDim.x) {
    const int zc = 1 << g.lzc, npt = g.na << g.lzc, na = g.na;
    __syncthreads();  // the previous slab is done with
#pragma unroll
    for (int u = 0; u < LPT; ++u) {
      const int t = threadIdx.x + u * FILTER_XY_BLOCK;
      if (t < npt) row[t] = ld[u];
    }
    __syncthreads();
    Item gn;
    const long long wn = w + gridDim.x;
    if (wn < items) {
      decode(wn, gn);
      issue(gn, ld);
    }
    const int ngr = (na + P - 1) / P;
    for (int t = threadIdx.x; t < (ngr << g.lzc); t += FILTER_XY_BLOCK) {
      const int kk = t & (zc - 1), ia0 = (t >> g.lzc) * P;
      if (kk >= g.kend) continue;
      R v[W];
      if (kk < g.kmax) {
        int idx = ((ia0 - HALO) % na + na) % na;  // periodic index of the first value
#pragma unroll
        for (int j = 0; j < W; ++j) {
          v[j] = row[(idx << g.lzc) + kk];
          if (++idx == na) idx = 0;
        }
        filter_passes<R, W>(v, g.npass, g.np);
      } else {
#pragma unroll
        for (int j = 0; j < W; ++j) v[j] = R(0);
      }
#pragma unroll
      for (int q = 0; q < P; ++q)
        if (ia0 + q < na) g.dst[(ia0 + q) * g.stride + kk] = v[HALO + q];
    }
    g = gn;
  }
}

template <int DIM, typename R, int HALO>
static void lfilter(const BatchTable* bt, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_filter_z<DIM, R, HALO>), dim3(grid), dim3(FILTER_Z_BLOCK), 0, s, bt);
  hipLaunchKernelGGL((k_filter_xy<DIM, R, HALO>), dim3(grid), dim3(FILTER_XY_BLOCK), 0, s, bt, 1);
  if (DIM == 3) hipLaunchKernelGGL((k_filter_xy<DIM, R, HALO>), dim3(grid), dim3(FILTER_XY_BLOCK), 0, s, bt, 2);
}

template <int DIM, typename R>
static void lf(const BatchTable* bt, int grid, int filter_stages, hipStream_t s) {
  // register halo: the most passes (plus compensation) of any run of the batch
  if (filter_stages / DIM <= 5) lfilter<DIM, R, 5>(bt, grid, s);
  else lfilter<DIM, R, FILTER_HMAX>(bt, grid, s);
}

void launch_filter(int dims, int prec, const BatchTable* bt, int grid, int filter_stages, hipStream_t s) {
  if (dims == 3) {
    if (prec) lf<3, double>(bt, grid, filter_stages, s);
    else lf<3, float>(bt, grid, filter_stages, s);
  } else {
    if (prec) lf<2, double>(bt, grid, filter_stages, s);
    else lf<2, float>(bt, grid, filter_stages, s);
  }
}

}  // namespace pic
