// Device-side run descriptor, batch table and small device helpers for the
// gfx950 boosted-frame PIC kernels.  Everything that changes during a run
// (step index, ping-pong buffer parities, particle counts, error word) lives
// in device memory, so every kernel sequence can be captured once in a HIP
// graph and replayed, and several runs can share one launch through a batch
// table of descriptors.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pic.h"

// Address spaces of the device pointers held in the run descriptor: global
// for the arrays, constant for the read-only descriptors.  Typed pointers let
// the compiler emit global and scalar loads instead of flat ones (a flat
// access counts against both the memory and the LDS wait counters, so every
// LDS wait would also wait for outstanding loads).  The host compilation
// sees plain pointers of the same size and layout.
#if defined(__HIP_DEVICE_COMPILE__)
#define PIC_G __attribute__((address_space(1)))
#define PIC_C __attribute__((address_space(4)))
#else
#define PIC_G
#define PIC_C
#endif

namespace pic {

// ---------------------------------------------------------------- constants
constexpr int MAX_BATCH = 256;

// Packed particle cell: k + KOFF in bits 0..10, i in bits 11..20, j in bits
// 21..30, bit 31 = removed.  KOFF lets a particle that just left through
// z = 0 keep its position for the continuity diagnostic.
constexpr int KOFF = 4;
constexpr int KBITS = 11, IBITS = 10, JBITS = 10;
constexpr int KMASK = (1 << KBITS) - 1, IMASK = (1 << IBITS) - 1, JMASK = (1 << JBITS) - 1;
constexpr unsigned DEAD = 0x80000000u;

// Tile geometry (cells) and the largest LDS window a tile may use.  The
// window spans the tile's particle bounding box widened by one cell below
// and two above (gather and deposit stencils): W = extent + 3, so a tile's
// particles may spread over TZ + 4 cells in z and TX + 2, TY + 2 across
// (the sort places some up to GZ cells above the tile's z range).
// The z extent W_z = 15 is odd, so the x offsets 15 i of a wavefront's 8x8
// transverse plane cover every residue mod 8, and the y stride is padded
// (below) to complete a bank-distinct pattern.
// 3D split precision: 8x8x8 cells, a 15x13x13 window (y stride padded to
// 200 cells) of 122 KiB (one 1024-thread workgroup per CU); 3D FP64: 8x8x4
// cells, 15x13x9, 123 KiB.
template <int DIM, typename R> struct Tile;
template <typename R> struct Tile<3, R> {
  static constexpr int LZ = 3, LX = 3, LY = sizeof(R) == 4 ? 3 : 2;
  static constexpr int TZ = 1 << LZ, TX = 1 << LX, TY = 1 << LY;
  static constexpr int WZ = TZ + 7, WX = TX + 5, WY = TY + 5;
  // LDS stride of y.  In split precision it is padded from WZ WX to the next
  // value = 8 (mod 64): with the odd x stride WZ, the word offsets
  // WZ i + SY j of an 8x8 transverse plane (the cells of one wavefront's
  // lanes) are then 64 distinct banks, so a pair read (z, z+1) or a 64-bit
  // atomic loads every bank exactly twice (unpadded: up to four times).
  static constexpr int SY = sizeof(R) == 4 ? WZ * WX + ((8 - WZ * WX) % 64 + 64) % 64 : WZ * WX;
  // z cells above the tile a group sorted by its lowest cell may reach
  // (the window still spans the tile plus this and the stencil)
  static constexpr int GZ = sizeof(R) == 4 ? 1 : 2;
};
// 2D: 16x16 cells, a 22x37 window (39 KiB; four 256-thread workgroups per
// CU): 21 cells of transverse slack, because electrons quivering in a
// strong laser at low gamma_b (a0 ~ 3, gamma_b ~ 2) spread across x by more
// than half a cell per step between sorts, and those that leave the window
// take the out-of-window path at tens of times the cost (a 37-wide window
// took the serving stream's p50 from 191 to 127 ms against 21).
template <typename R> struct Tile<2, R> {
  static constexpr int LZ = 4, LX = 4, LY = 0;
  static constexpr int TZ = 1 << LZ, TX = 1 << LX, TY = 1;
  static constexpr int WZ = TZ + 6, WX = TX + 21, WY = 1;
  static constexpr int SY = 0;  // no y
  static constexpr int GZ = 1;  // 2D groups interleave four columns: rarely whole
};

// Yee staggering per component (half-cell flags in z, x, y):
// Ex(0,1,0) Ey(0,0,1) Ez(1,0,0) Bx(1,0,1) By(1,1,0) Bz(0,1,1); J like E.
__host__ __device__ constexpr int stag(int comp, int d) {
  return (comp == 0) ? (d == 1) : (comp == 1) ? (d == 2) : (comp == 2) ? (d == 0)
       : (comp == 3) ? (d != 1) : (comp == 4) ? (d != 2) : (d != 0);
}

// ---------------------------------------------------------------- state
struct Counters {
  long long step;      // index n of the next step
  long long n_slots;   // particle slots in the current buffer (live + removed + tail)
  long long n_live;    // live particles after the last sort
  long long n_padded;  // slots after the last sort (tiles padded to 64 slots)
  long long next_col;  // next plasma lattice column to create
  long long last_sort; // step of the last sort (-1: none)
  long long n_new;     // particles created by the pending injection
  long long k_end;     // column bound of the pending injection
  int pbuf, fbuf, bbuf, fresh;
  unsigned err;
  int want_sort;       // sort at the next step: too many particles left their windows
  // continuity diagnostic (max over steps, as bit patterns of non-negative doubles)
  unsigned long long cont_res_bits, cont_rho_bits;
  double cont_max;
  double rho0_max;
  // diagnostic accumulators
  double acc[4];
  unsigned long long amax[4];
  unsigned long long cnt[2];
  unsigned long long n_slow;  // particles that took the HBM path (since the last diag)
  unsigned n_slowq;           // entries of this step's HBM-path queue
  unsigned pad1;
};

struct RunDev {
  int dims, nz, nx, ny, nzf, open, ppc, reservoir, ztop, inject_every;
  int ntz, ntx, nty, ntiles;
  int gx, gy, gz;       // wrap guards for tile-relative coordinates
  int pusher, diag_flags, pol_axis;
  // current filter: passes, compensation flag, and number of one-axis
  // stages ((passes + compensation) x axes; 0 = none)
  int filter_passes, filter_comp, filter_stages, pad_f;
  long long capacity, nperp, npts, max_new;
  double dt, dz, dx, dy;
  double beta_b, gamma_b, dminus, dplus, weight, jion_z, rho_ion, u_th;
  double k0_lab, E0_lab, L_lab, zc_boost, waist;
  double jscale, jinv;  // current stored as int64 = round(J * jscale)
  // particle-update constants: -dt/2 (q/m = -1), dt/dz, dt/dx, dt/dy, and the
  // current coefficients (times jscale) of Jz, Jx, Jy and the 2D out-of-plane Jy
  double pk[8];
  unsigned long long seed;
  // arrays (device addresses inside the caller's buffer); element type is
  // float (split-precision path) or double (FP64 path)
  PIC_G void* E[2][3];
  PIC_G void* B[2][3];  // B at half-integer time: B^{n-1/2} in B[fbuf]
  PIC_G void* J[2][3];  // int64 fixed point; the step deposits into J[fbuf], the
                        // field kernel reads it and clears J[fbuf^1] for the next step
  PIC_G int* cell[2];
  PIC_G void* off[2][3];
  PIC_G void* u[2][3];
  PIC_G unsigned* pid[2];
  PIC_G int* tile_start;  // ntiles + 1
  PIC_G int* tile_count;  // ntiles: particles per tile (counting), then zeroed
  PIC_G int* tile_cursor; // ntiles: next slot for particles that come in fragments
  PIC_G int* tile_full;   // ntiles: particles that come in whole wavefronts (counting),
                          // then the next slot for them
  PIC_G int* bbox[2];     // 6 ints per tile: lo z,x,y then hi z,x,y (tile-relative)
  PIC_G double* rho_a;
  PIC_G double* rho_b;
  PIC_G double* gauss0;
  PIC_G double* jlast[3];
  PIC_G int* cell_snap;
  PIC_G int* slowq;       // slots of particles deferred to the HBM path this step
  PIC_G void* jf[2][3];   // filtered current (R): stage s writes jf[s & 1]
  PIC_G double* ftmp[2];  // node scalar ping-pong (filtered Gauss diagnostic)
  PIC_G Counters* ctr;
  // laboratory-frame stations: count, first z (lab), spacing, transverse
  // stride, stored samples per station and transverse samples per record
  int n_stations, st_stride, st_cap, st_nxs, st_nys, pad_s;
  double st_z0, st_dz;
  PIC_G double* st_time;      // [station][st_cap] lab times
  PIC_G double* st_data;      // [station][st_cap][6][st_nys][st_nxs] lab fields
  PIC_G long long* st_count;  // [station] samples taken
  // laser antenna: on/off, lab z of the plane, lab time of the envelope peak
  int antenna, pad_a;
  double ant_z_lab, ant_t_peak;
};

// a run descriptor as the kernels see it (read-only, constant address space)
using RunC = const PIC_C RunDev;

// A set of runs advanced by the same launches.  Work items of the step's
// kernels are enumerated run by run; pre_* are exclusive prefix sums of the
// per-run item counts (tiles, field blocks).  The sort kernels count the
// live items of each run when they start.
struct BatchTable {
  int n;
  int pad;
  long long tiles, cellblk;
  RunC* run[MAX_BATCH];
  long long pre_tiles[MAX_BATCH + 1];
  long long pre_cellblk[MAX_BATCH + 1];
};

constexpr int CELL_BLOCK = 256;     // cells per field work item
constexpr int PART_CHUNK = 4096;    // particle slots per sort work item
constexpr int INJ_CHUNK = 4096;     // created particles per injection work item

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ int locate(const long long* pre, int n, long long w) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= w) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Persistent work distribution: workgroup b runs on XCD b % 8 (round-robin
// dispatch), so each XCD takes one contiguous eighth of the items and the
// tiles that share halo data meet in the same L2.
struct XcdSplit {
  long long beg, end, stride;
  __device__ XcdSplit(long long total) {
    const int G = gridDim.x;
    const int x = blockIdx.x & 7;
    const int per = G >> 3;
    const long long chunk = (total + 7) >> 3;
    beg = x * chunk + (blockIdx.x >> 3);
    end = (x + 1) * chunk < total ? (x + 1) * chunk : total;
    stride = per;
  }
};

__device__ __forceinline__ int wrapi(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}
// periodic wrap of an index in [-n, 2n) (one correction)
__device__ __forceinline__ int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }
// periodic wrap of an index in (-n, 2n) with one three-way unsigned minimum:
// of w, w + n and w - n exactly one lies in [0, n), and the others are >= n
// as unsigned numbers.  n = 0 leaves w unchanged.
__device__ __forceinline__ int wrapu(int w, int n) {
  const unsigned a = (unsigned)w, b = (unsigned)(w + n), c = (unsigned)(w - n);
  return (int)min(min(a, b), c);
}
// periodic wrap of an index in [-2n, 3n) (two corrections)
__device__ __forceinline__ int wrap2(int i, int n) {
  i = i < 0 ? i + n : (i >= n ? i - n : i);
  return i < 0 ? i + n : (i >= n ? i - n : i);
}
// tile-relative coordinate of a periodic index i in [0,n) for a tile origin
// t0 in [0,n) and a guard 0 <= g < n: result in [-g, n-g)
__device__ __forceinline__ int relw(int i, int t0, int n, int g) {
  int r = i - t0 + g;
  r = r < 0 ? r + n : (r >= n ? r - n : r);
  return r - g;
}

__device__ __forceinline__ int cell_k(int c) { return (c & KMASK) - KOFF; }
__device__ __forceinline__ int cell_i(int c) { return (c >> KBITS) & IMASK; }
__device__ __forceinline__ int cell_j(int c) { return (c >> (KBITS + IBITS)) & JMASK; }
__device__ __forceinline__ int cell_pack(int k, int i, int j) {
  return (k + KOFF) | (i << KBITS) | (j << (KBITS + IBITS));
}

// number of valid z indices of a component (open z: nodes 0..nz, half
// points 0..nz-1; periodic: nz)
__device__ __forceinline__ int zcount(RunC& r, int comp) {
  return r.open ? (stag(comp, 0) ? r.nz : r.nz + 1) : r.nz;
}

__device__ __forceinline__ long long gidx(RunC& r, int k, int i, int j) {
  return ((long long)j * r.nx + i) * r.nzf + k;
}

// E value at integer index with the open/periodic z rules
template <typename R>
__device__ __forceinline__ double ev(RunC& rd, R* const* E, int c, int k, int i, int j) {
  i = wrapi(i, rd.nx);
  j = rd.dims == 3 ? wrapi(j, rd.ny) : 0;
  if (rd.open) {
    if (k < 0 || k >= zcount(rd, c)) return 0.0;
  } else {
    k = wrapi(k, rd.nz);
  }
  return (double)E[c][gidx(rd, k, i, j)];
}

// curl of E at the B point of component c (0,1,2 = x,y,z)
template <typename R>
__device__ __forceinline__ double curl_e(RunC& rd, R* const* E, int c, int k, int i, int j) {
  const double idz = 1.0 / rd.dz, idx = 1.0 / rd.dx, idy = rd.dims == 3 ? 1.0 / rd.dy : 0.0;
  if (c == 0)
    return (ev(rd, E, 2, k, i, j + 1) - ev(rd, E, 2, k, i, j)) * idy -
           (ev(rd, E, 1, k + 1, i, j) - ev(rd, E, 1, k, i, j)) * idz;
  if (c == 1)
    return (ev(rd, E, 0, k + 1, i, j) - ev(rd, E, 0, k, i, j)) * idz -
           (ev(rd, E, 2, k, i + 1, j) - ev(rd, E, 2, k, i, j)) * idx;
  return (ev(rd, E, 1, k, i + 1, j) - ev(rd, E, 1, k, i, j)) * idx -
         (ev(rd, E, 0, k, i, j + 1) - ev(rd, E, 0, k, i, j)) * idy;
}

// Philox4x64-10 (Salmon et al., SC'11)
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
    uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
    uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    k0 += W0; k1 += W1;
  }
}
__device__ __forceinline__ double u01(uint64_t r) {
  return (double)(r >> 11) * (1.0 / 9007199254740992.0);
}

// x * scale rounded to the nearest integer as int64, for |x * scale| < 2^51:
// adding 1.5 * 2^52 places the rounded integer in the low mantissa bits
__device__ __forceinline__ long long to_fixed(double x, double scale) {
  const double magic = 6755399441055744.0;  // 1.5 * 2^52
  return __double_as_longlong(fma(x, scale, magic)) - 0x4338000000000000LL;
}

// relaxed device-scope atomics on global memory
template <typename T>
__device__ __forceinline__ T g_add(PIC_G T* a, T v) {
  return __hip_atomic_fetch_add(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T g_min(PIC_G T* a, T v) {
  return __hip_atomic_fetch_min(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T g_max(PIC_G T* a, T v) {
  return __hip_atomic_fetch_max(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T g_or(PIC_G T* a, T v) {
  return __hip_atomic_fetch_or(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// bit pattern max for non-negative doubles
__device__ __forceinline__ void atomic_max_pos(PIC_G unsigned long long* a, double v) {
  g_max(a, (unsigned long long)__double_as_longlong(v));
}

// the tile sort of a step runs when the step is a multiple of the cadence
// (the plasma-column injection runs only then) or when the previous step
// sent too many particles to the out-of-window path, and the step has not
// been sorted yet
__device__ __forceinline__ bool sort_due(const PIC_G Counters& c, int every) {
  return ((c.step % every) == 0 || c.want_sort != 0) && c.step != c.last_sort;
}

template <typename R> __device__ __forceinline__ PIC_G R* fptr(PIC_G void* p) { return (PIC_G R*)p; }

// Read-only view of global memory that no kernel writes while the caller
// runs (tile starts, the previous step's bounding boxes, buffer parities):
// through the constant address space, uniform reads become scalar loads,
// which wait on their own counter instead of on every outstanding vector
// memory operation.
template <typename T>
__device__ __forceinline__ const PIC_C T* ro(const PIC_G T* p) {
  return (const PIC_C T*)(size_t)p;
}

// element at byte offset b (32-bit, zero-extended) from a global base: the
// base stays in scalar registers and the offset in one vector register
template <typename T>
__device__ __forceinline__ PIC_G T& at32(PIC_G T* base, unsigned b) {
  return *(PIC_G T*)((PIC_G char*)base + b);
}

// the three component arrays of a field (or current) buffer
template <typename R>
struct Arr3 {
  PIC_G R* p[3];
  __device__ __forceinline__ PIC_G R* operator[](int c) const { return p[c]; }
};
#define PIC_ARR3(R, a) (::pic::Arr3<R>{{(PIC_G R*)(a)[0], (PIC_G R*)(a)[1], (PIC_G R*)(a)[2]}})

}  // namespace pic
