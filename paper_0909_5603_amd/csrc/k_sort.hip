// Plasma-column injection and the counting sort of particles by tile.
//
// Every sort_every steps, and (without (1)) at the first step carrying the
// sort chain after one in which more than 1/1024 of a run's particles left
// their tile windows:
// (1) create the lattice columns that have drifted
// into the reservoir beyond z_max (Philox-drawn positions, laboratory
// Maxwellian momenta boosted to the frame: Sec. 2, second paragraph - a
// plasma at rest in the laboratory streams toward -z here, its density
// raised by gamma_boost), appending them after
// the current slots; (2) count live particles per tile; (3) exclusive scan of
// the counts, each tile's range padded to a multiple of 64 slots with
// removed markers (one workgroup per run); (4) scatter into the other
// particle buffer, which also drops removed particles; (5) commit the new
// counts and flip the buffer.
// Wavefront groups.  The injection creates the plasma in groups of 64
// consecutive slots that lie in 64 different cells of one tile's transverse
// plane, and the step kernel gives each wavefront 64 consecutive slots of a
// tile starting at a multiple of 64; when the two coincide, the lanes of a
// wavefront add their currents to 64 different LDS cells that fall in
// distinct banks.  The sort keeps them coinciding: a source wavefront whose
// 64 slots are live and go to one tile (a whole group) is placed at the
// tile's front cursor, which advances by 64, and the particles of the other
// source wavefronts (groups split by a tile boundary, removed particles)
// follow behind the whole groups.  Per-tile atomics of those are aggregated
// over the wavefront with ballots: lanes with equal keys elect a leader that
// makes one atomic add, and each lane's rank inside its group is a popcount
// of the lower lanes.
#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "pic_dev.hpp"

namespace pic {

// columns and particles the pending injection of this step creates
__device__ __forceinline__ void pending(RunC& rd, const PIC_G Counters& c, long long& kend,
                                        long long& nnew) {
  if (c.step % rd.inject_every != 0) {  // a sort between cadence steps injects nothing
    kend = c.next_col;
    nnew = 0;
    return;
  }
  if (rd.open) {
    const double shift = rd.beta_b * ((double)c.step * rd.dt) / rd.dz;
    kend = (long long)rd.nz + rd.reservoir + (long long)ceil(shift);
  } else {
    kend = rd.nz;
  }
  long long ncol = kend - c.next_col;
  if (ncol < 0) ncol = 0;
  nnew = rd.ppc > 0 ? ncol * rd.nperp * rd.ppc : 0;
}

template <int DIM, typename R>
__device__ __forceinline__ int tile_of(RunC& rd, int c) {
  using T = Tile<DIM, R>;
  const int tz = cell_k(c) >> T::LZ;
  const int tx = cell_i(c) >> T::LX;
  const int ty = DIM == 3 ? (cell_j(c) >> T::LY) : 0;
  return (ty * rd.ntx + tx) * rd.ntz + tz;
}

// wavefront-aggregated atomic add of 1 per active lane to base[key];
// returns the lane's slot (old value + rank among equal keys).  The key
// groups are found with ballots first; then the leader of every group makes
// its atomic in one instruction, so the wavefront waits for one round trip
// whatever the number of distinct keys.
__device__ __forceinline__ int wave_agg_add(PIC_G int* base, int key, bool active) {
  const int lane = threadIdx.x & 63;
  unsigned long long pend = __ballot(active);
  unsigned long long mine = 0;
  int lead = 0;
  while (pend) {
    const int leader = __ffsll((long long)pend) - 1;
    const int lkey = __shfl(key, leader);
    const unsigned long long m = __ballot(active && key == lkey);
    if ((m >> lane) & 1ull) {
      mine = m;
      lead = leader;
    }
    pend &= ~m;
  }
  int b = 0;
  if (active && lane == lead) b = g_add(base + key, (int)__popcll(mine));
  b = __shfl(b, lead);
  return b + (int)__popcll(mine & ((1ull << lane) - 1ull));
}

// Sort key of the particles of one source wavefront (uniform decision).
// The wavefront is a whole group if its 64 slots are live, span at most
// GZ + 1 consecutive z cells (two in split precision, where a group is one
// column; more where it interleaves columns) and lie in one tile's
// transverse range: all of them then go to the tile of the group's lowest
// cell, so the drift of the plasma never splits a group at a tile boundary
// (the upper members may sit up to GZ cells above the tile's z range; the
// step kernel's window covers them).
// Otherwise every particle goes to the tile of its own cell.
template <int DIM, typename R>
__device__ __forceinline__ int sort_key(RunC& rd, int cc, bool act, bool& whole) {
  using T = Tile<DIM, R>;
  const int own = act ? tile_of<DIM, R>(rd, cc) : 0;
  whole = false;
  if (__ballot(act) != ~0ull) return own;
  // the z range of the group from ballots of the lanes' offsets to lane 0's
  // cell (uniform values, no cross-lane shuffles): it spans at most GZ + 1
  // cells iff every lane lies within GZ of lane 0 and the lowest and
  // highest offsets present are at most GZ apart
  const int k = cell_k(cc), k0 = __builtin_amdgcn_readfirstlane(k);
  unsigned long long seen = 0;
  int lo = T::GZ + 1, hi = -T::GZ - 1;
#pragma unroll
  for (int d = -T::GZ; d <= T::GZ; ++d) {
    const unsigned long long b = __ballot(k - k0 == d);
    if (b) {
      lo = min(lo, d);
      hi = max(hi, d);
      seen |= b;
    }
  }
  if (seen != ~0ull || hi - lo > T::GZ) return own;
  const int kmin = k0 + lo;
  const int key = own - ((k >> T::LZ) - (kmin >> T::LZ));  // tiles are z-fastest
  whole = __ballot(key == __builtin_amdgcn_readfirstlane(key)) == ~0ull;
  return whole ? key : own;
}

// The work items of the runs that sort at this step, as one flat range:
// thread t reads run t's counters (in parallel) and counts that run's live
// items with count(rd) (the particles it creates, or the slots it holds, in
// chunks), the workgroup scans the counts in LDS, and item w maps back to
// its run by a binary search of the scan.  Counting live items, not the
// run's largest possible number, keeps every XCD busy: a cadence injection
// creates a few columns of a box sized for all of them, and its items would
// otherwise all fall in the first XCD's share of the range.  A step where no
// run sorts (most steps) costs one round of loads; a step where one small run
// of a large batch sorts touches only its items.  Every thread of the
// workgroup must call it; returns the number of items.
struct SortItems {
  long long pre[MAX_BATCH + 1];
};

template <typename Count>
__device__ __forceinline__ long long sort_items(const BatchTable* bt, SortItems& si, Count count) {
  const int n = bt->n;
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
    RunC& rd = *bt->run[r];
    si.pre[r + 1] = sort_due(*rd.ctr, rd.inject_every) ? count(rd) : 0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    long long acc = 0;
    si.pre[0] = 0;
    for (int r = 0; r < n; ++r) {
      acc += si.pre[r + 1];
      si.pre[r + 1] = acc;
    }
  }
  __syncthreads();
  return si.pre[n];
}

// live items of a run that sorts: chunks of the particles it creates, and
// chunks of its slots (the current ones and the created ones)
__device__ __forceinline__ long long inject_items(RunC& rd) {
  long long kend, nnew;
  pending(rd, *rd.ctr, kend, nnew);
  return (nnew + INJ_CHUNK - 1) / INJ_CHUNK;
}
__device__ __forceinline__ long long slot_items(RunC& rd) {
  long long kend, nnew;
  pending(rd, *rd.ctr, kend, nnew);
  const long long total = min(rd.ctr->n_slots + nnew, rd.capacity);
  return (total + PART_CHUNK - 1) / PART_CHUNK;
}

// the run of sorting item w: the last r with pre[r] <= w
__device__ __forceinline__ int sort_item_run(const SortItems& si, int n, long long w) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (si.pre[mid] <= w) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------------------ inject
// The b-th transverse cell (i, j) of an nx x ny plane enumerated tile by
// tile: rows of tiles of tx x ty cells, the tiles of a row left to right,
// the cells of a tile row by row; the last row and column of tiles may be
// narrower.
__device__ __forceinline__ void blocked_cell(unsigned b, int nx, int ny, int tx, int ty, int& i, int& j) {
  const unsigned tyi = b / (unsigned)(ty * nx);
  unsigned r = b - tyi * (unsigned)(ty * nx);
  const int wy = min(ty, ny - (int)tyi * ty);
  const unsigned txi = r / (unsigned)(tx * wy);
  r -= txi * (unsigned)(tx * wy);
  const int wx = min(tx, nx - (int)txi * tx);
  const unsigned jr = r / (unsigned)wx;
  j = (int)tyi * ty + (int)jr;
  i = (int)txi * tx + (int)(r - jr * (unsigned)wx);
}

template <typename R>
__global__ __launch_bounds__(256) void k_inject(const BatchTable* __restrict__ bt) {
  __shared__ SortItems si;
  const long long items = sort_items(bt, si, inject_items);
  if (items == 0) return;
  const XcdSplit xs(items);
  for (long long w = xs.beg; w < xs.end; w += xs.stride) {
    const int r = __builtin_amdgcn_readfirstlane(sort_item_run(si, bt->n, w));
    RunC& rd = *bt->run[r];
    const PIC_G Counters& c = *rd.ctr;
    long long kend, nnew;
    pending(rd, c, kend, nnew);
    const long long blk = w - si.pre[r];
    if (blk * INJ_CHUNK >= nnew) continue;
    const int pb = c.pbuf;
    const long long per_col = rd.nperp * rd.ppc;
    const double shift = rd.open ? rd.beta_b * ((double)c.step * rd.dt) / rd.dz : 0.0;
    for (int t = threadIdx.x; t < INJ_CHUNK; t += 256) {
      const long long q = blk * INJ_CHUNK + t;
      if (q >= nnew) break;
      const long long slot = c.n_slots + q;
      if (slot >= rd.capacity) {
        g_or(&rd.ctr->err, 2u);
        break;
      }
      // slot outermost within a column, the transverse cells in tile-blocked
      // order: in split precision a wavefront creates one lattice slot of
      // the 8x8 cells of one tile's transverse plane, which the sort keeps
      // together, so the lanes of a wavefront of the step kernel start in 64
      // different cells and their LDS current atomics do not share
      // addresses; smaller planes interleave columns (below).  The lattice
      // id does not depend on this order.
      // q < nnew and per_col are below the capacity (< 2^31): 32-bit
      // unsigned divisions, a few instructions each instead of the long
      // 64-bit sequences
      const unsigned qu = (unsigned)q, pc = (unsigned)per_col, npu = (unsigned)rd.nperp;
      unsigned kq, slu, bq;
      // cells of one tile plane (8x8 split 3D, 8x4 FP64 3D, 16 in 2D) and
      // the columns a wavefront interleaves so that it still covers 64 cells
      const unsigned plane = rd.dims == 3 ? (unsigned)(Tile<3, R>::TX * Tile<3, R>::TY) : (unsigned)Tile<2, R>::TX;
      const unsigned ncw = 64 / plane;
      const unsigned ncol = (unsigned)(nnew / per_col);
      if (ncw > 1 && ncol >= ncw && qu / (ncw * pc) < ncol / ncw) {  // ncw * pc <= nnew < 2^31
        // columns in groups of ncw: a wavefront creates one slot of one
        // plane in each of columns K .. K+ncw-1 (different z cells), so the
        // step kernel's wavefronts still start in 64 different cells
        const unsigned kg = qu / (ncw * pc), r1 = qu - kg * ncw * pc;
        slu = r1 / (ncw * npu);
        const unsigned r2 = r1 - slu * ncw * npu, blk = r2 / 64, within = r2 - blk * 64;
        kq = ncw * kg + within / plane;
        bq = blk * plane + within % plane;
      } else {  // one column at a time (also the columns left over from the groups)
        kq = qu / pc;
        const unsigned rem = qu - kq * pc;
        slu = rem / npu;
        bq = rem - slu * npu;
      }
      const long long K = c.next_col + (long long)kq;
      const long long sl = (long long)slu;
      int i, j;
      blocked_cell(bq, rd.nx, rd.dims == 3 ? rd.ny : 1, rd.dims == 3 ? Tile<3, R>::TX : Tile<2, R>::TX,
                   rd.dims == 3 ? Tile<3, R>::TY : 1, i, j);
      const long long cperp = (long long)j * rd.nx + i;
      const uint64_t L = (uint64_t)((K * rd.nperp + cperp) * rd.ppc + sl);
      uint64_t a[4] = {L, 0, 0, 0}, b[4] = {L, 1, 0, 0};
      philox4x64_10(a, rd.seed, 0);
      philox4x64_10(b, rd.seed, 0);
      const double xz = u01(a[0]), xx = u01(a[1]), xy = u01(a[2]);
      // laboratory Maxwellian (Box-Muller on 1-U in (0,1]), then the boost
      const double m0 = sqrt(-2.0 * log(1.0 - u01(a[3])));
      const double p0 = 2.0 * M_PI * u01(b[0]);
      const double m1 = sqrt(-2.0 * log(1.0 - u01(b[1])));
      const double p1 = 2.0 * M_PI * u01(b[2]);
      const double lx = rd.u_th * m0 * cos(p0), ly = rd.u_th * m0 * sin(p0), lz = rd.u_th * m1 * cos(p1);
      const double gl = sqrt(1.0 + lx * lx + ly * ly + lz * lz);
      const double bz = rd.gamma_b * (lz - rd.beta_b * gl);
      // split positions: integer cell + offset stored in R
      double zeta[3] = {((double)K + xz) - shift, (double)i + xx, (double)j + xy};
      int cidx[3];
      R off[3];
      for (int d = 0; d < 3; ++d) {
        double fl = floor(zeta[d]);
        R o = R(zeta[d] - fl);
        if (o >= R(1)) {
          o = R(0);
          fl += 1.0;
        }
        cidx[d] = (int)fl;
        off[d] = o;
      }
      if (cidx[1] >= rd.nx) cidx[1] -= rd.nx;
      if (rd.dims == 3 && cidx[2] >= rd.ny) cidx[2] -= rd.ny;
      const int cj = rd.dims == 3 ? cidx[2] : 0;
      rd.cell[pb][slot] = cell_pack(cidx[0], cidx[1], cj);
      fptr<R>(rd.off[pb][0])[slot] = off[0];
      fptr<R>(rd.off[pb][1])[slot] = off[1];
      if (rd.dims == 3) fptr<R>(rd.off[pb][2])[slot] = off[2];
      fptr<R>(rd.u[pb][0])[slot] = R(lx);
      fptr<R>(rd.u[pb][1])[slot] = R(ly);
      fptr<R>(rd.u[pb][2])[slot] = R(bz);
      rd.pid[pb][slot] = (unsigned)L;
    }
  }
}

// ------------------------------------------------------------------ count
// Per-tile counts of a work item, gathered in a small LDS hash table first:
// the slots of an item (consecutive, sorted by tile at the previous sort)
// fall into a handful of tiles, so the global counters, which every item of
// a tile would otherwise hit wavefront by wavefront, take a few atomics per
// item.  A table that fills up (never with sorted input) counts directly.
constexpr int COUNT_HASH = 64;

template <int DIM, typename R>
__global__ __launch_bounds__(256) void k_count(const BatchTable* __restrict__ bt) {
  __shared__ SortItems si;
  __shared__ int hkey[COUNT_HASH], hcnt[COUNT_HASH], hfull[COUNT_HASH];
  const long long items = sort_items(bt, si, slot_items);
  if (items == 0) return;
  const int lane = threadIdx.x & 63;
  const XcdSplit xs(items);
  for (long long w = xs.beg; w < xs.end; w += xs.stride) {
    const int r = __builtin_amdgcn_readfirstlane(sort_item_run(si, bt->n, w));
    RunC& rd = *bt->run[r];
    const PIC_G Counters& c = *rd.ctr;
    long long kend, nnew;
    pending(rd, c, kend, nnew);
    long long total = c.n_slots + nnew;
    if (total > rd.capacity) total = rd.capacity;
    const long long blk = w - si.pre[r];
    if (blk * PART_CHUNK >= total) continue;  // uniform over the workgroup
    for (int e = threadIdx.x; e < COUNT_HASH; e += 256) {
      hkey[e] = -1;
      hcnt[e] = 0;
      hfull[e] = 0;
    }
    __syncthreads();
    // n particles go to tile key (full: as a whole group)
    auto tally = [&](int key, int n, bool full) {
      int h = key & (COUNT_HASH - 1);
#pragma nounroll
      for (int probe = 0; probe < COUNT_HASH; ++probe) {
        const int prev = atomicCAS(&hkey[h], -1, key);
        if (prev == -1 || prev == key) {
          atomicAdd(&hcnt[h], n);
          if (full) atomicAdd(&hfull[h], n);
          return;
        }
        h = (h + 1) & (COUNT_HASH - 1);
      }
      (void)g_add(rd.tile_count + key, n);
      if (full) (void)g_add(rd.tile_full + key, n);
    };
    const PIC_G int* cellp = rd.cell[c.pbuf];
    // all the item's loads first (the key computation below waits on each)
    constexpr int PER = PART_CHUNK / 256;
    int cv[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const long long q = blk * PART_CHUNK + threadIdx.x + u * 256;
      cv[u] = q < total ? cellp[q] : -1;
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int cc = cv[u];
      const bool act = cc >= 0;
      bool whole;
      const int key = sort_key<DIM, R>(rd, cc, act, whole);
      if (whole) {
        if (lane == 0) tally(key, 64, true);
      } else {
        // one tally per distinct key of the wavefront
        unsigned long long pend = __ballot(act);
        while (pend) {
          const int leader = __ffsll((long long)pend) - 1;
          const int lkey = __shfl(key, leader);
          const unsigned long long m = __ballot(act && key == lkey);
          if (lane == leader) tally(lkey, (int)__popcll(m), false);
          pend &= ~m;
        }
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < COUNT_HASH; e += 256) {
      const int k = hkey[e];
      if (k >= 0) {
        if (hcnt[e]) (void)g_add(rd.tile_count + k, hcnt[e]);
        if (hfull[e]) (void)g_add(rd.tile_full + k, hfull[e]);
      }
    }
    __syncthreads();  // the table is cleared for the next item
  }
}

// ------------------------------------------------------------------ scan
__global__ __launch_bounds__(1024) void k_scan(const BatchTable* __restrict__ bt) {
  if ((int)blockIdx.x >= bt->n) return;
  RunC& rd = *bt->run[blockIdx.x];
  PIC_G Counters* c = rd.ctr;
  if (!sort_due(*c, rd.inject_every)) return;
  __shared__ int wsum[16], lsum[16];
  const int n = rd.ntiles;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // tile t occupies pad64(count) slots
  auto pad64 = [](int v) { return (v + 63) & ~63; };
  PIC_G int* dcell = rd.cell[c->pbuf ^ 1];
  // blocks of 1024 consecutive tiles, one per thread (coalesced); the
  // running total (carry) is the same in every thread
  int carry = 0, live = 0;
  for (int base = 0; base < n; base += 1024) {
    const int t = base + (int)threadIdx.x;
    const int cnt = t < n ? rd.tile_count[t] : 0;
    const int full = t < n ? rd.tile_full[t] : 0;
    const int sz = pad64(cnt);
    live += cnt;
    // inclusive scan of the padded sizes: wavefront shuffles, then waves
    int v = sz;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int o = __shfl_up(v, d);
      if (lane >= d) v += o;
    }
    if (lane == 63) wsum[wave] = v;
    __syncthreads();
    int wpre = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int x = wsum[q];
      wpre += q < wave ? x : 0;
      tot += x;
    }
    const int start = carry + wpre + v - sz;  // exclusive prefix
    if (t < n) {
      rd.tile_start[t] = start;
      rd.tile_full[t] = start;            // whole groups from the front
      rd.tile_cursor[t] = start + full;   // then the other particles
      rd.tile_count[t] = 0;
    }
    // padding, marked removed: the tail of each tile's last 64-slot block
    // (every start is a multiple of 64), one wavefront store per tile
    const int padn = sz - cnt, pbeg = start + cnt;
#pragma unroll 8
    for (int j = 0; j < 64; ++j) {
      const int pj = __shfl(padn, j), ej = __shfl(pbeg, j);
      if (lane < pj) dcell[ej + lane] = -1;
    }
    carry += tot;
    __syncthreads();  // wsum is reused by the next block
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) live += __shfl_xor(live, d);
  if (lane == 0) lsum[wave] = live;
  __syncthreads();
  if (threadIdx.x == 0) {
    int lt = 0;
    for (int q = 0; q < 16; ++q) lt += lsum[q];
    rd.tile_start[n] = carry;
    c->n_live = lt;
    c->n_padded = carry;
  }
}

// ------------------------------------------------------------------ scatter
template <int DIM, typename R>
__global__ __launch_bounds__(256) void k_scatter(const BatchTable* __restrict__ bt) {
  __shared__ SortItems si;
  const long long items = sort_items(bt, si, slot_items);
  if (items == 0) return;
  const XcdSplit xs(items);
  for (long long w = xs.beg; w < xs.end; w += xs.stride) {
    const int r = __builtin_amdgcn_readfirstlane(sort_item_run(si, bt->n, w));
    RunC& rd = *bt->run[r];
    const PIC_G Counters& c = *rd.ctr;
    long long kend, nnew;
    pending(rd, c, kend, nnew);
    long long total = c.n_slots + nnew;
    if (total > rd.capacity) total = rd.capacity;
    const long long blk = w - si.pre[r];
    if (blk * PART_CHUNK >= total) continue;
    const int src = c.pbuf, dst = src ^ 1;
    const PIC_G int* cellp = rd.cell[src];
    for (int t = threadIdx.x; t < PART_CHUNK; t += 256) {
      const long long q = blk * PART_CHUNK + t;
      int cc = -1;
      if (q < total) cc = cellp[q];
      const bool act = cc >= 0;
      // the payload is loaded before the slot is known, so its latency
      // overlaps the cursor atomic's
      R v[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
      unsigned id = 0;
      if (act) {
        v[0] = fptr<R>(rd.off[src][0])[q];
        v[1] = fptr<R>(rd.off[src][1])[q];
        if (DIM == 3) v[2] = fptr<R>(rd.off[src][2])[q];
        v[3] = fptr<R>(rd.u[src][0])[q];
        v[4] = fptr<R>(rd.u[src][1])[q];
        v[5] = fptr<R>(rd.u[src][2])[q];
        id = rd.pid[src][q];
      }
      bool whole;
      const int key = sort_key<DIM, R>(rd, cc, act, whole);
      int slot;
      if (whole) {
        int b = 0;
        if ((threadIdx.x & 63) == 0) b = g_add(rd.tile_full + key, 64);
        slot = __shfl(b, 0) + (int)(threadIdx.x & 63);
      } else {
        slot = wave_agg_add(rd.tile_cursor, key, act);
      }
      if (act) {
        rd.cell[dst][slot] = cc;
        fptr<R>(rd.off[dst][0])[slot] = v[0];
        fptr<R>(rd.off[dst][1])[slot] = v[1];
        if (DIM == 3) fptr<R>(rd.off[dst][2])[slot] = v[2];
        fptr<R>(rd.u[dst][0])[slot] = v[3];
        fptr<R>(rd.u[dst][1])[slot] = v[4];
        fptr<R>(rd.u[dst][2])[slot] = v[5];
        rd.pid[dst][slot] = id;
      }
    }
  }
}

// The scan turned the whole-group counts into the front cursors the scatter
// used: zero them for the next sort's count (a flat range over the tiles of
// the runs that sort).
__global__ __launch_bounds__(256) void k_full_reset(const BatchTable* __restrict__ bt) {
  __shared__ SortItems si;
  const long long items = sort_items(bt, si, [](RunC& rd) { return (long long)rd.ntiles; });
  if (items == 0) return;
  for (long long w = (long long)blockIdx.x * 256 + threadIdx.x; w < items; w += (long long)gridDim.x * 256) {
    const int r = sort_item_run(si, bt->n, w);
    bt->run[r]->tile_full[w - si.pre[r]] = 0;
  }
}

// ------------------------------------------------------------------ commit
__global__ void k_commit(const BatchTable* __restrict__ bt) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= bt->n) return;
  RunC& rd = *bt->run[r];
  PIC_G Counters* c = rd.ctr;
  if (!sort_due(*c, rd.inject_every)) return;
  long long kend, nnew;
  pending(rd, *c, kend, nnew);
  if (c->n_slots + nnew > rd.capacity) c->err |= 2u;
  if (kend > c->next_col) c->next_col = kend;
  c->n_slots = c->n_padded;
  c->pbuf ^= 1;
  c->fresh = 1;
  c->last_sort = c->step;
  c->want_sort = 0;
}

template <int DIM, typename R>
static void chain(const BatchTable* bt, int nruns, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_inject<R>), dim3(grid), dim3(256), 0, s, bt);
  hipLaunchKernelGGL((k_count<DIM, R>), dim3(grid), dim3(256), 0, s, bt);
  hipLaunchKernelGGL(k_scan, dim3(nruns), dim3(1024), 0, s, bt);
  hipLaunchKernelGGL((k_scatter<DIM, R>), dim3(grid), dim3(256), 0, s, bt);
  hipLaunchKernelGGL(k_full_reset, dim3(grid), dim3(256), 0, s, bt);
  hipLaunchKernelGGL(k_commit, dim3((nruns + 63) / 64), dim3(64), 0, s, bt);
}

void launch_sort_chain(int dims, int prec, const BatchTable* bt, int nruns, int grid, hipStream_t s) {
  if (dims == 3) {
    if (prec) chain<3, double>(bt, nruns, grid, s); else chain<3, float>(bt, nruns, grid, s);
  } else {
    if (prec) chain<2, double>(bt, nruns, grid, s); else chain<2, float>(bt, nruns, grid, s);
  }
}

}  // namespace pic
