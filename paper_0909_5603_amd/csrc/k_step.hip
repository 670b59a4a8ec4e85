// One boosted-frame PIC step on gfx950: the fused particle kernel (gather,
// push, move, charge-conserving deposit) and the single-pass Yee update.
//
// Particle kernel.  Particles are stored tile by tile (counting sort every
// sort_every steps).  A workgroup takes one tile: it stages E^n and
// B^{n-1/2} of the tile's window in LDS, advances B to integer time there,
// zeroes an LDS current window, runs its particles through
//   gather (linear interpolation at each component's Yee stagger),
//   push (modified Lorentz force with analytic gamma, Vay 2008),
//   move (int cell + in-cell offset, one carry per dimension),
//   deposit (Esirkepov 2001, linear shape, into LDS in 64-bit fixed point
//   with ds_add_u64: the integer LDS atomics run ~30x faster than ds_add_f32
//   on gfx950 and make the sum independent of the order of the particles),
// and flushes the window's current to HBM with 64-bit integer atomics.  The window
// follows the bounding box of the tile's particles measured in the previous
// step, so it tracks the plasma as it streams through the boosted frame.
// Particles whose stencil leaves the window take a slow path that reads and
// deposits in HBM directly: results never depend on the window.
//
// Field update.  State is (E^n, B^{n-1/2}) in ping-pong buffers: B^{n+1/2} =
// B^{n-1/2} - dt curl E^n, then E^{n+1} = E^n + dt (curl B^{n+1/2} - J -
// J_ion), then first-order Mur on the tangential E at open z ends.  The
// current is double-buffered: the step deposits into J[fbuf], the E pass reads
// it and clears J[fbuf^1], into which the next step deposits.  This is the
// standard leapfrog, algebraically equal to two half steps of B around the E
// step with E and B both at integer time.
#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "pic_dev.hpp"
#include "pusher.hpp"

namespace pic {

// ------------------------------------------------------------------ helpers
template <typename R>
struct W1 {
  R n0, n1;  // node-centred weights at offsets 0, +1
  R h0, h1;  // half-cell weights at offsets hb, hb+1
  int hb;
};

template <typename R>
__device__ __forceinline__ W1<R> weights(R o) {
  W1<R> w;
  w.n0 = R(1) - o;
  w.n1 = o;
  const bool up = o >= R(0.5);
  w.hb = up ? 0 : -1;
  w.h0 = up ? R(1.5) - o : R(0.5) - o;
  w.h1 = up ? o - R(0.5) : R(0.5) + o;
  return w;
}

// linear interpolation of component C from its own stagger
template <int DIM, int C, typename R, class F>
__device__ __forceinline__ R interp(const W1<R>* w, F&& fetch) {
  constexpr bool sz = stag(C, 0), sx = stag(C, 1), sy = stag(C, 2);
  const R z0 = sz ? w[0].h0 : w[0].n0, z1 = sz ? w[0].h1 : w[0].n1;
  const R x0 = sx ? w[1].h0 : w[1].n0, x1 = sx ? w[1].h1 : w[1].n1;
  const int oz = sz ? w[0].hb : 0, ox = sx ? w[1].hb : 0;
  if constexpr (DIM == 3) {
    const R y0 = sy ? w[2].h0 : w[2].n0, y1 = sy ? w[2].h1 : w[2].n1;
    const int oy = sy ? w[2].hb : 0;
    // the 8 loads first, then the arithmetic: keeps four LDS reads in
    // flight instead of waiting on each one
    R v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = fetch(C, oz + (q & 1), ox + ((q >> 1) & 1), oy + (q >> 2));
    __builtin_amdgcn_sched_group_barrier(0x100, 8, 0);  // DS reads
    __builtin_amdgcn_sched_group_barrier(0x002, 14, 0);  // then VALU
    const R a = z0 * v[0] + z1 * v[1];
    const R b = z0 * v[2] + z1 * v[3];
    const R c = z0 * v[4] + z1 * v[5];
    const R d = z0 * v[6] + z1 * v[7];
    return y0 * (x0 * a + x1 * b) + y1 * (x0 * c + x1 * d);
  } else {
    const R a = z0 * fetch(C, oz, ox, 0) + z1 * fetch(C, oz + 1, ox, 0);
    const R b = z0 * fetch(C, oz, ox + 1, 0) + z1 * fetch(C, oz + 1, ox + 1, 0);
    return x0 * a + x1 * b;
  }
}

// Esirkepov shape data along one dimension.  The 3-node window starts at
// min(old cell, new cell) = old cell + base.  S0 = old node shapes, DS = new
// minus old, P[a] = sum_{a'<=a} DS[a'] (P[2] = 0), written directly from the
// offsets so that no cancellation is lost.
template <typename R>
struct Dep1 {
  R S0[3], DS[3], P[2];
  int base;
};

template <typename R>
__device__ __forceinline__ Dep1<R> dep1(R o0, R o1, int carry) {
  Dep1<R> d;
  const bool dn = carry < 0, up = carry > 0;
  const R a0 = R(1) - o0, a1 = R(1) - o1;
  d.S0[0] = dn ? R(0) : a0;
  d.S0[1] = dn ? a0 : o0;
  d.S0[2] = dn ? o0 : R(0);
  const R s10 = up ? R(0) : a1;
  const R s11 = up ? a1 : o1;
  const R s12 = up ? o1 : R(0);
  d.DS[0] = s10 - d.S0[0];
  d.DS[1] = s11 - d.S0[1];
  d.DS[2] = s12 - d.S0[2];
  // P[0] = o0 - o1, o0 - 1 or 1 - o1 (stay, up, down) as one rounded
  // difference; P[1] = -DS[2] = 0, -o1 or o0, exactly
  d.P[0] = (dn ? R(1) : o0) - (up ? R(1) : o1);
  d.P[1] = d.S0[2] - s12;
  d.base = dn ? -1 : 0;
  return d;
}

// Esirkepov shape data along a dimension in which no lane of the wavefront
// crossed a cell boundary: the window is the particle's own two nodes.  The
// values are rounded exactly as dep1 rounds them for a particle that stays,
// so a particle's current does not depend on the other lanes of its
// wavefront.
template <typename R>
__device__ __forceinline__ Dep1<R> dep1_stay(R o0, R o1) {
  Dep1<R> d;
  const R a0 = R(1) - o0;
  d.S0[0] = a0;
  d.S0[1] = o0;
  d.S0[2] = R(0);
  d.DS[0] = (R(1) - o1) - a0;
  d.DS[1] = o1 - o0;
  d.DS[2] = R(0);
  d.P[0] = o0 - o1;
  d.P[1] = R(0);
  d.base = 0;
  return d;
}

// offset carry after a move of less than one cell (CFL): o in (-1, 2) ->
// carry floor(o) in {-1, 0, 1} and offset o - floor(o), which is exact for
// o >= 0 and rounded for o < 0; when o + 1 rounds to 1 the particle stays
// in its cell at offset 0
template <typename R>
__device__ __forceinline__ int carry(R& o) {
  const R f = floor(o);
  const R on = o - f;
  const bool up1 = on == R(1);
  o = up1 ? R(0) : on;
  return (int)f + (up1 ? 1 : 0);
}

// A current contribution x, already in fixed-point units, as a 64-bit
// integer.  Split precision: |x| < 2^30 by the choice of the scale, one
// v_cvt_rpi_i32_f32 (floor(x + 1/2)) and a sign extension.  FP64: |x| < 2^51,
// adding 1.5 * 2^52 leaves the rounded integer in the low mantissa bits.
__device__ __forceinline__ long long fixq(float x) {
  int r;
  asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return (long long)r;
}
__device__ __forceinline__ long long fixq(double x) { return to_fixed(x, 1.0); }

// Charge-conserving current of one particle, linear shape (Esirkepov 2001),
// factored as J = c P[a] F(b,c): P is the running sum of the shape change
// along the current's direction and F the time-averaged shape across it.
// The coefficient c times the fixed-point scale is folded into P (cz, cx, cy
// below), and add(comp, a, b, c, q) receives node offsets from the start of
// the particle's 3-node window.  NX, NY = nodes visited across x and y: 3
// when some lane of the wavefront crossed a cell boundary in that dimension,
// else 2 (the third node and the second face then carry exact zeros).  Zero contributions are added like any other: a branch per
// contribution costs more than the LDS atomic it saves.
template <typename R, int NX, int NY, class A>
__device__ __forceinline__ void dep3(const Dep1<R>& Z, const Dep1<R>& X, const Dep1<R>& Y, R cz, R cx,
                                     R cy, A&& add) {
  R Ay[3], By[3], Ax[3], Bx[3];
#pragma unroll
  for (int c = 0; c < NY; ++c) {
    Ay[c] = Y.S0[c] + R(0.5) * Y.DS[c];
    By[c] = R(0.5) * Y.S0[c] + R(1.0 / 3.0) * Y.DS[c];
  }
#pragma unroll
  for (int b = 0; b < NX; ++b) {
    Ax[b] = X.S0[b] + R(0.5) * X.DS[b];
    Bx[b] = R(0.5) * X.S0[b] + R(1.0 / 3.0) * X.DS[b];
  }
  const R pz0 = Z.P[0] * cz, pz1 = Z.P[1] * cz;
  // J_z(face a; node b, c) = cz P_z[a] (S0x Ay + DSx By)
#pragma unroll
  for (int b = 0; b < NX; ++b)
#pragma unroll
    for (int c = 0; c < NY; ++c) {
      const R f = X.S0[b] * Ay[c] + X.DS[b] * By[c];
      add(2, 0, b, c, fixq(pz0 * f));
      add(2, 1, b, c, fixq(pz1 * f));
    }
  // J_x(node a; face b; node c) = cx P_x[b] (S0z Ay + DSz By)
  R px[2], py[2];
#pragma unroll
  for (int b = 0; b < NX - 1; ++b) px[b] = X.P[b] * cx;
#pragma unroll
  for (int c = 0; c < NY - 1; ++c) py[c] = Y.P[c] * cy;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < NY; ++c) {
      const R f = Z.S0[a] * Ay[c] + Z.DS[a] * By[c];
#pragma unroll
      for (int b = 0; b < NX - 1; ++b) add(0, a, b, c, fixq(px[b] * f));
    }
  // J_y(node a, b; face c) = cy P_y[c] (S0z Ax + DSz Bx)
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < NX; ++b) {
      const R f = Z.S0[a] * Ax[b] + Z.DS[a] * Bx[b];
#pragma unroll
      for (int c = 0; c < NY - 1; ++c) add(1, a, b, c, fixq(py[c] * f));
    }
}

// 2D3V: J_z = cz P_z (S0x + DSx/2), J_x = cx P_x (S0z + DSz/2), and the
// out-of-plane J_y = q w v_y times the time-averaged node shape (cyv = its
// coefficient times v_y).
template <typename R, int NX, class A>
__device__ __forceinline__ void dep2(const Dep1<R>& Z, const Dep1<R>& X, R cz, R cx, R cyv, A&& add) {
  R Ax[3], Bx[3];
#pragma unroll
  for (int b = 0; b < NX; ++b) {
    Ax[b] = X.S0[b] + R(0.5) * X.DS[b];
    Bx[b] = R(0.5) * X.S0[b] + R(1.0 / 3.0) * X.DS[b];
  }
  const R pz0 = Z.P[0] * cz, pz1 = Z.P[1] * cz;
#pragma unroll
  for (int b = 0; b < NX; ++b) {
    add(2, 0, b, 0, fixq(pz0 * Ax[b]));
    add(2, 1, b, 0, fixq(pz1 * Ax[b]));
  }
  R px[2];
#pragma unroll
  for (int b = 0; b < NX - 1; ++b) px[b] = X.P[b] * cx;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const R az = Z.S0[a] + R(0.5) * Z.DS[a];
#pragma unroll
    for (int b = 0; b < NX - 1; ++b) add(0, a, b, 0, fixq(px[b] * az));
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const R sa = Z.S0[a] * cyv, da = Z.DS[a] * cyv;
#pragma unroll
    for (int b = 0; b < NX; ++b) add(1, a, b, 0, fixq(sa * Ax[b] + da * Bx[b]));
  }
}

// The deposit of one particle, in the variant of its wavefront: the shape
// data across x and y are those of a 3-node window where some lane of the
// wavefront crossed a cell boundary in that dimension, else of the
// particle's own two nodes.  adder(zb, xb, yb) gives the accumulator of the
// window that starts at (zb, xb, yb) from the old cell.
template <int DIM, typename R, class AF>
__device__ __forceinline__ void deposit(const Dep1<R>& Z, const R* o, const R* on, const int* cr, R cz, R cx,
                                        R cy, R cyv, AF&& adder) {
  // wavefront-uniform: does any active lane cross a cell boundary in x, in y?
  if constexpr (DIM == 3) {
    const bool ax = __any(cr[1] != 0), ay = __any(cr[2] != 0);
    if (ax) {
      const Dep1<R> X = dep1(o[1], on[1], cr[1]);
      if (ay) {
        const Dep1<R> Y = dep1(o[2], on[2], cr[2]);
        dep3<R, 3, 3>(Z, X, Y, cz, cx, cy, adder(Z.base, X.base, Y.base));
      } else {
        dep3<R, 3, 2>(Z, X, dep1_stay(o[2], on[2]), cz, cx, cy, adder(Z.base, X.base, 0));
      }
    } else {
      const Dep1<R> X = dep1_stay(o[1], on[1]);
      if (ay) {
        const Dep1<R> Y = dep1(o[2], on[2], cr[2]);
        dep3<R, 2, 3>(Z, X, Y, cz, cx, cy, adder(Z.base, 0, Y.base));
      } else {
        dep3<R, 2, 2>(Z, X, dep1_stay(o[2], on[2]), cz, cx, cy, adder(Z.base, 0, 0));
      }
    }
  } else {
    if (__any(cr[1] != 0)) {
      const Dep1<R> X = dep1(o[1], on[1], cr[1]);
      dep2<R, 3>(Z, X, cz, cx, cyv, adder(Z.base, X.base, 0));
    } else {
      dep2<R, 2>(Z, dep1_stay(o[1], on[1]), cz, cx, cyv, adder(Z.base, 0, 0));
    }
  }
}

// E value with HBM index handling (zero outside an open z range).  Indices
// are at most a few cells outside the box, so one correction wraps them.
template <int DIM, typename R>
__device__ __forceinline__ R gE(RunC& rd, const Arr3<R>& E, int comp, int k, int i, int j) {
  i = wrap1(i, rd.nx);
  j = DIM == 3 ? wrap1(j, rd.ny) : 0;
  if (rd.open) {
    if (k < 0 || k >= zcount(rd, comp)) return R(0);
  } else {
    k = wrap1(k, rd.nz);
  }
  return E[comp][gidx(rd, k, i, j)];
}

// field value at integer time n for the HBM path: E directly, B advanced
// from n-1/2 on the fly
template <int DIM, typename R>
__device__ R fetch_hbm(RunC& rd, const Arr3<R>& E, const Arr3<R>& B, int comp, int k, int i, int j) {
  if (comp < 3) return gE<DIM, R>(rd, E, comp, k, i, j);
  int ii = wrap1(i, rd.nx), jj = DIM == 3 ? wrap1(j, rd.ny) : 0, kk = k;
  if (rd.open) {
    if (k < 0 || k >= zcount(rd, comp)) return R(0);
  } else {
    kk = wrap1(k, rd.nz);
  }
  const R b = B[comp - 3][gidx(rd, kk, ii, jj)];
  const R idz = R(1.0 / rd.dz), idx = R(1.0 / rd.dx), idy = DIM == 3 ? R(1.0 / rd.dy) : R(0);
  R curl;
  if (comp == 3)
    curl = (DIM == 3 ? (gE<DIM, R>(rd, E, 2, k, i, j + 1) - gE<DIM, R>(rd, E, 2, k, i, j)) * idy : R(0)) -
           (gE<DIM, R>(rd, E, 1, k + 1, i, j) - gE<DIM, R>(rd, E, 1, k, i, j)) * idz;
  else if (comp == 4)
    curl = (gE<DIM, R>(rd, E, 0, k + 1, i, j) - gE<DIM, R>(rd, E, 0, k, i, j)) * idz -
           (gE<DIM, R>(rd, E, 2, k, i + 1, j) - gE<DIM, R>(rd, E, 2, k, i, j)) * idx;
  else
    curl = (gE<DIM, R>(rd, E, 1, k, i + 1, j) - gE<DIM, R>(rd, E, 1, k, i, j)) * idx -
           (DIM == 3 ? (gE<DIM, R>(rd, E, 0, k, i, j + 1) - gE<DIM, R>(rd, E, 0, k, i, j)) * idy : R(0));
  return b - R(0.5 * rd.dt) * curl;
}

template <int DIM>
__device__ __forceinline__ void add_hbm(RunC& rd, int fb, int comp, int k, int i, int j, long long q) {
  i = wrap1(i, rd.nx);
  j = DIM == 3 ? wrap1(j, rd.ny) : 0;
  if (rd.open) {
    if (k < 0 || k >= zcount(rd, comp)) return;  // current outside the box is dropped
  } else {
    k = wrap1(k, rd.nz);
  }
  g_add((PIC_G unsigned long long*)rd.J[fb][comp] + gidx(rd, k, i, j), (unsigned long long)q);
}

// ------------------------------------------------------------------ particles
// constants of the particle update
template <typename R>
struct PConst {
  R eps, cdz, cdx, cdy;
  R cz, cx, cy, cyv;  // current coefficients times the fixed-point scale
};

template <int DIM, typename R>
__device__ __forceinline__ PConst<R> pconst(RunC& rd) {
  // computed once on the host (the FP64 divisions cost ~100 VALU
  // instructions per tile and wavefront when done here)
  PConst<R> K;
  K.eps = R(rd.pk[0]);
  K.cdz = R(rd.pk[1]);
  K.cdx = R(rd.pk[2]);
  K.cdy = R(rd.pk[3]);
  K.cz = R(rd.pk[4]);
  K.cx = R(rd.pk[5]);
  K.cy = R(rd.pk[6]);
  K.cyv = R(rd.pk[7]);
  return K;
}

// Gather, push, move and deposit of one particle.  o[] holds the old
// offsets on entry and the new ones on exit, cr[] receives the cell carries.
// fetch(comp, dk, di, dj) addresses fields relative to the particle's old
// cell; adder(dk, di, dj) returns the current accumulator add(comp, a, b, c,
// q) of the deposit window that starts at (dk, di, dj) from the old cell.
// Returns true if the new momentum is not finite.
template <int DIM, typename R, int PUSHER, class F, class A>
__device__ __forceinline__ bool advance(const PConst<R>& K, R* o, R& ux, R& uy, R& uz, int* cr,
                                        F&& fetch, A&& adder) {
  W1<R> wt[3];
  wt[0] = weights(o[0]);
  wt[1] = weights(o[1]);
  if (DIM == 3) wt[2] = weights(o[2]);
  const R ex = interp<DIM, 0, R>(wt, fetch);
  const R ey = interp<DIM, 1, R>(wt, fetch);
  const R ez = interp<DIM, 2, R>(wt, fetch);
  const R bx = interp<DIM, 3, R>(wt, fetch);
  const R by = interp<DIM, 4, R>(wt, fetch);
  const R bz = interp<DIM, 5, R>(wt, fetch);
  if (PUSHER == 1)
    push_boris<R>(ux, uy, uz, ex, ey, ez, bx, by, bz, K.eps);
  else
    push_vay<R>(ux, uy, uz, ex, ey, ez, bx, by, bz, K.eps);
  const R ig = frsq(R(1) + ux * ux + uy * uy + uz * uz);
  const bool bad = !(ig > R(0));  // 1 + u^2 infinite or NaN
  R on[3];
  on[0] = o[0] + K.cdz * uz * ig;
  on[1] = o[1] + K.cdx * ux * ig;
  on[2] = DIM == 3 ? o[2] + K.cdy * uy * ig : R(0);
  cr[0] = carry(on[0]);
  cr[1] = carry(on[1]);
  cr[2] = DIM == 3 ? carry(on[2]) : 0;
  deposit<DIM, R>(dep1(o[0], on[0], cr[0]), o, on, cr, K.cz, K.cx, K.cy, K.cyv * (uy * ig), adder);
  o[0] = on[0];
  o[1] = on[1];
  o[2] = on[2];
  return bad;
}

// new packed cell after the carries; removal at the open z ends.  wrap =
// false (uniform) when no particle of the tile can cross a periodic
// boundary: the carries are then added to the packed fields directly.
template <int DIM>
__device__ __forceinline__ int new_cell(RunC& rd, int c, int k, int i, int j, const int* cr, bool wrap,
                                        bool& dead, int& k1, int& i1, int& j1) {
  const bool open = rd.open != 0;
  int nc;
  if (wrap) {
    k1 = wrapu(k + cr[0], open ? 0 : rd.nz);
    i1 = wrapu(i + cr[1], rd.nx);
    j1 = DIM == 3 ? wrapu(j + cr[2], rd.ny) : 0;
    nc = cell_pack(k1, i1, j1);
  } else {
    k1 = k + cr[0];
    i1 = i + cr[1];
    j1 = DIM == 3 ? j + cr[2] : 0;
    nc = c + cr[0] + (cr[1] << KBITS) + (DIM == 3 ? cr[2] << (KBITS + IBITS) : 0);
  }
  dead = open && (unsigned)k1 >= (unsigned)rd.ztop;  // left through z = 0 or beyond ztop
  return nc | (dead ? (int)DEAD : 0);
}

// Per-tile geometry of a batch work item: the run, the tile, its particle
// slots, and the LDS window (the bounding box of the tile's particles in the
// previous step, widened by one cell below and two above for the gather and
// deposit stencils, capped at the allocated window).  All values are
// wavefront-uniform.  q -> (rz, rx, ry) of a window cell uses the per-tile
// multipliers m0, m1: floor(q / d) = (q * ceil(2^16 / d)) >> 16 exactly for
// q < 2^16 / (d - 1), which holds for every window here (at most 2197 cells
// in 3D, 814 in 2D, divisors at most 37).
template <int DIM>
struct TileGeo {
  int r, tile;
  unsigned p0, p1;
  int lo[3], w0[3], Wd[3];
  unsigned m0, m1;
  int nwin;
};

__device__ __forceinline__ unsigned magic16(int d) { return (65536u + (unsigned)d - 1u) / (unsigned)d; }

// window cell q -> (rz, rx, ry)
template <int DIM>
__device__ __forceinline__ void win_decode(const TileGeo<DIM>& g, int q, int& rz, int& rx, int& ry) {
  const int t = (int)(((unsigned)q * g.m0) >> 16);
  rz = q - t * g.Wd[0];
  ry = (int)(((unsigned)t * g.m1) >> 16);
  rx = t - ry * g.Wd[1];
}

// Tiles of the particle kernel dealt to the XCDs (workgroup b runs on XCD
// b % 8) in blocks of 64 consecutive tiles, round-robin: block q goes to XCD
// q % 8.  At 8 cells per tile a block is a row of tiles along z of a 512-cell
// box, so each XCD's share covers the whole transverse plane and the busier
// tiles near the laser axis (more crossings and bank conflicts once the wake
// forms) are spread over all XCDs instead of the two that hold the central
// slabs of a contiguous split; the XCDs working at the same time on
// neighbouring rows still share their halo reads in the last-level cache.
// Batches of fewer than 2048 tiles use smaller blocks (down to one tile),
// at least 32 of them, so that every XCD gets several.  The workgroups of an XCD step through its
// sequence of tiles together: workgroup j takes positions j, j + G/8, ...
struct XcdDeal {
  long long beg, end, stride, x;
  int sh;
  __device__ explicit XcdDeal(long long total) {
    x = blockIdx.x & 7;
    sh = 0;
    while (sh < 6 && (total >> (sh + 1)) >= 32) ++sh;
    const long long nb = (total + (1LL << sh) - 1) >> sh;
    const long long cx = nb > x ? (nb - 1 - x) / 8 + 1 : 0;  // blocks x, x + 8, ...
    long long len = cx << sh;
    if (cx > 0 && x + 8 * (cx - 1) == nb - 1) len -= (nb << sh) - total;  // the last block is short
    beg = blockIdx.x >> 3;
    end = len;
    stride = (long long)(gridDim.x >> 3);
  }
  // the tile at position k of this XCD's sequence
  __device__ long long tile(long long k) const { return ((x + 8 * (k >> sh)) << sh) + (k & ((1LL << sh) - 1)); }
};

template <int DIM, typename R>
__device__ __forceinline__ void tile_geo(const BatchTable* __restrict__ bt, long long w, TileGeo<DIM>& g) {
  using T = Tile<DIM, R>;
  g.r = __builtin_amdgcn_readfirstlane(locate(bt->pre_tiles, bt->n, w));
  RunC& rd = *bt->run[g.r];
  g.tile = (int)(w - bt->pre_tiles[g.r]);
  const int tz = g.tile % rd.ntz, rest = g.tile / rd.ntz;
  const int tx = rest % rd.ntx, ty = rest / rd.ntx;
  const int t0[3] = {tz * T::TZ, tx * T::TX, ty * T::TY};
  const PIC_C int* ts = ro(rd.tile_start);
  g.p0 = (unsigned)ts[g.tile];
  g.p1 = (unsigned)ts[g.tile + 1];
  const PIC_C Counters& ctr = *ro(rd.ctr);
  // right after a sort: the tile's cells, and GZ cells above in z, where the
  // upper members of a group sorted by its lowest cell may sit
  int hi[3] = {T::TZ - 1 + T::GZ, T::TX - 1, T::TY - 1};
  g.lo[0] = g.lo[1] = g.lo[2] = 0;
  if (!ctr.fresh) {
    const PIC_C int* bbr = ro(rd.bbox[ctr.bbuf]) + 6 * g.tile;
    if (bbr[0] <= bbr[3]) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        g.lo[d] = bbr[d];
        hi[d] = bbr[3 + d];
      }
    }
  }
  g.Wd[0] = min(hi[0] - g.lo[0] + 4, T::WZ);
  g.Wd[1] = min(hi[1] - g.lo[1] + 4, T::WX);
  g.Wd[2] = DIM == 3 ? min(hi[2] - g.lo[2] + 4, T::WY) : 1;
#pragma unroll
  for (int d = 0; d < 3; ++d) g.w0[d] = t0[d] + g.lo[d] - 1;
  if (DIM == 2) g.w0[2] = 0;
  g.m0 = magic16(g.Wd[0]);
  g.m1 = magic16(g.Wd[1]);
  g.nwin = g.Wd[0] * g.Wd[1] * g.Wd[2];
  // every value is uniform: keep them in scalar registers
  auto u = [](int v) { return __builtin_amdgcn_readfirstlane(v); };
  g.tile = u(g.tile);
  g.p0 = (unsigned)u((int)g.p0);
  g.p1 = (unsigned)u((int)g.p1);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    g.lo[d] = u(g.lo[d]);
    g.w0[d] = u(g.w0[d]);
    g.Wd[d] = u(g.Wd[d]);
  }
  g.m0 = (unsigned)u((int)g.m0);
  g.m1 = (unsigned)u((int)g.m1);
  g.nwin = u(g.nwin);
}

// Issue the global loads of a tile's window of E^n and B^{n-1/2} (NU cells
// per thread); nothing waits for them here.  zf: bit 0 = the z index is a
// valid node, bit 1 = a valid half point (open z), sidx = LDS index or -1.
template <int DIM, typename R, int BLOCK, int NU>
__device__ __forceinline__ void window_load(const BatchTable* __restrict__ bt, const TileGeo<DIM>& g,
                                            R (&ld)[NU][6], int (&sidx)[NU], unsigned (&zf)[NU]) {
  using T = Tile<DIM, R>;
  RunC& rd = *bt->run[g.r];
  const int fb = ro(rd.ctr)->fbuf;
  const Arr3<R> Eg = PIC_ARR3(R, rd.E[fb]);
  const Arr3<R> Bg = PIC_ARR3(R, rd.B[fb]);
  const int nx = rd.nx, ny = rd.ny, nz = rd.nz, nzf = rd.nzf;
  const bool open = rd.open != 0;
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int q = threadIdx.x + u * BLOCK;
    sidx[u] = -1;
    zf[u] = 0;
    if (q < g.nwin) {
      int rz, rx, ry;
      win_decode(g, q, rz, rx, ry);
      sidx[u] = ry * (DIM == 3 ? T::SY : 0) + rx * T::WZ + rz;
      const int gk = g.w0[0] + rz;
      const int gi = wrap2(g.w0[1] + rx, nx);
      const int gj = DIM == 3 ? wrap2(g.w0[2] + ry, ny) : 0;
      int kk;
      if (open) {
        zf[u] = (gk >= 0 && gk <= nz ? 1u : 0u) | (gk >= 0 && gk < nz ? 2u : 0u);
        kk = min(max(gk, 0), nzf - 1);
      } else {
        zf[u] = 3u;
        kk = wrap2(gk, nz);
      }
      const long long gq = ((long long)gj * nx + gi) * nzf + kk;
      ld[u][0] = Eg[0][gq];
      ld[u][1] = Eg[1][gq];
      ld[u][2] = Eg[2][gq];
      ld[u][3] = Bg[0][gq];
      ld[u][4] = Bg[1][gq];
      ld[u][5] = Bg[2][gq];
    }
  }
}

// Occupancy of the 3D particle kernel.  Its LDS window (122 KiB in split
// precision, 123 KiB in FP64) admits one workgroup per CU, so the workgroup
// is 1024 threads in split precision (16 resident waves per CU, registers
// capped at 128) and 512 in FP64 (8 waves; the FP64 state needs the
// registers).  The larger split-precision tile (8x8x8 cells, 8192 particles
// at 16 per cell) spreads the window load and the current flush over twice
// the particles of an 8x8x4 tile (11.0 against 11.9 ms per step at
// 512x256x256 when the change was made).
#ifndef PIC_PBLOCK3
#define PIC_PBLOCK3 1024
#endif
#ifndef PIC_WPE3
#define PIC_WPE3 4
#endif
#ifndef PIC_PBLOCK3D
#define PIC_PBLOCK3D 512
#endif
#ifndef PIC_WPE3D
#define PIC_WPE3D 2
#endif
template <int DIM, typename R>
struct PBlock {
  static constexpr int value = DIM == 3 ? (sizeof(R) == 4 ? PIC_PBLOCK3 : PIC_PBLOCK3D) : 256;
};
template <int DIM, typename R, int BLOCK>
struct PWaves {
  static constexpr int value = DIM == 3 ? (sizeof(R) == 4 ? PIC_WPE3 : PIC_WPE3D) : 1;
};

// Per tile: store the window (loaded during the previous tile's flush) in
// LDS, advance B to integer time there, run the tile's particles in chunks
// of one wavefront taken from a shared counter (so the wavefronts of a
// workgroup run out of work together), issue the next tile's window loads,
// reduce the bounding box of the new cells and flush the current window to
// HBM, zeroing it for the next tile.
template <int DIM, typename R, int BLOCK, int PUSHER>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(PWaves<DIM, R, BLOCK>::value)))
void k_particles(const BatchTable* __restrict__ bt) {
  using T = Tile<DIM, R>;
  constexpr int WZM = T::WZ, WXM = T::WX, WYM = T::WY;
  constexpr int SY = (DIM == 3) ? T::SY : 0;              // LDS stride of y
  constexpr int WV = (DIM == 3) ? SY * WYM : WZM * WXM;  // LDS stride of a component
  constexpr int NU = (WZM * WXM * WYM + BLOCK - 1) / BLOCK;  // window cells per thread
  static_assert(3 * WV * 8 <= 65536, "deposit offsets must fit the 16-bit LDS offset");
  // LDS: the current window first, so that every deposit address is one
  // per-particle base plus an immediate offset below 64 KiB
  struct Smem {
    long long J[3][WV];  // Jx Jy Jz, 64-bit fixed point
    R F[6][WV];          // Ex Ey Ez Bx By Bz of the tile window
    int bb[6];           // bounding box of the new cells (window coordinates)
    unsigned next;       // next unclaimed particle chunk of the tile
  };
  __shared__ Smem sm;
  auto& sJ = sm.J;
  auto& sF = sm.F;
  const int lane = threadIdx.x & 63;

  const XcdDeal xs(bt->tiles);
  TileGeo<DIM> g;
  R ld[NU][6];
  int sidx[NU];
  unsigned zf[NU];
  if (xs.beg < xs.end) {
    tile_geo<DIM, R>(bt, xs.tile(xs.beg), g);
    if (g.p0 < g.p1) window_load<DIM, R, BLOCK, NU>(bt, g, ld, sidx, zf);
  }
  for (int q = threadIdx.x; q < 3 * WV; q += BLOCK) (&sJ[0][0])[q] = 0;

  for (long long w = xs.beg; w < xs.end; w += xs.stride) {
    RunC& rd = *bt->run[g.r];
    const PIC_C Counters& ctr = *ro(rd.ctr);
    const int pb = ctr.pbuf, fb = ctr.fbuf, bb = ctr.bbuf;
    const int nx = rd.nx, ny = rd.ny, nz = rd.nz, nzf = rd.nzf;
    const bool open = rd.open != 0;
    PIC_G int* bbw = rd.bbox[bb ^ 1] + 6 * g.tile;
    const long long wn = w + xs.stride;
    __syncthreads();  // the previous tile's particles and flush are done with the LDS
    if (g.p0 >= g.p1) {
      if (threadIdx.x == 0) {
        bbw[0] = bbw[1] = bbw[2] = 1 << 20;
        bbw[3] = bbw[4] = bbw[5] = -(1 << 20);
      }
      if (wn < xs.end) {
        tile_geo<DIM, R>(bt, xs.tile(wn), g);
        if (g.p0 < g.p1) window_load<DIM, R, BLOCK, NU>(bt, g, ld, sidx, zf);
      }
      continue;
    }
    const int w00 = g.w0[0], w01 = g.w0[1], w02 = g.w0[2];
    const int Wd0 = g.Wd[0], Wd1 = g.Wd[1], Wd2 = g.Wd[2];
    // ---- store the window of E^n and B^{n-1/2} (zero outside an open z range)
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int s = sidx[u];
      if (s >= 0) {
        const bool zn = (zf[u] & 1u) != 0, zh = (zf[u] & 2u) != 0;
        sF[0][s] = zn ? ld[u][0] : R(0);
        sF[1][s] = zn ? ld[u][1] : R(0);
        sF[2][s] = zh ? ld[u][2] : R(0);
        sF[3][s] = zh ? ld[u][3] : R(0);
        sF[4][s] = zh ? ld[u][4] : R(0);
        sF[5][s] = zn ? ld[u][5] : R(0);
      }
    }
    if (threadIdx.x == 0) sm.next = 0;
    {
      // recomputed here (not hoisted out of the tile loop into a spill slot,
      // whose reload would wait on the next window's loads in flight)
      int t6 = (int)threadIdx.x, big = 1 << 20;
      asm volatile("" : "+v"(t6), "+v"(big));
      if (t6 < 6) sm.bb[t6] = t6 < 3 ? big : -big;
    }
    __syncthreads();
    // ---- B^n = B^{n-1/2} - dt/2 curl E^n on the window (last layer unused)
    {
      const R hdt = R(0.5 * rd.dt);
      const R idz = R(1.0 / rd.dz), idx = R(1.0 / rd.dx), idy = DIM == 3 ? R(1.0 / rd.dy) : R(0);
      const int bz_ = Wd0 - 1, bx_ = Wd1 - 1, by_ = DIM == 3 ? Wd2 - 1 : 1;
      const unsigned mb0 = magic16(bz_), mb1 = magic16(bx_);
      const int nb = bz_ * bx_ * by_;
      for (int q = threadIdx.x; q < nb; q += BLOCK) {
        const int t = (int)(((unsigned)q * mb0) >> 16);
        const int rz = q - t * bz_;
        const int ry = (int)(((unsigned)t * mb1) >> 16);
        const int rx = t - ry * bx_;
        const int s = ry * SY + rx * WZM + rz;
        const int gk = w00 + rz;
        const bool zn = !open || (gk >= 0 && gk <= nz);
        const bool zh = !open || (gk >= 0 && gk < nz);
        const R ex = sF[0][s], ey = sF[1][s], ez = sF[2][s];
        const R ex_z = sF[0][s + 1], ey_z = sF[1][s + 1];
        const R ez_x = sF[2][s + WZM], ey_x = sF[1][s + WZM];
        const R ez_y = sF[2][s + SY], ex_y = sF[0][s + SY];
        if (zh) {
          sF[3][s] -= hdt * ((ez_y - ez) * idy - (ey_z - ey) * idz);
          sF[4][s] -= hdt * ((ex_z - ex) * idz - (ez_x - ez) * idx);
        }
        if (zn) sF[5][s] -= hdt * ((ey_x - ey) * idx - (ex_y - ex) * idy);
      }
    }
    __syncthreads();

    // ---- particles whose stencil lies in the window; the others are queued
    // for the HBM kernel
    // The seven particle arrays are addressed from bases advanced to the
    // tile's first slot (scalar registers) plus one 32-bit byte offset per
    // particle, shared by all of them.  A tile holds far fewer than 2^28
    // particles; one that does not is flagged and left alone.
    const unsigned p0 = g.p0, nt = g.p1 - g.p0;
    bool tile_ok = nt < (1u << 28);
    if (!tile_ok && threadIdx.x == 0) g_or(&rd.ctr->err, (unsigned)PIC_ERR_TILE);
    PIC_G int* __restrict__ cellp = rd.cell[pb] + p0;
    PIC_G R* __restrict__ o0p = fptr<R>(rd.off[pb][0]) + p0;
    PIC_G R* __restrict__ o1p = fptr<R>(rd.off[pb][1]) + p0;
    PIC_G R* __restrict__ o2p = fptr<R>(rd.off[pb][2]) + p0;
    PIC_G R* __restrict__ uxp = fptr<R>(rd.u[pb][0]) + p0;
    PIC_G R* __restrict__ uyp = fptr<R>(rd.u[pb][1]) + p0;
    PIC_G R* __restrict__ uzp = fptr<R>(rd.u[pb][2]) + p0;
    const PConst<R> K = pconst<DIM, R>(rd);
    // Window coordinates of a particle are its cell minus the window origin;
    // a periodic correction is needed only where the window crosses the
    // periodic boundary (uniform per tile).  Open z never wraps.
    const int wrapz = (!open && (w00 < 0 || w00 + Wd0 > nz)) ? nz : 0;
    const int wrapx = (w01 < 0 || w01 + Wd1 > nx) ? nx : 0;
    const int wrapy = (DIM == 3 && (w02 < 0 || w02 + Wd2 > ny)) ? ny : 0;
    // a particle can cross a periodic boundary only in a tile whose window
    // (its cells -1 .. +2) crosses it
    const bool wrapany = (wrapz | wrapx | wrapy) != 0;
    // bounding box of the new cells, in window coordinates
    int bmin0 = 1 << 20, bmin1 = 1 << 20, bmin2 = 1 << 20;
    int bmax0 = -(1 << 20), bmax1 = -(1 << 20), bmax2 = -(1 << 20);
    bool bad = false;

    // Chunks of 64 consecutive slots are taken from the tile's counter, one
    // per wavefront and iteration; the state of the next chunk is loaded
    // while the current one is advanced (software pipeline).  Only one chunk
    // is held ahead, so the wavefronts run out of work within one iteration
    // of each other.
    auto grab = [&]() -> unsigned {
      unsigned v = 0;
      if (lane == 0) v = atomicAdd(&sm.next, 64u);
      return __builtin_amdgcn_readfirstlane(v);
    };
    unsigned cA = tile_ok ? grab() : nt;
    int sA = -1;
    R oA0 = R(0), oA1 = R(0), oA2 = R(0), uA0 = R(0), uA1 = R(0), uA2 = R(0);
    if (cA + lane < nt) {
      const unsigned u = cA + lane, bi = u * 4u, br = u * (unsigned)sizeof(R);
      sA = at32(cellp, bi);
      oA0 = at32(o0p, br);
      oA1 = at32(o1p, br);
      if (DIM == 3) oA2 = at32(o2p, br);
      uA0 = at32(uxp, br);
      uA1 = at32(uyp, br);
      uA2 = at32(uzp, br);
    }
    while (cA < nt) {
      const unsigned u = cA + lane;  // slot relative to the tile's first
      const int c = sA;
      R o[3] = {oA0, oA1, oA2};
      R ux = uA0, uy = uA1, uz = uA2;
      cA = grab();
      sA = -1;
      if (cA + lane < nt) {
        const unsigned un = cA + lane, bi = un * 4u, br = un * (unsigned)sizeof(R);
        sA = at32(cellp, bi);
        oA0 = at32(o0p, br);
        oA1 = at32(o1p, br);
        if (DIM == 3) oA2 = at32(o2p, br);
        uA0 = at32(uxp, br);
        uA1 = at32(uyp, br);
        uA2 = at32(uzp, br);
      }
      if (u >= nt || c < 0) continue;  // past the tile's last slot, or removed
      const int k = cell_k(c), i = cell_i(c), j = DIM == 3 ? cell_j(c) : 0;
      int wk = k - w00, wi = i - w01, wj = DIM == 3 ? j - w02 : 0;
      if (wrapany) {
        wk = wrapu(wk, wrapz);
        wi = wrapu(wi, wrapx);
        if (DIM == 3) wj = wrapu(wj, wrapy);
      }
      // the stencil (old cell -1 .. +2) lies in the window: 1 <= w <= Wd - 3
      const bool fast = (unsigned)(wk - 1) <= (unsigned)(Wd0 - 4) &&
                        (unsigned)(wi - 1) <= (unsigned)(Wd1 - 4) &&
                        (DIM == 2 || (unsigned)(wj - 1) <= (unsigned)(Wd2 - 4));
      if (!fast) {
        const unsigned e = g_add(&rd.ctr->n_slowq, 1u);
        if (e < (unsigned long long)rd.capacity) rd.slowq[e] = (int)(p0 + u);
        continue;
      }
      const int base = wj * SY + wi * WZM + wk;
      int cr[3];
      bad |= advance<DIM, R, PUSHER>(
          K, o, ux, uy, uz, cr,
          [&](int comp, int dk, int di, int dj) -> R { return sF[comp][base + dk + di * WZM + dj * SY]; },
          [&](int zb, int xb, int yb) {
            unsigned long long* jw = reinterpret_cast<unsigned long long*>(&sJ[0][base + zb + xb * WZM + yb * SY]);
            return [jw](int comp, int a, int b, int c, long long q) {
              atomicAdd(jw + comp * WV + a + b * WZM + c * SY, (unsigned long long)q);
            };
          });
      bool dead;
      int k1, i1, j1;
      const unsigned bi = u * 4u, br = u * (unsigned)sizeof(R);
      at32(cellp, bi) = new_cell<DIM>(rd, c, k, i, j, cr, wrapany, dead, k1, i1, j1);
      at32(o0p, br) = o[0];
      at32(o1p, br) = o[1];
      if (DIM == 3) at32(o2p, br) = o[2];
      at32(uxp, br) = ux;
      at32(uyp, br) = uy;
      at32(uzp, br) = uz;
      if (!dead) {
        const int nk = wk + cr[0];
        const int ni = wi + cr[1];
        bmin0 = min(bmin0, nk);
        bmax0 = max(bmax0, nk);
        bmin1 = min(bmin1, ni);
        bmax1 = max(bmax1, ni);
        if (DIM == 3) {
          const int nj = wj + cr[2];
          bmin2 = min(bmin2, nj);
          bmax2 = max(bmax2, nj);
        }
      }
    }
    // ---- the next tile's window loads, issued as soon as this wavefront has
    // no particles left: in flight during the tail, the reduction and the flush
    TileGeo<DIM> gn;
    gn.p0 = gn.p1 = 0;
    if (wn < xs.end) {
      tile_geo<DIM, R>(bt, xs.tile(wn), gn);
      if (gn.p0 < gn.p1) window_load<DIM, R, BLOCK, NU>(bt, gn, ld, sidx, zf);
    }
    if (bad) g_or(&rd.ctr->err, 1u);
    // ---- bounding box of the new positions
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
      bmin0 = min(bmin0, __shfl_xor(bmin0, m));
      bmin1 = min(bmin1, __shfl_xor(bmin1, m));
      bmin2 = min(bmin2, __shfl_xor(bmin2, m));
      bmax0 = max(bmax0, __shfl_xor(bmax0, m));
      bmax1 = max(bmax1, __shfl_xor(bmax1, m));
      bmax2 = max(bmax2, __shfl_xor(bmax2, m));
    }
    if (lane == 0) {
      atomicMin(&sm.bb[0], bmin0);
      atomicMin(&sm.bb[1], bmin1);
      atomicMin(&sm.bb[2], bmin2);
      atomicMax(&sm.bb[3], bmax0);
      atomicMax(&sm.bb[4], bmax1);
      atomicMax(&sm.bb[5], bmax2);
    }
    __syncthreads();
    int t6 = (int)threadIdx.x, big = 1 << 20;
    asm volatile("" : "+v"(t6), "+v"(big));
    if (t6 < 6) {
      const int t = t6;
      int v = sm.bb[t];
      // window -> tile-relative coordinates (window origin = tile origin + lo - 1)
      const int d = t < 3 ? t : t - 3;
      const int lod = d == 0 ? g.lo[0] : (d == 1 ? g.lo[1] : g.lo[2]);  // no dynamic index
      if (v != (t < 3 ? big : -big)) v += lod - 1;
      if (DIM == 2 && (t == 2 || t == 5)) v = 0;
      bbw[t] = v;
    }
    // ---- flush the current window to HBM and zero it for the next tile
    const Arr3<unsigned long long> Jg = PIC_ARR3(unsigned long long, rd.J[fb]);
    for (int q = threadIdx.x; q < g.nwin; q += BLOCK) {
      int rz, rx, ry;
      win_decode(g, q, rz, rx, ry);
      const int s = ry * SY + rx * WZM + rz;
      const long long jx = sJ[0][s], jy = sJ[1][s], jz = sJ[2][s];
      if ((jx | jy | jz) == 0) continue;
      sJ[0][s] = 0;
      sJ[1][s] = 0;
      sJ[2][s] = 0;
      int gk = w00 + rz;
      const int gi = wrap2(w01 + rx, nx);
      const int gj = DIM == 3 ? wrap2(w02 + ry, ny) : 0;
      bool zn = true, zh = true;
      if (open) {
        zn = gk >= 0 && gk <= nz;
        zh = gk >= 0 && gk < nz;
      } else {
        gk = wrap2(gk, nz);
      }
      const long long gq = ((long long)gj * nx + gi) * nzf + gk;
      if (zn && jx != 0) g_add(Jg[0] + gq, (unsigned long long)jx);
      if (zn && jy != 0) g_add(Jg[1] + gq, (unsigned long long)jy);
      if (zh && jz != 0) g_add(Jg[2] + gq, (unsigned long long)jz);
    }
    g = gn;
  }
}

// Particles whose stencil left their tile's window: gather from and deposit
// into HBM directly, then widen the tile's bounding box.  Normally a tiny
// queue (empty in the steady boosted-frame flow).  Every workgroup first
// reads all the runs' queue lengths in parallel (one thread per run) and
// scans them in LDS; the queued particles of all runs are then one flat range
// shared by the whole grid, so an empty launch costs one round of loads and a
// heavy run's queue is spread over every workgroup.
template <int DIM, typename R, int PUSHER>
__global__ __launch_bounds__(256) void k_particles_hbm(const BatchTable* __restrict__ bt) {
  using T = Tile<DIM, R>;
  __shared__ long long pre[MAX_BATCH + 1];
  const int nr = bt->n;
  for (int r = threadIdx.x; r < nr; r += blockDim.x) {
    RunC& rd = *bt->run[r];
    pre[r + 1] = min((long long)rd.ctr->n_slowq, rd.capacity);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    long long acc = 0;
    pre[0] = 0;
    for (int r = 0; r < nr; ++r) {
      acc += pre[r + 1];
      pre[r + 1] = acc;
    }
  }
  __syncthreads();
  const long long total = pre[nr];
  for (long long w = (long long)blockIdx.x * blockDim.x + threadIdx.x; w < total;
       w += (long long)gridDim.x * blockDim.x) {
    // the run of item w: the last r with pre[r] <= w
    int lo = 0, hi = nr - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (pre[mid] <= w) lo = mid; else hi = mid - 1;
    }
    const int r = lo;
    const long long e = w - pre[r];
    RunC& rd = *bt->run[r];
    const PIC_G Counters& ctr = *rd.ctr;
    const int pb = ctr.pbuf, fb = ctr.fbuf, bb = ctr.bbuf;
    const Arr3<R> Eg = PIC_ARR3(R, rd.E[fb]);
    const Arr3<R> Bg = PIC_ARR3(R, rd.B[fb]);
    const PConst<R> K = pconst<DIM, R>(rd);
    {
      const int p = rd.slowq[e];
      const int c = rd.cell[pb][p];
      const int k = cell_k(c), i = cell_i(c), j = DIM == 3 ? cell_j(c) : 0;
      R o[3];
      o[0] = fptr<R>(rd.off[pb][0])[p];
      o[1] = fptr<R>(rd.off[pb][1])[p];
      o[2] = DIM == 3 ? fptr<R>(rd.off[pb][2])[p] : R(0);
      R ux = fptr<R>(rd.u[pb][0])[p], uy = fptr<R>(rd.u[pb][1])[p], uz = fptr<R>(rd.u[pb][2])[p];
      int cr[3];
      const bool bad = advance<DIM, R, PUSHER>(
          K, o, ux, uy, uz, cr,
          [&](int comp, int dk, int di, int dj) -> R {
            return fetch_hbm<DIM, R>(rd, Eg, Bg, comp, k + dk, i + di, j + dj);
          },
          [&](int zb, int xb, int yb) {
            const int kw = k + zb, iw = i + xb, jw = j + yb;
            return [&rd, fb, kw, iw, jw](int comp, int a, int b, int c, long long q) {
              add_hbm<DIM>(rd, fb, comp, kw + a, iw + b, jw + c, q);
            };
          });
      if (bad) g_or(&rd.ctr->err, 1u);
      bool dead;
      int k1, i1, j1;
      rd.cell[pb][p] = new_cell<DIM>(rd, c, k, i, j, cr, true, dead, k1, i1, j1);
      fptr<R>(rd.off[pb][0])[p] = o[0];
      fptr<R>(rd.off[pb][1])[p] = o[1];
      if (DIM == 3) fptr<R>(rd.off[pb][2])[p] = o[2];
      fptr<R>(rd.u[pb][0])[p] = ux;
      fptr<R>(rd.u[pb][1])[p] = uy;
      fptr<R>(rd.u[pb][2])[p] = uz;
      if (!dead) {
        // the tile of slot p: last tile whose start is <= p
        int lo = 0, hi = rd.ntiles - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (rd.tile_start[mid] <= p) lo = mid; else hi = mid - 1;
        }
        const int tile = lo;
        const int tz = tile % rd.ntz, rest = tile / rd.ntz;
        const int tx = rest % rd.ntx, ty = rest / rd.ntx;
        PIC_G int* bbw = rd.bbox[bb ^ 1] + 6 * tile;
        const int nk = rd.open ? k1 - tz * T::TZ : relw(k1, tz * T::TZ, rd.nz, rd.gz);
        const int ni = relw(i1, tx * T::TX, rd.nx, rd.gx);
        g_min(bbw + 0, nk);
        g_max(bbw + 3, nk);
        g_min(bbw + 1, ni);
        g_max(bbw + 4, ni);
        if (DIM == 3) {
          const int nj = relw(j1, ty * T::TY, rd.ny, rd.gy);
          g_min(bbw + 2, nj);
          g_max(bbw + 5, nj);
        }
      }
    }
  }
}

// ------------------------------------------------------------------ fields
// Three passes, one thread per grid point each, so that every thread issues
// only a handful of coalesced loads:
//   k_bhalf: B^{n+1/2} = B^{n-1/2} - dt curl E^n           (B[fb] -> B[fb^1])
//   k_efull: E^{n+1} = E^n + dt (curl B^{n+1/2} - J - J_ion) (E[fb] -> E[fb^1]),
//            and clears the current buffer of the next step (J[fb^1])
//   k_mur:   first-order Mur on the tangential E at the open z ends, from
//            E^n (still in E[fb]) and the interior E^{n+1}.
// A grid point q = (j nx + i) nzf + k of one field work item and the flat
// indices of its six neighbours.  The work item's first point is decoded
// once (uniform), each thread then steps from it, so no thread divides;
// indices are 32-bit (a run holds fewer than 2^31 points).  Neighbour values
// outside the open z range of their component read as zero.
template <int DIM>
struct FieldPt {
  unsigned q, qzp, qzm, qxp, qxm, qyp, qym;
  int k;
  bool zp_n, zp_h, zm_ok, c_h;  // k+1 valid for node / half components, k-1 valid, k valid for half

  __device__ __forceinline__ bool init(RunC& rd, long long item) {
    const unsigned nzf = (unsigned)rd.nzf, nx = (unsigned)rd.nx, ny = (unsigned)rd.ny, nz = (unsigned)rd.nz;
    const unsigned q0 = (unsigned)item * CELL_BLOCK;
    const unsigned t0 = q0 / nzf;
    unsigned kk = q0 - t0 * nzf + threadIdx.x, t = t0;
    while (kk >= nzf) {
      kk -= nzf;
      ++t;
    }
    const unsigned j0 = t0 / nx;
    unsigned i = t0 - j0 * nx + (t - t0), j = j0;
    while (i >= nx) {
      i -= nx;
      ++j;
    }
    q = q0 + threadIdx.x;
    if (q >= (unsigned)rd.npts) return false;
    k = (int)kk;
    const unsigned sx = nzf, sy = nx * nzf;
    qxp = i + 1 == nx ? q - (nx - 1) * sx : q + sx;
    qxm = i == 0 ? q + (nx - 1) * sx : q - sx;
    if (DIM == 3) {
      qyp = j + 1 == ny ? q - (ny - 1) * sy : q + sy;
      qym = j == 0 ? q + (ny - 1) * sy : q - sy;
    } else {
      qyp = qym = q;
    }
    if (rd.open) {
      qzp = q + 1;
      qzm = q - 1;
      zp_n = kk + 1 <= nz;  // nodes 0..nz
      zp_h = kk + 1 < nz;   // half points 0..nz-1
      zm_ok = kk >= 1;      // k-1 >= 0 (then k-1 < nz is valid for both)
      c_h = kk < nz;
    } else {
      qzp = kk + 1 == nz ? q + 1 - nz : q + 1;
      qzm = kk == 0 ? q + nz - 1 : q - 1;
      zp_n = zp_h = zm_ok = c_h = true;
    }
    return true;
  }
};

template <int DIM, typename R>
__global__ __launch_bounds__(256) void k_bhalf(const BatchTable* __restrict__ bt) {
  const XcdSplit xs(bt->cellblk);
  for (long long w = xs.beg; w < xs.end; w += xs.stride) {
    const int r = __builtin_amdgcn_readfirstlane(locate(bt->pre_cellblk, bt->n, w));
    RunC& rd = *bt->run[r];
    FieldPt<DIM> P;
    if (!P.init(rd, w - bt->pre_cellblk[r])) continue;
    const int fb = rd.ctr->fbuf;
    const Arr3<R> E = PIC_ARR3(R, rd.E[fb]);
    const Arr3<R> Bm = PIC_ARR3(R, rd.B[fb]);
    const Arr3<R> Bh = PIC_ARR3(R, rd.B[fb ^ 1]);
    const R dt = R(rd.dt);
    const R idz = R(1.0 / rd.dz), idx = R(1.0 / rd.dx), idy = DIM == 3 ? R(1.0 / rd.dy) : R(0);
    const unsigned q = P.q;
    // Ex, Ey on nodes in z, Ez on half points
    const R ex = E[0][q], ey = E[1][q], ez = P.c_h ? E[2][q] : R(0);
    const R ey_z = P.zp_n ? E[1][P.qzp] : R(0), ex_z = P.zp_n ? E[0][P.qzp] : R(0);
    const R ez_x = P.c_h ? E[2][P.qxp] : R(0), ey_x = E[1][P.qxp];
    R ez_y = R(0), ex_y = R(0);
    if (DIM == 3) {
      ez_y = P.c_h ? E[2][P.qyp] : R(0);
      ex_y = E[0][P.qyp];
    }
    const R cx = (ez_y - ez) * idy - (ey_z - ey) * idz;
    const R cy = (ex_z - ex) * idz - (ez_x - ez) * idx;
    const R cz = (ey_x - ey) * idx - (ex_y - ex) * idy;
    // Bx, By on half points in z, Bz on nodes
    Bh[0][q] = P.c_h ? Bm[0][q] - dt * cx : R(0);
    Bh[1][q] = P.c_h ? Bm[1][q] - dt * cy : R(0);
    Bh[2][q] = Bm[2][q] - dt * cz;
  }
}

template <int DIM, typename R>
__global__ __launch_bounds__(256) void k_efull(const BatchTable* __restrict__ bt) {
  const XcdSplit xs(bt->cellblk);
  for (long long w = xs.beg; w < xs.end; w += xs.stride) {
    const int r = __builtin_amdgcn_readfirstlane(locate(bt->pre_cellblk, bt->n, w));
    RunC& rd = *bt->run[r];
    FieldPt<DIM> P;
    if (!P.init(rd, w - bt->pre_cellblk[r])) continue;
    const int fb = rd.ctr->fbuf;
    const Arr3<R> E = PIC_ARR3(R, rd.E[fb]);
    const Arr3<R> En = PIC_ARR3(R, rd.E[fb ^ 1]);
    const Arr3<R> Bh = PIC_ARR3(R, rd.B[fb ^ 1]);
    const Arr3<long long> J = PIC_ARR3(long long, rd.J[fb]);
    const Arr3<long long> Jnext = PIC_ARR3(long long, rd.J[fb ^ 1]);
    const R dt = R(rd.dt);
    const R idz = R(1.0 / rd.dz), idx = R(1.0 / rd.dx), idy = DIM == 3 ? R(1.0 / rd.dy) : R(0);
    const double jinv = rd.jinv;
    const unsigned q = P.q;
    // Bx, By on half points in z (k-1 is a half point whenever k-1 >= 0)
    const R bx = P.c_h ? Bh[0][q] : R(0), by = P.c_h ? Bh[1][q] : R(0), bz = Bh[2][q];
    const R by_z = P.zm_ok ? Bh[1][P.qzm] : R(0), bx_z = P.zm_ok ? Bh[0][P.qzm] : R(0);
    const R bz_x = Bh[2][P.qxm], by_x = P.c_h ? Bh[1][P.qxm] : R(0);
    R bz_y = R(0), bx_y = R(0);
    if (DIM == 3) {
      bz_y = Bh[2][P.qym];
      bx_y = P.c_h ? Bh[0][P.qym] : R(0);
    }
    R jx, jy, jz;
    if (rd.filter_stages > 0) {  // filtered current, already in physical units
      const Arr3<R> F = PIC_ARR3(R, rd.jf[(DIM == 3 ? 2 : 1) & 1]);
      jx = F[0][q];
      jy = F[1][q];
      jz = F[2][q];
    } else {
      jx = R((double)J[0][q] * jinv);
      jy = R((double)J[1][q] * jinv);
      jz = R((double)J[2][q] * jinv);
    }
    En[0][q] = E[0][q] + dt * ((bz - bz_y) * idy - (by - by_z) * idz - jx);
    En[1][q] = E[1][q] + dt * ((bx - bx_z) * idz - (bz - bz_x) * idx - jy);
    En[2][q] = P.c_h ? E[2][q] + dt * ((by - by_x) * idx - (bx - bx_y) * idy - jz - R(rd.jion_z)) : R(0);
    Jnext[0][q] = 0;
    Jnext[1][q] = 0;
    Jnext[2][q] = 0;
  }
}


template <typename R>
__global__ __launch_bounds__(256) void k_mur(const BatchTable* __restrict__ bt) {
  // 2 nperp boundary columns per open run; each workgroup serves one run of
  // the batch (the grid holds at least eight workgroups per run)
  const int nr = bt->n;
  const int parts = (int)gridDim.x / nr;
  if ((int)blockIdx.x >= parts * nr) return;
  {
    const int r = (int)blockIdx.x % nr, part = (int)blockIdx.x / nr;
    RunC& rd = *bt->run[r];
    if (!rd.open) return;
    const unsigned nperp = (unsigned)rd.nperp, nzf = (unsigned)rd.nzf;
    const int fb = rd.ctr->fbuf;
    const Arr3<R> E = PIC_ARR3(R, rd.E[fb]);
    const Arr3<R> En = PIC_ARR3(R, rd.E[fb ^ 1]);
    const R cm = R((rd.dt - rd.dz) / (rd.dt + rd.dz));
    for (unsigned q = (unsigned)part * 256u + threadIdx.x; q < 2u * nperp; q += (unsigned)parts * 256u) {
      const unsigned side = q >= nperp ? 1u : 0u;
      const unsigned col = (q - side * nperp) * nzf;
      const unsigned kb = side ? (unsigned)rd.nz : 0u, ki = side ? (unsigned)rd.nz - 1u : 1u;
      for (int c = 0; c < 2; ++c)
        En[c][col + kb] = E[c][col + ki] + cm * (En[c][col + ki] - E[c][col + kb]);
    }
  }
}

__global__ void k_advance(const BatchTable* __restrict__ bt) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= bt->n) return;
  PIC_G Counters* c = bt->run[r]->ctr;
  // more than 1/1024 of the particles took the out-of-window path (each costs
  // tens of window pushes): re-sort at the next step that carries the sort
  // chain (in the serving stream, 1/1024 against 1/128 took the p99 latency
  // from 0.75 to 0.67 s)
  if ((long long)c->n_slowq * 1024 > c->n_slots) c->want_sort = 1;
  c->n_slow += c->n_slowq;
  c->n_slowq = 0;
  c->step += 1;
  c->fbuf ^= 1;
  c->bbuf ^= 1;
  c->fresh = 0;
}

// ------------------------------------------------------------------ launch

int grid_particles(int dims, int prec, int ncu) {
  const size_t per_cell = 6 * sizeof(float) * (prec ? 2 : 1) + 3 * sizeof(long long);
  size_t lds;
  if (dims == 3)
    lds = prec ? per_cell * Tile<3, double>::SY * Tile<3, double>::WY
               : per_cell * Tile<3, float>::SY * Tile<3, float>::WY;
  else
    lds = per_cell * Tile<2, float>::WZ * Tile<2, float>::WX;
  int per_cu = (int)((160 * 1024) / (lds + 1024));
  if (per_cu < 1) per_cu = 1;
  if (per_cu > 8) per_cu = 8;
  int g = ncu * per_cu;
  return (g + 7) & ~7;
}

// (at least one workgroup per run of a full batch: k_mur serves one run per
// workgroup)
int grid_generic(int ncu) { return ncu * 8 > MAX_BATCH ? ncu * 8 : MAX_BATCH; }

template <int DIM, typename R>
static void lp(int pusher, const BatchTable* bt, int grid, hipStream_t s) {
  constexpr int B = PBlock<DIM, R>::value;
  if (pusher == 1) {
    hipLaunchKernelGGL((k_particles<DIM, R, B, 1>), dim3(grid), dim3(B), 0, s, bt);
    hipLaunchKernelGGL((k_particles_hbm<DIM, R, 1>), dim3(1024), dim3(256), 0, s, bt);
  } else {
    hipLaunchKernelGGL((k_particles<DIM, R, B, 0>), dim3(grid), dim3(B), 0, s, bt);
    hipLaunchKernelGGL((k_particles_hbm<DIM, R, 0>), dim3(1024), dim3(256), 0, s, bt);
  }
}

void launch_particles(int dims, int prec, int pusher, const BatchTable* bt, int grid, hipStream_t s) {
  if (dims == 3) {
    if (prec) lp<3, double>(pusher, bt, grid, s); else lp<3, float>(pusher, bt, grid, s);
  } else {
    if (prec) lp<2, double>(pusher, bt, grid, s); else lp<2, float>(pusher, bt, grid, s);
  }
}

template <int DIM, typename R>
static void lf(const BatchTable* bt, int grid, int filter_stages, long long ant_plane, hipStream_t s) {
  constexpr int prec = sizeof(R) == 8 ? 1 : 0;
  if (filter_stages > 0) launch_filter(DIM, prec, bt, grid, filter_stages, s);
  hipLaunchKernelGGL((k_bhalf<DIM, R>), dim3(grid), dim3(256), 0, s, bt);
  if (ant_plane > 0) launch_antenna(prec, bt, ant_plane, 0, grid, s);
  hipLaunchKernelGGL((k_efull<DIM, R>), dim3(grid), dim3(256), 0, s, bt);
  if (ant_plane > 0) launch_antenna(prec, bt, ant_plane, 1, grid, s);
  hipLaunchKernelGGL((k_mur<R>), dim3(grid), dim3(256), 0, s, bt);
}

void launch_fields(int dims, int prec, const BatchTable* bt, int grid, int filter_stages, long long ant_plane,
                   hipStream_t s) {
  if (dims == 3) {
    if (prec) lf<3, double>(bt, grid, filter_stages, ant_plane, s);
    else lf<3, float>(bt, grid, filter_stages, ant_plane, s);
  } else {
    if (prec) lf<2, double>(bt, grid, filter_stages, ant_plane, s);
    else lf<2, float>(bt, grid, filter_stages, ant_plane, s);
  }
}

void launch_advance(const BatchTable* bt, int nruns, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3((nruns + 63) / 64), dim3(64), 0, s, bt);
}

}  // namespace pic
