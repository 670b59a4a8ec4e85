// Host side of libpic: parameter validation and the derived boosted-frame
// quantities, the layout of the caller's device buffer, step orchestration
// (HIP graphs of one step, replayed), batched stepping of several runs,
// diagnostics and read-back.  See include/pic.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <atomic>
#include <mutex>
#include <vector>

#include "launch.hpp"
#include "pic.h"
#include "pic_dev.hpp"

using namespace pic;

namespace {

thread_local std::string g_err;

pic_status fail(pic_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIPCHK(expr)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(PIC_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// SI constants (CODATA 2018) for the laboratory density -> plasma units
constexpr double C_LIGHT = 299792458.0, Q_E = 1.602176634e-19, EPS_0 = 8.8541878128e-12,
                 M_ELECTRON = 9.1093837015e-31;

struct Derived {
  double dt, beta_b, gamma_b, dminus, dplus, skin_um, k0_lab, E0_lab, L_lab, L_boost, zc_boost;
  double weight, dV;
  double jscale;  // fixed-point scale of the current (a power of two)
  int reservoir, nzf, ztop;
  int ntz, ntx, nty, ntiles;
  long long nperp, npts, capacity, max_new;
  size_t rsz;
  // laboratory-frame stations: transverse samples per record (nxs, nys) and
  // the points one station pass visits (n_stations nxs nys; 0 = none)
  int st_nxs, st_nys;
  long long st_items;
  long long ant_plane;  // transverse points of an active laser antenna (0: none)
};

// what a captured step depends on besides the run table: current-filter
// stages, station points and antenna planes (the most any run of the table needs)
struct StepShape {
  int fstages = 0;
  long long st_items = 0, ant_plane = 0;
  bool operator==(const StepShape& o) const {
    return fstages == o.fstages && st_items == o.st_items && ant_plane == o.ant_plane;
  }
  bool operator!=(const StepShape& o) const { return !(*this == o); }
};

struct Layout {
  size_t rundev, ctr, tab1, tabB;
  size_t E[2][3], B[2][3], J[2][3];
  size_t cell[2], off[2][3], u[2][3], pid[2];
  size_t tile_start, tile_count, tile_cursor, tile_full, bbox[2];
  size_t rho_a, rho_b, gauss0, jlast[3], cell_snap, slowq;
  size_t jf[2][3];  // filtered current (R), ping-pong; only with the filter
  size_t ftmp[2];   // node scalar ping-pong of the filtered Gauss diagnostic (double)
  size_t st_count, st_time, st_data;  // stations (st_count is in the cleared range)
  size_t zero_end;  // [0, zero_end) is cleared at init
  size_t total;
};

constexpr size_t NOPT = (size_t)-1;

pic_status derive(const pic_lab_params* p, Derived& d) {
  if (!p) return fail(PIC_EINVAL, "params is NULL");
  if (p->dims != 2 && p->dims != 3) return fail(PIC_EINVAL, "dims must be 2 or 3");
  const bool f64 = p->precision == PIC_FP64;
  const int TZ = p->dims == 3 ? (f64 ? Tile<3, double>::TZ : Tile<3, float>::TZ) : Tile<2, float>::TZ;
  const int TX = p->dims == 3 ? (f64 ? Tile<3, double>::TX : Tile<3, float>::TX) : Tile<2, float>::TX;
  const int TY = p->dims == 3 ? (f64 ? Tile<3, double>::TY : Tile<3, float>::TY) : 1;
  const int ny = p->dims == 3 ? p->ny : 1;
  if (p->nz < 8) return fail(PIC_EINVAL, "nz must be >= 8");
  if (p->nx < TX || p->nx % TX || p->nx > (1 << IBITS))
    return fail(PIC_EINVAL, "nx must be a multiple of %d in [%d, %d]", TX, TX, 1 << IBITS);
  if (p->dims == 3 && (ny < TY || ny % TY || ny > (1 << JBITS)))
    return fail(PIC_EINVAL, "ny must be a multiple of %d in [%d, %d]", TY, TY, 1 << JBITS);
  if (!(p->dz > 0) || !(p->dx > 0) || (p->dims == 3 && !(p->dy > 0)))
    return fail(PIC_EINVAL, "cell sizes must be positive");
  if (!(p->cfl > 0) || !(p->cfl < 1)) return fail(PIC_ECFL, "cfl must be in (0, 1)");
  if (p->ppc < 0 || p->ppc > 4096) return fail(PIC_EINVAL, "ppc must be in [0, 4096]");
  if (!(p->gamma_boost >= 1.0)) return fail(PIC_EINVAL, "gamma_boost must be >= 1");
  if (!(p->n_lab_cm3 > 0) || !(p->lambda0_um > 0) || !(p->waist > 0))
    return fail(PIC_EINVAL, "density, wavelength and waist must be positive");
  if (!(p->u_th >= 0) || !(p->a0 >= 0)) return fail(PIC_EINVAL, "u_th and a0 must be >= 0");
  if (p->pol_axis != 1 && p->pol_axis != 2) return fail(PIC_EINVAL, "pol_axis must be 1 or 2");
  if (p->bc_z != PIC_BC_OPEN && p->bc_z != PIC_BC_PERIODIC) return fail(PIC_EINVAL, "bad bc_z");
  if (p->pusher != PIC_VAY && p->pusher != PIC_BORIS) return fail(PIC_EINVAL, "bad pusher");
  if (p->precision != PIC_FP32_SPLIT && p->precision != PIC_FP64) return fail(PIC_EINVAL, "bad precision");
  if (p->sort_every < 1) return fail(PIC_EINVAL, "sort_every must be >= 1");
  if (p->filter_passes < 0 || p->filter_passes > 16) return fail(PIC_EINVAL, "filter_passes must be in 0..16");
  if (p->filter_compensate != 0 && p->filter_compensate != 1)
    return fail(PIC_EINVAL, "filter_compensate must be 0 or 1");
  if (p->n_stations < 0 || p->n_stations > 65536) return fail(PIC_EINVAL, "n_stations must be in 0..65536");
  if (p->n_stations > 0) {
    if (p->station_stride < 1 || p->station_stride > p->nx || (p->dims == 3 && p->station_stride > ny))
      return fail(PIC_EINVAL, "station_stride must be in [1, nx] (and <= ny in 3D)");
    if (p->station_cap < 1) return fail(PIC_EINVAL, "station_cap must be >= 1");
    if (!std::isfinite(p->station_z0) || !std::isfinite(p->station_dz))
      return fail(PIC_EINVAL, "station_z0 and station_dz must be finite");
  }
  if (p->laser_antenna != 0 && p->laser_antenna != 1) return fail(PIC_EINVAL, "laser_antenna must be 0 or 1");
  if (p->laser_antenna && (!std::isfinite(p->antenna_z_lab) || !std::isfinite(p->antenna_t_peak)))
    return fail(PIC_EINVAL, "antenna_z_lab and antenna_t_peak must be finite");

  double inv2 = 1.0 / (p->dz * p->dz) + 1.0 / (p->dx * p->dx);
  if (p->dims == 3) inv2 += 1.0 / (p->dy * p->dy);
  d.dt = p->cfl / std::sqrt(inv2);
  d.gamma_b = p->gamma_boost;
  d.beta_b = std::sqrt(1.0 - 1.0 / (p->gamma_boost * p->gamma_boost));
  d.dplus = d.gamma_b * (1.0 + d.beta_b);
  d.dminus = 1.0 / d.dplus;
  const double wp = std::sqrt(p->n_lab_cm3 * 1e6 * Q_E * Q_E / (EPS_0 * M_ELECTRON));
  d.skin_um = C_LIGHT / wp * 1e6;
  d.k0_lab = 2.0 * M_PI * d.skin_um / p->lambda0_um;
  d.E0_lab = p->a0 * d.k0_lab;
  const double Lz = p->nz * p->dz;
  d.L_boost = p->tau_lab > 0 ? d.dplus * p->tau_lab : Lz / 8.0;
  d.L_lab = d.L_boost / d.dplus;
  d.zc_boost = 0.5 * Lz;
  d.dV = p->dz * p->dx * (p->dims == 3 ? p->dy : 1.0);
  d.weight = d.gamma_b * d.dV / (p->ppc > 0 ? p->ppc : 1);
  const bool open = p->bc_z == PIC_BC_OPEN;
  const double drift = d.beta_b * p->sort_every * d.dt / p->dz;  // cells per sort interval
  d.reservoir = open ? (int)std::ceil(drift) + 2 : 0;
  d.nzf = open ? p->nz + 1 : p->nz;
  d.ztop = open ? p->nz + d.reservoir + 2 : p->nz;
  if (d.ztop + KOFF > KMASK) return fail(PIC_EINVAL, "nz plus reservoir too large (%d)", d.ztop);
  d.ntz = (d.ztop + TZ - 1) / TZ;
  d.ntx = p->nx / TX;
  d.nty = p->dims == 3 ? ny / TY : 1;
  d.ntiles = d.ntz * d.ntx * d.nty;
  d.nperp = (long long)p->nx * ny;
  d.npts = (long long)d.nzf * d.nperp;
  if (open) {
    const long long cols = p->nz + d.reservoir + 2 + ((long long)std::ceil(drift) + 1) + 4;
    d.capacity = (long long)std::ceil(cols * (double)d.nperp * p->ppc * 1.05) + 4096;
    d.max_new = (long long)(p->nz + d.reservoir) * d.nperp * p->ppc;
  } else {
    d.capacity = (long long)p->nz * d.nperp * p->ppc + 64;
    d.max_new = (long long)p->nz * d.nperp * p->ppc;
  }
  // every tile's slot range is padded to a multiple of 64 (one wavefront)
  d.capacity += 64LL * d.ntiles;
  if (d.capacity >= (1LL << 31) - 1) return fail(PIC_EINVAL, "too many particles for one run");
  {
    // One particle's current contribution is at most cmax = w / (dA dt) (plus
    // w / (dz dx) for the 2D out-of-plane current).  FP64 path: scale 2^40,
    // contributions below 2^50.  Split precision: each contribution is
    // rounded to a 32-bit integer, so the scale is the largest power of two
    // with cmax * scale <= 2^30, at most 2^32 and at least 2^8.
    const double dA = p->dims == 3 ? std::min(p->dx * p->dy, std::min(p->dz * p->dy, p->dz * p->dx))
                                   : std::min(p->dx, p->dz);
    const double cmax = d.weight / (dA * d.dt) + d.weight / (p->dz * p->dx);
    if (p->precision == PIC_FP64) {
      if (!(cmax < 1024.0)) return fail(PIC_EINVAL, "current per particle %.3g exceeds the fixed-point range", cmax);
      d.jscale = 1099511627776.0;
    } else {
      if (!(cmax <= 4194304.0)) return fail(PIC_EINVAL, "current per particle %.3g exceeds the fixed-point range", cmax);
      int e = (int)std::floor(std::log2(1073741824.0 / cmax));
      if (std::ldexp(cmax, e) > 1073741824.0) --e;
      d.jscale = std::ldexp(1.0, std::min(e, 32));
    }
  }
  d.rsz = p->precision == PIC_FP64 ? sizeof(double) : sizeof(float);
  d.st_nxs = d.st_nys = 0;
  d.st_items = 0;
  d.ant_plane = (p->laser_antenna && p->a0 > 0) ? d.nperp : 0;
  if (p->n_stations > 0) {
    d.st_nxs = p->nx / p->station_stride;
    d.st_nys = p->dims == 3 ? ny / p->station_stride : 1;
    d.st_items = (long long)p->n_stations * d.st_nxs * d.st_nys;
    // 6 doubles per point and sample: keep the record addressable
    const double rec = 48.0 * (double)d.st_items * (double)p->station_cap;
    if (rec > 64.0 * (1LL << 30)) return fail(PIC_EINVAL, "station record of %.3g bytes exceeds 64 GiB", rec);
  }
  return PIC_OK;
}

void layout(const pic_lab_params* p, const Derived& d, Layout& L) {
  size_t o = 0;
  auto take = [&](size_t bytes) {
    o = (o + 255) & ~(size_t)255;
    size_t r = o;
    o += bytes;
    return r;
  };
  L.rundev = take(sizeof(RunDev));
  L.ctr = take(sizeof(Counters));
  L.tab1 = take(sizeof(BatchTable));
  L.tabB = take(sizeof(BatchTable));
  const size_t fb = d.npts * d.rsz;
  for (int b = 0; b < 2; ++b)
    for (int c = 0; c < 3; ++c) L.E[b][c] = take(fb);
  for (int b = 0; b < 2; ++b)
    for (int c = 0; c < 3; ++c) L.B[b][c] = take(fb);
  for (int b = 0; b < 2; ++b)
    for (int c = 0; c < 3; ++c) L.J[b][c] = take(sizeof(long long) * d.npts);
  L.tile_start = take(sizeof(int) * (d.ntiles + 1));
  L.tile_count = take(sizeof(int) * d.ntiles);
  L.tile_cursor = take(sizeof(int) * d.ntiles);
  L.tile_full = take(sizeof(int) * d.ntiles);
  L.bbox[0] = take(sizeof(int) * 6 * d.ntiles);
  L.bbox[1] = take(sizeof(int) * 6 * d.ntiles);
  const bool stn = p->n_stations > 0;
  L.st_count = stn ? take(sizeof(long long) * p->n_stations) : NOPT;
  L.zero_end = (o + 255) & ~(size_t)255;
  L.st_time = stn ? take(sizeof(double) * p->n_stations * (size_t)p->station_cap) : NOPT;
  L.st_data = stn ? take(sizeof(double) * 6 * (size_t)d.st_items * (size_t)p->station_cap) : NOPT;
  L.rho_a = take(sizeof(double) * d.npts);
  L.gauss0 = take(sizeof(double) * d.npts);
  const bool cont = (p->diag_flags & PIC_DIAGF_CONTINUITY) != 0;
  L.rho_b = cont ? take(sizeof(double) * d.npts) : NOPT;
  for (int c = 0; c < 3; ++c) L.jlast[c] = cont ? take(sizeof(double) * d.npts) : NOPT;
  L.cell_snap = cont ? take(sizeof(int) * d.capacity) : NOPT;
  const bool filt = p->filter_passes > 0;
  for (int b = 0; b < 2; ++b)
    for (int c = 0; c < 3; ++c) L.jf[b][c] = filt ? take(d.rsz * d.npts) : NOPT;
  for (int b = 0; b < 2; ++b) L.ftmp[b] = filt ? take(sizeof(double) * d.npts) : NOPT;
  const size_t cap = (size_t)d.capacity;
  L.slowq = take(sizeof(int) * cap);
  for (int b = 0; b < 2; ++b) {
    L.cell[b] = take(sizeof(int) * cap);
    for (int c = 0; c < 3; ++c) L.off[b][c] = (c < p->dims) ? take(d.rsz * cap) : NOPT;
    for (int c = 0; c < 3; ++c) L.u[b][c] = take(d.rsz * cap);
    L.pid[b] = take(sizeof(unsigned) * cap);
  }
  L.total = (o + 255) & ~(size_t)255;
}

}  // namespace

struct pic_run {
  pic_lab_params p;
  Derived d;
  Layout L;
  char* base;
  size_t bytes;
  hipStream_t stream;
  RunDev hrd;
  RunDev* drd;
  Counters* dctr;
  BatchTable* dtab1;
  BatchTable* dtabB;
  BatchTable htab1;
  unsigned long long serial;        // unique per run of the process
  std::vector<unsigned long long> tabB_runs;  // serials of the batch dtabB holds
  Counters hctr0;  // initial device counters (host staging of the asynchronous init)
  int ncu, gpart, ggen;
  bool use_graph;
  hipGraphExec_t g1[2];  // one single-run step: [1] with the sort chain, [0] without
  hipGraphExec_t gB[2];  // one batched step (this run's batch table), likewise
  StepShape gB_shape[2];  // what the batched graphs were captured for
  // host mirror of the device step counter (checked at every read-back).
  // The sort chain is enqueued on every cadence step and every CHAIN_EVERY-th
  // step in between; the device decides whether it sorts (cadence, or a
  // request left by a step with too many out-of-window particles, which
  // stays pending until a step that carries the chain) and its kernels
  // return at once otherwise.
  long long hstep;
};

namespace {

template <typename T>
T* at(pic_run* r, size_t off) {
  return off == NOPT ? nullptr : reinterpret_cast<T*>(r->base + off);
}

void fill_table(BatchTable& t, pic_run* const* runs, int n) {
  memset(&t, 0, sizeof(t));
  t.n = n;
  long long a = 0, b = 0;
  for (int i = 0; i < n; ++i) {
    const Derived& d = runs[i]->d;
    t.run[i] = runs[i]->drd;
    t.pre_tiles[i] = a;
    t.pre_cellblk[i] = b;
    a += d.ntiles;
    b += (d.npts + CELL_BLOCK - 1) / CELL_BLOCK;
  }
  t.pre_tiles[n] = t.tiles = a;
  t.pre_cellblk[n] = t.cellblk = b;
}

void host_advance(pic_run* r) { ++r->hstep; }

// steps that carry the sort chain: the cadence, and every CHAIN_EVERY-th
// step for sorts the device requests in between (an idle chain costs five
// small launches, a sizeable share of the step of small batched runs)
constexpr int CHAIN_EVERY = 4;
bool chain_step(const pic_run* r) {
  return r->hstep % r->p.sort_every == 0 || r->hstep % CHAIN_EVERY == 0;
}

// what one run needs of a captured step
StepShape shape_of(const pic_run* r) {
  StepShape sh;
  sh.fstages = r->hrd.filter_stages;
  sh.st_items = r->d.st_items;
  sh.ant_plane = r->d.ant_plane;
  return sh;
}

// enqueue one step for the runs of a batch table
void enqueue_step(pic_run* r0, const BatchTable* tab, bool cont, bool chain, const StepShape& sh) {
  const int dims = r0->p.dims, prec = r0->p.precision;
  hipStream_t s = r0->stream;
  if (chain) launch_sort_chain(dims, prec, tab, MAX_BATCH, r0->ggen, s);
  if (cont) {
    launch_cont_pre(dims, prec, r0->drd, r0->d.npts, r0->d.capacity, s);
    launch_rho(dims, prec, r0->drd, at<double>(r0, r0->L.rho_a), r0->d.npts, r0->d.capacity, 1, s);
  }
  launch_particles(dims, prec, r0->p.pusher, tab, r0->gpart, s);
  if (cont) {
    launch_rho(dims, prec, r0->drd, at<double>(r0, r0->L.rho_b), r0->d.npts, r0->d.capacity, 1, s);
    launch_cont_post(dims, prec, r0->drd, r0->d.npts, r0->d.capacity, s);
  }
  launch_fields(dims, prec, tab, r0->ggen, sh.fstages, sh.ant_plane, s);
  // E[fbuf] = E^n and B[fbuf] = B^{n-1/2} are intact until the advance flips fbuf
  if (sh.st_items > 0) launch_stations(prec, tab, sh.st_items, r0->ggen, s);
  launch_advance(tab, MAX_BATCH, s);
}

pic_status capture(pic_run* r, const BatchTable* tab, bool cont, bool chain, const StepShape& sh,
                   hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(r->stream, hipStreamCaptureModeThreadLocal));
  enqueue_step(r, tab, cont, chain, sh);
  hipError_t e = hipStreamEndCapture(r->stream, &g);
  if (e != hipSuccess) return fail(PIC_EHIP, "graph capture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(PIC_EHIP, "graph instantiate: %s", hipGetErrorString(e));
  return PIC_OK;
}

// the electron density the Gauss diagnostic compares div E with: rho_a as
// computed, or, with the current filter, rho_a filtered the same way
// (enqueued on the run's stream)
const double* gauss_rho(pic_run* r) {
  const double* rho = at<double>(r, r->L.rho_a);
  if (r->hrd.filter_stages == 0) return rho;
  return launch_filter_nodes(r->p.dims, r->drd, r->d.npts, r->hrd.filter_stages, rho,
                             at<double>(r, r->L.ftmp[0]), at<double>(r, r->L.ftmp[1]), r->stream);
}

pic_status read_counters(pic_run* r, Counters& c) {
  HIPCHK(hipMemcpyAsync(&c, r->dctr, sizeof(Counters), hipMemcpyDeviceToHost, r->stream));
  HIPCHK(hipStreamSynchronize(r->stream));
  if (c.step != r->hstep)
    return fail(PIC_ESTATE, "step counters disagree (device %lld, host %lld)", c.step, r->hstep);
  return PIC_OK;
}

double bits_to_double(unsigned long long b) {
  double v;
  memcpy(&v, &b, sizeof(v));
  return v;
}

}  // namespace

namespace {
template <typename R>
static pic_status read_parts(pic_run* r, const Counters& c, int64_t first, int64_t n, double* z,
                             double* x, double* y, double* ux, double* uy, double* uz, uint32_t* id,
                             int64_t* n_out) {
  const int pb = c.pbuf;
  std::vector<int> cell(n);
  std::vector<R> o[3], u[3];
  std::vector<unsigned> pid(n);
  HIPCHK(hipMemcpy(cell.data(), r->hrd.cell[pb] + first, sizeof(int) * n, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(pid.data(), r->hrd.pid[pb] + first, sizeof(unsigned) * n, hipMemcpyDeviceToHost));
  for (int d = 0; d < 3; ++d) {
    o[d].assign(n, R(0));
    u[d].resize(n);
    if (r->hrd.off[pb][d])
      HIPCHK(hipMemcpy(o[d].data(), static_cast<R*>(r->hrd.off[pb][d]) + first, sizeof(R) * n,
                       hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(u[d].data(), static_cast<R*>(r->hrd.u[pb][d]) + first, sizeof(R) * n,
                     hipMemcpyDeviceToHost));
  }
  int64_t w = 0;
  const double dy = r->p.dims == 3 ? r->p.dy : 0.0;
  for (int64_t q = 0; q < n; ++q) {
    const int cc = cell[q];
    if (cc < 0) continue;
    const int k = (cc & KMASK) - KOFF, i = (cc >> KBITS) & IMASK, j = (cc >> (KBITS + IBITS)) & JMASK;
    if (z) z[w] = (k + (double)o[0][q]) * r->p.dz;
    if (x) x[w] = (i + (double)o[1][q]) * r->p.dx;
    if (y) y[w] = r->p.dims == 3 ? (j + (double)o[2][q]) * dy : 0.0;
    if (ux) ux[w] = (double)u[0][q];
    if (uy) uy[w] = (double)u[1][q];
    if (uz) uz[w] = (double)u[2][q];
    if (id) id[w] = pid[q];
    ++w;
  }
  if (n_out) *n_out = w;
  return PIC_OK;
}

}  // namespace

extern "C" {

const char* pic_last_error(void) { return g_err.c_str(); }

pic_status pic_state_bytes(const pic_lab_params* p, size_t* bytes) {
  if (!bytes) return fail(PIC_EINVAL, "bytes is NULL");
  Derived d;
  pic_status s = derive(p, d);
  if (s != PIC_OK) return s;
  Layout L;
  layout(p, d, L);
  *bytes = L.total;
  return PIC_OK;
}

pic_status pic_init_boosted(const pic_lab_params* p, void* dev_buf, size_t bytes, void* hip_stream,
                            pic_run** out) {
  g_err.clear();
  if (!out) return fail(PIC_EINVAL, "out is NULL");
  *out = nullptr;
  if (!dev_buf) return fail(PIC_EINVAL, "dev_buf is NULL");
  Derived d;
  pic_status st = derive(p, d);
  if (st != PIC_OK) return st;
  pic_run* r = new pic_run();
  static std::atomic<unsigned long long> next_serial{1};
  r->serial = next_serial++;
  r->p = *p;
  if (r->p.dims == 2) r->p.ny = 1;
  r->d = d;
  layout(&r->p, d, r->L);
  if (bytes < r->L.total) {
    size_t need = r->L.total;
    delete r;
    return fail(PIC_EBUDGET, "buffer of %zu bytes is smaller than the %zu needed", bytes, need);
  }
  if (reinterpret_cast<uintptr_t>(dev_buf) % 256) {
    delete r;
    return fail(PIC_EINVAL, "dev_buf must be 256-byte aligned");
  }
  r->base = static_cast<char*>(dev_buf);
  r->bytes = bytes;
  r->stream = static_cast<hipStream_t>(hip_stream);
  r->use_graph = true;
  r->g1[0] = r->g1[1] = nullptr;
  r->gB[0] = r->gB[1] = nullptr;
  r->gB_shape[0] = r->gB_shape[1] = StepShape();
  r->hstep = 0;
  int dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&r->ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (r->ncu <= 0) r->ncu = 256;
  r->gpart = grid_particles(r->p.dims, r->p.precision, r->ncu);
  r->ggen = grid_generic(r->ncu);

  // ---- descriptor
  RunDev& h = r->hrd;
  memset(&h, 0, sizeof(h));
  h.dims = r->p.dims;
  h.nz = r->p.nz;
  h.nx = r->p.nx;
  h.ny = r->p.ny;
  h.nzf = d.nzf;
  h.open = r->p.bc_z == PIC_BC_OPEN;
  h.ppc = r->p.ppc;
  h.reservoir = d.reservoir;
  h.ztop = d.ztop;
  h.inject_every = r->p.sort_every;
  h.ntz = d.ntz;
  h.ntx = d.ntx;
  h.nty = d.nty;
  h.ntiles = d.ntiles;
  h.gx = r->p.nx / 4;
  h.gy = r->p.dims == 3 ? r->p.ny / 4 : 0;
  h.gz = r->p.nz / 4;
  h.pusher = r->p.pusher;
  h.diag_flags = (int)r->p.diag_flags;
  h.filter_passes = r->p.filter_passes;
  h.filter_comp = r->p.filter_compensate;
  h.filter_stages = r->p.filter_passes > 0
                        ? (r->p.filter_passes + r->p.filter_compensate) * (r->p.dims == 3 ? 3 : 2) : 0;
  h.pol_axis = r->p.pol_axis;
  h.capacity = d.capacity;
  h.nperp = d.nperp;
  h.npts = d.npts;
  h.max_new = d.max_new;
  h.dt = d.dt;
  h.dz = r->p.dz;
  h.dx = r->p.dx;
  h.dy = r->p.dims == 3 ? r->p.dy : 1.0;
  h.beta_b = d.beta_b;
  h.gamma_b = d.gamma_b;
  h.dminus = d.dminus;
  h.dplus = d.dplus;
  h.weight = d.weight;
  h.jion_z = r->p.ppc > 0 ? -d.gamma_b * d.beta_b : 0.0;
  h.rho_ion = r->p.ppc > 0 ? d.gamma_b : 0.0;
  h.u_th = r->p.u_th;
  h.k0_lab = d.k0_lab;
  h.E0_lab = d.E0_lab;
  h.L_lab = d.L_lab;
  h.zc_boost = d.zc_boost;
  h.waist = r->p.waist;
  // current in 64-bit fixed point (scale chosen in derive)
  h.jscale = d.jscale;
  h.jinv = 1.0 / h.jscale;
  {
    const double S = h.jscale, w = h.weight, dt = h.dt, dz = h.dz, dx = h.dx, dy = h.dy;
    h.pk[0] = -0.5 * dt;
    h.pk[1] = dt / dz;
    h.pk[2] = dt / dx;
    h.pk[3] = dt / dy;
    if (h.dims == 3) {
      h.pk[4] = S * w / (dx * dy * dt);
      h.pk[5] = S * w / (dz * dy * dt);
      h.pk[6] = S * w / (dz * dx * dt);
    } else {
      h.pk[4] = S * w / (dx * dt);
      h.pk[5] = S * w / (dz * dt);
      h.pk[6] = 0.0;
    }
    h.pk[7] = -S * w / (dz * dx);
  }
  h.seed = r->p.seed;
  const Layout& L = r->L;
  for (int b = 0; b < 2; ++b)
    for (int c = 0; c < 3; ++c) {
      h.E[b][c] = at<void>(r, L.E[b][c]);
      h.B[b][c] = at<void>(r, L.B[b][c]);
      h.off[b][c] = at<void>(r, L.off[b][c]);
      h.u[b][c] = at<void>(r, L.u[b][c]);
    }
  for (int c = 0; c < 3; ++c) {
    h.J[0][c] = at<void>(r, L.J[0][c]);
    h.J[1][c] = at<void>(r, L.J[1][c]);
    h.jlast[c] = at<double>(r, L.jlast[c]);
    h.jf[0][c] = at<void>(r, L.jf[0][c]);
    h.jf[1][c] = at<void>(r, L.jf[1][c]);
  }
  h.ftmp[0] = at<double>(r, L.ftmp[0]);
  h.ftmp[1] = at<double>(r, L.ftmp[1]);
  h.antenna = (r->p.laser_antenna && r->p.a0 > 0) ? 1 : 0;
  h.ant_z_lab = r->p.antenna_z_lab;
  h.ant_t_peak = r->p.antenna_t_peak;
  h.n_stations = r->p.n_stations;
  if (h.n_stations > 0) {
    h.st_stride = r->p.station_stride;
    h.st_cap = r->p.station_cap;
    h.st_nxs = d.st_nxs;
    h.st_nys = d.st_nys;
    h.st_z0 = r->p.station_z0;
    h.st_dz = r->p.station_dz;
    h.st_count = at<long long>(r, L.st_count);
    h.st_time = at<double>(r, L.st_time);
    h.st_data = at<double>(r, L.st_data);
  }
  for (int b = 0; b < 2; ++b) {
    h.cell[b] = at<int>(r, L.cell[b]);
    h.pid[b] = at<unsigned>(r, L.pid[b]);
    h.bbox[b] = at<int>(r, L.bbox[b]);
  }
  h.tile_start = at<int>(r, L.tile_start);
  h.tile_count = at<int>(r, L.tile_count);
  h.tile_cursor = at<int>(r, L.tile_cursor);
  h.tile_full = at<int>(r, L.tile_full);
  h.rho_a = at<double>(r, L.rho_a);
  h.rho_b = at<double>(r, L.rho_b);
  h.gauss0 = at<double>(r, L.gauss0);
  h.cell_snap = at<int>(r, L.cell_snap);
  h.slowq = at<int>(r, L.slowq);
  r->drd = at<RunDev>(r, L.rundev);
  r->dctr = at<Counters>(r, L.ctr);
  r->dtab1 = at<BatchTable>(r, L.tab1);
  r->dtabB = at<BatchTable>(r, L.tabB);
  h.ctr = r->dctr;

  // host staging of the copies below lives in the run handle (hrd, hctr0,
  // htab1), so the copies may still be in flight when this call returns
  Counters& c0 = r->hctr0;
  memset(&c0, 0, sizeof(c0));
  c0.last_sort = -1;
  pic_run* self = r;
  fill_table(r->htab1, &self, 1);

  hipStream_t s = r->stream;
  auto bail = [&](pic_status e) {
    (void)hipStreamSynchronize(s);  // nothing enqueued may still read the handle
    delete r;
    return e;
  };
#define INITCHK(expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return bail(fail(PIC_EHIP, "%s: %s", #expr, hipGetErrorString(e_))); \
  } while (0)
  INITCHK(hipMemsetAsync(r->base, 0, L.zero_end, s));
  INITCHK(hipMemcpyAsync(r->drd, &r->hrd, sizeof(RunDev), hipMemcpyHostToDevice, s));
  INITCHK(hipMemcpyAsync(r->dctr, &c0, sizeof(Counters), hipMemcpyHostToDevice, s));
  INITCHK(hipMemcpyAsync(r->dtab1, &r->htab1, sizeof(BatchTable), hipMemcpyHostToDevice, s));
  if (r->p.a0 > 0) {
    launch_init_fields(r->p.dims, r->p.precision, r->drd, d.npts, s);
    // leapfrog state: B^{-1/2} = B^0 + dt/2 curl E^0
    launch_bshift(r->p.precision, r->drd, d.npts, 0, 0, 0.5 * d.dt, s);
  }
  launch_sort_chain(r->p.dims, r->p.precision, r->dtab1, MAX_BATCH, r->ggen, s);
  launch_rho(r->p.dims, r->p.precision, r->drd, at<double>(r, L.rho_a), d.npts, d.capacity, 0, s);
  launch_gauss(r->p.precision, r->drd, d.npts, 0, gauss_rho(r), s);
  INITCHK(hipGetLastError());
#undef INITCHK
  *out = r;
  return PIC_OK;
}

pic_status pic_set_option(pic_run* r, int opt, int value) {
  if (!r) return fail(PIC_EINVAL, "run is NULL");
  if (opt == PIC_OPT_GRAPH) {
    r->use_graph = value != 0;
    return PIC_OK;
  }
  return fail(PIC_EINVAL, "unknown option %d", opt);
}

pic_status pic_step(pic_run* r, int nsteps) {
  if (!r) return fail(PIC_EINVAL, "run is NULL");
  if (nsteps < 0) return fail(PIC_EINVAL, "nsteps < 0");
  const bool cont = (r->p.diag_flags & PIC_DIAGF_CONTINUITY) != 0;
  // the legacy null stream cannot be captured: launch eagerly there
  const bool graph = r->use_graph && r->stream != nullptr && nsteps >= 2;
  for (int i = 0; i < nsteps; ++i) {
    const bool chain = chain_step(r);
    if (graph) {
      hipGraphExec_t& g = r->g1[chain ? 1 : 0];
      if (!g) {
        pic_status st = capture(r, r->dtab1, cont, chain, shape_of(r), &g);
        if (st != PIC_OK) return st;
      }
      HIPCHK(hipGraphLaunch(g, r->stream));
    } else {
      enqueue_step(r, r->dtab1, cont, chain, shape_of(r));
    }
    host_advance(r);
  }
  HIPCHK(hipGetLastError());
  return PIC_OK;
}

pic_status pic_step_timed(pic_run* r, int nsteps, double ms[4]) {
  if (!r || !ms) return fail(PIC_EINVAL, "NULL argument");
  if (nsteps <= 0) return fail(PIC_EINVAL, "nsteps must be positive");
  if (r->p.diag_flags & PIC_DIAGF_CONTINUITY)
    return fail(PIC_EINVAL, "timing is not available with continuity diagnostics");
  const int dims = r->p.dims, prec = r->p.precision;
  hipStream_t s = r->stream;
  std::vector<hipEvent_t> ev((size_t)nsteps * 4, nullptr);
  pic_status st = PIC_OK;
  for (auto& e : ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      st = fail(PIC_EHIP, "hipEventCreate failed");
      break;
    }
  }
  if (st == PIC_OK) {
    for (int i = 0; i < nsteps; ++i) {
      hipEvent_t* e = &ev[(size_t)i * 4];
      (void)hipEventRecord(e[0], s);
      if (chain_step(r)) launch_sort_chain(dims, prec, r->dtab1, MAX_BATCH, r->ggen, s);
      host_advance(r);
      (void)hipEventRecord(e[1], s);
      launch_particles(dims, prec, r->p.pusher, r->dtab1, r->gpart, s);
      (void)hipEventRecord(e[2], s);
      launch_fields(dims, prec, r->dtab1, r->ggen, r->hrd.filter_stages, r->d.ant_plane, s);
      if (r->d.st_items > 0) launch_stations(prec, r->dtab1, r->d.st_items, r->ggen, s);
      launch_advance(r->dtab1, MAX_BATCH, s);
      (void)hipEventRecord(e[3], s);
    }
    hipError_t err = hipStreamSynchronize(s);
    if (err != hipSuccess) st = fail(PIC_EHIP, "timed steps: %s", hipGetErrorString(err));
  }
  if (st == PIC_OK) {
    double acc[4] = {0, 0, 0, 0};
    for (int i = 0; i < nsteps; ++i) {
      hipEvent_t* e = &ev[(size_t)i * 4];
      float t01 = 0, t12 = 0, t23 = 0, t03 = 0;
      (void)hipEventElapsedTime(&t01, e[0], e[1]);
      (void)hipEventElapsedTime(&t12, e[1], e[2]);
      (void)hipEventElapsedTime(&t23, e[2], e[3]);
      (void)hipEventElapsedTime(&t03, e[0], e[3]);
      acc[0] += t01;
      acc[1] += t12;
      acc[2] += t23;
      acc[3] += t03;
    }
    for (int q = 0; q < 4; ++q) ms[q] = acc[q] / nsteps;
  }
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  return st;
}

// Pinned host staging of the batch tables that pic_step_batch uploads: a
// ring per device whose slots are reused once the copy that last read them
// has executed (one event per slot), so an upload never waits for the
// stream.  Allocated on first use, kept until the process ends.
namespace {
constexpr int TABLE_RING = 8;
constexpr int MAX_DEVICES = 16;
struct TableRing {
  BatchTable* host = nullptr;
  hipEvent_t ev[TABLE_RING] = {};
  int next = 0;
};
TableRing g_ring[MAX_DEVICES];
std::mutex g_ring_mutex;

pic_status upload_table(pic_run* r0, pic_run* const* act, int n) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES)
    return fail(PIC_EHIP, "no usable current device");
  std::lock_guard<std::mutex> lock(g_ring_mutex);
  TableRing& R = g_ring[dev];
  if (!R.host) {
    void* h = nullptr;
    HIPCHK(hipHostMalloc(&h, sizeof(BatchTable) * TABLE_RING, hipHostMallocDefault));
    for (int k = 0; k < TABLE_RING; ++k) {
      if (hipEventCreateWithFlags(&R.ev[k], hipEventDisableTiming) != hipSuccess) {
        for (int q = 0; q < k; ++q) (void)hipEventDestroy(R.ev[q]);
        (void)hipHostFree(h);
        return fail(PIC_EHIP, "hipEventCreateWithFlags failed");
      }
    }
    R.host = static_cast<BatchTable*>(h);
  }
  const int k = R.next;
  R.next = (k + 1) % TABLE_RING;
  HIPCHK(hipEventSynchronize(R.ev[k]));  // the copy that last read slot k has run
  fill_table(R.host[k], act, n);
  HIPCHK(hipMemcpyAsync(r0->dtabB, &R.host[k], sizeof(BatchTable), hipMemcpyHostToDevice, r0->stream));
  HIPCHK(hipEventRecord(R.ev[k], r0->stream));
  r0->tabB_runs.resize(n);
  for (int i = 0; i < n; ++i) r0->tabB_runs[i] = act[i]->serial;
  return PIC_OK;
}
}  // namespace

pic_status pic_step_batch(pic_run* const* runs, const int* nsteps, int n) {
  if (!runs || !nsteps || n <= 0) return fail(PIC_EINVAL, "empty batch");
  if (n > MAX_BATCH) return fail(PIC_EINVAL, "batch larger than %d", MAX_BATCH);
  pic_run* r0 = runs[0];
  for (int i = 0; i < n; ++i) {
    if (!runs[i]) return fail(PIC_EINVAL, "run %d is NULL", i);
    if (runs[i]->p.dims != r0->p.dims || runs[i]->p.precision != r0->p.precision ||
        runs[i]->p.pusher != r0->p.pusher)
      return fail(PIC_EINVAL, "batched runs must share dims, precision and pusher");
    if (runs[i]->p.diag_flags & PIC_DIAGF_CONTINUITY)
      return fail(PIC_EINVAL, "continuity diagnostics are single-run only");
    if (nsteps[i] < 0) return fail(PIC_EINVAL, "nsteps[%d] < 0", i);
  }
  int maxs = 0;
  for (int i = 0; i < n; ++i) maxs = nsteps[i] > maxs ? nsteps[i] : maxs;
  std::vector<pic_run*> act;
  for (int s = 0; s < maxs; ++s) {
    std::vector<pic_run*> a;
    for (int i = 0; i < n; ++i)
      if (nsteps[i] > s) a.push_back(runs[i]);
    if (a != act) {
      act = a;
      bool same = act.size() == r0->tabB_runs.size();
      for (size_t i = 0; same && i < act.size(); ++i) same = act[i]->serial == r0->tabB_runs[i];
      if (!same) {  // the device table holds another batch: upload this one
        pic_status st = upload_table(r0, act.data(), (int)act.size());
        if (st != PIC_OK) return st;
      }
    }
    StepShape sh;  // the most any run of the batch needs
    bool chain = false;
    for (pic_run* q : act) {
      chain = chain || chain_step(q);
      const StepShape qs = shape_of(q);
      sh.fstages = std::max(sh.fstages, qs.fstages);
      sh.st_items = std::max(sh.st_items, qs.st_items);
      sh.ant_plane = std::max(sh.ant_plane, qs.ant_plane);
    }
    if (r0->use_graph && r0->stream != nullptr) {
      hipGraphExec_t& g = r0->gB[chain ? 1 : 0];
      StepShape& gsh = r0->gB_shape[chain ? 1 : 0];
      if (g && gsh != sh) {
        HIPCHK(hipStreamSynchronize(r0->stream));
        (void)hipGraphExecDestroy(g);
        g = nullptr;
      }
      if (!g) {
        pic_status st = capture(r0, r0->dtabB, false, chain, sh, &g);
        if (st != PIC_OK) return st;
        gsh = sh;
      }
      HIPCHK(hipGraphLaunch(g, r0->stream));
    } else {
      enqueue_step(r0, r0->dtabB, false, chain, sh);
    }
    for (pic_run* q : act) host_advance(q);
  }
  HIPCHK(hipGetLastError());
  return PIC_OK;
}

pic_status pic_step_batch_noalloc(pic_run* const* runs, const int* nsteps, int n) {
  if (!runs || !nsteps || n <= 0) return fail(PIC_EINVAL, "empty batch");
  if (n > MAX_BATCH) return fail(PIC_EINVAL, "batch larger than %d", MAX_BATCH);
  pic_run* r0 = runs[0];
  int maxs = 0;
  for (int i = 0; i < n; ++i) {
    if (!runs[i]) return fail(PIC_EINVAL, "run %d is NULL", i);
    if (runs[i]->p.dims != r0->p.dims || runs[i]->p.precision != r0->p.precision ||
        runs[i]->p.pusher != r0->p.pusher)
      return fail(PIC_EINVAL, "batched runs must share dims, precision and pusher");
    if (runs[i]->p.diag_flags & PIC_DIAGF_CONTINUITY)
      return fail(PIC_EINVAL, "continuity diagnostics are single-run only");
    if (nsteps[i] < 0) return fail(PIC_EINVAL, "nsteps[%d] < 0", i);
    maxs = nsteps[i] > maxs ? nsteps[i] : maxs;
  }
  BatchTable* tab = nullptr;  // this device's table (set up on the first call)
  HIPCHK(batch_scratch(&tab));
  // everything below lives on the stack: no allocation of any kind
  BatchTable host;
  pic_run* act[MAX_BATCH];
  int nact = -1;
  for (int s = 0; s < maxs; ++s) {
    pic_run* a[MAX_BATCH];
    int na = 0;
    for (int i = 0; i < n; ++i)
      if (nsteps[i] > s) a[na++] = runs[i];
    bool same = na == nact;
    for (int i = 0; same && i < na; ++i) same = a[i] == act[i];
    if (!same) {
      // the whole table is rewritten (fill_table clears it first); a copy
      // from pageable memory is performed by HIP when it is enqueued, in
      // stream order after the steps already enqueued on r0's stream
      for (int i = 0; i < na; ++i) act[i] = a[i];
      nact = na;
      fill_table(host, act, nact);
      HIPCHK(hipMemcpyAsync(tab, &host, sizeof(BatchTable), hipMemcpyHostToDevice, r0->stream));
    }
    StepShape sh;
    bool chain = false;
    for (int i = 0; i < nact; ++i) {
      chain = chain || chain_step(act[i]);
      const StepShape qs = shape_of(act[i]);
      sh.fstages = std::max(sh.fstages, qs.fstages);
      sh.st_items = std::max(sh.st_items, qs.st_items);
      sh.ant_plane = std::max(sh.ant_plane, qs.ant_plane);
    }
    enqueue_step(r0, tab, false, chain, sh);  // direct launches: no graph is built
    for (int i = 0; i < nact; ++i) host_advance(act[i]);
  }
  HIPCHK(hipGetLastError());
  return PIC_OK;
}

pic_status pic_diag(pic_run* r, unsigned what, pic_diag_out* out) {
  if (!r || !out) return fail(PIC_EINVAL, "NULL argument");
  hipStream_t s = r->stream;
  HIPCHK(hipMemsetAsync(&r->dctr->acc[0], 0,
                        sizeof(r->dctr->acc) + sizeof(r->dctr->amax) + sizeof(r->dctr->cnt), s));
  launch_diag(r->p.dims, r->p.precision, r->drd, r->d.npts, r->d.capacity, what & 3u, s);
  if (what & PIC_DIAG_GAUSS) {
    launch_rho(r->p.dims, r->p.precision, r->drd, at<double>(r, r->L.rho_a), r->d.npts, r->d.capacity,
               0, s);
    launch_gauss(r->p.precision, r->drd, r->d.npts, 1, gauss_rho(r), s);
  }
  HIPCHK(hipGetLastError());
  Counters c;
  pic_status st = read_counters(r, c);
  if (st != PIC_OK) return st;
  memset(out, 0, sizeof(*out));
  out->step = c.step;
  out->t = c.step * r->d.dt;
  out->U_E = c.acc[0];
  out->U_B = c.acc[1];
  out->Ez_max = bits_to_double(c.amax[0]);
  out->KE = c.acc[2];
  out->n_particles = (int64_t)llround(c.acc[3]);
  const double rho0 = c.rho0_max;
  const double gd = bits_to_double(c.amax[1]);
  out->gauss_drift = (what & PIC_DIAG_GAUSS) ? (rho0 > 0 ? gd / rho0 : gd) : -1.0;
  if (r->p.diag_flags & PIC_DIAGF_CONTINUITY) {
    out->cont_resid = c.cont_max;
    HIPCHK(hipMemsetAsync(&r->dctr->cont_max, 0, sizeof(double), s));
  } else {
    out->cont_resid = -1.0;
  }
  out->err_bits = c.err;
  out->n_slow = (int64_t)c.n_slow;
  HIPCHK(hipMemsetAsync(&r->dctr->n_slow, 0, sizeof(c.n_slow), s));
  if (c.err) {
    HIPCHK(hipStreamSynchronize(s));
    if (c.err & PIC_ERR_NAN) return fail(PIC_ESTATE, "device error: non-finite momentum");
    if (c.err & PIC_ERR_CAPACITY) return fail(PIC_ESTATE, "device error: particle capacity exceeded");
    if (c.err & PIC_ERR_TILE) return fail(PIC_ESTATE, "device error: a tile holds 2^28 or more particles");
    return fail(PIC_ESTATE, "device error word 0x%x", c.err);
  }
  HIPCHK(hipStreamSynchronize(s));
  return PIC_OK;
}

pic_status pic_particle_count(pic_run* r, int64_t* slots, int64_t* live) {
  if (!r) return fail(PIC_EINVAL, "run is NULL");
  Counters c;
  pic_status st = read_counters(r, c);
  if (st != PIC_OK) return st;
  if (slots) *slots = c.n_slots;
  if (live) {
    // count the live slots
    std::vector<int> cell((size_t)c.n_slots);
    if (c.n_slots)
      HIPCHK(hipMemcpy(cell.data(), r->hrd.cell[c.pbuf], sizeof(int) * c.n_slots, hipMemcpyDeviceToHost));
    int64_t n = 0;
    for (int v : cell) n += v >= 0;
    *live = n;
  }
  return PIC_OK;
}

pic_status pic_read_particles(pic_run* r, int64_t first, int64_t count, double* z, double* x,
                              double* y, double* ux, double* uy, double* uz, uint32_t* id,
                              int64_t* n_out) {
  if (!r) return fail(PIC_EINVAL, "run is NULL");
  if (first < 0 || count < 0) return fail(PIC_EINVAL, "negative range");
  Counters c;
  pic_status st = read_counters(r, c);
  if (st != PIC_OK) return st;
  int64_t n = count;
  if (first >= c.n_slots) n = 0;
  else if (first + n > c.n_slots) n = c.n_slots - first;
  if (n == 0) {
    if (n_out) *n_out = 0;
    return PIC_OK;
  }
  if (r->p.precision == PIC_FP64) return read_parts<double>(r, c, first, n, z, x, y, ux, uy, uz, id, n_out);
  return read_parts<float>(r, c, first, n, z, x, y, ux, uy, uz, id, n_out);
}

pic_status pic_read_fields(pic_run* r, int comp, double* host, int64_t npts) {
  if (!r || !host) return fail(PIC_EINVAL, "NULL argument");
  if (npts < r->d.npts) return fail(PIC_EINVAL, "host array holds %lld < %lld points", (long long)npts,
                                    (long long)r->d.npts);
  Counters c;
  pic_status st = read_counters(r, c);
  if (st != PIC_OK) return st;
  const size_t n = (size_t)r->d.npts;
  if (comp >= PIC_F_JX_LAST && comp <= PIC_F_JZ_LAST) {
    double* src = r->hrd.jlast[comp - PIC_F_JX_LAST];
    if (!src) return fail(PIC_EINVAL, "J_LAST needs PIC_DIAGF_CONTINUITY");
    HIPCHK(hipMemcpy(host, src, sizeof(double) * n, hipMemcpyDeviceToHost));
    return PIC_OK;
  }
  if (comp < 0 || comp > PIC_F_BZ) return fail(PIC_EINVAL, "bad component %d", comp);
  void* src;
  if (comp < 3) {
    src = r->hrd.E[c.fbuf][comp];
  } else {
    // B^n = B^{n-1/2} - dt/2 curl E^n, written to the idle B buffer
    launch_bshift(r->p.precision, r->drd, r->d.npts, -1, -1, -0.5 * r->d.dt, r->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(r->stream));
    src = r->hrd.B[c.fbuf ^ 1][comp - 3];
  }
  if (r->p.precision == PIC_FP64) {
    HIPCHK(hipMemcpy(host, src, sizeof(double) * n, hipMemcpyDeviceToHost));
  } else {
    std::vector<float> tmp(n);
    HIPCHK(hipMemcpy(tmp.data(), src, sizeof(float) * n, hipMemcpyDeviceToHost));
    for (size_t q = 0; q < n; ++q) host[q] = tmp[q];
  }
  return PIC_OK;
}

pic_status pic_read_station(pic_run* r, int station, int64_t* count, double* times, double* data,
                            int64_t max_samples) {
  if (!r || !count) return fail(PIC_EINVAL, "NULL argument");
  if (r->p.n_stations <= 0) return fail(PIC_EINVAL, "the run has no stations");
  if (station < 0 || station >= r->p.n_stations)
    return fail(PIC_EINVAL, "station %d outside [0, %d)", station, r->p.n_stations);
  if (max_samples < 0) return fail(PIC_EINVAL, "max_samples < 0");
  if (max_samples > 0 && (!times || !data)) return fail(PIC_EINVAL, "times or data is NULL");
  Counters c;
  pic_status st = read_counters(r, c);
  if (st != PIC_OK) return st;
  long long n = 0;
  HIPCHK(hipMemcpy(&n, r->hrd.st_count + station, sizeof(n), hipMemcpyDeviceToHost));
  *count = n;
  const long long cap = r->p.station_cap;
  const long long m = std::min(std::min(n, cap), (long long)max_samples);
  if (m > 0) {
    const size_t rec = 6 * (size_t)r->d.st_nxs * (size_t)r->d.st_nys;
    HIPCHK(hipMemcpy(times, r->hrd.st_time + (size_t)station * cap, sizeof(double) * m,
                     hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(data, r->hrd.st_data + (size_t)station * cap * rec, sizeof(double) * m * rec,
                     hipMemcpyDeviceToHost));
  }
  return PIC_OK;
}

pic_status pic_get_derived(const pic_run* r, pic_derived* o) {
  if (!r || !o) return fail(PIC_EINVAL, "NULL argument");
  const Derived& d = r->d;
  o->dt = d.dt;
  o->beta_b = d.beta_b;
  o->gamma_b = d.gamma_b;
  o->dminus = d.dminus;
  o->dplus = d.dplus;
  o->skin_um = d.skin_um;
  o->k0_lab = d.k0_lab;
  o->E0_lab = d.E0_lab;
  o->L_lab = d.L_lab;
  o->L_boost = d.L_boost;
  o->zc_boost = d.zc_boost;
  o->weight = d.weight;
  o->dV = d.dV;
  o->reservoir = d.reservoir;
  o->nzf = d.nzf;
  o->capacity = d.capacity;
  o->ntiles = d.ntiles;
  return PIC_OK;
}

pic_status pic_free(pic_run* r) {
  if (!r) return PIC_OK;
  // no wait: the caller frees a run only after the work that uses it has
  // run (the host staging it holds is read by copies HIP performs when
  // they are enqueued, pageable memory being copied synchronously)
  for (int q = 0; q < 2; ++q) {
    if (r->g1[q]) (void)hipGraphExecDestroy(r->g1[q]);
    if (r->gB[q]) (void)hipGraphExecDestroy(r->gB[q]);
  }
  delete r;
  return PIC_OK;
}

pic_status pic_push_bench(int precision, int pusher, int64_t n, int nsteps, double dt, const double B[3],
                          void* Ex, void* u, int32_t* cell, void* off, void* hip_stream) {
  if (precision != PIC_FP32_SPLIT && precision != PIC_FP64) return fail(PIC_EINVAL, "bad precision");
  if (pusher != PIC_VAY && pusher != PIC_BORIS) return fail(PIC_EINVAL, "bad pusher");
  if (n < 0 || nsteps < 0) return fail(PIC_EINVAL, "negative size");
  if (!(dt > 0) || !(dt < 1)) return fail(PIC_ECFL, "dt must be in (0, 1) on the unit grid");
  if (!B) return fail(PIC_EINVAL, "B is NULL");
  if (n == 0 || nsteps == 0) return PIC_OK;
  if (!Ex || !u || !cell || !off) return fail(PIC_EINVAL, "NULL array");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  for (int i = 0; i < nsteps; ++i)
    launch_push_bench(precision, pusher, (long long)n, dt, B, Ex, u, cell, off, s);
  HIPCHK(hipGetLastError());
  return PIC_OK;
}

pic_status pic_copy_bench(const void* src, void* dst, int64_t nbytes, void* hip_stream) {
  if (nbytes < 0) return fail(PIC_EINVAL, "negative size");
  if (nbytes % 16 != 0) return fail(PIC_EINVAL, "nbytes must be a multiple of 16");
  if (nbytes == 0) return PIC_OK;
  if (!src || !dst) return fail(PIC_EINVAL, "NULL buffer");
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16 != 0)
    return fail(PIC_EINVAL, "buffers must be 16-byte aligned");
  launch_copy_bench(src, dst, (long long)(nbytes / 16), static_cast<hipStream_t>(hip_stream));
  HIPCHK(hipGetLastError());
  return PIC_OK;
}

pic_status pic_stream_bench(int mode, const void* src, void* dst, int64_t nbytes, void* hip_stream) {
  if (mode < 0 || mode > 2) return fail(PIC_EINVAL, "mode must be 0 (copy), 1 (read) or 2 (write)");
  if (nbytes < 0) return fail(PIC_EINVAL, "negative size");
  if (nbytes % 16 != 0) return fail(PIC_EINVAL, "nbytes must be a multiple of 16");
  if (nbytes == 0) return PIC_OK;
  if ((mode != 2 && !src) || !dst) return fail(PIC_EINVAL, "NULL buffer");
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16 != 0)
    return fail(PIC_EINVAL, "buffers must be 16-byte aligned");
  launch_stream_bench(mode, src, dst, (long long)(nbytes / 16), static_cast<hipStream_t>(hip_stream));
  HIPCHK(hipGetLastError());
  return PIC_OK;
}

}  // extern "C"
