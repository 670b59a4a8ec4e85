/*
 * libpic: one-GPU (MI355X, gfx950) boosted-frame electromagnetic
 * particle-in-cell step, after Vay, Fawley, Geddes, Cormier-Michel and Grote,
 * "Speeding up simulations of relativistic systems using an optimal boosted
 * frame" (2009).
 *
 * The calls follow the paper's statement of the problem (Sec. 2): inputs are
 * given in the laboratory frame (laser and plasma parameters, second
 * paragraph), the system is evolved by the relativistic PIC algorithm in the
 * boosted frame (third paragraph), and diagnostics are reported from the
 * boosted-frame state (plus the boost-invariant longitudinal field).
 *
 * Ownership.  The caller owns all device memory: it allocates one buffer of
 * pic_state_bytes() bytes and passes it to pic_init_boosted(), together with
 * the HIP stream everything is enqueued on.  The library never allocates
 * device memory; it owns only the small host-side handle and any HIP graphs
 * it captures.  The buffer must stay alive and untouched until pic_free().
 *
 * Device.  A run lives on the HIP device that is current when
 * pic_init_boosted() is called; every later call on it (and every batched
 * call, whose runs must all live there) must be made with that device
 * current.
 *
 * Errors.  No call throws.  Argument errors are returned synchronously as a
 * negative pic_status and described by pic_last_error() (thread-local).
 * Errors raised inside kernels (non-finite momentum, particle capacity
 * exceeded) set bits in a device error word; pic_diag() reports them and
 * returns PIC_ESTATE.
 *
 * Units: lengths in c/omega_p and times in 1/omega_p of the laboratory plasma
 * frequency; c = eps0 = 1; electron charge -1 and mass 1.
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PIC_OK = 0,
  PIC_EINVAL = -1,    /* bad argument */
  PIC_EBUDGET = -2,   /* device buffer smaller than pic_state_bytes() */
  PIC_EHIP = -3,      /* a HIP runtime call failed */
  PIC_ECFL = -4,      /* time step violates the CFL bound */
  PIC_ENAN = -5,      /* a kernel produced a non-finite momentum */
  PIC_ECAPACITY = -6, /* particle storage overflowed */
  PIC_ESTATE = -7     /* the run carries a device-side error */
} pic_status;

enum { PIC_BC_OPEN = 0, PIC_BC_PERIODIC = 1 };
enum { PIC_VAY = 0, PIC_BORIS = 1 };
enum { PIC_FP32_SPLIT = 0, PIC_FP64 = 1 };

/* device error-word bits: a non-finite momentum; particle storage full; a
 * tile holding 2^28 or more particles (its particles are then not advanced) */
enum { PIC_ERR_NAN = 1u, PIC_ERR_CAPACITY = 2u, PIC_ERR_TILE = 4u };

/* pic_lab_params.diag_flags */
enum {
  PIC_DIAGF_CONTINUITY = 1u /* measure the continuity residual every step */
};

/* Laboratory-frame problem description (Sec. 2, second paragraph: laser and
 * plasma parameters are given in the laboratory and transformed). */
typedef struct {
  int dims;              /* 2: (z,x) with three velocity components; 3: (z,x,y) */
  int nz, nx, ny;        /* boosted-frame cells; ny ignored in 2D.  nx, ny must be
                            multiples of the transverse tile (2D: 16; 3D: 8 x 8 in
                            split precision, 8 x 4 in FP64) */
  double dz, dx, dy;     /* cell sizes in c/omega_p */
  double cfl;            /* dt = cfl / sqrt(sum_d 1/d^2); must be in (0, 1) */
  int ppc;               /* electrons per cell (>= 0) */
  uint64_t seed;         /* Philox4x64-10 key for positions and thermal momenta */
  double gamma_boost;    /* Lorentz factor of the boosted frame (>= 1) */
  double n_lab_cm3;      /* laboratory plasma density; sets omega_p */
  double u_th;           /* laboratory thermal momentum spread per component */
  double a0;             /* laser normalised amplitude (0: no laser) */
  double lambda0_um;     /* laser wavelength, laboratory frame */
  double waist;          /* transverse 1/e field radius, c/omega_p */
  double tau_lab;        /* lab envelope e-fold length; <= 0: boosted length nz dz/8 */
  int pol_axis;          /* 1 = x, 2 = y */
  int bc_z;              /* PIC_BC_OPEN (Mur + plasma reservoir) or PIC_BC_PERIODIC */
  int pusher;            /* PIC_VAY (default) or PIC_BORIS */
  int precision;         /* PIC_FP32_SPLIT or PIC_FP64 */
  int sort_every;        /* tile sort and plasma-column injection cadence (>= 1) */
  unsigned diag_flags;   /* PIC_DIAGF_* */
  /* Low-pass digital filter of the current between the deposit and the field
   * update (Sec. 2: the short-wavelength instability of boosted-frame runs
   * is controlled with low-pass filtering): filter_passes (0..16) passes of
   * the binomial stencil (1/4, 1/2, 1/4) along every axis on each
   * component's own staggered grid, then, if filter_compensate = 1, one pass
   * of (-N/4, 1 + N/2, -N/4) per axis.  Periodic axes wrap; along an open z
   * axis a neighbour beyond a component's range repeats the value at that
   * end (a current streaming uniformly out through the end passes
   * unchanged); points outside the range stay zero.  The continuity
   * diagnostic uses the deposited current, the Gauss diagnostic the filtered
   * electron density.  0 = no filter. */
  int filter_passes;
  int filter_compensate;
  /* Laboratory-frame stations (Sec. 2, third paragraph: results are wanted
   * in the laboratory, so lab-fixed planes record the boosted-frame fields
   * at the lab times their events map to, interpolated because those events
   * are not on the boosted grid).
   * Station q (0 <= q < n_stations) is the plane z_lab = Z_q = station_z0 +
   * q station_dz (c/omega_p, lab frame).  At boosted time t' = n dt it sits
   * at z' = Z_q / gamma_b - beta_b t' and the event it samples has lab time
   * t_lab = t' / gamma_b + beta_b Z_q.  Every step whose z' lies in
   * [0, nz dz), the station records E^n and B^n (integer time) at that z':
   * each component linearly interpolated in z between its own staggered
   * points (zero outside its range on an open axis, wrapped on a periodic
   * one), on the transverse node indices (i, j) = (a, b) station_stride for
   * a < nxs = nx / station_stride, b < nys = ny / station_stride (3D; nys = 1
   * in 2D), then transformed back to the laboratory frame (boost of
   * velocity -beta_b along z).  The first station_cap samples are stored in
   * the run's buffer; later ones are counted but dropped.  n_stations = 0:
   * none (the other station fields are then ignored).  Limits: n_stations
   * <= 65536, 1 <= station_stride <= nx (and <= ny in 3D), station_cap >= 1,
   * finite station_z0 and station_dz. */
  int n_stations;
  double station_z0, station_dz;
  int station_stride;
  int station_cap;
  /* Laser source (Sec. 2, second paragraph: the pulse may enter through a
   * plane at rest in the laboratory, which moves at -beta_b in the boosted
   * frame).  laser_antenna = 0:
   * the pulse is placed in the box at t' = 0, centred at nz dz / 2.
   * laser_antenna = 1: the lab plane z = antenna_z_lab (c/omega_p) emits it;
   * the envelope peak crosses the plane at lab time antenna_t_peak.  In the
   * boosted frame the plane sits at z'_a = antenna_z_lab / gamma_b - beta_b
   * t'.  The grid is made to carry the boosted incident wave above the plane
   * and nothing below: the sources are the residual of the Yee update
   * applied to H times the incident wave (H = 1 above the plane, at each
   * point's own staggered z and time), an electric current in the E update
   * and a magnetic current in the B update, at the points whose update
   * involves both sides.  They act while 2 dz <= z'_a < (nz - 2) dz; at
   * t' = 0 the box holds the incident wave above the plane.  In 3D the
   * flat-phase-front pulse has div E != 0, and the antenna current leaves
   * the matching charge (reported by the Gauss diagnostic); in 2D with the
   * polarisation along y it is divergence-free. */
  int laser_antenna;
  double antenna_z_lab, antenna_t_peak;
} pic_lab_params;

typedef struct pic_run pic_run; /* opaque host handle */

/* Diagnostics of the boosted-frame state at step `step` (a8).  Energies and
 * maxima are taken over interior points: two cells are excluded at each open
 * z end. */
typedef struct {
  int64_t step;
  double t;
  double U_E, U_B;       /* 1/2 sum F^2 dV */
  double Ez_max;         /* max |E_z| (wake amplitude; invariant under the z boost) */
  double KE;             /* sum w (gamma - 1) over interior electrons */
  int64_t n_particles;   /* electrons inside the physical box */
  double cont_resid;     /* max over steps since the last call of
                            max|rho^{n+1}-rho^n+dt div J| / max|rho_e^n|
                            (needs PIC_DIAGF_CONTINUITY, else -1) */
  double gauss_drift;    /* max |(divE-rho)^n-(divE-rho)^0| / max|rho_e^0| */
  uint32_t err_bits;     /* device error word */
  int64_t n_slow;        /* particle pushes since the last call whose stencil left
                            the tile's LDS window (they read and deposit in HBM) */
} pic_diag_out;

enum { PIC_DIAG_FIELDS = 1u, PIC_DIAG_PARTICLES = 2u, PIC_DIAG_GAUSS = 4u, PIC_DIAG_ALL = 7u };

/* Bytes of device memory a run of these parameters needs (Sec. 2, second
 * paragraph: the run's size is that of the boosted-frame problem, a box of
 * nz x nx x ny cells holding the plasma at gamma_b times the laboratory
 * density as ppc electrons per cell, plus the reservoir and tile slack).
 * Pure host function, no device call; used for admission by memory budget.
 * Returns PIC_EINVAL for invalid parameters. */
pic_status pic_state_bytes(const pic_lab_params* p, size_t* bytes);

/* Transform the laboratory inputs to the boosted frame and lay out the run in
 * dev_buf (Sec. 2, second paragraph: Doppler-shifted laser, denser drifting
 * plasma).  Enqueues on `hip_stream` (a hipStream_t; NULL means the null
 * stream) the copies of the run's descriptors, the laser transform, the
 * plasma creation, the first tile sort and the Gauss-law reference, and
 * returns without waiting for the kernels.  The descriptor copies come from
 * pageable host memory kept in the handle, which HIP performs synchronously:
 * they wait for work enqueued earlier on the same stream (give a new run an
 * idle stream to start it without waiting).  dev_buf: device pointer to
 * >= pic_state_bytes() bytes, 256-byte aligned, owned by the caller and
 * untouched by anything else until pic_free.  Errors: PIC_EINVAL, PIC_ECFL,
 * PIC_EBUDGET (buffer too small) and PIC_EHIP are returned before anything
 * is left enqueued; device-side errors of the kernels show in err_bits of
 * the next pic_diag. */
pic_status pic_init_boosted(const pic_lab_params* p, void* dev_buf, size_t bytes,
                            void* hip_stream, pic_run** out);

/* Enqueue nsteps full PIC steps (Sec. 2, third paragraph: the system is
 * evolved in the boosted frame; Sec. 2, first paragraph: the pusher with the
 * modified Lorentz force): gather, modified-Lorentz push, move,
 * charge-conserving deposit, Yee update; tile sort and plasma injection
 * every sort_every steps, and a tile sort alone within four steps after a
 * step in which more than 1/1024 of the particles left their tiles' LDS
 * windows).  The storage
 * order of the particles changes only at sorts; results do not depend on
 * it.  Asynchronous. */
pic_status pic_step(pic_run* run, int nsteps);

/* Advance several runs together (the serving pattern: each run is the Sec. 2,
 * third paragraph, boosted-frame evolution of pic_step): their tiles share
 * the same kernel launches, enqueued on the first run's stream.  All runs
 * must have the same dims, precision and pusher, no continuity
 * diagnostics, and no work pending on another stream (order it before the
 * call, e.g. with an event).  nsteps[i] >= 0 may differ; runs drop out when
 * done.  Asynchronous; PIC_EINVAL for an invalid batch, nothing enqueued. */
pic_status pic_step_batch(pic_run* const* runs, const int* nsteps, int n);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same steps as
 * pic_step_batch, with the same arguments, rules and results, but the batch
 * table the kernels read lives in a device array of the library (one table,
 * sizeof(BatchTable) = 6 KiB, per GPU, kept until the process ends; the
 * current device's is used, and set up on the first call there) and the
 * steps are launched directly, so the call allocates no device or pinned
 * host memory and creates no graph or event.  Limit: n <= 256 runs
 * (PIC_EINVAL beyond).  Every call on a GPU shares that GPU's table, which
 * holds the last call's batch: calls that overlap on one GPU (on different
 * streams) race, and must be ordered by the caller. */
pic_status pic_step_batch_noalloc(pic_run* const* runs, const int* nsteps, int n);

/* Enqueue nsteps steps without graph replay, bracketing each stage with HIP
 * events recorded on the run's stream, synchronise, and return the mean
 * device time per step of each stage in milliseconds: ms[0] = injection and
 * tile sort, ms[1] = particle kernel (gather, push, move, deposit),
 * ms[2] = field kernel and step advance, ms[3] = the whole step.
 * For measurement; the state advances exactly as with pic_step. */
pic_status pic_step_timed(pic_run* run, int nsteps, double ms[4]);

/* Compute diagnostics (what = PIC_DIAG_* mask) of the boosted-frame state
 * (Sec. 2, third paragraph: the outputs of the run; Sec. 3.1 compares runs
 * by field and particle energies): field energies, wake amplitude, kinetic
 * energy, particle count, continuity residual and Gauss-law drift, defined
 * on pic_diag_out above.  Synchronises the run's stream.  Returns
 * PIC_ESTATE if the device error word is set (out is still filled). */
pic_status pic_diag(pic_run* run, unsigned what, pic_diag_out* out);

/* Number of particle slots in storage order (live and dead) and of live ones. */
pic_status pic_particle_count(pic_run* run, int64_t* slots, int64_t* live);

/* Copy live particles of storage slots [first, first+count) to host arrays
 * (absolute positions in c/omega_p, momenta u = gamma v, lattice ids).
 * Arrays must hold `count` entries; *n_out receives the number written.
 * Synchronises the run's stream. */
pic_status pic_read_particles(pic_run* run, int64_t first, int64_t count,
                              double* z, double* x, double* y,
                              double* ux, double* uy, double* uz, uint32_t* id,
                              int64_t* n_out);

/* Field component ids for pic_read_fields */
enum { PIC_F_EX = 0, PIC_F_EY, PIC_F_EZ, PIC_F_BX, PIC_F_BY, PIC_F_BZ,
       PIC_F_JX_LAST, PIC_F_JY_LAST, PIC_F_JZ_LAST };

/* Copy one field component at integer time n (B is advanced to integer
 * time on the fly) as doubles, layout [ny][nx][nzf] with z fastest,
 * nzf = nz+1 (open z) or nz (periodic).  The J_LAST components are the
 * current of the most recent step (only with PIC_DIAGF_CONTINUITY).
 * host must hold `npts` doubles.  Synchronises. */
pic_status pic_read_fields(pic_run* run, int comp, double* host, int64_t npts);

/* Copy the record of laboratory-frame station `station` (see
 * pic_lab_params.n_stations) to host memory, in double precision:
 *   *count = samples taken so far (stored or not);
 *   times[m] = lab time of sample m;
 *   data[((m * 6 + c) * nys + b) * nxs + a] = lab-frame component c
 *     (Ex, Ey, Ez, Bx, By, Bz) at transverse node (a, b) station_stride,
 * for m < min(*count, station_cap, max_samples).  times must hold
 * max_samples doubles and data 6 nys nxs max_samples; either may be NULL
 * when max_samples = 0.  Synchronises the run's stream.  PIC_EINVAL for a
 * station index out of range or a run without stations. */
pic_status pic_read_station(pic_run* run, int station, int64_t* count, double* times,
                            double* data, int64_t max_samples);

/* Boosted-frame quantities derived from the parameters. */
typedef struct {
  double dt, beta_b, gamma_b, dminus, dplus, skin_um, k0_lab, E0_lab;
  double L_lab, L_boost, zc_boost, weight, dV;
  int reservoir, nzf;
  int64_t capacity; /* particle slots per buffer */
  int ntiles;
} pic_derived;
pic_status pic_get_derived(const pic_run* run, pic_derived* out);

/* Options for pic_set_option */
enum { PIC_OPT_GRAPH = 1 /* 1 (default): replay each step as a captured HIP graph */ };
pic_status pic_set_option(pic_run* run, int opt, int value);

/* Release the host handle and graphs (device memory stays the caller's).
 * NULL-safe. */
pic_status pic_free(pic_run* run);

/* Message for the last error on this thread ("" if none). */
const char* pic_last_error(void);

/* Pusher microbenchmark (Sec. 2, first paragraph: the modified Lorentz-force
 * pusher against the Boris pusher).  n particles, each in its own uniform
 * field E = (Ex[p], 0, 0) and the common B, advanced nsteps steps of dt with
 * positions kept as an int32 cell plus an offset in [0,1) on a unit grid.
 * All arrays are caller-owned device memory, SoA:
 *   Ex[n]; u[3n] = ux|uy|uz; cell[3n] = cx|cy|cz; off[3n] = ox|oy|oz,
 * of float (PIC_FP32_SPLIT; the gamma solve still runs in FP64) or double
 * (PIC_FP64).  One kernel launch per step on hip_stream; asynchronous. */
pic_status pic_push_bench(int precision, int pusher, int64_t n, int nsteps, double dt,
                          const double B[3], void* Ex, void* u, int32_t* cell, void* off,
                          void* hip_stream);

/* Streaming copy of nbytes (a multiple of 16) from src to dst, both
 * caller-owned, 16-byte aligned, non-overlapping device buffers: one kernel
 * that reads and writes each byte once, the reference of known traffic for
 * calibrating hardware memory counters.  Asynchronous on hip_stream. */
pic_status pic_copy_bench(const void* src, void* dst, int64_t nbytes, void* hip_stream);

/* The HBM bandwidth a kernel can reach on this device, the practical
 * ceiling beside the peak: mode 0 copies nbytes from src to dst, mode 1 only
 * reads src (dst receives at most one word), mode 2 only writes dst (src is
 * not read and may be NULL).  Each thread moves eight 16-byte words per
 * iteration with non-temporal loads and stores.  nbytes a multiple of 16,
 * caller-owned 16-byte aligned device buffers that do not overlap; PIC_EINVAL
 * otherwise.  Asynchronous on hip_stream (time it with events there). */
pic_status pic_stream_bench(int mode, const void* src, void* dst, int64_t nbytes, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif
