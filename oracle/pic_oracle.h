/*
 * Plain, slow FP64 CPU oracle for the boosted-frame electromagnetic
 * particle-in-cell step (Vay et al., "Speeding up simulations of relativistic
 * systems using an optimal boosted frame", 2009).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the GPU library; the only thing the two sides
 * have in common is the seeded workload description they are both given.
 *
 * Every routine is written as plain loops over particles and grid points in
 * double precision, in the order the method defines:
 *   - the laboratory -> boosted frame transform of laser and plasma inputs
 *     (Sec. 2, the paragraph on inputs specified in the laboratory frame);
 *   - the field gather, the pusher with the modified Lorentz-force form and an
 *     analytic solution of its implicit gamma (Sec. 2, first paragraph;
 *     Vay 2008), the Boris pusher as the control it replaces;
 *   - charge-conserving current deposition (Esirkepov 2001, linear shape);
 *   - the Yee field update with first-order Mur boundaries at the open z ends.
 * Where the paper is silent, the choice made is stated at the routine that
 * makes it.
 *
 * Conventions: lengths in c/omega_p, times in 1/omega_p, c = eps0 = 1,
 * electron charge -1 and mass 1, laboratory plasma density 1.  Grid index
 * order is (k, i, j) = (z, x, y), z fastest in memory.  Vector quantities
 * (E, B, u) are ordered (x, y, z).
 */
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORA_BC_OPEN = 0, ORA_BC_PERIODIC = 1 };
enum { ORA_VAY = 0, ORA_BORIS = 1 };
/* field component ids */
enum { ORA_EX = 0, ORA_EY, ORA_EZ, ORA_BX, ORA_BY, ORA_BZ, ORA_JX, ORA_JY, ORA_JZ };

typedef struct {
  int dims;              /* 2 (z,x with 3 velocity components) or 3 (z,x,y) */
  int nz, nx, ny;        /* boosted-frame cells; ny = 1 in 2D */
  double dz, dx, dy;     /* cell sizes, c/omega_p */
  double cfl;            /* dt = cfl / sqrt(sum 1/d^2) */
  int ppc;               /* electrons per cell */
  uint64_t seed;
  double gamma_boost;    /* Lorentz factor of the boosted frame */
  double n_lab_cm3;      /* laboratory plasma density (sets omega_p) */
  double u_th;           /* laboratory thermal momentum spread per component */
  double a0, lambda0_um; /* laser strength and laboratory wavelength */
  double waist;          /* transverse 1/e field radius, c/omega_p */
  double tau_lab;        /* laboratory envelope e-fold length; <= 0: box/8 rule */
  int pol_axis;          /* 1 = x, 2 = y */
  int bc_z;              /* ORA_BC_OPEN or ORA_BC_PERIODIC */
  int pusher;            /* ORA_VAY or ORA_BORIS */
  int inject_every;      /* plasma columns are created every this many steps */
  int round_f32;         /* round created offsets and momenta to FP32 */
  int filter_passes;     /* passes of the 1-2-1 current filter per axis (0: none) */
  int filter_compensate; /* 1: one compensating pass per axis after them */
  /* laboratory-frame stations: planes z_lab = station_z0 + s station_dz,
   * s < n_stations, sampled every step while inside the box, transverse
   * stride station_stride, at most station_cap samples each */
  int n_stations;
  double station_z0, station_dz;
  int station_stride, station_cap;
  /* laser source: 0 = the pulse is placed in the box at t' = 0; 1 = it is
   * emitted by an antenna, the lab plane z = antenna_z_lab, whose envelope
   * peak crosses it at lab time antenna_t_peak */
  int laser_antenna;
  double antenna_z_lab, antenna_t_peak;
} ora_params;

typedef struct {
  double dt, beta_b, gamma_b, dminus, dplus;
  double skin_um;        /* c/omega_p in micrometres */
  double k0_lab;         /* laser wavenumber, lab frame */
  double E0_lab;         /* a0 * omega0 */
  double L_lab, L_boost; /* envelope e-fold lengths */
  double zc_boost;       /* pulse centre in the boosted frame at t'=0 */
  double weight;         /* macro-particle weight */
  double dV;
  int reservoir;         /* cells of plasma reservoir beyond z_max (open z) */
  int nzf;               /* z extent of the field arrays */
} ora_derived;

typedef struct {
  int64_t step;
  double t;
  double U_E, U_B;       /* field energies over interior points */
  double Ez_max;         /* max |E_z| over interior points (wake amplitude) */
  double KE;             /* kinetic energy of interior electrons */
  int64_t n_particles;   /* electrons inside the physical box */
  double gauss_drift;    /* max |(divE-rho)^n - (divE-rho)^0| / max|rho_e^0| */
} ora_diag_out;

typedef struct ora_state ora_state;

/* lifetime */
ora_state* ora_create(const ora_params* p);
void ora_destroy(ora_state* s);
void ora_get_derived(const ora_state* s, ora_derived* d);

/* advance nsteps full PIC steps; when cont_max is non-NULL every step also
 * measures the discrete continuity residual and keeps the maximum there. */
void ora_step(ora_state* s, int nsteps, double* cont_max);
void ora_diag(const ora_state* s, ora_diag_out* out);

/* state access (arrays owned by the state) */
int64_t ora_num_particles(const ora_state* s);
void ora_get_particles(const ora_state* s, double* z, double* x, double* y,
                       double* ux, double* uy, double* uz, uint32_t* id);
void ora_set_particles(ora_state* s, int64_t n, const double* z, const double* x,
                       const double* y, const double* ux, const double* uy,
                       const double* uz, const uint32_t* id);
double* ora_field(ora_state* s, int comp);           /* [ny][nx][nzf] */
int64_t ora_field_points(const ora_state* s);
void ora_reset_gauss_reference(ora_state* s);        /* re-take (divE-rho)^0 */
int64_t ora_step_index(const ora_state* s);

/* building blocks exposed for the physics pins */
void ora_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
void ora_push_vay(double u[3], const double E[3], const double B[3], double eps);
void ora_push_boris(double u[3], const double E[3], const double B[3], double eps);
void ora_boost_fields(double beta, const double E[3], const double B[3],
                      double Eo[3], double Bo[3]);
void ora_boost_momentum(double beta, const double u[3], double uo[3]);
void ora_gather(const ora_state* s, double z, double x, double y,
                double E[3], double B[3]);
void ora_deposit(ora_state* s, const double p0[3], const double p1[3], double vy);
void ora_rho(const ora_state* s, double* rho);        /* electron charge, nodes */
void ora_field_half_B(ora_state* s);                  /* B -= dt/2 curl E (no antenna) */
void ora_field_full_E(ora_state* s);                  /* E += dt (curl B - J - J_antenna) */
/* Station s's record: *count = samples taken (also those beyond the
 * capacity, which are dropped); times[t] = laboratory time of sample t;
 * data holds, per sample, the six laboratory-frame components
 * Ex Ey Ez Bx By Bz, each on the [ny/stride][nx/stride] transverse points
 * (i stride, j stride) of the component's own transverse stagger. */
void ora_station(const ora_state* s, int station, int64_t* count, const double** times,
                 const double** data);
/* low-pass filter of the current as configured (filter_passes,
 * filter_compensate), applied by ora_step between the deposit and the field
 * update; exposed for its pins */
void ora_filter_current(ora_state* s);
/* the same filter on a node-centred scalar array (rho), npts values */
void ora_filter_nodes(const ora_state* s, double* a);
void ora_laser_lab(const ora_state* s, double z, double t, double x, double y,
                   double E[3], double B[3]);

/* pusher microbenchmark: n particles, each in its own uniform field, advanced
 * nsteps with positions integrated on a unit grid (positions as doubles). */
void ora_push_many(int64_t n, double* u /*3n*/, const double* E /*3n*/,
                   const double* B /*3n*/, double* pos /*3n*/, double dt,
                   int nsteps, int pusher);

#ifdef __cplusplus
}
#endif
#endif
