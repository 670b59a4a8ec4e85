/*
 * Plain FP64 CPU oracle for the boosted-frame EM-PIC step.  TEST
 * INFRASTRUCTURE ONLY (tests, smoke check, CPU-baseline timing); see
 * pic_oracle.h for the conventions.  Nothing here is tuned: every stage is a
 * direct loop written in the order the method defines it.
 */
#include "pic_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* CODATA 2018 constants (SI), used only to turn the laboratory density and
 * wavelength into plasma units. */
#define ORA_C 299792458.0
#define ORA_QE 1.602176634e-19
#define ORA_EPS0 8.8541878128e-12
#define ORA_ME 9.1093837015e-31
#define ORA_PI 3.14159265358979323846

struct ora_state {
  ora_params p;
  ora_derived d;
  int64_t npts;
  double* F[9];       /* Ex Ey Ez Bx By Bz Jx Jy Jz at integer time n */
  double* G0;         /* (div E - rho) at the reference time, nodes */
  double rho0_max;    /* max |rho_e| at the reference time (interior) */
  int64_t np, cap;
  double *pz, *px, *py, *ux, *uy, *uz;
  uint32_t* id;
  int64_t next_col;
  int64_t step;
  /* laboratory-frame stations */
  double* st_data;    /* [station][sample][comp][ny/stride][nx/stride] */
  double* st_time;    /* [station][sample] */
  int64_t* st_count;  /* [station] */
};

/* Yee staggering per component: half-cell shift flags in (z, x, y).
 * E_x(i+1/2,j,k) E_y(i,j+1/2,k) E_z(i,j,k+1/2)
 * B_x(i,j+1/2,k+1/2) B_y(i+1/2,j,k+1/2) B_z(i+1/2,j+1/2,k); J like E.
 * In 2D (z,x) the y flags are dropped. */
static const int STAG[9][3] = {
    {0, 1, 0}, {0, 0, 1}, {1, 0, 0}, /* Ex Ey Ez */
    {1, 0, 1}, {1, 1, 0}, {0, 1, 1}, /* Bx By Bz */
    {0, 1, 0}, {0, 0, 1}, {1, 0, 0}, /* Jx Jy Jz */
};

/* ------------------------------------------------------------------------ */
/* small vector helpers                                                     */
static double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void cross3(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static int wrapi(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}
static double hat(double t) { /* linear (cloud-in-cell) particle shape */
  double a = fabs(t);
  return a < 1.0 ? 1.0 - a : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
 * 64x64->128 multiply/xor network with the published multipliers and Weyl
 * key increments. */
void ora_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    unsigned __int128 p0 = (unsigned __int128)M0 * c0;
    unsigned __int128 p1 = (unsigned __int128)M1 * c2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static double u01(uint64_t r) { /* 53-bit uniform in [0,1) */
  return (double)(r >> 11) * (1.0 / 9007199254740992.0);
}

/* ------------------------------------------------------------------------ */
/* Lorentz transforms for a frame moving at +beta along z (c = 1).
 * Parallel components are unchanged; perpendicular ones mix:
 *   E'_perp = gamma (E + beta z x B)_perp,  B'_perp = gamma (B - beta z x E)_perp */
void ora_boost_fields(double beta, const double E[3], const double B[3],
                      double Eo[3], double Bo[3]) {
  double g = 1.0 / sqrt(1.0 - beta * beta);
  double e0 = g * (E[0] - beta * B[1]);
  double e1 = g * (E[1] + beta * B[0]);
  double b0 = g * (B[0] + beta * E[1]);
  double b1 = g * (B[1] - beta * E[0]);
  Eo[0] = e0; Eo[1] = e1; Eo[2] = E[2];
  Bo[0] = b0; Bo[1] = b1; Bo[2] = B[2];
}

/* four-momentum: u'_z = gamma_b (u_z - beta_b gamma), u'_perp = u_perp */
void ora_boost_momentum(double beta, const double u[3], double uo[3]) {
  double gb = 1.0 / sqrt(1.0 - beta * beta);
  double g = sqrt(1.0 + dot3(u, u));
  uo[0] = u[0];
  uo[1] = u[1];
  uo[2] = gb * (u[2] - beta * g);
}

/* ------------------------------------------------------------------------ */
/* Pushers.  eps = q dt / (2 m).  u holds u^{n-1/2} on entry, u^{n+1/2} on exit. */

/* Vay (2008): the Lorentz force uses the average of the old and new velocity
 * in v x B; the resulting implicit equation for the new gamma is solved in
 * closed form. */
void ora_push_vay(double u[3], const double E[3], const double B[3], double eps) {
  double g = sqrt(1.0 + dot3(u, u));
  double v[3] = {u[0] / g, u[1] / g, u[2] / g};
  double vxb[3];
  cross3(v, B, vxb);
  double uh[3], up[3], tau[3];
  for (int a = 0; a < 3; ++a) {
    uh[a] = u[a] + eps * (E[a] + vxb[a]); /* half acceleration with old v */
    up[a] = uh[a] + eps * E[a];           /* u' */
    tau[a] = eps * B[a];
  }
  double ustar = dot3(up, tau);
  double tau2 = dot3(tau, tau);
  double sigma = 1.0 + dot3(up, up) - tau2; /* gamma'^2 - tau^2 */
  double a4 = 4.0 * (tau2 + ustar * ustar);
  double disc = sqrt(sigma * sigma + a4);
  double g2 = (sigma >= 0.0) ? 0.5 * (sigma + disc) : 0.5 * a4 / (disc - sigma);
  double gn = sqrt(g2);
  double t[3] = {tau[0] / gn, tau[1] / gn, tau[2] / gn};
  double s = 1.0 / (1.0 + dot3(t, t));
  double upt = dot3(up, t);
  double c[3];
  cross3(up, t, c);
  for (int a = 0; a < 3; ++a) u[a] = s * (up[a] + upt * t[a] + c[a]);
}

/* Boris (1970): half electric kick, magnetic rotation at the mid-step
 * gamma, half electric kick. */
void ora_push_boris(double u[3], const double E[3], const double B[3], double eps) {
  double um[3];
  for (int a = 0; a < 3; ++a) um[a] = u[a] + eps * E[a];
  double gm = sqrt(1.0 + dot3(um, um));
  double t[3] = {eps * B[0] / gm, eps * B[1] / gm, eps * B[2] / gm};
  double c[3], upp[3];
  cross3(um, t, c);
  for (int a = 0; a < 3; ++a) upp[a] = um[a] + c[a];
  double f = 2.0 / (1.0 + dot3(t, t));
  double st[3] = {f * t[0], f * t[1], f * t[2]};
  double c2[3];
  cross3(upp, st, c2);
  for (int a = 0; a < 3; ++a) u[a] = um[a] + c2[a] + eps * E[a];
}

void ora_push_many(int64_t n, double* u, const double* E, const double* B,
                   double* pos, double dt, int nsteps, int pusher) {
  double eps = -0.5 * dt; /* electron: q/m = -1 */
  for (int64_t p = 0; p < n; ++p) {
    double* up = u + 3 * p;
    for (int s = 0; s < nsteps; ++s) {
      if (pusher == ORA_BORIS)
        ora_push_boris(up, E + 3 * p, B + 3 * p, eps);
      else
        ora_push_vay(up, E + 3 * p, B + 3 * p, eps);
      double g = sqrt(1.0 + dot3(up, up));
      for (int a = 0; a < 3; ++a) pos[3 * p + a] += dt * up[a] / g;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* grid access                                                              */
static int64_t gidx(const ora_state* s, int k, int i, int j) {
  return ((int64_t)j * s->p.nx + i) * s->d.nzf + k;
}
static int zvalid_count(const ora_state* s, int comp) {
  if (s->p.bc_z == ORA_BC_PERIODIC) return s->p.nz;
  return STAG[comp][0] ? s->p.nz : s->p.nz + 1;
}
/* value of component comp at integer index (k,i,j); zero outside the open z
 * range, periodic wrap in x, y (and z when periodic). */
static double fval(const ora_state* s, int comp, int k, int i, int j) {
  i = wrapi(i, s->p.nx);
  j = wrapi(j, s->p.ny);
  if (s->p.bc_z == ORA_BC_PERIODIC)
    k = wrapi(k, s->p.nz);
  else if (k < 0 || k >= zvalid_count(s, comp))
    return 0.0;
  return s->F[comp][gidx(s, k, i, j)];
}
static void fadd(ora_state* s, int comp, int k, int i, int j, double v) {
  i = wrapi(i, s->p.nx);
  j = wrapi(j, s->p.ny);
  if (s->p.bc_z == ORA_BC_PERIODIC)
    k = wrapi(k, s->p.nz);
  else if (k < 0 || k >= zvalid_count(s, comp))
    return; /* current outside the box is discarded */
  s->F[comp][gidx(s, k, i, j)] += v;
}

/* ------------------------------------------------------------------------ */
/* Field gather: every component is linearly interpolated from its own
 * staggered location (cloud-in-cell in each dimension). */
static double interp(const ora_state* s, int comp, double z, double x, double y) {
  double xz = z / s->p.dz - 0.5 * STAG[comp][0];
  double xx = x / s->p.dx - 0.5 * STAG[comp][1];
  int kz = (int)floor(xz), kx = (int)floor(xx);
  double fz = xz - kz, fx = xx - kx;
  double wz[2] = {1.0 - fz, fz}, wx[2] = {1.0 - fx, fx};
  double acc = 0.0;
  if (s->p.dims == 3) {
    double xy = y / s->p.dy - 0.5 * STAG[comp][2];
    int ky = (int)floor(xy);
    double fy = xy - ky;
    double wy[2] = {1.0 - fy, fy};
    for (int c = 0; c < 2; ++c)
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a)
          acc += wz[a] * wx[b] * wy[c] * fval(s, comp, kz + a, kx + b, ky + c);
  } else {
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a)
        acc += wz[a] * wx[b] * fval(s, comp, kz + a, kx + b, 0);
  }
  return acc;
}

void ora_gather(const ora_state* s, double z, double x, double y, double E[3], double B[3]) {
  E[0] = interp(s, ORA_EX, z, x, y);
  E[1] = interp(s, ORA_EY, z, x, y);
  E[2] = interp(s, ORA_EZ, z, x, y);
  B[0] = interp(s, ORA_BX, z, x, y);
  B[1] = interp(s, ORA_BY, z, x, y);
  B[2] = interp(s, ORA_BZ, z, x, y);
}

/* ------------------------------------------------------------------------ */
/* Esirkepov (2001) charge-conserving deposit with the linear shape.
 * p0, p1 = old/new positions (z, x, y), unwrapped.  vy is the out-of-plane
 * velocity used by the 2D J_y term. */
void ora_deposit(ora_state* s, const double p0[3], const double p1[3], double vy) {
  const double dt = s->d.dt;
  const double qw = -s->d.weight; /* electron charge times weight */
  const double del[3] = {s->p.dz, s->p.dx, s->p.dy};
  const int nd = s->p.dims;
  int m[3] = {0, 0, 0};
  double S0[3][3] = {{0}}, DS[3][3] = {{0}};
  for (int d = 0; d < nd; ++d) {
    double a0 = p0[d] / del[d], a1 = p1[d] / del[d];
    int i0 = (int)floor(a0), i1 = (int)floor(a1);
    m[d] = i0 < i1 ? i0 : i1;
    for (int a = 0; a < 3; ++a) {
      double s0 = hat(a0 - (m[d] + a));
      double s1 = hat(a1 - (m[d] + a));
      S0[d][a] = s0;
      DS[d][a] = s1 - s0;
    }
  }
  enum { Z = 0, X = 1, Y = 2 };
  if (nd == 3) {
    /* W_z(a,b,c) = DS_z(a) (S0_x S0_y + DS_x S0_y/2 + S0_x DS_y/2 + DS_x DS_y/3)
     * and cyclic; J along d is the running sum of W_d along d. */
    double W[3][3][3][3]; /* [dim][a_z][b_x][c_y] */
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        for (int c = 0; c < 3; ++c) {
          double sz = S0[Z][a], dz = DS[Z][a];
          double sx = S0[X][b], dx = DS[X][b];
          double sy = S0[Y][c], dy = DS[Y][c];
          W[Z][a][b][c] = dz * (sx * sy + 0.5 * dx * sy + 0.5 * sx * dy + dx * dy / 3.0);
          W[X][a][b][c] = dx * (sz * sy + 0.5 * dz * sy + 0.5 * sz * dy + dz * dy / 3.0);
          W[Y][a][b][c] = dy * (sz * sx + 0.5 * dz * sx + 0.5 * sz * dx + dz * dx / 3.0);
        }
    double cz = -qw / (del[X] * del[Y] * dt);
    double cx = -qw / (del[Z] * del[Y] * dt);
    double cy = -qw / (del[Z] * del[X] * dt);
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c) {
        double run = 0.0;
        for (int a = 0; a < 3; ++a) {
          run += W[Z][a][b][c];
          fadd(s, ORA_JZ, m[Z] + a, m[X] + b, m[Y] + c, cz * run);
        }
      }
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) {
        double run = 0.0;
        for (int b = 0; b < 3; ++b) {
          run += W[X][a][b][c];
          fadd(s, ORA_JX, m[Z] + a, m[X] + b, m[Y] + c, cx * run);
        }
      }
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double run = 0.0;
        for (int c = 0; c < 3; ++c) {
          run += W[Y][a][b][c];
          fadd(s, ORA_JY, m[Z] + a, m[X] + b, m[Y] + c, cy * run);
        }
      }
  } else {
    /* 2D3V: W_z = DS_z (S0_x + DS_x/2), W_x = DS_x (S0_z + DS_z/2);
     * J_y uses the time-averaged shape times v_y. */
    double cz = -qw / (del[X] * dt);
    double cx = -qw / (del[Z] * dt);
    double cyv = qw * vy / (del[Z] * del[X]);
    for (int b = 0; b < 3; ++b) {
      double run = 0.0;
      for (int a = 0; a < 3; ++a) {
        run += DS[Z][a] * (S0[X][b] + 0.5 * DS[X][b]);
        fadd(s, ORA_JZ, m[Z] + a, m[X] + b, 0, cz * run);
      }
    }
    for (int a = 0; a < 3; ++a) {
      double run = 0.0;
      for (int b = 0; b < 3; ++b) {
        run += DS[X][b] * (S0[Z][a] + 0.5 * DS[Z][a]);
        fadd(s, ORA_JX, m[Z] + a, m[X] + b, 0, cx * run);
      }
    }
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double sz = S0[Z][a], dz = DS[Z][a], sx = S0[X][b], dx = DS[X][b];
        double sh = sz * sx + 0.5 * dz * sx + 0.5 * sz * dx + dz * dx / 3.0;
        fadd(s, ORA_JY, m[Z] + a, m[X] + b, 0, cyv * sh);
      }
  }
}

/* electron charge density on grid nodes (linear shape) */
void ora_rho(const ora_state* s, double* rho) {
  const double qw = -s->d.weight;
  const double inv_dv = 1.0 / s->d.dV;
  memset(rho, 0, sizeof(double) * s->npts);
  for (int64_t p = 0; p < s->np; ++p) {
    double az = s->pz[p] / s->p.dz, ax = s->px[p] / s->p.dx;
    int kz = (int)floor(az), kx = (int)floor(ax);
    double fz = az - kz, fx = ax - kx;
    double wz[2] = {1 - fz, fz}, wx[2] = {1 - fx, fx};
    int ncy = s->p.dims == 3 ? 2 : 1;
    double wy[2] = {1.0, 0.0};
    int ky = 0;
    if (s->p.dims == 3) {
      double ay = s->py[p] / s->p.dy;
      ky = (int)floor(ay);
      double fy = ay - ky;
      wy[0] = 1 - fy;
      wy[1] = fy;
    }
    for (int c = 0; c < ncy; ++c)
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
          int k = kz + a, i = wrapi(kx + b, s->p.nx), j = wrapi(ky + c, s->p.ny);
          if (s->p.bc_z == ORA_BC_PERIODIC)
            k = wrapi(k, s->p.nz);
          else if (k < 0 || k > s->p.nz)
            continue;
          rho[gidx(s, k, i, j)] += qw * wz[a] * wx[b] * wy[c] * inv_dv;
        }
  }
}

/* ------------------------------------------------------------------------ */
/* Yee update.  Curls are centred differences on the staggered grid.        */
static int zlimit(const ora_state* s, int comp) { return zvalid_count(s, comp); }

/* B -= dt/2 curl E  (one half step) */
/* ------------------------------------------------------------------------ */
/* Laser antenna (Sec. 2, second paragraph): the pulse enters through a    */
/* plane at rest in the laboratory, moving at -beta_b in the boosted frame. */
/* The lab plane z = Z_a sits at z'_a(t') = Z_a / gamma_b - beta_b t'.     */
/* Wanted: the boosted incident wave (E_i, B_i) above the plane   */
/* and nothing below, i.e. the field H (E_i, B_i) with H(z', t') = 1 where  */
/* z' > z'_a(t'), else 0.  In the continuum the step's derivatives leave    */
/* surface sources on the plane (an electric current J and a magnetic       */
/* current M in dB/dt = -curl E - M).  On the grid they are taken as what   */
/* the discrete update needs to carry H (E_i, B_i) from one time level to   */
/* the next:                                                                */
/*   J^{n+1/2} = curl_h (H B_i)^{n+1/2} - ((H E_i)^{n+1} - (H E_i)^n) / dt, */
/*   M^n = -curl_h (H E_i)^n - ((H B_i)^{n+1/2} - (H B_i)^{n-1/2}) / dt,    */
/* with curl_h the Yee differences of the field update, each point's H at   */
/* its own staggered z and time, and the source kept only at points whose   */
/* update involves both sides of the plane (elsewhere it is zero: above the */
/* plane the field evolves by the Yee update alone).  This is exact for any */
/* speed of the plane, where spreading a moving delta over the grid is not. */
/* The incident wave is the lab pulse evaluated at the lab event of each    */
/* grid point and boosted.  The antenna acts at level n while              */
/* 2 dz <= z'_a(n dt) < (nz - 2) dz; at t' = 0 the box holds H (E_i, B_i).  */
static double antenna_z(const ora_state* s, double t) {
  return s->p.antenna_z_lab / s->d.gamma_b - s->d.beta_b * t;
}

/* H times the incident boosted field, component comp at its point (k, i, j)
 * at boosted time t; *hmin / *hmax track the H values seen */
static double hinc(const ora_state* s, int comp, int k, int i, int j, double t, int* hmin, int* hmax) {
  const double z = (k + 0.5 * STAG[comp][0]) * s->p.dz;
  const int h = z > antenna_z(s, t) ? 1 : 0;
  if (h < *hmin) *hmin = h;
  if (h > *hmax) *hmax = h;
  if (!h) return 0.0;
  i = wrapi(i, s->p.nx);
  j = s->p.dims == 3 ? wrapi(j, s->p.ny) : 0;
  const double x = (i + 0.5 * STAG[comp][1]) * s->p.dx;
  const double y = s->p.dims == 3 ? (j + 0.5 * STAG[comp][2]) * s->p.dy : 0.0;
  double El[3], Bl[3], Ei[3], Bi[3];
  ora_laser_lab(s, s->d.gamma_b * (z + s->d.beta_b * t), s->d.gamma_b * (t + s->d.beta_b * z), x, y, El, Bl);
  ora_boost_fields(s->d.beta_b, El, Bl, Ei, Bi);
  return comp < 3 ? Ei[comp] : Bi[comp - 3];
}

static int antenna_on(const ora_state* s, int64_t n) {
  if (!s->p.laser_antenna || s->p.a0 == 0.0) return 0;
  const double za = antenna_z(s, n * s->d.dt);
  return za >= 2.0 * s->p.dz && za < (s->p.nz - 2) * s->p.dz;
}

/* J^{n+1/2} (comp = ORA_EX..EZ) or M^n (comp = ORA_BX..BZ) at (k, i, j);
 * *straddle (if given) tells whether the point's update involves both sides */
static double antenna_source_s(const ora_state* s, int comp, int64_t n, int k, int i, int j, int* straddle) {
  if (straddle) *straddle = 0;
  if (!antenna_on(s, n)) return 0.0;
  const double dt = s->d.dt;
  const double z = (k + 0.5 * STAG[comp][0]) * s->p.dz;
  if (fabs(z - antenna_z(s, n * dt)) > 3.0 * s->p.dz) return 0.0; /* cannot straddle */
  const double idz = 1.0 / s->p.dz, idx = 1.0 / s->p.dx;
  const double idy = s->p.dims == 3 ? 1.0 / s->p.dy : 0.0;
  int lo = 1, hi = 0;
  double r;
  if (comp <= ORA_EZ) {
    const double th = (n + 0.5) * dt, t0 = n * dt, t1 = (n + 1) * dt;
    double curl;
    if (comp == ORA_EX)
      curl = (hinc(s, ORA_BZ, k, i, j, th, &lo, &hi) - hinc(s, ORA_BZ, k, i, j - 1, th, &lo, &hi)) * idy -
             (hinc(s, ORA_BY, k, i, j, th, &lo, &hi) - hinc(s, ORA_BY, k - 1, i, j, th, &lo, &hi)) * idz;
    else if (comp == ORA_EY)
      curl = (hinc(s, ORA_BX, k, i, j, th, &lo, &hi) - hinc(s, ORA_BX, k - 1, i, j, th, &lo, &hi)) * idz -
             (hinc(s, ORA_BZ, k, i, j, th, &lo, &hi) - hinc(s, ORA_BZ, k, i - 1, j, th, &lo, &hi)) * idx;
    else
      curl = (hinc(s, ORA_BY, k, i, j, th, &lo, &hi) - hinc(s, ORA_BY, k, i - 1, j, th, &lo, &hi)) * idx -
             (hinc(s, ORA_BX, k, i, j, th, &lo, &hi) - hinc(s, ORA_BX, k, i, j - 1, th, &lo, &hi)) * idy;
    const double e1 = hinc(s, comp, k, i, j, t1, &lo, &hi), e0 = hinc(s, comp, k, i, j, t0, &lo, &hi);
    r = curl - (e1 - e0) / dt;
  } else {
    const double t0 = n * dt, tm = (n - 0.5) * dt, tq = (n + 0.5) * dt;
    double curl;
    if (comp == ORA_BX)
      curl = (hinc(s, ORA_EZ, k, i, j + 1, t0, &lo, &hi) - hinc(s, ORA_EZ, k, i, j, t0, &lo, &hi)) * idy -
             (hinc(s, ORA_EY, k + 1, i, j, t0, &lo, &hi) - hinc(s, ORA_EY, k, i, j, t0, &lo, &hi)) * idz;
    else if (comp == ORA_BY)
      curl = (hinc(s, ORA_EX, k + 1, i, j, t0, &lo, &hi) - hinc(s, ORA_EX, k, i, j, t0, &lo, &hi)) * idz -
             (hinc(s, ORA_EZ, k, i + 1, j, t0, &lo, &hi) - hinc(s, ORA_EZ, k, i, j, t0, &lo, &hi)) * idx;
    else
      curl = (hinc(s, ORA_EY, k, i + 1, j, t0, &lo, &hi) - hinc(s, ORA_EY, k, i, j, t0, &lo, &hi)) * idx -
             (hinc(s, ORA_EX, k, i, j + 1, t0, &lo, &hi) - hinc(s, ORA_EX, k, i, j, t0, &lo, &hi)) * idy;
    const double b1 = hinc(s, comp, k, i, j, tq, &lo, &hi), b0 = hinc(s, comp, k, i, j, tm, &lo, &hi);
    r = -curl - (b1 - b0) / dt;
  }
  if (straddle) *straddle = lo != hi;
  return lo != hi ? r : 0.0;
}

static double antenna_source(const ora_state* s, int comp, int64_t n, int k, int i, int j) {
  return antenna_source_s(s, comp, n, k, i, j, NULL);
}

/* B -= dt/2 curl E, and, with_m set, dt M^lev (the antenna's whole
 * magnetic current of level lev enters the first half step after it, so that
 * B at integer time is B^{n-1/2} - dt/2 curl E^n, as the gather sees it) */
static void half_B(ora_state* s, int64_t lev, int with_m) {
  const double h = 0.5 * s->d.dt;
  const double idz = 1.0 / s->p.dz, idx = 1.0 / s->p.dx;
  const double idy = s->p.dims == 3 ? 1.0 / s->p.dy : 0.0;
  const int nx = s->p.nx, ny = s->p.ny;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      for (int k = 0; k < zlimit(s, ORA_BX); ++k) { /* Bx at (i, j+1/2, k+1/2) */
        double curl = (fval(s, ORA_EZ, k, i, j + 1) - fval(s, ORA_EZ, k, i, j)) * idy -
                      (fval(s, ORA_EY, k + 1, i, j) - fval(s, ORA_EY, k, i, j)) * idz;
        s->F[ORA_BX][gidx(s, k, i, j)] -= h * curl + (with_m ? 2.0 * h * antenna_source(s, ORA_BX, lev, k, i, j) : 0.0);
      }
      for (int k = 0; k < zlimit(s, ORA_BY); ++k) { /* By at (i+1/2, j, k+1/2) */
        double curl = (fval(s, ORA_EX, k + 1, i, j) - fval(s, ORA_EX, k, i, j)) * idz -
                      (fval(s, ORA_EZ, k, i + 1, j) - fval(s, ORA_EZ, k, i, j)) * idx;
        s->F[ORA_BY][gidx(s, k, i, j)] -= h * curl + (with_m ? 2.0 * h * antenna_source(s, ORA_BY, lev, k, i, j) : 0.0);
      }
      for (int k = 0; k < zlimit(s, ORA_BZ); ++k) { /* Bz at (i+1/2, j+1/2, k) */
        double curl = (fval(s, ORA_EY, k, i + 1, j) - fval(s, ORA_EY, k, i, j)) * idx -
                      (fval(s, ORA_EX, k, i, j + 1) - fval(s, ORA_EX, k, i, j)) * idy;
        s->F[ORA_BZ][gidx(s, k, i, j)] -= h * curl + (with_m ? 2.0 * h * antenna_source(s, ORA_BZ, lev, k, i, j) : 0.0);
      }
    }
}

/* half step of B (Yee only, no antenna source) */
void ora_field_half_B(ora_state* s) { half_B(s, s->step, 0); }

/* E += dt (curl B - J - J_ion - J_antenna^{lev+1/2}); first-order Mur on the
 * tangential E at the open z ends. */
static void full_E(ora_state* s, int64_t lev) {
  const double dt = s->d.dt;
  const double idz = 1.0 / s->p.dz, idx = 1.0 / s->p.dx;
  const double idy = s->p.dims == 3 ? 1.0 / s->p.dy : 0.0;
  const int nx = s->p.nx, ny = s->p.ny, nz = s->p.nz;
  const int open = s->p.bc_z == ORA_BC_OPEN;
  /* ions at rest in the laboratory: density gamma_b, velocity -beta_b;
   * the background exists only together with the plasma electrons */
  const double jion_z = s->p.ppc > 0 ? -s->d.gamma_b * s->d.beta_b : 0.0;
  /* keep the old tangential E on planes 0, 1, nz-1, nz for Mur */
  int64_t plane = (int64_t)nx * ny;
  double* old = NULL;
  if (open) {
    old = (double*)malloc(sizeof(double) * plane * 8);
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        int64_t q = (int64_t)j * nx + i;
        int ks[4] = {0, 1, nz - 1, nz};
        for (int t = 0; t < 4; ++t) {
          old[(t * 2 + 0) * plane + q] = s->F[ORA_EX][gidx(s, ks[t], i, j)];
          old[(t * 2 + 1) * plane + q] = s->F[ORA_EY][gidx(s, ks[t], i, j)];
        }
      }
  }
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      for (int k = 0; k < zlimit(s, ORA_EX); ++k) { /* Ex at (i+1/2, j, k) */
        if (open && (k == 0 || k == nz)) continue;
        double curl = (fval(s, ORA_BZ, k, i, j) - fval(s, ORA_BZ, k, i, j - 1)) * idy -
                      (fval(s, ORA_BY, k, i, j) - fval(s, ORA_BY, k - 1, i, j)) * idz;
        int64_t g = gidx(s, k, i, j);
        s->F[ORA_EX][g] += dt * (curl - s->F[ORA_JX][g] - antenna_source(s, ORA_EX, lev, k, i, j));
      }
      for (int k = 0; k < zlimit(s, ORA_EY); ++k) { /* Ey at (i, j+1/2, k) */
        if (open && (k == 0 || k == nz)) continue;
        double curl = (fval(s, ORA_BX, k, i, j) - fval(s, ORA_BX, k - 1, i, j)) * idz -
                      (fval(s, ORA_BZ, k, i, j) - fval(s, ORA_BZ, k, i - 1, j)) * idx;
        int64_t g = gidx(s, k, i, j);
        s->F[ORA_EY][g] += dt * (curl - s->F[ORA_JY][g] - antenna_source(s, ORA_EY, lev, k, i, j));
      }
      for (int k = 0; k < zlimit(s, ORA_EZ); ++k) { /* Ez at (i, j, k+1/2) */
        double curl = (fval(s, ORA_BY, k, i, j) - fval(s, ORA_BY, k, i - 1, j)) * idx -
                      (fval(s, ORA_BX, k, i, j) - fval(s, ORA_BX, k, i, j - 1)) * idy;
        int64_t g = gidx(s, k, i, j);
        s->F[ORA_EZ][g] +=
            dt * (curl - s->F[ORA_JZ][g] - jion_z - antenna_source(s, ORA_EZ, lev, k, i, j));
      }
    }
  if (open) {
    /* Mur, first order, normal incidence:
     * E^{n+1}[0] = E^n[1] + (dt-dz)/(dt+dz) (E^{n+1}[1] - E^n[0]) */
    double cm = (dt - s->p.dz) / (dt + s->p.dz);
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        int64_t q = (int64_t)j * nx + i;
        for (int c = 0; c < 2; ++c) {
          int comp = c == 0 ? ORA_EX : ORA_EY;
          double e0 = old[(0 * 2 + c) * plane + q], e1 = old[(1 * 2 + c) * plane + q];
          double en1 = old[(2 * 2 + c) * plane + q], en = old[(3 * 2 + c) * plane + q];
          double n1 = s->F[comp][gidx(s, 1, i, j)];
          double nn1 = s->F[comp][gidx(s, nz - 1, i, j)];
          s->F[comp][gidx(s, 0, i, j)] = e1 + cm * (n1 - e0);
          s->F[comp][gidx(s, nz, i, j)] = en1 + cm * (nn1 - en);
        }
      }
    free(old);
  }
}

/* full E step from the current step (the antenna's J^{step+1/2}) */
void ora_field_full_E(ora_state* s) { full_E(s, s->step); }

/* ------------------------------------------------------------------------ */
/* laboratory laser: flat phase fronts, Gaussian transverse profile and
 * envelope, travelling along +z; B = z x E.  Placed in the box, its centre is
 * at z = zc_boost / D+ at t = 0 (so that at t' = 0 the boosted pulse is
 * centred at zc_boost); emitted by the antenna, the centre crosses the
 * antenna plane at t = antenna_t_peak. */
void ora_laser_lab(const ora_state* s, double z, double t, double x, double y,
                   double E[3], double B[3]) {
  double zeta = s->p.laser_antenna ? z - s->p.antenna_z_lab - (t - s->p.antenna_t_peak)
                                   : z - s->d.dminus * s->d.zc_boost - t;
  double Ll = s->d.L_lab;
  double env = exp(-zeta * zeta / (Ll * Ll)) * cos(s->d.k0_lab * zeta);
  double rx = x - 0.5 * s->p.nx * s->p.dx;
  double r2 = rx * rx;
  if (s->p.dims == 3) {
    double ry = y - 0.5 * s->p.ny * s->p.dy;
    r2 += ry * ry;
  }
  double amp = s->d.E0_lab * exp(-r2 / (s->p.waist * s->p.waist)) * env;
  E[0] = E[1] = E[2] = B[0] = B[1] = B[2] = 0.0;
  if (s->p.pol_axis == 1) {
    E[0] = amp;
    B[1] = amp;
  } else {
    E[1] = amp;
    B[0] = -amp;
  }
}

/* boosted-frame field at (z', x, y), t' = 0: the lab event is
 * z = gamma_b z', t = gamma_b beta_b z'; evaluate there and boost. */
static void laser_boosted(const ora_state* s, double zp, double x, double y,
                          double E[3], double B[3]) {
  double El[3], Bl[3];
  double z = s->d.gamma_b * zp, t = s->d.gamma_b * s->d.beta_b * zp;
  ora_laser_lab(s, z, t, x, y, El, Bl);
  ora_boost_fields(s->d.beta_b, El, Bl, E, B);
}

static void init_fields(ora_state* s) {
  for (int c = 0; c < 9; ++c) memset(s->F[c], 0, sizeof(double) * s->npts);
  if (s->p.a0 == 0.0) return;
  const int nx = s->p.nx, ny = s->p.ny;
  for (int comp = 0; comp < 6; ++comp) {
    int kl = zlimit(s, comp);
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i)
        for (int k = 0; k < kl; ++k) {
          double zp = (k + 0.5 * STAG[comp][0]) * s->p.dz;
          double x = (i + 0.5 * STAG[comp][1]) * s->p.dx;
          double y = s->p.dims == 3 ? (j + 0.5 * STAG[comp][2]) * s->p.dy : 0.0;
          double E[3], B[3];
          laser_boosted(s, zp, x, y, E, B);
          double v = comp < 3 ? E[comp] : B[comp - 3];
          if (s->p.laser_antenna) {
            /* antenna: the box holds the incident wave above the plane only;
             * a B point whose first update straddles the plane starts at
             * (H B_i)^{-1/2} - dt/2 curl_h (H E_i)^0, which equals the mean of
             * H B_i at t' = -dt/2 and dt/2 plus dt/2 M^0, so that the first
             * step of B lands on H B_i at t' = dt/2 */
            int lo = 1, hi = 0, st = 0;
            double m0 = 0.0;
            if (comp >= 3) m0 = antenna_source_s(s, comp, 0, k, i, j, &st);
            if (st) {
              const double h = 0.5 * s->d.dt;
              v = 0.5 * (hinc(s, comp, k, i, j, -h, &lo, &hi) + hinc(s, comp, k, i, j, h, &lo, &hi)) + h * m0;
            } else {
              v = hinc(s, comp, k, i, j, 0.0, &lo, &hi);
            }
          }
          s->F[comp][gidx(s, k, i, j)] = v;
        }
  }
}

/* ------------------------------------------------------------------------ */
/* plasma columns                                                           */
static void ensure_cap(ora_state* s, int64_t need) {
  if (need <= s->cap) return;
  int64_t nc = s->cap ? s->cap : 1024;
  while (nc < need) nc *= 2;
  s->pz = (double*)realloc(s->pz, sizeof(double) * nc);
  s->px = (double*)realloc(s->px, sizeof(double) * nc);
  s->py = (double*)realloc(s->py, sizeof(double) * nc);
  s->ux = (double*)realloc(s->ux, sizeof(double) * nc);
  s->uy = (double*)realloc(s->uy, sizeof(double) * nc);
  s->uz = (double*)realloc(s->uz, sizeof(double) * nc);
  s->id = (uint32_t*)realloc(s->id, sizeof(uint32_t) * nc);
  s->cap = nc;
}

/* position along one axis from a coordinate in cell units; with round_f32
 * the in-cell offset is rounded to FP32 the way split storage keeps it. */
static double place(const ora_state* s, double zeta, double delta) {
  if (!s->p.round_f32) return zeta * delta;
  double c = floor(zeta);
  float o = (float)(zeta - c);
  if (o >= 1.0f) {
    o = 0.0f;
    c += 1.0;
  }
  return (c + (double)o) * delta;
}

/* create lattice columns [k_begin, k_end) at time step n.  Each cell gets
 * ppc electrons at Philox-drawn in-cell positions, with a laboratory
 * Maxwellian momentum (spread u_th) that is then boosted. */
static void create_columns(ora_state* s, int64_t k_begin, int64_t k_end, int64_t n) {
  const int nx = s->p.nx, ny = s->p.ny, ppc = s->p.ppc;
  const int64_t nperp = (int64_t)nx * ny;
  const double shift = s->d.beta_b * ((double)n * s->d.dt) / s->p.dz;
  const uint64_t key[2] = {s->p.seed, 0};
  ensure_cap(s, s->np + (k_end - k_begin) * nperp * ppc);
  for (int64_t K = k_begin; K < k_end; ++K)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i)
        for (int sl = 0; sl < ppc; ++sl) {
          uint64_t L = ((uint64_t)K * nperp + (uint64_t)(i + (int64_t)nx * j)) * ppc + sl;
          uint64_t c0[4] = {L, 0, 0, 0}, c1[4] = {L, 1, 0, 0}, r[4], q[4];
          ora_philox4x64_10(c0, key, r);
          ora_philox4x64_10(c1, key, q);
          double xz = u01(r[0]), xx = u01(r[1]), xy = u01(r[2]);
          /* Box-Muller with 1-U in (0,1] */
          double m0 = sqrt(-2.0 * log(1.0 - u01(r[3])));
          double a0 = 2.0 * ORA_PI * u01(q[0]);
          double m1 = sqrt(-2.0 * log(1.0 - u01(q[1])));
          double a1 = 2.0 * ORA_PI * u01(q[2]);
          double ul[3] = {s->p.u_th * m0 * cos(a0), s->p.u_th * m0 * sin(a0),
                          s->p.u_th * m1 * cos(a1)};
          double ub[3];
          ora_boost_momentum(s->d.beta_b, ul, ub);
          int64_t p = s->np++;
          s->pz[p] = place(s, ((double)K + xz) - shift, s->p.dz);
          s->px[p] = place(s, (double)i + xx, s->p.dx);
          s->py[p] = s->p.dims == 3 ? place(s, (double)j + xy, s->p.dy) : 0.0;
          if (s->p.round_f32) {
            ub[0] = (double)(float)ub[0];
            ub[1] = (double)(float)ub[1];
            ub[2] = (double)(float)ub[2];
          }
          s->ux[p] = ub[0];
          s->uy[p] = ub[1];
          s->uz[p] = ub[2];
          s->id[p] = (uint32_t)L;
        }
}

/* columns K are created at steps n that are multiples of inject_every, for
 * every K with K dz - beta_b t_n < L_z + R dz (open z). */
static void inject(ora_state* s, int64_t n) {
  int64_t kend;
  if (s->p.bc_z == ORA_BC_PERIODIC) {
    kend = s->p.nz;
  } else {
    double shift = s->d.beta_b * ((double)n * s->d.dt) / s->p.dz;
    kend = (int64_t)s->p.nz + s->d.reservoir + (int64_t)ceil(shift);
  }
  if (kend > s->next_col) {
    create_columns(s, s->next_col, kend, n);
    s->next_col = kend;
  }
}

/* ------------------------------------------------------------------------ */
/* Low-pass digital filter of the current (Sec. 2: the short-wavelength     */
/* instability of boosted-frame runs is controlled with low-dispersion      */
/* solvers and low-pass digital filtering; the paper gives no filter, the   */
/* one here is the standard binomial one).  A pass along one axis replaces  */
/* every value by wm a[q] + ws (a[q-1] + a[q+1]) on the component's own     */
/* staggered grid: periodic axes wrap; along an open z axis a value beyond  */
/* the component's range repeats the value at that end of the range, so a  */
/* current that streams uniformly out through an end (the drifting plasma)  */
/* passes unchanged (with zeros beyond the ends, the cut of the end values  */
/* would act as a steady charge source there).  N passes of (1/4,1/2,1/4)   */
/* along each axis have the transfer function cos^2N(theta/2) per axis      */
/* (theta = k * cell); the optional compensating pass (-N/4, 1+N/2, -N/4)   */
/* multiplies it by 1 + N sin^2(theta/2), which restores the long-wave      */
/* response to second order.                                                */
static void filter_pass(const ora_state* s, double* a, int zcount, int axis, double ws, double wm) {
  const int nx = s->p.nx, ny = s->p.ny;
  const int periodic_z = s->p.bc_z == ORA_BC_PERIODIC;
  double* t = (double*)malloc(sizeof(double) * s->npts);
  memcpy(t, a, sizeof(double) * s->npts);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i)
      for (int k = 0; k < zcount; ++k) {
        double lo, hi;
        if (axis == 0) {
          int km = k - 1, kp = k + 1;
          if (periodic_z) {
            km = wrapi(km, s->p.nz);
            kp = wrapi(kp, s->p.nz);
            lo = a[gidx(s, km, i, j)];
            hi = a[gidx(s, kp, i, j)];
          } else {
            lo = a[gidx(s, km >= 0 ? km : k, i, j)];
            hi = a[gidx(s, kp < zcount ? kp : k, i, j)];
          }
        } else if (axis == 1) {
          lo = a[gidx(s, k, wrapi(i - 1, nx), j)];
          hi = a[gidx(s, k, wrapi(i + 1, nx), j)];
        } else {
          lo = a[gidx(s, k, i, wrapi(j - 1, ny))];
          hi = a[gidx(s, k, i, wrapi(j + 1, ny))];
        }
        t[gidx(s, k, i, j)] = wm * a[gidx(s, k, i, j)] + ws * (lo + hi);
      }
  memcpy(a, t, sizeof(double) * s->npts);
  free(t);
}

static void filter_array(const ora_state* s, double* a, int zcount) {
  const int naxes = s->p.dims == 3 ? 3 : 2;
  const int N = s->p.filter_passes;
  for (int n = 0; n < N; ++n)
    for (int ax = 0; ax < naxes; ++ax) filter_pass(s, a, zcount, ax, 0.25, 0.5);
  if (N > 0 && s->p.filter_compensate)
    for (int ax = 0; ax < naxes; ++ax) filter_pass(s, a, zcount, ax, -0.25 * N, 1.0 + 0.5 * N);
}

void ora_filter_current(ora_state* s) {
  for (int c = ORA_JX; c <= ORA_JZ; ++c) filter_array(s, s->F[c], zvalid_count(s, c));
}

void ora_filter_nodes(const ora_state* s, double* a) { filter_array(s, a, zvalid_count(s, ORA_EX)); }

/* ------------------------------------------------------------------------ */
/* Laboratory-frame stations (Sec. 2: quantities are recorded at stations   */
/* immobile in the laboratory, at a succession of times, with interpolation */
/* because lab space-time points do not coincide with the boosted grid).    */
/* A station is the plane z_lab = Z.  At boosted time t' it sits at         */
/* z' = Z / gamma_b - beta_b t' (from z_lab = gamma_b (z' + beta_b t')),    */
/* and the event it samples has lab time t_lab = gamma_b (t' + beta_b z')   */
/* = t' / gamma_b + beta_b Z.  Every step, each station inside [0, L_z)     */
/* records E^n, B^n at its plane: each component linearly interpolated in z */
/* from its own staggered points (zero outside its range), transformed back */
/* to the laboratory frame with the boost of velocity -beta_b.              */
static double zinterp(const ora_state* s, int comp, double z, int i, int j) {
  double u = z / s->p.dz - 0.5 * STAG[comp][0];
  int k = (int)floor(u);
  double f = u - k;
  return (1.0 - f) * fval(s, comp, k, i, j) + f * fval(s, comp, k + 1, i, j);
}

static void record_stations(ora_state* s) {
  const int S = s->p.n_stations, st = s->p.station_stride, T = s->p.station_cap;
  if (S <= 0) return;
  const int nxs = s->p.nx / st, nys = s->p.dims == 3 ? s->p.ny / st : 1;
  const double Lz = s->p.nz * s->p.dz, tp = s->step * s->d.dt;
  for (int q = 0; q < S; ++q) {
    const double Z = s->p.station_z0 + q * s->p.station_dz;
    const double zp = Z / s->d.gamma_b - s->d.beta_b * tp;
    if (!(zp >= 0.0 && zp < Lz)) continue;
    const int64_t t = s->st_count[q]++;
    if (t >= T) continue;
    s->st_time[(int64_t)q * T + t] = tp / s->d.gamma_b + s->d.beta_b * Z;
    double* out = s->st_data + ((int64_t)q * T + t) * 6 * nys * nxs;
    for (int js = 0; js < nys; ++js)
      for (int is = 0; is < nxs; ++is) {
        double Eb[3], Bb[3], El[3], Bl[3];
        for (int c = 0; c < 3; ++c) {
          Eb[c] = zinterp(s, ORA_EX + c, zp, is * st, js * st);
          Bb[c] = zinterp(s, ORA_BX + c, zp, is * st, js * st);
        }
        ora_boost_fields(-s->d.beta_b, Eb, Bb, El, Bl);
        for (int c = 0; c < 3; ++c) {
          out[((int64_t)c * nys + js) * nxs + is] = El[c];
          out[((int64_t)(3 + c) * nys + js) * nxs + is] = Bl[c];
        }
      }
  }
}

void ora_station(const ora_state* s, int station, int64_t* count, const double** times,
                 const double** data) {
  const int T = s->p.station_cap;
  const int nxs = s->p.nx / s->p.station_stride;
  const int nys = s->p.dims == 3 ? s->p.ny / s->p.station_stride : 1;
  *count = s->st_count[station];
  *times = s->st_time + (int64_t)station * T;
  *data = s->st_data + (int64_t)station * T * 6 * nys * nxs;
}

/* ------------------------------------------------------------------------ */
/* diagnostics                                                              */
static int interior_k(const ora_state* s, int comp, int k) {
  if (s->p.bc_z == ORA_BC_PERIODIC) return 1;
  int hi = STAG[comp][0] ? s->p.nz - 3 : s->p.nz - 2;
  return k >= 2 && k <= hi;
}

static void div_field(const ora_state* s, int cx, int cy, int cz, double* out) {
  /* divergence at nodes of a field staggered like E */
  const int nx = s->p.nx, ny = s->p.ny;
  const double idz = 1.0 / s->p.dz, idx = 1.0 / s->p.dx;
  const double idy = s->p.dims == 3 ? 1.0 / s->p.dy : 0.0;
  int kl = zlimit(s, ORA_EX); /* node-type z range */
  memset(out, 0, sizeof(double) * s->npts);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i)
      for (int k = 0; k < kl; ++k)
        out[gidx(s, k, i, j)] =
            (fval(s, cx, k, i, j) - fval(s, cx, k, i - 1, j)) * idx +
            (fval(s, cy, k, i, j) - fval(s, cy, k, i, j - 1)) * idy +
            (fval(s, cz, k, i, j) - fval(s, cz, k - 1, i, j)) * idz;
}

/* div E - rho - rho_ion on nodes.  With the current filter, E follows the
 * filtered current, so the conserved quantity is div E - F(rho_e) - rho_ion
 * (the filter commutes with the difference operators away from open ends). */
static void gauss_field(const ora_state* s, double* G) {
  double* rho = (double*)malloc(sizeof(double) * s->npts);
  ora_rho(s, rho);
  if (s->p.filter_passes > 0) ora_filter_nodes(s, rho);
  div_field(s, ORA_EX, ORA_EY, ORA_EZ, G);
  const double rho_ion = s->p.ppc > 0 ? s->d.gamma_b : 0.0;
  for (int64_t q = 0; q < s->npts; ++q) G[q] -= rho[q] + rho_ion;
  free(rho);
}

static double max_abs_interior_nodes(const ora_state* s, const double* a) {
  double m = 0.0;
  const int nx = s->p.nx, ny = s->p.ny;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i)
      for (int k = 0; k < zlimit(s, ORA_EX); ++k)
        if (interior_k(s, ORA_EX, k)) {
          double v = fabs(a[gidx(s, k, i, j)]);
          if (v > m) m = v;
        }
  return m;
}

void ora_reset_gauss_reference(ora_state* s) {
  gauss_field(s, s->G0);
  double* rho = (double*)malloc(sizeof(double) * s->npts);
  ora_rho(s, rho);
  s->rho0_max = max_abs_interior_nodes(s, rho);
  free(rho);
}

void ora_diag(const ora_state* s, ora_diag_out* o) {
  memset(o, 0, sizeof(*o));
  o->step = s->step;
  o->t = s->step * s->d.dt;
  const int nx = s->p.nx, ny = s->p.ny;
  for (int comp = 0; comp < 6; ++comp) {
    double acc = 0.0;
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i)
        for (int k = 0; k < zlimit(s, comp); ++k)
          if (interior_k(s, comp, k)) {
            double v = s->F[comp][gidx(s, k, i, j)];
            acc += v * v;
            if (comp == ORA_EZ && fabs(v) > o->Ez_max) o->Ez_max = fabs(v);
          }
    if (comp < 3)
      o->U_E += 0.5 * acc * s->d.dV;
    else
      o->U_B += 0.5 * acc * s->d.dV;
  }
  const int open = s->p.bc_z == ORA_BC_OPEN;
  double zlo = 2.0 * s->p.dz, zhi = (s->p.nz - 2) * s->p.dz, zmax = s->p.nz * s->p.dz;
  for (int64_t p = 0; p < s->np; ++p) {
    double z = s->pz[p];
    if (!open || (z >= 0.0 && z < zmax)) o->n_particles++;
    if (!open || (z >= zlo && z < zhi)) {
      double g = sqrt(1.0 + s->ux[p] * s->ux[p] + s->uy[p] * s->uy[p] + s->uz[p] * s->uz[p]);
      o->KE += s->d.weight * (g - 1.0);
    }
  }
  double* G = (double*)malloc(sizeof(double) * s->npts);
  gauss_field(s, G);
  for (int64_t q = 0; q < s->npts; ++q) G[q] -= s->G0[q];
  double gd = max_abs_interior_nodes(s, G);
  o->gauss_drift = s->rho0_max > 0 ? gd / s->rho0_max : gd;
  free(G);
}

/* ------------------------------------------------------------------------ */
ora_state* ora_create(const ora_params* p) {
  ora_state* s = (ora_state*)calloc(1, sizeof(ora_state));
  s->p = *p;
  if (s->p.dims == 2) s->p.ny = 1;
  if (s->p.inject_every < 1) s->p.inject_every = 1;
  ora_derived* d = &s->d;
  double inv2 = 1.0 / (p->dz * p->dz) + 1.0 / (p->dx * p->dx);
  if (p->dims == 3) inv2 += 1.0 / (p->dy * p->dy);
  d->dt = p->cfl / sqrt(inv2);
  d->gamma_b = p->gamma_boost;
  d->beta_b = sqrt(1.0 - 1.0 / (p->gamma_boost * p->gamma_boost));
  d->dplus = d->gamma_b * (1.0 + d->beta_b);
  d->dminus = 1.0 / d->dplus;
  double wp = sqrt(p->n_lab_cm3 * 1e6 * ORA_QE * ORA_QE / (ORA_EPS0 * ORA_ME));
  d->skin_um = ORA_C / wp * 1e6;
  d->k0_lab = 2.0 * ORA_PI * d->skin_um / p->lambda0_um;
  d->E0_lab = p->a0 * d->k0_lab;
  double Lz = p->nz * p->dz;
  d->L_boost = p->tau_lab > 0 ? d->dplus * p->tau_lab : Lz / 8.0;
  d->L_lab = d->L_boost / d->dplus;
  d->zc_boost = 0.5 * Lz;
  d->dV = p->dz * p->dx * (p->dims == 3 ? p->dy : 1.0);
  /* with no plasma (ppc = 0, field-only runs and hand-placed particles) the
   * weight is that of one electron per cell */
  d->weight = d->gamma_b * d->dV / (p->ppc > 0 ? p->ppc : 1);
  d->reservoir = p->bc_z == ORA_BC_OPEN
                     ? (int)ceil(d->beta_b * s->p.inject_every * d->dt / p->dz) + 2
                     : 0;
  d->nzf = p->bc_z == ORA_BC_OPEN ? p->nz + 1 : p->nz;
  s->npts = (int64_t)d->nzf * s->p.nx * s->p.ny;
  for (int c = 0; c < 9; ++c) s->F[c] = (double*)calloc(s->npts, sizeof(double));
  s->G0 = (double*)calloc(s->npts, sizeof(double));
  if (s->p.n_stations > 0) {
    if (s->p.station_stride < 1) s->p.station_stride = 1;
    const int64_t per = 6 * (int64_t)(s->p.nx / s->p.station_stride) *
                        (s->p.dims == 3 ? s->p.ny / s->p.station_stride : 1);
    s->st_data = (double*)calloc((size_t)s->p.n_stations * s->p.station_cap * per, sizeof(double));
    s->st_time = (double*)calloc((size_t)s->p.n_stations * s->p.station_cap, sizeof(double));
    s->st_count = (int64_t*)calloc((size_t)s->p.n_stations, sizeof(int64_t));
  }
  init_fields(s);
  if (p->ppc > 0) inject(s, 0);
  ora_reset_gauss_reference(s);
  return s;
}

void ora_destroy(ora_state* s) {
  if (!s) return;
  for (int c = 0; c < 9; ++c) free(s->F[c]);
  free(s->G0);
  free(s->pz); free(s->px); free(s->py);
  free(s->ux); free(s->uy); free(s->uz); free(s->id);
  free(s->st_data); free(s->st_time); free(s->st_count);
  free(s);
}

void ora_get_derived(const ora_state* s, ora_derived* d) { *d = s->d; }
int64_t ora_num_particles(const ora_state* s) { return s->np; }
int64_t ora_field_points(const ora_state* s) { return s->npts; }
double* ora_field(ora_state* s, int comp) { return s->F[comp]; }
int64_t ora_step_index(const ora_state* s) { return s->step; }

void ora_get_particles(const ora_state* s, double* z, double* x, double* y,
                       double* ux, double* uy, double* uz, uint32_t* id) {
  size_t n = (size_t)s->np;
  memcpy(z, s->pz, n * sizeof(double));
  memcpy(x, s->px, n * sizeof(double));
  memcpy(y, s->py, n * sizeof(double));
  memcpy(ux, s->ux, n * sizeof(double));
  memcpy(uy, s->uy, n * sizeof(double));
  memcpy(uz, s->uz, n * sizeof(double));
  memcpy(id, s->id, n * sizeof(uint32_t));
}

void ora_set_particles(ora_state* s, int64_t n, const double* z, const double* x,
                       const double* y, const double* ux, const double* uy,
                       const double* uz, const uint32_t* id) {
  s->np = 0;
  ensure_cap(s, n);
  s->np = n;
  size_t b = (size_t)n;
  memcpy(s->pz, z, b * sizeof(double));
  memcpy(s->px, x, b * sizeof(double));
  memcpy(s->py, y, b * sizeof(double));
  memcpy(s->ux, ux, b * sizeof(double));
  memcpy(s->uy, uy, b * sizeof(double));
  memcpy(s->uz, uz, b * sizeof(double));
  memcpy(s->id, id, b * sizeof(uint32_t));
}

/* ------------------------------------------------------------------------ */
/* one full step, in this order: (inject) gather -> push -> move -> deposit,
 * then B half step, E full step (+Mur), B half step, then particle boundary
 * conditions. */
void ora_step(ora_state* s, int nsteps, double* cont_max) {
  const double eps = -0.5 * s->d.dt;
  const int open = s->p.bc_z == ORA_BC_OPEN;
  const double Lz = s->p.nz * s->p.dz, Lx = s->p.nx * s->p.dx, Ly = s->p.ny * s->p.dy;
  const double ztop = (s->p.nz + s->d.reservoir + 2) * s->p.dz;
  for (int it = 0; it < nsteps; ++it) {
    if (open && s->step % s->p.inject_every == 0) inject(s, s->step);
    record_stations(s);
    double *rho0 = NULL, *rho1 = NULL;
    if (cont_max) {
      rho0 = (double*)malloc(sizeof(double) * s->npts);
      ora_rho(s, rho0);
    }
    memset(s->F[ORA_JX], 0, sizeof(double) * s->npts);
    memset(s->F[ORA_JY], 0, sizeof(double) * s->npts);
    memset(s->F[ORA_JZ], 0, sizeof(double) * s->npts);
    for (int64_t p = 0; p < s->np; ++p) {
      double E[3], B[3];
      ora_gather(s, s->pz[p], s->px[p], s->py[p], E, B);
      double u[3] = {s->ux[p], s->uy[p], s->uz[p]};
      if (s->p.pusher == ORA_BORIS)
        ora_push_boris(u, E, B, eps);
      else
        ora_push_vay(u, E, B, eps);
      double g = sqrt(1.0 + dot3(u, u));
      double p0[3] = {s->pz[p], s->px[p], s->py[p]};
      double p1[3] = {p0[0] + s->d.dt * u[2] / g, p0[1] + s->d.dt * u[0] / g,
                      s->p.dims == 3 ? p0[2] + s->d.dt * u[1] / g : p0[2]};
      ora_deposit(s, p0, p1, u[1] / g);
      s->pz[p] = p1[0];
      s->px[p] = p1[1];
      s->py[p] = p1[2];
      s->ux[p] = u[0];
      s->uy[p] = u[1];
      s->uz[p] = u[2];
    }
    if (cont_max) {
      rho1 = (double*)malloc(sizeof(double) * s->npts);
      ora_rho(s, rho1);
      double* divj = (double*)malloc(sizeof(double) * s->npts);
      div_field(s, ORA_JX, ORA_JY, ORA_JZ, divj);
      for (int64_t q = 0; q < s->npts; ++q) rho1[q] = rho1[q] - rho0[q] + s->d.dt * divj[q];
      double r = max_abs_interior_nodes(s, rho1);
      double nrm = max_abs_interior_nodes(s, rho0);
      double rel = nrm > 0 ? r / nrm : r;
      if (rel > *cont_max) *cont_max = rel;
      free(divj);
      free(rho0);
      free(rho1);
    }
    if (s->p.filter_passes > 0) ora_filter_current(s);
    half_B(s, s->step, 1);
    full_E(s, s->step);
    half_B(s, s->step + 1, 0);
    /* particle boundary conditions */
    int64_t w = 0;
    for (int64_t p = 0; p < s->np; ++p) {
      double z = s->pz[p];
      if (open) {
        if (z < 0.0 || z >= ztop) continue; /* leaves the box */
      } else {
        z = fmod(z, Lz);
        if (z < 0) z += Lz;
      }
      double x = fmod(s->px[p], Lx);
      if (x < 0) x += Lx;
      double y = s->py[p];
      if (s->p.dims == 3) {
        y = fmod(y, Ly);
        if (y < 0) y += Ly;
      }
      s->pz[w] = z; s->px[w] = x; s->py[w] = y;
      s->ux[w] = s->ux[p]; s->uy[w] = s->uy[p]; s->uz[w] = s->uz[p];
      s->id[w] = s->id[p];
      ++w;
    }
    s->np = w;
    s->step++;
  }
}
