// Relativistic pushers (u = gamma v), device side.
//
// push_vay: the modified Lorentz-force form of the paper (Sec. 2, first
// paragraph; Vay, Phys. Plasmas 15, 056701 (2008)): the magnetic force uses
// the average of the old and new velocity, so for E + v x B = 0 the electric
// and magnetic kicks cancel exactly; the resulting implicit equation for the
// new gamma is solved in closed form.  The vector algebra runs in R (float
// or double); the gamma solve always runs in double, because at large gamma
// the "1 +" and the tau^2 terms of sigma vanish below FP32 resolution.
//
// push_boris: the Boris pusher the paper replaces (kept as a control).
#pragma once

#include <hip/hip_runtime.h>

namespace pic {

// u'^2 above which the gamma solve runs in FP64 (gamma ~ 1000)
#ifndef PIC_GAMMA2_FP64
#define PIC_GAMMA2_FP64 1.0e6
#endif
constexpr double GAMMA2_FP64 = PIC_GAMMA2_FP64;

// Reciprocal, reciprocal square root and square root: one hardware
// instruction each in FP32 (v_rcp_f32, v_rsq_f32, v_sqrt_f32, about 1 ulp
// instead of the ~12-instruction correctly rounded sequences), IEEE in FP64.
// Their arguments here are 1 + u^2, 1 + t^2 and positive sums: never
// denormal.
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double frcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double frsq(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fsqrt(double x) { return sqrt(x); }

template <typename R>
__device__ __forceinline__ void push_vay(R& ux, R& uy, R& uz, R ex, R ey, R ez, R bx, R by, R bz,
                                         R eps) {
  const R ig = frsq(R(1) + ux * ux + uy * uy + uz * uz);
  const R vx = ux * ig, vy = uy * ig, vz = uz * ig;
  // half electric kick plus magnetic force with the old velocity, then the
  // second electric half kick: u' = u + eps (2E + v x B)
  const R upx = ux + eps * (R(2) * ex + (vy * bz - vz * by));
  const R upy = uy + eps * (R(2) * ey + (vz * bx - vx * bz));
  const R upz = uz + eps * (R(2) * ez + (vx * by - vy * bx));
  const R tx = eps * bx, ty = eps * by, tz = eps * bz;
  // gamma_new^2 = (sigma + sqrt(sigma^2 + 4 (tau^2 + u*^2))) / 2,
  // sigma = 1 + u'^2 - tau^2, u* = u'.tau.  At large gamma the "1 +" and the
  // tau^2 terms of sigma drop below FP32 resolution (the "1" is lost entirely
  // above u'^2 ~ 2^24), so the solve runs in FP64 whenever some lane of the
  // wavefront has u'^2 > GAMMA2_FP64 (gamma above ~1000, where the "1" is
  // still 16 FP32 ulps of u'^2); below that the FP32 solve keeps gamma_new
  // to ~1.3e-7 relative, the rounding level of the FP32 momentum itself.
  // The switch is wavefront-uniform, so no lane pays for both.
  R ign;
  const R up2 = upx * upx + upy * upy + upz * upz;
  if (sizeof(R) == 8 || __any(up2 > R(GAMMA2_FP64))) {
    const double dux = upx, duy = upy, duz = upz, dtx = tx, dty = ty, dtz = tz;
    const double ustar = dux * dtx + duy * dty + duz * dtz;
    const double tau2 = dtx * dtx + dty * dty + dtz * dtz;
    const double sigma = 1.0 + (dux * dux + duy * duy + duz * duz) - tau2;
    const double a4 = 4.0 * (tau2 + ustar * ustar);
    const double disc = sqrt(sigma * sigma + a4);
    const double g2 = sigma >= 0.0 ? 0.5 * (sigma + disc) : 0.5 * a4 / (disc - sigma);
    // gamma_new^2 carries the FP64 accuracy; its reciprocal square root is
    // taken in R (for FP32 one v_rsq_f32, relative error ~1e-7)
    ign = R(frsq(R(g2)));
  } else {
    const R ustar = upx * tx + upy * ty + upz * tz;
    const R tau2 = tx * tx + ty * ty + tz * tz;
    const R sigma = R(1) + up2 - tau2;
    const R a4 = R(4) * (tau2 + ustar * ustar);
    const R disc = fsqrt(sigma * sigma + a4);
    // both forms evaluated and selected (no divergent branch); the second
    // avoids the cancellation when sigma < 0
    const R g2p = R(0.5) * (sigma + disc), g2n = R(0.5) * a4 * frcp(disc - sigma);
    const R g2 = sigma >= R(0) ? g2p : g2n;
    ign = frsq(g2);
  }
  // u_new = s (u' + (u'.t) t + u' x t),  t = tau / gamma_new,  s = 1/(1+t^2),
  // evaluated as u' + s ((u'.t) t + u' x t - t^2 u'): the small rotation is
  // formed on its own and added once, so the large components of u' are
  // rounded once per step instead of being scaled by s
  const R ttx = tx * ign, tty = ty * ign, ttz = tz * ign;
  const R t2 = ttx * ttx + tty * tty + ttz * ttz;
  const R s = frcp(R(1) + t2);
  const R upt = upx * ttx + upy * tty + upz * ttz;
  ux = upx + s * (upt * ttx + (upy * ttz - upz * tty) - t2 * upx);
  uy = upy + s * (upt * tty + (upz * ttx - upx * ttz) - t2 * upy);
  uz = upz + s * (upt * ttz + (upx * tty - upy * ttx) - t2 * upz);
}

template <typename R>
__device__ __forceinline__ void push_boris(R& ux, R& uy, R& uz, R ex, R ey, R ez, R bx, R by,
                                           R bz, R eps) {
  const R mx = ux + eps * ex, my = uy + eps * ey, mz = uz + eps * ez;
  const R ig = frsq(R(1) + mx * mx + my * my + mz * mz);
  const R tx = eps * bx * ig, ty = eps * by * ig, tz = eps * bz * ig;
  const R px = mx + (my * tz - mz * ty);
  const R py = my + (mz * tx - mx * tz);
  const R pz = mz + (mx * ty - my * tx);
  const R f = R(2) * frcp(R(1) + tx * tx + ty * ty + tz * tz);
  const R sx = f * tx, sy = f * ty, sz = f * tz;
  ux = mx + (py * sz - pz * sy) + eps * ex;
  uy = my + (pz * sx - px * sz) + eps * ey;
  uz = mz + (px * sy - py * sx) + eps * ez;
}

}  // namespace pic
