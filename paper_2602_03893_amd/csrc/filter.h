// filter.h -- constants of the float32 window filter for one (reference
// block, sensor), shared by the isotropic and the anisotropic operators.
//
// For a kernel at offset dk = c_k - c_B from the float32-rounded centre c_B
// of its reference block, seen from sensor s at distance R = |s - c_B|,
// D = r^2 - R^2 = |dk|^2 - 2 (s - c_B).dk, and r - R = dr solves
// dr = (D - dr^2) / (2R), reached by a few fixed-point steps (the planner sets
// their number per block).  The window position in samples is then
// X + dr / (v dt) with X = R / (v dt) - t0 / dt - nb split into an integer and
// a float32 fraction, so every float32 quantity stays small.
#pragma once

#include "gpair_internal.h"

namespace gpair {

// Guard of the float32 window filter (samples): the planner admits a block
// to the filter only when the filter's error bound is below kGuard / 2.
constexpr float kGuard = (float)kFilterGuard;

// Constants of the float32 filter for one (reference block, sensor).
struct BlockLane {
  float m2ux, m2uy, m2uz;  // -2 (s - c_B)
  float inv2R;             // 1 / (2R)
  float Rf;                // R
  float Xf;                // X - Xi, X = R/(v dt) - t0/dt - nb
  int Xi;                  // floor(X)
};

// Fills bl for the sensor at s (double4: x, y, z, |s|^2) and the block B
// (its float32-rounded centre is the reference point).  The number of
// fixed-point steps, or -1 (every pair in float64), is the block's
// filter_steps, set by the planner from its closest sensor so that the
// forward and the adjoint run the same arithmetic for every pair.
__device__ __forceinline__ void block_lane(const double4 &s, const TileInfo &B, int nb,
                                           double inv_vdt, double t0_over_dt, BlockLane &bl) {
  const float bx = (float)B.cx, by = (float)B.cy, bz = (float)B.cz;
  const double ux = s.x - (double)bx, uy = s.y - (double)by, uz = s.z - (double)bz;
  const double R = sqrt(fma(uz, uz, fma(uy, uy, ux * ux)));
  const double X = fma(R, inv_vdt, -t0_over_dt) - (double)nb;
  const double Xi = floor(X);
  bl.m2ux = (float)(-2.0 * ux);
  bl.m2uy = (float)(-2.0 * uy);
  bl.m2uz = (float)(-2.0 * uz);
  bl.inv2R = (float)(0.5 / R);
  bl.Rf = (float)R;
  bl.Xf = (float)(X - Xi);
  bl.Xi = (int)Xi;
}

}  // namespace gpair
