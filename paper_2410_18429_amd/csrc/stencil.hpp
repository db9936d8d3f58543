// Stencil arithmetic shared by every kernel that applies A or A^H (the fused
// CGLS kernels, the single-operator kernel and the off-grid path), so that all
// of them round identically.  Device-only inline functions.
#pragma once

#include <hip/hip_runtime.h>

namespace wri {

__device__ __forceinline__ double sponge_axis_d(int i, int n, int nb, double inv_nb) {
  const int d = max(0, max(nb - i, i - (n - 1 - nb)));
  const double f = (double)d * inv_nb;
  return f * f;
}

// One cell of A c (kim = -omega b) or A^H c (kim = +omega b):
//   sum over the 6 neighbours of (nb - c) / h^2  +  (omega^2 m + i kim) c.
// Storage is complex float32; the arithmetic is float64 in registers and the
// result is rounded once.  (Float32 arithmetic here loses several digits to
// cancellation between the Laplacian and the mass term and slows CGLS; the
// kernels are bandwidth-bound, so the float64 pipe costs nothing measurable.)
// The difference form limits cancellation for smooth fields.  This function
// is the only place the stencil arithmetic lives, so every tiling (and the
// single-operator kernel) rounds identically.
__device__ __forceinline__ double2 helm(float2 c, float2 xm, float2 xp, float2 ym, float2 yp,
                                        float2 zm, float2 zp, double h2inv, double kre, double kim) {
  const double cr = c.x, ci = c.y;
  const double lr = ((((double)xm.x - cr) + ((double)xp.x - cr)) + (((double)ym.x - cr) + ((double)yp.x - cr))) +
                    (((double)zm.x - cr) + ((double)zp.x - cr));
  const double li = ((((double)xm.y - ci) + ((double)xp.y - ci)) + (((double)ym.y - ci) + ((double)yp.y - ci))) +
                    (((double)zm.y - ci) + ((double)zp.y - ci));
  return make_double2(lr * h2inv + (kre * cr - kim * ci), li * h2inv + (kre * ci + kim * cr));
}

__device__ __forceinline__ float2 round2(double2 v) { return make_float2((float)v.x, (float)v.y); }

}  // namespace wri
