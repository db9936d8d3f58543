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
//   (sum of the 6 neighbours - 6 c) / h^2  +  (omega^2 m + i kim) c.
// Storage is complex float32; the arithmetic is float64 in registers and the
// result is rounded once.  (Float32 arithmetic here loses several digits to
// cancellation between the Laplacian and the mass term and slows CGLS.)  The
// inputs are float32, so the float64 sum of the six neighbours and the fused
// subtraction of 6 c are exact unless the magnitudes of a neighbourhood span
// more than 2^26: no difference form is needed, and the stencil takes 9
// float64 operations per component.  This function is the only place the
// stencil arithmetic lives, so every tiling, the recomputed t of the adjoint
// pass and the single-operator kernel round identically.
__device__ __forceinline__ double2 helm(float2 c, float2 xm, float2 xp, float2 ym, float2 yp,
                                        float2 zm, float2 zp, double h2inv, double kre, double kim) {
  const double cr = c.x, ci = c.y;
  const double sr = (((double)xm.x + (double)xp.x) + ((double)ym.x + (double)yp.x)) + ((double)zm.x + (double)zp.x);
  const double si = (((double)xm.y + (double)xp.y) + ((double)ym.y + (double)yp.y)) + ((double)zm.y + (double)zp.y);
  const double lr = fma(-6.0, cr, sr), li = fma(-6.0, ci, si);
  return make_double2(fma(lr, h2inv, fma(kre, cr, -(kim * ci))), fma(li, h2inv, fma(kre, ci, kim * cr)));
}

__device__ __forceinline__ float2 round2(double2 v) { return make_float2((float)v.x, (float)v.y); }

}  // namespace wri
