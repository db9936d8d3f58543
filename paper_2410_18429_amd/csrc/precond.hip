// Preconditioned CGLS: the batched augmented solve with S preconditioned on the
// right by one multigrid V(1,1) cycle of the complex-shifted Helmholtz operator
//   A_beta = L_h + diag(omega^2 (1 - i beta) m - i omega b),   beta = 1/2,
// i.e. CGLS on min ||S M y - b|| with x = M y.  This goes beyond the paper,
// whose only reducer of the iteration count is the adaptive tolerance of
// Algorithm 2: the minimiser is that of eq. SimpObj, the iterates and their
// number differ.  S is the printed one (source column -e, weight 1), and the
// stopping test is the plain solver's, on the true normal residual
// ||S^H r|| <= rtol ||S^H b||.
//
// Per iteration, over all systems of a grid in lockstep (finished systems skip
// inside the kernels; step scalars live in device memory; chunks of iterations
// replay from a hipGraph between host checks of the statuses):
//   p = z + beta p;  q = M p (V-cycle);  t = S q;  a = gamma / ||t||^2;
//   x += a q;  r -= a t;  s = S^H r (stopping test);  z = M^H s (V-cycle on
//   conj(A_beta), M being complex symmetric);  beta = ||z||^2 / gamma.
// The V-cycle on a level with right-hand side f: y = w D^-1 f (one damped
// Jacobi step from zero), the residual f - A_beta y restricted with P^T / 8 to
// the next level (halved along every axis, h doubled, m and sponge restricted
// as weighted means), the next level's result prolonged (trilinear) and added,
// one more Jacobi step; four Jacobi steps from zero on the coarsest level.
// Every reduction sums fixed per-block partials in one fixed order.
#include "../../include/wri.h"
#include "wri_impl.hpp"
#include "stencil.hpp"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <vector>

namespace wri {
namespace {

constexpr int kThr = 256;
constexpr int kParts = 256;        // blocks (and partial sums) per system for the level-0 passes
constexpr int kMaxLev = 12;
constexpr int kCheck = 16;         // iterations between host checks of the statuses
constexpr double kBeta = 0.5;      // imaginary shift of the mass term in A_beta
constexpr double kJac = 0.7;       // Jacobi damping
constexpr int kCoarseSweeps = 4;   // Jacobi steps on the coarsest level
constexpr int64_t kCoarsestCells = 512;
constexpr size_t kAl = 256;
size_t al(size_t v) { return (v + kAl - 1) / kAl * kAl; }

#define PC_HIP(expr)                                                                                \
  do {                                                                                              \
    hipError_t e_ = (expr);                                                                         \
    if (e_ != hipSuccess) return report_error(WRI_EHIP, "%s: %s", #expr, hipGetErrorString(e_));   \
  } while (0)

// One level of one system's V-cycle.  m and b are the grid's (shared by its
// systems); f, y, o, res are the system's: right-hand side, the prolonged and
// corrected iterate, the level's result, the restricted residual's source.
struct PcLevel {
  int nx, ny, nz, n;
  double h2inv;
  const float* m;
  const float* b;
  const float2* wdinv;   // w D^-1 of A_beta on this level (per grid and frequency), complex64
  float2 *f, *y, *o, *res;
};

struct PcSys {
  float2 *x, *r, *p, *q, *t, *s, *z, *r2, *t2;
  const float2* d;
  const int* rec;
  const float* m;
  int n, nx, ny, nz, nb, nr, est, max_iter, nlev, src, pad_[2];
  double lam, rtol2, omega, omega2, h2inv, sp_scale, inv_nb;
  double2 alpha;  // KNOWN-mode weight
  PcLevel lev[kMaxLev];
};

// Mutable scalars of one system (float64).
struct PcState {
  double gamma, ss0, ss, ssmin, a, beta, J;
  double2 xa, pa, za;
  int status, iters, pad_[2];
};

__device__ __forceinline__ double bsum(double v, double* red) {  // block total, every thread
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < kThr / 64; ++i) r += red[i];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double nrm(float2 v) { return (double)v.x * v.x + (double)v.y * v.y; }
__device__ __forceinline__ float2 fd(double a, double b) { return make_float2((float)a, (float)b); }

// partials of one system's level-0 pass: kParts values, summed in index order
__device__ double sum_parts(const double* __restrict__ part, double* red) {
  double v = 0.0;
  for (int i = threadIdx.x; i < kParts; i += kThr) v += part[i];
  return bsum(v, red);
}

// ---------------------------------------------------------------------------
// level-0 CGLS passes (grid (kParts, systems of the group))
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool active(const PcState* stv, int k) { return stv[k].status == kActive; }

// x = 0, r = 0, p = 0
__global__ void __launch_bounds__(kThr) k_pc_zero(const PcSys* __restrict__ sy, int g0) {
  const PcSys& S = sy[g0 + blockIdx.y];
  const float2 z = make_float2(0.f, 0.f);
  for (int c = blockIdx.x * kThr + threadIdx.x; c < S.n; c += gridDim.x * kThr) {
    S.x[c] = z;
    S.r[c] = z;
    S.p[c] = z;
  }
}

// r1[src] = alpha (KNOWN), r2 = lam d, scalars reset (one block per system)
__global__ void __launch_bounds__(kThr) k_pc_init(const PcSys* __restrict__ sy, PcState* __restrict__ stv, int g0) {
  const int k = g0 + blockIdx.x;
  const PcSys& S = sy[k];
  for (int q = threadIdx.x; q < S.nr; q += kThr) {
    const float2 dv = S.d[q];
    S.r2[q] = fd(S.lam * dv.x, S.lam * dv.y);
  }
  if (threadIdx.x == 0) {
    if (!S.est) S.r[S.src] = fd(S.alpha.x, S.alpha.y);
    PcState& T = stv[k];
    T = PcState{};
    T.status = kActive;
  }
}

// p = z + beta p (beta of the state; 0 at the start)
__global__ void __launch_bounds__(kThr) k_pc_pupd(const PcSys* __restrict__ sy, const PcState* __restrict__ stv,
                                                  int g0) {
  const int k = g0 + blockIdx.y;
  if (!active(stv, k)) return;
  const PcSys& S = sy[k];
  const double be = stv[k].beta;
  for (int c = blockIdx.x * kThr + threadIdx.x; c < S.n; c += gridDim.x * kThr) {
    const float2 zv = S.z[c], pv = S.p[c];
    S.p[c] = fd((double)zv.x + be * pv.x, (double)zv.y + be * pv.y);
  }
}

__device__ __forceinline__ double sponge_at(const PcSys& S, int x, int y, int z) {
  return S.sp_scale * ((sponge_axis_d(x, S.nx, S.nb, S.inv_nb) + sponge_axis_d(y, S.ny, S.nb, S.inv_nb)) +
                       sponge_axis_d(z, S.nz, S.nb, S.inv_nb));
}

// one cell of A v (adj = 0) or A^H v (adj = 1) in float64 from float32 storage
__device__ __forceinline__ double2 apply_cell(const PcSys& S, const float2* __restrict__ v, int c, bool adj) {
  const int plane = S.nx * S.ny;
  const int z = c / plane, rem = c - z * plane, y = rem / S.nx, x = rem - y * S.nx;
  const float2 zero = make_float2(0.f, 0.f);
  const float2 xm = x > 0 ? v[c - 1] : zero, xp = x < S.nx - 1 ? v[c + 1] : zero;
  const float2 ym = y > 0 ? v[c - S.nx] : zero, yp = y < S.ny - 1 ? v[c + S.nx] : zero;
  const float2 zm = z > 0 ? v[c - plane] : zero, zp = z < S.nz - 1 ? v[c + plane] : zero;
  const double kim = S.omega * sponge_at(S, x, y, z);
  return helm(v[c], xm, xp, ym, yp, zm, zp, S.h2inv, S.omega2 * (double)S.m[c], adj ? kim : -kim);
}

// t = A q - p_alpha e_src (ESTIMATE; q_alpha = p_alpha); partials of ||t||^2
__global__ void __launch_bounds__(kThr) k_pc_fwd(const PcSys* __restrict__ sy, const PcState* __restrict__ stv,
                                                 double* __restrict__ part, int g0) {
  __shared__ double red[kThr / 64];
  const int k = g0 + blockIdx.y;
  if (!active(stv, k)) return;
  const PcSys& S = sy[k];
  const double2 pa = stv[k].pa;
  double acc = 0.0;
  for (int c = blockIdx.x * kThr + threadIdx.x; c < S.n; c += gridDim.x * kThr) {
    double2 tv = apply_cell(S, S.q, c, false);
    if (S.est && c == S.src) { tv.x -= pa.x; tv.y -= pa.y; }
    const float2 t = round2(tv);
    S.t[c] = t;
    acc += nrm(t);
  }
  const double tot = bsum(acc, red);
  if (threadIdx.x == 0) part[(size_t)k * kParts + blockIdx.x] = tot;
}

// receiver rows t2 = lam q[rec]; delta, a; x_alpha += a p_alpha; r2 -= a t2
// (one block per system)
__global__ void __launch_bounds__(kThr) k_pc_step(const PcSys* __restrict__ sy, PcState* __restrict__ stv,
                                                  const double* __restrict__ part, int g0) {
  __shared__ double red[kThr / 64];
  const int k = g0 + blockIdx.x;
  if (!active(stv, k)) return;
  const PcSys& S = sy[k];
  PcState& T = stv[k];
  double acc = 0.0;
  for (int q = threadIdx.x; q < S.nr; q += kThr) {
    const float2 qv = S.q[S.rec[q]];
    const float2 t2 = fd(S.lam * qv.x, S.lam * qv.y);
    S.t2[q] = t2;
    acc += nrm(t2);
  }
  const double delta = sum_parts(part + (size_t)k * kParts, red) + bsum(acc, red);
  const bool bad = !(delta > 0.0) || !(delta <= DBL_MAX) || !(T.gamma <= DBL_MAX);
  const double a = bad ? 0.0 : T.gamma / delta;
  for (int q = threadIdx.x; q < S.nr; q += kThr) {
    const float2 r2 = S.r2[q], t2 = S.t2[q];
    S.r2[q] = fd((double)r2.x - a * t2.x, (double)r2.y - a * t2.y);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    T.a = a;
    if (bad) {
      T.status = kBreakdown;
    } else if (S.est) {
      T.xa = make_double2(T.xa.x + a * T.pa.x, T.xa.y + a * T.pa.y);
    }
  }
}

// r -= a t, x += a q
__global__ void __launch_bounds__(kThr) k_pc_rupd(const PcSys* __restrict__ sy, const PcState* __restrict__ stv,
                                                  int g0) {
  const int k = g0 + blockIdx.y;
  if (!active(stv, k)) return;
  const PcSys& S = sy[k];
  const double a = stv[k].a;
  for (int c = blockIdx.x * kThr + threadIdx.x; c < S.n; c += gridDim.x * kThr) {
    const float2 r = S.r[c], t = S.t[c], x = S.x[c], q = S.q[c];
    S.r[c] = fd((double)r.x - a * t.x, (double)r.y - a * t.y);
    S.x[c] = fd((double)x.x + a * q.x, (double)x.y + a * q.y);
  }
}

// s = A^H r (the receiver and source-row terms are added per system); partials of ||s||^2
__global__ void __launch_bounds__(kThr) k_pc_adj(const PcSys* __restrict__ sy, const PcState* __restrict__ stv,
                                                 double* __restrict__ part, int g0) {
  __shared__ double red[kThr / 64];
  const int k = g0 + blockIdx.y;
  if (!active(stv, k)) return;
  const PcSys& S = sy[k];
  double acc = 0.0;
  for (int c = blockIdx.x * kThr + threadIdx.x; c < S.n; c += gridDim.x * kThr) {
    const float2 s = round2(apply_cell(S, S.r, c, true));
    S.s[c] = s;
    acc += nrm(s);
  }
  const double tot = bsum(acc, red);
  if (threadIdx.x == 0) part[(size_t)k * kParts + blockIdx.x] = tot;
}

// s += lam P^H r2 (distinct receiver cells), s_alpha = -r1[src] (ESTIMATE);
// ||s||^2, the stopping test (one block per system).  setup = 1: ||s_0||^2.
__global__ void __launch_bounds__(kThr) k_pc_check(const PcSys* __restrict__ sy, PcState* __restrict__ stv,
                                                   const double* __restrict__ part, int g0, int setup) {
  __shared__ double red[kThr / 64];
  const int k = g0 + blockIdx.x;
  if (!active(stv, k)) return;
  const PcSys& S = sy[k];
  PcState& T = stv[k];
  double corr = 0.0;
  for (int q = threadIdx.x; q < S.nr; q += kThr) {
    const int c = S.rec[q];
    const float2 s0 = S.s[c], r2 = S.r2[q];
    const float2 s1 = fd((double)s0.x + S.lam * r2.x, (double)s0.y + S.lam * r2.y);
    S.s[c] = s1;
    corr += nrm(s1) - nrm(s0);
  }
  const double ss_u = sum_parts(part + (size_t)k * kParts, red) + bsum(corr, red);
  if (threadIdx.x == 0) {
    double2 sa = make_double2(0.0, 0.0);
    if (S.est) {
      const float2 r1 = S.r[S.src];
      sa = make_double2(-(double)r1.x, -(double)r1.y);
    }
    const double ss = ss_u + sa.x * sa.x + sa.y * sa.y;
    T.za = sa;  // M leaves the source-weight component as it is: z_alpha = s_alpha
    T.ss = ss;
    if (setup) {
      T.ss0 = ss;
      T.ssmin = ss;
      if (ss == 0.0) T.status = kZeroRhs;
      else if (!(ss <= DBL_MAX)) T.status = kBreakdown;
      else if (S.rtol2 >= 1.0) T.status = kConverged;   // ||s_0|| <= rtol ||s_0||
      else if (S.max_iter <= 0) T.status = kMaxIter;
    } else {
      T.iters += 1;
      // below what float32 storage resolves the recurrences iterate on
      // rounding noise: a rise of ||S^H r|| 1e4 times above its running
      // minimum stops the system (as in the plain solver)
      T.ssmin = fmin(T.ssmin, ss);
      if (!(ss <= DBL_MAX)) T.status = kBreakdown;
      else if (ss <= S.rtol2 * T.ss0) T.status = kConverged;
      else if (T.iters >= S.max_iter) T.status = kMaxIter;
      else if (ss > kDivergeRatio * T.ssmin) T.status = kDiverged;
    }
  }
}

// gamma' = ||z||^2, beta = gamma'/gamma, p_alpha = z_alpha + beta p_alpha
// (one block per system).  setup = 1: gamma = ||z_0||^2, beta = 0.
__global__ void __launch_bounds__(kThr) k_pc_beta(const PcSys* __restrict__ sy, PcState* __restrict__ stv,
                                                  const double* __restrict__ part, int g0, int setup) {
  __shared__ double red[kThr / 64];
  const int k = g0 + blockIdx.x;
  if (!active(stv, k)) return;
  PcState& T = stv[k];
  const double zz = sum_parts(part + (size_t)k * kParts, red) + (T.za.x * T.za.x + T.za.y * T.za.y);
  if (threadIdx.x == 0) {
    const double be = setup ? 0.0 : zz / T.gamma;
    T.beta = be;
    T.gamma = zz;
    T.pa = make_double2(T.za.x + be * T.pa.x, T.za.y + be * T.pa.y);
    if (!(zz > 0.0) || !(zz <= DBL_MAX)) T.status = (T.ss == 0.0) ? T.status : kBreakdown;
  }
}

// ---------------------------------------------------------------------------
// V-cycle passes (grid (blocks, systems of the group)); conj = 1: the cycle on
// conj(A_beta).  A level-0 pass reads its right-hand side from `in0` (p or s)
// and the level-0 result goes to `out0` (q or z).
// ---------------------------------------------------------------------------

// diagonal of A_beta (or its conjugate) at a cell: -6/h^2 + omega^2 (1 - i beta) m - i omega b
__device__ __forceinline__ double2 diag_beta(const PcSys& S, const PcLevel& L, int c, int conj) {
  const double m = L.m[c], b = L.b[c];
  const double im = -kBeta * S.omega2 * m - S.omega * b;
  return make_double2(-6.0 * L.h2inv + S.omega2 * m, conj ? -im : im);
}
// w D^-1 v with the tabulated w D^-1 (conjugated for the cycle on conj(A_beta))
__device__ __forceinline__ double2 jac(const PcLevel& L, int c, int conj, float2 v) {
  const float2 w = L.wdinv[c];
  const double wr = w.x, wi = conj ? -(double)w.y : (double)w.y;
  return make_double2(wr * v.x - wi * v.y, wr * v.y + wi * v.x);
}
__device__ __forceinline__ void coords(const PcLevel& L, int c, int& x, int& y, int& z) {
  const int plane = L.nx * L.ny;
  z = c / plane;
  const int rem = c - z * plane;
  y = rem / L.nx;
  x = rem - y * L.nx;
}

__device__ __forceinline__ const float2* level_in(const PcSys& S, int l, int which) {
  return l > 0 ? S.lev[l].f : (which ? S.s : S.p);
}

// res = f - A_beta (w D^-1 f) on level l (w D^-1 f recomputed at each neighbour)
__global__ void __launch_bounds__(kThr) k_pc_vdown(const PcSys* __restrict__ sy, const PcState* __restrict__ stv,
                                                   int g0, int l, int which, int conj) {
  const int k = g0 + blockIdx.y;
  if (!active(stv, k)) return;
  const PcSys& S = sy[k];
  if (l >= S.nlev - 1) return;
  const PcLevel& L = S.lev[l];
  const float2* __restrict__ f = level_in(S, l, which);
  for (int c = blockIdx.x * kThr + threadIdx.x; c < L.n; c += gridDim.x * kThr) {
    int x, y, z;
    coords(L, c, x, y, z);
    const int plane = L.nx * L.ny;
    double sr = 0.0, si = 0.0;
    const int nb[6] = {x > 0 ? c - 1 : -1, x < L.nx - 1 ? c + 1 : -1, y > 0 ? c - L.nx : -1,
                       y < L.ny - 1 ? c + L.nx : -1, z > 0 ? c - plane : -1, z < L.nz - 1 ? c + plane : -1};
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      if (nb[i] < 0) continue;
      const double2 yn = jac(L, nb[i], conj, f[nb[i]]);
      sr += yn.x;
      si += yn.y;
    }
    const double2 d = diag_beta(S, L, c, conj);
    const float2 fc = f[c];
    const double2 yc = jac(L, c, conj, fc);
    const double ar = sr * L.h2inv + (d.x * yc.x - d.y * yc.y);
    const double ai = si * L.h2inv + (d.x * yc.y + d.y * yc.x);
    L.res[c] = fd((double)fc.x - ar, (double)fc.y - ai);
  }
}

// f_{l+1} = P^T res_l / 8 (27 fine cells around fine (2i+1, 2j+1, 2k+1))
__global__ void __launch_bounds__(kThr) k_pc_vrestrict(const PcSys* __restrict__ sy, const PcState* __restrict__ stv,
                                                       int g0, int l) {
  const int k = g0 + blockIdx.y;
  if (!active(stv, k)) return;
  const PcSys& S = sy[k];
  if (l >= S.nlev - 1) return;
  const PcLevel& F = S.lev[l];
  const PcLevel& C = S.lev[l + 1];
  for (int c = blockIdx.x * kThr + threadIdx.x; c < C.n; c += gridDim.x * kThr) {
    int cx, cy, cz;
    coords(C, c, cx, cy, cz);
    double sr = 0.0, si = 0.0;
    for (int dz = -1; dz <= 1; ++dz) {
      const int fz = 2 * cz + 1 + dz;
      if (fz < 0 || fz >= F.nz) continue;
      for (int dy = -1; dy <= 1; ++dy) {
        const int fy = 2 * cy + 1 + dy;
        if (fy < 0 || fy >= F.ny) continue;
        for (int dx = -1; dx <= 1; ++dx) {
          const int fx = 2 * cx + 1 + dx;
          if (fx < 0 || fx >= F.nx) continue;
          const double w = (dz ? 0.5 : 1.0) * (dy ? 0.5 : 1.0) * (dx ? 0.5 : 1.0);
          const float2 v = F.res[((size_t)fz * F.ny + fy) * F.nx + fx];
          sr += w * v.x;
          si += w * v.y;
        }
      }
    }
    C.f[c] = fd(0.125 * sr, 0.125 * si);
  }
}

// Jacobi step on the coarsest level: sweep 0: o = w D^-1 f; sweep j > 0:
// out = in + w D^-1 (f - A_beta in), in/out alternating o (j odd reads o) and y
__global__ void __launch_bounds__(kThr) k_pc_vcoarse(const PcSys* __restrict__ sy, const PcState* __restrict__ stv,
                                                     int g0, int which, int conj, int sweep) {
  const int k = g0 + blockIdx.y;
  if (!active(stv, k)) return;
  const PcSys& S = sy[k];
  const int l = S.nlev - 1;
  const PcLevel& L = S.lev[l];
  const float2* __restrict__ f = level_in(S, l, which);
  const float2* __restrict__ in = (sweep & 1) ? L.o : L.y;
  float2* __restrict__ out = (sweep & 1) ? L.y : L.o;
  for (int c = blockIdx.x * kThr + threadIdx.x; c < L.n; c += gridDim.x * kThr) {
    const double2 d = diag_beta(S, L, c, conj);
    if (sweep == 0) {
      const double2 v = jac(L, c, conj, f[c]);
      out[c] = fd(v.x, v.y);
      continue;
    }
    int x, y, z;
    coords(L, c, x, y, z);
    const int plane = L.nx * L.ny;
    const float2 zero = make_float2(0.f, 0.f);
    const float2 xm = x > 0 ? in[c - 1] : zero, xp = x < L.nx - 1 ? in[c + 1] : zero;
    const float2 ym = y > 0 ? in[c - L.nx] : zero, yp = y < L.ny - 1 ? in[c + L.nx] : zero;
    const float2 zm = z > 0 ? in[c - plane] : zero, zp = z < L.nz - 1 ? in[c + plane] : zero;
    const float2 xc = in[c];
    const double sr = (((double)xm.x + xp.x) + ((double)ym.x + yp.x)) + ((double)zm.x + zp.x);
    const double si = (((double)xm.y + xp.y) + ((double)ym.y + yp.y)) + ((double)zm.y + zp.y);
    const double ar = sr * L.h2inv + (d.x * xc.x - d.y * xc.y);
    const double ai = si * L.h2inv + (d.x * xc.y + d.y * xc.x);
    const float2 fc = f[c];
    const double2 corr = jac(L, c, conj, fd((double)fc.x - ar, (double)fc.y - ai));
    out[c] = fd((double)xc.x + corr.x, (double)xc.y + corr.y);
  }
}

// the coarsest level's result: after kCoarseSweeps sweeps it is in o (odd count) or y
__device__ __forceinline__ const float2* coarse_out(const PcSys& S, int l) {
  const PcLevel& L = S.lev[l];
  if (l < S.nlev - 1) return L.o;
  return (kCoarseSweeps & 1) ? L.o : L.y;
}

// y_l = w D^-1 f_l + P e_{l+1} (trilinear)
__global__ void __launch_bounds__(kThr) k_pc_vprolong(const PcSys* __restrict__ sy, const PcState* __restrict__ stv,
                                                      int g0, int l, int which, int conj) {
  const int k = g0 + blockIdx.y;
  if (!active(stv, k)) return;
  const PcSys& S = sy[k];
  if (l >= S.nlev - 1) return;
  const PcLevel& F = S.lev[l];
  const PcLevel& C = S.lev[l + 1];
  const float2* __restrict__ e = coarse_out(S, l + 1);
  const float2* __restrict__ f = level_in(S, l, which);
  for (int c = blockIdx.x * kThr + threadIdx.x; c < F.n; c += gridDim.x * kThr) {
    int x, y, z;
    coords(F, c, x, y, z);
    // 1D interpolation: odd fine f <- coarse (f-1)/2 (1); even f <- f/2 - 1 and f/2 (1/2 each)
    int ix[2], iy[2], iz[2];
    double wx[2], wy[2], wz[2];
    auto axis = [](int fi, int nc, int* id, double* w) {
      if (fi & 1) { id[0] = (fi - 1) >> 1; w[0] = 1.0; id[1] = -1; w[1] = 0.0; }
      else {
        id[0] = (fi >> 1) - 1; w[0] = 0.5; id[1] = fi >> 1; w[1] = 0.5;
        if (id[1] >= nc) id[1] = -1;
      }
      if (id[0] >= nc) id[0] = -1;
    };
    axis(x, C.nx, ix, wx);
    axis(y, C.ny, iy, wy);
    axis(z, C.nz, iz, wz);
    double sr = 0.0, si = 0.0;
    for (int a = 0; a < 2; ++a) {
      if (iz[a] < 0) continue;
      for (int b = 0; b < 2; ++b) {
        if (iy[b] < 0) continue;
        for (int cc = 0; cc < 2; ++cc) {
          if (ix[cc] < 0) continue;
          const double w = wz[a] * wy[b] * wx[cc];
          const float2 v = e[((size_t)iz[a] * C.ny + iy[b]) * C.nx + ix[cc]];
          sr += w * v.x;
          si += w * v.y;
        }
      }
    }
    const double2 j = jac(F, c, conj, f[c]);
    F.y[c] = fd(j.x + sr, j.y + si);
  }
}

// o_l = y + w D^-1 (f - A_beta y); level 0 writes `out0` (q: which = 0, z:
// which = 1) and, for z, the partials of ||z||^2
__global__ void __launch_bounds__(kThr) k_pc_vsmooth(const PcSys* __restrict__ sy, const PcState* __restrict__ stv,
                                                     double* __restrict__ part, int g0, int l, int which, int conj) {
  __shared__ double red[kThr / 64];
  const int k = g0 + blockIdx.y;
  if (!active(stv, k)) return;
  const PcSys& S = sy[k];
  if (l >= S.nlev - 1) return;
  const PcLevel& L = S.lev[l];
  const float2* __restrict__ f = level_in(S, l, which);
  const float2* __restrict__ in = L.y;
  float2* __restrict__ out = l > 0 ? L.o : (which ? S.z : S.q);
  double acc = 0.0;
  for (int c = blockIdx.x * kThr + threadIdx.x; c < L.n; c += gridDim.x * kThr) {
    int x, y, z;
    coords(L, c, x, y, z);
    const int plane = L.nx * L.ny;
    const float2 zero = make_float2(0.f, 0.f);
    const float2 xm = x > 0 ? in[c - 1] : zero, xp = x < L.nx - 1 ? in[c + 1] : zero;
    const float2 ym = y > 0 ? in[c - L.nx] : zero, yp = y < L.ny - 1 ? in[c + L.nx] : zero;
    const float2 zm = z > 0 ? in[c - plane] : zero, zp = z < L.nz - 1 ? in[c + plane] : zero;
    const float2 xc = in[c];
    const double2 d = diag_beta(S, L, c, conj);
    const double sr = (((double)xm.x + xp.x) + ((double)ym.x + yp.x)) + ((double)zm.x + zp.x);
    const double si = (((double)xm.y + xp.y) + ((double)ym.y + yp.y)) + ((double)zm.y + zp.y);
    const double ar = sr * L.h2inv + (d.x * xc.x - d.y * xc.y);
    const double ai = si * L.h2inv + (d.x * xc.y + d.y * xc.x);
    const float2 fc = f[c];
    const double2 corr = jac(L, c, conj, fd((double)fc.x - ar, (double)fc.y - ai));
    const float2 o = fd((double)xc.x + corr.x, (double)xc.y + corr.y);
    out[c] = o;
    acc += nrm(o);
  }
  if (l == 0 && which && part != nullptr) {
    const double tot = bsum(acc, red);
    if (threadIdx.x == 0) part[(size_t)k * kParts + blockIdx.x] = tot;
  }
}

// A V-cycle whose only level is level 0 (a grid too small or too thin to
// coarsen): kCoarseSweeps Jacobi steps on level 0 itself; the last result is
// copied to out0 with the partials of ||out0||^2 when which = 1.
__global__ void __launch_bounds__(kThr) k_pc_vsingle_out(const PcSys* __restrict__ sy, const PcState* __restrict__ stv,
                                                         double* __restrict__ part, int g0, int which) {
  __shared__ double red[kThr / 64];
  const int k = g0 + blockIdx.y;
  if (!active(stv, k)) return;
  const PcSys& S = sy[k];
  if (S.nlev != 1) return;
  const float2* __restrict__ src = coarse_out(S, 0);
  float2* __restrict__ out = which ? S.z : S.q;
  double acc = 0.0;
  for (int c = blockIdx.x * kThr + threadIdx.x; c < S.n; c += gridDim.x * kThr) {
    const float2 o = src[c];
    out[c] = o;
    acc += nrm(o);
  }
  if (which && part != nullptr) {
    const double tot = bsum(acc, red);
    if (threadIdx.x == 0) part[(size_t)k * kParts + blockIdx.x] = tot;
  }
}

// ---------------------------------------------------------------------------
// grid set-up and results
// ---------------------------------------------------------------------------

// w D^-1 of A_beta on one level for one frequency: w / (-6/h^2 + omega^2 (1 - i beta) m - i omega b)
__global__ void __launch_bounds__(kThr) k_pc_wdinv(const float* __restrict__ m, const float* __restrict__ b, int n,
                                                   double h2inv, double omega, float2* __restrict__ out) {
  for (int c = blockIdx.x * kThr + threadIdx.x; c < n; c += gridDim.x * kThr) {
    const double mm = m[c], bb = b[c];
    const double dr = -6.0 * h2inv + omega * omega * mm;
    const double di = -kBeta * omega * omega * mm - omega * bb;
    const double den = dr * dr + di * di;
    out[c] = fd(kJac * dr / den, -kJac * di / den);
  }
}

// b_0 = the sponge of the grid (float32)
__global__ void __launch_bounds__(kThr) k_pc_sponge(float* __restrict__ b, int nx, int ny, int nz, int nb,
                                                    double sp_scale, double inv_nb) {
  const int n = nx * ny * nz, plane = nx * ny;
  for (int c = blockIdx.x * kThr + threadIdx.x; c < n; c += gridDim.x * kThr) {
    const int z = c / plane, rem = c - z * plane, y = rem / nx, x = rem - y * nx;
    b[c] = (float)(sp_scale * ((sponge_axis_d(x, nx, nb, inv_nb) + sponge_axis_d(y, ny, nb, inv_nb)) +
                               sponge_axis_d(z, nz, nb, inv_nb)));
  }
}

// coarse = P^T fine / P^T 1 (weighted mean over the 27 fine cells)
__global__ void __launch_bounds__(kThr) k_pc_restrict_mean(const float* __restrict__ fine, float* __restrict__ coarse,
                                                           int fnx, int fny, int fnz, int cnx, int cny, int cnz) {
  const int n = cnx * cny * cnz, plane = cnx * cny;
  for (int c = blockIdx.x * kThr + threadIdx.x; c < n; c += gridDim.x * kThr) {
    const int cz = c / plane, rem = c - cz * plane, cy = rem / cnx, cx = rem - cy * cnx;
    double s = 0.0, wsum = 0.0;
    for (int dz = -1; dz <= 1; ++dz) {
      const int fz = 2 * cz + 1 + dz;
      if (fz < 0 || fz >= fnz) continue;
      for (int dy = -1; dy <= 1; ++dy) {
        const int fy = 2 * cy + 1 + dy;
        if (fy < 0 || fy >= fny) continue;
        for (int dx = -1; dx <= 1; ++dx) {
          const int fx = 2 * cx + 1 + dx;
          if (fx < 0 || fx >= fnx) continue;
          const double w = (dz ? 0.5 : 1.0) * (dy ? 0.5 : 1.0) * (dx ? 0.5 : 1.0);
          s += w * fine[((size_t)fz * fny + fy) * fnx + fx];
          wsum += w;
        }
      }
    }
    coarse[c] = (float)(s / wsum);
  }
}

// J = ||r1||^2 + ||r2||^2 (recurred), alpha_ls = (A u)[src] in float64
// (one block per system)
__global__ void __launch_bounds__(kThr) k_pc_final(const PcSys* __restrict__ sy, PcState* __restrict__ stv, int g0) {
  __shared__ double red[kThr / 64];
  const int k = g0 + blockIdx.x;
  const PcSys& S = sy[k];
  PcState& T = stv[k];
  double acc = 0.0;
  for (int c = threadIdx.x; c < S.n; c += kThr) acc += nrm(S.r[c]);
  for (int q = threadIdx.x; q < S.nr; q += kThr) acc += nrm(S.r2[q]);
  const double J = bsum(acc, red);
  if (threadIdx.x == 0) {
    T.J = J;
    if (S.est) {
      const double2 au = apply_cell(S, S.x, S.src, false);
      T.za = au;  // alpha_ls
    }
  }
}

// g = -sum over the grid's systems of 2 omega^2 Re(conj(u) r1); systems
// idx[0..cnt) in fixed order
__global__ void __launch_bounds__(kThr) k_pc_grad(const PcSys* __restrict__ sy, const int* __restrict__ idx, int cnt,
                                                  int n, float* __restrict__ g) {
  for (int c = blockIdx.x * kThr + threadIdx.x; c < n; c += gridDim.x * kThr) {
    double acc = 0.0;
    for (int i = 0; i < cnt; ++i) {
      const PcSys& S = sy[idx[i]];
      const float2 u = S.x[c], r = S.r[c];
      acc -= 2.0 * S.omega2 * ((double)u.x * r.x + (double)u.y * r.y);
    }
    g[c] = (float)acc;
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

struct LevelDims {
  int nx, ny, nz;
  double h;
};

// levels: halve every axis (n -> n/2) while all axes have >= 4 cells and the
// level holds more than kCoarsestCells cells
std::vector<LevelDims> levels_of(const wri_grid& g) {
  std::vector<LevelDims> v;
  LevelDims d{g.nx, g.ny, g.nz, g.h};
  v.push_back(d);
  while (std::min({d.nx, d.ny, d.nz}) >= 4 && (int64_t)d.nx * d.ny * d.nz > kCoarsestCells &&
         (int)v.size() < kMaxLev) {
    d = LevelDims{d.nx / 2, d.ny / 2, d.nz / 2, 2.0 * d.h};
    v.push_back(d);
  }
  return v;
}

int64_t cells_of(const LevelDims& d) { return (int64_t)d.nx * d.ny * d.nz; }

struct PcLayout {
  size_t sys = 0, state = 0, parts = 0, idx = 0, total = 0;
  std::vector<size_t> grid_arrays;   // per grid: m_l (l >= 1) and b_l (l >= 0)
  std::vector<std::pair<int, double>> pairs;   // distinct (grid, omega) of the systems
  std::vector<int> pair_of;                    // per system
  std::vector<size_t> pair_arrays;             // per pair: w D^-1 on every level
  std::vector<size_t> vec, rvec, rec;
};

PcLayout pc_layout(const wri_grid* grids, int n_grids, const wri_system* sys, int n_sys) {
  PcLayout L;
  size_t o = 0;
  auto take = [&](size_t b) { size_t r = o; o = al(o + std::max<size_t>(b, 1)); return r; };
  L.sys = take(sizeof(PcSys) * std::max(n_sys, 1));
  L.state = take(sizeof(PcState) * std::max(n_sys, 1));
  L.parts = take(sizeof(double) * (size_t)kParts * std::max(n_sys, 1));
  L.idx = take(sizeof(int) * std::max(n_sys, 1));
  L.grid_arrays.resize(n_grids);
  for (int g = 0; g < n_grids; ++g) {
    size_t b = 0;
    for (const auto& d : levels_of(grids[g])) b += 2 * al(sizeof(float) * (size_t)cells_of(d));
    L.grid_arrays[g] = take(b);
  }
  L.pair_of.assign(n_sys, -1);
  for (int k = 0; k < n_sys; ++k) {
    const std::pair<int, double> key(sys[k].grid, sys[k].omega);
    auto it = std::find(L.pairs.begin(), L.pairs.end(), key);
    L.pair_of[k] = (int)(it - L.pairs.begin());
    if (it == L.pairs.end()) L.pairs.push_back(key);
  }
  for (const auto& pr : L.pairs) {
    size_t b = 0;
    for (const auto& d : levels_of(grids[pr.first])) b += al(sizeof(float2) * (size_t)cells_of(d));
    L.pair_arrays.push_back(take(b));
  }
  L.vec.resize(n_sys);
  L.rvec.resize(n_sys);
  L.rec.resize(n_sys);
  for (int k = 0; k < n_sys; ++k) {
    const wri_grid& g = grids[sys[k].grid];
    const auto lv = levels_of(g);
    size_t b = 9 * al(sizeof(float2) * (size_t)cells_of(lv[0]));   // x r p q t s z res0 y0
    for (size_t l = 1; l < lv.size(); ++l) b += 4 * al(sizeof(float2) * (size_t)cells_of(lv[l]));
    L.vec[k] = take(b);
    L.rvec[k] = take(2 * al(sizeof(float2) * (size_t)sys[k].n_rec));
    L.rec[k] = take(sizeof(int) * (size_t)sys[k].n_rec);
  }
  L.total = o + kAl;
  return L;
}

int blocks_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + kThr - 1) / kThr, 1024)); }

int pc_run(const wri_grid* grids, int n_grids, const float* const* m, const wri_system* sys, int n_sys, int mode,
           int max_iter, int flags, double* J_out, float* const* grad, wri_c32* const* u_out, wri_result* res,
           void* ws, size_t ws_bytes, hipStream_t st) {
  int rc = wri_validate(grids, n_grids, sys, n_sys, mode, max_iter);
  if (rc != WRI_OK) return rc;
  if (n_sys > 0 && res == nullptr) return report_error(WRI_EINVAL, "res is NULL");
  if (flags & ~WRI_FLAG_NO_GRAPH)
    return report_error(WRI_EINVAL, "the preconditioned solver takes only WRI_FLAG_NO_GRAPH");
  if (n_grids > 0 && m == nullptr) return report_error(WRI_EINVAL, "m is NULL");
  for (int g = 0; g < n_grids; ++g)
    if (m[g] == nullptr || (grad != nullptr && grad[g] == nullptr))
      return report_error(WRI_EINVAL, "m[%d] or grad[%d] is NULL", g, g);
  const PcLayout L = pc_layout(grids, n_grids, sys, n_sys);
  if (ws == nullptr || ws_bytes < L.total)
    return report_error(WRI_ENOWS, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, L.total);
  char* base = reinterpret_cast<char*>(al(reinterpret_cast<uintptr_t>(ws)));
  if (J_out) *J_out = 0.0;
  // per-grid level arrays: b_0 from the sponge, m_l and b_l restricted
  std::vector<std::vector<const float*>> gm(n_grids), gb(n_grids);
  for (int g = 0; g < n_grids; ++g) {
    const wri_grid& G = grids[g];
    const auto lv = levels_of(G);
    char* p = base + L.grid_arrays[g];
    std::vector<float*> mm(lv.size()), bb(lv.size());
    for (size_t l = 0; l < lv.size(); ++l) {
      const size_t nb = al(sizeof(float) * (size_t)cells_of(lv[l]));
      mm[l] = reinterpret_cast<float*>(p);
      bb[l] = reinterpret_cast<float*>(p + nb);
      p += 2 * nb;
    }
    double sp = 0.0, inb = 0.0;
    if (G.nb > 0) {
      const double d0 = 3.0 * G.v_ref * std::log(1000.0) / (2.0 * G.nb * G.h);
      sp = 2.0 * d0 / (G.v_ref * G.v_ref);
      inb = 1.0 / G.nb;
    }
    hipLaunchKernelGGL(k_pc_sponge, dim3(blocks_for(cells_of(lv[0]))), dim3(kThr), 0, st, bb[0], G.nx, G.ny, G.nz,
                       G.nb, sp, inb);
    PC_HIP(hipGetLastError());
    gm[g].assign(lv.size(), nullptr);
    gb[g].assign(lv.size(), nullptr);
    gm[g][0] = m[g];
    gb[g][0] = bb[0];
    for (size_t l = 1; l < lv.size(); ++l) {
      const float* fm = (l == 1) ? m[g] : mm[l - 1];
      hipLaunchKernelGGL(k_pc_restrict_mean, dim3(blocks_for(cells_of(lv[l]))), dim3(kThr), 0, st, fm, mm[l],
                         lv[l - 1].nx, lv[l - 1].ny, lv[l - 1].nz, lv[l].nx, lv[l].ny, lv[l].nz);
      hipLaunchKernelGGL(k_pc_restrict_mean, dim3(blocks_for(cells_of(lv[l]))), dim3(kThr), 0, st, bb[l - 1], bb[l],
                         lv[l - 1].nx, lv[l - 1].ny, lv[l - 1].nz, lv[l].nx, lv[l].ny, lv[l].nz);
      PC_HIP(hipGetLastError());
      gm[g][l] = mm[l];
      gb[g][l] = bb[l];
    }
  }
  // w D^-1 per distinct (grid, frequency) and level
  std::vector<std::vector<const float2*>> pw(L.pairs.size());
  for (size_t q = 0; q < L.pairs.size(); ++q) {
    const int g = L.pairs[q].first;
    const double om = L.pairs[q].second;
    const auto lv = levels_of(grids[g]);
    char* p = base + L.pair_arrays[q];
    for (size_t l = 0; l < lv.size(); ++l) {
      float2* w = reinterpret_cast<float2*>(p);
      const int64_t nl = cells_of(lv[l]);
      hipLaunchKernelGGL(k_pc_wdinv, dim3(blocks_for(nl)), dim3(kThr), 0, st, gm[g][l], gb[g][l], (int)nl,
                         1.0 / (lv[l].h * lv[l].h), om, w);
      PC_HIP(hipGetLastError());
      pw[q].push_back(w);
      p += al(sizeof(float2) * (size_t)nl);
    }
  }
  if (n_sys == 0) {
    if (grad != nullptr)
      for (int g = 0; g < n_grids; ++g) PC_HIP(launch_zero_f32(grad[g], (size_t)grids[g].nx * grids[g].ny * grids[g].nz, st));
    PC_HIP(hipStreamSynchronize(st));
    return WRI_OK;
  }
  // systems in grid order; groups of consecutive systems on one grid
  std::vector<int> order(n_sys);
  for (int k = 0; k < n_sys; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return sys[a].grid < sys[b].grid; });
  struct Group { int grid, p0, cnt; int64_t n; };
  std::vector<Group> groups;
  std::vector<PcSys> hs(n_sys);
  for (int p = 0; p < n_sys; ++p) {
    const int k = order[p];
    const wri_system& s = sys[k];
    const wri_grid& g = grids[s.grid];
    const auto lv = levels_of(g);
    const int64_t n = cells_of(lv[0]);
    if (groups.empty() || groups.back().grid != s.grid) groups.push_back({s.grid, p, 0, n});
    groups.back().cnt++;
    PcSys& S = hs[p];
    S = PcSys{};
    const size_t vb = al(sizeof(float2) * (size_t)n);
    char* v = base + L.vec[k];
    auto vec = [&](int i) { return reinterpret_cast<float2*>(v + i * vb); };
    S.x = (u_out != nullptr && u_out[k] != nullptr) ? reinterpret_cast<float2*>(u_out[k]) : vec(0);
    S.r = vec(1); S.p = vec(2); S.q = vec(3); S.t = vec(4); S.s = vec(5); S.z = vec(6);
    char* cv = v + 9 * vb;
    for (size_t l = 0; l < lv.size(); ++l) {
      PcLevel& Lv = S.lev[l];
      Lv.nx = lv[l].nx; Lv.ny = lv[l].ny; Lv.nz = lv[l].nz; Lv.n = (int)cells_of(lv[l]);
      Lv.h2inv = 1.0 / (lv[l].h * lv[l].h);
      Lv.m = gm[s.grid][l];
      Lv.b = gb[s.grid][l];
      Lv.wdinv = pw[L.pair_of[k]][l];
      if (l == 0) {
        Lv.f = nullptr; Lv.o = nullptr;
        Lv.res = vec(7); Lv.y = vec(8);
      } else {
        const size_t cb = al(sizeof(float2) * (size_t)Lv.n);
        Lv.f = reinterpret_cast<float2*>(cv);
        Lv.y = reinterpret_cast<float2*>(cv + cb);
        Lv.o = reinterpret_cast<float2*>(cv + 2 * cb);
        Lv.res = reinterpret_cast<float2*>(cv + 3 * cb);
        cv += 4 * cb;
      }
    }
    if (lv.size() == 1) S.lev[0].o = vec(7);   // single-level cycle: Jacobi steps ping-pong between y and o
    S.nlev = (int)lv.size();
    const size_t rb = al(sizeof(float2) * (size_t)s.n_rec);
    S.r2 = reinterpret_cast<float2*>(base + L.rvec[k]);
    S.t2 = reinterpret_cast<float2*>(base + L.rvec[k] + rb);
    S.d = reinterpret_cast<const float2*>(s.d);
    int* drec = reinterpret_cast<int*>(base + L.rec[k]);
    if (s.n_rec > 0) PC_HIP(hipMemcpyAsync(drec, s.rec, sizeof(int) * s.n_rec, hipMemcpyHostToDevice, st));
    S.rec = drec;
    S.m = m[s.grid];
    S.n = (int)n; S.nx = g.nx; S.ny = g.ny; S.nz = g.nz; S.nb = g.nb; S.nr = s.n_rec;
    S.est = mode == WRI_ESTIMATE;
    S.max_iter = max_iter;
    S.src = s.src;
    S.lam = s.lambda;
    S.rtol2 = s.rtol * s.rtol;
    S.omega = s.omega;
    S.omega2 = s.omega * s.omega;
    S.h2inv = 1.0 / (g.h * g.h);
    if (g.nb > 0) {
      const double d0 = 3.0 * g.v_ref * std::log(1000.0) / (2.0 * g.nb * g.h);
      S.sp_scale = 2.0 * d0 / (g.v_ref * g.v_ref);
      S.inv_nb = 1.0 / g.nb;
    }
    S.alpha = make_double2(s.alpha.re, s.alpha.im);
  }
  PcSys* dsys = reinterpret_cast<PcSys*>(base + L.sys);
  PcState* dst = reinterpret_cast<PcState*>(base + L.state);
  double* parts = reinterpret_cast<double*>(base + L.parts);
  int* didx = reinterpret_cast<int*>(base + L.idx);
  std::vector<int> ident(n_sys);
  for (int p = 0; p < n_sys; ++p) ident[p] = p;
  PC_HIP(hipMemcpyAsync(dsys, hs.data(), sizeof(PcSys) * n_sys, hipMemcpyHostToDevice, st));
  PC_HIP(hipMemcpyAsync(didx, ident.data(), sizeof(int) * n_sys, hipMemcpyHostToDevice, st));
  PC_HIP(hipStreamSynchronize(st));  // host tables are read by the copies above

  // one V-cycle (which = 0: q = M p, 1: z = M^H s with the partials of ||z||^2)
  auto vcycle = [&](const Group& G, hipStream_t sq, int which) -> int {
    const int conj = which;
    const std::vector<LevelDims> lv = levels_of(grids[G.grid]);
    const int nl = (int)lv.size();
    for (int l = 0; l + 1 < nl; ++l) {
      hipLaunchKernelGGL(k_pc_vdown, dim3(blocks_for(cells_of(lv[l])), G.cnt), dim3(kThr), 0, sq, dsys, dst, G.p0,
                         l, which, conj);
      hipLaunchKernelGGL(k_pc_vrestrict, dim3(blocks_for(cells_of(lv[l + 1])), G.cnt), dim3(kThr), 0, sq, dsys, dst,
                         G.p0, l);
    }
    for (int j = 0; j < kCoarseSweeps; ++j)
      hipLaunchKernelGGL(k_pc_vcoarse, dim3(blocks_for(cells_of(lv[nl - 1])), G.cnt), dim3(kThr), 0, sq, dsys, dst,
                         G.p0, which, conj, j);
    if (nl == 1) {
      hipLaunchKernelGGL(k_pc_vsingle_out, dim3(kParts, G.cnt), dim3(kThr), 0, sq, dsys, dst, parts, G.p0, which);
    } else {
      for (int l = nl - 2; l >= 0; --l) {
        const int nbk = (l == 0) ? kParts : blocks_for(cells_of(lv[l]));
        hipLaunchKernelGGL(k_pc_vprolong, dim3(blocks_for(cells_of(lv[l])), G.cnt), dim3(kThr), 0, sq, dsys, dst,
                           G.p0, l, which, conj);
        hipLaunchKernelGGL(k_pc_vsmooth, dim3(nbk, G.cnt), dim3(kThr), 0, sq, dsys, dst, parts, G.p0, l, which, conj);
      }
    }
    PC_HIP(hipGetLastError());
    return WRI_OK;
  };
  auto iteration = [&](hipStream_t sq) -> int {
    for (const Group& G : groups) {
      const dim3 pg(kParts, G.cnt);
      hipLaunchKernelGGL(k_pc_pupd, pg, dim3(kThr), 0, sq, dsys, dst, G.p0);
      int e = vcycle(G, sq, 0);
      if (e != WRI_OK) return e;
      hipLaunchKernelGGL(k_pc_fwd, pg, dim3(kThr), 0, sq, dsys, dst, parts, G.p0);
      hipLaunchKernelGGL(k_pc_step, dim3(G.cnt), dim3(kThr), 0, sq, dsys, dst, parts, G.p0);
      hipLaunchKernelGGL(k_pc_rupd, pg, dim3(kThr), 0, sq, dsys, dst, G.p0);
      hipLaunchKernelGGL(k_pc_adj, pg, dim3(kThr), 0, sq, dsys, dst, parts, G.p0);
      hipLaunchKernelGGL(k_pc_check, dim3(G.cnt), dim3(kThr), 0, sq, dsys, dst, parts, G.p0, 0);
      e = vcycle(G, sq, 1);
      if (e != WRI_OK) return e;
      hipLaunchKernelGGL(k_pc_beta, dim3(G.cnt), dim3(kThr), 0, sq, dsys, dst, parts, G.p0, 0);
      PC_HIP(hipGetLastError());
    }
    return WRI_OK;
  };
  // set-up: x = 0, r = b, s_0 = S^H b, z_0 = M^H s_0, p_0 = z_0
  for (const Group& G : groups) {
    const dim3 pg(kParts, G.cnt);
    hipLaunchKernelGGL(k_pc_zero, pg, dim3(kThr), 0, st, dsys, G.p0);
    hipLaunchKernelGGL(k_pc_init, dim3(G.cnt), dim3(kThr), 0, st, dsys, dst, G.p0);
    hipLaunchKernelGGL(k_pc_adj, pg, dim3(kThr), 0, st, dsys, dst, parts, G.p0);
    hipLaunchKernelGGL(k_pc_check, dim3(G.cnt), dim3(kThr), 0, st, dsys, dst, parts, G.p0, 1);
    rc = vcycle(G, st, 1);
    if (rc != WRI_OK) return rc;
    hipLaunchKernelGGL(k_pc_beta, dim3(G.cnt), dim3(kThr), 0, st, dsys, dst, parts, G.p0, 1);
    PC_HIP(hipGetLastError());
  }
  std::vector<PcState> hst(n_sys);
  auto read = [&]() -> int {
    PC_HIP(hipMemcpyAsync(hst.data(), dst, sizeof(PcState) * n_sys, hipMemcpyDeviceToHost, st));
    PC_HIP(hipStreamSynchronize(st));
    return WRI_OK;
  };
  if ((rc = read()) != WRI_OK) return rc;
  const bool use_graph = !(flags & WRI_FLAG_NO_GRAPH);
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  auto drop_graph = [&]() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  };
  int64_t done = 0;
  while (true) {
    bool any = false;
    for (const auto& T : hst) any = any || (T.status == kActive);
    if (!any) break;
    if (done > (int64_t)max_iter + kCheck) {
      drop_graph();
      return report_error(WRI_EHIP, "internal: systems still active after max_iter iterations");
    }
    if (use_graph) {
      if (exec == nullptr) {
        hipStream_t cs = nullptr;
        PC_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipError_t eb = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (eb != hipSuccess) {
          (void)hipStreamDestroy(cs);
          return report_error(WRI_EHIP, "hipStreamBeginCapture: %s", hipGetErrorString(eb));
        }
        int e = WRI_OK;
        for (int i = 0; i < kCheck && e == WRI_OK; ++i) e = iteration(cs);
        const hipError_t ee = hipStreamEndCapture(cs, &graph);
        (void)hipStreamDestroy(cs);
        if (e != WRI_OK) { drop_graph(); return e; }
        if (ee != hipSuccess) { drop_graph(); return report_error(WRI_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(ee)); }
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ei != hipSuccess) { drop_graph(); return report_error(WRI_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(ei)); }
      }
      const hipError_t el = hipGraphLaunch(exec, st);
      if (el != hipSuccess) { drop_graph(); return report_error(WRI_EHIP, "hipGraphLaunch: %s", hipGetErrorString(el)); }
    } else {
      for (int i = 0; i < kCheck; ++i) {
        rc = iteration(st);
        if (rc != WRI_OK) return rc;
      }
    }
    done += kCheck;
    if ((rc = read()) != WRI_OK) { drop_graph(); return rc; }
  }
  drop_graph();
  // results: J, alpha_ls, gradient per grid
  for (const Group& G : groups)
    hipLaunchKernelGGL(k_pc_final, dim3(G.cnt), dim3(kThr), 0, st, dsys, dst, G.p0);
  PC_HIP(hipGetLastError());
  if (grad != nullptr) {
    for (int g = 0; g < n_grids; ++g) {
      const Group* G = nullptr;
      for (const auto& gg : groups)
        if (gg.grid == g) G = &gg;
      const int64_t n = (int64_t)grids[g].nx * grids[g].ny * grids[g].nz;
      if (G == nullptr) {
        PC_HIP(launch_zero_f32(grad[g], (size_t)n, st));
        continue;
      }
      hipLaunchKernelGGL(k_pc_grad, dim3(blocks_for(n)), dim3(kThr), 0, st, dsys, didx + G->p0, G->cnt, (int)n,
                         grad[g]);
      PC_HIP(hipGetLastError());
    }
  }
  if ((rc = read()) != WRI_OK) return rc;
  int ret = WRI_OK;
  double J = 0.0;
  for (int p = 0; p < n_sys; ++p) {
    const int k = order[p];
    const PcState& T = hst[p];
    wri_result& r = res[k];
    r.iters = T.iters;
    r.status = T.status;
    r.relres = (T.ss0 > 0.0) ? std::sqrt(std::max(T.ss, 0.0) / T.ss0) : 0.0;
    r.J = T.J;
    if (mode == WRI_ESTIMATE) {
      r.alpha.re = T.xa.x; r.alpha.im = T.xa.y;
      r.alpha_ls.re = T.za.x; r.alpha_ls.im = T.za.y;
    } else {
      r.alpha = sys[k].alpha;
      r.alpha_ls = sys[k].alpha;
    }
    J += T.J;
    if (T.status == kBreakdown) ret = WRI_EBREAKDOWN;
    else if ((T.status == kMaxIter || T.status == kDiverged) && ret == WRI_OK) ret = WRI_NOT_CONVERGED;
  }
  if (J_out) *J_out = J;
  if (ret == WRI_EBREAKDOWN) report_error(WRI_EBREAKDOWN, "at least one system broke down");
  return ret;
}

}  // namespace
}  // namespace wri

using namespace wri;

extern "C" {

size_t wri_precond_workspace_bytes(const wri_grid* grids, int32_t n_grids, const wri_system* sys, int32_t n_sys,
                                   int32_t mode) {
  if (wri_validate(grids, n_grids, sys, n_sys, mode, 0) != WRI_OK) return 0;
  return pc_layout(grids, n_grids, sys, n_sys).total;
}

int wri_objective_grad_precond(const wri_grid* grids, int32_t n_grids, const float* const* m, const wri_system* sys,
                               int32_t n_sys, int32_t mode, int32_t max_iter, int32_t flags, double* J_out,
                               float* const* grad, wri_c32* const* u_out, wri_result* res, void* ws, size_t ws_bytes,
                               void* stream) {
  try {
    return pc_run(grids, n_grids, m, sys, n_sys, mode, max_iter, flags, J_out, grad, u_out, res, ws, ws_bytes,
                  reinterpret_cast<hipStream_t>(stream));
  } catch (const std::exception& e) {
    return report_error(WRI_EINVAL, "exception: %s", e.what());
  }
}

}  // extern "C"
