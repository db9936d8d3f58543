// HIP kernels (gfx950) of the augmented-wavefield solver.
//
// The hot loop is CGLS on S = [[A, -e],[lambda P, 0]] (KNOWN: [A; lambda P]),
// the conjugate-gradient-on-the-normal-equations reading of the paper's
// Algorithm 1, whose cost is dominated by the products S p and S^H r
// ("GPU acceleration" section).  Each iteration is two fused, bandwidth-bound
// launches over every active system:
//
//   fwd (k):  p_k = s_k + beta_k p_{k-1};  on even k >= 2 (and when the
//             system stops) x += a_{k-2} p_{k-2} + a_{k-1} p_{k-1}, the two
//             pending steps (p_{k-2} still sits in the buffer p_k overwrites);
//             t = S p_k (7-point stencil + source column + receiver gather);
//             float64 partials of ||t||^2.
//   adj (k):  a_k = gamma_k / ||t||^2;  r_{k+1} = r_k - a_k t;
//             s_{k+1} = S^H r_{k+1} (stencil + receiver scatter, s_alpha = -r1[src]);
//             float64 partials of ||s_{k+1}||^2.
//
// A workgroup owns a 64 x TY x TZ slab tile of one system: lanes run along x
// (coalesced 512-byte rows of complex64), waves stack along y, and the tile
// marches along z with the (z-1, z, z+1) column values in registers and the
// current x-y plane (plus a one-cell halo) in LDS.  The neighbour values of the
// updated vector (p_k in fwd, r_{k+1} in adj) are recomputed from the stored
// inputs at halo cells, so the updated vector never needs a grid-wide barrier
// before the stencil.
//
// Scalars: every workgroup of a system sums the previous launch's per-tile
// partials in the same fixed order, so all workgroups derive bit-identical
// float64 scalars (no atomics, deterministic for a given tiling).
#include "wri_impl.hpp"
#include "stencil.hpp"

#include <cfloat>
#include <climits>

namespace wri {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

// Vector pointers read from the device-resident system table are generic
// (flat) to the compiler; flat accesses also count against the LDS wait
// counter, which ties every LDS wait to the outstanding HBM loads.  All solver
// vectors live in global memory, so the fused kernels access them through
// address-space-1 pointers (global_load / global_store).
#define GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ GLOBAL T* gptr(T* p) { return (GLOBAL T*)p; }
template <class T>
__device__ __forceinline__ const GLOBAL T* gptr(const T* p) { return (const GLOBAL T*)p; }
// 8-byte element access through a global pointer (one dwordx2 load/store)
__device__ __forceinline__ float2 ld2(const GLOBAL float2* p, int i) {
  return __builtin_bit_cast(float2, *((const GLOBAL unsigned long long*)p + i));
}
__device__ __forceinline__ void st2(GLOBAL float2* p, int i, float2 v) {
  *((GLOBAL unsigned long long*)p + i) = __builtin_bit_cast(unsigned long long, v);
}
// Stores of values that no other workgroup reads in the same launch (every
// output of the fused kernels) carry the non-temporal hint: measured about
// 1.5 % faster on the forward kernel and 1 % on the adjoint.  (The same hint on
// loads of halo-free inputs was slower.)
__device__ __forceinline__ void st2s(GLOBAL float2* p, int i, float2 v) {
  __builtin_nontemporal_store(__builtin_bit_cast(unsigned long long, v), (GLOBAL unsigned long long*)p + i);
}
__device__ __forceinline__ int2 ld2i(const GLOBAL int2* p, int i) {
  return __builtin_bit_cast(int2, *((const GLOBAL unsigned long long*)p + i));
}

// Block order inside a group: system-major (tile_major 0: all tiles of one
// system, then the next), tile-major over all systems (1), or tile-major
// within bundles of tile_major >= 2 systems (the same tile of the bundle's
// systems on consecutive blocks, so the bundle shares m and its halo rows in
// L2; the last bundle may be smaller).
__device__ __forceinline__ void block_map(const GroupDesc& d, int local, int* rl, int* tile) {
  const int n = d.nrhs, nt = d.ntiles, ord = d.tile_major;
  if (ord == 0) {
    *rl = local / nt;
    *tile = local - *rl * nt;
    return;
  }
  const int bsz = (ord == 1 || ord > n) ? n : ord;
  const int full = n / bsz, span = bsz * nt;
  const int b = local / span;
  if (b < full) {
    const int w = local - b * span;
    *tile = w / bsz;
    *rl = b * bsz + (w - *tile * bsz);
  } else {
    const int bt = n - full * bsz;
    const int w = local - full * span;
    *tile = w / bt;
    *rl = full * bsz + (w - *tile * bt);
  }
}

__device__ __forceinline__ int xcd_remap(int b, int nb, int q) {
  // Blocks go round-robin to the XCDs (b % 8).  The logical sequence of
  // (group, system, tile) is cut into chunks of q consecutive tiles, dealt to the
  // XCDs round-robin as well: the tiles of a chunk are spatial neighbours on
  // one XCD (halo re-reads hit its L2), and every XCD holds a share of every
  // system, so no XCD idles while others still work when some systems of the
  // batch have converged.  Blocks past the last complete round keep their index.
  const int xcd = b % kXCD, local = b / kXCD;
  const int full = nb / (kXCD * q) * (kXCD * q);
  if (b >= full) return b;
  const int round = local / q, off = local - round * q;
  return (round * kXCD + xcd) * q + off;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of n partials by one wave in a fixed order, broadcast to the block.
template <int NW>
__device__ __forceinline__ double block_sum_slots(const double* __restrict__ p, int n, double* red) {
  const int tid = threadIdx.x;
  if (tid < 64) {
    double v = 0.0;
    for (int i = tid; i < n; i += 64) v += p[i];
    v = wave_sum(v);
    if (tid == 0) red[NW] = v;
  }
  __syncthreads();
  const double r = red[NW];
  __syncthreads();
  return r;
}

// Block reduction; the result is valid in thread 0 only.
template <int NW>
__device__ __forceinline__ double block_reduce(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NW; ++i) r += red[i];
  }
  __syncthreads();
  return r;
}

// Squared sponge depth along one axis, in units of nb (0 outside the sponge).
__device__ __forceinline__ float sponge_axis(int i, int n, int nb, float inv_nb) {
  const int d = max(0, max(nb - i, i - (n - 1 - nb)));
  const float f = (float)d * inv_nb;
  return f * f;
}
// sponge_axis_d, helm and round2 (the stencil arithmetic) live in stencil.hpp

__device__ __forceinline__ float2 f2(float a, float b) { return make_float2(a, b); }
// y + a x as one float64 fused multiply-add, rounded once to complex float32
__device__ __forceinline__ float2 axpy2(float2 y, double a, float2 x) {
  return f2((float)fma(a, (double)x.x, (double)y.x), (float)fma(a, (double)x.y, (double)y.y));
}
// x + c2 p2 + c1 p1 in float64 arithmetic, rounded once (the x update that
// takes two CGLS steps at a time; with c2 = 0 and finite p2 it equals axpy2(x, c1, p1))
__device__ __forceinline__ float2 xupd2(float2 x, double c2, float2 p2, double c1, float2 p1) {
  return f2((float)fma(c1, (double)p1.x, fma(c2, (double)p2.x, (double)x.x)),
            (float)fma(c1, (double)p1.y, fma(c2, (double)p2.y, (double)x.y)));
}
__device__ __forceinline__ double norm2d(float2 v) {
  return (double)v.x * (double)v.x + (double)v.y * (double)v.y;
}

// ---------------------------------------------------------------------------
// initialisation: x = 0, p0 = 0, r1 = b1 (KNOWN: alpha e; ESTIMATE: 0),
// r2 = lambda d, state reset.  grid = (blocks per system, nsys).
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_init(const SysDev* __restrict__ sysv, SysState* __restrict__ stv,
                                              int warm, int rhs_rec) {
  const int rhs = blockIdx.y;
  const SysDev& S = sysv[rhs];
  const int n = S.nx * S.ny * S.nz;
  const float2 z = f2(0.f, 0.f);
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    if (!warm) S.x[c] = z;
    S.p[0][c] = z;
    float2 r = z;
    if (S.mode == 0 && !rhs_rec && c == S.src) r = f2((float)S.alpha.x, (float)S.alpha.y);
    S.r[1][c] = r;
  }
  if (blockIdx.x == 0) {
    for (int q = threadIdx.x; q < S.n_rec; q += blockDim.x) {
      const float2 dq = S.d[q];
      S.r2[q] = f2((float)(S.lam_d * dq.x), (float)(S.lam_d * dq.y));
      S.t2[q] = z;
    }
    if (threadIdx.x == 0) {
      SysState* T = stv + rhs;
      T->gamma[0] = T->gamma[1] = 0.0;
      T->gmin[0] = T->gmin[1] = 0.0;
      T->gamma0 = 0.0;
      T->a[0] = T->a[1] = 0.0;
      // warm start in ESTIMATE mode: the unknown is alpha / c
      T->xa = (warm && S.mode == 1) ? make_double2(S.alpha.x / S.alpha_c, S.alpha.y / S.alpha_c)
                                    : make_double2(0.0, 0.0);
      T->pa = make_double2(0.0, 0.0);
      T->sa = make_double2(0.0, 0.0);
      T->J = 0.0;
      T->alpha_ls = make_double2(0.0, 0.0);
      T->iterA = 0;
      T->iterB = -1;
      T->status = kActive;
      T->iters = 0;
      T->brk = 0;
      T->warm = warm;
    }
  }
}

// Receiver sources: r1 = P^H d, the observed-data values placed at the
// receiver cells (stream-ordered after k_init has zeroed r1; the cells of one
// system are distinct).  grid = nsys blocks.
__global__ void __launch_bounds__(256) k_rhs_at_receivers(const SysDev* __restrict__ sysv) {
  const SysDev& S = sysv[blockIdx.x];
  for (int q = threadIdx.x; q < S.n_rec; q += blockDim.x) S.r[1][S.rec[q]] = S.d[q];
}

hipError_t launch_init(const SysDev* sys, SysState* st, int nsys, hipStream_t s, int warm, int rhs_rec) {
  if (nsys <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_init, dim3(256, nsys), dim3(256), 0, s, sys, st, warm, rhs_rec);
  if (rhs_rec) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rhs_at_receivers, dim3(nsys), dim3(256), 0, s, sys);
  }
  return hipGetLastError();
}

// Warm start, after a set-up adjoint pass on r = b: gamma0 = ||S^H b||^2 from
// that pass's partials (summed by one wave in a fixed order), then
// r1 = b1 - (A x0 - c xa e) and r2 = lambda (d - P x0).  b = 0 (gamma0 = 0)
// has the solution 0: x0 and xa are zeroed instead, so the solve ends with the
// zero-right-hand-side status.  grid = (blocks, nsys).
__global__ void __launch_bounds__(256) k_warm_residual(const SysDev* __restrict__ sysv, SysState* __restrict__ stv,
                                                      const double* __restrict__ part_s,
                                                      const int* __restrict__ nparts) {
  __shared__ double g0s;
  const int rhs = blockIdx.y;
  const SysDev& S = sysv[rhs];
  SysState* T = stv + rhs;
  if (threadIdx.x < 64) {
    double v = 0.0;
    for (int i = threadIdx.x; i < nparts[rhs]; i += 64) v += part_s[S.slot_base + i];
    v = wave_sum(v);
    if (threadIdx.x == 0) g0s = v;
  }
  __syncthreads();
  const double g0 = g0s;
  const double2 xa = T->xa;  // read by every block before block 0 may clear it
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    T->gamma0 = g0;
    if (g0 == 0.0) T->xa = make_double2(0.0, 0.0);
  }
  const int nx = S.nx, ny = S.ny, nz = S.nz, plane = nx * ny, n = plane * nz;
  const float2 z = f2(0.f, 0.f);
  const double w2 = S.omega_d * S.omega_d;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    if (g0 == 0.0) {
      S.x[c] = z;
      continue;
    }
    const int x = c % nx, y = (c / nx) % ny, zz = c / plane;
    const float2 xc = S.x[c];
    const float2 xm = x > 0 ? S.x[c - 1] : z, xp = x + 1 < nx ? S.x[c + 1] : z;
    const float2 ym = y > 0 ? S.x[c - nx] : z, yp = y + 1 < ny ? S.x[c + nx] : z;
    const float2 zm = zz > 0 ? S.x[c - plane] : z, zp = zz + 1 < nz ? S.x[c + plane] : z;
    const double b = S.sp_scale_d * (sponge_axis_d(x, nx, S.nb, S.inv_nb_d) + sponge_axis_d(y, ny, S.nb, S.inv_nb_d) +
                                     sponge_axis_d(zz, nz, S.nb, S.inv_nb_d));
    double2 ax = helm(xc, xm, xp, ym, yp, zm, zp, S.h2inv_d, w2 * (double)S.m[c], -(S.omega_d * b));
    if (S.mode == 1 && c == S.src) {  // the source column: A x - c xa e
      ax.x -= S.alpha_c * xa.x;
      ax.y -= S.alpha_c * xa.y;
    }
    const float2 r = S.r[1][c];
    S.r[1][c] = f2((float)((double)r.x - ax.x), (float)((double)r.y - ax.y));
  }
  if (blockIdx.x == 0 && g0 != 0.0) {
    for (int q = threadIdx.x; q < S.n_rec; q += blockDim.x) {
      const float2 xq = S.x[S.rec[q]];
      const float2 r2 = S.r2[q];
      S.r2[q] = f2((float)((double)r2.x - S.lam_d * (double)xq.x), (float)((double)r2.y - S.lam_d * (double)xq.y));
    }
  }
}

hipError_t launch_warm_residual(const SysDev* sys, SysState* st, const double* part_s, const int* nparts, int nsys,
                                hipStream_t s) {
  if (nsys <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_warm_residual, dim3(256, nsys), dim3(256), 0, s, sys, st, part_s, nparts);
  return hipGetLastError();
}

// A change of tiling between two iterations: the adjoint pass of the old
// tiling left the partials of ||s_k||^2 in n_old slots per system.  They are
// folded into slot 0 in the order in which the forward pass sums its slots
// (lane 0's value of the same wave sum), and the slots up to n_new are
// cleared, so the forward pass of the new tiling sums exactly the same
// gamma_k.  grid = one 64-thread block per system of a group.
__global__ void __launch_bounds__(64) k_fold_partials(const SysDev* __restrict__ sysv, double* __restrict__ part_s,
                                                     int rhs0, int n_old, int n_new) {
  double* __restrict__ p = part_s + sysv[rhs0 + blockIdx.x].slot_base;
  double v = 0.0;
  for (int i = threadIdx.x; i < n_old; i += 64) v += p[i];
  v = wave_sum(v);
  const int n = max(n_old, n_new);
  for (int i = threadIdx.x; i < n; i += 64) p[i] = (i == 0) ? v : 0.0;
}

hipError_t launch_fold_partials(const SysDev* sys, double* part_s, int rhs0, int nrhs, int n_old, int n_new,
                                hipStream_t s) {
  if (nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fold_partials, dim3(nrhs), dim3(64), 0, s, sys, part_s, rhs0, n_old, n_new);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Tile geometry shared by the fused kernels
// ---------------------------------------------------------------------------

template <int W, int RY>
struct TileCtx {
  static constexpr int TY = W * RY;
  static constexpr int LX = kTX + 2;
  static constexpr int LY = TY + 2;
  static constexpr int NH = 2 * LX + 2 * TY;  // halo cells of one plane
  int x0, y0, z0, z1;
  int gx;
  int gy[RY];
  bool in[RY];
  int plane;  // nx*ny

  __device__ void setup(const SysDev& S, int tile, int lane, int w, int tiles_x, int tiles_y, int tz) {
    const int txi = tile % tiles_x;
    const int rem = tile / tiles_x;
    const int tyi = rem % tiles_y;
    const int tzi = rem / tiles_y;
    x0 = txi * kTX;
    y0 = tyi * TY;
    z0 = tzi * tz;
    z1 = min(z0 + tz, S.nz);
    gx = x0 + lane;
    plane = S.nx * S.ny;
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      gy[j] = y0 + w * RY + j;
      in[j] = (gx < S.nx) && (gy[j] < S.ny);
    }
  }
  // LDS halo slot h -> (hx, hy) in LDS coordinates
  __device__ static void halo_xy(int h, int& hx, int& hy) {
    if (h < LX) { hx = h; hy = 0; }
    else if (h < 2 * LX) { hx = h - LX; hy = LY - 1; }
    else { const int h2 = h - 2 * LX; hy = 1 + (h2 >> 1); hx = (h2 & 1) ? (LX - 1) : 0; }
  }
};

// Per-thread receiver cursors for its RY columns.
template <int RY>
struct RecCursor {
  int cur[RY], end[RY], nz_[RY];
  __device__ void setup(const SysDev& S, int gx, const int* gy, const bool* in, int z0) {
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      cur[j] = 0; end[j] = 0; nz_[j] = INT_MAX;
      if (S.colmap != nullptr && in[j]) {
        const int2 be = ld2i(gptr(S.colmap), gy[j] * S.nx + gx);
        int c = be.x;
        while (c < be.y && ld2i(gptr(S.entries), c).x < z0) ++c;
        cur[j] = c; end[j] = be.y;
        nz_[j] = (c < be.y) ? ld2i(gptr(S.entries), c).x : INT_MAX;
      }
    }
  }
  __device__ int take(const SysDev& S, int j) {  // receiver index at the current z; advance
    const int q = ld2i(gptr(S.entries), cur[j]).y;
    ++cur[j];
    nz_[j] = (cur[j] < end[j]) ? ld2i(gptr(S.entries), cur[j]).x : INT_MAX;
    return q;
  }
};

// ---------------------------------------------------------------------------
// fused forward kernel: x update, p update, t = S p, ||t||^2 partials
// ---------------------------------------------------------------------------

template <int W, int RY>
__global__ void __launch_bounds__(64 * W)
k_fwd(const SysDev* __restrict__ sysv, SysState* __restrict__ stv, const double* __restrict__ part_s,
      double* __restrict__ part_d, const GroupDesc* __restrict__ gd, int ngroups) {
  using Ctx = TileCtx<W, RY>;
  __shared__ float2 pl[2][Ctx::LY][Ctx::LX];
  __shared__ double red[W + 1];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int logical = xcd_remap(blockIdx.x, gridDim.x, gd[0].xchunk);
  int g = 0;
  while (g + 1 < ngroups && logical >= gd[g + 1].block0) ++g;
  const int ntiles = gd[g].ntiles, tiles_x = gd[g].tiles_x, tiles_y = gd[g].tiles_y, tz = gd[g].tz;
  const int local = logical - gd[g].block0;
  int rl, tile;
  block_map(gd[g], local, &rl, &tile);
  const int rhs = gd[g].rhs0 + rl;
  const SysDev& S = sysv[rhs];
  SysState* T = stv + rhs;
  if (T->status != kActive) return;
  const int k = T->iterA;

  const double gk = block_sum_slots<W>(part_s + S.slot_base, ntiles, red);
  const bool warm = T->warm != 0;  // gamma0 = ||S^H b||^2 was set by the warm-start set-up
  const double g0 = (k == 0 && !warm) ? gk : T->gamma0;
  const double gmin = (k == 0) ? gk : T->gmin[(k - 1) & 1];
  // brk: the adjoint launch of this same k broke down; this launch only finishes x
  const bool brk = T->brk != 0;
  const bool stop = brk || (g0 == 0.0) || (gk <= S.rtol2 * g0) || (k >= S.max_iter) || (gk > kDivergeRatio * gmin);
  const double beta = (k == 0) ? 0.0 : gk / T->gamma[(k - 1) & 1];
  const double aprev = (k == 0) ? 0.0 : T->a[(k - 1) & 1];
  // x takes the pending steps on even iterations and when the system stops:
  // c1 p_{k-1} (+ c2 p_{k-2} at even k >= 2; a_{k-2} is still in a[k & 1]).
  // After a breakdown this k already ran once: only an odd k left a step pending.
  const bool xstep = brk ? (k & 1) == 1 : stop ? (k >= 1) : (k >= 2 && (k & 1) == 0);
  const double c1 = xstep ? aprev : 0.0;
  const double c2 = (xstep && !brk && k >= 2 && (k & 1) == 0) ? T->a[k & 1] : 0.0;
  if (tile == 0 && tid == 0) {
    T->gamma[k & 1] = gk;
    T->gmin[k & 1] = fmin(gmin, gk);
    if (k == 0 && !warm) T->gamma0 = gk;
    T->iterB = k;
  }

  Ctx C;
  C.setup(S, tile, lane, w, tiles_x, tiles_y, tz);
  const int plane = C.plane;
  const double bf = beta;
  const double w2 = S.omega_d * S.omega_d;
  const GLOBAL float2* __restrict__ sv = gptr((const float2*)S.s);
  const GLOBAL float2* __restrict__ po = gptr((const float2*)S.p[k & 1]);
  GLOBAL float2* __restrict__ pn = gptr(S.p[(k + 1) & 1]);
  GLOBAL float2* __restrict__ xv = gptr(S.x);
  const GLOBAL float* __restrict__ mv = gptr(S.m);
  GLOBAL float2* __restrict__ tout = gptr(S.t);
  GLOBAL float2* __restrict__ t2v = gptr(S.t2);

  // source cell: which of my rows (if any) holds it
  const int sxy = S.src % plane, sz = S.src / plane;
  const int sx = sxy % S.nx, sy = sxy / S.nx;
  int srcj = -1;
  if (S.mode == 1 && sx == C.gx && sz >= C.z0 && sz < C.z1) {
#pragma unroll
    for (int j = 0; j < RY; ++j)
      if (C.gy[j] == sy) srcj = j;
  }

  if (stop) {
    // finish x with the pending steps; the adjoint kernel records the status
    if (xstep) {
      for (int z = C.z0; z < C.z1; ++z) {
#pragma unroll
        for (int j = 0; j < RY; ++j) {
          if (!C.in[j]) continue;
          const int c = z * plane + C.gy[j] * S.nx + C.gx;
          const float2 p2 = (c2 != 0.0) ? ld2(pn, c) : f2(0.f, 0.f);
          st2s(xv, c, xupd2(ld2(xv, c), c2, p2, c1, ld2(po, c)));
        }
      }
      if (srcj >= 0 && !brk) {
        const double2 pa = T->pa;
        T->xa = make_double2(T->xa.x + aprev * pa.x, T->xa.y + aprev * pa.y);
      }
    }
    return;
  }

  // source-weight direction p_a = s_a + beta p_a (owned by the source thread)
  double2 pa_new = make_double2(0.0, 0.0);
  if (srcj >= 0) {
    const double2 pa = T->pa, sa = T->sa;
    pa_new = make_double2(sa.x + beta * pa.x, sa.y + beta * pa.y);
    T->xa = make_double2(T->xa.x + aprev * pa.x, T->xa.y + aprev * pa.y);
  }

  RecCursor<RY> rc;
  rc.setup(S, C.gx, C.gy, C.in, C.z0);

  double sxy2[RY];
  const double sx2 = sponge_axis_d(C.gx, S.nx, S.nb, S.inv_nb_d);
#pragma unroll
  for (int j = 0; j < RY; ++j) sxy2[j] = sx2 + sponge_axis_d(C.gy[j], S.ny, S.nb, S.inv_nb_d);

  auto pval = [&](int c) -> float2 { return axpy2(ld2(sv, c), bf, ld2(po, c)); };

  float2 pm[RY], pc[RY], pnx[RY], poc[RY], pon[RY];
  // plane z0 - 1 and z0
#pragma unroll
  for (int j = 0; j < RY; ++j) {
    pm[j] = f2(0.f, 0.f);
    pc[j] = f2(0.f, 0.f);
    poc[j] = f2(0.f, 0.f);
    if (C.in[j]) {
      const int c = C.z0 * plane + C.gy[j] * S.nx + C.gx;
      if (C.z0 > 0) pm[j] = pval(c - plane);
      poc[j] = ld2(po, c);
      pc[j] = axpy2(ld2(sv, c), bf, poc[j]);
    }
    pl[0][1 + w * RY + j][1 + lane] = pc[j];
  }
  for (int h = tid; h < Ctx::NH; h += 64 * W) {
    int hx, hy;
    Ctx::halo_xy(h, hx, hy);
    const int xx = C.x0 + hx - 1, yy = C.y0 + hy - 1;
    float2 v = f2(0.f, 0.f);
    if (xx >= 0 && xx < S.nx && yy >= 0 && yy < S.ny) v = pval(C.z0 * plane + yy * S.nx + xx);
    pl[0][hy][hx] = v;
  }
  __syncthreads();

  double acc = 0.0;
  int cur = 0;
  for (int z = C.z0; z < C.z1; ++z) {
    const int nxt = cur ^ 1;
    const bool has_next = (z + 1) < S.nz;
    // plane z+1: own cells and halo
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      pnx[j] = f2(0.f, 0.f);
      pon[j] = f2(0.f, 0.f);
      if (C.in[j] && has_next) {
        const int c = (z + 1) * plane + C.gy[j] * S.nx + C.gx;
        pon[j] = ld2(po, c);
        pnx[j] = axpy2(ld2(sv, c), bf, pon[j]);
      }
    }
    for (int h = tid; h < Ctx::NH; h += 64 * W) {
      int hx, hy;
      Ctx::halo_xy(h, hx, hy);
      const int xx = C.x0 + hx - 1, yy = C.y0 + hy - 1;
      float2 v = f2(0.f, 0.f);
      if (has_next && xx >= 0 && xx < S.nx && yy >= 0 && yy < S.ny)
        v = pval((z + 1) * plane + yy * S.nx + xx);
      pl[nxt][hy][hx] = v;
    }
#pragma unroll
    for (int j = 0; j < RY; ++j) pl[nxt][1 + w * RY + j][1 + lane] = pnx[j];

    // t = S p at plane z
    const double sz2 = sponge_axis_d(z, S.nz, S.nb, S.inv_nb_d);
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      if (!C.in[j]) continue;
      const int ly = w * RY + j;
      const int c = z * plane + C.gy[j] * S.nx + C.gx;
      const float2 xm = pl[cur][ly + 1][lane];
      const float2 xp = pl[cur][ly + 1][lane + 2];
      const float2 ym = (j > 0) ? pc[j > 0 ? j - 1 : 0] : pl[cur][ly][lane + 1];
      const float2 yp = (j < RY - 1) ? pc[j < RY - 1 ? j + 1 : 0] : pl[cur][ly + 2][lane + 1];
      const double b = S.sp_scale_d * (sxy2[j] + sz2);
      double2 td = helm(pc[j], xm, xp, ym, yp, pm[j], pnx[j], S.h2inv_d, w2 * (double)mv[c], -(S.omega_d * b));
      if (j == srcj && z == sz) {
        td.x -= S.alpha_c * pa_new.x;
        td.y -= S.alpha_c * pa_new.y;
      }
      const float2 tv = round2(td);
      if (xstep) {  // read p_{k-2} before p_k replaces it
        const float2 p2 = (c2 != 0.0) ? ld2(pn, c) : f2(0.f, 0.f);
        st2s(xv, c, xupd2(ld2(xv, c), c2, p2, c1, poc[j]));
      }
      st2s(tout, c, tv);
      st2s(pn, c, pc[j]);
      acc += norm2d(tv);
      while (rc.nz_[j] == z) {
        const int q = rc.take(S, j);
        const float2 tq = f2((float)(S.lam_d * pc[j].x), (float)(S.lam_d * pc[j].y));
        st2(t2v, q, tq);
        acc += norm2d(tq);
      }
    }
    __syncthreads();
    cur = nxt;
#pragma unroll
    for (int j = 0; j < RY; ++j) { pm[j] = pc[j]; pc[j] = pnx[j]; poc[j] = pon[j]; }
  }

  const double tot = block_reduce<W>(acc, red);
  if (tid == 0) part_d[S.slot_base + tile] = tot;
  if (srcj >= 0) T->pa = pa_new;
}

// ---------------------------------------------------------------------------
// fused adjoint kernel: step, r update, s = S^H r, ||s||^2 partials
// (k < 0: the set-up pass s_0 = S^H b with a = 0)
// ---------------------------------------------------------------------------

template <int W, int RY>
__global__ void __launch_bounds__(64 * W)
k_adj(const SysDev* __restrict__ sysv, SysState* __restrict__ stv, const double* __restrict__ part_d,
      double* __restrict__ part_s, const GroupDesc* __restrict__ gd, int ngroups, int setup_only) {
  using Ctx = TileCtx<W, RY>;
  __shared__ float2 pl[2][Ctx::LY][Ctx::LX];
  __shared__ double red[W + 1];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int logical = xcd_remap(blockIdx.x, gridDim.x, gd[0].xchunk);
  int g = 0;
  while (g + 1 < ngroups && logical >= gd[g + 1].block0) ++g;
  const int ntiles = gd[g].ntiles, tiles_x = gd[g].tiles_x, tiles_y = gd[g].tiles_y, tz = gd[g].tz;
  const int local = logical - gd[g].block0;
  int rl, tile;
  block_map(gd[g], local, &rl, &tile);
  const int rhs = gd[g].rhs0 + rl;
  const SysDev& S = sysv[rhs];
  SysState* T = stv + rhs;
  if (T->status != kActive) return;
  const int k = T->iterB;
  const bool setup = k < 0;
  if (setup_only && !setup) return;

  double a = 0.0;
  if (!setup) {
    const double gk = T->gamma[k & 1];
    const double g0 = T->gamma0;
    const double gmin = (k == 0) ? gk : T->gmin[(k - 1) & 1];
    const bool brk = T->brk != 0;
    const bool stop = brk || (g0 == 0.0) || (gk <= S.rtol2 * g0) || (k >= S.max_iter) || (gk > kDivergeRatio * gmin);
    if (stop) {
      if (tile == 0 && tid == 0) {
        T->status = brk ? kBreakdown
                  : (g0 == 0.0) ? kZeroRhs
                  : (gk <= S.rtol2 * g0) ? kConverged
                  : (gk > kDivergeRatio * gmin) ? kDiverged : kMaxIter;
        T->iters = k;
      }
      return;
    }
    const double dk = block_sum_slots<W>(part_d + S.slot_base, ntiles, red);
    if (!(dk > 0.0) || !(dk <= DBL_MAX) || !(gk <= DBL_MAX)) {
      // x may still lack a step: the next forward launch (same k) finishes it
      // and the adjoint launch after it records the status
      if (tile == 0 && tid == 0) T->brk = 1;
      return;
    }
    a = gk / dk;
    if (tile == 0 && tid == 0) T->a[k & 1] = a;
  }

  Ctx C;
  C.setup(S, tile, lane, w, tiles_x, tiles_y, tz);
  const int plane = C.plane;
  const double af = a;
  const double w2 = S.omega_d * S.omega_d;
  const GLOBAL float2* __restrict__ ro = gptr((const float2*)S.r[setup ? 1 : (k & 1)]);
  GLOBAL float2* __restrict__ rn = gptr(S.r[setup ? 0 : ((k + 1) & 1)]);
  const GLOBAL float2* __restrict__ tv = gptr((const float2*)S.t);
  GLOBAL float2* __restrict__ sout = gptr(S.s);
  const GLOBAL float* __restrict__ mv = gptr(S.m);
  GLOBAL float2* __restrict__ r2v = gptr(S.r2);
  const GLOBAL float2* __restrict__ t2v = gptr((const float2*)S.t2);

  const int sxy = S.src % plane, sz = S.src / plane;
  const int sx = sxy % S.nx, sy = sxy / S.nx;
  int srcj = -1;
  if (S.mode == 1 && sx == C.gx && sz >= C.z0 && sz < C.z1) {
#pragma unroll
    for (int j = 0; j < RY; ++j)
      if (C.gy[j] == sy) srcj = j;
  }

  RecCursor<RY> rc;
  rc.setup(S, C.gx, C.gy, C.in, C.z0);

  double sxy2[RY];
  const double sx2 = sponge_axis_d(C.gx, S.nx, S.nb, S.inv_nb_d);
#pragma unroll
  for (int j = 0; j < RY; ++j) sxy2[j] = sx2 + sponge_axis_d(C.gy[j], S.ny, S.nb, S.inv_nb_d);

  auto rval = [&](int c) -> float2 {
    const float2 r = ld2(ro, c);
    return setup ? r : axpy2(r, -af, ld2(tv, c));
  };

  float2 rm[RY], rc_[RY], rnx[RY];
#pragma unroll
  for (int j = 0; j < RY; ++j) {
    rm[j] = f2(0.f, 0.f);
    rc_[j] = f2(0.f, 0.f);
    if (C.in[j]) {
      const int c = C.z0 * plane + C.gy[j] * S.nx + C.gx;
      if (C.z0 > 0) rm[j] = rval(c - plane);
      rc_[j] = rval(c);
    }
    pl[0][1 + w * RY + j][1 + lane] = rc_[j];
  }
  for (int h = tid; h < Ctx::NH; h += 64 * W) {
    int hx, hy;
    Ctx::halo_xy(h, hx, hy);
    const int xx = C.x0 + hx - 1, yy = C.y0 + hy - 1;
    float2 v = f2(0.f, 0.f);
    if (xx >= 0 && xx < S.nx && yy >= 0 && yy < S.ny) v = rval(C.z0 * plane + yy * S.nx + xx);
    pl[0][hy][hx] = v;
  }
  __syncthreads();

  double acc = 0.0;
  double2 sa = make_double2(0.0, 0.0);
  int cur = 0;
  for (int z = C.z0; z < C.z1; ++z) {
    const int nxt = cur ^ 1;
    const bool has_next = (z + 1) < S.nz;
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      rnx[j] = f2(0.f, 0.f);
      if (C.in[j] && has_next) rnx[j] = rval((z + 1) * plane + C.gy[j] * S.nx + C.gx);
    }
    for (int h = tid; h < Ctx::NH; h += 64 * W) {
      int hx, hy;
      Ctx::halo_xy(h, hx, hy);
      const int xx = C.x0 + hx - 1, yy = C.y0 + hy - 1;
      float2 v = f2(0.f, 0.f);
      if (has_next && xx >= 0 && xx < S.nx && yy >= 0 && yy < S.ny)
        v = rval((z + 1) * plane + yy * S.nx + xx);
      pl[nxt][hy][hx] = v;
    }
#pragma unroll
    for (int j = 0; j < RY; ++j) pl[nxt][1 + w * RY + j][1 + lane] = rnx[j];

    const double sz2 = sponge_axis_d(z, S.nz, S.nb, S.inv_nb_d);
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      if (!C.in[j]) continue;
      const int ly = w * RY + j;
      const int c = z * plane + C.gy[j] * S.nx + C.gx;
      const float2 xm = pl[cur][ly + 1][lane];
      const float2 xp = pl[cur][ly + 1][lane + 2];
      const float2 ym = (j > 0) ? rc_[j > 0 ? j - 1 : 0] : pl[cur][ly][lane + 1];
      const float2 yp = (j < RY - 1) ? rc_[j < RY - 1 ? j + 1 : 0] : pl[cur][ly + 2][lane + 1];
      const double b = S.sp_scale_d * (sxy2[j] + sz2);
      double2 sd = helm(rc_[j], xm, xp, ym, yp, rm[j], rnx[j], S.h2inv_d, w2 * (double)mv[c], S.omega_d * b);
      while (rc.nz_[j] == z) {
        const int q = rc.take(S, j);
        float2 r2 = ld2(r2v, q);
        if (!setup) {
          r2 = axpy2(r2, -af, ld2(t2v, q));
          st2(r2v, q, r2);
        }
        sd.x += S.lam_d * r2.x;
        sd.y += S.lam_d * r2.y;
      }
      const float2 s = round2(sd);
      if (j == srcj && z == sz) {
        sa = make_double2(-S.alpha_c * (double)rc_[j].x, -S.alpha_c * (double)rc_[j].y);
        acc += sa.x * sa.x + sa.y * sa.y;
      }
      st2s(sout, c, s);
      st2s(rn, c, rc_[j]);
      acc += norm2d(s);
    }
    __syncthreads();
    cur = nxt;
#pragma unroll
    for (int j = 0; j < RY; ++j) { rm[j] = rc_[j]; rc_[j] = rnx[j]; }
  }

  const double tot = block_reduce<W>(acc, red);
  if (tid == 0) part_s[S.slot_base + tile] = tot;
  if (tile == 0 && tid == 0) T->iterA = k + 1;
  if (srcj >= 0) T->sa = sa;
}

// ---------------------------------------------------------------------------
// Software-pipelined variants (same arithmetic, same outputs bit for bit).
// While plane z is computed, the raw inputs of plane z+3 are in flight and
// plane z+2 is committed to LDS; x, m (and p_{k-2}) of plane z+1 are loaded one
// step ahead.  LDS holds three planes (z, z+1, z+2).
//
// Every vector access of the z-march is an unconditional buffer instruction:
// each workgroup builds buffer resources that cover exactly the planes of its
// slab (plus the one-plane halo for the stencil inputs), and cells outside the
// grid get an out-of-range offset, so reads outside the domain return zero and
// stores there are dropped by the hardware.  Without branches around memory
// instructions the compiler's wait counts stay exact and a wavefront waits only
// for the plane it is about to use, not for its own prefetches.  The march is
// unrolled by two so that the one-plane-ahead registers swap roles instead of
// being copied (a copy of a pending load would force a wait).  Receivers are
// located with a per-column bit mask of the slab's planes, so the per-plane
// test touches no memory.
// ---------------------------------------------------------------------------

typedef __amdgpu_buffer_rsrc_t BufRes;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr unsigned kOOB = 0x80000000u;   // beyond any resource (records < 2^31)
constexpr int kBufFlags = 0x00020000;    // raw 32-bit buffer, gfx9 family
constexpr int kStoreNT = 2;              // non-temporal store

// Resource over elements [first, first + count) of v (elem bytes each).
__device__ __forceinline__ BufRes mkbuf(const void* v, int64_t first, int64_t count, int elem) {
  const char* b = static_cast<const char*>(v) + first * elem;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(b), (short)0, (int)(count * elem), kBufFlags);
}
__device__ __forceinline__ float2 bld2(BufRes r, unsigned off) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ float bld1(BufRes r, unsigned off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ void bst2(BufRes r, unsigned off, float2 v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, kStoreNT);
}

// Receivers of a thread's RY columns inside the slab [z0, z1): bit (z - z0) of
// mask[j] is set where a receiver sits (at most one per cell, duplicates are
// rejected on the host); cur[j] is its first entry.  Requires z1 - z0 <= 64.
template <int RY>
struct RecMask {
  uint64_t mask[RY];
  int cur[RY];
  __device__ void setup(const SysDev& S, int gx, const int* gy, const bool* in, int z0, int z1) {
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      mask[j] = 0; cur[j] = 0;
      if (S.colmap != nullptr && in[j]) {
        const int2 be = ld2i(gptr(S.colmap), gy[j] * S.nx + gx);
        int c = be.x;
        while (c < be.y && ld2i(gptr(S.entries), c).x < z0) ++c;
        cur[j] = c;
        for (int e = c; e < be.y; ++e) {
          const int ze = ld2i(gptr(S.entries), e).x;
          if (ze >= z1) break;
          mask[j] |= uint64_t(1) << (ze - z0);
        }
      }
    }
  }
  __device__ bool at(int j, int dz) const { return dz < 64 && ((mask[j] >> dz) & 1); }
  __device__ int take(const SysDev& S, int j) { return ld2i(gptr(S.entries), cur[j]++).y; }
};

// TR = 1: t is not stored (the adjoint pass k_adj_rc recomputes it from p_k);
// the receiver rows t2 and the partials of ||t||^2 are the same.
template <int W, int RY, int XS, int TR>
__global__ void __launch_bounds__(64 * W)
k_fwd_pf(const SysDev* __restrict__ sysv, SysState* __restrict__ stv, const double* __restrict__ part_s,
         double* __restrict__ part_d, const GroupDesc* __restrict__ gd, int ngroups) {
  using Ctx = TileCtx<W, RY>;
  constexpr int NT = 64 * W;
  constexpr int HS = (Ctx::NH + NT - 1) / NT;  // halo slots per thread
  __shared__ float2 pl[3][Ctx::LY][Ctx::LX];
  __shared__ double red[W + 1];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int logical = xcd_remap(blockIdx.x, gridDim.x, gd[0].xchunk);
  int g = 0;
  while (g + 1 < ngroups && logical >= gd[g + 1].block0) ++g;
  const int ntiles = gd[g].ntiles, tiles_x = gd[g].tiles_x, tiles_y = gd[g].tiles_y, tz = gd[g].tz;
  const int local = logical - gd[g].block0;
  int rl, tile;
  block_map(gd[g], local, &rl, &tile);
  const int rhs = gd[g].rhs0 + rl;
  const SysDev& S = sysv[rhs];
  SysState* T = stv + rhs;
  if (T->status != kActive) return;
  const int k = T->iterA;

  const double gk = block_sum_slots<W>(part_s + S.slot_base, ntiles, red);
  const bool warm = T->warm != 0;  // gamma0 = ||S^H b||^2 was set by the warm-start set-up
  const double g0 = (k == 0 && !warm) ? gk : T->gamma0;
  const double gmin = (k == 0) ? gk : T->gmin[(k - 1) & 1];
  // brk: the adjoint launch of this same k broke down; this launch only finishes x
  const bool brk = T->brk != 0;
  const bool stop = brk || (g0 == 0.0) || (gk <= S.rtol2 * g0) || (k >= S.max_iter) || (gk > kDivergeRatio * gmin);
  const double beta = (k == 0) ? 0.0 : gk / T->gamma[(k - 1) & 1];
  const double aprev = (k == 0) ? 0.0 : T->a[(k - 1) & 1];
  // x takes the pending steps on even iterations and when the system stops:
  // c1 p_{k-1} (+ c2 p_{k-2} at even k >= 2; a_{k-2} is still in a[k & 1]).
  // After a breakdown this k already ran once: only an odd k left a step pending.
  const bool xstep = brk ? (k & 1) == 1 : stop ? (k >= 1) : (k >= 2 && (k & 1) == 0);
  const double c1 = xstep ? aprev : 0.0;
  const double c2 = (xstep && !brk && k >= 2 && (k & 1) == 0) ? T->a[k & 1] : 0.0;
  if (tile == 0 && tid == 0) {
    T->gamma[k & 1] = gk;
    T->gmin[k & 1] = fmin(gmin, gk);
    if (k == 0 && !warm) T->gamma0 = gk;
    T->iterB = k;
  }

  Ctx C;
  C.setup(S, tile, lane, w, tiles_x, tiles_y, tz);
  const int plane = C.plane;
  const double bf = beta;
  const double w2 = S.omega_d * S.omega_d;
  // the table's scalars that the march uses, read once (the receiver-row
  // stores could alias the table, so reads through S would be repeated)
  const double sp_scale = S.sp_scale_d, h2inv = S.h2inv_d, om = S.omega_d, inv_nb = S.inv_nb_d;
  const double lam = S.lam_d, acol = S.alpha_c;
  const int nz = S.nz, nbw = S.nb;
  int coff[RY];
#pragma unroll
  for (int j = 0; j < RY; ++j) coff[j] = C.gy[j] * S.nx + C.gx;

  const int sxy = S.src % plane, sz = S.src / plane;
  const int sx = sxy % S.nx, sy = sxy / S.nx;
  int srcj = -1;
  if (S.mode == 1 && sx == C.gx && sz >= C.z0 && sz < C.z1) {
#pragma unroll
    for (int j = 0; j < RY; ++j)
      if (C.gy[j] == sy) srcj = j;
  }

  // x still owes the pending steps when the host's x pattern for this launch
  // does not match this system's own (the host keeps them equal; kept correct anyway)
  if (stop || (!XS && xstep)) {
    if (xstep) {
      const GLOBAL float2* __restrict__ po = gptr((const float2*)S.p[k & 1]);
      const GLOBAL float2* __restrict__ p2v = gptr((const float2*)S.p[(k + 1) & 1]);
      GLOBAL float2* __restrict__ xv = gptr(S.x);
      for (int z = C.z0; z < C.z1; ++z) {
#pragma unroll
        for (int j = 0; j < RY; ++j) {
          if (!C.in[j]) continue;
          const int c = z * plane + coff[j];
          const float2 p2 = (c2 != 0.0) ? ld2(p2v, c) : f2(0.f, 0.f);
          st2s(xv, c, xupd2(ld2(xv, c), c2, p2, c1, ld2(po, c)));
        }
      }
      if (srcj >= 0 && stop && !brk) {
        const double2 pa = T->pa;
        T->xa = make_double2(T->xa.x + aprev * pa.x, T->xa.y + aprev * pa.y);
      }
    }
    if (stop) return;
  }

  double2 pa_new = make_double2(0.0, 0.0);
  if (srcj >= 0) {
    const double2 pa = T->pa, sa = T->sa;
    pa_new = make_double2(sa.x + beta * pa.x, sa.y + beta * pa.y);
    T->xa = make_double2(T->xa.x + aprev * pa.x, T->xa.y + aprev * pa.y);
  }

  RecMask<RY> rc;
  rc.setup(S, C.gx, C.gy, C.in, C.z0, C.z1);

  double sxy2[RY];
  const double sx2 = sponge_axis_d(C.gx, S.nx, S.nb, S.inv_nb_d);
#pragma unroll
  for (int j = 0; j < RY; ++j) sxy2[j] = sx2 + sponge_axis_d(C.gy[j], S.ny, S.nb, S.inv_nb_d);

  // buffer resources: stencil inputs over planes [zlo, zhi) (slab plus halo),
  // the rest over the slab's own planes [z0, z1)
  const int zlo = max(C.z0 - 1, 0), zhi = min(C.z1 + 1, S.nz);
  const int64_t pl64 = plane;
  const BufRes Rs = mkbuf(S.s, zlo * pl64, (zhi - zlo) * pl64, 8);
  const BufRes Rpo = mkbuf(S.p[k & 1], zlo * pl64, (zhi - zlo) * pl64, 8);
  const BufRes Rpn = mkbuf(S.p[(k + 1) & 1], C.z0 * pl64, (C.z1 - C.z0) * pl64, 8);
  const BufRes Rx = mkbuf(S.x, C.z0 * pl64, (C.z1 - C.z0) * pl64, 8);
  const BufRes Rt = mkbuf(S.t, C.z0 * pl64, (C.z1 - C.z0) * pl64, 8);
  const BufRes Rm = mkbuf(S.m, C.z0 * pl64, (C.z1 - C.z0) * pl64, 4);
  GLOBAL float2* __restrict__ t2v = gptr(S.t2);

  // halo slot geometry (fixed for the whole march)
  int hx[HS], hy[HS], hoff[HS];
  bool hin[HS];
#pragma unroll
  for (int q = 0; q < HS; ++q) {
    const int h = tid + q * NT;
    hx[q] = 0; hy[q] = 0; hoff[q] = 0; hin[q] = false;
    if (h < Ctx::NH) {
      Ctx::halo_xy(h, hx[q], hy[q]);
      const int xx = C.x0 + hx[q] - 1, yy = C.y0 + hy[q] - 1;
      hin[q] = xx >= 0 && xx < S.nx && yy >= 0 && yy < S.ny;
      hoff[q] = yy * S.nx + xx;
    }
  }
  // byte offset of an own cell (plane zz) in a stencil-input resource / a slab resource
  // Byte offsets of a cell in a stencil-input resource (planes from zlo) and in
  // a slab resource (planes from z0).  Cells outside the grid get the
  // out-of-range bit ORed in (arithmetic, so that no branch forms around the
  // access); planes outside a resource's range are out of range by themselves.
  unsigned obit[RY], hbit[HS];
#pragma unroll
  for (int j = 0; j < RY; ++j) obit[j] = C.in[j] ? 0u : kOOB;
#pragma unroll
  for (int q = 0; q < HS; ++q) hbit[q] = hin[q] ? 0u : kOOB;
  auto hoff_b = [&](int zz, int cell, unsigned bit) -> unsigned {
    return (unsigned)(((zz - zlo) * plane + cell) * 8) | bit;
  };
  auto own_b = [&](int zz, int j, int elem) -> unsigned {
    return (unsigned)(((zz - C.z0) * plane + coff[j]) * elem) | obit[j];
  };

  // Raw inputs of one plane: s and p_{k-1} of the own rows and the halo, and
  // (x-step launches) x and p_{k-2} of the own rows.  The x update of a plane
  // is applied when the plane is committed, so every raw load is consumed right
  // after its one wait and no loaded register lives on across planes.
  float2 rs[RY], rp[RY], hs_[HS], hp_[HS], rx[RY], rq[RY];
  auto issue = [&](int zz) {
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      const unsigned o = hoff_b(zz, coff[j], obit[j]);
      rs[j] = bld2(Rs, o);
      rp[j] = bld2(Rpo, o);
      if constexpr (XS != 0) {
        const unsigned o8 = own_b(zz, j, 8);
        rx[j] = bld2(Rx, o8);
        rq[j] = bld2(Rpn, o8);
      }
    }
#pragma unroll
    for (int q = 0; q < HS; ++q) {
      const unsigned o = hoff_b(zz, hoff[q], hbit[q]);
      hs_[q] = bld2(Rs, o);
      hp_[q] = bld2(Rpo, o);
    }
  };
  // p_k = s + beta p_{k-1} of plane zz into LDS buffer b and pnew; x of plane zz
  // (planes outside the slab are out of range of Rx: the store is dropped)
  float2 pnew[RY];
  auto commit = [&](int b, int zz) {
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      pnew[j] = axpy2(rs[j], bf, rp[j]);
      pl[b][1 + w * RY + j][1 + lane] = pnew[j];
      if constexpr (XS != 0)
        bst2(Rx, own_b(zz, j, 8), xstep ? xupd2(rx[j], c2, rq[j], c1, rp[j]) : rx[j]);
    }
#pragma unroll
    for (int q = 0; q < HS; ++q)
      if (tid + q * NT < Ctx::NH) pl[b][hy[q]][hx[q]] = axpy2(hs_[q], bf, hp_[q]);
  };

  // m of the current / next plane.  Plane z0's m is loaded first: the loop's
  // wait for it then counts every later load of the prologue, and the count the
  // compiler derives for the loop header is the loop's own, not a drain.
  float mA[RY], mB[RY];
#pragma unroll
  for (int j = 0; j < RY; ++j) mA[j] = bld1(Rm, own_b(C.z0, j, 4));
  float2 pm[RY], pc[RY], pnx[RY];
  // plane z0-1 (own rows only; zero below the grid)
#pragma unroll
  for (int j = 0; j < RY; ++j) {
    const unsigned o = hoff_b(C.z0 - 1, coff[j], obit[j]);
    pm[j] = axpy2(bld2(Rs, o), bf, bld2(Rpo, o));
  }
  issue(C.z0);
  commit(0, C.z0);
#pragma unroll
  for (int j = 0; j < RY; ++j) pc[j] = pnew[j];
  issue(C.z0 + 1);
  commit(1, C.z0 + 1);
#pragma unroll
  for (int j = 0; j < RY; ++j) pnx[j] = pnew[j];
  issue(C.z0 + 2);
  __syncthreads();

  double acc = 0.0;
  int cur = 0;
  // one plane: uses m of plane z (mz) and loads that of plane z+1 into mn.  A
  // step with z >= z1 (odd slab length) computes nothing that is stored or summed.
  auto step = [&](int z, float (&mz)[RY], float (&mn)[RY]) {
#pragma unroll
    for (int j = 0; j < RY; ++j) mn[j] = bld1(Rm, own_b(z + 1, j, 4));
    const bool zin = z < C.z1;
    const unsigned zbit = zin ? 0u : kOOB;
    const double sz2 = sponge_axis_d(z, nz, nbw, inv_nb);
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      const int ly = w * RY + j;
      const float2 xm = pl[cur][ly + 1][lane];
      const float2 xp = pl[cur][ly + 1][lane + 2];
      const float2 ym = (j > 0) ? pc[j > 0 ? j - 1 : 0] : pl[cur][ly][lane + 1];
      const float2 yp = (j < RY - 1) ? pc[j < RY - 1 ? j + 1 : 0] : pl[cur][ly + 2][lane + 1];
      const double b = sp_scale * (sxy2[j] + sz2);
      double2 td = helm(pc[j], xm, xp, ym, yp, pm[j], pnx[j], h2inv, w2 * (double)mz[j], -(om * b));
      if (j == srcj && z == sz) {
        td.x -= acol * pa_new.x;
        td.y -= acol * pa_new.y;
      }
      const float2 tv = round2(td);
      const bool live = C.in[j] && zin;
      const unsigned o8 = own_b(z, j, 8) | zbit;
      if constexpr (TR == 0) bst2(Rt, o8, tv);
      bst2(Rpn, o8, pc[j]);
      acc += live ? norm2d(tv) : 0.0;
      if (rc.at(j, z - C.z0)) {  // receiver row of S p: lambda p at the receiver cell
        const int q = rc.take(S, j);
        const float2 tq = f2((float)(lam * pc[j].x), (float)(lam * pc[j].y));
        st2(t2v, q, tq);
        acc += norm2d(tq);
      }
    }
    // plane z+2 (its loads were issued one step ago) into LDS; then prefetch z+3
    commit((cur + 2) % 3, z + 2);
    float2 pn2[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) pn2[j] = pnew[j];
    // keep the next plane's loads below the commit: hoisted above it, they would
    // need registers of their own and a copy (a wait) at the loop back-edge
    __builtin_amdgcn_sched_barrier(0);
    issue(z + 3);
    __syncthreads();
    cur = (cur + 1) % 3;
#pragma unroll
    for (int j = 0; j < RY; ++j) { pm[j] = pc[j]; pc[j] = pnx[j]; pnx[j] = pn2[j]; }
  };
  for (int z = C.z0; z < C.z1; z += 2) {
    step(z, mA, mB);
    step(z + 1, mB, mA);
  }

  const double tot = block_reduce<W>(acc, red);
  if (tid == 0) part_d[S.slot_base + tile] = tot;
  if (srcj >= 0) T->pa = pa_new;
}

template <int W, int RY>
__global__ void __launch_bounds__(64 * W)
k_adj_pf(const SysDev* __restrict__ sysv, SysState* __restrict__ stv, const double* __restrict__ part_d,
         double* __restrict__ part_s, const GroupDesc* __restrict__ gd, int ngroups, int setup_only) {
  using Ctx = TileCtx<W, RY>;
  constexpr int NT = 64 * W;
  constexpr int HS = (Ctx::NH + NT - 1) / NT;
  __shared__ float2 pl[3][Ctx::LY][Ctx::LX];
  __shared__ double red[W + 1];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int logical = xcd_remap(blockIdx.x, gridDim.x, gd[0].xchunk);
  int g = 0;
  while (g + 1 < ngroups && logical >= gd[g + 1].block0) ++g;
  const int ntiles = gd[g].ntiles, tiles_x = gd[g].tiles_x, tiles_y = gd[g].tiles_y, tz = gd[g].tz;
  const int local = logical - gd[g].block0;
  int rl, tile;
  block_map(gd[g], local, &rl, &tile);
  const int rhs = gd[g].rhs0 + rl;
  const SysDev& S = sysv[rhs];
  SysState* T = stv + rhs;
  if (T->status != kActive) return;
  const int k = T->iterB;
  const bool setup = k < 0;
  if (setup_only && !setup) return;

  double a = 0.0;
  if (!setup) {
    const double gk = T->gamma[k & 1];
    const double g0 = T->gamma0;
    const double gmin = (k == 0) ? gk : T->gmin[(k - 1) & 1];
    const bool brk = T->brk != 0;
    const bool stop = brk || (g0 == 0.0) || (gk <= S.rtol2 * g0) || (k >= S.max_iter) || (gk > kDivergeRatio * gmin);
    if (stop) {
      if (tile == 0 && tid == 0) {
        T->status = brk ? kBreakdown
                  : (g0 == 0.0) ? kZeroRhs
                  : (gk <= S.rtol2 * g0) ? kConverged
                  : (gk > kDivergeRatio * gmin) ? kDiverged : kMaxIter;
        T->iters = k;
      }
      return;
    }
    const double dk = block_sum_slots<W>(part_d + S.slot_base, ntiles, red);
    if (!(dk > 0.0) || !(dk <= DBL_MAX) || !(gk <= DBL_MAX)) {
      // x may still lack a step: the next forward launch (same k) finishes it
      // and the adjoint launch after it records the status
      if (tile == 0 && tid == 0) T->brk = 1;
      return;
    }
    a = gk / dk;
    if (tile == 0 && tid == 0) T->a[k & 1] = a;
  }

  Ctx C;
  C.setup(S, tile, lane, w, tiles_x, tiles_y, tz);
  const int plane = C.plane;
  const double af = a;
  const double w2 = S.omega_d * S.omega_d;
  int coff[RY];
#pragma unroll
  for (int j = 0; j < RY; ++j) coff[j] = C.gy[j] * S.nx + C.gx;

  const int sxy = S.src % plane, sz = S.src / plane;
  const int sx = sxy % S.nx, sy = sxy / S.nx;
  int srcj = -1;
  if (S.mode == 1 && sx == C.gx && sz >= C.z0 && sz < C.z1) {
#pragma unroll
    for (int j = 0; j < RY; ++j)
      if (C.gy[j] == sy) srcj = j;
  }

  RecMask<RY> rc;
  rc.setup(S, C.gx, C.gy, C.in, C.z0, C.z1);

  double sxy2[RY];
  const double sx2 = sponge_axis_d(C.gx, S.nx, S.nb, S.inv_nb_d);
#pragma unroll
  for (int j = 0; j < RY; ++j) sxy2[j] = sx2 + sponge_axis_d(C.gy[j], S.ny, S.nb, S.inv_nb_d);

  const int zlo = max(C.z0 - 1, 0), zhi = min(C.z1 + 1, S.nz);
  const int64_t pl64 = plane;
  const BufRes Rro = mkbuf(S.r[setup ? 1 : (k & 1)], zlo * pl64, (zhi - zlo) * pl64, 8);
  const BufRes Rt = mkbuf(S.t, zlo * pl64, (zhi - zlo) * pl64, 8);
  const BufRes Rrn = mkbuf(S.r[setup ? 0 : ((k + 1) & 1)], C.z0 * pl64, (C.z1 - C.z0) * pl64, 8);
  const BufRes Rso = mkbuf(S.s, C.z0 * pl64, (C.z1 - C.z0) * pl64, 8);
  const BufRes Rm = mkbuf(S.m, C.z0 * pl64, (C.z1 - C.z0) * pl64, 4);
  GLOBAL float2* __restrict__ r2v = gptr(S.r2);
  const GLOBAL float2* __restrict__ t2v = gptr((const float2*)S.t2);

  int hx[HS], hy[HS], hoff[HS];
  bool hin[HS];
#pragma unroll
  for (int q = 0; q < HS; ++q) {
    const int h = tid + q * NT;
    hx[q] = 0; hy[q] = 0; hoff[q] = 0; hin[q] = false;
    if (h < Ctx::NH) {
      Ctx::halo_xy(h, hx[q], hy[q]);
      const int xx = C.x0 + hx[q] - 1, yy = C.y0 + hy[q] - 1;
      hin[q] = xx >= 0 && xx < S.nx && yy >= 0 && yy < S.ny;
      hoff[q] = yy * S.nx + xx;
    }
  }
  // Byte offsets of a cell in a stencil-input resource (planes from zlo) and in
  // a slab resource (planes from z0).  Cells outside the grid get the
  // out-of-range bit ORed in (arithmetic, so that no branch forms around the
  // access); planes outside a resource's range are out of range by themselves.
  unsigned obit[RY], hbit[HS];
#pragma unroll
  for (int j = 0; j < RY; ++j) obit[j] = C.in[j] ? 0u : kOOB;
#pragma unroll
  for (int q = 0; q < HS; ++q) hbit[q] = hin[q] ? 0u : kOOB;
  auto hoff_b = [&](int zz, int cell, unsigned bit) -> unsigned {
    return (unsigned)(((zz - zlo) * plane + cell) * 8) | bit;
  };
  auto own_b = [&](int zz, int j, int elem) -> unsigned {
    return (unsigned)(((zz - C.z0) * plane + coff[j]) * elem) | obit[j];
  };
  // the set-up pass (s_0 = S^H b) reads no t
  const unsigned tbit = setup ? kOOB : 0u;

  float2 rr[RY], rt[RY], hr[HS], ht[HS];
  auto issue = [&](int zz) {
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      const unsigned o = hoff_b(zz, coff[j], obit[j]);
      rr[j] = bld2(Rro, o);
      rt[j] = bld2(Rt, o | tbit);
    }
#pragma unroll
    for (int q = 0; q < HS; ++q) {
      const unsigned o = hoff_b(zz, hoff[q], hbit[q]);
      hr[q] = bld2(Rro, o);
      ht[q] = bld2(Rt, o | tbit);
    }
  };
  float2 rnew[RY];
  auto commit = [&](int b) {
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      rnew[j] = setup ? rr[j] : axpy2(rr[j], -af, rt[j]);
      pl[b][1 + w * RY + j][1 + lane] = rnew[j];
    }
#pragma unroll
    for (int q = 0; q < HS; ++q)
      if (tid + q * NT < Ctx::NH) pl[b][hy[q]][hx[q]] = setup ? hr[q] : axpy2(hr[q], -af, ht[q]);
  };

  // m of plane z0 first (see the forward kernel)
  float mA[RY], mB[RY];
#pragma unroll
  for (int j = 0; j < RY; ++j) mA[j] = bld1(Rm, own_b(C.z0, j, 4));
  float2 rm[RY], rc_[RY], rnx[RY];
#pragma unroll
  for (int j = 0; j < RY; ++j) {
    const unsigned o = hoff_b(C.z0 - 1, coff[j], obit[j]);
    const float2 r0 = bld2(Rro, o);
    const float2 t0 = bld2(Rt, o | tbit);
    rm[j] = setup ? r0 : axpy2(r0, -af, t0);
  }
  issue(C.z0);
  commit(0);
#pragma unroll
  for (int j = 0; j < RY; ++j) rc_[j] = rnew[j];
  issue(C.z0 + 1);
  commit(1);
#pragma unroll
  for (int j = 0; j < RY; ++j) rnx[j] = rnew[j];
  issue(C.z0 + 2);
  __syncthreads();

  double acc = 0.0;
  double2 sa = make_double2(0.0, 0.0);
  int cur = 0;
  auto step = [&](int z, float (&mz)[RY], float (&mn)[RY]) {
#pragma unroll
    for (int j = 0; j < RY; ++j) mn[j] = bld1(Rm, own_b(z + 1, j, 4));
    const bool zin = z < C.z1;
    const unsigned zbit = zin ? 0u : kOOB;
    const double sz2 = sponge_axis_d(z, S.nz, S.nb, S.inv_nb_d);
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      const int ly = w * RY + j;
      const float2 xm = pl[cur][ly + 1][lane];
      const float2 xp = pl[cur][ly + 1][lane + 2];
      const float2 ym = (j > 0) ? rc_[j > 0 ? j - 1 : 0] : pl[cur][ly][lane + 1];
      const float2 yp = (j < RY - 1) ? rc_[j < RY - 1 ? j + 1 : 0] : pl[cur][ly + 2][lane + 1];
      const double b = S.sp_scale_d * (sxy2[j] + sz2);
      double2 sd = helm(rc_[j], xm, xp, ym, yp, rm[j], rnx[j], S.h2inv_d, w2 * (double)mz[j], S.omega_d * b);
      if (rc.at(j, z - C.z0)) {  // receiver column of S^H: lambda r2 at the receiver cell
        const int q = rc.take(S, j);
        float2 r2 = ld2(r2v, q);
        if (!setup) {
          r2 = axpy2(r2, -af, ld2(t2v, q));
          st2(r2v, q, r2);
        }
        sd.x += S.lam_d * r2.x;
        sd.y += S.lam_d * r2.y;
      }
      const float2 s = round2(sd);
      if (j == srcj && z == sz) {
        sa = make_double2(-S.alpha_c * (double)rc_[j].x, -S.alpha_c * (double)rc_[j].y);
        acc += sa.x * sa.x + sa.y * sa.y;
      }
      const bool live = C.in[j] && zin;
      const unsigned o8 = own_b(z, j, 8) | zbit;
      bst2(Rso, o8, s);
      bst2(Rrn, o8, rc_[j]);
      acc += live ? norm2d(s) : 0.0;
    }
    commit((cur + 2) % 3);
    float2 rn2[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) rn2[j] = rnew[j];
    __builtin_amdgcn_sched_barrier(0);
    issue(z + 3);
    __syncthreads();
    cur = (cur + 1) % 3;
#pragma unroll
    for (int j = 0; j < RY; ++j) { rm[j] = rc_[j]; rc_[j] = rnx[j]; rnx[j] = rn2[j]; }
  };
  for (int z = C.z0; z < C.z1; z += 2) {
    step(z, mA, mB);
    step(z + 1, mB, mA);
  }

  const double tot = block_reduce<W>(acc, red);
  if (tid == 0) part_s[S.slot_base + tile] = tot;
  if (tile == 0 && tid == 0) T->iterA = k + 1;
  if (srcj >= 0) T->sa = sa;
}

// ---------------------------------------------------------------------------
// fused adjoint kernel with t recomputed: the forward pass stores no t
// ---------------------------------------------------------------------------

// A register copy the compiler cannot coalesce with its source: a loaded
// register that is kept for later planes is copied out once it has been used,
// so the load's own register dies there and the next load of the march can
// land in it (a coalesced copy keeps it alive, and the next load then goes to
// a fresh register that has to be copied, with a wait, at the loop back-edge).
__device__ __forceinline__ float keep1(float v) {
  float r;
  asm("v_mov_b32 %0, %1" : "=&v"(r) : "v"(v));
  return r;
}
__device__ __forceinline__ float2 keep2(float2 v) { return make_float2(keep1(v.x), keep1(v.y)); }

// r_{k+1} = r_k - a_k t is needed on the tile and on a one-cell ring around it
// (the stencil of s = A^H r_{k+1}), so t = S p_k is evaluated there, which
// takes p_k on a two-cell ring.  t comes from the same stencil routine, with
// the same operands in the same order, as in the forward pass, so it has the
// bits the forward pass would have stored, and the iterates are identical to
// those of k_adj_pf.  Bytes per (system, cell): read r_k, p_k, m (8+8+4), write
// r_{k+1}, s (8+8) = 36 B; the forward pass drops its 8 B store of t.
//
// March over the slab, step for plane z: s of plane z from the r_{k+1} planes
// z-1..z+1 (LDS ring of three, z-neighbours of the own rows in registers);
// then t and r_{k+1} of plane z+2 on tile + ring 1 from the p_k plane z+2 (LDS,
// two rings) and the p_k planes z+1, z+3 (registers); then p_k of plane z+3 is
// committed to the other LDS buffer and the loads of plane z+2+NS (r_k, m) and
// z+3+NS (p_k) are issued.  There are NS sets of raw load registers: with
// NS = 2 even and odd steps use their own set, so a load has two steps to
// arrive (at the cost of registers, i.e. of resident waves).  A loaded register
// is consumed where it lands and never copied while in flight.
template <int W, int RY, int NS>
__global__ void __launch_bounds__(64 * W)
k_adj_rc(const SysDev* __restrict__ sysv, SysState* __restrict__ stv, const double* __restrict__ part_d,
         double* __restrict__ part_s, const GroupDesc* __restrict__ gd, int ngroups, int setup_only) {
  using Ctx = TileCtx<W, RY>;
  constexpr int NT = 64 * W;
  constexpr int LX = Ctx::LX, LY = Ctx::LY;  // r_{k+1} plane: tile and ring 1
  constexpr int PX = LX + 2, PY = LY + 2;    // p_k plane: tile and rings 1, 2
  constexpr int NH = Ctx::NH;                // ring-1 cells
  constexpr int NH2 = 2 * PX + 2 * LY;       // ring-2 cells
  constexpr int HS = (NH + NT - 1) / NT;
  constexpr int HS2 = (NH2 + NT - 1) / NT;
  __shared__ float2 pl[3][LY][LX];
  __shared__ float2 pp[2][PY][PX];
  __shared__ double red[W + 1];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int logical = xcd_remap(blockIdx.x, gridDim.x, gd[0].xchunk);
  int g = 0;
  while (g + 1 < ngroups && logical >= gd[g + 1].block0) ++g;
  const int ntiles = gd[g].ntiles, tiles_x = gd[g].tiles_x, tiles_y = gd[g].tiles_y, tz = gd[g].tz;
  const int local = logical - gd[g].block0;
  int rl, tile;
  block_map(gd[g], local, &rl, &tile);
  const int rhs = gd[g].rhs0 + rl;
  const SysDev& S = sysv[rhs];
  SysState* T = stv + rhs;
  if (T->status != kActive) return;
  const int k = T->iterB;
  const bool setup = k < 0;
  if (setup_only && !setup) return;

  double a = 0.0;
  double2 pa = make_double2(0.0, 0.0);
  if (!setup) {
    const double gk = T->gamma[k & 1];
    const double g0 = T->gamma0;
    const double gmin = (k == 0) ? gk : T->gmin[(k - 1) & 1];
    const bool brk = T->brk != 0;
    const bool stop = brk || (g0 == 0.0) || (gk <= S.rtol2 * g0) || (k >= S.max_iter) || (gk > kDivergeRatio * gmin);
    if (stop) {
      if (tile == 0 && tid == 0) {
        T->status = brk ? kBreakdown
                  : (g0 == 0.0) ? kZeroRhs
                  : (gk <= S.rtol2 * g0) ? kConverged
                  : (gk > kDivergeRatio * gmin) ? kDiverged : kMaxIter;
        T->iters = k;
      }
      return;
    }
    const double dk = block_sum_slots<W>(part_d + S.slot_base, ntiles, red);
    if (!(dk > 0.0) || !(dk <= DBL_MAX) || !(gk <= DBL_MAX)) {
      if (tile == 0 && tid == 0) T->brk = 1;
      return;
    }
    a = gk / dk;
    if (tile == 0 && tid == 0) T->a[k & 1] = a;
    if (S.mode == 1) pa = T->pa;  // p_alpha of this k (the forward pass wrote it)
  }

  Ctx C;
  C.setup(S, tile, lane, w, tiles_x, tiles_y, tz);
  const int plane = C.plane;
  const double af = a;
  const double w2 = S.omega_d * S.omega_d;
  // the table's scalars that the march uses, read once: the receiver-row
  // stores go through a global pointer that could alias the table, so reads
  // through S inside the loop would be repeated after every store
  const double sp_scale = S.sp_scale_d, h2inv = S.h2inv_d, om = S.omega_d, inv_nb = S.inv_nb_d;
  const double lam = S.lam_d, acol = S.alpha_c;
  const int nz = S.nz, nbw = S.nb;
  int coff[RY];
#pragma unroll
  for (int j = 0; j < RY; ++j) coff[j] = C.gy[j] * S.nx + C.gx;

  const int sxy = S.src % plane, sz = S.src / plane;
  const int sx = sxy % S.nx, sy = sxy / S.nx;
  int srcj = -1;  // own row holding the source column (mode 1)
  if (S.mode == 1 && sx == C.gx) {
#pragma unroll
    for (int j = 0; j < RY; ++j)
      if (C.gy[j] == sy) srcj = j;
  }
  const bool src_in_slab = sz >= C.z0 && sz < C.z1;

  RecMask<RY> rc;
  rc.setup(S, C.gx, C.gy, C.in, C.z0, C.z1);

  double sxy2[RY];
  const double sx2 = sponge_axis_d(C.gx, S.nx, S.nb, S.inv_nb_d);
#pragma unroll
  for (int j = 0; j < RY; ++j) sxy2[j] = sx2 + sponge_axis_d(C.gy[j], S.ny, S.nb, S.inv_nb_d);

  // r_k and m over planes [zlo, zhi) (t and r_{k+1} are needed one plane
  // beyond the slab), p_k over [plo, phi) (two planes beyond)
  const int zlo = max(C.z0 - 1, 0), zhi = min(C.z1 + 1, S.nz);
  const int plo = max(C.z0 - 2, 0), phi = min(C.z1 + 2, S.nz);
  const int64_t pl64 = plane;
  const BufRes Rro = mkbuf(S.r[setup ? 1 : (k & 1)], zlo * pl64, (zhi - zlo) * pl64, 8);
  const BufRes Rp = mkbuf(S.p[(k + 1) & 1], plo * pl64, (phi - plo) * pl64, 8);
  const BufRes Rm = mkbuf(S.m, zlo * pl64, (zhi - zlo) * pl64, 4);
  const BufRes Rrn = mkbuf(S.r[setup ? 0 : ((k + 1) & 1)], C.z0 * pl64, (C.z1 - C.z0) * pl64, 8);
  const BufRes Rso = mkbuf(S.s, C.z0 * pl64, (C.z1 - C.z0) * pl64, 8);
  GLOBAL float2* __restrict__ r2v = gptr(S.r2);
  const GLOBAL float2* __restrict__ t2v = gptr((const float2*)S.t2);

  // ring 1: LDS coordinates in the r_{k+1} plane (the p_k plane has them +1),
  // cell offset, inside-grid flag, sponge of its column, source column flag
  int hx[HS], hy[HS], hoff[HS];
  bool hin[HS], hsrc[HS];
  double hsxy[HS];
#pragma unroll
  for (int q = 0; q < HS; ++q) {
    const int h = tid + q * NT;
    hx[q] = 0; hy[q] = 0; hoff[q] = 0; hin[q] = false; hsrc[q] = false; hsxy[q] = 0.0;
    if (h < NH) {
      Ctx::halo_xy(h, hx[q], hy[q]);
      const int xx = C.x0 + hx[q] - 1, yy = C.y0 + hy[q] - 1;
      hin[q] = xx >= 0 && xx < S.nx && yy >= 0 && yy < S.ny;
      hoff[q] = yy * S.nx + xx;
      hsrc[q] = S.mode == 1 && xx == sx && yy == sy;
      hsxy[q] = sponge_axis_d(xx, S.nx, S.nb, S.inv_nb_d) + sponge_axis_d(yy, S.ny, S.nb, S.inv_nb_d);
    }
  }
  // ring 2: LDS coordinates in the p_k plane and cell offset
  int gx2[HS2], gy2[HS2], goff[HS2];
  bool gin[HS2];
#pragma unroll
  for (int q = 0; q < HS2; ++q) {
    const int h = tid + q * NT;
    gx2[q] = 0; gy2[q] = 0; goff[q] = 0; gin[q] = false;
    if (h < NH2) {
      if (h < PX) { gx2[q] = h; gy2[q] = 0; }
      else if (h < 2 * PX) { gx2[q] = h - PX; gy2[q] = PY - 1; }
      else { const int h2 = h - 2 * PX; gy2[q] = 1 + (h2 >> 1); gx2[q] = (h2 & 1) ? (PX - 1) : 0; }
      const int xx = C.x0 + gx2[q] - 2, yy = C.y0 + gy2[q] - 2;
      gin[q] = xx >= 0 && xx < S.nx && yy >= 0 && yy < S.ny;
      goff[q] = yy * S.nx + xx;
    }
  }
  // Byte offsets (see k_adj_pf): out-of-grid cells carry the out-of-range bit;
  // planes outside a resource's range are out of range by themselves.  The
  // set-up pass (s_0 = S^H b) reads no p.
  const unsigned pbit = setup ? kOOB : 0u;
  unsigned obit[RY], hbit[HS], gbit[HS2];
#pragma unroll
  for (int j = 0; j < RY; ++j) obit[j] = C.in[j] ? 0u : kOOB;
#pragma unroll
  for (int q = 0; q < HS; ++q) hbit[q] = hin[q] ? 0u : kOOB;
#pragma unroll
  for (int q = 0; q < HS2; ++q) gbit[q] = gin[q] ? 0u : kOOB;
  auto off_r = [&](int zz, int cell, unsigned bit, int elem) -> unsigned {
    return (unsigned)(((zz - zlo) * plane + cell) * elem) | bit;
  };
  auto off_p = [&](int zz, int cell, unsigned bit) -> unsigned {
    return (unsigned)(((zz - plo) * plane + cell) * 8) | bit | pbit;
  };
  auto own_b = [&](int zz, int j) -> unsigned {
    return (unsigned)(((zz - C.z0) * plane + coff[j]) * 8) | obit[j];
  };

  // raw loads of one step, NS sets: p_k (own, ring 1, ring 2), r_k and m (own, ring 1)
  float2 rp[NS][RY], hp[NS][HS], gp[NS][HS2], rr[NS][RY], hr[NS][HS];
  float rmr[NS][RY], hmr[NS][HS];
  auto issue = [&](const int st, int zr, int zp) __attribute__((always_inline)) {
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      rp[st][j] = bld2(Rp, off_p(zp, coff[j], obit[j]));
      rr[st][j] = bld2(Rro, off_r(zr, coff[j], obit[j], 8));
      rmr[st][j] = bld1(Rm, off_r(zr, coff[j], obit[j], 4));
    }
#pragma unroll
    for (int q = 0; q < HS; ++q) {
      hp[st][q] = bld2(Rp, off_p(zp, hoff[q], hbit[q]));
      hr[st][q] = bld2(Rro, off_r(zr, hoff[q], hbit[q], 8));
      hmr[st][q] = bld1(Rm, off_r(zr, hoff[q], hbit[q], 4));
    }
#pragma unroll
    for (int q = 0; q < HS2; ++q) gp[st][q] = bld2(Rp, off_p(zp, goff[q], gbit[q]));
  };
  // p_k of planes zz-1, zz (own rows and ring 1); the raw load holds plane zz+1
  float2 pzm[RY], pzc[RY], hpm[HS], hpc[HS];
  // m of the own rows: planes z, z+1 (for s), then plane z+2 after tphase
  float mq0[RY], mq1[RY], mq2[RY];
  float2 rnew[RY];
  // t and r_{k+1} of plane zz on tile + ring 1 from LDS p buffer bp; r_{k+1}
  // into LDS buffer br (br < 0: own rows only) from raw set st; commit p_k of
  // plane zz+1 to LDS buffer bp ^ 1 and move the p registers up one plane.
  auto tphase = [&](const int st, int zz, int bp, int br) __attribute__((always_inline)) {
    const bool zok = zz >= 0 && zz < nz;
    const double sz2 = sponge_axis_d(zz, nz, nbw, inv_nb);
    const bool zsrc = zz == sz;
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      const int ly = w * RY + j + 2;
      const float2 xm = pp[bp][ly][lane + 1];
      const float2 xp = pp[bp][ly][lane + 3];
      const float2 ym = (j > 0) ? pzc[j > 0 ? j - 1 : 0] : pp[bp][ly - 1][lane + 2];
      const float2 yp = (j < RY - 1) ? pzc[j < RY - 1 ? j + 1 : 0] : pp[bp][ly + 1][lane + 2];
      const double b = sp_scale * (sxy2[j] + sz2);
      double2 td = helm(pzc[j], xm, xp, ym, yp, pzm[j], rp[st][j], h2inv, w2 * (double)rmr[st][j],
                         -(om * b));
      if (j == srcj && zsrc) {
        td.x -= acol * pa.x;
        td.y -= acol * pa.y;
      }
      const double ae = (zok && C.in[j]) ? af : 0.0;
      rnew[j] = setup ? rr[st][j] : axpy2(rr[st][j], -ae, round2(td));
      if (br >= 0) pl[br][ly - 1][lane + 1] = rnew[j];
      mq2[j] = keep1(rmr[st][j]);
    }
#pragma unroll
    for (int q = 0; q < HS; ++q) {
      if (tid + q * NT < NH) {
        const int cx = hx[q] + 1, cy = hy[q] + 1;
        const float2 xm = pp[bp][cy][cx - 1];
        const float2 xp = pp[bp][cy][cx + 1];
        const float2 ym = pp[bp][cy - 1][cx];
        const float2 yp = pp[bp][cy + 1][cx];
        const double b = sp_scale * (hsxy[q] + sz2);
        double2 td = helm(hpc[q], xm, xp, ym, yp, hpm[q], hp[st][q], h2inv, w2 * (double)hmr[st][q],
                           -(om * b));
        if (hsrc[q] && zsrc) {
          td.x -= acol * pa.x;
          td.y -= acol * pa.y;
        }
        const double ae = (zok && hin[q]) ? af : 0.0;
        const float2 rv = setup ? hr[st][q] : axpy2(hr[st][q], -ae, round2(td));
        if (br >= 0) pl[br][hy[q]][hx[q]] = rv;
      }
    }
    // p_k of plane zz+1 into the other buffer
    const int bq = bp ^ 1;
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      pp[bq][w * RY + j + 2][lane + 2] = rp[st][j];
      pzm[j] = pzc[j];
      pzc[j] = keep2(rp[st][j]);
    }
#pragma unroll
    for (int q = 0; q < HS; ++q) {
      if (tid + q * NT < NH) pp[bq][hy[q] + 1][hx[q] + 1] = hp[st][q];
      hpm[q] = hpc[q];
      hpc[q] = keep2(hp[st][q]);
    }
#pragma unroll
    for (int q = 0; q < HS2; ++q)
      if (tid + q * NT < NH2) pp[bq][gy2[q]][gx2[q]] = gp[st][q];
  };

  // prologue (raw set 0): p_k planes z0-2, z0-1 into registers (z0-1 also
  // into LDS 0), then t / r_{k+1} of planes z0-1 (own rows), z0 (LDS 0) and
  // z0+1 (LDS 1); then the raw sets of the first NS steps in flight
  issue(0, C.z0 - 1, C.z0 - 2);
#pragma unroll
  for (int j = 0; j < RY; ++j) pzc[j] = rp[0][j];
#pragma unroll
  for (int q = 0; q < HS; ++q) hpc[q] = hp[0][q];
  issue(0, C.z0 - 1, C.z0 - 1);
#pragma unroll
  for (int j = 0; j < RY; ++j) {
    pp[0][w * RY + j + 2][lane + 2] = rp[0][j];
    pzm[j] = pzc[j];
    pzc[j] = rp[0][j];
  }
#pragma unroll
  for (int q = 0; q < HS; ++q) {
    if (tid + q * NT < NH) pp[0][hy[q] + 1][hx[q] + 1] = hp[0][q];
    hpm[q] = hpc[q];
    hpc[q] = hp[0][q];
  }
#pragma unroll
  for (int q = 0; q < HS2; ++q)
    if (tid + q * NT < NH2) pp[0][gy2[q]][gx2[q]] = gp[0][q];
  issue(0, C.z0 - 1, C.z0);
  __syncthreads();
  float2 rm[RY], rc_[RY], rnx[RY];
  tphase(0, C.z0 - 1, 0, -1);
#pragma unroll
  for (int j = 0; j < RY; ++j) rm[j] = rnew[j];
  issue(0, C.z0, C.z0 + 1);
  __syncthreads();
  tphase(0, C.z0, 1, 0);
#pragma unroll
  for (int j = 0; j < RY; ++j) { rc_[j] = rnew[j]; mq0[j] = mq2[j]; }
  issue(0, C.z0 + 1, C.z0 + 2);
  __syncthreads();
  tphase(0, C.z0 + 1, 0, 1);
#pragma unroll
  for (int j = 0; j < RY; ++j) { rnx[j] = rnew[j]; mq1[j] = mq2[j]; }
  issue(0, C.z0 + 2, C.z0 + 3);
  if constexpr (NS == 2) issue(NS - 1, C.z0 + 3, C.z0 + 4);
  __syncthreads();

  double acc = 0.0;
  double2 sa = make_double2(0.0, 0.0);
  int cur = 0, bp = 1;
  // one plane of s; a step with z >= z1 (odd slab length) stores and sums nothing
  auto step = [&](const int st, int z) __attribute__((always_inline)) {
    const bool zin = z < C.z1;
    const unsigned zbit = zin ? 0u : kOOB;
    const double sz2 = sponge_axis_d(z, nz, nbw, inv_nb);
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      const int ly = w * RY + j;
      const float2 xm = pl[cur][ly + 1][lane];
      const float2 xp = pl[cur][ly + 1][lane + 2];
      const float2 ym = (j > 0) ? rc_[j > 0 ? j - 1 : 0] : pl[cur][ly][lane + 1];
      const float2 yp = (j < RY - 1) ? rc_[j < RY - 1 ? j + 1 : 0] : pl[cur][ly + 2][lane + 1];
      const double b = sp_scale * (sxy2[j] + sz2);
      double2 sd = helm(rc_[j], xm, xp, ym, yp, rm[j], rnx[j], h2inv, w2 * (double)mq0[j], om * b);
      if (rc.at(j, z - C.z0)) {  // receiver column of S^H: lambda r2 at the receiver cell
        const int q = rc.take(S, j);
        float2 r2 = ld2(r2v, q);
        if (!setup) {
          r2 = axpy2(r2, -af, ld2(t2v, q));
          st2(r2v, q, r2);
        }
        sd.x += lam * r2.x;
        sd.y += lam * r2.y;
      }
      const float2 s = round2(sd);
      if (j == srcj && src_in_slab && z == sz) {
        sa = make_double2(-acol * (double)rc_[j].x, -acol * (double)rc_[j].y);
        acc += sa.x * sa.x + sa.y * sa.y;
      }
      const bool live = C.in[j] && zin;
      const unsigned o8 = own_b(z, j) | zbit;
      bst2(Rso, o8, s);
      bst2(Rrn, o8, rc_[j]);
      acc += live ? norm2d(s) : 0.0;
    }
    tphase(st, z + 2, bp, (cur + 2) % 3);
    float2 rn2[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) rn2[j] = rnew[j];
    __builtin_amdgcn_sched_barrier(0);
    issue(st, z + 2 + NS, z + 3 + NS);
    __syncthreads();
    cur = (cur + 1) % 3;
    bp ^= 1;
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      rm[j] = rc_[j]; rc_[j] = rnx[j]; rnx[j] = rn2[j];
      mq0[j] = mq1[j]; mq1[j] = mq2[j];
    }
  };
  for (int z = C.z0; z < C.z1; z += 2) {
    step(0, z);
    step(NS - 1, z + 1);
  }

  const double tot = block_reduce<W>(acc, red);
  if (tid == 0) part_s[S.slot_base + tile] = tot;
  if (tile == 0 && tid == 0) T->iterA = k + 1;
  if (srcj >= 0 && src_in_slab) T->sa = sa;
}

// ---------------------------------------------------------------------------
// dispatch over the supported tile shapes
// ---------------------------------------------------------------------------

#define WRI_TILE_LIST(X) X(4, 1) X(4, 2) X(4, 4) X(8, 1) X(8, 2) X(2, 8) X(8, 4)

bool cfg_supported(const TileCfg& c) {
#define X(W_, R_) if (c.w == W_ && c.ry == R_) return c.tz >= 1 && c.tz <= 64 && c.pf >= 0 && c.pf <= 3;
  WRI_TILE_LIST(X)
#undef X
  return false;
}

hipError_t launch_fwd(const TileCfg& c, const SysDev* sys, SysState* st, const double* part_s, double* part_d,
                      const GroupDesc* gd, int ngroups, int nblocks, int k, hipStream_t s) {
  if (nblocks <= 0 || ngroups <= 0) return hipSuccess;
  const unsigned nb = (unsigned)nblocks;
#define X(W_, R_)                                                                                   \
  if (c.w == W_ && c.ry == R_) {                                                                    \
    if (c.pf == 1 && fwd_x_step(k))                                                                 \
      hipLaunchKernelGGL((k_fwd_pf<W_, R_, 1, 0>), dim3(nb), dim3(64 * W_), 0, s, sys, st, part_s,     \
                         part_d, gd, ngroups);                                                      \
    else if (c.pf == 1)                                                                             \
      hipLaunchKernelGGL((k_fwd_pf<W_, R_, 0, 0>), dim3(nb), dim3(64 * W_), 0, s, sys, st, part_s,     \
                         part_d, gd, ngroups);                                                      \
    else if (c.pf >= 2 && fwd_x_step(k))                                                            \
      hipLaunchKernelGGL((k_fwd_pf<W_, R_, 1, 1>), dim3(nb), dim3(64 * W_), 0, s, sys, st, part_s,     \
                         part_d, gd, ngroups);                                                      \
    else if (c.pf >= 2)                                                                             \
      hipLaunchKernelGGL((k_fwd_pf<W_, R_, 0, 1>), dim3(nb), dim3(64 * W_), 0, s, sys, st, part_s,     \
                         part_d, gd, ngroups);                                                      \
    else                                                                                            \
      hipLaunchKernelGGL((k_fwd<W_, R_>), dim3(nb), dim3(64 * W_), 0, s, sys, st, part_s, part_d,     \
                         gd, ngroups);                                                              \
    return hipGetLastError();                                                                       \
  }
  WRI_TILE_LIST(X)
#undef X
  return hipErrorInvalidValue;
}

int adj_blocks_per_cu(const TileCfg& c) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
#define X(W_, R_)                                                                                   \
  if (c.w == W_ && c.ry == R_) {                                                                    \
    if (c.pf == 1) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_adj_pf<W_, R_>, 64 * W_, 0);  \
    else if (c.pf == 2) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_adj_rc<W_, R_, 1>, 64 * W_, 0); \
    else if (c.pf == 3) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_adj_rc<W_, R_, 2>, 64 * W_, 0); \
    else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_adj<W_, R_>, 64 * W_, 0);         \
  }
  WRI_TILE_LIST(X)
#undef X
  return e == hipSuccess ? nb : 0;
}

hipError_t launch_adj(const TileCfg& c, const SysDev* sys, SysState* st, const double* part_d, double* part_s,
                      const GroupDesc* gd, int ngroups, int nblocks, hipStream_t s, int setup_only) {
  if (nblocks <= 0 || ngroups <= 0) return hipSuccess;
  const unsigned nb = (unsigned)nblocks;
#define X(W_, R_)                                                                                   \
  if (c.w == W_ && c.ry == R_) {                                                                    \
    if (c.pf == 1)                                                                                  \
      hipLaunchKernelGGL((k_adj_pf<W_, R_>), dim3(nb), dim3(64 * W_), 0, s, sys, st, part_d, part_s,  \
                         gd, ngroups, setup_only);                                                  \
    else if (c.pf == 2)                                                                             \
      hipLaunchKernelGGL((k_adj_rc<W_, R_, 1>), dim3(nb), dim3(64 * W_), 0, s, sys, st, part_d, part_s, \
                         gd, ngroups, setup_only);                                                  \
    else if (c.pf == 3)                                                                             \
      hipLaunchKernelGGL((k_adj_rc<W_, R_, 2>), dim3(nb), dim3(64 * W_), 0, s, sys, st, part_d, part_s, \
                         gd, ngroups, setup_only);                                                  \
    else                                                                                            \
      hipLaunchKernelGGL((k_adj<W_, R_>), dim3(nb), dim3(64 * W_), 0, s, sys, st, part_d, part_s,     \
                         gd, ngroups, setup_only);                                                  \
    return hipGetLastError();                                                                       \
  }
  WRI_TILE_LIST(X)
#undef X
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// gradient  g = sum_rhs 2 omega^2 Re(conj(u) (A u - a e)) = -sum 2 omega^2 Re(conj(u) r1)
// and the per-block partials of ||r1||^2 for J.  Systems of one grid only.
// ---------------------------------------------------------------------------

constexpr int kGradThreads = 256;
constexpr int kGradCells = 4;   // cells per thread

int grad_blocks(int n) {
  const int per = kGradThreads * kGradCells;
  return (n + per - 1) / per;
}

__global__ void __launch_bounds__(kGradThreads)
k_grad(const SysDev* __restrict__ sysv, const SysState* __restrict__ stv, int rhs0, int nrhs, int n,
       float* __restrict__ grad, double* __restrict__ part_j, int stride, int accumulate) {
  __shared__ double red[kGradThreads / 64 + 1];
  const int base = blockIdx.x * (kGradThreads * kGradCells);
  double g[kGradCells];
#pragma unroll
  for (int i = 0; i < kGradCells; ++i) g[i] = 0.0;
  for (int r = 0; r < nrhs; ++r) {
    const SysDev& S = sysv[rhs0 + r];
    const SysState& T = stv[rhs0 + r];
    const bool ok = T.status != kBreakdown;
    const float2* __restrict__ r1 = S.r[T.iterA & 1];
    const float2* __restrict__ u = S.x;
    const double w2 = -2.0 * (double)S.omega_d * (double)S.omega_d;
    double jj = 0.0;
#pragma unroll
    for (int i = 0; i < kGradCells; ++i) {
      const int c = base + i * kGradThreads + threadIdx.x;
      if (ok && c < n) {
        const float2 rv = r1[c], uv = u[c];
        g[i] += w2 * ((double)uv.x * (double)rv.x + (double)uv.y * (double)rv.y);
        jj += norm2d(rv);
      }
    }
    const double tot = block_reduce<kGradThreads / 64>(jj, red);
    if (threadIdx.x == 0) part_j[(size_t)(rhs0 + r) * stride + blockIdx.x] = tot;
  }
  if (grad == nullptr) return;
#pragma unroll
  for (int i = 0; i < kGradCells; ++i) {
    const int c = base + i * kGradThreads + threadIdx.x;
    if (c < n) grad[c] = accumulate ? (float)((double)grad[c] + g[i]) : (float)g[i];
  }
}

hipError_t launch_grad(const SysDev* sys, SysState* st, int rhs0, int nrhs, int n, float* grad,
                       double* part_j, int stride, int accumulate, hipStream_t s) {
  const int nb = grad_blocks(n);
  if (nb == 0 || nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_grad, dim3(nb), dim3(kGradThreads), 0, s, sys, st, rhs0, nrhs, n, grad, part_j,
                     stride, accumulate);
  return hipGetLastError();
}

// One block per system: J = sum(part_j) + ||r2||^2, and (A u)[src] in float64.
__global__ void __launch_bounds__(64)
k_finalize(const SysDev* __restrict__ sysv, SysState* __restrict__ stv, const double* __restrict__ part_j,
           int nparts, int stride, int rhs0) {
  const int rhs = rhs0 + blockIdx.x;
  const SysDev& S = sysv[rhs];
  SysState* T = stv + rhs;
  double v = 0.0;
  if (part_j != nullptr)
    for (int i = threadIdx.x; i < nparts; i += 64) v += part_j[(size_t)rhs * stride + i];
  for (int q = threadIdx.x; q < S.n_rec; q += 64) v += norm2d(S.r2[q]);
  v = wave_sum(v);
  if (threadIdx.x == 0) {
    T->J = v;
    if (S.mode == 1) {
      const int plane = S.nx * S.ny;
      const int c = S.src;
      const int z = c / plane, y = (c % plane) / S.nx, x = c % S.nx;
      const float2* u = S.x;
      const double2 uc = make_double2(u[c].x, u[c].y);
      double lr = 0.0, li = 0.0;
      auto nb = [&](bool inside, int cc) {
        double vr = 0.0, vi = 0.0;
        if (inside) { vr = u[cc].x; vi = u[cc].y; }
        lr += vr - uc.x;
        li += vi - uc.y;
      };
      nb(x > 0, c - 1);
      nb(x < S.nx - 1, c + 1);
      nb(y > 0, c - S.nx);
      nb(y < S.ny - 1, c + S.nx);
      nb(z > 0, c - plane);
      nb(z < S.nz - 1, c + plane);
      const double b = S.sp_scale_d * (sponge_axis_d(x, S.nx, S.nb, S.inv_nb_d) +
                                       sponge_axis_d(y, S.ny, S.nb, S.inv_nb_d) +
                                       sponge_axis_d(z, S.nz, S.nb, S.inv_nb_d));
      const double kre = S.omega_d * S.omega_d * (double)S.m[c];
      const double kim = -S.omega_d * b;
      T->alpha_ls = make_double2(lr * S.h2inv_d + kre * uc.x - kim * uc.y,
                                 li * S.h2inv_d + kre * uc.y + kim * uc.x);
    } else {
      T->alpha_ls = S.alpha;
    }
  }
}

hipError_t launch_finalize(const SysDev* sys, SysState* st, const double* part_j, int nparts, int stride,
                           int rhs0, int nrhs, hipStream_t s) {
  if (nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize, dim3(nrhs), dim3(64), 0, s, sys, st, part_j, nparts, stride, rhs0);
  return hipGetLastError();
}

__global__ void k_zero_f32(float* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

hipError_t launch_zero_f32(float* p, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_f32, dim3(1024), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// single-operator stencil (one thread per cell; same cell arithmetic) and the
// unfused kernels of the plain baseline
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256)
k_apply(int nx, int ny, int nz, int nbw, double h2inv, double sp_scale, double inv_nb, double omega,
        const float* __restrict__ m, const float2* __restrict__ in, float2* __restrict__ out, int adjoint, int src,
        double2 src_sub) {
  const int plane = nx * ny;
  const int n = plane * nz;
  const double w2 = omega * omega;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    const int z = c / plane, rem = c - z * plane, y = rem / nx, x = rem - y * nx;
    const float2 zero = f2(0.f, 0.f);
    const float2 cc = in[c];
    const float2 xm = x > 0 ? in[c - 1] : zero;
    const float2 xp = x < nx - 1 ? in[c + 1] : zero;
    const float2 ym = y > 0 ? in[c - nx] : zero;
    const float2 yp = y < ny - 1 ? in[c + nx] : zero;
    const float2 zm = z > 0 ? in[c - plane] : zero;
    const float2 zp = z < nz - 1 ? in[c + plane] : zero;
    const double b = sp_scale * ((sponge_axis_d(x, nx, nbw, inv_nb) + sponge_axis_d(y, ny, nbw, inv_nb)) +
                                 sponge_axis_d(z, nz, nbw, inv_nb));
    const double kim = adjoint ? (omega * b) : -(omega * b);
    double2 o = helm(cc, xm, xp, ym, yp, zm, zp, h2inv, w2 * (double)m[c], kim);
    if (c == src) { o.x -= src_sub.x; o.y -= src_sub.y; }
    out[c] = round2(o);
  }
}

static unsigned blocks_for(size_t n, unsigned threads = 256, unsigned cap = 65535u * 4u) {
  size_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

hipError_t launch_apply(int nx, int ny, int nz, int nb, double h2inv, double sp_scale, double inv_nb,
                        double omega, const float* m, const float2* in, float2* out, int adjoint, int src,
                        double2 src_sub, hipStream_t s) {
  const size_t n = (size_t)nx * ny * nz;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_apply, dim3(blocks_for(n)), dim3(256), 0, s, nx, ny, nz, nb, h2inv, sp_scale, inv_nb,
                     omega, m, in, out, adjoint, src, src_sub);
  return hipGetLastError();
}

__global__ void k_gather(float2* __restrict__ t2, const float2* __restrict__ p, const int* __restrict__ rec,
                         int n_rec, double lam) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n_rec) {
    const float2 v = p[rec[q]];
    t2[q] = f2((float)(lam * v.x), (float)(lam * v.y));
  }
}

hipError_t launch_gather(float2* t2, const float2* p, const int* rec, int n_rec, double lam, hipStream_t s) {
  if (n_rec <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather, dim3((n_rec + 255) / 256), dim3(256), 0, s, t2, p, rec, n_rec, lam);
  return hipGetLastError();
}

// receiver indices are distinct within a system: no two threads touch one cell
__global__ void k_scatter(float2* __restrict__ sv, const float2* __restrict__ r2, const int* __restrict__ rec,
                          int n_rec, double lam) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n_rec) {
    const int c = rec[q];
    sv[c] = axpy2(sv[c], lam, r2[q]);
  }
}

hipError_t launch_scatter(float2* sv, const float2* r2, const int* rec, int n_rec, double lam, hipStream_t s) {
  if (n_rec <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter, dim3((n_rec + 255) / 256), dim3(256), 0, s, sv, r2, rec, n_rec, lam);
  return hipGetLastError();
}

constexpr int kDotThreads = 256;

int dot_parts(int n) {
  int b = (n + kDotThreads * 8 - 1) / (kDotThreads * 8);
  if (b < 1) b = 1;
  if (b > 2048) b = 2048;
  return b;
}

__global__ void __launch_bounds__(kDotThreads) k_dot(const float2* __restrict__ v, int n, double* __restrict__ part) {
  __shared__ double red[kDotThreads / 64 + 1];
  double acc = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) acc += norm2d(v[i]);
  const double tot = block_reduce<kDotThreads / 64>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

hipError_t launch_dot(const float2* v, int n, double* part, int nparts, hipStream_t s) {
  hipLaunchKernelGGL(k_dot, dim3(nparts), dim3(kDotThreads), 0, s, v, n, part);
  return hipGetLastError();
}

__global__ void k_sum(const double* __restrict__ part, int nparts, double* __restrict__ out) {
  double v = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 64) v += part[i];
  v = wave_sum(v);
  if (threadIdx.x == 0) *out = v;
}

hipError_t launch_sum(const double* part, int nparts, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(64), 0, s, part, nparts, out);
  return hipGetLastError();
}

__global__ void k_axpy(float2* __restrict__ y, const float2* __restrict__ x, double a, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    y[i] = axpy2(y[i], a, x[i]);
}

hipError_t launch_axpy(float2* y, const float2* x, double a, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy, dim3(blocks_for(n)), dim3(256), 0, s, y, x, a, n);
  return hipGetLastError();
}

__global__ void k_xpby(float2* __restrict__ p, const float2* __restrict__ sv, double b, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    p[i] = axpy2(sv[i], b, p[i]);
}

hipError_t launch_xpby(float2* p, const float2* sv, double b, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_xpby, dim3(blocks_for(n)), dim3(256), 0, s, p, sv, b, n);
  return hipGetLastError();
}

__global__ void k_copy_f2(float2* __restrict__ d, const float2* __restrict__ sv, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) d[i] = sv[i];
}

hipError_t launch_copy_f2(float2* dst, const float2* src, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_f2, dim3(blocks_for(n)), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}

__global__ void k_fill_f2(float2* __restrict__ d, float2 v, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) d[i] = v;
}

hipError_t launch_fill_f2(float2* dst, float2 v, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f2, dim3(blocks_for(n)), dim3(256), 0, s, dst, v, n);
  return hipGetLastError();
}

__global__ void k_scale_f2(float2* __restrict__ d, const float2* __restrict__ sv, float a, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    d[i] = f2(a * sv[i].x, a * sv[i].y);
}

hipError_t launch_scale_f2(float2* dst, const float2* src, float a, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_f2, dim3(blocks_for(n)), dim3(256), 0, s, dst, src, a, n);
  return hipGetLastError();
}

__global__ void k_set_state(SysState* st, int rhs, int iters, int status, double2 xa, double gamma,
                            double gamma0) {
  if (threadIdx.x == 0) {
    SysState* T = st + rhs;
    T->iters = iters;
    T->status = status;
    T->xa = xa;
    T->gamma[iters & 1] = gamma;
    T->gamma0 = gamma0;
    T->iterA = 0;
  }
}

hipError_t launch_set_state(SysState* st, int rhs, int iters, int status, double2 xa, double gamma,
                            double gamma0, hipStream_t s) {
  hipLaunchKernelGGL(k_set_state, dim3(1), dim3(64), 0, s, st, rhs, iters, status, xa, gamma, gamma0);
  return hipGetLastError();
}

}  // namespace wri
