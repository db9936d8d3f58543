// Sources and receivers off the grid nodes: the source vector e and the
// receiver sampling P of eqs. ObjPen / SimpObj become trilinear interpolation
// weights over up to 8 cells each, and the same CGLS (the reading of
// Algorithm 1 used throughout the library) runs for all systems of a call in
// lockstep, four launches per iteration: a forward pass (p update and
// t = A p at each cell from its neighbours' recomputed p), a one-block-per-
// system pass for the source column, P p and the step a, an adjoint pass
// (r update, s = A^H r, x update) and a one-block-per-system pass for P^H r2,
// the source row and beta.  The stencil arithmetic is the fused kernels'
// (stencil.hpp); step scalars live in device memory; chunks of iterations
// replay from a hipGraph and the host checks the statuses between them.
//
// P p: one thread per receiver sums its weighted cells (reads only).  P^H r2:
// a gather over the distinct receiver cells of a system (each cell's list of
// (receiver, weight) pairs is built on the host), so cells shared by several
// receivers need no atomics.  Source cells are distinct by construction.
// Every reduction runs in one fixed order.
#include "../../include/wri.h"
#include "wri_impl.hpp"
#include "stencil.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <vector>

namespace wri {
namespace {

constexpr int kThreads = 256;
constexpr size_t kAl = 256;
size_t al(size_t v) { return (v + kAl - 1) / kAl * kAl; }

#define OG_HIP(expr)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return report_error(WRI_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

int nblk(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + kThreads - 1) / kThreads, 4096)); }

constexpr int kParts = 128;  // blocks (and partial sums) per system in the stencil passes
constexpr int kCheck = 32;   // iterations between host checks of the statuses

// One system, resident in the workspace.  r and p are ping-pong pairs (the
// stencil passes read neighbours of the old vector while writing the new one).
struct OgSys {
  float2 *x, *r[2], *p[2], *s, *t, *r2, *t2;
  const float2* d;
  const int* scell; const double* sw;
  const int* rptr; const int* rcell; const double* rw;
  const int* uptr; const int* ucell; const int* uq; const double* uw;
  const float* m;
  int n, ns, nr, nu;
  int est, max_iter, nx, ny, nz, nb, zc, pad2_;
  double c, lam, rtol2, omega, omega2, h2inv, sp_scale, inv_nb;
  double2 alpha;  // KNOWN-mode weight
};

// Mutable scalars of one system (float64).  iters = k while iteration k runs:
// p_k is in p[k & 1], r_k in r[k & 1].
struct OgState {
  double gamma, gamma0, a, beta, J;
  double2 xa, pa, sa, eau;
  int status, iters, pad_[2];
};

__device__ __forceinline__ double bsum(double v, double* red) {  // all threads get the block total
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < kThreads / 64; ++i) r += red[i];
  __syncthreads();
  return r;
}

__device__ __forceinline__ float2 f2d(double a, double b) { return make_float2((float)a, (float)b); }
__device__ __forceinline__ double nrm(float2 v) { return (double)v.x * v.x + (double)v.y * v.y; }
// y + a x in float64, rounded once: the value every neighbour recomputes identically
__device__ __forceinline__ float2 axpyd(float2 y, double a, float2 x) {
  return f2d((double)y.x + a * (double)x.x, (double)y.y + a * (double)x.y);
}

__device__ __forceinline__ double sponge_at(const OgSys& S, int x, int y, int z) {
  return S.sp_scale * ((sponge_axis_d(x, S.nx, S.nb, S.inv_nb) + sponge_axis_d(y, S.ny, S.nb, S.inv_nb)) +
                       sponge_axis_d(z, S.nz, S.nb, S.inv_nb));
}

// x = 0, r_0 = 0, p_{-1} = 0 (grid (blocks, nsys))
__global__ void __launch_bounds__(kThreads) k_og_zero(const OgSys* __restrict__ sy) {
  const OgSys& S = sy[blockIdx.y];
  const float2 z = make_float2(0.f, 0.f);
  for (int c = blockIdx.x * kThreads + threadIdx.x; c < S.n; c += gridDim.x * kThreads) {
    S.x[c] = z;
    S.r[0][c] = z;
    S.p[1][c] = z;
  }
}

// t = A x (the least-squares source weight of the result)  (grid (blocks, nsys))
__global__ void __launch_bounds__(kThreads) k_og_ax(const OgSys* __restrict__ sy) {
  const OgSys& S = sy[blockIdx.y];
  const int nx = S.nx, ny = S.ny, nz = S.nz, plane = nx * ny;
  const float2 zero = make_float2(0.f, 0.f);
  const float2* __restrict__ in = S.x;
  for (int c = blockIdx.x * kThreads + threadIdx.x; c < S.n; c += gridDim.x * kThreads) {
    const int z = c / plane, rem = c - z * plane, y = rem / nx, x = rem - y * nx;
    const float2 xm = x > 0 ? in[c - 1] : zero, xp = x < nx - 1 ? in[c + 1] : zero;
    const float2 ym = y > 0 ? in[c - nx] : zero, yp = y < ny - 1 ? in[c + nx] : zero;
    const float2 zm = z > 0 ? in[c - plane] : zero, zp = z < nz - 1 ? in[c + plane] : zero;
    S.t[c] = round2(helm(in[c], xm, xp, ym, yp, zm, zp, S.h2inv, S.omega2 * (double)S.m[c],
                         -(S.omega * sponge_at(S, x, y, z))));
  }
}

// r_0[src] = alpha e (KNOWN), r2 = lam d, state reset (grid nsys)
__global__ void __launch_bounds__(kThreads) k_og_init(const OgSys* __restrict__ sy, OgState* __restrict__ stv) {
  const OgSys& S = sy[blockIdx.x];
  if (!S.est && (int)threadIdx.x < S.ns) {
    const double w = S.sw[threadIdx.x];
    S.r[0][S.scell[threadIdx.x]] = f2d(S.alpha.x * w, S.alpha.y * w);
  }
  for (int q = threadIdx.x; q < S.nr; q += kThreads)
    S.r2[q] = f2d(S.lam * (double)S.d[q].x, S.lam * (double)S.d[q].y);
  if (threadIdx.x == 0) {
    OgState& T = stv[blockIdx.x];
    T = OgState{};
    T.status = kActive;
  }
}

// Work items of the stencil passes: a 64 x 4 tile of (x, y) columns (one
// thread each) and a chunk of S.zc planes marched in z.  Each plane of the
// recomputed vector (p_k or r_{k+1}) is staged with a one-cell halo in LDS for
// the x/y neighbours; the z-neighbours stay in registers.  Every block runs
// the same number of items and planes (the barriers are uniform); threads
// outside the grid hold zeros.
constexpr int kZc = 16;
constexpr int kTy = kThreads / 64;               // tile rows
constexpr int kHalo = 2 * (64 + 2) + 2 * kTy;    // halo cells of one tile plane

struct TileWork {
  int x, y, z0, z1, col;
  bool in;
};

__device__ __forceinline__ int tile_items(const OgSys& S) {
  return ((S.nx + 63) / 64) * ((S.ny + kTy - 1) / kTy) * ((S.nz + S.zc - 1) / S.zc);
}

__device__ __forceinline__ TileWork tile_work(const OgSys& S, int w) {
  const int tx_n = (S.nx + 63) / 64, ty_n = (S.ny + kTy - 1) / kTy;
  const int t = w % (tx_n * ty_n), zc = w / (tx_n * ty_n);
  TileWork W;
  W.x = (t % tx_n) * 64 + (threadIdx.x & 63);
  W.y = (t / tx_n) * kTy + (threadIdx.x >> 6);
  W.z0 = zc * S.zc;
  W.z1 = min(W.z0 + S.zc, S.nz);
  W.in = W.x < S.nx && W.y < S.ny;
  W.col = W.y * S.nx + W.x;
  return W;
}

// halo cell h of the tile containing (x0, y0) (its corner cell): LDS slot and grid cell
__device__ __forceinline__ void halo_cell(int h, int x0, int y0, int* hx, int* hy, int* gx, int* gy) {
  if (h < 66) { *hy = 0; *hx = h; }
  else if (h < 132) { *hy = kTy + 1; *hx = h - 66; }
  else { const int q = h - 132; *hy = 1 + (q >> 1); *hx = (q & 1) ? 65 : 0; }
  *gx = x0 + *hx - 1;
  *gy = y0 + *hy - 1;
}

// Forward pass of iteration k: p_k = s_k + beta p_{k-1} (computed at the cell
// and its neighbours), t = A p_k, per-block partials of ||t||^2 (the
// source-column term is added by k_og_alpha).  grid (kParts, nsys).
__global__ void __launch_bounds__(kThreads) k_og_fwd(const OgSys* __restrict__ sy, const OgState* __restrict__ stv,
                                                     double* __restrict__ parts) {
  __shared__ double red[kThreads / 64];
  __shared__ float2 pl[kTy + 2][66];
  const OgSys& S = sy[blockIdx.y];
  const OgState& T = stv[blockIdx.y];
  double acc = 0.0;
  if (T.status == kActive) {  // uniform over the block
    const int k = T.iters;
    const float2* __restrict__ sv = S.s;
    const float2* __restrict__ po = S.p[(k + 1) & 1];
    float2* __restrict__ pn = S.p[k & 1];
    const double beta = T.beta;
    const int nx = S.nx, ny = S.ny, nz = S.nz, plane = nx * ny;
    const float2 zero = make_float2(0.f, 0.f);
    const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
    auto P = [&](int c) { return axpyd(sv[c], beta, po[c]); };
    const int items = tile_items(S);
    for (int w = blockIdx.x; w < items; w += kParts) {
      const TileWork W = tile_work(S, w);
      int hx = 0, hy = 0, gx = -1, gy = -1;
      if ((int)threadIdx.x < kHalo) halo_cell(threadIdx.x, W.x - lx, W.y - ly, &hx, &hy, &gx, &gy);
      const bool hin = (int)threadIdx.x < kHalo && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
      const double sxy = W.in ? sponge_axis_d(W.x, nx, S.nb, S.inv_nb) + sponge_axis_d(W.y, ny, S.nb, S.inv_nb) : 0.0;
      float2 vm = (W.in && W.z0 > 0) ? P((W.z0 - 1) * plane + W.col) : zero;
      float2 vc = W.in ? P(W.z0 * plane + W.col) : zero;
      for (int z = W.z0; z < W.z1; ++z) {
        pl[ly + 1][lx + 1] = vc;
        if ((int)threadIdx.x < kHalo) pl[hy][hx] = hin ? P(z * plane + gy * nx + gx) : zero;
        __syncthreads();
        const int c = z * plane + W.col;
        const float2 vp = (W.in && z + 1 < nz) ? P(c + plane) : zero;
        if (W.in) {
          pn[c] = vc;
          const double b = S.sp_scale * (sxy + sponge_axis_d(z, nz, S.nb, S.inv_nb));
          const float2 tv = round2(helm(vc, pl[ly + 1][lx], pl[ly + 1][lx + 2], pl[ly][lx + 1], pl[ly + 2][lx + 1], vm,
                                        vp, S.h2inv, S.omega2 * (double)S.m[c], -(S.omega * b)));
          S.t[c] = tv;
          acc += nrm(tv);
        }
        __syncthreads();
        vm = vc;
        vc = vp;
      }
    }
  }
  acc = bsum(acc, red);
  if (threadIdx.x == 0) parts[blockIdx.y * kParts + blockIdx.x] = acc;
}

// delta = ||t||^2 with the source column (t[src] -= c p_a w) + ||t2||^2 with
// t2 = lam P p_k; a = gamma / delta; x_a += a p_a; r2 -= a t2  (grid nsys)
__global__ void __launch_bounds__(kThreads) k_og_alpha(const OgSys* __restrict__ sy, OgState* __restrict__ stv,
                                                       const double* __restrict__ parts) {
  __shared__ double red[kThreads / 64];
  const OgSys& S = sy[blockIdx.x];
  OgState& T = stv[blockIdx.x];
  if (T.status != kActive) return;  // uniform over the block
  const float2* __restrict__ pk = S.p[T.iters & 1];
  double v = 0.0;
  for (int i = threadIdx.x; i < kParts; i += kThreads) v += parts[blockIdx.x * kParts + i];
  if (S.est && (int)threadIdx.x < S.ns) {  // distinct source cells, one per thread
    const int c = S.scell[threadIdx.x];
    const double w = S.sw[threadIdx.x];
    const float2 t0 = S.t[c];
    const float2 t1 = f2d((double)t0.x - S.c * T.pa.x * w, (double)t0.y - S.c * T.pa.y * w);
    S.t[c] = t1;
    v += nrm(t1) - nrm(t0);
  }
  for (int q = threadIdx.x; q < S.nr; q += kThreads) {
    double re = 0.0, im = 0.0;
    for (int j = S.rptr[q]; j < S.rptr[q + 1]; ++j) {
      const float2 x = pk[S.rcell[j]];
      re += S.rw[j] * (double)x.x;
      im += S.rw[j] * (double)x.y;
    }
    const float2 t2 = f2d(S.lam * re, S.lam * im);
    S.t2[q] = t2;
    v += nrm(t2);
  }
  const double delta = bsum(v, red);
  const double gamma = T.gamma;
  const bool bad = !(delta > 0.0) || !isfinite(delta) || !isfinite(gamma);
  const double a = bad ? 0.0 : gamma / delta;
  if (!bad)
    for (int q = threadIdx.x; q < S.nr; q += kThreads) S.r2[q] = axpyd(S.r2[q], -a, S.t2[q]);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (bad) {
      T.status = kBreakdown;
    } else {
      T.a = a;
      T.xa = make_double2(T.xa.x + a * T.pa.x, T.xa.y + a * T.pa.y);
    }
  }
}

// Adjoint pass: r_{k+1} = r_k - a t (at the cell and its neighbours),
// s = A^H r_{k+1}, x += a p_k, per-block partials of ||s||^2 (the receiver
// rows are added by k_og_beta).  setup = 1: the pass on r_0 with no update
// (s_0 = A^H r_0, copied r_0 into r_1).  Same tiles as k_og_fwd.
// grid (kParts, nsys).
__global__ void __launch_bounds__(kThreads) k_og_adj(const OgSys* __restrict__ sy, const OgState* __restrict__ stv,
                                                     double* __restrict__ parts, int setup) {
  __shared__ double red[kThreads / 64];
  __shared__ float2 pl[kTy + 2][66];
  const OgSys& S = sy[blockIdx.y];
  const OgState& T = stv[blockIdx.y];
  double acc = 0.0;
  if (setup || T.status == kActive) {  // uniform over the block
    const int k = setup ? 0 : T.iters;
    const double a = setup ? 0.0 : T.a;
    const float2* __restrict__ ro = S.r[k & 1];
    float2* __restrict__ rn = S.r[(k + 1) & 1];
    const float2* __restrict__ tv = S.t;
    const float2* __restrict__ pk = S.p[k & 1];
    const int nx = S.nx, ny = S.ny, nz = S.nz, plane = nx * ny;
    const float2 zero = make_float2(0.f, 0.f);
    const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
    auto R = [&](int c) { return setup ? ro[c] : axpyd(ro[c], -a, tv[c]); };
    const int items = tile_items(S);
    for (int w = blockIdx.x; w < items; w += kParts) {
      const TileWork W = tile_work(S, w);
      int hx = 0, hy = 0, gx = -1, gy = -1;
      if ((int)threadIdx.x < kHalo) halo_cell(threadIdx.x, W.x - lx, W.y - ly, &hx, &hy, &gx, &gy);
      const bool hin = (int)threadIdx.x < kHalo && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
      const double sxy = W.in ? sponge_axis_d(W.x, nx, S.nb, S.inv_nb) + sponge_axis_d(W.y, ny, S.nb, S.inv_nb) : 0.0;
      float2 vm = (W.in && W.z0 > 0) ? R((W.z0 - 1) * plane + W.col) : zero;
      float2 vc = W.in ? R(W.z0 * plane + W.col) : zero;
      for (int z = W.z0; z < W.z1; ++z) {
        pl[ly + 1][lx + 1] = vc;
        if ((int)threadIdx.x < kHalo) pl[hy][hx] = hin ? R(z * plane + gy * nx + gx) : zero;
        __syncthreads();
        const int c = z * plane + W.col;
        const float2 vp = (W.in && z + 1 < nz) ? R(c + plane) : zero;
        if (W.in) {
          rn[c] = vc;
          const double b = S.sp_scale * (sxy + sponge_axis_d(z, nz, S.nb, S.inv_nb));
          const float2 sv = round2(helm(vc, pl[ly + 1][lx], pl[ly + 1][lx + 2], pl[ly][lx + 1], pl[ly + 2][lx + 1], vm,
                                        vp, S.h2inv, S.omega2 * (double)S.m[c], S.omega * b));
          S.s[c] = sv;
          acc += nrm(sv);
          if (!setup) S.x[c] = axpyd(S.x[c], a, pk[c]);
        }
        __syncthreads();
        vm = vc;
        vc = vp;
      }
    }
  }
  acc = bsum(acc, red);
  if (threadIdx.x == 0) parts[blockIdx.y * kParts + blockIdx.x] = acc;
}

// The receiver rows of S^H r (s += lam P^H r2 over the distinct receiver
// cells) and the source row s_a = -c e^H r, with gamma = ||s||^2 + |s_a|^2:
// shared by the set-up (gamma0) and every iteration (beta, statuses).
__device__ void og_finish_s(const OgSys& S, const float2* __restrict__ r, double pv, double* red, double* gs,
                            double2* sa) {
  double v = pv;
  for (int u = threadIdx.x; u < S.nu; u += kThreads) {
    double re = 0.0, im = 0.0;
    for (int j = S.uptr[u]; j < S.uptr[u + 1]; ++j) {
      const float2 x = S.r2[S.uq[j]];
      re += S.uw[j] * (double)x.x;
      im += S.uw[j] * (double)x.y;
    }
    const int c = S.ucell[u];
    const float2 s0 = S.s[c];
    const float2 s1 = f2d((double)s0.x + S.lam * re, (double)s0.y + S.lam * im);
    S.s[c] = s1;
    v += nrm(s1) - nrm(s0);
  }
  v = bsum(v, red);
  double sr = 0.0, si = 0.0;
  if (S.est)
    for (int i = 0; i < S.ns; ++i) {
      const float2 x = r[S.scell[i]];
      sr -= S.c * S.sw[i] * (double)x.x;
      si -= S.c * S.sw[i] * (double)x.y;
    }
  *gs = v + sr * sr + si * si;
  *sa = make_double2(sr, si);
}

// gamma0 = ||S^H b||^2 after the set-up pass; p_a = s_a, beta = 0 (p_{-1} = 0)  (grid nsys)
__global__ void __launch_bounds__(kThreads) k_og_start(const OgSys* __restrict__ sy, OgState* __restrict__ stv,
                                                       const double* __restrict__ parts) {
  __shared__ double red[kThreads / 64];
  const OgSys& S = sy[blockIdx.x];
  OgState& T = stv[blockIdx.x];
  double v = 0.0;
  for (int i = threadIdx.x; i < kParts; i += kThreads) v += parts[blockIdx.x * kParts + i];
  double g;
  double2 sa;
  og_finish_s(S, S.r[0], v, red, &g, &sa);
  if (threadIdx.x == 0) {
    T.gamma = T.gamma0 = g;
    T.sa = T.pa = sa;
    T.beta = 0.0;
    if (g == 0.0) T.status = kZeroRhs;
    else if (g <= S.rtol2 * g) T.status = kConverged;
    else if (S.max_iter <= 0) T.status = kMaxIter;
  }
}

// s_{k+1} completed, gamma' , beta, statuses, p_a; iteration k done  (grid nsys)
__global__ void __launch_bounds__(kThreads) k_og_beta(const OgSys* __restrict__ sy, OgState* __restrict__ stv,
                                                      const double* __restrict__ parts) {
  __shared__ double red[kThreads / 64];
  const OgSys& S = sy[blockIdx.x];
  OgState& T = stv[blockIdx.x];
  if (T.status != kActive) return;  // uniform over the block
  double v = 0.0;
  for (int i = threadIdx.x; i < kParts; i += kThreads) v += parts[blockIdx.x * kParts + i];
  double gnew;
  double2 sa;
  og_finish_s(S, S.r[(T.iters + 1) & 1], v, red, &gnew, &sa);
  if (threadIdx.x == 0) {
    const double beta = gnew / T.gamma;
    T.beta = beta;
    T.gamma = gnew;
    T.sa = sa;
    T.pa = make_double2(sa.x + beta * T.pa.x, sa.y + beta * T.pa.y);
    T.iters += 1;
    if (gnew <= S.rtol2 * T.gamma0) T.status = kConverged;
    else if (!isfinite(gnew)) T.status = kBreakdown;
    else if (T.iters >= S.max_iter) T.status = kMaxIter;
  }
}

// per-system partials of ||r||^2 for the final residual r[iters & 1]  (grid (kParts, nsys))
__global__ void __launch_bounds__(kThreads) k_og_rnorm(const OgSys* __restrict__ sy, const OgState* __restrict__ stv,
                                                       double* __restrict__ parts) {
  __shared__ double red[kThreads / 64];
  const OgSys& S = sy[blockIdx.y];
  const float2* __restrict__ r = S.r[stv[blockIdx.y].iters & 1];
  double acc = 0.0;
  for (int c = blockIdx.x * kThreads + threadIdx.x; c < S.n; c += kParts * kThreads) acc += nrm(r[c]);
  acc = bsum(acc, red);
  if (threadIdx.x == 0) parts[blockIdx.y * kParts + blockIdx.x] = acc;
}

// J = ||r||^2 + ||r2||^2; e^H (A u) from t = A x  (grid nsys)
__global__ void __launch_bounds__(kThreads) k_og_final(const OgSys* __restrict__ sy, OgState* __restrict__ stv,
                                                       const double* __restrict__ parts) {
  __shared__ double red[kThreads / 64];
  const OgSys& S = sy[blockIdx.x];
  OgState& T = stv[blockIdx.x];
  double v = 0.0;
  for (int i = threadIdx.x; i < kParts; i += kThreads) v += parts[blockIdx.x * kParts + i];
  for (int q = threadIdx.x; q < S.nr; q += kThreads) v += nrm(S.r2[q]);
  v = bsum(v, red);
  if (threadIdx.x == 0) {
    T.J = v;
    double er = 0.0, ei = 0.0;
    if (S.est)
      for (int i = 0; i < S.ns; ++i) {
        const float2 x = S.t[S.scell[i]];
        er += S.sw[i] * (double)x.x;
        ei += S.sw[i] * (double)x.y;
      }
    T.eau = make_double2(er, ei);
  }
}

// g = -sum over the grid's systems of 2 omega^2 Re(conj(x) r)  (systems idx[0..k))
__global__ void __launch_bounds__(kThreads) k_og_grad(const OgSys* __restrict__ sy, const OgState* __restrict__ stv,
                                                      const int* __restrict__ idx, int k, int n,
                                                      float* __restrict__ g) {
  for (int c = blockIdx.x * kThreads + threadIdx.x; c < n; c += gridDim.x * kThreads) {
    double acc = 0.0;
    for (int j = 0; j < k; ++j) {
      const int i = idx[j];
      if (stv[i].status == kBreakdown) continue;
      const OgSys& S = sy[i];
      const float2 a = S.x[c], b = S.r[stv[i].iters & 1][c];
      acc -= 2.0 * S.omega2 * ((double)a.x * b.x + (double)a.y * b.y);
    }
    g[c] = (float)acc;
  }
}

// ---- host-side tables ------------------------------------------------------

struct Point {
  std::vector<int> cells;
  std::vector<double> w;
};

// trilinear cells and weights of point xyz [m] on grid g (distinct cells,
// zero weights dropped); the point is clamped into the grid
Point trilinear(const wri_grid& g, const double* xyz) {
  const int n[3] = {g.nx, g.ny, g.nz};
  int i0[3], i1[3];
  double w0[3], w1[3];
  for (int a = 0; a < 3; ++a) {
    if (n[a] == 1) {
      i0[a] = i1[a] = 0;
      w0[a] = 1.0;
      w1[a] = 0.0;
      continue;
    }
    double xi = xyz[a] / g.h;
    xi = xi < 0.0 ? 0.0 : (xi > n[a] - 1.0 ? n[a] - 1.0 : xi);
    int k = (int)std::floor(xi);
    if (k > n[a] - 2) k = n[a] - 2;
    i0[a] = k;
    i1[a] = k + 1;
    w1[a] = xi - k;
    w0[a] = 1.0 - w1[a];
  }
  std::map<int, double> acc;
  for (int cz = 0; cz < 2; ++cz)
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx) {
        const int x = cx ? i1[0] : i0[0], y = cy ? i1[1] : i0[1], z = cz ? i1[2] : i0[2];
        const double w = (cx ? w1[0] : w0[0]) * (cy ? w1[1] : w0[1]) * (cz ? w1[2] : w0[2]);
        acc[(z * g.ny + y) * g.nx + x] += w;
      }
  Point p;
  for (const auto& kv : acc)
    if (kv.second != 0.0) {
      p.cells.push_back(kv.first);
      p.w.push_back(kv.second);
    }
  return p;
}

struct SysTables {
  Point src;
  std::vector<int> rptr, rcell;      // receiver q: cells rcell[rptr[q] .. rptr[q+1])
  std::vector<double> rw;
  std::vector<int> uptr, ucell, uq;  // distinct cell u: pairs [uptr[u] .. uptr[u+1])
  std::vector<double> uw;
  size_t off = 0;                    // device copy in the workspace
  size_t bytes() const {
    return al(sizeof(int) * src.cells.size()) + al(sizeof(double) * src.w.size()) + al(sizeof(int) * rptr.size()) +
           al(sizeof(int) * rcell.size()) + al(sizeof(double) * rw.size()) + al(sizeof(int) * uptr.size()) +
           al(sizeof(int) * ucell.size()) + al(sizeof(int) * uq.size()) + al(sizeof(double) * uw.size());
  }
};

SysTables build_tables(const wri_grid& g, const wri_positions& pos, int n_rec) {
  SysTables T;
  T.src = trilinear(g, pos.src);
  T.rptr.push_back(0);
  std::map<int, std::vector<std::pair<int, double>>> by_cell;
  for (int q = 0; q < n_rec; ++q) {
    Point r = trilinear(g, pos.rec + 3 * q);
    for (size_t j = 0; j < r.cells.size(); ++j) {
      T.rcell.push_back(r.cells[j]);
      T.rw.push_back(r.w[j]);
      by_cell[r.cells[j]].push_back({q, r.w[j]});
    }
    T.rptr.push_back((int)T.rcell.size());
  }
  T.uptr.push_back(0);
  for (const auto& kv : by_cell) {
    T.ucell.push_back(kv.first);
    for (const auto& pr : kv.second) {
      T.uq.push_back(pr.first);
      T.uw.push_back(pr.second);
    }
    T.uptr.push_back((int)T.uq.size());
  }
  return T;
}

struct DevTables {  // pointers into the workspace
  int* scell; double* sw;
  int* rptr; int* rcell; double* rw;
  int* uptr; int* ucell; int* uq; double* uw;
};

DevTables place(char* base, const SysTables& T) {
  DevTables D;
  size_t o = T.off;
  auto take = [&](size_t bytes) { char* p = base + o; o += al(bytes); return p; };
  D.scell = reinterpret_cast<int*>(take(sizeof(int) * T.src.cells.size()));
  D.sw = reinterpret_cast<double*>(take(sizeof(double) * T.src.w.size()));
  D.rptr = reinterpret_cast<int*>(take(sizeof(int) * T.rptr.size()));
  D.rcell = reinterpret_cast<int*>(take(sizeof(int) * T.rcell.size()));
  D.rw = reinterpret_cast<double*>(take(sizeof(double) * T.rw.size()));
  D.uptr = reinterpret_cast<int*>(take(sizeof(int) * T.uptr.size()));
  D.ucell = reinterpret_cast<int*>(take(sizeof(int) * T.ucell.size()));
  D.uq = reinterpret_cast<int*>(take(sizeof(int) * T.uq.size()));
  D.uw = reinterpret_cast<double*>(take(sizeof(double) * T.uw.size()));
  return D;
}

template <class V>
hipError_t up(void* dst, const std::vector<V>& v, hipStream_t st) {
  if (v.empty()) return hipSuccess;
  return hipMemcpyAsync(dst, v.data(), sizeof(V) * v.size(), hipMemcpyHostToDevice, st);
}

int64_t ncell(const wri_grid& g) { return (int64_t)g.nx * g.ny * g.nz; }

struct OgLayout {
  std::vector<size_t> vec, rvec;  // per system: 5 wavefield vectors (x unless u_out), r2 and t2
  size_t sys = 0, state = 0, parts = 0, idx = 0, total = 0;
};

int validate_offgrid(const wri_grid* grids, int n_grids, const wri_system* sys, int n_sys, const wri_positions* pos,
                     int mode, int max_iter) {
  if (n_grids < 0 || n_sys < 0) return report_error(WRI_EINVAL, "negative n_grids or n_sys");
  if (n_grids > 0 && grids == nullptr) return report_error(WRI_EINVAL, "grids is NULL");
  if (n_sys > 0 && (sys == nullptr || pos == nullptr)) return report_error(WRI_EINVAL, "sys or pos is NULL");
  if (mode != WRI_KNOWN && mode != WRI_ESTIMATE) return report_error(WRI_EINVAL, "bad mode %d", mode);
  if (max_iter < 0) return report_error(WRI_EINVAL, "max_iter < 0");
  for (int i = 0; i < n_grids; ++i) {
    const wri_grid& g = grids[i];
    if (g.nx < 1 || g.ny < 1 || g.nz < 1 || ncell(g) >= (int64_t(1) << 31))
      return report_error(WRI_EINVAL, "grid %d: bad size", i);
    if (!(g.h > 0.0) || !std::isfinite(g.h)) return report_error(WRI_EINVAL, "grid %d: h must be > 0", i);
    if (g.nb < 0 || (g.nb > 0 && !(g.v_ref > 0.0))) return report_error(WRI_EINVAL, "grid %d: bad sponge", i);
  }
  for (int k = 0; k < n_sys; ++k) {
    const wri_system& s = sys[k];
    if (s.grid < 0 || s.grid >= n_grids) return report_error(WRI_EINVAL, "system %d: grid index out of range", k);
    if (!(s.omega >= 0.0) || !std::isfinite(s.omega) || !(s.lambda >= 0.0) || !std::isfinite(s.lambda) ||
        !(s.rtol >= 0.0) || !std::isfinite(s.rtol))
      return report_error(WRI_EINVAL, "system %d: omega, lambda and rtol must be finite and >= 0", k);
    if (s.n_rec < 0) return report_error(WRI_EINVAL, "system %d: n_rec < 0", k);
    if (s.n_rec > 0 && (s.d == nullptr || pos[k].rec == nullptr))
      return report_error(WRI_EINVAL, "system %d: d or receiver positions NULL", k);
    if (mode == WRI_KNOWN && (!std::isfinite(s.alpha.re) || !std::isfinite(s.alpha.im)))
      return report_error(WRI_EINVAL, "system %d: alpha not finite", k);
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(pos[k].src[a])) return report_error(WRI_EINVAL, "system %d: source position not finite", k);
    for (int q = 0; q < 3 * s.n_rec; ++q)
      if (!std::isfinite(pos[k].rec[q])) return report_error(WRI_EINVAL, "system %d: receiver position not finite", k);
  }
  return WRI_OK;
}

int og_layout(const wri_grid* grids, const wri_system* sys, int n_sys, std::vector<SysTables>* tabs, OgLayout* L) {
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = al(o + std::max<size_t>(bytes, 1)); return r; };
  L->vec.resize(n_sys);
  L->rvec.resize(n_sys);
  for (int k = 0; k < n_sys; ++k) {
    L->vec[k] = take(7 * al(sizeof(float2) * (size_t)ncell(grids[sys[k].grid])));
    L->rvec[k] = take(2 * al(sizeof(float2) * (size_t)sys[k].n_rec));
  }
  L->sys = take(sizeof(OgSys) * (size_t)std::max(n_sys, 1));
  L->state = take(sizeof(OgState) * (size_t)std::max(n_sys, 1));
  L->parts = take(sizeof(double) * (size_t)kParts * std::max(n_sys, 1));
  L->idx = take(sizeof(int) * (size_t)std::max(n_sys, 1));
  for (auto& T : *tabs) {
    T.off = o;
    o = al(o + T.bytes());
  }
  L->total = o + kAl;
  return WRI_OK;
}

int og_run(const wri_grid* grids, int n_grids, const float* const* m, const wri_system* sys, int n_sys,
           const wri_positions* pos, int mode, int max_iter, int flags, double* J_out, float* const* grad,
           wri_c32* const* u_out, wri_result* res, void* ws, size_t ws_bytes, hipStream_t st) {
  int rc = validate_offgrid(grids, n_grids, sys, n_sys, pos, mode, max_iter);
  if (rc != WRI_OK) return rc;
  if (n_sys > 0 && res == nullptr) return report_error(WRI_EINVAL, "res is NULL");
  if (flags & (WRI_FLAG_WARM_START | WRI_FLAG_ADJOINT_SOURCE))
    return report_error(WRI_EINVAL, "off-grid solves take no WRI_FLAG_WARM_START or WRI_FLAG_ADJOINT_SOURCE");
  if (n_grids > 0 && m == nullptr) return report_error(WRI_EINVAL, "m is NULL");
  for (int g = 0; g < n_grids; ++g)
    if (m[g] == nullptr || (grad != nullptr && grad[g] == nullptr))
      return report_error(WRI_EINVAL, "m[%d] or grad[%d] is NULL", g, g);
  std::vector<SysTables> tabs(n_sys);
  for (int k = 0; k < n_sys; ++k) tabs[k] = build_tables(grids[sys[k].grid], pos[k], sys[k].n_rec);
  OgLayout L;
  og_layout(grids, sys, n_sys, &tabs, &L);
  if (ws == nullptr || ws_bytes < L.total)
    return report_error(WRI_ENOWS, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, L.total);
  char* base = reinterpret_cast<char*>(al(reinterpret_cast<uintptr_t>(ws)));
  if (J_out) *J_out = 0.0;
  if (n_sys == 0) {
    if (grad != nullptr)
      for (int g = 0; g < n_grids; ++g) OG_HIP(launch_zero_f32(grad[g], (size_t)ncell(grids[g]), st));
    OG_HIP(hipStreamSynchronize(st));
    return WRI_OK;
  }
  // device tables
  std::vector<OgSys> hs(n_sys);
  int64_t nmax = 1;
  int rmax = 1, umax = 1;
  for (int k = 0; k < n_sys; ++k) {
    const wri_system& s = sys[k];
    const wri_grid& g = grids[s.grid];
    const SysTables& T = tabs[k];
    const DevTables D = place(base, T);
    OG_HIP(up(D.scell, T.src.cells, st)); OG_HIP(up(D.sw, T.src.w, st));
    OG_HIP(up(D.rptr, T.rptr, st)); OG_HIP(up(D.rcell, T.rcell, st)); OG_HIP(up(D.rw, T.rw, st));
    OG_HIP(up(D.uptr, T.uptr, st)); OG_HIP(up(D.ucell, T.ucell, st)); OG_HIP(up(D.uq, T.uq, st));
    OG_HIP(up(D.uw, T.uw, st));
    const int64_t n = ncell(g);
    const size_t vb = al(sizeof(float2) * (size_t)n);
    const size_t rb = al(sizeof(float2) * (size_t)s.n_rec);
    float2* v = reinterpret_cast<float2*>(base + L.vec[k]);
    OgSys& S = hs[k];
    S = OgSys{};
    S.x = (u_out != nullptr && u_out[k] != nullptr) ? reinterpret_cast<float2*>(u_out[k]) : v;
    S.r[0] = reinterpret_cast<float2*>(base + L.vec[k] + vb);
    S.r[1] = reinterpret_cast<float2*>(base + L.vec[k] + 2 * vb);
    S.p[0] = reinterpret_cast<float2*>(base + L.vec[k] + 3 * vb);
    S.p[1] = reinterpret_cast<float2*>(base + L.vec[k] + 4 * vb);
    S.s = reinterpret_cast<float2*>(base + L.vec[k] + 5 * vb);
    S.t = reinterpret_cast<float2*>(base + L.vec[k] + 6 * vb);
    S.r2 = reinterpret_cast<float2*>(base + L.rvec[k]);
    S.t2 = reinterpret_cast<float2*>(base + L.rvec[k] + rb);
    S.d = reinterpret_cast<const float2*>(s.d);
    S.scell = D.scell; S.sw = D.sw;
    S.rptr = D.rptr; S.rcell = D.rcell; S.rw = D.rw;
    S.uptr = D.uptr; S.ucell = D.ucell; S.uq = D.uq; S.uw = D.uw;
    S.n = (int)n;
    S.ns = (int)T.src.cells.size();
    S.nr = s.n_rec;
    S.nu = (int)T.ucell.size();
    S.est = mode == WRI_ESTIMATE;
    S.max_iter = max_iter;
    S.c = (flags & WRI_FLAG_UNSCALED_ALPHA) ? 1.0 : std::sqrt(42.0) / (g.h * g.h);
    S.lam = s.lambda;
    S.rtol2 = s.rtol * s.rtol;
    S.omega = s.omega;
    S.omega2 = s.omega * s.omega;
    S.alpha = make_double2(s.alpha.re, s.alpha.im);
    S.m = m[s.grid];
    S.nx = g.nx; S.ny = g.ny; S.nz = g.nz; S.nb = g.nb;
    S.zc = (int)std::max<int64_t>(1, std::min<int64_t>(kZc, n / ((int64_t)kParts * kThreads)));  // >= kParts items
    S.h2inv = 1.0 / (g.h * g.h);
    if (g.nb > 0) {
      const double d0 = 3.0 * g.v_ref * std::log(1000.0) / (2.0 * g.nb * g.h);
      S.sp_scale = 2.0 * d0 / (g.v_ref * g.v_ref);
      S.inv_nb = 1.0 / g.nb;
    }
    nmax = std::max<int64_t>(nmax, n);
    rmax = std::max(rmax, S.nr);
    umax = std::max(umax, S.nu);
  }
  OgSys* dsys = reinterpret_cast<OgSys*>(base + L.sys);
  OgState* dst = reinterpret_cast<OgState*>(base + L.state);
  double* parts = reinterpret_cast<double*>(base + L.parts);
  int* didx = reinterpret_cast<int*>(base + L.idx);
  OG_HIP(hipMemcpyAsync(dsys, hs.data(), sizeof(OgSys) * n_sys, hipMemcpyHostToDevice, st));
  // systems grouped by grid for the gradient pass
  std::vector<int> order(n_sys);
  for (int k = 0; k < n_sys; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return sys[a].grid < sys[b].grid; });
  OG_HIP(hipMemcpyAsync(didx, order.data(), sizeof(int) * n_sys, hipMemcpyHostToDevice, st));
  OG_HIP(hipStreamSynchronize(st));  // the host tables are read by the copies above

  const dim3 vgrid(nblk(nmax), n_sys), pgrid(kParts, n_sys);
  (void)rmax;
  (void)umax;
  // kCheck iterations of every system (finished systems skip inside the
  // kernels), enqueued on stream sq: four launches per iteration
  auto enqueue_chunk = [&](hipStream_t sq) -> int {
    for (int it = 0; it < kCheck; ++it) {
      hipLaunchKernelGGL(k_og_fwd, pgrid, dim3(kThreads), 0, sq, dsys, dst, parts);
      hipLaunchKernelGGL(k_og_alpha, dim3(n_sys), dim3(kThreads), 0, sq, dsys, dst, parts);
      hipLaunchKernelGGL(k_og_adj, pgrid, dim3(kThreads), 0, sq, dsys, dst, parts, 0);
      hipLaunchKernelGGL(k_og_beta, dim3(n_sys), dim3(kThreads), 0, sq, dsys, dst, parts);
      OG_HIP(hipGetLastError());
    }
    return WRI_OK;
  };
  // set-up: x = 0, r_0 = b, s_0 = S^H b, gamma0
  hipLaunchKernelGGL(k_og_zero, vgrid, dim3(kThreads), 0, st, dsys);
  hipLaunchKernelGGL(k_og_init, dim3(n_sys), dim3(kThreads), 0, st, dsys, dst);
  hipLaunchKernelGGL(k_og_adj, pgrid, dim3(kThreads), 0, st, dsys, dst, parts, 1);
  hipLaunchKernelGGL(k_og_start, dim3(n_sys), dim3(kThreads), 0, st, dsys, dst, parts);
  OG_HIP(hipGetLastError());
  std::vector<OgState> hst(n_sys);
  auto read = [&]() -> int {
    OG_HIP(hipMemcpyAsync(hst.data(), dst, sizeof(OgState) * n_sys, hipMemcpyDeviceToHost, st));
    OG_HIP(hipStreamSynchronize(st));
    return WRI_OK;
  };
  if ((rc = read()) != WRI_OK) return rc;
  // A chunk of kCheck iterations is captured once into a hipGraph (kernel
  // nodes only) and replayed on the caller's stream; the graph lives for this
  // call only (it holds this workspace's pointers).
  hipStream_t cs = nullptr;
  std::map<int, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
  auto release = [&]() {
    for (auto& kv : graphs) {
      (void)hipGraphExecDestroy(kv.second.second);
      (void)hipGraphDestroy(kv.second.first);
    }
    graphs.clear();
    if (cs != nullptr) (void)hipStreamDestroy(cs);
    cs = nullptr;
  };
  auto run_chunk = [&]() -> int {
    auto it = graphs.find(0);
    if (it == graphs.end()) {
      if (cs == nullptr) OG_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      OG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      const int e = enqueue_chunk(cs);
      hipGraph_t graph = nullptr;
      const hipError_t ec = hipStreamEndCapture(cs, &graph);
      if (e != WRI_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return e;
      }
      if (ec != hipSuccess) return report_error(WRI_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(ec));
      hipGraphExec_t exec = nullptr;
      const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      if (ei != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return report_error(WRI_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(ei));
      }
      it = graphs.emplace(0, std::make_pair(graph, exec)).first;
    }
    OG_HIP(hipGraphLaunch(it->second.second, st));
    return WRI_OK;
  };
  std::vector<int> active;
  for (int64_t done = 0;; done += kCheck) {
    active.clear();
    for (int k = 0; k < n_sys; ++k)
      if (hst[k].status == kActive) active.push_back(k);
    if (active.empty()) break;
    if (done > (int64_t)max_iter + kCheck) {
      release();
      return report_error(WRI_EHIP, "internal: systems active past max_iter");
    }
    rc = (flags & WRI_FLAG_NO_GRAPH) ? enqueue_chunk(st) : run_chunk();
    if (rc == WRI_OK) rc = read();
    if (rc != WRI_OK) {
      release();
      return rc;
    }
  }
  release();
  // objective, source weights, gradient
  hipLaunchKernelGGL(k_og_rnorm, pgrid, dim3(kThreads), 0, st, dsys, dst, parts);
  if (mode == WRI_ESTIMATE) hipLaunchKernelGGL(k_og_ax, vgrid, dim3(kThreads), 0, st, dsys);
  OG_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_og_final, dim3(n_sys), dim3(kThreads), 0, st, dsys, dst, parts);
  OG_HIP(hipGetLastError());
  if (grad != nullptr)
    for (int g = 0, p0 = 0; g < n_grids; ++g) {
      int cnt = 0;
      while (p0 + cnt < n_sys && sys[order[p0 + cnt]].grid == g) ++cnt;
      const int64_t n = ncell(grids[g]);
      hipLaunchKernelGGL(k_og_grad, dim3(nblk(n)), dim3(kThreads), 0, st, dsys, dst, didx + p0, cnt, (int)n,
                         grad[g]);
      OG_HIP(hipGetLastError());
      p0 += cnt;
    }
  if ((rc = read()) != WRI_OK) return rc;
  double Jtot = 0.0;
  int ret = WRI_OK;
  for (int k = 0; k < n_sys; ++k) {
    const OgState& T = hst[k];
    double ee = 0.0;
    for (double w : tabs[k].src.w) ee += w * w;
    wri_result& r = res[k];
    r.iters = T.iters;
    r.status = T.status;
    r.relres = T.gamma0 > 0.0 ? std::sqrt(std::max(T.gamma, 0.0) / T.gamma0) : 0.0;
    r.J = T.J;
    if (mode == WRI_ESTIMATE) {
      r.alpha = wri_c64{hs[k].c * T.xa.x, hs[k].c * T.xa.y};
      r.alpha_ls = ee > 0.0 ? wri_c64{T.eau.x / ee, T.eau.y / ee} : wri_c64{0.0, 0.0};
    } else {
      r.alpha = sys[k].alpha;
      r.alpha_ls = sys[k].alpha;
    }
    Jtot += T.J;
    if (T.status == kBreakdown) ret = WRI_EBREAKDOWN;
    else if (T.status == kMaxIter && ret == WRI_OK) ret = WRI_NOT_CONVERGED;
  }
  if (J_out) *J_out = Jtot;
  if (ret == WRI_EBREAKDOWN) report_error(WRI_EBREAKDOWN, "at least one system broke down");
  return ret;
}

}  // namespace
}  // namespace wri

using namespace wri;

extern "C" {

size_t wri_offgrid_workspace_bytes(const wri_grid* grids, int32_t n_grids, const wri_system* sys, int32_t n_sys,
                                   const wri_positions* pos) {
  try {
    if (validate_offgrid(grids, n_grids, sys, n_sys, pos, WRI_ESTIMATE, 0) != WRI_OK) return 0;
    std::vector<SysTables> tabs(n_sys);
    for (int k = 0; k < n_sys; ++k) tabs[k] = build_tables(grids[sys[k].grid], pos[k], sys[k].n_rec);
    OgLayout L;
    og_layout(grids, sys, n_sys, &tabs, &L);
    return L.total;
  } catch (const std::exception& e) {
    report_error(WRI_EINVAL, "exception: %s", e.what());
    return 0;
  }
}

int wri_objective_grad_offgrid(const wri_grid* grids, int32_t n_grids, const float* const* m, const wri_system* sys,
                               int32_t n_sys, const wri_positions* pos, int32_t mode, int32_t max_iter,
                               int32_t flags, double* J_out, float* const* grad, wri_c32* const* u_out,
                               wri_result* res, void* ws, size_t ws_bytes, void* stream) {
  try {
    return og_run(grids, n_grids, m, sys, n_sys, pos, mode, max_iter, flags, J_out, grad, u_out, res, ws, ws_bytes,
                  reinterpret_cast<hipStream_t>(stream));
  } catch (const std::exception& e) {
    return report_error(WRI_EINVAL, "exception: %s", e.what());
  }
}

}  // extern "C"
