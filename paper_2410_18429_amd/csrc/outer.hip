// Outer loop of the inversion (section "SF-AWRI with total variation
// regularization", eq. TVAWRI, Algorithm 2): the smoothed total-variation term
// and its gradient, limited-memory BFGS directions, and the adaptive-tolerance
// driver that calls the augmented solve (wri_objective_grad) for every
// objective evaluation.
//
// Every reduction runs with a fixed grid and sums its per-block float64
// partials in one fixed order, so results are deterministic.  The l-BFGS
// two-loop recursion keeps its coefficients in device memory: a chain of small
// launches on the caller's stream, no host round trip.
#include "../../include/wri.h"
#include "wri_impl.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

namespace wri {
namespace {

constexpr int kRedThreads = 256;
constexpr int kRedBlocks = 1024;  // partial sums per reduction (fixed: deterministic order)

#define OUTER_HIP(expr)                                                                 \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return report_error(WRI_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kRedThreads / 64; ++i) r += red[i];
  return r;  // valid in thread 0
}

__device__ __forceinline__ float block_max(float v, float* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  __syncthreads();
  float r = 0.f;
  if (threadIdx.x == 0)
    for (int i = 0; i < kRedThreads / 64; ++i) r = fmaxf(r, red[i]);
  return r;
}

// ---- total variation --------------------------------------------------------
// phi_c = sqrt(|D m|_c^2 + eps^2) with forward differences (zero in the last
// cell of each axis); q_a = (D_a m) / phi.  Partials of sum phi per block.
__global__ void __launch_bounds__(kRedThreads)
k_tv_q(int nx, int ny, int nz, double inv_h, double eps2, const float* __restrict__ m,
       double* __restrict__ qx, double* __restrict__ qy, double* __restrict__ qz, double* __restrict__ part) {
  __shared__ double red[kRedThreads / 64];
  const int64_t n = (int64_t)nx * ny * nz, plane = (int64_t)nx * ny;
  double acc = 0.0;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(c % nx), y = (int)((c / nx) % ny), z = (int)(c / plane);
    const double mc = m[c];
    const double dx = (x + 1 < nx) ? ((double)m[c + 1] - mc) * inv_h : 0.0;
    const double dy = (y + 1 < ny) ? ((double)m[c + nx] - mc) * inv_h : 0.0;
    const double dz = (z + 1 < nz) ? ((double)m[c + plane] - mc) * inv_h : 0.0;
    const double phi = sqrt(dx * dx + dy * dy + dz * dz + eps2);
    qx[c] = dx / phi;
    qy[c] = dy / phi;
    qz[c] = dz / phi;
    acc += phi;
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// grad_c += gamma / h * sum_a (q_a[c - e_a] - q_a[c])
__global__ void __launch_bounds__(kRedThreads)
k_tv_grad(int nx, int ny, int nz, double scale, const double* __restrict__ qx, const double* __restrict__ qy,
          const double* __restrict__ qz, float* __restrict__ grad) {
  const int64_t n = (int64_t)nx * ny * nz, plane = (int64_t)nx * ny;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(c % nx), y = (int)((c / nx) % ny), z = (int)(c / plane);
    double v = -(qx[c] + qy[c] + qz[c]);
    if (x > 0) v += qx[c - 1];
    if (y > 0) v += qy[c - nx];
    if (z > 0) v += qz[c - plane];
    grad[c] = (float)((double)grad[c] + scale * v);
  }
}

// ---- vector kernels of the l-BFGS recursion and the model update -------------
__global__ void __launch_bounds__(kRedThreads)
k_dot32(const float* __restrict__ a, const float* __restrict__ b, int64_t n, double* __restrict__ part) {
  __shared__ double red[kRedThreads / 64];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    acc += (double)a[i] * (double)b[i];
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Device scalars of the recursion (index into sc): rho[i], alpha[i] for the
// ring slots, then H0 and two temporaries.
enum CoefOp : int { kOpSum = 0, kOpRho = 1, kOpAlpha = 2, kOpBeta = 3, kOpRatio = 4 };

// One block: s = fixed-order sum of the partials; then
//   kOpSum:   sc[dst] = s
//   kOpRho:   sc[dst] = 1 / s
//   kOpAlpha: sc[dst] = sc[a] * s                  (alpha_i = rho_i s_i.q)
//   kOpBeta:  sc[dst] = sc[a] - sc[b] * s          (alpha_i - rho_i y_i.r)
//   kOpRatio: sc[dst] = sc[a] / s                  (H0 = s.y / y.y)
__global__ void __launch_bounds__(64) k_coef(const double* __restrict__ part, int nparts, double* __restrict__ sc,
                                             int op, int dst, int a, int b) {
  double v = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 64) v += part[i];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if (threadIdx.x == 0) {
    double r = v;
    if (op == kOpRho) r = 1.0 / v;
    else if (op == kOpAlpha) r = sc[a] * v;
    else if (op == kOpBeta) r = sc[a] - sc[b] * v;
    else if (op == kOpRatio) r = sc[a] / v;
    sc[dst] = r;
  }
}

// y = y + sign * sc[k] * x   (float64 arithmetic, one rounding; x, y distinct)
__global__ void k_axpy_sc(float* __restrict__ y, const float* __restrict__ x, int64_t n, double sign,
                          const double* __restrict__ sc, int k) {
  const double a = sign * sc[k];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)((double)y[i] + a * (double)x[i]);
}

// y = sc[k] * y
__global__ void k_scale_sc(float* __restrict__ y, int64_t n, const double* __restrict__ sc, int k) {
  const double a = sc[k];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)(a * (double)y[i]);
}

__global__ void k_copy32(float* __restrict__ d, const float* __restrict__ s, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    d[i] = s[i];
}

// d = a - b
__global__ void k_sub32(float* __restrict__ d, const float* __restrict__ a, const float* __restrict__ b, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    d[i] = (float)((double)a[i] - (double)b[i]);
}

__global__ void __launch_bounds__(kRedThreads) k_absmax32(const float* __restrict__ a, int64_t n, float* __restrict__ part) {
  __shared__ float red[kRedThreads / 64];
  float v = 0.f;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v = fmaxf(v, fabsf(a[i]));
  const float t = block_max(v, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__device__ __forceinline__ bool in_sponge(int64_t c, int nx, int ny, int nz, int nb) {
  if (nb <= 0) return false;
  const int x = (int)(c % nx), y = (int)((c / nx) % ny), z = (int)(c / ((int64_t)nx * ny));
  return x < nb || x > nx - 1 - nb || y < nb || y > ny - 1 - nb || z < nb || z > nz - 1 - nb;
}

__global__ void k_zero_sponge(float* __restrict__ v, int nx, int ny, int nz, int nb) {
  const int64_t n = (int64_t)nx * ny * nz;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (in_sponge(i, nx, ny, nz, nb)) v[i] = 0.f;
}

// out = clamp(m + scale * dir) (bounds <= 0 are off)
__global__ void k_update(float* __restrict__ out, const float* __restrict__ m, const float* __restrict__ dir, int64_t n,
                         double scale, double lo, double hi) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double v = (double)m[i] + scale * (double)dir[i];
    if (lo > 0.0) v = fmax(v, lo);
    if (hi > 0.0) v = fmin(v, hi);
    out[i] = (float)v;
  }
}

int grid_blocks(int64_t n) { return (int)std::min<int64_t>(kRedBlocks, std::max<int64_t>(1, (n + kRedThreads - 1) / kRedThreads)); }

// ---- host helpers ----------------------------------------------------------------
size_t al(size_t x) { return (x + 255) & ~size_t(255); }

struct TvWs { double *qx, *qy, *qz, *part, *sum; };
size_t tv_ws_bytes(int64_t n) { return 3 * al(sizeof(double) * n) + al(sizeof(double) * (kRedBlocks + 1)); }
TvWs tv_ws(char* ws, int64_t n) {
  TvWs w;
  w.qx = reinterpret_cast<double*>(ws);
  w.qy = reinterpret_cast<double*>(ws + al(sizeof(double) * n));
  w.qz = reinterpret_cast<double*>(ws + 2 * al(sizeof(double) * n));
  w.part = reinterpret_cast<double*>(ws + 3 * al(sizeof(double) * n));
  w.sum = w.part + kRedBlocks;
  return w;
}

// TV(m) (host value) and, if grad != null, grad += gamma * grad TV
int tv_run(const wri_grid& g, const float* m, double eps, double gamma, double* value, float* grad, char* ws,
           hipStream_t st) {
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  TvWs w = tv_ws(ws, n);
  const int nbk = kRedBlocks;
  hipLaunchKernelGGL(k_tv_q, dim3(nbk), dim3(kRedThreads), 0, st, g.nx, g.ny, g.nz, 1.0 / g.h, eps * eps, m, w.qx,
                     w.qy, w.qz, w.part);
  OUTER_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_coef, dim3(1), dim3(64), 0, st, w.part, nbk, w.sum, (int)kOpSum, 0, 0, 0);
  OUTER_HIP(hipGetLastError());
  if (grad != nullptr && gamma != 0.0) {
    hipLaunchKernelGGL(k_tv_grad, dim3(grid_blocks(n)), dim3(kRedThreads), 0, st, g.nx, g.ny, g.nz, gamma / g.h, w.qx,
                       w.qy, w.qz, grad);
    OUTER_HIP(hipGetLastError());
  }
  OUTER_HIP(hipMemcpyAsync(value, w.sum, sizeof(double), hipMemcpyDeviceToHost, st));
  OUTER_HIP(hipStreamSynchronize(st));
  return WRI_OK;
}

struct LbWs { double* part; double* sc; };
size_t lb_ws_bytes(int cap) { return al(sizeof(double) * kRedBlocks) + al(sizeof(double) * (2 * cap + 4)); }
LbWs lb_ws(char* ws) {
  LbWs w;
  w.part = reinterpret_cast<double*>(ws);
  w.sc = reinterpret_cast<double*>(ws + al(sizeof(double) * kRedBlocks));
  return w;
}

int dot_to(const float* a, const float* b, int64_t n, const LbWs& w, int op, int dst, int ia, int ib, hipStream_t st) {
  hipLaunchKernelGGL(k_dot32, dim3(kRedBlocks), dim3(kRedThreads), 0, st, a, b, n, w.part);
  OUTER_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_coef, dim3(1), dim3(64), 0, st, w.part, kRedBlocks, w.sc, op, dst, ia, ib);
  OUTER_HIP(hipGetLastError());
  return WRI_OK;
}

// dir = -H g, two-loop recursion over `count` ring slots ending at `newest`.
// h0 > 0: H0 = h0 I; otherwise H0 = s.y / y.y of the newest pair.
int lbfgs_run(int64_t n, const float* g, const float* S, const float* Y, int cap, int count, int newest, double h0,
              float* dir, char* ws, hipStream_t st) {
  LbWs w = lb_ws(ws);
  const int rho0 = 0, alp0 = cap, ih0 = 2 * cap, it0 = 2 * cap + 1, it1 = 2 * cap + 2;
  const int nbk = grid_blocks(n);
  auto slot = [&](int j) { return ((newest - (count - 1) + j) % cap + cap) % cap; };  // j = 0 oldest
  hipLaunchKernelGGL(k_copy32, dim3(nbk), dim3(kRedThreads), 0, st, dir, g, n);
  OUTER_HIP(hipGetLastError());
  int rc;
  for (int j = count - 1; j >= 0; --j) {
    const int i = slot(j);
    const float* s = S + (int64_t)i * n;
    const float* y = Y + (int64_t)i * n;
    if ((rc = dot_to(y, s, n, w, kOpRho, rho0 + i, 0, 0, st)) != WRI_OK) return rc;
    if ((rc = dot_to(s, dir, n, w, kOpAlpha, alp0 + i, rho0 + i, 0, st)) != WRI_OK) return rc;
    hipLaunchKernelGGL(k_axpy_sc, dim3(nbk), dim3(kRedThreads), 0, st, dir, y, n, -1.0, w.sc, alp0 + i);
    OUTER_HIP(hipGetLastError());
  }
  if (h0 > 0.0 || count == 0) {
    const double hh = h0;
    OUTER_HIP(hipMemcpyAsync(w.sc + ih0, &hh, sizeof(double), hipMemcpyHostToDevice, st));
  } else {
    const float* s = S + (int64_t)slot(count - 1) * n;
    const float* y = Y + (int64_t)slot(count - 1) * n;
    if ((rc = dot_to(s, y, n, w, kOpSum, it0, 0, 0, st)) != WRI_OK) return rc;
    if ((rc = dot_to(y, y, n, w, kOpRatio, ih0, it0, 0, st)) != WRI_OK) return rc;
  }
  // r = H0 q
  hipLaunchKernelGGL(k_scale_sc, dim3(nbk), dim3(kRedThreads), 0, st, dir, n, w.sc, ih0);
  OUTER_HIP(hipGetLastError());
  for (int j = 0; j < count; ++j) {
    const int i = slot(j);
    const float* s = S + (int64_t)i * n;
    const float* y = Y + (int64_t)i * n;
    if ((rc = dot_to(y, dir, n, w, kOpBeta, it1, alp0 + i, rho0 + i, st)) != WRI_OK) return rc;
    hipLaunchKernelGGL(k_axpy_sc, dim3(nbk), dim3(kRedThreads), 0, st, dir, s, n, 1.0, w.sc, it1);
    OUTER_HIP(hipGetLastError());
  }
  // dir = -r
  const double minus_one = -1.0;
  OUTER_HIP(hipMemcpyAsync(w.sc + it0, &minus_one, sizeof(double), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_scale_sc, dim3(nbk), dim3(kRedThreads), 0, st, dir, n, w.sc, it0);
  OUTER_HIP(hipGetLastError());
  return WRI_OK;
}

// ---- the adaptive-tolerance driver (Algorithm 2) ------------------------------------
struct AwriLayout {
  size_t solver = 0, off_vec = 0, off_tv = 0, off_lb = 0, off_red = 0, off_u = 0, total = 0;
};
AwriLayout awri_layout(int64_t n, size_t solver_bytes, int memory, int n_sys, bool warm) {
  AwriLayout L;
  L.solver = al(solver_bytes);
  L.off_vec = L.solver;
  const size_t vb = al(sizeof(float) * n);
  size_t off = L.off_vec + vb * (size_t)(5 + 2 * std::max(memory, 0));  // g, g_try, m_try, dir, tmp, S, Y
  L.off_tv = off;
  off += tv_ws_bytes(n);
  L.off_lb = off;
  off += lb_ws_bytes(std::max(memory, 1));
  L.off_red = off;
  off += al(sizeof(float) * kRedBlocks) + al(sizeof(double) * kRedBlocks);
  L.off_u = off;  // warm start: wavefields at the current model, then at the trial model
  if (warm) off += 2 * (size_t)std::max(n_sys, 0) * al(sizeof(float) * 2 * n);
  L.total = off + 256;
  return L;
}

int absmax_host(const float* a, int64_t n, float* part, hipStream_t st, double* out) {
  hipLaunchKernelGGL(k_absmax32, dim3(kRedBlocks), dim3(kRedThreads), 0, st, a, n, part);
  OUTER_HIP(hipGetLastError());
  std::vector<float> h(kRedBlocks);
  OUTER_HIP(hipMemcpyAsync(h.data(), part, sizeof(float) * kRedBlocks, hipMemcpyDeviceToHost, st));
  OUTER_HIP(hipStreamSynchronize(st));
  float v = 0.f;
  for (float x : h) v = std::max(v, x);
  *out = v;
  return WRI_OK;
}

int dot_host(const float* a, const float* b, int64_t n, double* part, hipStream_t st, double* out) {
  hipLaunchKernelGGL(k_dot32, dim3(kRedBlocks), dim3(kRedThreads), 0, st, a, b, n, part);
  OUTER_HIP(hipGetLastError());
  std::vector<double> h(kRedBlocks);
  OUTER_HIP(hipMemcpyAsync(h.data(), part, sizeof(double) * kRedBlocks, hipMemcpyDeviceToHost, st));
  OUTER_HIP(hipStreamSynchronize(st));
  double v = 0.0;
  for (double x : h) v += x;
  *out = v;
  return WRI_OK;
}

}  // namespace
}  // namespace wri

using namespace wri;

extern "C" {

size_t wri_tv_workspace_bytes(const wri_grid* grid) {
  if (grid == nullptr || grid->nx < 1 || grid->ny < 1 || grid->nz < 1) return 0;
  return tv_ws_bytes((int64_t)grid->nx * grid->ny * grid->nz) + 256;
}

int wri_tv(const wri_grid* grid, const float* m, double eps, double gamma, double* value, float* grad, void* ws,
           size_t ws_bytes, void* stream) {
  if (grid == nullptr || m == nullptr || value == nullptr) return report_error(WRI_EINVAL, "grid, m and value are required");
  if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1 || !(grid->h > 0.0)) return report_error(WRI_EINVAL, "invalid grid");
  if (!(eps >= 0.0) || !std::isfinite(gamma)) return report_error(WRI_EINVAL, "eps must be >= 0 and gamma finite");
  const size_t need = wri_tv_workspace_bytes(grid);
  if (ws == nullptr || ws_bytes < need) return report_error(WRI_ENOWS, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
  char* w = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
  return tv_run(*grid, m, eps, gamma, value, grad, w, reinterpret_cast<hipStream_t>(stream));
}

size_t wri_lbfgs_workspace_bytes(int32_t capacity) {
  if (capacity < 0) return 0;
  return lb_ws_bytes(std::max(capacity, 1)) + 256;
}

int wri_lbfgs_direction(int64_t n, const float* g, const float* S, const float* Y, int32_t capacity, int32_t count,
                        int32_t newest, double h0, float* dir, void* ws, size_t ws_bytes, void* stream) {
  if (n < 1 || g == nullptr || dir == nullptr) return report_error(WRI_EINVAL, "n >= 1, g and dir are required");
  if (capacity < 0 || count < 0 || count > capacity || (count > 0 && (S == nullptr || Y == nullptr)) ||
      (count > 0 && (newest < 0 || newest >= capacity)))
    return report_error(WRI_EINVAL, "invalid pair ring (capacity %d, count %d, newest %d)", capacity, count, newest);
  if (count == 0 && !(h0 > 0.0)) return report_error(WRI_EINVAL, "h0 must be > 0 without curvature pairs");
  if (!std::isfinite(h0)) return report_error(WRI_EINVAL, "h0 is not finite");
  const size_t need = wri_lbfgs_workspace_bytes(capacity);
  if (ws == nullptr || ws_bytes < need) return report_error(WRI_ENOWS, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
  char* w = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
  return lbfgs_run(n, g, S, Y, std::max(capacity, 1), count, newest, h0, dir, w, reinterpret_cast<hipStream_t>(stream));
}

size_t wri_awri_workspace_bytes(const wri_grid* grid, const wri_system* sys, int32_t n_sys, int32_t mode,
                                int32_t flags, int32_t memory) {
  if (grid == nullptr || memory < 0) return 0;
  const size_t sb = wri_workspace_bytes(grid, 1, sys, n_sys, mode, flags);
  if (sb == 0) return 0;
  return awri_layout((int64_t)grid->nx * grid->ny * grid->nz, sb, memory, n_sys,
                     (flags & WRI_FLAG_WARM_START) != 0).total;
}

int wri_awri(const wri_grid* grid, float* m, const wri_system* sys, int32_t n_sys, int32_t mode,
             const wri_awri_options* opt, wri_awri_record* history, int32_t history_cap, int32_t* n_records,
             void* ws, size_t ws_bytes, void* stream) {
  if (grid == nullptr || m == nullptr || opt == nullptr || n_records == nullptr)
    return report_error(WRI_EINVAL, "grid, m, opt and n_records are required");
  *n_records = 0;
  const wri_awri_options o = *opt;
  if (!(o.eps0 > 0.0) || !(o.eps_min > 0.0) || o.eps_min > o.eps0 || o.max_outer < 0 || o.memory < 0 ||
      !(o.gamma >= 0.0) || !(o.eps_tv >= 0.0) || !(o.step0 > 0.0) || !(o.max_step >= 0.0) || o.max_iter < 0 ||
      (o.m_min > 0.0 && o.m_max > 0.0 && o.m_min > o.m_max))
    return report_error(WRI_EINVAL, "invalid options");
  if (history_cap > 0 && history == nullptr) return report_error(WRI_EINVAL, "history is NULL");
  const size_t sb = wri_workspace_bytes(grid, 1, sys, n_sys, mode, o.flags);
  if (sb == 0) return report_error(WRI_EINVAL, "invalid grid or systems: %s", wri_last_error());
  const int64_t n = (int64_t)grid->nx * grid->ny * grid->nz;
  const bool warm = o.warm_start != 0;
  const AwriLayout L = awri_layout(n, sb, o.memory, n_sys, warm);
  if (ws == nullptr || ws_bytes < L.total)
    return report_error(WRI_ENOWS, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, L.total);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
  char* solver_ws = base;
  const size_t vb = al(sizeof(float) * n);
  float* g = reinterpret_cast<float*>(base + L.off_vec);
  float* g_try = reinterpret_cast<float*>(base + L.off_vec + vb);
  float* m_try = reinterpret_cast<float*>(base + L.off_vec + 2 * vb);
  float* dir = reinterpret_cast<float*>(base + L.off_vec + 3 * vb);
  float* tmp = reinterpret_cast<float*>(base + L.off_vec + 4 * vb);
  float* Sring = reinterpret_cast<float*>(base + L.off_vec + 5 * vb);
  float* Yring = Sring + (size_t)o.memory * (vb / sizeof(float));
  char* tvw = base + L.off_tv;
  char* lbw = base + L.off_lb;
  float* fpart = reinterpret_cast<float*>(base + L.off_red);
  double* dpart = reinterpret_cast<double*>(base + L.off_red + al(sizeof(float) * kRedBlocks));
  const int nbk = grid_blocks(n);
  const int nbs = (o.mask_sponge && grid->nb > 0) ? grid->nb : 0;

  std::vector<wri_system> se(sys, sys + n_sys);
  std::vector<wri_result> res(std::max(n_sys, 1));
  // warm start: wavefields (and source weights) of the current model and of the trial
  const size_t ub = al(sizeof(float) * 2 * n);
  std::vector<wri_c32*> ucur(n_sys), utry(n_sys);
  for (int i = 0; i < n_sys; ++i) {
    ucur[i] = reinterpret_cast<wri_c32*>(base + L.off_u + (size_t)i * ub);
    utry[i] = reinterpret_cast<wri_c32*>(base + L.off_u + (size_t)(n_sys + i) * ub);
  }
  std::vector<wri_c64> acur(n_sys), atry(n_sys);
  bool have_cur = false;
  int recs = 0;
  auto record = [&](double F, double J, double T, double eps, int kind, int iters, double secs) {
    if (recs < history_cap) history[recs] = wri_awri_record{F, J, T, eps, kind, iters, secs};
    ++recs;
  };
  // F = J + gamma TV and its gradient (masked in the sponge) at model mm, tolerance eps.
  // Warm start: the solves start from the current model's wavefields `from`
  // (copied into `into` unless they are the same set) and source weights.
  auto evaluate_w = [&](const float* mm, double eps, float* grad, double* F, double* J, double* T, int* iters,
                        double* secs, std::vector<wri_c32*>* into, std::vector<wri_c32*>* from,
                        std::vector<wri_c64>* alphas_out) -> int {
    const auto t0 = std::chrono::steady_clock::now();
    int fl = o.flags & ~WRI_FLAG_WARM_START;  // the driver decides per solve
    for (int i = 0; i < n_sys; ++i) {
      se[i].rtol = eps;
      if (warm && have_cur && mode == WRI_ESTIMATE) se[i].alpha = acur[i];
    }
    if (warm && have_cur) {
      fl |= WRI_FLAG_WARM_START;
      if (from != into)
        for (int i = 0; i < n_sys; ++i)
          OUTER_HIP(hipMemcpyAsync((*into)[i], (*from)[i], sizeof(float) * 2 * n, hipMemcpyDeviceToDevice, st));
    }
    const float* mp[1] = {mm};
    float* gp[1] = {grad};
    int rc = wri_objective_grad(grid, 1, mp, se.data(), n_sys, mode, o.max_iter, fl, J, gp,
                                warm ? into->data() : nullptr, res.data(), solver_ws, sb, stream);
    if (rc < 0) return rc;
    if (warm)
      for (int i = 0; i < n_sys; ++i) (*alphas_out)[i] = res[i].alpha;
    int it = 0;
    for (int i = 0; i < n_sys; ++i) it += res[i].iters;
    *iters = it;
    rc = tv_run(*grid, mm, o.eps_tv, o.gamma, T, grad, tvw, st);
    if (rc != WRI_OK) return rc;
    if (nbs > 0) {
      hipLaunchKernelGGL(k_zero_sponge, dim3(nbk), dim3(kRedThreads), 0, st, grad, grid->nx, grid->ny, grid->nz, nbs);
      OUTER_HIP(hipGetLastError());
    }
    OUTER_HIP(hipStreamSynchronize(st));
    *F = *J + o.gamma * *T;
    *secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return WRI_OK;
  };

  // the current model (start, or again after eps was halved): warm from its own wavefields
  auto evaluate = [&](const float* mm, double eps, float* grad, double* F, double* J, double* T, int* iters,
                      double* secs) -> int {
    const int r = evaluate_w(mm, eps, grad, F, J, T, iters, secs, &ucur, &ucur, &acur);
    if (r == WRI_OK) have_cur = true;
    return r;
  };
  double eps = o.eps0, F = 0, J = 0, T = 0, secs = 0;
  int iters = 0, rc;
  if ((rc = evaluate(m, eps, g, &F, &J, &T, &iters, &secs)) != WRI_OK) return rc;
  record(F, J, T, eps, WRI_AWRI_EVAL, iters, secs);
  int count = 0, newest = -1, accepted = 0;
  double last_sy = 0.0, last_yy = 0.0;
  int status = WRI_OK;
  while (accepted < o.max_outer) {
    double h0;
    if (count > 0) {
      h0 = last_sy / last_yy;
    } else {
      double mmax = 0.0, gmax = 0.0;
      if ((rc = absmax_host(m, n, fpart, st, &mmax)) != WRI_OK) return rc;
      if ((rc = absmax_host(g, n, fpart, st, &gmax)) != WRI_OK) return rc;
      if (!(gmax > 0.0)) break;  // stationary
      h0 = o.step0 * mmax / gmax;
    }
    if ((rc = lbfgs_run(n, g, Sring, Yring, std::max(o.memory, 1), count, std::max(newest, 0), h0, dir, lbw, st)) !=
        WRI_OK)
      return rc;
    double scale = 1.0;
    if (o.max_step > 0.0) {
      double mmax = 0.0, dmax = 0.0;
      if ((rc = absmax_host(m, n, fpart, st, &mmax)) != WRI_OK) return rc;
      if ((rc = absmax_host(dir, n, fpart, st, &dmax)) != WRI_OK) return rc;
      if (dmax > o.max_step * mmax) scale = o.max_step * mmax / dmax;
    }
    hipLaunchKernelGGL(k_update, dim3(nbk), dim3(kRedThreads), 0, st, m_try, m, dir, n, scale, o.m_min, o.m_max);
    OUTER_HIP(hipGetLastError());
    double F1 = 0, J1 = 0, T1 = 0;
    if ((rc = evaluate_w(m_try, eps, g_try, &F1, &J1, &T1, &iters, &secs, &utry, &ucur, &atry)) != WRI_OK)
      return rc;
    const bool ok = F1 <= F;
    record(F1, J1, T1, eps, ok ? WRI_AWRI_ACCEPTED : WRI_AWRI_REJECTED, iters, secs);
    if (!ok) {
      if (0.5 * eps < o.eps_min) { status = WRI_NOT_CONVERGED; break; }
      eps *= 0.5;
      // pairs formed at the looser tolerance are dropped: the next trial is a
      // scaled gradient step (without a line search a stale pair repeats the
      // rejected step)
      count = 0;
      newest = -1;
      if ((rc = evaluate(m, eps, g, &F, &J, &T, &iters, &secs)) != WRI_OK) return rc;
      record(F, J, T, eps, WRI_AWRI_EVAL, iters, secs);
      continue;
    }
    // curvature pair (s, y) = (m_try - m, g_try - g): kept (in the next ring
    // slot, replacing the oldest pair once the ring is full) only if s.y > 0
    if (o.memory > 0) {
      float* s = tmp;
      float* y = dir;  // the direction is no longer needed
      hipLaunchKernelGGL(k_sub32, dim3(nbk), dim3(kRedThreads), 0, st, s, m_try, m, n);
      hipLaunchKernelGGL(k_sub32, dim3(nbk), dim3(kRedThreads), 0, st, y, g_try, g, n);
      OUTER_HIP(hipGetLastError());
      double sy = 0.0, yy = 0.0;
      if ((rc = dot_host(s, y, n, dpart, st, &sy)) != WRI_OK) return rc;
      if ((rc = dot_host(y, y, n, dpart, st, &yy)) != WRI_OK) return rc;
      if (sy > 0.0 && yy > 0.0) {
        const int slot = (newest + 1) % o.memory;
        hipLaunchKernelGGL(k_copy32, dim3(nbk), dim3(kRedThreads), 0, st, Sring + (size_t)slot * (vb / sizeof(float)), s, n);
        hipLaunchKernelGGL(k_copy32, dim3(nbk), dim3(kRedThreads), 0, st, Yring + (size_t)slot * (vb / sizeof(float)), y, n);
        OUTER_HIP(hipGetLastError());
        newest = slot;
        count = std::min(count + 1, o.memory);
        last_sy = sy;
        last_yy = yy;
      }
    }
    hipLaunchKernelGGL(k_copy32, dim3(nbk), dim3(kRedThreads), 0, st, m, m_try, n);
    OUTER_HIP(hipGetLastError());
    std::swap(g, g_try);
    if (warm) {
      std::swap(ucur, utry);
      std::swap(acur, atry);
    }
    F = F1; J = J1; T = T1;
    ++accepted;
  }
  OUTER_HIP(hipStreamSynchronize(st));
  *n_records = recs;
  if (status != WRI_OK) report_error(status, "the objective did not decrease at the smallest tolerance %.3g", o.eps_min);
  return status;
}

}  // extern "C"
