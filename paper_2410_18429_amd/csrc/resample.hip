// One model grid tied to per-frequency simulation grids: trilinear resampling
// of the squared slowness from the model grid onto each simulation grid, the
// adjoint (transpose) of that map for gradients, and an objective-and-gradient
// entry point whose model lives on the model grid.  Each frequency is then
// simulated at its own cell size (a fixed number of points per wavelength)
// while the inversion updates one model.
//
// Geometry: every grid has its cell (i, j, k) at (i h, j h, k h) — a common
// origin at cell 0.  A simulation cell samples the model grid at
// xi = clamp(i h / h_m, 0, n_m - 1) per axis, i0 = min(floor(xi), n_m - 2),
// t = xi - i0, weights (1 - t, t) on (i0, i0 + 1) (one model cell: i0 = 0,
// weight 1).  The 3-D weight is the product of the three axes.
//
// The adjoint runs as a gather over model cells (no atomics, fixed order):
// for each axis, the simulation cells whose i0 is a - 1 or a are listed with
// their weights, recomputed by the same function as the forward map.
#include "../../include/wri.h"
#include "wri_impl.hpp"

#include <algorithm>
#include <cmath>
#include <vector>

namespace wri {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxAxisList = 16;  // simulation cells per axis that can touch one model cell
constexpr size_t kAl = 256;
size_t al(size_t v) { return (v + kAl - 1) / kAl * kAl; }

#define RS_HIP(expr)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return report_error(WRI_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

struct Axis {
  int n_m, n_g;
  double ratio;  // h_g / h_m
};

// model-grid interval and weight of simulation index i along one axis
__host__ __device__ inline void axis_weight(const Axis& a, int i, int* i0, double* t) {
  if (a.n_m == 1) {
    *i0 = 0;
    *t = 0.0;
    return;
  }
  double xi = (double)i * a.ratio;
  xi = xi < 0.0 ? 0.0 : (xi > (double)(a.n_m - 1) ? (double)(a.n_m - 1) : xi);
  int k = (int)floor(xi);
  if (k > a.n_m - 2) k = a.n_m - 2;
  *i0 = k;
  *t = xi - (double)k;
}

// simulation indices i (with weight) whose interpolation touches model index m
__device__ inline int axis_list(const Axis& a, int m, int* idx, double* w) {
  int lo, hi;
  if (a.n_m == 1) {  // then n_g == 1 (the model grid covers the simulation grid)
    lo = 0;
    hi = a.n_g - 1;
  } else {  // xi = i * ratio in [m - 1, m + 1], one index of margin for rounding
    lo = (int)floor((double)(m - 1) / a.ratio) - 1;
    hi = (int)ceil((double)(m + 1) / a.ratio) + 1;
    lo = lo < 0 ? 0 : lo;
    hi = hi > a.n_g - 1 ? a.n_g - 1 : hi;
  }
  int cnt = 0;
  for (int i = lo; i <= hi && cnt < kMaxAxisList; ++i) {
    int i0;
    double t;
    axis_weight(a, i, &i0, &t);
    double wt = 0.0;
    if (a.n_m == 1) wt = 1.0;
    else if (i0 == m) wt = 1.0 - t;
    else if (i0 + 1 == m) wt = t;
    if (wt != 0.0) {
      idx[cnt] = i;
      w[cnt] = wt;
      ++cnt;
    }
  }
  return cnt;
}

__global__ void __launch_bounds__(kThreads) k_model_to_grid(Axis ax, Axis ay, Axis az, const float* __restrict__ mm,
                                                            float* __restrict__ mg) {
  const int64_t n = (int64_t)ax.n_g * ay.n_g * az.n_g;
  const int64_t pm = (int64_t)ax.n_m * ay.n_m;
  for (int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x; c < n; c += (int64_t)gridDim.x * kThreads) {
    const int i = (int)(c % ax.n_g), j = (int)((c / ax.n_g) % ay.n_g), k = (int)(c / ((int64_t)ax.n_g * ay.n_g));
    int x0, y0, z0;
    double tx, ty, tz;
    axis_weight(ax, i, &x0, &tx);
    axis_weight(ay, j, &y0, &ty);
    axis_weight(az, k, &z0, &tz);
    const int x1 = ax.n_m > 1 ? x0 + 1 : x0, y1 = ay.n_m > 1 ? y0 + 1 : y0, z1 = az.n_m > 1 ? z0 + 1 : z0;
    auto at = [&](int x, int y, int z) { return (double)mm[(int64_t)z * pm + (int64_t)y * ax.n_m + x]; };
    const double v = (1.0 - tz) * ((1.0 - ty) * ((1.0 - tx) * at(x0, y0, z0) + tx * at(x1, y0, z0)) +
                                   ty * ((1.0 - tx) * at(x0, y1, z0) + tx * at(x1, y1, z0))) +
                     tz * ((1.0 - ty) * ((1.0 - tx) * at(x0, y0, z1) + tx * at(x1, y0, z1)) +
                           ty * ((1.0 - tx) * at(x0, y1, z1) + tx * at(x1, y1, z1)));
    mg[c] = (float)v;
  }
}

// g_model[M] (+)= sum over simulation cells c of weight(c, M) * g_grid[c].
// One block per model row (b, d): the y and z lists are the same for the whole
// row and live in LDS; each thread builds the x list of its own model cells.
// Reads of g_grid along a list are contiguous across neighbouring threads.
__global__ void __launch_bounds__(kThreads) k_grid_to_model(Axis ax, Axis ay, Axis az, const float* __restrict__ gg,
                                                            float* __restrict__ gm, int accumulate) {
  __shared__ int sy[kMaxAxisList], sz[kMaxAxisList], cnt[2];
  __shared__ double swy[kMaxAxisList], swz[kMaxAxisList];
  const int64_t pg = (int64_t)ax.n_g * ay.n_g;
  const int64_t rows = (int64_t)ay.n_m * az.n_m;
  for (int64_t rw = blockIdx.x; rw < rows; rw += gridDim.x) {
  const int b = (int)(rw % ay.n_m), d = (int)(rw / ay.n_m);
  __syncthreads();  // the previous row's lists are no longer read
  if (threadIdx.x == 0) cnt[0] = axis_list(ay, b, sy, swy);
  if (threadIdx.x == 64) cnt[1] = axis_list(az, d, sz, swz);
  __syncthreads();
  const int ny = cnt[0], nz = cnt[1];
  const int64_t row_m = rw * ax.n_m;
  for (int a = threadIdx.x; a < ax.n_m; a += kThreads) {
    int ix[kMaxAxisList];
    double wx[kMaxAxisList];
    const int nx = axis_list(ax, a, ix, wx);
    double acc = 0.0;
    for (int r = 0; r < nz; ++r)
      for (int q = 0; q < ny; ++q) {
        const int64_t row = (int64_t)sz[r] * pg + (int64_t)sy[q] * ax.n_g;
        double s = 0.0;
        for (int p = 0; p < nx; ++p) s += wx[p] * (double)gg[row + ix[p]];
        acc += swz[r] * swy[q] * s;
      }
    const int64_t c = row_m + a;
    gm[c] = accumulate ? (float)((double)gm[c] + acc) : (float)acc;
  }
  }
}

int blocks_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + kThreads - 1) / kThreads, 8192)); }

int check_pair(const wri_grid* model, const wri_grid* grid) {
  if (model == nullptr || grid == nullptr) return report_error(WRI_EINVAL, "grid is NULL");
  for (const wri_grid* g : {model, grid}) {
    if (g->nx < 1 || g->ny < 1 || g->nz < 1) return report_error(WRI_EINVAL, "non-positive grid size");
    if ((int64_t)g->nx * g->ny * g->nz >= (int64_t(1) << 31)) return report_error(WRI_EINVAL, "grid too large");
    if (!(g->h > 0.0) || !std::isfinite(g->h)) return report_error(WRI_EINVAL, "h must be > 0");
  }
  // a model cell is touched by at most 2 h_m / h_g + 1 simulation cells per axis
  // (searched with one index of margin on each side)
  if (2.0 * model->h / grid->h + 3.0 > (double)kMaxAxisList)
    return report_error(WRI_EINVAL, "simulation grid finer than the model grid by more than %.1f x",
                        (kMaxAxisList - 3) / 2.0);
  // the model grid must cover the simulation grid: (n_g - 1) h_g <= (n_m - 1) h_m
  const int ng[3] = {grid->nx, grid->ny, grid->nz}, nm[3] = {model->nx, model->ny, model->nz};
  for (int a = 0; a < 3; ++a)
    if ((double)(ng[a] - 1) * grid->h > (double)(nm[a] - 1) * model->h * (1.0 + 1e-12))
      return report_error(WRI_EINVAL, "simulation grid extends beyond the model grid along axis %d", a);
  return WRI_OK;
}

void axes(const wri_grid* model, const wri_grid* grid, Axis* ax, Axis* ay, Axis* az) {
  const double r = grid->h / model->h;
  *ax = Axis{model->nx, grid->nx, r};
  *ay = Axis{model->ny, grid->ny, r};
  *az = Axis{model->nz, grid->nz, r};
}

int model_to_grid(const wri_grid* model, const float* mm, const wri_grid* grid, float* mg, hipStream_t st) {
  int rc = check_pair(model, grid);
  if (rc != WRI_OK) return rc;
  if (mm == nullptr || mg == nullptr) return report_error(WRI_EINVAL, "model or output is NULL");
  Axis ax, ay, az;
  axes(model, grid, &ax, &ay, &az);
  hipLaunchKernelGGL(k_model_to_grid, dim3(blocks_for((int64_t)grid->nx * grid->ny * grid->nz)), dim3(kThreads), 0,
                     st, ax, ay, az, mm, mg);
  RS_HIP(hipGetLastError());
  return WRI_OK;
}

int grid_to_model(const wri_grid* model, const wri_grid* grid, const float* gg, float* gm, int accumulate,
                  hipStream_t st) {
  int rc = check_pair(model, grid);
  if (rc != WRI_OK) return rc;
  if (gg == nullptr || gm == nullptr) return report_error(WRI_EINVAL, "gradient pointer is NULL");
  Axis ax, ay, az;
  axes(model, grid, &ax, &ay, &az);
  const int64_t rows = (int64_t)model->ny * model->nz;
  hipLaunchKernelGGL(k_grid_to_model, dim3((unsigned)std::min<int64_t>(rows, 1 << 20)), dim3(kThreads), 0, st, ax, ay,
                     az, gg, gm, accumulate);
  RS_HIP(hipGetLastError());
  return WRI_OK;
}

struct ModelLayout {
  size_t solver = 0, solver_bytes = 0, total = 0;
  std::vector<size_t> m, g;
};

int model_layout(const wri_grid* model, const wri_grid* grids, int n_grids, const wri_system* sys, int n_sys,
                 int mode, int flags, ModelLayout* L) {
  for (int gi = 0; gi < n_grids; ++gi) {
    int rc = check_pair(model, grids + gi);
    if (rc != WRI_OK) return rc;
  }
  const size_t sb = wri_workspace_bytes(grids, n_grids, sys, n_sys, mode, flags);
  if (sb == 0) return WRI_EINVAL;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = al(o + std::max<size_t>(bytes, 1)); return r; };
  L->solver_bytes = sb;
  L->solver = take(sb);
  L->m.resize(n_grids);
  L->g.resize(n_grids);
  for (int gi = 0; gi < n_grids; ++gi) {
    const size_t nb = sizeof(float) * (size_t)grids[gi].nx * grids[gi].ny * grids[gi].nz;
    L->m[gi] = take(nb);
    L->g[gi] = take(nb);
  }
  L->total = o + kAl;
  return WRI_OK;
}

}  // namespace
}  // namespace wri

using namespace wri;

extern "C" {

int wri_model_to_grid(const wri_grid* model_grid, const float* m_model, const wri_grid* grid, float* m_grid,
                      void* stream) {
  try {
    return model_to_grid(model_grid, m_model, grid, m_grid, reinterpret_cast<hipStream_t>(stream));
  } catch (const std::exception& e) {
    return report_error(WRI_EINVAL, "exception: %s", e.what());
  }
}

int wri_grid_to_model_adjoint(const wri_grid* model_grid, const wri_grid* grid, const float* g_grid, float* g_model,
                              int32_t accumulate, void* stream) {
  try {
    return grid_to_model(model_grid, grid, g_grid, g_model, accumulate, reinterpret_cast<hipStream_t>(stream));
  } catch (const std::exception& e) {
    return report_error(WRI_EINVAL, "exception: %s", e.what());
  }
}

size_t wri_model_workspace_bytes(const wri_grid* model_grid, const wri_grid* grids, int32_t n_grids,
                                 const wri_system* sys, int32_t n_sys, int32_t mode, int32_t flags) {
  try {
    if (n_grids < 0 || (n_grids > 0 && grids == nullptr)) {
      report_error(WRI_EINVAL, "bad grids");
      return 0;
    }
    ModelLayout L;
    if (model_layout(model_grid, grids, n_grids, sys, n_sys, mode, flags, &L) != WRI_OK) return 0;
    return L.total;
  } catch (const std::exception& e) {
    report_error(WRI_EINVAL, "exception: %s", e.what());
    return 0;
  }
}

int wri_objective_grad_model(const wri_grid* model_grid, const float* m_model, const wri_grid* grids,
                             int32_t n_grids, const wri_system* sys, int32_t n_sys, int32_t mode, int32_t max_iter,
                             int32_t flags, double* J_out, float* grad_model, wri_c32* const* u_out, wri_result* res,
                             void* ws, size_t ws_bytes, void* stream) {
  try {
    if (J_out == nullptr) return report_error(WRI_EINVAL, "J_out is NULL");
    if (m_model == nullptr) return report_error(WRI_EINVAL, "m_model is NULL");
    if (n_grids < 1 || grids == nullptr) return report_error(WRI_EINVAL, "need at least one simulation grid");
    int rc = wri_validate(grids, n_grids, sys, n_sys, mode, max_iter);
    if (rc != WRI_OK) return rc;
    ModelLayout L;
    rc = model_layout(model_grid, grids, n_grids, sys, n_sys, mode, flags, &L);
    if (rc != WRI_OK) return rc;
    if (ws == nullptr || ws_bytes < L.total)
      return report_error(WRI_ENOWS, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, L.total);
    char* base = reinterpret_cast<char*>(al(reinterpret_cast<uintptr_t>(ws)));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    std::vector<const float*> mp(n_grids);
    std::vector<float*> gp(n_grids);
    for (int gi = 0; gi < n_grids; ++gi) {
      float* mg = reinterpret_cast<float*>(base + L.m[gi]);
      rc = model_to_grid(model_grid, m_model, grids + gi, mg, st);
      if (rc != WRI_OK) return rc;
      mp[gi] = mg;
      gp[gi] = reinterpret_cast<float*>(base + L.g[gi]);
    }
    const int rs = wri_objective_grad(grids, n_grids, mp.data(), sys, n_sys, mode, max_iter, flags, J_out,
                                      gp.data(), u_out, res, base + L.solver, L.solver_bytes, stream);
    if (rs < 0) return rs;
    if (grad_model != nullptr) {
      for (int gi = 0; gi < n_grids; ++gi) {
        rc = grid_to_model(model_grid, grids + gi, gp[gi], grad_model, gi > 0 ? 1 : 0, st);
        if (rc != WRI_OK) return rc;
      }
    }
    RS_HIP(hipStreamSynchronize(st));
    return rs;
  } catch (const std::exception& e) {
    return report_error(WRI_EINVAL, "exception: %s", e.what());
  }
}

}  // extern "C"
