// Reduced (conventional) FWI, the objective that WRI relaxes (eqs. FWI,
// PDEsolve, FWI2): forward and adjoint Helmholtz solves by the batched solver
// with lambda = 0, the misfit-minimising source weight, the data residual and
// the adjoint-state gradient.
//
// Per system the forward solve gives w = A^{-1} e (ESTIMATE; KNOWN solves
// A u = alpha e directly).  One block per system then forms, in float64, the
// weight alpha = (P w)^H d / ||P w||^2, the residual rho = alpha P w - d, its
// share of f = 1/2 ||rho||^2 and the adjoint source conj(rho).  The adjoint
// solve (receiver sources, WRI_FLAG_ADJOINT_SOURCE) gives z = A^{-1} P^H conj(rho),
// so v = conj(z) solves A^H v = P^H rho, and one pass per grid writes
// df/dm = -sum omega^2 Re(z * alpha w).  Reductions run in one fixed order.
#include "../../include/wri.h"
#include "wri_impl.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace wri {
namespace {

constexpr int kThreads = 256;
constexpr size_t kAl = 256;
size_t al(size_t v) { return (v + kAl - 1) / kAl * kAl; }

#define FWI_HIP(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return report_error(WRI_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// One system's pointers and scalars, resident in the workspace.
struct FwiSys {
  const float2* w;    // forward solution (A^{-1} e, or A^{-1} alpha e in KNOWN mode)
  const float2* z;    // adjoint solution A^{-1} P^H conj(rho)
  const float2* d;    // observed data, n_rec
  const int* rec;     // receiver cells, n_rec (device copy)
  float2* adj;        // adjoint source values conj(rho), n_rec
  float2* u;          // optional output u = mult * w (null: not requested)
  double omega2;
  double2 mult;       // written by k_fwi_residual: u = mult * w
  double f;           // written by k_fwi_residual: 1/2 ||rho||^2
  int n_rec, estimate, n, pad_;
};

// Sum over a 256-thread block, returned to every thread (fixed order).
__device__ __forceinline__ double block_sum_all(double v, double* red) {
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

// grid = n_sys blocks of 256 threads.
__global__ void __launch_bounds__(kThreads) k_fwi_residual(FwiSys* __restrict__ tab) {
  __shared__ double red[kThreads / 64];
  FwiSys& S = tab[blockIdx.x];
  const int nr = S.n_rec;
  double cr = 0.0, ci = 0.0, den = 0.0;
  for (int q = threadIdx.x; q < nr; q += kThreads) {
    const float2 pw = S.w[S.rec[q]], dq = S.d[q];
    const double wr = pw.x, wi = pw.y, dr = dq.x, di = dq.y;
    cr += wr * dr + wi * di;  // conj(P w) * d
    ci += wr * di - wi * dr;
    den += wr * wr + wi * wi;
  }
  cr = block_sum_all(cr, red);
  ci = block_sum_all(ci, red);
  den = block_sum_all(den, red);
  double ar = 1.0, ai = 0.0;
  if (S.estimate) {
    ar = den > 0.0 ? cr / den : 0.0;
    ai = den > 0.0 ? ci / den : 0.0;
  }
  double f = 0.0;
  for (int q = threadIdx.x; q < nr; q += kThreads) {
    const float2 pw = S.w[S.rec[q]], dq = S.d[q];
    const double rr = ar * pw.x - ai * pw.y - dq.x;
    const double ri = ar * pw.y + ai * pw.x - dq.y;
    f += rr * rr + ri * ri;
    S.adj[q] = make_float2((float)rr, (float)-ri);
  }
  f = block_sum_all(f, red);
  if (threadIdx.x == 0) {
    S.mult = make_double2(ar, ai);
    S.f = 0.5 * f;
  }
}

// df/dm on one grid: systems [s0, s0 + ns) of the table (all on this grid).
__global__ void __launch_bounds__(kThreads) k_fwi_grad(const FwiSys* __restrict__ tab, int s0, int ns, int n,
                                                       float* __restrict__ g) {
  for (int c = blockIdx.x * kThreads + threadIdx.x; c < n; c += gridDim.x * kThreads) {
    double acc = 0.0;
    for (int k = s0; k < s0 + ns; ++k) {
      const FwiSys& S = tab[k];
      const float2 w = S.w[c], z = S.z[c];
      const double ur = S.mult.x * w.x - S.mult.y * w.y;
      const double ui = S.mult.x * w.y + S.mult.y * w.x;
      acc -= S.omega2 * (ur * z.x - ui * z.y);  // Re(u * z)
    }
    g[c] = (float)acc;
  }
}

// u = mult * w for every system that asked for it.  grid = (blocks, n_sys).
__global__ void __launch_bounds__(kThreads) k_fwi_scale(const FwiSys* __restrict__ tab) {
  const FwiSys& S = tab[blockIdx.y];
  if (S.u == nullptr) return;
  for (int c = blockIdx.x * kThreads + threadIdx.x; c < S.n; c += gridDim.x * kThreads) {
    const float2 w = S.w[c];
    S.u[c] = make_float2((float)(S.mult.x * w.x - S.mult.y * w.y), (float)(S.mult.x * w.y + S.mult.y * w.x));
  }
}

__global__ void __launch_bounds__(kThreads) k_fwi_zero(float* __restrict__ g, int n) {
  for (int c = blockIdx.x * kThreads + threadIdx.x; c < n; c += gridDim.x * kThreads) g[c] = 0.f;
}

int64_t ncells(const wri_grid& g) { return (int64_t)g.nx * g.ny * g.nz; }

int pass_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + kThreads - 1) / kThreads, 4096)); }

// The systems of the forward solve: lambda = 0, and alpha = 1 when the weight
// is estimated afterwards.
std::vector<wri_system> forward_systems(const wri_system* sys, int n_sys, int mode) {
  std::vector<wri_system> s(sys, sys + n_sys);
  for (auto& x : s) {
    x.lambda = 0.0;
    if (mode == WRI_ESTIMATE) x.alpha = wri_c64{1.0, 0.0};
  }
  return s;
}

struct FwiLayout {
  size_t solver = 0, solver_bytes = 0, tab = 0, total = 0;
  std::vector<size_t> w, z, adj, rec;
};

int fwi_layout(const wri_grid* grids, int n_grids, const std::vector<wri_system>& sf, int mode, int flags,
               FwiLayout* L) {
  (void)mode;
  const int n_sys = (int)sf.size();
  const size_t a = wri_workspace_bytes(grids, n_grids, sf.data(), n_sys, WRI_KNOWN, flags);
  if (a == 0) return WRI_EINVAL;
  const size_t b = wri_workspace_bytes(grids, n_grids, sf.data(), n_sys, WRI_KNOWN, flags | WRI_FLAG_ADJOINT_SOURCE);
  if (b == 0) return WRI_EINVAL;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = al(o + std::max<size_t>(bytes, 1)); return r; };
  L->solver_bytes = std::max(a, b);
  L->solver = take(L->solver_bytes);
  L->tab = take(sizeof(FwiSys) * (size_t)std::max(n_sys, 1));
  L->w.resize(n_sys); L->z.resize(n_sys); L->adj.resize(n_sys); L->rec.resize(n_sys);
  for (int i = 0; i < n_sys; ++i) {
    const size_t vb = sizeof(float2) * (size_t)ncells(grids[sf[i].grid]);
    L->w[i] = take(vb);
    L->z[i] = take(vb);
    L->adj[i] = take(sizeof(float2) * (size_t)sf[i].n_rec);
    L->rec[i] = take(sizeof(int32_t) * (size_t)sf[i].n_rec);
  }
  L->total = o + kAl;  // slack for aligning the caller's base pointer
  return WRI_OK;
}

int fwi_run(const wri_grid* grids, int32_t n_grids, const float* const* m, const wri_system* sys, int32_t n_sys,
            int32_t mode, int32_t max_iter, int32_t flags, double* f_out, float* const* grad,
            wri_c32* const* u_out, wri_fwi_result* res, void* ws, size_t ws_bytes, void* stream) {
  if (f_out == nullptr) return report_error(WRI_EINVAL, "f_out is NULL");
  if (n_sys > 0 && res == nullptr) return report_error(WRI_EINVAL, "res is NULL");
  if (flags & WRI_FLAG_WARM_START) return report_error(WRI_EINVAL, "the FWI baseline takes no WRI_FLAG_WARM_START");
  if (flags & WRI_FLAG_ADJOINT_SOURCE)
    return report_error(WRI_EINVAL, "WRI_FLAG_ADJOINT_SOURCE is set internally for the adjoint solve");
  int rc = wri_validate(grids, n_grids, sys, n_sys, mode, max_iter);
  if (rc != WRI_OK) return rc;
  if (grad != nullptr)
    for (int g = 0; g < n_grids; ++g)
      if (grad[g] == nullptr) return report_error(WRI_EINVAL, "grad[%d] is NULL", g);
  if (u_out != nullptr)
    for (int i = 0; i < n_sys; ++i)
      if (u_out[i] == nullptr) return report_error(WRI_EINVAL, "u_out[%d] is NULL", i);
  std::vector<wri_system> sf = forward_systems(sys, n_sys, mode);
  FwiLayout L;
  rc = fwi_layout(grids, n_grids, sf, mode, flags, &L);
  if (rc != WRI_OK) return rc;
  if (ws == nullptr || ws_bytes < L.total)
    return report_error(WRI_ENOWS, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, L.total);
  char* base = reinterpret_cast<char*>(al(reinterpret_cast<uintptr_t>(ws)));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  *f_out = 0.0;
  if (n_sys == 0) {
    if (grad != nullptr)
      for (int g = 0; g < n_grids; ++g) {
        const int n = (int)ncells(grids[g]);
        hipLaunchKernelGGL(k_fwi_zero, dim3(pass_blocks(n)), dim3(kThreads), 0, st, grad[g], n);
        FWI_HIP(hipGetLastError());
      }
    FWI_HIP(hipStreamSynchronize(st));
    return WRI_OK;
  }

  // 1. forward solves
  std::vector<wri_c32*> wp(n_sys), zp(n_sys);
  for (int i = 0; i < n_sys; ++i) {
    wp[i] = reinterpret_cast<wri_c32*>(base + L.w[i]);
    zp[i] = reinterpret_cast<wri_c32*>(base + L.z[i]);
  }
  std::vector<wri_result> rf(n_sys), ra(n_sys);
  const int rcf = wri_solve(grids, n_grids, m, sf.data(), n_sys, WRI_KNOWN, max_iter, flags, wp.data(), rf.data(),
                            base + L.solver, L.solver_bytes, stream);
  if (rcf < 0 && rcf != WRI_EBREAKDOWN) return rcf;
  for (int i = 0; i < n_sys; ++i) {
    res[i] = wri_fwi_result{};
    res[i].iters_fwd = rf[i].iters;
    res[i].status_fwd = rf[i].status;
    res[i].status_adj = WRI_SYS_ZERO_RHS;
  }
  if (rcf == WRI_EBREAKDOWN) return report_error(WRI_EBREAKDOWN, "a forward solve broke down");

  // 2. source weights, residuals, adjoint sources (systems grouped by grid)
  std::vector<int> order(n_sys);
  for (int i = 0; i < n_sys; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return sys[a].grid < sys[b].grid; });
  std::vector<FwiSys> tab(n_sys);
  for (int p = 0; p < n_sys; ++p) {
    const int i = order[p];
    FwiSys& T = tab[p];
    std::memset(&T, 0, sizeof(T));
    T.w = reinterpret_cast<const float2*>(wp[i]);
    T.z = reinterpret_cast<const float2*>(zp[i]);
    T.d = reinterpret_cast<const float2*>(sys[i].d);
    T.rec = reinterpret_cast<const int*>(base + L.rec[i]);
    T.adj = reinterpret_cast<float2*>(base + L.adj[i]);
    T.u = u_out != nullptr ? reinterpret_cast<float2*>(u_out[i]) : nullptr;
    T.omega2 = sys[i].omega * sys[i].omega;
    T.n_rec = sys[i].n_rec;
    T.estimate = mode == WRI_ESTIMATE;
    T.n = (int)ncells(grids[sys[i].grid]);
    if (sys[i].n_rec > 0)
      FWI_HIP(hipMemcpyAsync(base + L.rec[i], sys[i].rec, sizeof(int32_t) * sys[i].n_rec, hipMemcpyHostToDevice, st));
  }
  FwiSys* dtab = reinterpret_cast<FwiSys*>(base + L.tab);
  FWI_HIP(hipMemcpyAsync(dtab, tab.data(), sizeof(FwiSys) * n_sys, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_fwi_residual, dim3(n_sys), dim3(kThreads), 0, st, dtab);
  FWI_HIP(hipGetLastError());
  FWI_HIP(hipStreamSynchronize(st));  // the host table and receiver lists are read by the copies above

  // 3. adjoint solves: A z = P^H conj(rho)
  std::vector<wri_system> sa = sf;
  for (int i = 0; i < n_sys; ++i) sa[i].d = reinterpret_cast<const wri_c32*>(base + L.adj[i]);
  const int rca = wri_solve(grids, n_grids, m, sa.data(), n_sys, WRI_KNOWN, max_iter,
                            flags | WRI_FLAG_ADJOINT_SOURCE, zp.data(), ra.data(), base + L.solver, L.solver_bytes,
                            stream);
  if (rca < 0 && rca != WRI_EBREAKDOWN) return rca;
  for (int i = 0; i < n_sys; ++i) {
    res[i].iters_adj = ra[i].iters;
    res[i].status_adj = ra[i].status;
  }

  // 4. gradient per grid, wavefield output
  if (rca != WRI_EBREAKDOWN && grad != nullptr) {
    for (int g = 0; g < n_grids; ++g) {
      int s0 = n_sys, ns = 0;
      for (int p = 0; p < n_sys; ++p)
        if (sys[order[p]].grid == g) { s0 = std::min(s0, p); ++ns; }
      const int n = (int)ncells(grids[g]);
      if (ns == 0) hipLaunchKernelGGL(k_fwi_zero, dim3(pass_blocks(n)), dim3(kThreads), 0, st, grad[g], n);
      else hipLaunchKernelGGL(k_fwi_grad, dim3(pass_blocks(n)), dim3(kThreads), 0, st, dtab, s0, ns, n, grad[g]);
      FWI_HIP(hipGetLastError());
    }
  }
  if (u_out != nullptr) {
    int64_t nmax = 1;
    for (int i = 0; i < n_sys; ++i) nmax = std::max<int64_t>(nmax, ncells(grids[sys[i].grid]));
    hipLaunchKernelGGL(k_fwi_scale, dim3(pass_blocks(nmax), n_sys), dim3(kThreads), 0, st, dtab);
    FWI_HIP(hipGetLastError());
  }
  FWI_HIP(hipMemcpyAsync(tab.data(), dtab, sizeof(FwiSys) * n_sys, hipMemcpyDeviceToHost, st));
  FWI_HIP(hipStreamSynchronize(st));
  double f = 0.0;
  bool not_conv = false;
  for (int p = 0; p < n_sys; ++p) {
    const int i = order[p];
    res[i].f = tab[p].f;
    res[i].alpha = mode == WRI_ESTIMATE ? wri_c64{tab[p].mult.x, tab[p].mult.y} : sys[i].alpha;
    f += tab[p].f;
    for (int st2 : {res[i].status_fwd, res[i].status_adj})
      not_conv = not_conv || st2 == WRI_SYS_MAX_ITER || st2 == WRI_SYS_DIVERGED;
  }
  *f_out = f;
  if (rca == WRI_EBREAKDOWN) return report_error(WRI_EBREAKDOWN, "an adjoint solve broke down");
  return not_conv ? WRI_NOT_CONVERGED : WRI_OK;
}

}  // namespace
}  // namespace wri

using namespace wri;

extern "C" {

size_t wri_fwi_workspace_bytes(const wri_grid* grids, int32_t n_grids, const wri_system* sys, int32_t n_sys,
                               int32_t mode, int32_t flags) {
  try {
    if (wri_validate(grids, n_grids, sys, n_sys, mode, 0) != WRI_OK) return 0;
    FwiLayout L;
    if (fwi_layout(grids, n_grids, forward_systems(sys, n_sys, mode), mode, flags, &L) != WRI_OK) return 0;
    return L.total;
  } catch (const std::exception& e) {
    report_error(WRI_EINVAL, "exception: %s", e.what());
    return 0;
  }
}

int wri_fwi_objective_grad(const wri_grid* grids, int32_t n_grids, const float* const* m, const wri_system* sys,
                           int32_t n_sys, int32_t mode, int32_t max_iter, int32_t flags, double* f_out,
                           float* const* grad, wri_c32* const* u_out, wri_fwi_result* res, void* ws,
                           size_t ws_bytes, void* stream) {
  try {
    return fwi_run(grids, n_grids, m, sys, n_sys, mode, max_iter, flags, f_out, grad, u_out, res, ws, ws_bytes,
                   stream);
  } catch (const std::exception& e) {
    return report_error(WRI_EINVAL, "exception: %s", e.what());
  }
}

}  // extern "C"
