// Sources and receivers off the grid nodes: the source vector e and the
// receiver sampling P of eqs. ObjPen / SimpObj become trilinear interpolation
// weights over up to 8 cells each, and the same CGLS (the reading of
// Algorithm 1 used throughout the library) runs system by system with the
// library's single-operator stencil and vector kernels plus the weighted
// source and receiver kernels below.  Scalars are float64 on the host, every
// reduction runs in one fixed order.
//
// P p: one thread per receiver sums its weighted cells (reads only).  P^H r2:
// a gather over the distinct receiver cells of a system (each cell's list of
// (receiver, weight) pairs is built on the host), so cells shared by several
// receivers need no atomics.  Source cells are distinct by construction.
#include "../../include/wri.h"
#include "wri_impl.hpp"

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

// r[cells] = alpha * w
__global__ void k_og_src_set(float2* __restrict__ r, const int* __restrict__ cells, const double* __restrict__ w,
                             int nc, double2 a) {
  const int i = threadIdx.x;
  if (i < nc) r[cells[i]] = make_float2((float)(a.x * w[i]), (float)(a.y * w[i]));
}

// t[cells] -= cp * w
__global__ void k_og_src_sub(float2* __restrict__ t, const int* __restrict__ cells, const double* __restrict__ w,
                             int nc, double2 cp) {
  const int i = threadIdx.x;
  if (i < nc) {
    const float2 v = t[cells[i]];
    t[cells[i]] = make_float2((float)((double)v.x - cp.x * w[i]), (float)((double)v.y - cp.y * w[i]));
  }
}

// out = sum_k w_k v[cells_k] (one thread, fixed order)
__global__ void k_og_src_dot(const float2* __restrict__ v, const int* __restrict__ cells,
                             const double* __restrict__ w, int nc, double2* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double re = 0.0, im = 0.0;
  for (int i = 0; i < nc; ++i) {
    const float2 x = v[cells[i]];
    re += w[i] * (double)x.x;
    im += w[i] * (double)x.y;
  }
  *out = make_double2(re, im);
}

// t2[q] = lam * sum_j w_j p[cell_j] over receiver q's cells
__global__ void k_og_gather(float2* __restrict__ t2, const float2* __restrict__ p, const int* __restrict__ ptr,
                            const int* __restrict__ cell, const double* __restrict__ w, int n_rec, double lam) {
  const int q = blockIdx.x * kThreads + threadIdx.x;
  if (q >= n_rec) return;
  double re = 0.0, im = 0.0;
  for (int j = ptr[q]; j < ptr[q + 1]; ++j) {
    const float2 x = p[cell[j]];
    re += w[j] * (double)x.x;
    im += w[j] * (double)x.y;
  }
  t2[q] = make_float2((float)(lam * re), (float)(lam * im));
}

// s[ucell[u]] += lam * sum_j w_j r2[q_j] over the (receiver, weight) pairs of
// distinct cell u
__global__ void k_og_scatter(float2* __restrict__ s, const float2* __restrict__ r2, const int* __restrict__ ptr,
                             const int* __restrict__ ucell, const int* __restrict__ uq, const double* __restrict__ uw,
                             int n_u, double lam) {
  const int u = blockIdx.x * kThreads + threadIdx.x;
  if (u >= n_u) return;
  double re = 0.0, im = 0.0;
  for (int j = ptr[u]; j < ptr[u + 1]; ++j) {
    const float2 x = r2[uq[j]];
    re += uw[j] * (double)x.x;
    im += uw[j] * (double)x.y;
  }
  const float2 v = s[ucell[u]];
  s[ucell[u]] = make_float2((float)((double)v.x + lam * re), (float)((double)v.y + lam * im));
}

// r2 = lam * d
__global__ void k_og_r2(float2* __restrict__ r2, const float2* __restrict__ d, int n, double lam) {
  const int q = blockIdx.x * kThreads + threadIdx.x;
  if (q < n) r2[q] = make_float2((float)(lam * (double)d[q].x), (float)(lam * (double)d[q].y));
}

// g += -2 omega^2 Re(conj(u) r1)  (r1 = alpha e - A u, the recurred PDE residual)
__global__ void k_og_grad(float* __restrict__ g, const float2* __restrict__ u, const float2* __restrict__ r, int n,
                          double w2) {
  for (int c = blockIdx.x * kThreads + threadIdx.x; c < n; c += gridDim.x * kThreads) {
    const float2 a = u[c], b = r[c];
    g[c] = (float)((double)g[c] - 2.0 * w2 * ((double)a.x * b.x + (double)a.y * b.y));
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
  size_t vec = 0, rvec = 0, dots = 0, tables = 0, total = 0;
  size_t vb = 0, rb = 0;
  int dparts = 1;
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
  int64_t nmax = 1, rmax = 1;
  for (int k = 0; k < n_sys; ++k) {
    nmax = std::max<int64_t>(nmax, ncell(grids[sys[k].grid]));
    rmax = std::max<int64_t>(rmax, sys[k].n_rec);
  }
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = al(o + std::max<size_t>(bytes, 1)); return r; };
  L->vb = al(sizeof(float2) * (size_t)nmax);
  L->rb = al(sizeof(float2) * (size_t)rmax);
  L->vec = take(5 * L->vb);
  L->rvec = take(2 * L->rb);
  L->dparts = dot_parts((int)std::max(nmax, rmax));
  L->dots = take(sizeof(double) * (size_t)(16 + L->dparts));
  L->tables = o;
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
  std::vector<DevTables> dt(n_sys);
  for (int k = 0; k < n_sys; ++k) {
    const SysTables& T = tabs[k];
    DevTables& D = dt[k];
    D = place(base, T);
    OG_HIP(up(D.scell, T.src.cells, st)); OG_HIP(up(D.sw, T.src.w, st));
    OG_HIP(up(D.rptr, T.rptr, st)); OG_HIP(up(D.rcell, T.rcell, st)); OG_HIP(up(D.rw, T.rw, st));
    OG_HIP(up(D.uptr, T.uptr, st)); OG_HIP(up(D.ucell, T.ucell, st)); OG_HIP(up(D.uq, T.uq, st));
    OG_HIP(up(D.uw, T.uw, st));
  }
  OG_HIP(hipStreamSynchronize(st));  // the host tables are read by the copies above
  float2* xw = reinterpret_cast<float2*>(base + L.vec);
  float2* rv = reinterpret_cast<float2*>(base + L.vec + L.vb);
  float2* pv = reinterpret_cast<float2*>(base + L.vec + 2 * L.vb);
  float2* sv = reinterpret_cast<float2*>(base + L.vec + 3 * L.vb);
  float2* tv = reinterpret_cast<float2*>(base + L.vec + 4 * L.vb);
  float2* r2 = reinterpret_cast<float2*>(base + L.rvec);
  float2* t2 = reinterpret_cast<float2*>(base + L.rvec + L.rb);
  double* dres = reinterpret_cast<double*>(base + L.dots);  // [0] |t|^2 [1] |t2|^2 [2] |s|^2 [3] |r2|^2
  double2* dsrc = reinterpret_cast<double2*>(dres + 8);      // e^H r1, e^H (A u)
  double* part = dres + 16;                                  // dot-product partials
  if (grad != nullptr)
    for (int g = 0; g < n_grids; ++g) OG_HIP(launch_zero_f32(grad[g], (size_t)ncell(grids[g]), st));
  double Jtot = 0.0;
  int ret = WRI_OK;
  for (int k = 0; k < n_sys; ++k) {
    const wri_system& s = sys[k];
    const wri_grid& g = grids[s.grid];
    const DevTables& D = dt[k];
    const int n = (int)ncell(g);
    const int nr = s.n_rec;
    const int ns = (int)tabs[k].src.cells.size();
    const int nu = (int)tabs[k].ucell.size();
    const bool est = mode == WRI_ESTIMATE;
    const double h2inv = 1.0 / (g.h * g.h);
    double sp_scale = 0.0, inv_nb = 0.0;
    if (g.nb > 0) {
      const double d0 = 3.0 * g.v_ref * std::log(1000.0) / (2.0 * g.nb * g.h);
      sp_scale = 2.0 * d0 / (g.v_ref * g.v_ref);
      inv_nb = 1.0 / g.nb;
    }
    const double c = (flags & WRI_FLAG_UNSCALED_ALPHA) ? 1.0 : std::sqrt(42.0) * h2inv;
    const double lam = s.lambda;
    const double rtol2 = s.rtol * s.rtol;
    float2* x = (u_out != nullptr && u_out[k] != nullptr) ? reinterpret_cast<float2*>(u_out[k]) : xw;
    const float2 z = make_float2(0.f, 0.f);
    const int dp = dot_parts(n), dpr = dot_parts(std::max(nr, 1));
    auto dot = [&](const float2* v, int len, double* out) -> int {
      const int npp = len == n ? dp : dpr;
      OG_HIP(launch_dot(v, len, part, npp, st));
      OG_HIP(launch_sum(part, npp, out, st));
      return WRI_OK;
    };
    // x = 0, r1 = alpha e (KNOWN), r2 = lam d
    OG_HIP(launch_fill_f2(x, z, n, st));
    OG_HIP(launch_fill_f2(rv, z, n, st));
    if (!est && ns > 0) {
      hipLaunchKernelGGL(k_og_src_set, dim3(1), dim3(64), 0, st, rv, D.scell, D.sw, ns,
                         make_double2(s.alpha.re, s.alpha.im));
      OG_HIP(hipGetLastError());
    }
    if (nr > 0) {
      hipLaunchKernelGGL(k_og_r2, dim3(nblk(nr)), dim3(kThreads), 0, st, r2, reinterpret_cast<const float2*>(s.d), nr,
                         lam);
      OG_HIP(hipGetLastError());
    }
    double hres[4] = {0, 0, 0, 0};
    double2 hsrc = make_double2(0.0, 0.0);
    double sa_re = 0.0, sa_im = 0.0;
    // s = S^H r: wavefield rows A^H r1 + lam P^H r2; source row -c e^H r1
    auto apply_SH = [&]() -> int {
      OG_HIP(launch_apply(g.nx, g.ny, g.nz, g.nb, h2inv, sp_scale, inv_nb, s.omega, m[s.grid], rv, sv, 1, -1,
                          make_double2(0.0, 0.0), st));
      if (nu > 0) {
        hipLaunchKernelGGL(k_og_scatter, dim3(nblk(nu)), dim3(kThreads), 0, st, sv, r2, D.uptr, D.ucell, D.uq, D.uw,
                           nu, lam);
        OG_HIP(hipGetLastError());
      }
      int e = dot(sv, n, dres + 2);
      if (e != WRI_OK) return e;
      if (est && ns > 0) {
        hipLaunchKernelGGL(k_og_src_dot, dim3(1), dim3(64), 0, st, rv, D.scell, D.sw, ns, dsrc);
        OG_HIP(hipGetLastError());
      }
      OG_HIP(hipMemcpyAsync(hres + 2, dres + 2, sizeof(double), hipMemcpyDeviceToHost, st));
      OG_HIP(hipMemcpyAsync(&hsrc, dsrc, sizeof(double2), hipMemcpyDeviceToHost, st));
      OG_HIP(hipStreamSynchronize(st));
      sa_re = (est && ns > 0) ? -c * hsrc.x : 0.0;
      sa_im = (est && ns > 0) ? -c * hsrc.y : 0.0;
      return WRI_OK;
    };
    rc = apply_SH();
    if (rc != WRI_OK) return rc;
    double gamma = hres[2] + sa_re * sa_re + sa_im * sa_im;
    const double gamma0 = gamma;
    OG_HIP(launch_copy_f2(pv, sv, n, st));
    double pa_re = sa_re, pa_im = sa_im, xa_re = 0.0, xa_im = 0.0;
    int it = 0, status = kActive;
    while (true) {
      if (gamma0 == 0.0) { status = kZeroRhs; break; }
      if (gamma <= rtol2 * gamma0) { status = kConverged; break; }
      if (it >= max_iter) { status = kMaxIter; break; }
      // t = S p: A p_u - c p_a e ; t2 = lam P p_u
      OG_HIP(launch_apply(g.nx, g.ny, g.nz, g.nb, h2inv, sp_scale, inv_nb, s.omega, m[s.grid], pv, tv, 0, -1,
                          make_double2(0.0, 0.0), st));
      if (est && ns > 0) {
        hipLaunchKernelGGL(k_og_src_sub, dim3(1), dim3(64), 0, st, tv, D.scell, D.sw, ns,
                           make_double2(c * pa_re, c * pa_im));
        OG_HIP(hipGetLastError());
      }
      if (nr > 0) {
        hipLaunchKernelGGL(k_og_gather, dim3(nblk(nr)), dim3(kThreads), 0, st, t2, pv, D.rptr, D.rcell, D.rw, nr,
                           lam);
        OG_HIP(hipGetLastError());
      }
      rc = dot(tv, n, dres + 0);
      if (rc != WRI_OK) return rc;
      if (nr > 0) {
        rc = dot(t2, nr, dres + 1);
        if (rc != WRI_OK) return rc;
      }
      OG_HIP(hipMemcpyAsync(hres, dres, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
      OG_HIP(hipStreamSynchronize(st));
      const double delta = hres[0] + (nr > 0 ? hres[1] : 0.0);
      if (!(delta > 0.0) || !std::isfinite(delta) || !std::isfinite(gamma)) { status = kBreakdown; break; }
      const double a = gamma / delta;
      OG_HIP(launch_axpy(x, pv, a, n, st));
      OG_HIP(launch_axpy(rv, tv, -a, n, st));
      OG_HIP(launch_axpy(r2, t2, -a, nr, st));
      xa_re += a * pa_re;
      xa_im += a * pa_im;
      rc = apply_SH();
      if (rc != WRI_OK) return rc;
      const double gnew = hres[2] + sa_re * sa_re + sa_im * sa_im;
      const double beta = gnew / gamma;
      gamma = gnew;
      OG_HIP(launch_xpby(pv, sv, beta, n, st));
      pa_re = sa_re + beta * pa_re;
      pa_im = sa_im + beta * pa_im;
      ++it;
    }
    // objective from the recurred residuals, gradient, source weights
    rc = dot(rv, n, dres + 0);
    if (rc != WRI_OK) return rc;
    if (nr > 0) {
      rc = dot(r2, nr, dres + 3);
      if (rc != WRI_OK) return rc;
    }
    if (grad != nullptr && status != kBreakdown) {
      hipLaunchKernelGGL(k_og_grad, dim3(nblk(n)), dim3(kThreads), 0, st, grad[s.grid], x, rv, n,
                         s.omega * s.omega);
      OG_HIP(hipGetLastError());
    }
    double2 eau = make_double2(0.0, 0.0);
    if (est && ns > 0) {  // alpha_ls = e^H (A u) / e^H e
      OG_HIP(launch_apply(g.nx, g.ny, g.nz, g.nb, h2inv, sp_scale, inv_nb, s.omega, m[s.grid], x, tv, 0, -1,
                          make_double2(0.0, 0.0), st));
      hipLaunchKernelGGL(k_og_src_dot, dim3(1), dim3(64), 0, st, tv, D.scell, D.sw, ns, dsrc + 1);
      OG_HIP(hipGetLastError());
      OG_HIP(hipMemcpyAsync(&eau, dsrc + 1, sizeof(double2), hipMemcpyDeviceToHost, st));
    }
    OG_HIP(hipMemcpyAsync(hres, dres, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
    OG_HIP(hipStreamSynchronize(st));
    double ee = 0.0;
    for (double w : tabs[k].src.w) ee += w * w;
    wri_result& r = res[k];
    r.iters = it;
    r.status = status;
    r.relres = gamma0 > 0.0 ? std::sqrt(std::max(gamma, 0.0) / gamma0) : 0.0;
    r.J = hres[0] + (nr > 0 ? hres[3] : 0.0);
    if (est) {
      r.alpha = wri_c64{c * xa_re, c * xa_im};
      r.alpha_ls = ee > 0.0 ? wri_c64{eau.x / ee, eau.y / ee} : wri_c64{0.0, 0.0};
    } else {
      r.alpha = s.alpha;
      r.alpha_ls = s.alpha;
    }
    Jtot += r.J;
    if (status == kBreakdown) ret = WRI_EBREAKDOWN;
    else if (status == kMaxIter && ret == WRI_OK) ret = WRI_NOT_CONVERGED;
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
