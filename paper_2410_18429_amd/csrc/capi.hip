// Host side of the library: argument validation, the work planner (workspace
// layout, receiver column maps, per-grid slab tiles), the slab-tile autotuner,
// hipGraph capture of the batched CGLS iterations, the unfused one-system
// baseline, and the C ABI declared in include/wri.h.
#include "../../include/wri.h"
#include "wri_impl.hpp"

#include <chrono>
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

namespace wri {
namespace {

thread_local std::string g_last_error;

// Algorithmic HBM bytes per cell of the fused launches (complex64 vectors,
// float32 model), the figures the roofline is quoted on.
//   forward k: reads s, p_{k-1}, m; writes p_k, t                       36 B
//              + at even k >= 2 reads x, p_{k-2} and writes x           24 B
//   adjoint k: reads r_k, t, m; writes r_{k+1}, s                       36 B
// With t recomputed in the adjoint pass (tile pf >= 2) the forward pass does
// not write t (28 B) and the adjoint pass reads p_k in its place (36 B).
// Halo re-reads and the receiver rows are not counted.
constexpr int kFwdBytesPerCell = 36, kFwdXBytesPerCell = 24, kAdjBytesPerCell = 36, kTBytesPerCell = 8;
inline int fwd_bytes_per_cell(int64_t k, int pf) {
  return kFwdBytesPerCell - (pf >= 2 ? kTBytesPerCell : 0) + ((k >= 2 && (k & 1) == 0) ? kFwdXBytesPerCell : 0);
}

struct KernelTimes {
  bool valid = false;
  wri_timing t{};
};
thread_local KernelTimes g_times;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define WRI_HIP(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(WRI_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                  __LINE__);                                                            \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Slab-tile candidates explored by the autotuner; the first is the default.
const TileCfg kCands[] = {
    {4, 4, 32, 0, 0}, {4, 2, 32, 1, 0}, {4, 2, 32, 1, 1}, {4, 2, 16, 1, 1}, {4, 2, 64, 1, 1},
    {8, 1, 32, 1, 0}, {8, 1, 32, 1, 1}, {8, 1, 16, 1, 1}, {8, 2, 32, 1, 0}, {8, 2, 32, 1, 1},
    {4, 1, 32, 1, 1}, {4, 1, 64, 1, 1}, {4, 4, 32, 1, 1}, {4, 2, 32, 0, 1}, {8, 1, 16, 0, 1},
    {8, 2, 16, 0, 1}, {4, 2, 16, 0, 0}, {8, 1, 16, 0, 0}, {2, 8, 32, 0, 0}, {4, 4, 16, 0, 1},
    {8, 1, 32, 1, 2}, {8, 1, 32, 1, 4}, {8, 1, 32, 1, 8}, {4, 2, 32, 1, 2},
    {8, 1, 32, 2, 4}, {8, 2, 32, 2, 4}, {4, 4, 32, 2, 4}, {4, 2, 32, 2, 4}, {8, 1, 32, 2, 0},
    {8, 1, 32, 3, 4}, {4, 2, 32, 3, 4}, {4, 2, 64, 2, 4}, {4, 2, 16, 2, 4}, {8, 1, 64, 3, 4},
    {4, 4, 32, 1, 4}, {8, 4, 64, 2, 4}, {8, 4, 32, 2, 4}, {4, 4, 64, 2, 4}, {8, 4, 32, 1, 4},
    {8, 4, 64, 2, 8}, {8, 4, 64, 2, 2},
};
constexpr int kNumCands = sizeof(kCands) / sizeof(kCands[0]);

struct Tiling {
  TileCfg cfg;
  int tx, ty, tz;  // tile counts per axis
  int ntiles() const { return tx * ty * tz; }
};

Tiling make_tiling(const TileCfg& c, const wri_grid& g) {
  Tiling t;
  t.cfg = c;
  t.tx = (g.nx + kTX - 1) / kTX;
  t.ty = (g.ny + c.ty() - 1) / c.ty();
  t.tz = (g.nz + c.tz - 1) / c.tz;
  return t;
}

int max_tiles(const wri_grid& g) {
  int m = 1;
  for (int i = 0; i < kNumCands; ++i) m = std::max(m, make_tiling(kCands[i], g).ntiles());
  return m;
}

int64_t cells(const wri_grid& g) { return (int64_t)g.nx * g.ny * g.nz; }

// ---------------------------------------------------------------------------
// validation (host only)
// ---------------------------------------------------------------------------

constexpr int64_t kMaxPlaneSpan = 72;  // planes a slab's buffer offsets may span (z-slab <= 64, halo, prefetch)

int validate(const wri_grid* grids, int32_t n_grids, const wri_system* sys, int32_t n_sys, int32_t mode,
             int32_t max_iter) {
  if (n_grids < 0 || n_sys < 0) return fail(WRI_EINVAL, "negative n_grids or n_sys");
  if (n_grids > 0 && grids == nullptr) return fail(WRI_EINVAL, "grids is NULL");
  if (n_sys > 0 && sys == nullptr) return fail(WRI_EINVAL, "sys is NULL");
  if (mode != WRI_KNOWN && mode != WRI_ESTIMATE) return fail(WRI_EINVAL, "mode %d is not WRI_KNOWN/WRI_ESTIMATE", mode);
  if (max_iter < 0) return fail(WRI_EINVAL, "max_iter < 0");
  for (int i = 0; i < n_grids; ++i) {
    const wri_grid& g = grids[i];
    if (g.nx < 1 || g.ny < 1 || g.nz < 1) return fail(WRI_EINVAL, "grid %d: non-positive size", i);
    if (cells(g) >= (int64_t(1) << 31)) return fail(WRI_EINVAL, "grid %d: more than 2^31-1 cells", i);
    // the fused kernels address up to 72 planes of complex64 with 32-bit byte offsets
    if ((int64_t)g.nx * g.ny * kMaxPlaneSpan * 8 >= (int64_t(1) << 31))
      return fail(WRI_EINVAL, "grid %d: more than %lld cells in one x-y plane", i,
                  (long long)(((int64_t(1) << 31) - 1) / (kMaxPlaneSpan * 8)));
    if (!(g.h > 0.0) || !std::isfinite(g.h)) return fail(WRI_EINVAL, "grid %d: h must be > 0", i);
    if (g.nb < 0) return fail(WRI_EINVAL, "grid %d: nb < 0", i);
    if (g.nb > 0 && (!(g.v_ref > 0.0) || !std::isfinite(g.v_ref)))
      return fail(WRI_EINVAL, "grid %d: v_ref must be > 0 when nb > 0", i);
  }
  std::vector<int32_t> tmp;
  for (int k = 0; k < n_sys; ++k) {
    const wri_system& s = sys[k];
    if (s.grid < 0 || s.grid >= n_grids) return fail(WRI_EINVAL, "system %d: grid index %d out of range", k, s.grid);
    const wri_grid& g = grids[s.grid];
    const int64_t n = cells(g);
    if (!(s.omega >= 0.0) || !std::isfinite(s.omega)) return fail(WRI_EINVAL, "system %d: omega must be finite and >= 0", k);
    if (!(s.lambda >= 0.0) || !std::isfinite(s.lambda)) return fail(WRI_EINVAL, "system %d: lambda must be finite and >= 0", k);
    if (!(s.rtol >= 0.0) || !std::isfinite(s.rtol)) return fail(WRI_EINVAL, "system %d: rtol must be finite and >= 0", k);
    if (s.src < 0 || s.src >= n) return fail(WRI_ERANGE, "system %d: source cell %d outside grid", k, s.src);
    if (s.n_rec < 0) return fail(WRI_EINVAL, "system %d: n_rec < 0", k);
    if (s.n_rec > 0 && (s.rec == nullptr || s.d == nullptr))
      return fail(WRI_EINVAL, "system %d: rec or d is NULL", k);
    if (mode == WRI_KNOWN && (!std::isfinite(s.alpha.re) || !std::isfinite(s.alpha.im)))
      return fail(WRI_EINVAL, "system %d: alpha not finite", k);
    tmp.assign(s.rec, s.rec + s.n_rec);
    for (int32_t c : tmp)
      if (c < 0 || c >= n) return fail(WRI_ERANGE, "system %d: receiver cell %d outside grid", k, c);
    std::sort(tmp.begin(), tmp.end());
    for (size_t q = 1; q < tmp.size(); ++q)
      if (tmp[q] == tmp[q - 1]) return fail(WRI_EDUP, "system %d: duplicate receiver cell %d", k, tmp[q]);
  }
  return WRI_OK;
}

// ---------------------------------------------------------------------------
// planner: workspace layout (deterministic in the arguments)
// ---------------------------------------------------------------------------

struct RecSet {       // one distinct receiver list on one grid
  int grid;
  std::vector<int32_t> rec;
  size_t off_rec = 0, off_colmap = 0, off_entries = 0;
};

struct Layout {
  bool plain = false;
  std::vector<int> order;           // processing order -> original system index (grouped by grid)
  std::vector<int> set_of;          // original system -> receiver-set id
  std::vector<RecSet> sets;
  size_t off_sysdev = 0, off_state = 0, off_part_d = 0, off_part_s = 0, off_part_j = 0, off_dot = 0;
  size_t off_gdesc = 0;
  size_t off_nparts = 0;            // per processing slot: partial sums of a set-up pass (warm start)
  std::vector<size_t> off_vec;      // per processing slot: base of its 7 vectors (batched) ; plain: one slot
  std::vector<size_t> off_rvec;     // per processing slot: r2, t2
  std::vector<int> slot_base;       // per processing slot
  int part_j_stride = 1;
  int dot_nparts = 1;
  size_t vec_bytes_plain = 0, rvec_bytes_plain = 0;
  size_t total = 0;
};

struct Group {
  int grid;
  int rhs0, nrhs;  // processing slots
};

Layout make_layout(const wri_grid* grids, int n_grids, const wri_system* sys, int n_sys, int flags) {
  Layout L;
  L.plain = (flags & WRI_FLAG_PLAIN) != 0;
  L.order.resize(n_sys);
  for (int i = 0; i < n_sys; ++i) L.order[i] = i;
  std::stable_sort(L.order.begin(), L.order.end(), [&](int a, int b) { return sys[a].grid < sys[b].grid; });
  // distinct receiver sets
  L.set_of.assign(n_sys, -1);
  std::map<std::pair<int, std::vector<int32_t>>, int> seen;
  for (int i = 0; i < n_sys; ++i) {
    std::vector<int32_t> r(sys[i].rec, sys[i].rec + sys[i].n_rec);
    auto key = std::make_pair(sys[i].grid, r);
    auto it = seen.find(key);
    if (it == seen.end()) {
      RecSet rs;
      rs.grid = sys[i].grid;
      rs.rec = std::move(r);
      seen.emplace(std::make_pair(sys[i].grid, rs.rec), (int)L.sets.size());
      L.set_of[i] = (int)L.sets.size();
      L.sets.push_back(std::move(rs));
    } else {
      L.set_of[i] = it->second;
    }
  }
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + std::max<size_t>(bytes, 1)); return r; };
  L.off_sysdev = take(sizeof(SysDev) * std::max(n_sys, 1));
  L.off_state = take(sizeof(SysState) * std::max(n_sys, 1));
  int slots = 0;
  L.slot_base.resize(n_sys);
  for (int p = 0; p < n_sys; ++p) {
    L.slot_base[p] = slots;
    slots += max_tiles(grids[sys[L.order[p]].grid]);
  }
  L.off_part_d = take(sizeof(double) * std::max(slots, 1));
  L.off_part_s = take(sizeof(double) * std::max(slots, 1));
  int gb = 1;
  for (int g = 0; g < n_grids; ++g) gb = std::max(gb, grad_blocks((int)cells(grids[g])));
  L.part_j_stride = gb;
  L.off_part_j = take(sizeof(double) * (size_t)gb * std::max(n_sys, 1));
  int64_t nmax = 1, rmax = 1;
  for (int i = 0; i < n_sys; ++i) {
    nmax = std::max<int64_t>(nmax, cells(grids[sys[i].grid]));
    rmax = std::max<int64_t>(rmax, sys[i].n_rec);
  }
  L.dot_nparts = dot_parts((int)nmax);
  L.off_dot = take(sizeof(double) * (size_t)(L.dot_nparts * 2 + 16));
  L.off_gdesc = take(sizeof(GroupDesc) * (size_t)std::max(n_grids, 1));
  L.off_nparts = take(sizeof(int32_t) * (size_t)std::max(n_sys, 1));
  for (auto& rs : L.sets) {
    const wri_grid& g = grids[rs.grid];
    rs.off_rec = take(sizeof(int32_t) * rs.rec.size());
    rs.off_colmap = take(sizeof(int32_t) * 2 * (size_t)g.nx * g.ny);
    rs.off_entries = take(sizeof(int32_t) * 2 * rs.rec.size());
  }
  if (!L.plain) {
    L.off_vec.resize(n_sys);
    L.off_rvec.resize(n_sys);
    for (int p = 0; p < n_sys; ++p) {
      const wri_system& s = sys[L.order[p]];
      const size_t vb = align_up(sizeof(float2) * (size_t)cells(grids[s.grid]));
      L.off_vec[p] = take(7 * vb);
      L.off_rvec[p] = take(2 * align_up(sizeof(float2) * (size_t)s.n_rec));
    }
  } else {
    const size_t vb = align_up(sizeof(float2) * (size_t)nmax);
    L.vec_bytes_plain = vb;
    L.off_vec.assign(1, take(5 * vb));   // x, r, p, s, t
    L.rvec_bytes_plain = align_up(sizeof(float2) * (size_t)rmax);
    L.off_rvec.assign(1, take(2 * L.rvec_bytes_plain));
  }
  L.total = o + kAlign;  // slack for aligning the caller's base pointer
  return L;
}

// host-side receiver structures: column map and (z, q) entries sorted by z
void build_colmap(const wri_grid& g, const std::vector<int32_t>& rec, std::vector<int32_t>& colmap,
                  std::vector<int32_t>& entries) {
  const int64_t plane = (int64_t)g.nx * g.ny;
  std::vector<std::tuple<int64_t, int32_t, int32_t>> v;  // (column, z, q)
  v.reserve(rec.size());
  for (size_t q = 0; q < rec.size(); ++q) v.emplace_back(rec[q] % plane, (int32_t)(rec[q] / plane), (int32_t)q);
  std::sort(v.begin(), v.end());
  colmap.assign(2 * (size_t)plane, 0);
  entries.resize(2 * rec.size());
  size_t i = 0;
  while (i < v.size()) {
    const int64_t col = std::get<0>(v[i]);
    size_t j = i;
    while (j < v.size() && std::get<0>(v[j]) == col) {
      entries[2 * j] = std::get<1>(v[j]);
      entries[2 * j + 1] = std::get<2>(v[j]);
      ++j;
    }
    colmap[2 * col] = (int32_t)i;
    colmap[2 * col + 1] = (int32_t)j;
    i = j;
  }
}

// ---------------------------------------------------------------------------
// process-wide caches: tuned tiles per shape, captured graphs
// ---------------------------------------------------------------------------

std::mutex g_mutex;
std::map<std::string, TileCfg> g_tuned;  // batch signature -> tile shape

struct GraphEntry {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};
std::map<std::string, GraphEntry> g_graphs;
std::map<int, hipStream_t> g_capture_stream;

hipStream_t capture_stream(int dev) {
  auto it = g_capture_stream.find(dev);
  if (it != g_capture_stream.end()) return it->second;
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
  g_capture_stream[dev] = s;
  return s;
}

// ---------------------------------------------------------------------------
// solver context for one call
// ---------------------------------------------------------------------------

struct Ctx {
  const wri_grid* grids;
  int n_grids;
  const float* const* m;
  const wri_system* sys;
  int n_sys;
  int mode, max_iter, flags;
  wri_c32* const* u_out;
  char* ws;
  hipStream_t st;
  Layout L;
  std::vector<SysDev> hsys;          // processing order
  std::vector<Group> groups;
  std::vector<Tiling> tiling;        // per group (one tile shape for all groups)
  std::vector<GroupDesc> hgd;        // host copy of the device group table
  int nblocks = 0;                   // blocks of one fused launch over all groups
  GroupDesc* dgd = nullptr;
  SysDev* dsys = nullptr;
  SysState* dstate = nullptr;
  double* part_d = nullptr;
  double* part_s = nullptr;
  double* part_j = nullptr;
  double* dot = nullptr;
  int dev = 0;
};

template <class T>
T* at(char* ws, size_t off) { return reinterpret_cast<T*>(ws + off); }

void fill_sysdev(Ctx& C, int p, SysDev& S, float2* x, float2* r0, float2* r1, float2* p0, float2* p1,
                 float2* sv, float2* tv, float2* r2, float2* t2) {
  const int i = C.L.order.empty() ? p : C.L.order[p];
  const wri_system& s = C.sys[i];
  const wri_grid& g = C.grids[s.grid];
  const RecSet& rs = C.L.sets[C.L.set_of[i]];
  std::memset(&S, 0, sizeof(S));
  S.x = x;
  S.r[0] = r0; S.r[1] = r1;
  S.p[0] = p0; S.p[1] = p1;
  S.s = sv; S.t = tv; S.r2 = r2; S.t2 = t2;
  S.m = C.m[s.grid];
  S.d = reinterpret_cast<const float2*>(s.d);
  S.colmap = s.n_rec > 0 ? at<const int2>(C.ws, rs.off_colmap) : nullptr;
  S.entries = s.n_rec > 0 ? at<const int2>(C.ws, rs.off_entries) : nullptr;
  S.rec = s.n_rec > 0 ? at<const int>(C.ws, rs.off_rec) : nullptr;
  S.nx = g.nx; S.ny = g.ny; S.nz = g.nz; S.nb = g.nb;
  S.h2inv_d = 1.0 / (g.h * g.h);
  if (g.nb > 0) {
    const double d0 = 3.0 * g.v_ref * std::log(1000.0) / (2.0 * g.nb * g.h);
    S.sp_scale_d = 2.0 * d0 / (g.v_ref * g.v_ref);
    S.inv_nb_d = 1.0 / g.nb;
  }
  S.h2inv = (float)S.h2inv_d;
  S.sp_scale = (float)S.sp_scale_d;
  S.inv_nb = (float)S.inv_nb_d;
  S.omega_d = s.omega;
  S.omega = (float)s.omega;
  S.omega2 = (float)(s.omega * s.omega);
  S.lam_d = s.lambda;
  S.lam = (float)s.lambda;
  S.src = s.src;
  S.n_rec = s.n_rec;
  S.mode = C.mode;
  S.max_iter = C.max_iter;
  S.rtol2 = s.rtol * s.rtol;
  S.alpha = make_double2(s.alpha.re, s.alpha.im);
  // Column equilibration of S in ESTIMATE mode: the source column -e is scaled
  // to -c e with c = sqrt(42)/h^2, the norm of a Laplacian column, so that the
  // unknown alpha/c does not dominate the spectrum of S^H S.
  S.alpha_c = (C.flags & WRI_FLAG_UNSCALED_ALPHA) ? 1.0 : std::sqrt(42.0) * S.h2inv_d;
  S.slot_base = C.L.slot_base[p];
  S.grid_id = s.grid;
}

int upload_receivers(Ctx& C) {
  for (auto& rs : C.L.sets) {
    if (rs.rec.empty()) continue;
    std::vector<int32_t> colmap, entries;
    build_colmap(C.grids[rs.grid], rs.rec, colmap, entries);
    WRI_HIP(hipMemcpyAsync(C.ws + rs.off_rec, rs.rec.data(), rs.rec.size() * 4, hipMemcpyHostToDevice, C.st));
    WRI_HIP(hipMemcpyAsync(C.ws + rs.off_colmap, colmap.data(), colmap.size() * 4, hipMemcpyHostToDevice, C.st));
    WRI_HIP(hipMemcpyAsync(C.ws + rs.off_entries, entries.data(), entries.size() * 4, hipMemcpyHostToDevice, C.st));
    // the host vectors die at scope exit: make the copies complete first
    WRI_HIP(hipStreamSynchronize(C.st));
  }
  return WRI_OK;
}

int read_states(Ctx& C, std::vector<SysState>& hs) {
  hs.resize(C.n_sys);
  if (C.n_sys == 0) return WRI_OK;
  WRI_HIP(hipMemcpyAsync(hs.data(), C.dstate, sizeof(SysState) * C.n_sys, hipMemcpyDeviceToHost, C.st));
  WRI_HIP(hipStreamSynchronize(C.st));
  return WRI_OK;
}

// one CGLS iteration (fwd then adj) for every group
struct EventPool {
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  ~EventPool() { for (auto e : ev) (void)hipEventDestroy(e); }
  hipEvent_t next() {
    if (used == ev.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      ev.push_back(e);
    }
    return ev[used++];
  }
};

// One tile shape for every group: per-group tile counts and the device table
// that maps a block of a fused launch to (group, system, tile).
int set_config(Ctx& C, const TileCfg& cfg) {
  C.tiling.resize(C.groups.size());
  C.hgd.resize(C.groups.size());
  int b0 = 0;
  for (size_t gi = 0; gi < C.groups.size(); ++gi) {
    const wri_grid& g = C.grids[C.groups[gi].grid];
    const Tiling t = make_tiling(cfg, g);
    // each system has max_tiles(g) partial-sum slots (the layout's count)
    if (!cfg_supported(cfg) || t.ntiles() > max_tiles(g))
      return fail(WRI_EINVAL, "tile w=%d ry=%d tz=%d pf=%d: %d tiles per system, %d partial slots", cfg.w, cfg.ry,
                  cfg.tz, cfg.pf, t.ntiles(), max_tiles(g));
    C.tiling[gi] = t;
    GroupDesc& d = C.hgd[gi];
    d.rhs0 = C.groups[gi].rhs0;
    d.nrhs = C.groups[gi].nrhs;
    d.tiles_x = t.tx;
    d.tiles_y = t.ty;
    d.tz = cfg.tz;
    d.ntiles = t.ntiles();
    d.block0 = b0;
    d.tile_major = cfg.order;
    b0 += d.nrhs * d.ntiles;
  }
  C.nblocks = b0;
  // XCD chunk: half of the largest system's tiles, and at least 16 workgroups.
  // Measured on the 48-system 128^3 batch (whole solves): with the 64 x 16 x 32
  // tile (64 tiles per system) halves 18.20 solves/s, whole systems 18.15,
  // eighths 18.06, sixteenths 17.58 -- smaller chunks balance the convergence
  // tail better but lose more halo rows to other XCDs' L2; with the 64 x 32 x 64
  // tile (16 tiles per system) chunks of 8, 16 and 32 workgroups took 2.424,
  // 2.399 and 2.401 s per evaluation.
  constexpr int kMinXChunk = 16;
  int tmax = 1;
  for (const auto& d : C.hgd) tmax = std::max(tmax, d.ntiles);
  for (auto& d : C.hgd) d.xchunk = std::max(kMinXChunk, tmax / 2);
  if (!C.hgd.empty()) {
    WRI_HIP(hipMemcpyAsync(C.dgd, C.hgd.data(), sizeof(GroupDesc) * C.hgd.size(), hipMemcpyHostToDevice, C.st));
    WRI_HIP(hipStreamSynchronize(C.st));  // C.hgd may change before an asynchronous copy would finish
  }
  return WRI_OK;
}

const TileCfg& cur_cfg(const Ctx& C) { return C.tiling.front().cfg; }

// the tile counts of t fit every group's partial-sum slots
bool tiles_fit(const Ctx& C, const TileCfg& t) {
  for (const auto& G : C.groups)
    if (make_tiling(t, C.grids[G.grid]).ntiles() > max_tiles(C.grids[G.grid])) return false;
  return true;
}

// Convergence tail.  Once few systems still iterate, the tiling tuned for the
// full batch leaves compute units idle, or ends every launch with a partly
// filled round of workgroups.  At every chunk boundary the solve takes the
// z-slab of the tuned tile's shape (the tuned slab, halved down to 16 planes)
// with the least modelled time for the systems still iterating,
//   rounds x planes,  rounds = ceil(workgroups / resident workgroups of the
//   chip),  planes = min(slab, nz) + 2
// (the adjoint pass forms t one plane beyond each face of its slab; the chip
// holds compute units x the adjoint kernel's resident workgroups per unit).
// Measured steady state, 128^3 workload, 64 x 32 tile, ms per iteration for
// slabs of 64 / 32 / 16 planes: 48 systems 1.496 / 1.500 / 1.602, 24 systems
// 0.881 / 0.774 / 0.811, 16 systems 0.511 / 0.521 / 0.564, 12 systems 0.459 /
// 0.467 / 0.417, 8 systems 0.424 / 0.279 / 0.290, 4 systems 0.385 / 0.235 /
// 0.163; the model picks the fastest slab in each row.  Only for a
// recomputed-t tile chosen by the autotuner; WRI_TAIL_UNITS sets the chip's
// resident workgroups and applies the model to a forced tile too, and
// WRI_TAIL_TILE ("w,ry,tz,pf[,order]", or "0" for no switch) instead asks for
// one switch to that tile once at most WRI_TAIL_CELLS cells (default 2^25)
// still iterate (tests, experiments).
constexpr int kTailTZ = 16;
constexpr int kTailFacePlanes = 2;
struct TailPlan {
  int kind = 0;              // 0: none; 1: one switch to tile (WRI_TAIL_TILE); 2: slab by the model
  TileCfg tile{0, 0, 0, 0, 0};
  int64_t max_cells = 0;     // kind 1
  int64_t units = 0;         // kind 2: resident workgroups of the chip
  int full_tz = 0;           // kind 2: the model's slab for the whole batch
};

// The slab of P.tile's shape with the least modelled time for the systems
// flagged in active (ties keep the longer slab).
int model_tz(const Ctx& C, const TailPlan& P, const std::vector<char>& active) {
  int best_tz = P.tile.tz;
  double best_cost = -1.0;
  for (int tz = P.tile.tz; tz >= kTailTZ; tz /= 2) {
    TileCfg t = P.tile;
    t.tz = tz;
    if (!cfg_supported(t) || !tiles_fit(C, t)) continue;
    int64_t blocks = 0;
    int planes = 0;
    for (int p = 0; p < C.n_sys; ++p) {
      if (!active[p]) continue;
      const wri_grid& g = C.grids[C.sys[C.L.order[p]].grid];
      blocks += make_tiling(t, g).ntiles();
      planes = std::max(planes, std::min(tz, g.nz) + kTailFacePlanes);
    }
    const double cost = (double)((blocks + P.units - 1) / P.units) * planes;
    if (best_cost < 0.0 || cost < best_cost) {
      best_cost = cost;
      best_tz = tz;
    }
  }
  return best_tz;
}

TailPlan tail_plan(const Ctx& C, const TileCfg& main, bool forced_main) {
  TailPlan P;
  const char* e = getenv("WRI_TAIL_TILE");
  if (e != nullptr && *e) {
    if (*e == '0') return P;
    TileCfg t{0, 0, 0, 0, 0};
    const int got = sscanf(e, "%d,%d,%d,%d,%d", &t.w, &t.ry, &t.tz, &t.pf, &t.order);
    if (got < 4 || !cfg_supported(t)) return P;
    if (got == 4) t.order = 0;
    if (!tiles_fit(C, t)) return P;
    // t is produced and consumed within one iteration, so any march may follow
    P.kind = 1;
    P.tile = t;
    P.max_cells = (int64_t)1 << 25;
    if (const char* c = getenv("WRI_TAIL_CELLS"); c != nullptr && *c) P.max_cells = atoll(c);
    return P;
  }
  const char* u = getenv("WRI_TAIL_UNITS");
  const bool u_set = u != nullptr && *u;
  if ((forced_main && !u_set) || main.pf < 2 || main.tz <= kTailTZ) return P;
  int64_t units = 0;
  if (u_set) {
    units = atoll(u);
  } else {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, C.dev) != hipSuccess) return P;
    units = (int64_t)cus * adj_blocks_per_cu(main);
  }
  if (units <= 0) return P;
  P.kind = 2;
  P.tile = main;
  P.units = units;
  P.full_tz = model_tz(C, P, std::vector<char>(C.n_sys, 1));
  return P;
}

// Plan kind 2: the tile for the systems still iterating.  The tuned slab stays
// while the model picks for them what it picks for the whole batch (the
// autotuner measured the whole batch; the model only tracks the change).
TileCfg tail_tile(const Ctx& C, const std::vector<SysState>& hs, const TailPlan& P) {
  std::vector<char> active(C.n_sys);
  for (int p = 0; p < C.n_sys; ++p) active[p] = hs[p].status == kActive;
  TileCfg t = P.tile;
  const int tz = model_tz(C, P, active);
  if (tz != P.full_tz) t.tz = tz;
  return t;
}

// Switch the tiling between two iterations: the new group table, then the
// partials of ||s||^2 that the next forward launch reads folded to the new tile
// count.
int switch_tiling(Ctx& C, const TileCfg& cfg) {
  std::vector<int> n_old(C.hgd.size());
  for (size_t gi = 0; gi < C.hgd.size(); ++gi) n_old[gi] = C.hgd[gi].ntiles;
  const int rc = set_config(C, cfg);
  if (rc != WRI_OK) return rc;
  for (size_t gi = 0; gi < C.hgd.size(); ++gi)
    WRI_HIP(launch_fold_partials(C.dsys, C.part_s, C.hgd[gi].rhs0, C.hgd[gi].nrhs, n_old[gi], C.hgd[gi].ntiles, C.st));
  return WRI_OK;
}

// eager iteration with an event pair around the forward and adjoint launches
int launch_iteration_timed(Ctx& C, int k, EventPool& pool, std::vector<std::pair<hipEvent_t, hipEvent_t>>& fwd,
                           std::vector<std::pair<hipEvent_t, hipEvent_t>>& adj) {
  for (int phase = 0; phase < 2; ++phase) {
    hipEvent_t a = pool.next(), b = pool.next();
    if (!a || !b) return fail(WRI_EHIP, "hipEventCreate failed");
    WRI_HIP(hipEventRecord(a, C.st));
    if (phase == 0)
      WRI_HIP(launch_fwd(cur_cfg(C), C.dsys, C.dstate, C.part_s, C.part_d, C.dgd, (int)C.hgd.size(), C.nblocks, k,
                         C.st));
    else
      WRI_HIP(launch_adj(cur_cfg(C), C.dsys, C.dstate, C.part_d, C.part_s, C.dgd, (int)C.hgd.size(), C.nblocks, C.st));
    WRI_HIP(hipEventRecord(b, C.st));
    (phase == 0 ? fwd : adj).emplace_back(a, b);
  }
  return WRI_OK;
}

// CGLS iteration k: the forward launch then the adjoint launch, each over all groups
int launch_iteration(Ctx& C, int k, hipStream_t s) {
  WRI_HIP(launch_fwd(cur_cfg(C), C.dsys, C.dstate, C.part_s, C.part_d, C.dgd, (int)C.hgd.size(), C.nblocks, k, s));
  WRI_HIP(launch_adj(cur_cfg(C), C.dsys, C.dstate, C.part_d, C.part_s, C.dgd, (int)C.hgd.size(), C.nblocks, s));
  return WRI_OK;
}

int launch_setup(Ctx& C) {
  WRI_HIP(launch_init(C.dsys, C.dstate, C.n_sys, C.st, 0, (C.flags & WRI_FLAG_ADJOINT_SOURCE) ? 1 : 0));
  WRI_HIP(launch_adj(cur_cfg(C), C.dsys, C.dstate, C.part_d, C.part_s, C.dgd, (int)C.hgd.size(), C.nblocks, C.st));
  return WRI_OK;
}

// Warm start (WRI_FLAG_WARM_START): x holds x0.  S^H b gives the reference
// ||S^H b||^2, then r = b - S x0 and s0 = S^H r.
int launch_setup_warm(Ctx& C) {
  WRI_HIP(launch_init(C.dsys, C.dstate, C.n_sys, C.st, 1));
  WRI_HIP(launch_adj(cur_cfg(C), C.dsys, C.dstate, C.part_d, C.part_s, C.dgd, (int)C.hgd.size(), C.nblocks, C.st));
  std::vector<int32_t> np(C.n_sys);
  for (size_t gi = 0; gi < C.hgd.size(); ++gi)
    for (int r = 0; r < C.hgd[gi].nrhs; ++r) np[C.hgd[gi].rhs0 + r] = C.hgd[gi].ntiles;
  int32_t* dnp = at<int32_t>(C.ws, C.L.off_nparts);
  WRI_HIP(hipMemcpyAsync(dnp, np.data(), sizeof(int32_t) * np.size(), hipMemcpyHostToDevice, C.st));
  WRI_HIP(launch_warm_residual(C.dsys, C.dstate, C.part_s, dnp, C.n_sys, C.st));
  WRI_HIP(launch_adj(cur_cfg(C), C.dsys, C.dstate, C.part_d, C.part_s, C.dgd, (int)C.hgd.size(), C.nblocks, C.st));
  WRI_HIP(hipStreamSynchronize(C.st));  // np is host memory
  return WRI_OK;
}

bool verbose() {
  static const bool v = [] { const char* e = getenv("WRI_VERBOSE"); return e && *e && *e != '0'; }();
  return v;
}

// WRI_TILE="w,ry,tz,pf[,order]" forces a tile (tests, experiments): any
// supported shape whose tile count fits the partial-sum slots of every grid
bool forced_tile(const Ctx& C, TileCfg* out) {
  const char* e = getenv("WRI_TILE");
  if (e == nullptr || *e == 0) return false;
  TileCfg t{0, 0, 0, 0, 0};
  const int got = sscanf(e, "%d,%d,%d,%d,%d", &t.w, &t.ry, &t.tz, &t.pf, &t.order);
  if (got < 4 || !cfg_supported(t)) return false;
  if (got == 4) t.order = 0;
  if (!tiles_fit(C, t)) return false;
  *out = t;
  return true;
}

// Time a few real iterations of the whole batch per candidate tile shape and
// keep the fastest; cached per (device, mode, grid shapes and system counts).
int autotune(Ctx& C) {
  std::string key;
  int64_t total = 0;
  {
    char buf[96];
    snprintf(buf, sizeof(buf), "%d|%d|", C.dev, C.mode);
    key = buf;
    for (const auto& G : C.groups) {
      const wri_grid& g = C.grids[G.grid];
      snprintf(buf, sizeof(buf), "%dx%dx%d:%d;", g.nx, g.ny, g.nz, G.nrhs);
      key += buf;
      total += cells(g) * G.nrhs;
    }
  }
  auto it = g_tuned.find(key);
  if (it != g_tuned.end()) return set_config(C, it->second);
  if (total < (int64_t)64 * 64 * 64) {  // too small for the choice to matter
    g_tuned[key] = kCands[0];
    return set_config(C, kCands[0]);
  }
  hipEvent_t e0, e1;
  WRI_HIP(hipEventCreate(&e0));
  WRI_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  TileCfg best_cfg = kCands[0];
  for (int c = 0; c < kNumCands; ++c) {
    int rc = set_config(C, kCands[c]);
    if (rc == WRI_OK) rc = launch_setup(C);
    if (rc == WRI_OK) rc = launch_iteration(C, 0, C.st);  // warm
    if (rc != WRI_OK) return rc;
    WRI_HIP(hipEventRecord(e0, C.st));
    for (int it2 = 1; it2 <= 4 && rc == WRI_OK; ++it2) rc = launch_iteration(C, it2, C.st);
    if (rc != WRI_OK) return rc;
    WRI_HIP(hipEventRecord(e1, C.st));
    WRI_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    WRI_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (verbose())
      fprintf(stderr, "[wri] autotune %s w=%d ry=%d tz=%d pf=%d order=%d -> %.3f ms / 4 iterations\n",
              key.c_str(), kCands[c].w, kCands[c].ry, kCands[c].tz, kCands[c].pf, kCands[c].order, ms);
    if (ms < best) { best = ms; best_cfg = kCands[c]; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  g_tuned[key] = best_cfg;
  return set_config(C, best_cfg);
}

// A captured chunk bakes in every kernel argument of its launches: the tile
// (template and grid size), the group count and the five table pointers.  The
// table pointers are workspace offsets that depend on every grid's cell count,
// the number of grids and the receiver sets, so two batches that share the
// workspace base and the tile can still place them differently; the key holds
// the pointers themselves, not only the base.
std::string graph_key(const Ctx& C, int64_t k0, int chunk) {
  std::string k;
  char buf[256];
  // the kernels of a chunk depend on k0 only through fwd_x_step(k0 + i)
  snprintf(buf, sizeof(buf), "%d|%d|%d|%d|", C.dev, chunk, (int)(k0 & 1), k0 >= 2 ? 1 : (int)k0);
  k += buf;
  snprintf(buf, sizeof(buf), "%p,%p,%p,%p,%p,%d|", (const void*)C.dsys, (const void*)C.dstate,
           (const void*)C.part_s, (const void*)C.part_d, (const void*)C.dgd, (int)C.hgd.size());
  k += buf;
  const TileCfg& c = cur_cfg(C);
  snprintf(buf, sizeof(buf), "%d,%d,%d,%d,%d,%d;", c.w, c.ry, c.tz, c.pf, c.order, C.nblocks);
  k += buf;
  for (const auto& d : C.hgd) {
    snprintf(buf, sizeof(buf), "%d,%d,%d,%d,%d,%d;", d.rhs0, d.nrhs, d.tiles_x, d.tiles_y, d.tz, d.block0);
    k += buf;
  }
  return k;
}

int get_graph(Ctx& C, int64_t k0, int chunk, hipGraphExec_t* out) {
  const std::string key = graph_key(C, k0, chunk);
  auto it = g_graphs.find(key);
  if (it != g_graphs.end()) { *out = it->second.exec; return WRI_OK; }
  hipStream_t cs = capture_stream(C.dev);
  if (cs == nullptr) return fail(WRI_EHIP, "cannot create the capture stream");
  GraphEntry e;
  WRI_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  int rc = WRI_OK;
  for (int i = 0; i < chunk && rc == WRI_OK; ++i) rc = launch_iteration(C, (int)(k0 + i), cs);
  hipGraph_t graph = nullptr;
  hipError_t ec = hipStreamEndCapture(cs, &graph);
  if (rc != WRI_OK) { if (graph) (void)hipGraphDestroy(graph); return rc; }
  if (ec != hipSuccess) return fail(WRI_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(ec));
  e.graph = graph;
  WRI_HIP(hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0));
  if (g_graphs.size() > 64) {  // bound the cache: drop everything (rare)
    for (auto& kv : g_graphs) { (void)hipGraphExecDestroy(kv.second.exec); (void)hipGraphDestroy(kv.second.graph); }
    g_graphs.clear();
  }
  g_graphs[key] = e;
  *out = e.exec;
  return WRI_OK;
}

// ---------------------------------------------------------------------------
// batched driver
// ---------------------------------------------------------------------------

int run_batched(Ctx& C, float* const* grad, std::vector<SysState>& hs) {
  const Layout& L = C.L;
  const bool warm = (C.flags & WRI_FLAG_WARM_START) != 0;
  C.hsys.resize(C.n_sys);
  // user_x = 1: x is the caller's u_out where given; 0: the workspace vector
  // (the autotuner of a warm start must not overwrite the initial guess)
  auto fill_tables = [&](bool user_x) {
    for (int p = 0; p < C.n_sys; ++p) {
      const int i = L.order[p];
      const wri_system& s = C.sys[i];
      const size_t vb = align_up(sizeof(float2) * (size_t)cells(C.grids[s.grid]));
      char* base = C.ws + L.off_vec[p];
      float2* v[7];
      for (int q = 0; q < 7; ++q) v[q] = reinterpret_cast<float2*>(base + q * vb);
      float2* x = (user_x && C.u_out != nullptr && C.u_out[i] != nullptr) ? reinterpret_cast<float2*>(C.u_out[i])
                                                                          : v[0];
      const size_t rb = align_up(sizeof(float2) * (size_t)s.n_rec);
      float2* r2 = reinterpret_cast<float2*>(C.ws + L.off_rvec[p]);
      float2* t2 = reinterpret_cast<float2*>(C.ws + L.off_rvec[p] + rb);
      fill_sysdev(C, p, C.hsys[p], x, v[1], v[2], v[3], v[4], v[5], v[6], r2, t2);
    }
  };
  fill_tables(!warm);
  // groups: consecutive processing slots on one grid
  C.groups.clear();
  for (int p = 0; p < C.n_sys; ++p) {
    const int g = C.sys[L.order[p]].grid;
    if (C.groups.empty() || C.groups.back().grid != g) C.groups.push_back({g, p, 0});
    C.groups.back().nrhs++;
  }

  TileCfg main_cfg = kCands[0];  // the tile of the full batch (reported by the timing)
  int n_switches = 0;            // tiling changes of the convergence tail
  if (C.n_sys > 0) {
    WRI_HIP(hipMemcpyAsync(C.dsys, C.hsys.data(), sizeof(SysDev) * C.n_sys, hipMemcpyHostToDevice, C.st));
    int rc = upload_receivers(C);
    if (rc != WRI_OK) return rc;
    TileCfg forced;
    const bool is_forced = forced_tile(C, &forced);
    if (is_forced) rc = set_config(C, forced);
    else if (!(C.flags & WRI_FLAG_NO_AUTOTUNE)) rc = autotune(C);
    else rc = set_config(C, kCands[0]);
    if (rc != WRI_OK) return rc;
    if (warm) {  // the tuned tile is known; now point x at the caller's initial guess
      fill_tables(true);
      WRI_HIP(hipMemcpyAsync(C.dsys, C.hsys.data(), sizeof(SysDev) * C.n_sys, hipMemcpyHostToDevice, C.st));
    }
    if (verbose())
      for (size_t gi = 0; gi < C.groups.size(); ++gi)
        fprintf(stderr, "[wri] grid %d (%d systems): tile w=%d ry=%d tz=%d pf=%d order=%d, %d tiles per system\n",
                C.groups[gi].grid, C.groups[gi].nrhs, C.tiling[gi].cfg.w, C.tiling[gi].cfg.ry, C.tiling[gi].cfg.tz,
                C.tiling[gi].cfg.pf, C.tiling[gi].cfg.order, C.tiling[gi].ntiles());
    rc = warm ? launch_setup_warm(C) : launch_setup(C);
    if (rc != WRI_OK) return rc;
    const bool timing = (C.flags & WRI_FLAG_TIMING) != 0;
    const bool use_graph = !(C.flags & WRI_FLAG_NO_GRAPH) && !timing;
    int chunk = 8;
    int64_t launched = 0;
    auto last_report = std::chrono::steady_clock::now();
    main_cfg = cur_cfg(C);
    TailPlan tail = tail_plan(C, main_cfg, is_forced);
    EventPool pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_fwd, ev_adj;
    if (timing) g_times = KernelTimes();
    while (true) {
      if (timing) {
        pool.used = 0;
        ev_fwd.clear();
        ev_adj.clear();
        for (int i = 0; i < chunk; ++i) {
          rc = launch_iteration_timed(C, (int)(launched + i), pool, ev_fwd, ev_adj);
          if (rc != WRI_OK) return rc;
        }
      } else if (use_graph) {
        hipGraphExec_t ex = nullptr;
        rc = get_graph(C, launched, chunk, &ex);
        if (rc != WRI_OK) return rc;
        WRI_HIP(hipGraphLaunch(ex, C.st));
      } else {
        for (int i = 0; i < chunk; ++i) {
          rc = launch_iteration(C, (int)(launched + i), C.st);
          if (rc != WRI_OK) return rc;
        }
      }
      const int64_t kstart = launched;
      launched += chunk;
      rc = read_states(C, hs);
      if (rc != WRI_OK) return rc;
      if (timing) {
        bool all_active = true;
        for (const auto& st : hs) all_active = all_active && (st.status == kActive);
        float ms = 0.f;
        wri_timing& T = g_times.t;
        // algorithmic bytes of each launch of the chunk: a system takes part in
        // launch k with full work while k < its final iteration count
        const int pf = cur_cfg(C).pf;
        for (int i = 0; i < chunk; ++i) {
          const int64_t k = kstart + i;
          double fb = 0.0, ab = 0.0;
          for (int p = 0; p < C.n_sys; ++p) {
            if (hs[p].status != kActive && hs[p].iters <= k) continue;
            const double n = (double)cells(C.grids[C.sys[L.order[p]].grid]);
            fb += n * (double)fwd_bytes_per_cell(k, pf);
            ab += n * (double)kAdjBytesPerCell;
          }
          T.fwd_bytes += fb;
          T.adj_bytes += ab;
          if (all_active) { T.fwd_bytes_full += fb; T.adj_bytes_full += ab; }
        }
        for (auto& e : ev_fwd) {
          WRI_HIP(hipEventElapsedTime(&ms, e.first, e.second));
          T.fwd_ms += ms;
          if (all_active) { T.fwd_ms_full += ms; T.fwd_launches_full++; }
        }
        for (auto& e : ev_adj) {
          WRI_HIP(hipEventElapsedTime(&ms, e.first, e.second));
          T.adj_ms += ms;
          if (all_active) { T.adj_ms_full += ms; T.adj_launches_full++; }
        }
        T.fwd_launches += (int64_t)ev_fwd.size();
        T.adj_launches += (int64_t)ev_adj.size();
      }
      bool active = false;
      int n_active = 0;
      for (const auto& s : hs) {
        active = active || (s.status == kActive);
        n_active += (s.status == kActive) ? 1 : 0;
      }
      if (verbose() && active) {  // progress of long solves, at most every 30 s
        const auto now = std::chrono::steady_clock::now();
        if (now - last_report > std::chrono::seconds(30)) {
          fprintf(stderr, "[wri] iteration %lld: %d of %d systems iterating\n", (long long)launched, n_active,
                  C.n_sys);
          last_report = now;
        }
      }
      if (!active) break;
      if (tail.kind == 1) {
        int64_t act_cells = 0;
        for (int p = 0; p < C.n_sys; ++p)
          if (hs[p].status == kActive) act_cells += cells(C.grids[C.sys[L.order[p]].grid]);
        if (act_cells <= tail.max_cells) {
          rc = switch_tiling(C, tail.tile);
          if (rc != WRI_OK) return rc;
          tail.kind = 0;
          ++n_switches;
          if (verbose())
            fprintf(stderr, "[wri] iteration %lld: %d systems (%lld cells) iterating, tile w=%d ry=%d tz=%d pf=%d order=%d\n",
                    (long long)launched, n_active, (long long)act_cells, tail.tile.w, tail.tile.ry, tail.tile.tz,
                    tail.tile.pf, tail.tile.order);
        }
      } else if (tail.kind == 2) {
        const TileCfg t = tail_tile(C, hs, tail);
        if (t.tz != cur_cfg(C).tz) {
          rc = switch_tiling(C, t);
          if (rc != WRI_OK) return rc;
          ++n_switches;
          if (verbose())
            fprintf(stderr, "[wri] iteration %lld: %d systems iterating, slab %d planes\n", (long long)launched,
                    n_active, t.tz);
        }
      }
      if (launched > (int64_t)C.max_iter + 2)
        return fail(WRI_EHIP, "internal: systems still active after max_iter+2 iterations");
      chunk = std::min(chunk * 2, 128);
    }
  }
  if (C.flags & WRI_FLAG_TIMING) {
    if (!C.tiling.empty()) {
      const TileCfg& c = main_cfg;
      g_times.t.tile_w = c.w; g_times.t.tile_ry = c.ry; g_times.t.tile_tz = c.tz;
      g_times.t.tile_pf = c.pf; g_times.t.tile_order = c.order;
    }
    g_times.t.tail_switches = n_switches;
    g_times.valid = true;
  }
  // objective partials and gradient, per grid
  for (int g = 0; g < C.n_grids; ++g) {
    const Group* G = nullptr;
    for (const auto& gg : C.groups)
      if (gg.grid == g) G = &gg;
    const int n = (int)cells(C.grids[g]);
    float* gp = (grad != nullptr) ? grad[g] : nullptr;
    if (G == nullptr) {
      if (gp) WRI_HIP(launch_zero_f32(gp, (size_t)n, C.st));
      continue;
    }
    WRI_HIP(launch_grad(C.dsys, C.dstate, G->rhs0, G->nrhs, n, gp, C.part_j, L.part_j_stride, 0, C.st));
    WRI_HIP(launch_finalize(C.dsys, C.dstate, C.part_j, grad_blocks(n), L.part_j_stride, G->rhs0, G->nrhs, C.st));
  }
  return read_states(C, hs);
}

// ---------------------------------------------------------------------------
// plain driver: one system at a time, unfused kernels, host-side scalars
// ---------------------------------------------------------------------------

int plain_dot(Ctx& C, const float2* v, int n, double* out) {
  WRI_HIP(launch_dot(v, n, C.dot, C.L.dot_nparts, C.st));
  WRI_HIP(launch_sum(C.dot, C.L.dot_nparts, out, C.st));
  return WRI_OK;
}

int run_plain(Ctx& C, float* const* grad, std::vector<SysState>& hs) {
  const Layout& L = C.L;
  const size_t vb = L.vec_bytes_plain;
  char* base = C.ws + L.off_vec[0];
  float2* xw = reinterpret_cast<float2*>(base);
  float2* rv = reinterpret_cast<float2*>(base + vb);
  float2* pv = reinterpret_cast<float2*>(base + 2 * vb);
  float2* sv = reinterpret_cast<float2*>(base + 3 * vb);
  float2* tv = reinterpret_cast<float2*>(base + 4 * vb);
  float2* r2 = reinterpret_cast<float2*>(C.ws + L.off_rvec[0]);
  float2* t2 = reinterpret_cast<float2*>(C.ws + L.off_rvec[0] + L.rvec_bytes_plain);
  double* res = C.dot + L.dot_nparts * 2;  // [0]=|t|^2 [1]=|t2|^2 [2]=|s|^2
  // tables in original order (processing order = identity); one system's
  // vectors at a time, r[0] == r[1] and p[0] == p[1]
  C.hsys.resize(C.n_sys);
  for (int i = 0; i < C.n_sys; ++i) C.L.order[i] = i;
  for (int i = 0; i < C.n_sys; ++i) {
    float2* x = (C.u_out != nullptr && C.u_out[i] != nullptr) ? reinterpret_cast<float2*>(C.u_out[i]) : xw;
    fill_sysdev(C, i, C.hsys[i], x, rv, rv, pv, pv, sv, tv, r2, t2);
  }
  if (C.n_sys > 0) {
    WRI_HIP(hipMemcpyAsync(C.dsys, C.hsys.data(), sizeof(SysDev) * C.n_sys, hipMemcpyHostToDevice, C.st));
    int rc = upload_receivers(C);
    if (rc != WRI_OK) return rc;
  }
  for (int g = 0; g < C.n_grids; ++g)
    if (grad != nullptr && grad[g] != nullptr) WRI_HIP(launch_zero_f32(grad[g], (size_t)cells(C.grids[g]), C.st));

  double hres[3];
  for (int i = 0; i < C.n_sys; ++i) {
    const SysDev& S = C.hsys[i];
    const int n = S.nx * S.ny * S.nz;
    const bool est = C.mode == WRI_ESTIMATE;
    const double c = S.alpha_c;
    WRI_HIP(launch_init(C.dsys + i, C.dstate + i, 1, C.st, 0,   // x = 0, r1 = b1, r2 = lambda d
                        (C.flags & WRI_FLAG_ADJOINT_SOURCE) ? 1 : 0));
    double sa_re = 0.0, sa_im = 0.0;
    // s = S^H r (wavefield rows on the device, source-weight row on the host)
    auto apply_SH = [&]() -> int {
      WRI_HIP(launch_apply(S.nx, S.ny, S.nz, S.nb, S.h2inv_d, S.sp_scale_d, S.inv_nb_d, S.omega_d, S.m, rv, sv, 1,
                           -1, make_double2(0.0, 0.0), C.st));
      WRI_HIP(launch_scatter(sv, r2, S.rec, S.n_rec, S.lam_d, C.st));
      int rc = plain_dot(C, sv, n, res + 2);
      if (rc != WRI_OK) return rc;
      WRI_HIP(hipMemcpyAsync(hres + 2, res + 2, sizeof(double), hipMemcpyDeviceToHost, C.st));
      float2 r1s;
      WRI_HIP(hipMemcpyAsync(&r1s, rv + S.src, sizeof(float2), hipMemcpyDeviceToHost, C.st));
      WRI_HIP(hipStreamSynchronize(C.st));
      sa_re = est ? -c * (double)r1s.x : 0.0;
      sa_im = est ? -c * (double)r1s.y : 0.0;
      return WRI_OK;
    };
    int rc = apply_SH();
    if (rc != WRI_OK) return rc;
    double gamma = hres[2] + sa_re * sa_re + sa_im * sa_im;
    const double gamma0 = gamma;
    WRI_HIP(launch_copy_f2(pv, sv, n, C.st));
    double pa_re = sa_re, pa_im = sa_im, xa_re = 0.0, xa_im = 0.0;
    int k = 0, status = kActive;
    while (true) {
      if (gamma0 == 0.0) { status = kZeroRhs; break; }
      if (gamma <= S.rtol2 * gamma0) { status = kConverged; break; }
      if (k >= C.max_iter) { status = kMaxIter; break; }
      // t = S p
      WRI_HIP(launch_apply(S.nx, S.ny, S.nz, S.nb, S.h2inv_d, S.sp_scale_d, S.inv_nb_d, S.omega_d, S.m, pv, tv, 0,
                           est ? S.src : -1, make_double2(c * pa_re, c * pa_im), C.st));
      WRI_HIP(launch_gather(t2, pv, S.rec, S.n_rec, S.lam_d, C.st));
      rc = plain_dot(C, tv, n, res + 0);
      if (rc != WRI_OK) return rc;
      if (S.n_rec > 0) {
        rc = plain_dot(C, t2, S.n_rec, res + 1);
        if (rc != WRI_OK) return rc;
      }
      WRI_HIP(hipMemcpyAsync(hres, res, 2 * sizeof(double), hipMemcpyDeviceToHost, C.st));
      WRI_HIP(hipStreamSynchronize(C.st));
      const double delta = hres[0] + (S.n_rec > 0 ? hres[1] : 0.0);
      if (!(delta > 0.0) || !std::isfinite(delta) || !std::isfinite(gamma)) { status = kBreakdown; break; }
      const double a = gamma / delta;
      WRI_HIP(launch_axpy(S.x, pv, a, n, C.st));
      WRI_HIP(launch_axpy(rv, tv, -a, n, C.st));
      WRI_HIP(launch_axpy(r2, t2, -a, S.n_rec, C.st));
      xa_re += a * pa_re;
      xa_im += a * pa_im;
      rc = apply_SH();
      if (rc != WRI_OK) return rc;
      const double gnew = hres[2] + sa_re * sa_re + sa_im * sa_im;
      const double beta = gnew / gamma;
      gamma = gnew;
      WRI_HIP(launch_xpby(pv, sv, beta, n, C.st));
      pa_re = sa_re + beta * pa_re;
      pa_im = sa_im + beta * pa_im;
      ++k;
    }
    WRI_HIP(launch_set_state(C.dstate, i, k, status, make_double2(xa_re, xa_im), gamma, gamma0, C.st));
    const int g = C.sys[i].grid;
    float* gp = (grad != nullptr) ? grad[g] : nullptr;
    if (status != kBreakdown) {
      WRI_HIP(launch_grad(C.dsys, C.dstate, i, 1, n, gp, C.part_j, L.part_j_stride, 1, C.st));
      WRI_HIP(launch_finalize(C.dsys, C.dstate, C.part_j, grad_blocks(n), L.part_j_stride, i, 1, C.st));
    }
  }
  return read_states(C, hs);
}

// ---------------------------------------------------------------------------
// common entry
// ---------------------------------------------------------------------------

int solve_common(const wri_grid* grids, int32_t n_grids, const float* const* m, const wri_system* sys,
                 int32_t n_sys, int32_t mode, int32_t max_iter, int32_t flags, wri_c32* const* u_out,
                 wri_result* res, void* ws, size_t ws_bytes, void* stream, float* const* grad, double* J_out,
                 wri_c64* alpha_out) {
  int rc = validate(grids, n_grids, sys, n_sys, mode, max_iter);
  if (rc != WRI_OK) return rc;
  if (n_sys > 0 && res == nullptr) return fail(WRI_EINVAL, "res is NULL");
  if (m == nullptr && n_grids > 0) return fail(WRI_EINVAL, "m is NULL");
  for (int g = 0; g < n_grids; ++g)
    if (m[g] == nullptr) return fail(WRI_EINVAL, "m[%d] is NULL", g);
  if (grad != nullptr)
    for (int g = 0; g < n_grids; ++g)
      if (grad[g] == nullptr) return fail(WRI_EINVAL, "grad[%d] is NULL", g);
  if (flags & WRI_FLAG_WARM_START) {
    if (flags & WRI_FLAG_PLAIN) return fail(WRI_EINVAL, "WRI_FLAG_WARM_START is for the batched path only");
    if (n_sys > 0 && u_out == nullptr) return fail(WRI_EINVAL, "WRI_FLAG_WARM_START needs u_out (the initial guess)");
    for (int i = 0; i < n_sys; ++i)
      if (u_out[i] == nullptr) return fail(WRI_EINVAL, "WRI_FLAG_WARM_START: u_out[%d] is NULL", i);
  }
  if (flags & WRI_FLAG_ADJOINT_SOURCE) {
    if (mode != WRI_KNOWN) return fail(WRI_EINVAL, "WRI_FLAG_ADJOINT_SOURCE needs WRI_KNOWN");
    if (flags & WRI_FLAG_WARM_START) return fail(WRI_EINVAL, "WRI_FLAG_ADJOINT_SOURCE with WRI_FLAG_WARM_START");
    for (int i = 0; i < n_sys; ++i)
      if (sys[i].lambda != 0.0) return fail(WRI_EINVAL, "WRI_FLAG_ADJOINT_SOURCE: system %d has lambda != 0", i);
  }
  Ctx C;
  C.grids = grids; C.n_grids = n_grids; C.m = m; C.sys = sys; C.n_sys = n_sys;
  C.mode = mode; C.max_iter = max_iter; C.flags = flags; C.u_out = u_out;
  C.st = reinterpret_cast<hipStream_t>(stream);
  C.L = make_layout(grids, n_grids, sys, n_sys, flags);
  if (ws == nullptr || ws_bytes < C.L.total)
    return fail(WRI_ENOWS, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, C.L.total);
  C.ws = reinterpret_cast<char*>(align_up(reinterpret_cast<uintptr_t>(ws)));
  C.dsys = at<SysDev>(C.ws, C.L.off_sysdev);
  C.dstate = at<SysState>(C.ws, C.L.off_state);
  C.part_d = at<double>(C.ws, C.L.off_part_d);
  C.part_s = at<double>(C.ws, C.L.off_part_s);
  C.part_j = at<double>(C.ws, C.L.off_part_j);
  C.dot = at<double>(C.ws, C.L.off_dot);
  C.dgd = at<GroupDesc>(C.ws, C.L.off_gdesc);
  std::lock_guard<std::mutex> lock(g_mutex);
  WRI_HIP(hipGetDevice(&C.dev));
  std::vector<SysState> hs;
  rc = (flags & WRI_FLAG_PLAIN) ? run_plain(C, grad, hs) : run_batched(C, grad, hs);
  if (rc != WRI_OK) return rc;
  // results (the state array is in processing order)
  std::vector<int> slot_of(n_sys);
  for (int p = 0; p < n_sys; ++p) slot_of[C.L.order[p]] = p;
  int ret = WRI_OK;
  double J = 0.0;
  for (int i = 0; i < n_sys; ++i) {
    const SysState& T = hs[slot_of[i]];
    wri_result& r = res[i];
    r.iters = T.iters;
    r.status = T.status;
    const int slot = slot_of[i];
    const double gk = (flags & WRI_FLAG_PLAIN) ? T.gamma[T.iters & 1] : T.gamma[T.iterA & 1];
    r.relres = (T.gamma0 > 0.0) ? std::sqrt(std::max(gk, 0.0) / T.gamma0) : 0.0;
    r.J = T.J;
    if (mode == WRI_ESTIMATE) {
      const double c = C.hsys[(flags & WRI_FLAG_PLAIN) ? i : slot].alpha_c;
      r.alpha.re = c * T.xa.x; r.alpha.im = c * T.xa.y;
      r.alpha_ls.re = T.alpha_ls.x; r.alpha_ls.im = T.alpha_ls.y;
    } else {
      r.alpha = sys[i].alpha;
      r.alpha_ls = sys[i].alpha;
    }
    if (alpha_out) alpha_out[i] = r.alpha_ls;
    J += T.J;
    if (T.status == kBreakdown) ret = WRI_EBREAKDOWN;
    else if ((T.status == kMaxIter || T.status == kDiverged) && ret == WRI_OK) ret = WRI_NOT_CONVERGED;
  }
  if (J_out) *J_out = J;
  if (ret == WRI_EBREAKDOWN) fail(WRI_EBREAKDOWN, "at least one system broke down (non-finite or non-positive curvature)");
  return ret;
}

// ---------------------------------------------------------------------------
// fixed device scratch of the entry point that allocates nothing
// ---------------------------------------------------------------------------

// The workspace of wri_solve_noalloc: a file-scope device array, one copy per
// device, held by the loaded code object until the process ends.  On the host
// the name `scratch` is only a stand-in symbol: every kernel argument and copy
// uses the per-device address that hipGetSymbolAddress returns.
constexpr size_t kNoAllocBytes = WRI_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_scratch_mutex;
std::map<int, char*> g_scratch_addr;  // device -> address of its copy of `scratch`

// Address of the current device's copy, looked up once per device (with that
// device current) on its first call.
int scratch_address(int dev, char** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  auto it = g_scratch_addr.find(dev);
  if (it != g_scratch_addr.end()) {
    *out = it->second;
    return WRI_OK;
  }
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr)
    return fail(WRI_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
  g_scratch_addr[dev] = static_cast<char*>(ptr);
  *out = static_cast<char*>(ptr);
  return WRI_OK;
}

}  // namespace

int report_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

}  // namespace wri

using namespace wri;

extern "C" {

size_t wri_workspace_bytes(const wri_grid* grids, int32_t n_grids, const wri_system* sys, int32_t n_sys,
                           int32_t mode, int32_t flags) {
  if (validate(grids, n_grids, sys, n_sys, mode, 0) != WRI_OK) return 0;
  return make_layout(grids, n_grids, sys, n_sys, flags).total;
}

int wri_validate(const wri_grid* grids, int32_t n_grids, const wri_system* sys, int32_t n_sys, int32_t mode,
                 int32_t max_iter) {
  return validate(grids, n_grids, sys, n_sys, mode, max_iter);
}

int wri_solve(const wri_grid* grids, int32_t n_grids, const float* const* m, const wri_system* sys, int32_t n_sys,
              int32_t mode, int32_t max_iter, int32_t flags, wri_c32* const* u_out, wri_result* res, void* ws,
              size_t ws_bytes, void* stream) {
  try {
    return solve_common(grids, n_grids, m, sys, n_sys, mode, max_iter, flags, u_out, res, ws, ws_bytes, stream,
                        nullptr, nullptr, nullptr);
  } catch (const std::exception& e) {
    return fail(WRI_EINVAL, "exception: %s", e.what());
  }
}

int wri_solve_noalloc(const wri_grid* grids, int32_t n_grids, const float* const* m, const wri_system* sys,
                      int32_t n_sys, int32_t mode, int32_t max_iter, int32_t flags, wri_c32* const* u_out,
                      wri_result* res, void* stream) {
  try {
    if (flags & WRI_FLAG_TIMING) return fail(WRI_EINVAL, "wri_solve_noalloc: WRI_FLAG_TIMING creates events");
    int rc = validate(grids, n_grids, sys, n_sys, mode, max_iter);
    if (rc != WRI_OK) return rc;
    const size_t need = make_layout(grids, n_grids, sys, n_sys, flags).total;
    if (need > kNoAllocBytes)
      return fail(WRI_ENOWS,
                  "wri_solve_noalloc: these systems need %zu bytes of workspace; the fixed scratch holds %zu "
                  "(call wri_solve with a workspace of wri_workspace_bytes())", need, kNoAllocBytes);
    int dev = 0;
    WRI_HIP(hipGetDevice(&dev));
    char* ws = nullptr;
    rc = scratch_address(dev, &ws);
    if (rc != WRI_OK) return rc;
    // eager launches on the caller's stream (graph instantiation and the
    // autotuner's events would allocate); the default tile unless WRI_TILE forces one
    return solve_common(grids, n_grids, m, sys, n_sys, mode, max_iter,
                        flags | WRI_FLAG_NO_GRAPH | WRI_FLAG_NO_AUTOTUNE, u_out, res, ws, kNoAllocBytes, stream,
                        nullptr, nullptr, nullptr);
  } catch (const std::exception& e) {
    return fail(WRI_EINVAL, "exception: %s", e.what());
  }
}

int wri_objective_grad(const wri_grid* grids, int32_t n_grids, const float* const* m, const wri_system* sys,
                       int32_t n_sys, int32_t mode, int32_t max_iter, int32_t flags, double* J_out,
                       float* const* grad, wri_c32* const* u_out, wri_result* res, void* ws, size_t ws_bytes,
                       void* stream) {
  if (J_out == nullptr) return fail(WRI_EINVAL, "J_out is NULL");
  if (grad == nullptr && n_grids > 0) return fail(WRI_EINVAL, "grad is NULL");
  try {
    return solve_common(grids, n_grids, m, sys, n_sys, mode, max_iter, flags, u_out, res, ws, ws_bytes, stream,
                        grad, J_out, nullptr);
  } catch (const std::exception& e) {
    return fail(WRI_EINVAL, "exception: %s", e.what());
  }
}

int estimate_source(const wri_grid* grids, int32_t n_grids, const float* const* m, const wri_system* sys,
                    int32_t n_sys, int32_t max_iter, int32_t flags, wri_c64* alpha_out, wri_c32* const* u_out,
                    wri_result* res, void* ws, size_t ws_bytes, void* stream) {
  if (alpha_out == nullptr && n_sys > 0) return fail(WRI_EINVAL, "alpha_out is NULL");
  try {
    return solve_common(grids, n_grids, m, sys, n_sys, WRI_ESTIMATE, max_iter, flags, u_out, res, ws, ws_bytes,
                        stream, nullptr, nullptr, alpha_out);
  } catch (const std::exception& e) {
    return fail(WRI_EINVAL, "exception: %s", e.what());
  }
}

int wri_apply_helmholtz(const wri_grid* grid, const float* m, double omega, const wri_c32* in, wri_c32* out,
                        int32_t adjoint, void* stream) {
  if (grid == nullptr || m == nullptr || in == nullptr || out == nullptr)
    return fail(WRI_EINVAL, "NULL argument");
  if (validate(grid, 1, nullptr, 0, WRI_KNOWN, 0) != WRI_OK) return WRI_EINVAL;
  if (!(omega >= 0.0) || !std::isfinite(omega)) return fail(WRI_EINVAL, "omega must be finite and >= 0");
  if ((const void*)in == (const void*)out) return fail(WRI_EINVAL, "in and out must be distinct");
  const wri_grid& g = *grid;
  double sp = 0.0, inb = 0.0;
  if (g.nb > 0) {
    const double d0 = 3.0 * g.v_ref * std::log(1000.0) / (2.0 * g.nb * g.h);
    sp = 2.0 * d0 / (g.v_ref * g.v_ref);
    inb = 1.0 / g.nb;
  }
  WRI_HIP(launch_apply(g.nx, g.ny, g.nz, g.nb, 1.0 / (g.h * g.h), sp, inb, omega, m,
                       reinterpret_cast<const float2*>(in), reinterpret_cast<float2*>(out), adjoint ? 1 : 0, -1,
                       make_double2(0.0, 0.0), reinterpret_cast<hipStream_t>(stream)));
  return WRI_OK;
}

const char* wri_strerror(int code) {
  switch (code) {
    case WRI_OK: return "ok";
    case WRI_NOT_CONVERGED: return "some system reached max_iter before its tolerance";
    case WRI_EINVAL: return "invalid argument";
    case WRI_ERANGE: return "cell index outside its grid";
    case WRI_EDUP: return "duplicate receiver index within a system";
    case WRI_ENOWS: return "workspace missing or too small";
    case WRI_EHIP: return "HIP runtime error";
    case WRI_EBREAKDOWN: return "CGLS breakdown (non-finite or non-positive curvature)";
    default: return "unknown error";
  }
}

const char* wri_last_error(void) { return g_last_error.c_str(); }

int wri_kernel_times(wri_timing* out) {
  if (!g_times.valid) return fail(WRI_EINVAL, "no WRI_FLAG_TIMING call has completed on this thread");
  if (out == nullptr) return fail(WRI_EINVAL, "out is NULL");
  *out = g_times.t;
  return WRI_OK;
}
int wri_version(void) { return 100; }

}  // extern "C"
