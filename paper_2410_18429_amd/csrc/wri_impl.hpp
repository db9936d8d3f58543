// Internal declarations shared by the HIP kernels (kernels.hip) and the host
// side of the library (capi.hip).  Not part of the public ABI (include/wri.h).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace wri {

// x-extent of a slab tile: one 64-wide wavefront spans a row of cells.
constexpr int kTX = 64;
// Workgroups are dispatched round-robin over the 8 XCDs of an MI355X.
constexpr int kXCD = 8;

// Per-system status while iterating (final values mirror WRI_SYS_*).
enum : int { kActive = -1, kConverged = 0, kMaxIter = 1, kBreakdown = 2, kZeroRhs = 3, kDiverged = 4 };
// The recurred ||S^H r_k||^2 growing this far above its running minimum means
// the float32 recurrences have lost the solution (tolerance below what the
// storage precision can resolve): stop instead of iterating on noise.
constexpr double kDivergeRatio = 1e8;

// Read-only description of one right-hand side, resident in device memory.
// All vectors of one system live on that system's grid (n = nx*ny*nz cells,
// x fastest); int32 indexing inside a grid, 64-bit base pointers per system.
struct SysDev {
  float2* x;          // u (the wavefield unknown)
  float2* r[2];       // PDE-row residual r1 = q - A u (+ alpha e), ping-pong
  float2* p[2];       // search direction, ping-pong
  float2* s;          // S^H r (wavefield rows)
  float2* t;          // S p (PDE rows)
  float2* r2;         // receiver-row residual lambda (d - P u), n_rec
  float2* t2;         // receiver rows of S p, n_rec
  const float* m;     // squared slowness of the grid
  const float2* d;    // observed data, n_rec
  const int2* colmap; // [ny*nx] (begin, end) into entries for each (x, y) column; null if n_rec == 0
  const int2* entries;// (z, receiver index q), sorted by z within a column
  const int* rec;     // receiver cell indices (n_rec), used by the unfused path
  int nx, ny, nz, nb;
  float h2inv;        // 1/h^2
  float sp_scale;     // 2 d0 / v_ref^2 (0 when nb == 0)
  float inv_nb;       // 1/nb (0 when nb == 0)
  float omega, omega2, lam;
  int src, n_rec;
  int mode, max_iter;
  double rtol2;
  double omega_d, h2inv_d, sp_scale_d, inv_nb_d, lam_d;  // float64 copies for the final kernels
  double2 alpha;      // KNOWN-mode source weight
  double alpha_c;     // ESTIMATE: the source column of S is -alpha_c e (unknown alpha/alpha_c)
  int slot_base;      // first partial-sum slot of this system
  int grid_id;
};

// Mutable per-system scalars (float64), updated only by the kernels.
// Fields written inside a launch are never read by another workgroup of the
// same launch (double-buffered by iteration parity or by kernel), so no
// grid-wide synchronisation is needed beyond kernel boundaries.
struct SysState {
  double gamma[2];    // ||s_k||^2 by iteration parity (written by the forward kernel)
  double gamma0;
  double gmin[2];     // running minimum of gamma by parity (written by the forward kernel)
  double a[2];        // step gamma_k / ||t_k||^2 by parity (written by the adjoint kernel)
  double2 xa, pa, sa; // source-weight components of x, p, s (ESTIMATE)
  double J;           // objective share of this system
  double2 alpha_ls;   // (A u)[src] (ESTIMATE) or the given weight (KNOWN)
  int iterA;          // iteration index read by the forward kernel
  int iterB;          // iteration index read by the adjoint kernel
  int status;         // kActive or final
  int iters;
  int brk;            // set by the adjoint kernel on a breakdown; the next pair of
                      // launches finishes x and records the status
  int warm;           // warm start: gamma0 holds ||S^H b||^2 from the set-up, not ||S^H r_0||^2
  int pad_[2];
};

struct TileCfg {
  int w;       // wavefronts per workgroup
  int ry;      // rows per wavefront  (tile height TY = w*ry)
  int tz;      // z-slab length
  int pf = 0;  // 1: software-pipelined z march (loads of plane z+2 in flight during plane z);
               // 2: pipelined, and the adjoint pass recomputes t = S p instead of reading it;
               // 3: as 2, with the adjoint pass's loads two planes ahead
  int order = 0;  // 1: tile-major block order (see GroupDesc::tile_major)
  int ty() const { return w * ry; }
};

// One group = the systems of one grid.  A fused launch covers every group:
// blocks [block0, block0 + nrhs*ntiles) belong to the group, ntiles =
// tiles_x*tiles_y*tiles_z slab tiles per system.
struct GroupDesc {
  int rhs0, nrhs;
  int tiles_x, tiles_y, tz;
  int ntiles;
  int block0;
  int tile_major;  // 1: consecutive blocks take the same tile of successive systems
                   //    (the tile of m is then read once per XCD for the whole group)
  int xchunk;      // tiles per XCD chunk (same value in every entry of a table)
};

// Records a failure for wri_last_error (thread-local) and returns code.
int report_error(int code, const char* fmt, ...);

// ---- launchers (kernels.hip) -------------------------------------------
// rhs_rec = 1: the PDE rows' right-hand side is P^H d (receiver sources) instead
// of alpha e (KNOWN mode with lambda = 0; the adjoint solve of reduced FWI).
hipError_t launch_init(const SysDev* sys, SysState* st, int nsys, hipStream_t s, int warm = 0, int rhs_rec = 0);
// Warm start, after a set-up adjoint pass on r = b: gamma0 = ||S^H b||^2 from the
// pass's partials (nparts per system), then r = b - S x0 (x0 = 0 when b = 0).
hipError_t launch_warm_residual(const SysDev* sys, SysState* st, const double* part_s, const int* nparts,
                                int nsys, hipStream_t s);
// Before the first forward launch of a new tiling: the ||s||^2 partials of the
// group's systems [rhs0, rhs0 + nrhs) folded from n_old tiles into slot 0,
// slots up to n_new cleared.
hipError_t launch_fold_partials(const SysDev* sys, double* part_s, int rhs0, int nrhs, int n_old, int n_new,
                                hipStream_t s);
// Fused CGLS launches over all groups (same tile shape c for all of them).
// k: the iteration every active system of the launch is at (systems of one
// call iterate in lockstep); selects the variant of the forward kernel that
// updates x (even k >= 2) or leaves it alone (odd k, k = 0).
inline bool fwd_x_step(int64_t k) { return k >= 2 && (k & 1) == 0; }
hipError_t launch_fwd(const TileCfg& c, const SysDev* sys, SysState* st, const double* part_s, double* part_d,
                      const GroupDesc* gd, int ngroups, int nblocks, int k, hipStream_t s);
hipError_t launch_adj(const TileCfg& c, const SysDev* sys, SysState* st, const double* part_d, double* part_s,
                      const GroupDesc* gd, int ngroups, int nblocks, hipStream_t s, int setup_only = 0);
hipError_t launch_grad(const SysDev* sys, SysState* st, int rhs0, int nrhs, int n, float* grad,
                       double* part_j, int stride, int accumulate, hipStream_t s);
hipError_t launch_finalize(const SysDev* sys, SysState* st, const double* part_j, int nparts,
                           int stride, int rhs0, int nrhs, hipStream_t s);
hipError_t launch_zero_f32(float* p, size_t n, hipStream_t s);
int grad_blocks(int n);
bool cfg_supported(const TileCfg& c);
// workgroups of the adjoint kernel of tile c resident on one compute unit (0 on error)
int adj_blocks_per_cu(const TileCfg& c);

// single-operator and unfused kernels (test hook and the plain baseline)
hipError_t launch_apply(int nx, int ny, int nz, int nb, double h2inv, double sp_scale, double inv_nb,
                        double omega, const float* m, const float2* in, float2* out, int adjoint, int src,
                        double2 src_sub, hipStream_t s);
hipError_t launch_gather(float2* t2, const float2* p, const int* rec, int n_rec, double lam, hipStream_t s);
hipError_t launch_scatter(float2* sv, const float2* r2, const int* rec, int n_rec, double lam, hipStream_t s);
hipError_t launch_dot(const float2* v, int n, double* part, int nparts, hipStream_t s);
hipError_t launch_sum(const double* part, int nparts, double* out, hipStream_t s);
hipError_t launch_axpy(float2* y, const float2* x, double a, int n, hipStream_t s);
hipError_t launch_xpby(float2* p, const float2* sv, double b, int n, hipStream_t s);
hipError_t launch_copy_f2(float2* dst, const float2* src, int n, hipStream_t s);
hipError_t launch_fill_f2(float2* dst, float2 v, int n, hipStream_t s);
hipError_t launch_scale_f2(float2* dst, const float2* src, float a, int n, hipStream_t s);
hipError_t launch_set_state(SysState* st, int rhs, int iters, int status, double2 xa, double gamma,
                            double gamma0, hipStream_t s);
int dot_parts(int n);

}  // namespace wri
