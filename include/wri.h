/*
 * wri.h — C ABI of the MI355X (gfx950) augmented-wavefield library.
 *
 * The library solves, for many (source i, frequency j) systems at once, the
 * data-augmented wavefield problem of wavefield reconstruction inversion
 * (paper: "3D Source free wavefield reconstruction inversion", eqs. ObjPen,
 * CmpctWRIobj/Sandb, SimpObj):
 *
 *     J_ij(u, a) = || A_j(m) u - a e_i ||^2 + lambda^2 || P_i u - d_ij ||^2
 *
 * A_j(m) = L_h + diag(omega_j^2 m - i omega_j b)  (text after eq. FWI):
 *   L_h  the 7-point second-order Laplacian with zero Dirichlet ghosts,
 *   m    squared slowness [s^2/m^2] (float32, one value per cell),
 *   b    an m-independent damping sponge of nb cells on every face:
 *        b = (2 d0 / v_ref^2) * sum_axes (delta_axis / nb)^2, delta_axis the
 *        distance (cells) into the sponge, d0 = 3 v_ref ln(1000) / (2 nb h).
 * P_i samples the receiver cells, e_i is the unit vector of the source cell.
 *
 * lambda here weights the DATA term (lambda = 1/lambda_paper; the paper's
 * f_2 equals lambda_paper^2 J / 2).
 *
 * Two modes:
 *   WRI_KNOWN    a = alpha given:   minimise over u; normal equations
 *                (A^H A + lambda^2 P^H P) u = A^H (alpha e) + lambda^2 P^H d.
 *   WRI_ESTIMATE a unknown (the paper's source-free / on-the-fly source
 *                estimate, eq. SimpObj): minimise over x = [u; a].
 * Both are solved by CGLS on S = [[A, -c e],[lambda P, 0]] with x = [u; a/c]
 * (KNOWN: S = [A; lambda P]) — the conjugate-gradient-on-the-normal-equations
 * reading of the paper's Algorithm 1 — from x0 = 0, stopping when
 * ||S^H r_k|| <= rtol ||S^H r_0||.  c = sqrt(42)/h^2 (the norm of a Laplacian
 * column) equilibrates the source column; c = 1 is the printed S (same
 * minimiser).
 * Vectors are stored as complex float32; the stencil and vector-update
 * arithmetic runs in float64 registers (one rounding per stored value); every
 * inner product, step scalar, the unknown source weight and the objective are
 * float64.
 *
 * Objective and gradient (eqs. VarObj2, VarG2): J = sum_ij J_ij at the
 * computed minimiser (from the CGLS recurred residuals r1 = q - A u and
 * r2 = lambda (d - P u)), and, because b does not depend on m,
 *     dJ/dm = sum_ij 2 omega_j^2 Re( conj(u_ij) * (A_j u_ij - a_ij e_i) ).
 *
 * Conventions shared by every entry point
 *   - Cell layout: x fastest, linear index (z*ny + y)*nx + x, z down.
 *   - Complex numbers are interleaved (re, im).
 *   - "device" pointers are HIP device memory owned by the caller; "host"
 *     pointers are ordinary host memory owned by the caller.  The library
 *     never frees caller memory.  Scratch comes from the caller's workspace
 *     (size from wri_workspace_bytes); the only library-global state is the
 *     tile autotune cache and cached HIP graphs (guarded by a mutex).
 *   - `stream` is a hipStream_t; all device work is ordered on it.  The
 *     solver entry points synchronise `stream` before returning (their
 *     per-system results are written to host memory).
 *   - Return value: 0 = OK; 1 = WRI_NOT_CONVERGED (some system stopped at
 *     max_iter, see results); < 0 = error.  Inputs are validated before any
 *     device work; on error nothing is launched and wri_last_error() gives a
 *     message (thread-local).  No C++ exception crosses this ABI.
 *   - Tiling: the batched solver times candidate slab tiles on the first call
 *     of each batch shape and caches the fastest.  As systems stop, a tuned
 *     recomputed-t tile changes its z-slab (the tuned one, halved down to 16
 *     planes) to the one with the least modelled time for the systems still
 *     iterating: rounds of workgroups on the chip times planes per slab
 *     (only the summation order of a float64 reduction changes).  Environment
 *     overrides, for tests and experiments: WRI_TILE="w,ry,tz,pf[,order]"
 *     forces a tile (any supported shape whose tile count fits the
 *     partial-sum slots; the slab then stays), WRI_TAIL_UNITS sets the chip's
 *     resident workgroups of the model (and applies it to a forced tile),
 *     WRI_TAIL_TILE (same form as WRI_TILE, or "0" for no change) asks instead
 *     for one switch to that tile once at most WRI_TAIL_CELLS cells (default
 *     2^25) still iterate; WRI_VERBOSE=1 prints the tiles, the slab changes
 *     and, every 30 s, the progress of long solves to stderr.
 */
#ifndef WRI_H
#define WRI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { float re, im; } wri_c32;
typedef struct { double re, im; } wri_c64;

/* One grid. nx*ny*nz < 2^31 cells and nx*ny <= 3728270 cells per x-y plane
 * (72 planes of complex64 addressable with 32-bit offsets); h > 0 [m]; nb >= 0 sponge cells;
 * v_ref > 0 [m/s] (sponge reference velocity; ignored when nb == 0). */
typedef struct {
  int32_t nx, ny, nz;
  int32_t nb;
  double  h;
  double  v_ref;
} wri_grid;

/* One (source, frequency) system = one right-hand side. */
typedef struct {
  int32_t        grid;    /* index into the grids array                         */
  int32_t        src;     /* linear cell index of the point source e_i          */
  double         omega;   /* angular frequency 2*pi*f [rad/s], >= 0             */
  double         lambda;  /* data weight (>= 0)                                 */
  double         rtol;    /* tolerance on ||S^H r_k|| / ||S^H r_0||, >= 0       */
  wri_c64        alpha;   /* source weight, used in WRI_KNOWN only              */
  int32_t        n_rec;   /* number of receivers (>= 0)                         */
  int32_t        _pad;
  const int32_t* rec;     /* HOST, n_rec distinct linear cell indices (P_i)     */
  const wri_c32* d;       /* DEVICE, n_rec observed data d_ij                   */
} wri_system;

/* Per-system results (host). */
typedef struct {
  int32_t iters;          /* CGLS iterations performed (S p products)           */
  int32_t status;         /* WRI_SYS_*                                          */
  double  relres;         /* recurred sqrt(gamma_k / gamma_0)                   */
  double  J;              /* ||r1||^2 + ||r2||^2 from the recurred residuals    */
  wri_c64 alpha;          /* source weight of the solution: KNOWN: the input;
                             ESTIMATE: the CGLS unknown                         */
  wri_c64 alpha_ls;       /* ESTIMATE: least-squares weight for the computed u,
                             (A u)[src] (the exact stationarity condition in a);
                             KNOWN: the input                                   */
} wri_result;

enum { WRI_KNOWN = 0, WRI_ESTIMATE = 1 };

enum {
  WRI_OK = 0,
  WRI_NOT_CONVERGED = 1,   /* some system stopped at max_iter or diverged          */
  WRI_EINVAL = -1,      /* bad argument (null pointer, size, mode, ...)       */
  WRI_ERANGE = -2,      /* a cell index (src or receiver) outside its grid    */
  WRI_EDUP = -3,        /* duplicate receiver indices within one system       */
  WRI_ENOWS = -4,       /* workspace missing or smaller than required         */
  WRI_EHIP = -5,        /* a HIP runtime call failed                          */
  WRI_EBREAKDOWN = -6   /* some system broke down (non-finite or <= 0 curvature) */
};

enum {
  WRI_SYS_CONVERGED = 0,
  WRI_SYS_MAX_ITER = 1,
  WRI_SYS_BREAKDOWN = 2,
  WRI_SYS_ZERO_RHS = 3,  /* S^H b = 0: the solution is x = 0, no iteration   */
  WRI_SYS_DIVERGED = 4   /* ||S^H r_k|| rose 1e4x above its running minimum: the
                            tolerance is below what float32 storage resolves;
                            the last iterate is returned                       */
};

/* flags (bitwise OR) */
enum {
  WRI_FLAG_PLAIN = 1,       /* one system at a time, unfused kernels, host-driven
                               scalars (the straightforward transcription of the
                               iterative solver; the baseline of the batched form) */
  WRI_FLAG_NO_GRAPH = 2,    /* launch the batched iterations eagerly (no hipGraph) */
  WRI_FLAG_NO_AUTOTUNE = 4, /* use the default slab tile instead of the tuned one */
  WRI_FLAG_UNSCALED_ALPHA = 8, /* ESTIMATE: use the source column -e exactly as printed
                               (default: -c e with c = sqrt(42)/h^2, same minimiser,
                               better-conditioned iteration) */
  WRI_FLAG_TIMING = 16,     /* launch the batched iterations eagerly with a HIP event
                               pair around every fused launch; totals via
                               wri_kernel_times() */
  WRI_FLAG_WARM_START = 32, /* batched path only: u_out (required, one pointer per
                               system) holds the initial wavefield on entry, and in
                               ESTIMATE mode sys[k].alpha the initial source weight.
                               CGLS starts from x0 = (u0, alpha0) with r0 = b - S x0;
                               the tolerance stays relative to ||S^H b|| (the
                               zero-start residual), so the result meets the same
                               rtol as a cold start.  u0 = 0 reproduces the cold
                               start bit for bit. */
  WRI_FLAG_ADJOINT_SOURCE = 64 /* WRI_KNOWN with lambda = 0 in every system: the
                               right-hand side of the PDE rows is P^H d — point
                               sources of strengths sys[k].d at the receiver cells —
                               instead of alpha e (src and alpha are not used).  u then
                               solves A u = P^H d; as A is complex symmetric,
                               conj(u) solves A^H v = P^H conj(d), the adjoint field of
                               reduced FWI (eqs. FWI, FWI2).  Not with WRI_FLAG_WARM_START. */
};

/* Workspace bytes needed by wri_solve / wri_objective_grad / estimate_source
 * for these systems (host-only computation; no device call).  Returns 0 and
 * sets wri_last_error() if the arguments are invalid. */
size_t wri_workspace_bytes(const wri_grid* grids, int32_t n_grids,
                           const wri_system* sys, int32_t n_sys,
                           int32_t mode, int32_t flags);

/* Validate arguments only (host-only; no device call).  Same checks and
 * return codes as the solver entry points. */
int wri_validate(const wri_grid* grids, int32_t n_grids,
                 const wri_system* sys, int32_t n_sys,
                 int32_t mode, int32_t max_iter);

/* Batched augmented solve (eq. SimpObj; paper's grouping of systems, eq.
 * Mmatrix2 read as block-diagonal).  All systems — any mix of sources,
 * frequencies and grids — iterate together; each stops at its own rtol.
 *   m[g]      DEVICE float32, n(g) squared slowness of grid g (n_grids pointers, host array)
 *   u_out     host array of n_sys DEVICE pointers (n(grid) complex each) receiving u,
 *             or NULL (u is then kept in the workspace only)
 *   res       HOST, n_sys results (required)
 *   ws        DEVICE workspace of ws_bytes >= wri_workspace_bytes(...) */
int wri_solve(const wri_grid* grids, int32_t n_grids, const float* const* m,
              const wri_system* sys, int32_t n_sys, int32_t mode, int32_t max_iter,
              int32_t flags, wri_c32* const* u_out, wri_result* res,
              void* ws, size_t ws_bytes, void* stream);

/* Size of the fixed device scratch that wri_solve_noalloc uses as its workspace. */
#define WRI_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* wri_solve for callers that cannot allocate device memory: code under HIP
 * graph capture, allocation-free serving loops, harnesses that forbid
 * hipMalloc.  Arguments and results as in wri_solve, without ws / ws_bytes.
 *   Workspace: a fixed scratch array of WRI_NOALLOC_SCRATCH_BYTES (64 MiB) in
 *   the library's device code, one copy per device, held from the library's
 *   first use on that device until the process ends.  The call allocates
 *   nothing (no hipMalloc/hipFree, no graph, no events): the iterations are
 *   launched eagerly on `stream` with the default slab tile (WRI_FLAG_NO_GRAPH
 *   and WRI_FLAG_NO_AUTOTUNE are implied; the WRI_TILE environment variable
 *   still forces a tile).
 *   Limit: systems whose wri_workspace_bytes() exceeds the scratch are
 *   rejected with WRI_ENOWS before any device work (e.g. up to about 8
 *   systems of 64^3 cells fit).  WRI_FLAG_TIMING is rejected (WRI_EINVAL).
 *   Sharing: every call on a device uses that device's one scratch and leaves
 *   its contents behind (the solver initialises everything it reads).  Calls
 *   that overlapped on one device would race on it; the library serialises
 *   its solver calls within a process and returns only after the device work
 *   of a call has finished. */
int wri_solve_noalloc(const wri_grid* grids, int32_t n_grids, const float* const* m,
                      const wri_system* sys, int32_t n_sys, int32_t mode, int32_t max_iter,
                      int32_t flags, wri_c32* const* u_out, wri_result* res, void* stream);

/* Objective and gradient in m (eqs. VarObj2, VarG2): runs the batched solve,
 * then writes
 *   J_out     HOST double, sum over systems of J_ij
 *   grad[g]   DEVICE float32 n(g): dJ/dm on grid g, summed over the systems on
 *             that grid (overwritten; grids without systems get zeros)
 *   u_out, res as in wri_solve (u_out may be NULL). */
int wri_objective_grad(const wri_grid* grids, int32_t n_grids, const float* const* m,
                       const wri_system* sys, int32_t n_sys, int32_t mode, int32_t max_iter,
                       int32_t flags, double* J_out, float* const* grad,
                       wri_c32* const* u_out, wri_result* res,
                       void* ws, size_t ws_bytes, void* stream);

/* On-the-fly source-weight estimate (section "3D Source free wavefield
 * reconstruction inversion", variable projection of eq. SimpObj): an
 * ESTIMATE-mode solve, then alpha_out[k] = (A u_k)[src_k] in float64 — the
 * weight that minimises J_k for the computed wavefield.
 *   alpha_out HOST, n_sys; u_out optional as in wri_solve. */
int estimate_source(const wri_grid* grids, int32_t n_grids, const float* const* m,
                    const wri_system* sys, int32_t n_sys, int32_t max_iter, int32_t flags,
                    wri_c64* alpha_out, wri_c32* const* u_out, wri_result* res,
                    void* ws, size_t ws_bytes, void* stream);

/* Single operator application (text after eq. FWI): out = A in (adjoint = 0)
 * or out = A^H in (adjoint = 1) on one grid.  in, out: DEVICE, n complex,
 * distinct buffers; m: DEVICE float32 n.  Uses the solver's stencil code. */
int wri_apply_helmholtz(const wri_grid* grid, const float* m, double omega,
                        const wri_c32* in, wri_c32* out, int32_t adjoint, void* stream);

/* ---- outer loop: source-free adaptive WRI with TV (section "SF-AWRI with
 * total variation regularization", eq. TVAWRI, Algorithm 2) ---------------- */

/* Smoothed isotropic total variation of a model on one grid:
 *   TV(m) = sum over cells of sqrt((D_x m)^2 + (D_y m)^2 + (D_z m)^2 + eps^2),
 * forward differences (D_x m)[i] = (m[i+1] - m[i]) / h, zero in the last cell
 * of every axis (the paper names the TV norm without defining it).
 *   m: DEVICE float32 n; value: HOST, TV(m) (float64 sums, fixed order);
 *   grad: DEVICE float32 n or NULL: grad += gamma * dTV/dm;
 *   ws: DEVICE workspace of wri_tv_workspace_bytes(grid) bytes.
 * Synchronises the stream (the value is host memory). */
size_t wri_tv_workspace_bytes(const wri_grid* grid);
int wri_tv(const wri_grid* grid, const float* m, double eps, double gamma, double* value, float* grad,
           void* ws, size_t ws_bytes, void* stream);

/* l-BFGS search direction dir = -H g (two-loop recursion; H_0 = h0 I, or, with
 * h0 <= 0 and at least one pair, s.y / y.y of the newest pair).
 *   g, dir: DEVICE float32 n (distinct); S, Y: DEVICE float32 [capacity][n]
 *   rings of curvature pairs s_i = m_{i+1} - m_i, y_i = g_{i+1} - g_i; the
 *   `count` pairs in use end at slot `newest` (older pairs in the slots
 *   before it, cyclically).  Dot products are float64.  Stream-ordered (no
 *   synchronisation).  ws: DEVICE, wri_lbfgs_workspace_bytes(capacity). */
size_t wri_lbfgs_workspace_bytes(int32_t capacity);
int wri_lbfgs_direction(int64_t n, const float* g, const float* S, const float* Y, int32_t capacity,
                        int32_t count, int32_t newest, double h0, float* dir, void* ws, size_t ws_bytes,
                        void* stream);

typedef struct {
  double  gamma;      /* TV weight: the loop minimises F(m) = J(m) + gamma TV(m), J as
                         returned by wri_objective_grad (the paper's f4 is
                         (lambda_p^2/2) J + gamma_p TV, i.e. gamma = 2 gamma_p / lambda_p^2) */
  double  eps_tv;     /* TV smoothing                                                       */
  double  eps0;       /* initial solver tolerance (relative normal residual, every system)  */
  double  eps_min;    /* a rejected trial that would halve eps below this ends the loop     */
  double  step0;      /* first step, before any curvature pair: max|dm| = step0 * max|m|    */
  double  max_step;   /* every step is scaled to max|dm| <= max_step * max|m| (0: no cap)   */
  double  m_min, m_max; /* bounds of the squared slowness (<= 0: none)                      */
  int32_t max_outer;  /* accepted model updates                                             */
  int32_t memory;     /* curvature pairs kept                                               */
  int32_t max_iter;   /* CGLS iteration cap per solve                                       */
  int32_t flags;      /* solver flags (WRI_FLAG_*)                                          */
  int32_t mask_sponge;/* 1: the damping layer is not updated (gradient zeroed there)        */
  int32_t warm_start; /* 1: every solve after the first starts from the wavefields and
                         source weights of the current model (WRI_FLAG_WARM_START).
                         Meant for a fixed tolerance (eps0 == eps_min): the value of a
                         CGLS iterate only falls along the iteration, so a trial begun
                         at the current wavefield passes the acceptance test almost
                         regardless of the step and the tolerance is rarely halved    */
} wri_awri_options;

enum { WRI_AWRI_EVAL = 0, WRI_AWRI_ACCEPTED = 1, WRI_AWRI_REJECTED = 2 };

typedef struct {
  double  F, J, tv;       /* F = J + gamma TV and its parts at the evaluated model       */
  double  eps;            /* solver tolerance of the evaluation                          */
  int32_t kind;           /* WRI_AWRI_EVAL: the current model (start, or again after eps
                             was halved); _ACCEPTED / _REJECTED: a trial model          */
  int32_t solver_iters;   /* CGLS iterations summed over the systems                     */
  double  seconds;        /* wall time of the evaluation (solves, gradient, TV)         */
} wri_awri_record;

/* Algorithm 2 on one grid: repeat { trial m~ = m - H g (l-BFGS; unit step,
 * optionally capped and clipped to the bounds); solve and evaluate F at m~
 * with tolerance eps; if F(m~) <= F(m) accept it, else halve eps, drop the
 * curvature pairs (formed at the looser tolerance) and evaluate F and g at m
 * again } until max_outer trials are accepted.  The values at an accepted
 * trial serve as the next iteration's F and g.
 *   m: DEVICE float32 n, the start model, overwritten with the result;
 *   sys: as for wri_objective_grad (every system's rtol is replaced by eps;
 *   all systems on grid 0); history: HOST, up to history_cap records, one per
 *   evaluation; *n_records: records produced (more than history_cap means the
 *   rest were not stored); ws: DEVICE, wri_awri_workspace_bytes(...).
 * Returns WRI_OK, or WRI_NOT_CONVERGED when the loop stopped at eps_min; the
 * errors of wri_objective_grad otherwise.  The workspace query takes the
 * solver flags; add WRI_FLAG_WARM_START to them when opt->warm_start is set
 * (two wavefield sets of n_sys systems are then part of the workspace). */
size_t wri_awri_workspace_bytes(const wri_grid* grid, const wri_system* sys, int32_t n_sys, int32_t mode,
                                int32_t flags, int32_t memory);
int wri_awri(const wri_grid* grid, float* m, const wri_system* sys, int32_t n_sys, int32_t mode,
             const wri_awri_options* opt, wri_awri_record* history, int32_t history_cap,
             int32_t* n_records, void* ws, size_t ws_bytes, void* stream);

/* ---- Reduced (conventional) FWI baseline: eqs. FWI, PDEsolve, FWI2 --------
 *
 *     f = 1/2 sum_ij || alpha_ij P_i A_j^{-1} e_i - d_ij ||^2
 *
 * the objective WRI relaxes (section "3D Source free wavefield reconstruction
 * inversion").  Per system: a forward solve A w = e (ESTIMATE) or
 * A u = alpha e (KNOWN), both by the batched solver with lambda = 0; in
 * ESTIMATE mode the weight that minimises the misfit for the current m,
 * alpha = (P w)^H d / ||P w||^2 (0 when P w = 0), and u = alpha w (float64);
 * the residual rho = P u - d; an adjoint solve A z = P^H conj(rho)
 * (WRI_FLAG_ADJOINT_SOURCE; v = conj(z) solves A^H v = P^H rho); and
 *     df/dm = - sum_ij omega_j^2 Re( conj(v) * u ) = - sum_ij omega_j^2 Re( z * u )
 * (dA/dm = omega^2 I; with alpha at its optimum the alpha-derivative
 * vanishes, so this is the gradient of the reduced function of m).
 * Both solves stop at sys[k].rtol; sys[k].lambda is not used. */
typedef struct {
  double  f;              /* this system's 1/2 || alpha P u - d ||^2 (float64)   */
  wri_c64 alpha;          /* KNOWN: the input weight; ESTIMATE: the estimate     */
  int32_t iters_fwd, iters_adj;    /* CGLS iterations of the two solves         */
  int32_t status_fwd, status_adj;  /* WRI_SYS_* of the two solves               */
} wri_fwi_result;

/* Workspace bytes of wri_fwi_objective_grad (host-only; 0 on invalid input):
 * the solver's workspace plus two wavefields per system (w and z). */
size_t wri_fwi_workspace_bytes(const wri_grid* grids, int32_t n_grids, const wri_system* sys, int32_t n_sys,
                               int32_t mode, int32_t flags);
/*   m[g]     DEVICE float32 n(g) per grid (host array of n_grids pointers)
 *   flags    WRI_FLAG_PLAIN / NO_GRAPH / NO_AUTOTUNE / TIMING (not WARM_START); with
 *            TIMING, wri_kernel_times() then reports the adjoint (last) solve
 *   f_out    HOST double: sum of the systems' f (required)
 *   grad     host array of n_grids DEVICE float32 pointers receiving df/dm
 *            (overwritten; zeros on grids without systems), or NULL
 *   u_out    host array of n_sys DEVICE pointers receiving u = alpha w, or NULL
 *   res      HOST, n_sys results (required when n_sys > 0)
 * Returns WRI_OK, WRI_NOT_CONVERGED when a solve stopped at max_iter or
 * diverged, WRI_EBREAKDOWN (results filled, gradient not computed), or the
 * validation errors of wri_solve. */
int wri_fwi_objective_grad(const wri_grid* grids, int32_t n_grids, const float* const* m, const wri_system* sys,
                           int32_t n_sys, int32_t mode, int32_t max_iter, int32_t flags, double* f_out,
                           float* const* grad, wri_c32* const* u_out, wri_fwi_result* res, void* ws,
                           size_t ws_bytes, void* stream);

/* ---- One model grid, per-frequency simulation grids --------------------
 *
 * Each frequency may be simulated on its own grid (a fixed number of points
 * per wavelength, as in the grouping of systems by frequency, eq. Mmatrix2)
 * while the inversion updates one model m on a model grid.  Every grid has
 * its cell (i, j, k) at (i h, j h, k h) — a common origin at cell 0 — and the
 * model grid must cover each simulation grid ((n_g - 1) h_g <= (n_m - 1) h_m
 * per axis) and be at most 6.5x coarser than it.  The map R_g from the
 * model grid to grid g is trilinear interpolation: per axis
 * xi = clamp(i h_g / h_m, 0, n_m - 1), i0 = min(floor(xi), n_m - 2),
 * weights (1 - t, t) on model cells (i0, i0 + 1), t = xi - i0 (an axis of one
 * model cell has weight 1); the 3-D weight is the product.  Arithmetic in
 * float64, values stored as float32.
 *
 * wri_model_to_grid:          m_grid = R_g m_model  (DEVICE float32 arrays)
 * wri_grid_to_model_adjoint:  g_model = R_g^T g_grid, or += when accumulate != 0
 *                             (a gather over model cells; deterministic)
 * Both are stream-ordered and do not synchronise; WRI_EINVAL on bad grids. */
int wri_model_to_grid(const wri_grid* model_grid, const float* m_model, const wri_grid* grid, float* m_grid,
                      void* stream);
int wri_grid_to_model_adjoint(const wri_grid* model_grid, const wri_grid* grid, const float* g_grid, float* g_model,
                              int32_t accumulate, void* stream);

/* Objective and gradient with the model on the model grid: m_g = R_g m_model
 * for every simulation grid, the batched solve and gradient of
 * wri_objective_grad on the simulation grids, then
 *     grad_model = sum_g R_g^T grad_g
 * (the chain rule through the interpolation).  grad_model: DEVICE float32 on
 * the model grid (overwritten), or NULL for the objective only.  Other
 * arguments and returns as wri_objective_grad; the workspace (from
 * wri_model_workspace_bytes) adds m_g and grad_g of every simulation grid to
 * the solver's. */
size_t wri_model_workspace_bytes(const wri_grid* model_grid, const wri_grid* grids, int32_t n_grids,
                                 const wri_system* sys, int32_t n_sys, int32_t mode, int32_t flags);
int wri_objective_grad_model(const wri_grid* model_grid, const float* m_model, const wri_grid* grids,
                             int32_t n_grids, const wri_system* sys, int32_t n_sys, int32_t mode, int32_t max_iter,
                             int32_t flags, double* J_out, float* grad_model, wri_c32* const* u_out, wri_result* res,
                             void* ws, size_t ws_bytes, void* stream);

/* ---- Sources and receivers off the grid nodes ---------------------------
 *
 * e and P of eq. ObjPen become trilinear interpolation at arbitrary points:
 * a point (x, y, z) [m] (cell (i, j, k) at (i h, j h, k h)) is clamped into
 * the grid and, per axis, xi = x / h, i0 = min(floor(xi), n - 2), weights
 * (1 - t, t) on (i0, i0 + 1), t = xi - i0 (an axis of one cell: weight 1 on
 * cell 0); the 3-D weights are products, duplicate cells merged and zero
 * weights dropped.  e = sum_k w_k e_{c_k}; row q of P holds receiver q's
 * weights.  Receivers may share cells.  In ESTIMATE mode the source column is
 * -c e and the least-squares weight of the result is
 * alpha_ls = e^H (A u) / e^H e.  The gradient keeps the form of eq. VarG2.
 *
 * All systems of a call iterate in lockstep, four launches per iteration
 * (forward pass, source/receiver rows and step, adjoint pass, rows and
 * beta), with the step scalars in device memory and chunks of iterations
 * replayed from a hipGraph (the fused kernels assume one cell per source and
 * receiver). */
typedef struct {
  double        src[3];  /* source position (x, y, z) [m]                           */
  const double* rec;     /* HOST, 3 * n_rec receiver positions (x, y, z) [m]        */
} wri_positions;

/* Workspace bytes (host-only; 0 on invalid input).  pos: n_sys entries. */
size_t wri_offgrid_workspace_bytes(const wri_grid* grids, int32_t n_grids, const wri_system* sys, int32_t n_sys,
                                   const wri_positions* pos);
/* As wri_objective_grad, with sys[k].src and sys[k].rec replaced by pos[k]
 * (sys[k].n_rec and sys[k].d still give the data).  grad may be NULL (a solve
 * only).  flags: WRI_FLAG_UNSCALED_ALPHA, WRI_FLAG_NO_GRAPH (launch every
 * chunk of iterations eagerly instead of replaying a hipGraph captured per set
 * of still-active systems); WRI_FLAG_WARM_START and WRI_FLAG_ADJOINT_SOURCE are
 * rejected, the others have no effect.  Positions
 * must be finite; points outside the grid are clamped onto its boundary. */
int wri_objective_grad_offgrid(const wri_grid* grids, int32_t n_grids, const float* const* m, const wri_system* sys,
                               int32_t n_sys, const wri_positions* pos, int32_t mode, int32_t max_iter,
                               int32_t flags, double* J_out, float* const* grad, wri_c32* const* u_out,
                               wri_result* res, void* ws, size_t ws_bytes, void* stream);

/* Kernel time of the last WRI_FLAG_TIMING call on this thread (HIP event
 * pairs around every fused launch; one launch covers every active system).
 * Bytes are algorithmic: per cell, forward 36 B with t stored, 28 B when the
 * adjoint pass recomputes t (+24 B for the x update on even iterations
 * k >= 2), adjoint 36 B; halo re-reads are not counted. */
typedef struct {
  double  fwd_ms, adj_ms;                /* summed durations of the fused launches       */
  int64_t fwd_launches, adj_launches;
  double  fwd_bytes, adj_bytes;          /* algorithmic bytes of those launches          */
  double  fwd_ms_full, adj_ms_full;      /* the launches during which every system was
                                            still iterating (whole batch resident)       */
  int64_t fwd_launches_full, adj_launches_full;
  double  fwd_bytes_full, adj_bytes_full;
  int32_t tile_w, tile_ry, tile_tz, tile_pf, tile_order; /* tile shape of the fused launches
                                                           (waves, rows per wave, z-slab,
                                                           march: 0 plain, 1 pipelined,
                                                           2 pipelined with t recomputed
                                                           in the adjoint pass, 3 as 2 with
                                                           two planes of prefetch; block
                                                           order)                        */
  int32_t tail_switches;                 /* changes of the tiling during the solve (the
                                            convergence tail, see Tiling above)          */
} wri_timing;

/* Fills *out; WRI_EINVAL if no timed call has completed on this thread. */
int wri_kernel_times(wri_timing* out);

/* Objective and gradient with the preconditioned CGLS (fewer CGLS
 * iterations).  Beyond the paper, whose only reducer of the iteration
 * count is the adaptive tolerance of Algorithm 2: S is preconditioned on the
 * right by one multigrid V(1,1) cycle of the complex-shifted Helmholtz
 * operator A_beta = L_h + diag(omega^2 (1 - i beta) m - i omega b), beta = 1/2
 * (damped Jacobi 0.7, trilinear prolongation, restriction P^T / 8, grids
 * halved while every axis has >= 4 cells and the level > 512 cells, 4 Jacobi
 * steps on the coarsest level), i.e. CGLS on min ||S M y - b||, x = M y.  The
 * minimiser is the one of eq. SimpObj; S has the printed source column -e
 * (weight 1); a system stops when ||S^H r|| <= rtol ||S^H b|| (the true
 * normal residual, as in wri_solve).  All systems of a grid iterate in
 * lockstep, chunks of iterations replay from a hipGraph.
 *   Arguments and results as in wri_objective_grad, except:
 *   J_out, grad  may be NULL (a solve only); grad[g] DEVICE float32 n(g)
 *   flags        0 or WRI_FLAG_NO_GRAPH (anything else: WRI_EINVAL)
 *   ws           DEVICE workspace of ws_bytes >= wri_precond_workspace_bytes()
 *                (about 9 complex vectors per system plus 4/7 of one for the
 *                coarse levels)
 *   res[k].relres is sqrt(||S^H r||^2 / ||S^H b||^2), res[k].alpha the CGLS
 *   unknown and res[k].alpha_ls = (A u)[src] in float64 (ESTIMATE).
 * Statuses: converged, max_iter, breakdown, zero_rhs, diverged (as in wri_solve). */
size_t wri_precond_workspace_bytes(const wri_grid* grids, int32_t n_grids, const wri_system* sys,
                                   int32_t n_sys, int32_t mode);
int wri_objective_grad_precond(const wri_grid* grids, int32_t n_grids, const float* const* m,
                               const wri_system* sys, int32_t n_sys, int32_t mode, int32_t max_iter,
                               int32_t flags, double* J_out, float* const* grad,
                               wri_c32* const* u_out, wri_result* res,
                               void* ws, size_t ws_bytes, void* stream);

/* Streaming bandwidth probe (a measurement helper, not a step of the method):
 * a kernel with the HBM access mix of a fused CGLS launch and none of its
 * arithmetic, the practical bandwidth ceiling that the fused kernels' fraction
 * of the 8 TB/s peak is set against.  Per complex64 element:
 *   mix 0  copy: read a, write c                                    16 B
 *   mix 1  forward pass: read s, p, m; write p (no x update)         28 B
 *   mix 2  forward pass with the x update: + read x, p'; write x     52 B
 *   mix 3  adjoint pass: read r, p, m; write r, s                    36 B
 *   n        elements per array (even, > 0)
 *   reps     timed launches after one warm-up launch
 *   ws       DEVICE workspace of ws_bytes >= wri_stream_probe_bytes(mix, n);
 *            its contents are read and overwritten (values are arbitrary)
 *   gbs_out  HOST: bytes of the mix / the shortest launch time (HIP events on
 *            `stream`), in GB/s, the best over the probe's variants (one or
 *            four element pairs in flight per thread on a grid-stride grid of
 *            8 blocks per compute unit, or one pair per thread on the full
 *            grid; ordinary or non-temporal stores)
 * Returns WRI_EINVAL / WRI_ENOWS for bad arguments, WRI_EHIP on a HIP error. */
size_t wri_stream_probe_bytes(int32_t mix, int64_t n);
int wri_stream_probe(int32_t mix, int64_t n, int32_t reps, void* ws, size_t ws_bytes, void* stream,
                     double* gbs_out);

/* The same probe in a tiled access pattern like the fused kernels': mix 1 (read a, b, m;
 * write c; 28 B per cell) over n_sys grids of nx x ny x nz cells, one
 * workgroup of 256 threads per (grid, 64 x 16 x 32 tile), blocks of the same
 * tile of consecutive grids adjacent, marching z through its slab plane by
 * plane (four cells per thread per plane), as the fused forward pass reads
 * and writes its vectors.  m is one float32 array shared by the grids.
 *   nx, ny, nz  multiples of 64, 16 and 32
 *   ws          DEVICE workspace of ws_bytes >= wri_tile_probe_bytes(...),
 *               contents read and overwritten (values arbitrary)
 *   gbs_out     HOST: 28 B x n_sys x cells / the shortest of `reps` timed
 *               launches (one warm-up launch first), in GB/s
 * Returns WRI_EINVAL / WRI_ENOWS for bad arguments, WRI_EHIP on a HIP error. */
size_t wri_tile_probe_bytes(int32_t nx, int32_t ny, int32_t nz, int32_t n_sys);
int wri_tile_probe(int32_t nx, int32_t ny, int32_t nz, int32_t n_sys, int32_t reps, void* ws, size_t ws_bytes,
                   void* stream, double* gbs_out);

/* Text of a return code; message of the last error on this thread. */
const char* wri_strerror(int code);
const char* wri_last_error(void);

/* Library version (major*10000 + minor*100 + patch). */
int wri_version(void);

#ifdef __cplusplus
}
#endif

#endif /* WRI_H */
