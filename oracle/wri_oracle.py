"""CPU reference (oracle) for the augmented-wavefield solve, the on-the-fly
source-weight estimate, and the WRI objective and gradient.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this module: it is used by the test-suite, by the smoke check and by the
benchmark's CPU-baseline leg.  It shares no code with the GPU library (its only
shared dependency is the seeded input generator ``wri_synth``, which holds no
arithmetic of the method).

Everything here is plain NumPy/SciPy in complex128 / float64, written from the
paper's statement of the method (section "3D Source free wavefield
reconstruction inversion"):

* the Helmholtz operator A_j(m) = omega_j^2 diag(m) + Laplacian (text after
  eq. FWI), with the 7-point second-order Laplacian, zero Dirichlet ghosts and
  an m-independent damping sponge (read as -i*omega*diag(b));
* the penalty objective (eq. ObjPen) in the scaling
  J = sum ||A u - alpha e||^2 + lam^2 ||P u - d||^2, i.e. lam = 1/lambda_paper and
  J = 2 f_2 / lambda_paper^2;
* the closed-form minimiser over (u, alpha) for fixed m (eq. SimpObj, read with
  conjugate transposes and P^H d), computed three independent ways;
* the reduced objective (eq. VarObj2) and its gradient (eq. VarG2, read with
  omega_j and a real part): g = sum 2 omega^2 Re(conj(u) * (A u - alpha e));
* a reference CGLS (the CG-on-the-normal-equations reading of the paper's
  Algorithm 1) with the stopping rule ||S^H r_k|| <= rtol ||S^H r_0||.
"""
from __future__ import annotations

import time
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spl

KNOWN = "known"
ESTIMATE = "estimate"


# --------------------------------------------------------------------------
# Operators (text after eq. FWI: A_j(m) = omega_j^2 diag(m) + Delta, P_i, e_i)
# --------------------------------------------------------------------------

def sponge(grid) -> np.ndarray:
    """Damping profile b >= 0 (one value per cell, x fastest).

    The paper is silent on the boundary; the workloads call for a "damped
    boundary" of nb cells.  Reading: b = (2 d0 / v_ref^2) * sum over axes of
    (delta/nb)^2, delta = distance (cells) into the sponge along that axis,
    d0 = 3 v_ref ln(1000) / (2 nb h).  nb = 0 gives b = 0."""
    if grid.nb <= 0:
        return np.zeros(grid.n)
    nb = float(grid.nb)
    d0 = 3.0 * grid.v_ref * np.log(1000.0) / (2.0 * nb * grid.h)

    def depth(n):
        i = np.arange(n, dtype=np.float64)
        return np.maximum(0.0, np.maximum(nb - i, i - (n - 1 - nb))) / nb

    dz, dy, dx = np.meshgrid(depth(grid.nz), depth(grid.ny), depth(grid.nx), indexing="ij")
    return ((2.0 * d0 / grid.v_ref ** 2) * (dx ** 2 + dy ** 2 + dz ** 2)).reshape(-1)


def _second_difference(n: int, h: float) -> sp.csr_matrix:
    """1D second difference (u[i-1] - 2u[i] + u[i+1]) / h^2, zero ghosts."""
    e = np.ones(n)
    return sp.diags([e[:-1], -2.0 * e, e[:-1]], [-1, 0, 1], shape=(n, n)) / h ** 2


def laplacian(grid) -> sp.csr_matrix:
    """7-point second-order Laplacian with zero Dirichlet ghosts, as the sum of
    1D second differences along x, y and z (x fastest in the linear index)."""
    Ix, Iy, Iz = (sp.identity(k, format="csr") for k in (grid.nx, grid.ny, grid.nz))
    Dx, Dy, Dz = (_second_difference(k, grid.h) for k in (grid.nx, grid.ny, grid.nz))
    L = sp.kron(Iz, sp.kron(Iy, Dx)) + sp.kron(Iz, sp.kron(Dy, Ix)) + sp.kron(Dz, sp.kron(Iy, Ix))
    return L.tocsr()


def helmholtz(grid, m: np.ndarray, omega: float, b: Optional[np.ndarray] = None) -> sp.csr_matrix:
    """A = L_h + diag(omega^2 m - i omega b)   (complex128 CSR).

    b defaults to the sponge profile of the grid; any non-negative array may
    be passed (tests use a constant one)."""
    if b is None:
        b = sponge(grid)
    diag = omega ** 2 * np.asarray(m, dtype=np.float64).reshape(-1) - 1j * omega * np.asarray(b).reshape(-1)
    return (laplacian(grid).astype(np.complex128) + sp.diags(diag)).tocsr()


def helmholtz_apply(grid, m: np.ndarray, omega: float, u: np.ndarray, b: Optional[np.ndarray] = None,
                    adjoint: bool = False) -> np.ndarray:
    """A u (or A^H u) in complex128 without forming A, for full-size checks.

    Same operator as `helmholtz`: the sum over the three axes of the second
    difference (u[i-1] - 2 u[i] + u[i+1]) / h^2 with zero ghost values, plus
    (omega^2 m - i omega b) u; the adjoint conjugates the diagonal (the
    Laplacian is real symmetric)."""
    if b is None:
        b = sponge(grid)
    v = np.asarray(u, dtype=np.complex128).reshape(grid.shape)
    out = np.zeros_like(v)
    for ax in range(3):
        d = -2.0 * v
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, -1)
        hi[ax] = slice(1, None)
        d[tuple(lo)] += v[tuple(hi)]     # u[i+1]
        d[tuple(hi)] += v[tuple(lo)]     # u[i-1]
        out += d
    out /= grid.h ** 2
    sgn = 1.0 if adjoint else -1.0
    diag = omega ** 2 * np.asarray(m, dtype=np.float64).reshape(grid.shape) + sgn * 1j * omega * np.asarray(b).reshape(grid.shape)
    out += diag * v
    return out.reshape(-1)


def helmholtz_rows(grid, m: np.ndarray, omega: float, cells, b: Optional[np.ndarray] = None):
    """Rows `cells` of A (same operator as `helmholtz`) straight from the
    stencil: (cols, vals), each of shape (len(cells), 7), the centre first and
    then the -x, +x, -y, +y, -z, +z neighbours.  A neighbour outside the grid
    (zero ghost) gets value 0 and the centre as its column."""
    if b is None:
        b = sponge(grid)
    cells = np.asarray(cells, dtype=np.int64).reshape(-1)
    x = cells % grid.nx
    y = (cells // grid.nx) % grid.ny
    z = cells // (grid.nx * grid.ny)
    h2 = 1.0 / grid.h ** 2
    mm = np.asarray(m, dtype=np.float64).reshape(-1)
    bb = np.asarray(b, dtype=np.float64).reshape(-1)
    cols = np.empty((cells.size, 7), dtype=np.int64)
    vals = np.zeros((cells.size, 7), dtype=np.complex128)
    cols[:, 0] = cells
    vals[:, 0] = -6.0 * h2 + omega ** 2 * mm[cells] - 1j * omega * bb[cells]
    steps = [(x, grid.nx, 1), (y, grid.ny, grid.nx), (z, grid.nz, grid.nx * grid.ny)]
    k = 1
    for coord, n, stride in steps:
        for dirn in (-1, 1):
            inside = (coord + dirn >= 0) & (coord + dirn < n)
            cols[:, k] = np.where(inside, cells + dirn * stride, cells)
            vals[:, k] = np.where(inside, h2, 0.0)
            k += 1
    return cols, vals


def restriction(n: int, rec: np.ndarray) -> sp.csr_matrix:
    """P: n_r x n selection of the receiver cells."""
    rec = np.asarray(rec, dtype=np.int64)
    return sp.csr_matrix((np.ones(rec.size), (np.arange(rec.size), rec)), shape=(rec.size, n),
                         dtype=np.complex128)


def unit_vector(n: int, src: int) -> np.ndarray:
    e = np.zeros(n, dtype=np.complex128)
    e[src] = 1.0
    return e


def system_operators(problem, k: int, m=None, b=None):
    """(A, P, e) of system k, at model m (defaults to problem.m of its grid)."""
    s = problem.systems[k]
    g = problem.grids[s.grid]
    mm = problem.m[s.grid] if m is None else m
    A = helmholtz(g, mm, s.omega, b)
    return A, restriction(g.n, s.rec), unit_vector(g.n, s.src)


# --------------------------------------------------------------------------
# Exact minimisers (eq. SimpObj and its KNOWN-source counterpart)
# --------------------------------------------------------------------------

def normal_matrix(A, P, lam) -> sp.csc_matrix:
    """N = A^H A + lam^2 P^H P."""
    AH = A.conj().T.tocsr()
    return (AH @ A + lam ** 2 * (P.conj().T @ P)).tocsc()


def factor(M):
    return spl.splu(sp.csc_matrix(M), permc_spec="COLAMD")


class NormalInverse:
    """x = N^{-1} y for N = A^H A + lam^2 P^H P, through the LU factors of A
    instead of a factor of N (A is a 7-point operator; N has a 25-point
    pattern and far more fill, so this route reaches larger grids).

    With B = (A^H A)^{-1} = A^{-1} A^{-H}, the Sherman-Morrison-Woodbury
    identity for the rank-n_r update lam^2 P^H P gives
        N^{-1} = B - B P^H (lam^{-2} I + P B P^H)^{-1} P B,
    where B P^H takes 2 n_r solves with the factors of A and the middle
    matrix is n_r x n_r.  lam = 0 or no receivers leaves N^{-1} = B.
    Same interface as a SuperLU factor of N (`solve`)."""

    def __init__(self, A, P, lam):
        self.lu = spl.splu(sp.csc_matrix(A), permc_spec="MMD_AT_PLUS_A")
        self.P = sp.csr_matrix(P)
        self.Z = None
        nr = P.shape[0]
        if lam != 0.0 and nr > 0:
            PH = self.P.conj().T.toarray()                 # n x n_r
            self.Z = self._B(PH)                           # B P^H
            M = np.eye(nr) / lam ** 2 + self.P @ self.Z    # lam^-2 I + P B P^H
            self.M = M

    def _B(self, y):
        return self.lu.solve(self.lu.solve(y, trans="H"))

    def solve(self, y):
        x = self._B(np.asarray(y, dtype=np.complex128))
        if self.Z is not None:
            x = x - self.Z @ np.linalg.solve(self.M, self.P @ x)
        return x


def solve_known(A, P, lam, alpha, e, d, lu=None) -> np.ndarray:
    """u = argmin ||A u - alpha e||^2 + lam^2 ||P u - d||^2
       = (A^H A + lam^2 P^H P)^{-1} (A^H (alpha e) + lam^2 P^H d)."""
    lu = lu or factor(normal_matrix(A, P, lam))
    rhs = A.conj().T @ (alpha * e) + lam ** 2 * (P.conj().T @ d)
    return lu.solve(rhs)


def solve_estimate(A, P, lam, src, d, route="varpro", lu=None) -> Tuple[np.ndarray, complex]:
    """(u, alpha) = argmin over u and alpha of ||A u - alpha e||^2 + lam^2 ||P u - d||^2.

    route "augmented": the (n+1) normal system of S = [[A, -e], [lam P, 0]],
      b = [0; lam d]: [[N, -A^H e], [-e^H A, 1]] [u; alpha] = [lam^2 P^H d; 0].
    route "varpro": u(alpha) = u0 + alpha u1 from the factor of N, then the
      scalar least-squares problem in alpha.
    route "projected": eliminate alpha first (its optimum is (A u)[src]), so
      u minimises ||(I - e e^H) A u||^2 + lam^2 ||P u - d||^2.
    """
    n = A.shape[0]
    e = unit_vector(n, src)
    PH = P.conj().T
    if route == "augmented":
        N = normal_matrix(A, P, lam)
        c = (A.conj().T @ e).reshape(-1, 1)
        r = (e.conj() @ A).reshape(1, -1)
        K = sp.bmat([[N, sp.csc_matrix(-c)], [sp.csc_matrix(-r), sp.csc_matrix([[1.0 + 0j]])]]).tocsc()
        rhs = np.concatenate([lam ** 2 * (PH @ d), [0.0]])
        x = factor(K).solve(rhs)
        return x[:n], complex(x[n])
    if route == "varpro":
        lu = lu or factor(normal_matrix(A, P, lam))
        u0 = lu.solve(lam ** 2 * (PH @ d))
        u1 = lu.solve(A.conj().T @ e)
        a = np.concatenate([A @ u1 - e, lam * (P @ u1)])
        c = np.concatenate([-(A @ u0), lam * (d - P @ u0)])
        alpha = complex(np.vdot(a, c) / np.vdot(a, a))
        return u0 + alpha * u1, alpha
    if route == "projected":
        keep = np.ones(n)
        keep[src] = 0.0
        At = (sp.diags(keep) @ A).tocsr()
        u = factor(normal_matrix(At, P, lam)).solve(lam ** 2 * (PH @ d))
        return u, complex((A @ u)[src])
    raise ValueError(route)


def objective_terms(A, P, lam, u, alpha, e, d):
    """(||A u - alpha e||^2, lam^2 ||P u - d||^2)."""
    r1 = A @ u - alpha * e
    r2 = P @ u - d
    return float(np.vdot(r1, r1).real), float(lam ** 2 * np.vdot(r2, r2).real)


def gradient_term(omega, u, A, alpha, e) -> np.ndarray:
    """2 omega^2 Re(conj(u) * (A u - alpha e)) : one system's share of dJ/dm."""
    return 2.0 * omega ** 2 * np.real(np.conj(u) * (A @ u - alpha * e))


def objective_grad(problem, m_list=None, mode=None, route="varpro", b_list=None,
                   return_fields=True, normal_solver="factor_N") -> Dict:
    """Exact variable-projection objective and gradient over all systems.

    normal_solver: "factor_N" (SuperLU of N = A^H A + lam^2 P^H P) or
    "woodbury" (`NormalInverse`, through the LU of A; for grids where the fill
    of N is too large).  The "augmented" and "projected" routes always factor
    their own matrices.

    Returns dict(J, J_sys, g (list per grid, float64 (nz,ny,nx)), u (list),
    alpha (array))."""
    mode = mode or problem.mode
    m_list = problem.m if m_list is None else m_list
    grads = [np.zeros(g.n) for g in problem.grids]
    us, alphas, Js = [None] * len(problem.systems), np.zeros(len(problem.systems), complex), \
        np.zeros(len(problem.systems))
    cache = {}
    for k, s in enumerate(problem.systems):
        g = problem.grids[s.grid]
        b = None if b_list is None else b_list[s.grid]
        key = (s.grid, s.freq, s.lam, tuple(np.asarray(s.rec).tolist()))
        if key not in cache:
            A = helmholtz(g, m_list[s.grid], s.omega, b)
            P = restriction(g.n, s.rec)
            if normal_solver == "woodbury":
                inv = NormalInverse(A, P, s.lam)
            elif normal_solver == "factor_N":
                inv = factor(normal_matrix(A, P, s.lam))
            else:
                raise ValueError(normal_solver)
            cache = {key: (A, P, inv)}
        A, P, lu = cache[key]
        e = unit_vector(g.n, s.src)
        if mode == KNOWN:
            u, alpha = solve_known(A, P, s.lam, s.alpha, e, s.d, lu=lu), s.alpha
        else:
            u, alpha = solve_estimate(A, P, s.lam, s.src, s.d, route=route,
                                      lu=lu if route == "varpro" else None)
        t1, t2 = objective_terms(A, P, s.lam, u, alpha, e, s.d)
        Js[k] = t1 + t2
        alphas[k] = alpha
        grads[s.grid] += gradient_term(s.omega, u, A, alpha, e)
        if return_fields:
            us[k] = u
    out = dict(J=float(Js.sum()), J_sys=Js, g=[gr.reshape(g.shape) for gr, g in zip(grads, problem.grids)],
               alpha=alphas)
    if return_fields:
        out["u"] = us
    return out


def plain_helmholtz_solution(A, q) -> np.ndarray:
    """u = A^{-1} q (the reduced-FWI wavefield, eq. PDEsolve)."""
    return spl.splu(A.tocsc(), permc_spec="COLAMD").solve(q)


def observed_data(problem, seed=0, noise=0.01) -> List[np.ndarray]:
    """Clean data d = P A(m_true)^{-1} (alpha_true e) per system, plus noise
    (via the generator's noise routine)."""
    import wri_synth
    rng = np.random.default_rng(seed + 1000)
    out = []
    cache = {}
    for s in problem.systems:
        g = problem.grids[s.grid]
        key = (s.grid, s.freq)
        if key not in cache:
            A = helmholtz(g, problem.m_true[s.grid], s.omega)
            cache = {key: spl.splu(A.tocsc(), permc_spec="COLAMD")}
        lu = cache[key]
        u = lu.solve(s.alpha * unit_vector(g.n, s.src))
        d = u[np.asarray(s.rec)]
        out.append(wri_synth.add_noise(d, rng, noise) if noise > 0 else d)
    return out


# --------------------------------------------------------------------------
# Residual of the normal equations and the reference CGLS (Algorithm 1 read as
# CG on S^H S; convergence on ||S^H r_k|| / ||S^H r_0||)
# --------------------------------------------------------------------------

def apply_S(A, P, lam, src, mode, x, c=1.0):
    """S x: KNOWN S = [A; lam P] (x = u); ESTIMATE S = [[A, -c e], [lam P, 0]]
    (x = [u; alpha / c]; c = 1 is the paper's S, any c > 0 has the same
    minimiser in (u, alpha))."""
    n = A.shape[0]
    u = x[:n]
    t1 = A @ u
    if mode == ESTIMATE:
        t1 = t1.copy()
        t1[src] -= c * x[n]
    return np.concatenate([t1, lam * (P @ u)])


def apply_SH(A, P, lam, src, mode, r, AH=None, PH=None, c=1.0):
    """S^H r for r = [r1 (n); r2 (n_r)]."""
    n = A.shape[0]
    AH = A.conj().T if AH is None else AH
    PH = P.conj().T if PH is None else PH
    s = AH @ r[:n] + lam * (PH @ r[n:])
    if mode == ESTIMATE:
        return np.concatenate([s, [-c * r[src]]])
    return s


def rhs_vector(n, lam, src, mode, alpha, d):
    """b: KNOWN [alpha e; lam d]; ESTIMATE [0; lam d]."""
    b1 = np.zeros(n, dtype=np.complex128)
    if mode == KNOWN:
        b1[src] = alpha
    return np.concatenate([b1, lam * np.asarray(d, dtype=np.complex128)])


def normal_residual(A, P, lam, src, mode, alpha_known, d, u, alpha=None) -> float:
    """||S^H (b - S x)|| / ||S^H b|| in complex128 (x = u, or [u; alpha])."""
    n = A.shape[0]
    x = np.asarray(u, dtype=np.complex128)
    if mode == ESTIMATE:
        x = np.concatenate([x, [complex(alpha)]])
    b = rhs_vector(n, lam, src, mode, alpha_known, d)
    num = apply_SH(A, P, lam, src, mode, b - apply_S(A, P, lam, src, mode, x))
    den = apply_SH(A, P, lam, src, mode, b)
    dn = np.linalg.norm(den)
    return float(np.linalg.norm(num) / dn) if dn > 0 else float(np.linalg.norm(num))


def cgls(A, P, lam, src, mode, alpha_known, d, rtol, maxiter, vec_dtype=np.complex128,
         time_limit=None, alpha_scale=1.0):
    """Reference CGLS on min ||S x - b||.

    x0 = 0, r = b, s = S^H r, p = s, gamma = ||s||^2; per iteration
    t = S p, a = gamma/||t||^2, x += a p, r -= a t, s = S^H r,
    beta = ||s||^2/gamma, p = s + beta p.  Stops before forming t when
    sqrt(gamma/gamma0) <= rtol.  Inner products and scalars are float64;
    vectors are stored in vec_dtype (complex64 emulates the GPU's storage).

    Returns dict(u, alpha, iters, relres, status, seconds)."""
    t0 = time.perf_counter()
    n = A.shape[0]
    AH, PH = A.conj().T.tocsr(), P.conj().T.tocsr()
    b = rhs_vector(n, lam, src, mode, alpha_known, d).astype(vec_dtype)
    nx = n + (1 if mode == ESTIMATE else 0)

    def dot(v):
        v = v.astype(np.complex128, copy=False)
        return float(np.vdot(v, v).real)

    x = np.zeros(nx, dtype=vec_dtype)
    r = b.copy()
    c = float(alpha_scale)
    s = apply_SH(A, P, lam, src, mode, r.astype(np.complex128), AH, PH, c).astype(vec_dtype)
    p = s.copy()
    gamma = dot(s)
    gamma0 = gamma
    k = 0
    status = "converged"
    if gamma0 == 0.0:
        return dict(u=x[:n].astype(np.complex128), alpha=c * complex(x[n]) if mode == ESTIMATE else None,
                    iters=0, relres=0.0, status="zero_rhs", seconds=time.perf_counter() - t0)
    while True:
        if np.sqrt(gamma / gamma0) <= rtol:
            break
        if k >= maxiter or (time_limit is not None and time.perf_counter() - t0 > time_limit):
            status = "max_iter"
            break
        t = apply_S(A, P, lam, src, mode, p.astype(np.complex128), c).astype(vec_dtype)
        delta = dot(t)
        if not np.isfinite(delta) or delta <= 0.0:
            status = "breakdown"
            break
        a = gamma / delta
        x = (x + a * p).astype(vec_dtype)
        r = (r - a * t).astype(vec_dtype)
        s = apply_SH(A, P, lam, src, mode, r.astype(np.complex128), AH, PH, c).astype(vec_dtype)
        gnew = dot(s)
        beta = gnew / gamma
        gamma = gnew
        p = (s + beta * p).astype(vec_dtype)
        k += 1
    x = x.astype(np.complex128)
    return dict(u=x[:n], alpha=c * complex(x[n]) if mode == ESTIMATE else None, iters=k,
                relres=float(np.sqrt(gamma / gamma0)), status=status,
                r=r.astype(np.complex128), seconds=time.perf_counter() - t0)


# --------------------------------------------------------------------------
# Preconditioned CGLS.  Beyond the paper, whose only iteration reducer is the
# adaptive tolerance of Algorithm 2: S is preconditioned on the right by one
# multigrid V-cycle of the complex-shifted Helmholtz operator
#   A_beta = L_h + diag(omega^2 (1 - i beta) m - i omega b),
# the same Laplacian, model and sponge as A with an imaginary shift of the
# mass term.  The minimiser does not change; the iterates and their number do.
# --------------------------------------------------------------------------

CSL_BETA = 0.5            # imaginary shift of the mass term in A_beta
CSL_JACOBI = 0.7          # damping of the Jacobi smoother
CSL_COARSE_SWEEPS = 4     # Jacobi steps on the coarsest level
CSL_COARSEST_CELLS = 512  # levels are halved while they hold more cells than this


def csl_prolongation_1d(n: int) -> sp.csr_matrix:
    """Linear interpolation from n // 2 coarse points to n fine points along
    one axis: coarse point i sits on fine point 2i + 1, so fine 2i + 1 takes
    coarse i with weight 1 and fine 2i takes coarse i - 1 and i with weight
    1/2 each; coarse values outside the grid are zero."""
    nc = n // 2
    rows, cols, vals = [], [], []
    for i in range(nc):
        f = 2 * i + 1
        rows.append(f); cols.append(i); vals.append(1.0)
        for ff in (f - 1, f + 1):
            if 0 <= ff < n:
                rows.append(ff); cols.append(i); vals.append(0.5)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, nc))


def csl_levels(grid, m: np.ndarray) -> List[Dict]:
    """The V-cycle's grid hierarchy.  Level 0 is the grid itself (its model m
    and sponge b).  A level is halved along every axis (n -> n // 2, h -> 2 h)
    while every axis has at least 4 cells and the level holds more than
    CSL_COARSEST_CELLS cells; the coarse m and b are the fine values
    restricted with P^T and divided by the restricted ones (weighted means).
    Each level but the last carries P, the prolongation from the next level
    (3D trilinear: the product of the 1D interpolations, x fastest)."""
    nz, ny, nx = grid.shape
    levels = [dict(shape=(nz, ny, nx), h=float(grid.h), m=np.asarray(m, dtype=np.float64).reshape(-1),
                   b=sponge(grid))]
    while min(nz, ny, nx) >= 4 and nz * ny * nx > CSL_COARSEST_CELLS:
        lev = levels[-1]
        Pm = sp.kron(csl_prolongation_1d(nz), sp.kron(csl_prolongation_1d(ny), csl_prolongation_1d(nx))).tocsr()
        lev["P"] = Pm
        w = np.asarray(Pm.sum(axis=0)).ravel()          # P^T 1
        nz, ny, nx = nz // 2, ny // 2, nx // 2
        levels.append(dict(shape=(nz, ny, nx), h=2.0 * lev["h"], m=(Pm.T @ lev["m"]) / w, b=(Pm.T @ lev["b"]) / w))
    return levels


def csl_operator(level: Dict, omega: float, beta: float = CSL_BETA) -> sp.csr_matrix:
    """A_beta on one level: 7-point Laplacian with zero ghosts at the level's
    spacing plus diag(omega^2 (1 - i beta) m - i omega b)."""
    nz, ny, nx = level["shape"]
    g = type("G", (), {})()
    g.nx, g.ny, g.nz, g.h = nx, ny, nz, level["h"]
    diag = omega ** 2 * (1.0 - 1j * beta) * level["m"] - 1j * omega * level["b"]
    return (laplacian(g).astype(np.complex128) + sp.diags(diag)).tocsr()


def csl_vcycle(levels: List[Dict], omega: float, v: np.ndarray, adjoint: bool = False, beta: float = CSL_BETA,
               wj: float = CSL_JACOBI, coarse_sweeps: int = CSL_COARSE_SWEEPS) -> np.ndarray:
    """One V(1,1) cycle from a zero initial guess: the fixed linear map
    M v ~ A_beta^{-1} v.  On a level with right-hand side f: x = wj D^-1 f
    (one damped Jacobi step from zero, D the diagonal of A_beta); the residual
    f - A_beta x restricted with R = P^T / 8 is the next level's right-hand
    side; the next level's result is prolonged and added (x += P e); then one
    more Jacobi step x += wj D^-1 (f - A_beta x).  On the coarsest level,
    coarse_sweeps Jacobi steps from zero.  With R proportional to P^T and the
    same smoother on both sides, M is complex symmetric (M^T = M), so
    M^H v = conj(M conj v): adjoint=True runs the cycle on conj(A_beta)."""
    ops = [csl_operator(lev, omega, beta) for lev in levels]
    if adjoint:
        ops = [A.conj() for A in ops]

    def cycle(l, f):
        A = ops[l]
        dinv = 1.0 / A.diagonal()
        if l == len(levels) - 1:
            x = wj * dinv * f
            for _ in range(coarse_sweeps - 1):
                x = x + wj * dinv * (f - A @ x)
            return x
        Pm = levels[l]["P"]
        x = wj * dinv * f
        x = x + Pm @ cycle(l + 1, (Pm.T @ (f - A @ x)) / 8.0)
        return x + wj * dinv * (f - A @ x)

    return cycle(0, np.asarray(v, dtype=np.complex128))


def pcgls(A, P, lam, src, mode, alpha_known, d, rtol, maxiter, M, MH, alpha_scale=1.0):
    """CGLS on min ||S M y - b|| with x = M y: right preconditioning by M on
    the wavefield part of x (the source weight of ESTIMATE mode is left as it
    is).  x0 = 0, r = b, s = S^H r, z = M^H s, p = z, gamma = ||z||^2; per
    iteration q = M p, t = S q, a = gamma / ||t||^2, x += a q, r -= a t,
    s = S^H r, z = M^H s, beta = ||z||^2 / gamma, p = z + beta p.  Stops
    before forming q when ||s|| <= rtol ||s_0||: the same test on the true
    normal residual as the unpreconditioned CGLS.  M and MH act on vectors of
    the grid's cells.  Returns dict(u, alpha, iters, relres, status, r)."""
    n = A.shape[0]
    AH, PH = A.conj().T.tocsr(), P.conj().T.tocsr()
    est = mode == ESTIMATE
    c = float(alpha_scale)
    b = rhs_vector(n, lam, src, mode, alpha_known, d)

    def prec(f, y):
        out = np.array(y, dtype=np.complex128)
        out[:n] = f(y[:n])
        return out

    x = np.zeros(n + (1 if est else 0), dtype=np.complex128)
    r = b.copy()
    s = apply_SH(A, P, lam, src, mode, r, AH, PH, c)
    s0 = float(np.vdot(s, s).real)
    if s0 == 0.0:
        return dict(u=x[:n], alpha=c * complex(x[n]) if est else None, iters=0, relres=0.0, status="zero_rhs", r=r)
    z = prec(MH, s)
    p = z.copy()
    gamma = float(np.vdot(z, z).real)
    k, status = 0, "converged"
    while True:
        ss = float(np.vdot(s, s).real)
        if np.sqrt(ss / s0) <= rtol:
            break
        if k >= maxiter:
            status = "max_iter"
            break
        q = prec(M, p)
        t = apply_S(A, P, lam, src, mode, q, c)
        delta = float(np.vdot(t, t).real)
        if not np.isfinite(delta) or delta <= 0.0:
            status = "breakdown"
            break
        a = gamma / delta
        x = x + a * q
        r = r - a * t
        s = apply_SH(A, P, lam, src, mode, r, AH, PH, c)
        z = prec(MH, s)
        gnew = float(np.vdot(z, z).real)
        p = z + (gnew / gamma) * p
        gamma = gnew
        k += 1
    return dict(u=x[:n], alpha=c * complex(x[n]) if est else None, iters=k,
                relres=float(np.sqrt(float(np.vdot(s, s).real) / s0)), status=status, r=r)


def precond_objective_grad(problem, rtol, mode=None, alpha_scale=1.0, maxiter=10 ** 6) -> Dict:
    """J, g, u, alpha and iteration counts with every system solved by the
    V-cycle-preconditioned CGLS (`pcgls`) to the relative normal residual
    rtol.  J and g use the recurred residual r1 as the GPU path does:
    J = sum ||r||^2, g = -sum 2 omega^2 Re(conj(u) r1); alpha of ESTIMATE
    mode is the least-squares weight (A u)[src] of the computed u."""
    mode = mode or problem.mode
    J = 0.0
    grads = [np.zeros(gr.n) for gr in problem.grids]
    us, alphas, iters = [], [], []
    for k, s in enumerate(problem.systems):
        gr = problem.grids[s.grid]
        A, P, e = system_operators(problem, k)
        levels = csl_levels(gr, problem.m[s.grid])
        M = lambda v, lv=levels, om=s.omega: csl_vcycle(lv, om, v)
        MH = lambda v, lv=levels, om=s.omega: csl_vcycle(lv, om, v, adjoint=True)
        out = pcgls(A, P, s.lam, s.src, mode, s.alpha, s.d, rtol, maxiter, M, MH, alpha_scale)
        r = out["r"]
        J += float(np.vdot(r, r).real)
        grads[s.grid] += -2.0 * s.omega ** 2 * np.real(np.conj(out["u"]) * r[:gr.n])
        us.append(out["u"])
        alphas.append(complex((A @ out["u"])[s.src]) if mode == ESTIMATE else s.alpha)
        iters.append(out["iters"])
    return dict(J=J, g=grads, u=us, alpha=np.array(alphas), iters=iters)


# --------------------------------------------------------------------------
# The paper's own scaling (eqs. ObjPen, CmpctWRIobj, Sandb)
# --------------------------------------------------------------------------

def paper_S_and_b(A, P, src, d, lam_p):
    """S = [[lam_p A, -lam_p e], [P, 0]], b = [0; d] exactly as printed."""
    n = A.shape[0]
    e = sp.csr_matrix(([1.0 + 0j], ([src], [0])), shape=(n, 1))
    S = sp.bmat([[lam_p * A, -lam_p * e], [P, None]]).tocsr()
    b = np.concatenate([np.zeros(n, np.complex128), np.asarray(d, np.complex128)])
    return S, b


def paper_f2(A, P, lam_p, u, alpha, e, d) -> float:
    """f_2 = 1/2 (||P u - d||^2 + lam_p^2 ||A u - alpha e||^2)."""
    r1 = A @ u - alpha * e
    r2 = P @ u - d
    return 0.5 * float(np.vdot(r2, r2).real + lam_p ** 2 * np.vdot(r1, r1).real)


# --------------------------------------------------------------------------
# Outer loop: source-free adaptive WRI with TV regularisation
# (section "SF-AWRI with total variation regularization", eq. TVAWRI,
#  Algorithm 2)
# --------------------------------------------------------------------------

def tv(grid, m: np.ndarray, eps: float) -> float:
    """Smoothed isotropic total variation (the paper names the TV norm without
    defining it; reading): TV(m) = sum over cells of
    sqrt((D_x m)^2 + (D_y m)^2 + (D_z m)^2 + eps^2), with forward differences
    (D_x m)[i] = (m[i+1] - m[i]) / h and a zero difference in the last cell of
    every axis (the model is not extended past the grid)."""
    phi, _ = _tv_parts(grid, m, eps)
    return float(phi.sum())


def _tv_parts(grid, m, eps):
    v = np.asarray(m, dtype=np.float64).reshape(grid.shape)
    d = []
    for ax in range(3):
        dd = np.zeros_like(v)
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, -1)
        hi[ax] = slice(1, None)
        dd[tuple(lo)] = (v[tuple(hi)] - v[tuple(lo)]) / grid.h
        d.append(dd)
    phi = np.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2 + eps ** 2)
    return phi, d


def tv_grad(grid, m: np.ndarray, eps: float) -> np.ndarray:
    """Gradient of `tv` with respect to m (same shape as m, flattened).

    Cell c enters its own forward differences with weight -1/h and the
    difference of its lower neighbour along each axis with weight +1/h:
    dTV/dm_c = (1/h) * sum over axes a of (q_a[c - e_a] - q_a[c]),
    q_a = (D_a m) / phi (q_a is zero where D_a m is)."""
    phi, d = _tv_parts(grid, m, eps)
    out = np.zeros(grid.shape)
    for ax in range(3):
        q = d[ax] / phi
        out -= q
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, -1)
        hi[ax] = slice(1, None)
        out[tuple(hi)] += q[tuple(lo)]
    return (out / grid.h).reshape(-1)


def lbfgs_two_loop(g: np.ndarray, pairs, h0: float) -> np.ndarray:
    """H g for the limited-memory BFGS inverse-Hessian approximation built from
    the curvature pairs (s_i, y_i), oldest first, with H_0 = h0 * I (the
    two-loop recursion; Nocedal and Wright, Numerical Optimization, Alg. 7.4).
    The model update of Algorithm 2 is m - H g."""
    q = np.asarray(g, dtype=np.float64).copy()
    coef = []
    for s, y in reversed(pairs):
        rho = 1.0 / float(np.dot(y, s))
        a = rho * float(np.dot(s, q))
        q -= a * y
        coef.append((rho, a))
    r = h0 * q
    for (s, y), (rho, a) in zip(pairs, reversed(coef)):
        b = rho * float(np.dot(y, r))
        r += (a - b) * s
    return r


def inexact_objective_grad(problem, m, rtol, mode=None, alpha_scale=1.0):
    """J and g at model m with every system solved by the reference CGLS to
    the relative normal-residual tolerance rtol (complex128).  J and g use the
    recurred residual r1 = b1 - (A u - alpha e) of CGLS, as the GPU path does:
    J = sum ||r||^2, g = -sum 2 omega^2 Re(conj(u) r1).

    alpha_scale is the weight c of the source column of S = [[A, -c e],
    [lam P, 0]] in ESTIMATE mode; the default 1 is S as eq. SimpObj prints it.
    Any c > 0 has the same minimiser but different iterates, so a caller that
    compares iterates with a solver using another column weight passes it."""
    mode = mode or problem.mode
    J = 0.0
    grads = [np.zeros(gr.n) for gr in problem.grids]
    iters = []
    for k, s in enumerate(problem.systems):
        gr = problem.grids[s.grid]
        A = helmholtz(gr, m[s.grid], s.omega)
        P = restriction(gr.n, s.rec)
        out = cgls(A, P, s.lam, s.src, mode, s.alpha, s.d, rtol=rtol, maxiter=10 ** 6,
                   alpha_scale=float(alpha_scale))
        r = out["r"]
        J += float(np.vdot(r, r).real)
        grads[s.grid] += -2.0 * s.omega ** 2 * np.real(np.conj(out["u"]) * r[:gr.n])
        iters.append(out["iters"])
    return J, grads, iters


def awri(problem, m0, gamma: float, eps0: float, n_outer: int, memory: int = 5, eps_tv: float = 1e-9,
         step0: float = 0.01, eps_min: float = 1e-8, solver: str = "exact", m_min: float = 0.0,
         m_max: float = 0.0, max_step: float = 0.0, mask_sponge: bool = False,
         alpha_scale: float = 1.0) -> Dict:
    """Algorithm 2 (source-free AWRI with TV) on a single-grid problem.

    Objective F(m) = J(m) + gamma * TV(m) in this package's scaling
    (J = sum ||A u - alpha e||^2 + lam^2 ||P u - d||^2; the paper's f4 equals
    (lambda_p^2 / 2) J + gamma_p TV, so gamma = 2 gamma_p / lambda_p^2).
    Each trial model is m - H g (l-BFGS, unit step; with no curvature pair
    yet, H = step0 * max|m| / max|g| * I).  A trial whose F does not decrease
    halves the solver tolerance eps and recomputes F, g and the l-BFGS
    approximation at the current model (the paper's "go back"); the
    curvature pairs collected at the looser tolerance are dropped (reading:
    they mix gradients of two accuracies, and without a line search a stale
    pair repeats the same rejected step), so the next trial is a scaled
    gradient step.  The loop stops when eps would fall below eps_min.  Accepted trials add the pair (s, y) = (dm, dg) when s.y > 0 and
    keep the last `memory` pairs.  The values at an accepted trial serve as the
    next iteration's F and g (same model, same tolerance).  Optional bounds
    clip the trial model to [m_min, m_max] (0 disables a bound).  Two
    safeguards that the algorithm as printed does not have (readings): the
    update is scaled down so that max|dm| <= max_step * max|m| (0: no cap), and
    with mask_sponge the update is zero inside the damping layer (b > 0), which
    is an extension of the physical model rather than part of it.

    solver: "exact" (sparse direct, eps only drives the schedule) or "cgls"
    (reference CGLS to tolerance eps, see `inexact_objective_grad`, with the
    source-column weight alpha_scale).
    Returns dict(m, history) with one record per trial:
    (F, J, TV, eps, accepted, solver iterations)."""
    grid = problem.grids[0]
    assert len(problem.grids) == 1
    m = np.asarray(m0, dtype=np.float64).reshape(-1).copy()

    def evaluate(mm, eps):
        if solver == "exact":
            o = objective_grad(problem, [mm.reshape(grid.shape)], return_fields=False)
            J, g, it = o["J"], o["g"][0].reshape(-1), 0
        else:
            J, gl, its = inexact_objective_grad(problem, [mm], eps, alpha_scale=alpha_scale)
            g, it = gl[0], int(sum(its))
        t = tv(grid, mm, eps_tv)
        gg = g + gamma * tv_grad(grid, mm, eps_tv)
        if mask_sponge:
            gg = np.where(sponge(grid) > 0.0, 0.0, gg)
        return J + gamma * t, gg, J, t, it

    eps = float(eps0)
    F, g, J, T, it = evaluate(m, eps)
    history = [dict(F=F, J=J, TV=T, eps=eps, accepted=True, iters=it)]
    pairs = []
    accepted = 0
    while accepted < n_outer:
        if pairs:
            s_new, y_new = pairs[-1]
            h0 = float(np.dot(s_new, y_new) / np.dot(y_new, y_new))
        else:
            gmax = float(np.abs(g).max())
            if gmax == 0.0:
                break
            h0 = step0 * float(np.abs(m).max()) / gmax
        dm = -lbfgs_two_loop(g, pairs, h0)
        if mask_sponge:
            dm[sponge(grid) > 0.0] = 0.0
        if max_step > 0.0:
            cap = max_step * float(np.abs(m).max())
            big = float(np.abs(dm).max())
            if big > cap:
                dm *= cap / big
        m_try = m + dm
        if m_min > 0.0:
            m_try = np.maximum(m_try, m_min)
        if m_max > 0.0:
            m_try = np.minimum(m_try, m_max)
        F_try, g_try, J_try, T_try, it = evaluate(m_try, eps)
        ok = F_try <= F
        history.append(dict(F=F_try, J=J_try, TV=T_try, eps=eps, accepted=ok, iters=it))
        if not ok:
            if 0.5 * eps < eps_min:
                break
            eps *= 0.5
            pairs = []
            F, g, J, T, it = evaluate(m, eps)
            history.append(dict(F=F, J=J, TV=T, eps=eps, accepted=True, iters=it, reeval=True))
            continue
        s, y = m_try - m, g_try - g
        if float(np.dot(s, y)) > 0.0:
            pairs.append((s, y))
            pairs = pairs[-memory:] if memory > 0 else []
        m, F, g = m_try, F_try, g_try
        accepted += 1
    return dict(m=m, history=history)


# --------------------------------------------------------------------------
# Reduced (conventional) FWI: eqs. FWI, PDEsolve, FWI2 — the baseline that WRI
# is compared against.  Sparse direct solves; no iteration.
# --------------------------------------------------------------------------

def fwi_alpha(Pw: np.ndarray, d: np.ndarray) -> complex:
    """Source weight minimising ||alpha P w - d||^2 for fixed w = A^{-1} e:
    alpha = (P w)^H d / ||P w||^2 (0 when P w = 0)."""
    den = float(np.vdot(Pw, Pw).real)
    return complex(np.vdot(Pw, d) / den) if den > 0.0 else 0j


def fwi_objective_grad(problem, m_list=None, mode=None, b_list=None) -> Dict:
    """Reduced FWI objective and gradient (eq. FWI2 with the wavefield of eq.
    PDEsolve):  f = 1/2 sum_ij ||alpha_ij P_i A_j^{-1} e_i - d_ij||^2.

    KNOWN: alpha_ij = the system's given weight.  ESTIMATE: alpha_ij minimises
    f for the current m (`fwi_alpha`, the minimisation over alpha that eq. FWI2
    keeps), so the gradient below is that of the reduced function of m alone
    (the alpha-derivative vanishes at the optimum).

    Gradient by the adjoint-state method: with u = alpha A^{-1} e and
    v = A^{-H} P^H (P u - d),  df/dm = -sum_ij omega_j^2 Re(conj(v) * u),
    because dA/dm = omega^2 I (the sponge does not depend on m).

    Returns dict(f, f_sys, g (list per grid, (nz, ny, nx)), alpha, u, v)."""
    mode = mode or problem.mode
    m_list = problem.m if m_list is None else m_list
    grads = [np.zeros(g.n) for g in problem.grids]
    ns = len(problem.systems)
    f_sys, alphas, us, vs = np.zeros(ns), np.zeros(ns, complex), [None] * ns, [None] * ns
    cache = {}
    for k, s in enumerate(problem.systems):
        g = problem.grids[s.grid]
        key = (s.grid, s.freq)
        if key not in cache:
            b = None if b_list is None else b_list[s.grid]
            A = helmholtz(g, m_list[s.grid], s.omega, b)
            cache = {key: spl.splu(A.tocsc(), permc_spec="COLAMD")}
        lu = cache[key]
        P = restriction(g.n, s.rec)
        d = np.asarray(s.d, dtype=np.complex128)
        w = lu.solve(unit_vector(g.n, s.src))
        alpha = complex(s.alpha) if mode == KNOWN else fwi_alpha(P @ w, d)
        u = alpha * w
        rho = P @ u - d
        v = lu.solve(np.asarray(P.conj().T @ rho), trans="H")
        f_sys[k] = 0.5 * float(np.vdot(rho, rho).real)
        alphas[k] = alpha
        grads[s.grid] += -(s.omega ** 2) * np.real(np.conj(v) * u)
        us[k], vs[k] = u, v
    return dict(f=float(f_sys.sum()), f_sys=f_sys, alpha=alphas, u=us, v=vs,
                g=[gr.reshape(g.shape) for gr, g in zip(grads, problem.grids)])


def receiver_source_solution(A, n: int, rec, values) -> np.ndarray:
    """z = A^{-1} (P^H c): the wavefield of point sources of strengths c at the
    receiver cells (the adjoint source of the reduced method, solved with A;
    A is complex symmetric, so A^{-H} y = conj(A^{-1} conj(y)))."""
    q = np.asarray(restriction(n, rec).conj().T @ np.asarray(values, dtype=np.complex128))
    return spl.splu(A.tocsc(), permc_spec="COLAMD").solve(q)


# --------------------------------------------------------------------------
# One model grid tied to per-frequency simulation grids (trilinear resampling)
# --------------------------------------------------------------------------

def _axis_interp(n_model: int, h_model: float, n_grid: int, h_grid: float) -> sp.csr_matrix:
    """1-D linear interpolation from model nodes a*h_model to simulation nodes
    i*h_grid (common origin), clamped to the model's extent."""
    rows, cols, vals = [], [], []
    for i in range(n_grid):
        if n_model == 1:
            rows.append(i); cols.append(0); vals.append(1.0)
            continue
        xi = min(max(i * h_grid / h_model, 0.0), n_model - 1.0)
        a = min(int(np.floor(xi)), n_model - 2)
        t = xi - a
        rows += [i, i]; cols += [a, a + 1]; vals += [1.0 - t, t]
    return sp.csr_matrix((vals, (rows, cols)), shape=(n_grid, n_model))


def resample_matrix(model_grid, grid) -> sp.csr_matrix:
    """R: trilinear interpolation of a model on `model_grid` at the nodes of
    `grid` (cell (i, j, k) at (i h, j h, k h) on both), as the Kronecker product
    of the three axes in the x-fastest cell order."""
    Rx = _axis_interp(model_grid.nx, model_grid.h, grid.nx, grid.h)
    Ry = _axis_interp(model_grid.ny, model_grid.h, grid.ny, grid.h)
    Rz = _axis_interp(model_grid.nz, model_grid.h, grid.nz, grid.h)
    return sp.kron(Rz, sp.kron(Ry, Rx)).tocsr()


def objective_grad_model(problem, model_grid, m_model, mode=None) -> Dict:
    """J and dJ/dm_model when every simulation grid takes its model as
    m_g = R_g m_model: J from `objective_grad` at those models and, by the
    chain rule, g_model = sum_g R_g^T g_g."""
    mm = np.asarray(m_model, dtype=np.float64).reshape(-1)
    Rs = [resample_matrix(model_grid, g) for g in problem.grids]
    m_list = [(R @ mm).reshape(g.shape) for R, g in zip(Rs, problem.grids)]
    out = objective_grad(problem, m_list=m_list, mode=mode, return_fields=False)
    g = np.zeros(mm.size)
    for R, gg in zip(Rs, out["g"]):
        g += R.T @ gg.reshape(-1)
    return dict(J=out["J"], g=g.reshape(model_grid.shape), m_list=m_list, alpha=out["alpha"])


# --------------------------------------------------------------------------
# Sources and receivers off the grid nodes (trilinear e and P)
# --------------------------------------------------------------------------

def trilinear_point(grid, xyz) -> Tuple[np.ndarray, np.ndarray]:
    """Cells and weights of trilinear interpolation at the point xyz = (x, y, z)
    [m], cell (i, j, k) at (i h, j h, k h), the point clamped into the grid.
    Per axis xi = clamp(x / h, 0, n - 1), i0 = min(floor(xi), n - 2), weights
    (1 - t, t) on (i0, i0 + 1); an axis of one cell has weight 1 on cell 0.
    Returns the distinct cells (duplicates merged, zero weights dropped) and
    their weights."""
    per_axis = []
    for coord, n in zip(xyz, (grid.nx, grid.ny, grid.nz)):
        if n == 1:
            per_axis.append([(0, 1.0)])
            continue
        xi = min(max(float(coord) / grid.h, 0.0), n - 1.0)
        i0 = min(int(np.floor(xi)), n - 2)
        t = xi - i0
        per_axis.append([(i0, 1.0 - t), (i0 + 1, t)])
    acc: Dict[int, float] = {}
    for (k, wz) in per_axis[2]:
        for (j, wy) in per_axis[1]:
            for (i, wx) in per_axis[0]:
                c = (k * grid.ny + j) * grid.nx + i
                acc[c] = acc.get(c, 0.0) + wz * wy * wx
    cells = np.array(sorted(c for c in acc if acc[c] != 0.0), dtype=np.int64)
    return cells, np.array([acc[c] for c in cells])


def offgrid_operators(grid, src_xyz, rec_xyz) -> Tuple[np.ndarray, sp.csr_matrix]:
    """e (dense, the source spread over its cells) and P (n_rec x n, one
    interpolation row per receiver)."""
    e = np.zeros(grid.n, dtype=np.complex128)
    cs, ws = trilinear_point(grid, src_xyz)
    e[cs] = ws
    rows, cols, vals = [], [], []
    for q, r in enumerate(np.asarray(rec_xyz, dtype=np.float64).reshape(-1, 3)):
        cr, wr = trilinear_point(grid, r)
        rows += [q] * len(cr); cols += list(cr); vals += list(wr)
    P = sp.csr_matrix((np.asarray(vals, dtype=np.complex128), (rows, cols)),
                      shape=(len(np.asarray(rec_xyz).reshape(-1, 3)), grid.n))
    return e, P


def solve_estimate_general(A, P, lam, e, d, route="varpro") -> Tuple[np.ndarray, complex]:
    """(u, alpha) = argmin ||A u - alpha e||^2 + lam^2 ||P u - d||^2 for a
    general source vector e (eq. SimpObj with e spread over several cells).
    route "varpro": u(alpha) = u0 + alpha u1 from the normal matrix, then the
    scalar least-squares problem; route "augmented": the (n+1) normal system
    of S = [[A, -e], [lam P, 0]]."""
    n = A.shape[0]
    PH = P.conj().T
    if route == "augmented":
        N = normal_matrix(A, P, lam)
        c = (A.conj().T @ e).reshape(-1, 1)
        r = (e.conj() @ A).reshape(1, -1)
        K = sp.bmat([[N, sp.csc_matrix(-c)], [sp.csc_matrix(-r), sp.csc_matrix([[np.vdot(e, e)]])]]).tocsc()
        x = factor(K).solve(np.concatenate([lam ** 2 * (PH @ d), [0.0]]))
        return x[:n], complex(x[n])
    lu = factor(normal_matrix(A, P, lam))
    u0 = lu.solve(lam ** 2 * (PH @ d))
    u1 = lu.solve(A.conj().T @ e)
    a = np.concatenate([A @ u1 - e, lam * (P @ u1)])
    c = np.concatenate([-(A @ u0), lam * (d - P @ u0)])
    alpha = complex(np.vdot(a, c) / np.vdot(a, a))
    return u0 + alpha * u1, alpha


def objective_grad_offgrid(problem, src_xyz, rec_xyz, m_list=None, mode=None) -> Dict:
    """Objective and gradient (eqs. VarObj2, VarG2) with off-grid sources and
    receivers: system k uses e and P of `offgrid_operators` at src_xyz[k] and
    rec_xyz[k] (its own rec and src cell indices are not used)."""
    mode = mode or problem.mode
    m_list = problem.m if m_list is None else m_list
    grads = [np.zeros(g.n) for g in problem.grids]
    ns = len(problem.systems)
    Js, alphas, us = np.zeros(ns), np.zeros(ns, complex), [None] * ns
    for k, s in enumerate(problem.systems):
        g = problem.grids[s.grid]
        A = helmholtz(g, m_list[s.grid], s.omega)
        e, P = offgrid_operators(g, src_xyz[k], rec_xyz[k])
        d = np.asarray(s.d, dtype=np.complex128)
        if mode == KNOWN:
            alpha = complex(s.alpha)
            u = solve_known(A, P, s.lam, alpha, e, d)
        else:
            u, alpha = solve_estimate_general(A, P, s.lam, e, d)
        r1 = A @ u - alpha * e
        r2 = P @ u - d
        Js[k] = float(np.vdot(r1, r1).real + s.lam ** 2 * np.vdot(r2, r2).real)
        alphas[k] = alpha
        grads[s.grid] += 2.0 * s.omega ** 2 * np.real(np.conj(u) * r1)
        us[k] = u
    return dict(J=float(Js.sum()), J_sys=Js, alpha=alphas, u=us,
                g=[gr.reshape(g.shape) for gr, g in zip(grads, problem.grids)])
