"""Pins of the CPU oracle against facts fixed by the paper or by mathematics
(closed forms, textbook/library routines, special cases, invariants, brute
force).  None of these re-types the oracle's own formula: each checks it
through a different route, chosen so that a dropped term, a wrong sign, a
conjugate-vs-transpose slip or a transposed operand fails at least one test.
"""
import dataclasses
import json
import os

import numpy as np
import pytest
import scipy.fft
import scipy.sparse as sp
import scipy.sparse.linalg as spl

import oracle
import wri_synth
from wri_synth import Grid

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed=0):
    return np.random.default_rng(seed)


def _crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _dst_eigs(grid):
    """Eigenvalues of the zero-ghost 7-point Laplacian on the DST-I basis."""
    def one(n):
        k = np.arange(1, n + 1)
        return -(4.0 / grid.h ** 2) * np.sin(np.pi * k / (2.0 * (n + 1))) ** 2
    lz, ly, lx = one(grid.nz), one(grid.ny), one(grid.nx)
    return lz[:, None, None] + ly[None, :, None] + lx[None, None, :]


def _dst(u, grid):
    return scipy.fft.dstn(u.reshape(grid.shape), type=1, norm="ortho")


def _idst(U, grid):
    return scipy.fft.idstn(U, type=1, norm="ortho").reshape(-1)


# --------------------------------------------------------------------------
# Operator pins
# --------------------------------------------------------------------------

def test_laplacian_matches_dst_closed_form():
    """L_h is diagonalised by the 3D DST-I with eigenvalues
    -(4/h^2) sum sin^2(pi k / (2(n+1))) (textbook)."""
    g = Grid(7, 5, 6, 12.5, 0, 1500.0)
    u = _crandn(_rng(1), g.n)
    ref = _idst(_dst(u, g) * _dst_eigs(g), g)
    np.testing.assert_allclose(oracle.laplacian(g) @ u, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_helmholtz_bruteforce_small():
    """A assembled by explicit neighbour loops on a 3x4x5 grid (brute force)."""
    g = Grid(3, 4, 5, 7.0, 1, 1700.0)
    rng = _rng(2)
    m = rng.uniform(1e-7, 4e-7, g.n)
    om = 2 * np.pi * 7.0
    b = oracle.sponge(g)
    A = oracle.helmholtz(g, m, om).toarray()
    B = np.zeros((g.n, g.n), complex)
    for z in range(g.nz):
        for y in range(g.ny):
            for x in range(g.nx):
                c = (z * g.ny + y) * g.nx + x
                B[c, c] = -6.0 / g.h ** 2 + om ** 2 * m[c] - 1j * om * b[c]
                for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    xx, yy, zz = x + dx, y + dy, z + dz
                    if 0 <= xx < g.nx and 0 <= yy < g.ny and 0 <= zz < g.nz:
                        B[c, (zz * g.ny + yy) * g.nx + xx] = 1.0 / g.h ** 2
    np.testing.assert_allclose(A, B, rtol=0, atol=1e-15)


def test_sponge_zero_inside_and_damps():
    """b = 0 away from the faces, b > 0 on them, b = 0 everywhere when nb = 0;
    and the damping term dissipates: Im<u, A u> = -omega sum b |u|^2 <= 0 for
    every u (L_h + omega^2 m is real symmetric)."""
    g = Grid(20, 18, 16, 10.0, 4, 1500.0)
    b = oracle.sponge(g).reshape(g.shape)
    assert np.all(b[4:-4, 4:-4, 4:-4] == 0.0)
    assert np.all(b[0] > 0) and np.all(b[:, :, 0] > 0) and np.all(b >= 0)
    assert np.all(oracle.sponge(Grid(5, 5, 5, 10.0, 0, 1500.0)) == 0.0)
    A = oracle.helmholtz(g, np.full(g.n, 1 / 2000.0 ** 2), 2 * np.pi * 6)
    rng = _rng(3)
    for _ in range(3):
        u = _crandn(rng, g.n)
        assert np.vdot(u, A @ u).imag < 0.0


def test_sponge_values_at_named_cells():
    """Values of the damping reading b = (2 d0 / v_ref^2) sum_axes (delta/nb)^2,
    d0 = 3 v_ref ln(1000) / (2 nb h), worked out by hand for nb = 3, h = 10 m,
    v_ref = 1500 m/s:  d0 = 3*1500*ln(1000)/60 = 225 ln 10, so
    2 d0 / v_ref^2 = 450 ln 10 / 2.25e6 = 2e-4 ln 10.  On a 12 x 11 x 10 grid the
    depth into the sponge along an axis of n cells is 3, 2, 1 at i = 0, 1, 2 and
    at i = n-1, n-2, n-3, and 0 for 3 <= i <= n-4 (the sponge is nb cells thick;
    an off-by-one such as nb-1-i or a wrong d0 constant fails here)."""
    g = Grid(12, 11, 10, 10.0, 3, 1500.0)
    b = oracle.sponge(g).reshape(g.shape)      # (z, y, x)
    k = 2e-4 * np.log(10.0)
    interior = (5, 5, 5)
    cases = {
        # (z, y, x): sum of (delta/3)^2 over the three axes
        (5, 5, 0): 1.0,                 # x-face, outermost cell (depth 3)
        (5, 5, 1): 4.0 / 9.0,           # depth 2
        (5, 5, 2): 1.0 / 9.0,           # depth 1
        (5, 5, 3): 0.0,                 # first interior cell next to the x-face
        (5, 5, 11): 1.0,                # opposite x-face (n = 12: i = 11, 10, 9, 8)
        (5, 5, 10): 4.0 / 9.0,
        (5, 5, 9): 1.0 / 9.0,
        (5, 5, 8): 0.0,
        (5, 0, 5): 1.0,                 # y-face
        (5, 8, 5): 1.0 / 9.0,           # n = 11: depth 1 at i = 8
        (5, 7, 5): 0.0,
        (9, 5, 5): 1.0,                 # z-face, n = 10: depth 3 at i = 9
        (6, 5, 5): 0.0,
        (5, 0, 0): 2.0,                 # x-y edge, both depth 3
        (0, 1, 2): 1.0 + 4.0 / 9.0 + 1.0 / 9.0,   # corner region, depths 3 (z), 2 (y), 1 (x)
        (0, 0, 0): 3.0,                 # corner
        (9, 10, 11): 3.0,               # opposite corner
        interior: 0.0,
    }
    for (z, y, x), q in cases.items():
        assert abs(b[z, y, x] - k * q) <= 1e-14 * k, ((z, y, x), b[z, y, x], k * q)


def test_sponge_round_trip_attenuation_is_one_in_a_thousand():
    """Independent route to the sponge constant: b = 2 d / v^2 turns the damped
    wave equation u_tt + 2 d u_t = v^2 Lap u into A = Lap + omega^2 m - i omega b
    (m = 1/v^2, transform with exp(-i omega t)), so d is an amplitude decay rate
    per second.  A plane wave crossing the layer and coming back loses
    exp(-2 int d dx / v); the quadratic profile d(x) = d0 (x/L)^2 with
    d0 = 3 v ln(1000) / (2 L) gives int d dx = d0 L / 3, a round-trip factor of
    exactly 1e-3.  The cell sum of the oracle's values (depths 1..nb, cell width
    h, L = nb h) approaches that integral as nb grows (midpoint-like error
    O(1/nb))."""
    v = 1500.0
    ratio = {}
    for nb in (50, 100, 200):
        g = Grid(2 * nb + 2, 1, 1, 7.5, nb, v)
        b = oracle.sponge(g).reshape(-1)
        # along x only; y and z have one cell each (the sponge of the thin
        # axes is the same constant in every cell and cancels below)
        bx = b - b[nb]                      # cell nb is the first interior cell along x
        d = bx[:nb] * v ** 2 / 2.0          # decay rate per cell, depths nb..1
        factor = np.exp(-2.0 * np.sum(d) * g.h / v)
        ratio[nb] = np.log(factor) / np.log(1e-3)
        assert abs(ratio[nb] - 1.0) < 2.0 / nb, (nb, ratio[nb])
    # the cell sum converges to the integral at first order in 1/nb: one
    # Richardson step removes that term and must land on the design value
    assert abs(2.0 * ratio[200] - ratio[100] - 1.0) < 1e-3, ratio


def test_point_source_is_outgoing_wave():
    """Convention pin (the paper's source tables use exp(-i 2 pi f t0), i.e.
    forward transform with exp(-i omega t)).  Under that convention an
    outgoing wave is exp(-i k r): the solution of A u = e_s in a homogeneous
    medium with the sponge must track -h^3 exp(-i k r) / (4 pi r), and not the
    incoming exp(+i k r); its shell-averaged amplitude decays through the
    sponge."""
    n, h, v, f = 28, 10.0, 1500.0, 18.75       # 8 points per wavelength
    g = Grid(n, n, n, h, 6, v)
    m = np.full(g.n, 1.0 / v ** 2)
    A = oracle.helmholtz(g, m, 2 * np.pi * f)
    c = n // 2
    src = (c * n + c) * n + c
    u = oracle.plain_helmholtz_solution(A, oracle.unit_vector(g.n, src)).reshape(g.shape)
    zz, yy, xx = np.meshgrid(*(np.arange(n),) * 3, indexing="ij")
    r = h * np.sqrt((xx - c) ** 2 + (yy - c) ** 2 + (zz - c) ** 2)
    sel = (r >= 3 * h) & (r <= 7 * h)
    k = 2 * np.pi * f / v
    out = -h ** 3 * np.exp(-1j * k * r[sel]) / (4 * np.pi * r[sel])
    inc = -h ** 3 * np.exp(+1j * k * r[sel]) / (4 * np.pi * r[sel])
    us = u[sel]
    corr = lambda a, b: abs(np.vdot(a, b)) / (np.linalg.norm(a) * np.linalg.norm(b))
    assert corr(us, out) > 0.95
    assert corr(us, inc) < 0.6
    # amplitude within 15 % of the continuum Green's function at these distances
    assert 0.85 < np.linalg.norm(us) / np.linalg.norm(out) < 1.15
    # decay through the sponge: mean |u| on shells
    shells = [np.abs(u[(r >= a * h) & (r < (a + 1) * h)]).mean() for a in (8, 10, 12, 14)]
    assert all(s1 > s2 for s1, s2 in zip(shells, shells[1:]))


# --------------------------------------------------------------------------
# KNOWN-source solve
# --------------------------------------------------------------------------

def test_known_solve_matches_dst_closed_form_complex_shift():
    """Homogeneous m, constant damping b (complex diagonal shift), P = I:
    the normal equations diagonalise under DST-I,
    u_k = (conj(a_k) q_k + lam^2 d_k) / (|a_k|^2 + lam^2),
    a_k = omega^2 m - i omega b + eig_k(L_h).  The complex shift makes A
    non-Hermitian, so conjugate-vs-transpose mistakes fail here."""
    g = Grid(6, 7, 5, 10.0, 0, 1500.0)
    om, m0, b0, lam = 2 * np.pi * 9.0, 1 / 1900.0 ** 2, 2e-5, 0.07
    rng = _rng(4)
    src = 37
    alpha = complex(_crandn(rng, 1)[0])
    d = _crandn(rng, g.n)
    A = oracle.helmholtz(g, np.full(g.n, m0), om, b=np.full(g.n, b0))
    P = oracle.restriction(g.n, np.arange(g.n))
    u = oracle.solve_known(A, P, lam, alpha, oracle.unit_vector(g.n, src), d)
    a = om ** 2 * m0 - 1j * om * b0 + _dst_eigs(g)
    q = np.zeros(g.n, complex)
    q[src] = alpha
    # DST-I ortho is real, symmetric and orthogonal: transform real/imag alike
    Q = lambda v: _dst(v.real, g) + 1j * _dst(v.imag, g)
    Qi = lambda V: _idst(V.real, g) + 1j * _idst(V.imag, g)
    U = (np.conj(a) * Q(q) + lam ** 2 * Q(d)) / (np.abs(a) ** 2 + lam ** 2)
    ref = Qi(U)
    assert np.linalg.norm(u - ref) / np.linalg.norm(ref) < 1e-11


def test_known_lambda_to_zero_gives_plain_helmholtz():
    """lam -> 0: u -> A^{-1} (alpha e) (reduced FWI wavefield, eq. PDEsolve),
    error O(lam^2)."""
    p = wri_synth.custom_problem((9, 8, 7), nb=2, n_src=1, n_rec=6, seed=5)
    A, P, e = oracle.system_operators(p, 0)
    s = p.systems[0]
    uref = oracle.plain_helmholtz_solution(A, s.alpha * e)
    errs = []
    for lam in (1e-4, 1e-5, 1e-6):
        u = oracle.solve_known(A, P, lam, s.alpha, e, s.d)
        errs.append(np.linalg.norm(u - uref) / np.linalg.norm(uref))
    assert errs[-1] < 1e-6
    assert 50 < errs[0] / errs[1] < 200 and 50 < errs[1] / errs[2] < 200


# --------------------------------------------------------------------------
# Source-estimating (source-free) solve, eq. SimpObj
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def small_problem():
    return wri_synth.custom_problem((10, 9, 8), nb=2, n_src=2, n_rec=7, seed=6, lam=0.05)


def test_estimate_three_routes_agree(small_problem):
    p = small_problem
    for k in range(len(p.systems)):
        A, P, e = oracle.system_operators(p, k)
        s = p.systems[k]
        outs = [oracle.solve_estimate(A, P, s.lam, s.src, s.d, route=r)
                for r in ("augmented", "varpro", "projected")]
        for u, a in outs[1:]:
            assert np.linalg.norm(u - outs[0][0]) / np.linalg.norm(outs[0][0]) < 1e-10
            assert abs(a - outs[0][1]) / abs(outs[0][1]) < 1e-10


def test_estimate_alpha_stationarity(small_problem):
    """At the optimum alpha = e^H A u / e^H e = (A u)[src]; hence the gradient
    vanishes at the source cell."""
    p = small_problem
    out = oracle.objective_grad(p, mode=oracle.ESTIMATE)
    for k, s in enumerate(p.systems):
        A, P, e = oracle.system_operators(p, k)
        au = (A @ out["u"][k])[s.src]
        assert abs(au - out["alpha"][k]) <= 1e-12 * abs(au)
        gk = oracle.gradient_term(s.omega, out["u"][k], A, out["alpha"][k], e)
        assert abs(gk[s.src]) <= 1e-9 * np.abs(gk).max()


def test_estimate_lambda_to_zero_gives_fwi_source_estimate():
    """lam -> 0: alpha -> (P G)^H d / ||P G||^2 with G = A^{-1} e (the classic
    frequency-domain FWI source estimate), error O(lam^2)."""
    p = wri_synth.custom_problem((9, 8, 7), nb=2, n_src=1, n_rec=6, seed=7)
    A, P, e = oracle.system_operators(p, 0)
    s = p.systems[0]
    G = P @ oracle.plain_helmholtz_solution(A, e)
    aref = np.vdot(G, s.d) / np.vdot(G, G)
    errs = [abs(oracle.solve_estimate(A, P, lam, s.src, s.d)[1] - aref) / abs(aref)
            for lam in (1e-4, 1e-5, 1e-6)]
    assert errs[-1] < 1e-6
    assert 50 < errs[0] / errs[1] < 200


def test_noise_free_data_recovers_true_source_and_zero_gradient():
    """d = P A(m)^{-1} (alpha_t e) exactly and the same m: the minimum is J = 0
    at (u, alpha) = (A^{-1} alpha_t e, alpha_t), so g = 0."""
    p = wri_synth.custom_problem((10, 9, 8), nb=2, n_src=2, n_rec=8, seed=8, data="none")
    p.m_true = [m.copy() for m in p.m]
    p = p.with_data(oracle.observed_data(p, noise=0.0))
    out = oracle.objective_grad(p, mode=oracle.ESTIMATE)
    for k, s in enumerate(p.systems):
        assert abs(out["alpha"][k] - s.alpha) / abs(s.alpha) < 1e-9
        A, P, e = oracle.system_operators(p, k)
        uref = oracle.plain_helmholtz_solution(A, s.alpha * e)
        assert np.linalg.norm(out["u"][k] - uref) / np.linalg.norm(uref) < 1e-9
    dn = sum(np.vdot(s.d, s.d).real for s in p.systems)
    assert out["J"] < 1e-18 * dn
    # gradient relative to the size of one system's gradient at a perturbed model
    pert = [m * 1.05 for m in p.m]
    gref = np.abs(oracle.objective_grad(p, m_list=pert)["g"][0]).max()
    assert np.abs(out["g"][0]).max() < 1e-8 * gref


def test_normal_equations_hold_with_explicit_S(small_problem):
    """Brute force: assemble S = [[A, -e], [lam P, 0]] explicitly and check
    ||S^H (b - S x)|| / ||S^H b|| ~ 0 at the oracle's minimiser, for both
    modes (KNOWN: S = [A; lam P], b = [alpha e; lam d])."""
    p = small_problem
    for k, s in enumerate(p.systems):
        A, P, e = oracle.system_operators(p, k)
        n = A.shape[0]
        ecol = sp.csr_matrix(([1.0 + 0j], ([s.src], [0])), shape=(n, 1))
        S = sp.bmat([[A, -ecol], [s.lam * P, None]]).tocsr()
        b = np.concatenate([np.zeros(n), s.lam * s.d])
        u, a = oracle.solve_estimate(A, P, s.lam, s.src, s.d)
        x = np.concatenate([u, [a]])
        res = np.linalg.norm(S.conj().T @ (b - S @ x)) / np.linalg.norm(S.conj().T @ b)
        assert res < 1e-10
        assert abs(oracle.normal_residual(A, P, s.lam, s.src, oracle.ESTIMATE, 0, s.d, u, a) - res) < 1e-10
        SK = sp.bmat([[A], [s.lam * P]]).tocsr()
        bK = np.concatenate([s.alpha * e, s.lam * s.d])
        uK = oracle.solve_known(A, P, s.lam, s.alpha, e, s.d)
        resK = np.linalg.norm(SK.conj().T @ (bK - SK @ uK)) / np.linalg.norm(SK.conj().T @ bK)
        assert resK < 1e-10


def test_apply_S_adjoint(small_problem):
    """<S x, y> = <x, S^H y> for the matrix-free S used by the reference CGLS."""
    p = small_problem
    rng = _rng(9)
    s = p.systems[0]
    A, P, e = oracle.system_operators(p, 0)
    n = A.shape[0]
    for mode, nx in ((oracle.KNOWN, n), (oracle.ESTIMATE, n + 1)):
        x = _crandn(rng, nx)
        y = _crandn(rng, n + s.rec.size)
        lhs = np.vdot(y, oracle.apply_S(A, P, s.lam, s.src, mode, x))
        rhs = np.vdot(oracle.apply_SH(A, P, s.lam, s.src, mode, y), x)
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_paper_scaling_lsqr_on_printed_S():
    """The paper's own compact form (eqs. CmpctWRIobj, Sandb): S with lambda_p
    on the PDE rows, b = [0; d].  scipy's LSQR on that printed system gives the
    same (u, alpha) as the oracle at lam = 1/lambda_p, and
    J = 2 f_2 / lambda_p^2."""
    p = wri_synth.custom_problem((8, 7, 6), nb=2, n_src=1, n_rec=6, seed=10)
    A, P, e = oracle.system_operators(p, 0)
    s = p.systems[0]
    lam_p = 4.0
    Sp, bp = oracle.paper_S_and_b(A, P, s.src, s.d, lam_p)
    sol = spl.lsqr(Sp, bp, atol=1e-15, btol=1e-15, conlim=1e12, iter_lim=200000)[0]
    u, a = oracle.solve_estimate(A, P, 1.0 / lam_p, s.src, s.d)
    assert np.linalg.norm(sol[:-1] - u) / np.linalg.norm(u) < 1e-7
    assert abs(sol[-1] - a) / abs(a) < 1e-7
    t1, t2 = oracle.objective_terms(A, P, 1.0 / lam_p, u, a, e, s.d)
    f2 = oracle.paper_f2(A, P, lam_p, u, a, e, s.d)
    assert abs((t1 + t2) - 2.0 * f2 / lam_p ** 2) < 1e-12 * (t1 + t2)


# --------------------------------------------------------------------------
# Objective and gradient (eqs. VarObj2, VarG2)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("mode", ["estimate", "known"])
def test_gradient_matches_central_differences(mode):
    """Central differences of the exact reduced objective (direct solves,
    complex128) at a handful of cells, relative step 1e-4, plus a Taylor test
    along a random direction: |J(m + t dm) - J(m) - t g.dm| = O(t^2)."""
    p = wri_synth.custom_problem((9, 8, 7), nb=2, n_src=2, n_rec=7, seed=11, freqs=(6.0, 9.0),
                                 lam=0.03)
    out = oracle.objective_grad(p, mode=mode)
    g = out["g"][0].reshape(-1)
    m = p.m[0].reshape(-1)
    rng = _rng(12)
    cells = list(rng.choice(np.arange(m.size), 4, replace=False)) + [int(np.argmax(np.abs(g)))]
    for c in cells:
        step = 1e-4 * m[c]
        mp, mm = m.copy(), m.copy()
        mp[c] += step
        mm[c] -= step
        Jp = oracle.objective_grad(p, m_list=[mp.reshape(p.grids[0].shape)], mode=mode, return_fields=False)["J"]
        Jm = oracle.objective_grad(p, m_list=[mm.reshape(p.grids[0].shape)], mode=mode, return_fields=False)["J"]
        fd = (Jp - Jm) / (2 * step)
        assert abs(fd - g[c]) <= 1e-6 * np.abs(g).max(), (c, fd, g[c])
    dm = rng.standard_normal(m.size) * m * 0.01
    J0 = out["J"]
    res = []
    for t in (1.0, 0.5, 0.25):
        Jt = oracle.objective_grad(p, m_list=[(m + t * dm).reshape(p.grids[0].shape)], mode=mode,
                                   return_fields=False)["J"]
        res.append(abs(Jt - J0 - t * g @ dm))
    assert 3.0 < res[0] / res[1] < 5.0 and 3.0 < res[1] / res[2] < 5.0


def test_scaling_laws(small_problem):
    """ESTIMATE: d -> c d scales (u, alpha) by c and (J, g) by |c|^2.
    KNOWN: (d, alpha) -> c (d, alpha) does the same."""
    p = small_problem
    c = 0.3 - 1.7j
    base_e = oracle.objective_grad(p, mode="estimate")
    base_k = oracle.objective_grad(p, mode="known")
    q = p.with_data([c * s.d for s in p.systems])
    from dataclasses import replace
    q = replace(q, systems=[replace(s, alpha=c * s.alpha) for s in q.systems])
    sc_e = oracle.objective_grad(q, mode="estimate")
    sc_k = oracle.objective_grad(q, mode="known")
    for base, sc in ((base_e, sc_e), (base_k, sc_k)):
        assert abs(sc["J"] - abs(c) ** 2 * base["J"]) < 1e-10 * sc["J"]
        np.testing.assert_allclose(sc["g"][0], abs(c) ** 2 * base["g"][0], rtol=0,
                                   atol=1e-10 * np.abs(sc["g"][0]).max())
        for u1, u0 in zip(sc["u"], base["u"]):
            assert np.linalg.norm(u1 - c * u0) < 1e-10 * np.linalg.norm(u1)
    np.testing.assert_allclose(sc_e["alpha"], c * base_e["alpha"], rtol=1e-10)


# --------------------------------------------------------------------------
# Reference CGLS (Algorithm 1 read as CG on the normal equations)
# --------------------------------------------------------------------------

def test_cgls_iterates_equal_lsqr_iterates(small_problem):
    """CGLS and LSQR (Paige & Saunders, cited by the paper) generate the same
    Krylov iterates in exact arithmetic: compare with scipy's LSQR after k
    steps on the explicitly assembled S."""
    p = small_problem
    s = p.systems[0]
    A, P, e = oracle.system_operators(p, 0)
    n = A.shape[0]
    ecol = sp.csr_matrix(([1.0 + 0j], ([s.src], [0])), shape=(n, 1))
    S = sp.bmat([[A, -ecol], [s.lam * P, None]]).tocsr()
    b = np.concatenate([np.zeros(n), s.lam * s.d])
    for k in (1, 3, 8):
        xl = spl.lsqr(S, b, atol=0, btol=0, conlim=0, iter_lim=k)[0]
        out = oracle.cgls(A, P, s.lam, s.src, "estimate", 0, s.d, rtol=0.0, maxiter=k)
        xc = np.concatenate([out["u"], [out["alpha"]]])
        assert out["iters"] == k
        # rounding separates the two recurrences slowly (~1e-8 after 8 steps)
        assert np.linalg.norm(xc - xl) / np.linalg.norm(xl) < 1e-6


def test_cgls_converges_to_exact_minimiser():
    p = wri_synth.custom_problem((8, 7, 6), nb=2, n_src=1, n_rec=6, seed=13, lam=0.12)
    s = p.systems[0]
    A, P, e = oracle.system_operators(p, 0)
    u, a = oracle.solve_estimate(A, P, s.lam, s.src, s.d)
    out = oracle.cgls(A, P, s.lam, s.src, "estimate", 0, s.d, rtol=1e-12, maxiter=100000)
    assert out["status"] == "converged"
    assert np.linalg.norm(out["u"] - u) / np.linalg.norm(u) < 1e-8
    assert abs(out["alpha"] - a) / abs(a) < 1e-8
    # the recurred stopping quantity agrees with the true normal residual
    tr = oracle.normal_residual(A, P, s.lam, s.src, "estimate", 0, s.d, out["u"], out["alpha"])
    assert tr < 1e-10
    uk = oracle.cgls(A, P, s.lam, s.src, "known", s.alpha, s.d, rtol=1e-12, maxiter=100000)
    assert np.linalg.norm(uk["u"] - oracle.solve_known(A, P, s.lam, s.alpha, e, s.d)) < 1e-8 * np.linalg.norm(uk["u"])


def test_cgls_zero_rhs_and_max_iter():
    p = wri_synth.custom_problem((6, 6, 6), nb=1, n_src=1, n_rec=4, seed=14)
    s = p.systems[0]
    A, P, e = oracle.system_operators(p, 0)
    z = oracle.cgls(A, P, s.lam, s.src, "estimate", 0, np.zeros_like(s.d), rtol=1e-6, maxiter=10)
    assert z["status"] == "zero_rhs" and z["iters"] == 0 and not np.any(z["u"])
    one = oracle.cgls(A, P, s.lam, s.src, "estimate", 0, s.d, rtol=1e-12, maxiter=1)
    assert one["status"] == "max_iter" and one["iters"] == 1


# --------------------------------------------------------------------------
# The paper's printed numbers (source tables): convention pins for the inputs
# --------------------------------------------------------------------------

def test_paper_source_tables():
    with open(os.path.join(GOLDEN, "paper_source_tables.json")) as f:
        tab = json.load(f)
    cam = tab["camembert"]
    at = np.array([wri_synth.alpha_true(f) for f in cam["freqs_hz"]])
    a0 = np.array([wri_synth.alpha_initial(f) for f in cam["freqs_hz"]])
    np.testing.assert_allclose(at, [complex(*z) for z in cam["alpha_true"]], atol=0.06)
    np.testing.assert_allclose(a0, [complex(*z) for z in cam["alpha_initial"]], atol=0.06)
    err = 100 * np.linalg.norm(a0 - at) / np.linalg.norm(at)
    assert abs(err - cam["rel_err_initial_pct"]) < 0.15
    vsp = tab["vsp"]
    at5 = wri_synth.alpha_true(5.0)
    a05 = wri_synth.alpha_initial(5.0)
    assert abs(100 * abs(a05 - at5) / abs(at5) - vsp["rel_err_initial_pct"]) < 0.15
    # the printed final estimates reproduce the printed final errors
    af = np.array([complex(*z) for z in cam["alpha_final"]])
    atp = np.array([complex(*z) for z in cam["alpha_true"]])
    assert abs(100 * np.linalg.norm(af - atp) / np.linalg.norm(atp) - cam["rel_err_final_pct"]) < 0.15


def test_cgls_column_scaling_keeps_minimiser():
    """Scaling the source column of S (-c e, unknown alpha/c) is a right
    diagonal preconditioner: the converged (u, alpha) must not depend on c."""
    p = wri_synth.custom_problem((8, 7, 6), nb=2, n_src=1, n_rec=6, seed=19, lam=0.12)
    s = p.systems[0]
    A, P, e = oracle.system_operators(p, 0)
    u, a = oracle.solve_estimate(A, P, s.lam, s.src, s.d)
    for c in (1.0, 42 ** 0.5 / p.grids[0].h ** 2, 7.0):
        out = oracle.cgls(A, P, s.lam, s.src, "estimate", 0, s.d, rtol=1e-12, maxiter=100000, alpha_scale=c)
        assert np.linalg.norm(out["u"] - u) / np.linalg.norm(u) < 1e-8
        assert abs(out["alpha"] - a) / abs(a) < 1e-8


def test_matrix_free_helmholtz_equals_assembled_operator():
    """The full-size helpers (matrix-free A u, A^H u and single stencil rows)
    reproduce the assembled sparse operator on a ragged grid with a sponge."""
    p = wri_synth.custom_problem((7, 5, 6), nb=2, n_src=1, n_rec=3, seed=31)
    g = p.grids[0]
    omega = p.systems[0].omega
    A = oracle.helmholtz(g, p.m[0], omega)
    rng = np.random.default_rng(3)
    u = rng.standard_normal(g.n) + 1j * rng.standard_normal(g.n)
    assert np.allclose(oracle.helmholtz_apply(g, p.m[0], omega, u), A @ u, rtol=1e-13, atol=1e-12 * np.abs(A @ u).max())
    AH = A.conj().T.tocsr()
    assert np.allclose(oracle.helmholtz_apply(g, p.m[0], omega, u, adjoint=True), AH @ u, rtol=1e-13,
                       atol=1e-12 * np.abs(AH @ u).max())
    cells = np.array([0, 1, g.nx - 1, g.nx * g.ny + 3, g.n - 1, g.n // 2])
    cols, vals = oracle.helmholtz_rows(g, p.m[0], omega, cells)
    dense = A.toarray()
    for i, c in enumerate(cells):
        row = np.zeros(g.n, dtype=np.complex128)
        np.add.at(row, cols[i], vals[i])
        assert np.allclose(row, dense[c], rtol=1e-14, atol=1e-14 * np.abs(dense[c]).max())


# --------------------------------------------------------------------------
# outer loop: TV, l-BFGS, Algorithm 2
# --------------------------------------------------------------------------

def test_tv_closed_forms():
    """Constant model: every cell contributes eps.  A ramp along x: the
    interior cells contribute sqrt((a/h)^2 + eps^2), the last x-column eps."""
    g = Grid(7, 5, 4, 10.0, 0, 1500.0)
    eps = 1e-6
    assert oracle.tv(g, np.full(g.n, 3.3e-7), eps) == pytest.approx(g.n * eps, rel=1e-12)
    a = 2.0e-9
    ramp = (a * np.arange(g.nx))[None, None, :] * np.ones(g.shape)
    want = (g.nx - 1) * g.ny * g.nz * np.sqrt((a / g.h) ** 2 + eps ** 2) + g.ny * g.nz * eps
    assert oracle.tv(g, ramp, eps) == pytest.approx(want, rel=1e-12)
    # the ramp along z instead (axis order check)
    rz = (a * np.arange(g.nz))[:, None, None] * np.ones(g.shape)
    want_z = (g.nz - 1) * g.ny * g.nx * np.sqrt((a / g.h) ** 2 + eps ** 2) + g.ny * g.nx * eps
    assert oracle.tv(g, rz, eps) == pytest.approx(want_z, rel=1e-12)


def test_tv_gradient_matches_finite_differences():
    g = Grid(5, 4, 6, 10.0, 0, 1500.0)
    rng = np.random.default_rng(5)
    m = 3e-7 * (1.0 + 0.1 * rng.standard_normal(g.n))
    eps = 1e-10
    gr = oracle.tv_grad(g, m, eps)
    h = 1e-11
    for c in rng.choice(g.n, 12, replace=False):
        mp, mm = m.copy(), m.copy()
        mp[c] += h
        mm[c] -= h
        fd = (oracle.tv(g, mp, eps) - oracle.tv(g, mm, eps)) / (2 * h)
        assert gr[c] == pytest.approx(fd, rel=1e-5, abs=1e-9 * np.abs(gr).max())
    assert np.allclose(oracle.tv_grad(g, np.full(g.n, 2e-7), eps), 0.0)


def test_lbfgs_two_loop_secant_and_exact_inverse():
    """With pairs y = A s the recursion satisfies the secant condition for the
    newest pair; when the s_i are A-conjugate and span the space, H = A^-1."""
    rng = np.random.default_rng(2)
    n = 6
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.linspace(1.0, 9.0, n)
    A = Q @ np.diag(lam) @ Q.T
    g = rng.standard_normal(n)
    assert np.allclose(oracle.lbfgs_two_loop(g, [], 0.37), 0.37 * g)
    pairs = [(s, A @ s) for s in rng.standard_normal((3, n))]
    H_y = oracle.lbfgs_two_loop(pairs[-1][1], pairs, 0.5)
    assert np.allclose(H_y, pairs[-1][0], rtol=1e-12, atol=1e-12)
    eig_pairs = [(Q[:, i], A @ Q[:, i]) for i in range(n)]
    Hg = oracle.lbfgs_two_loop(g, eig_pairs, 0.123)
    assert np.allclose(Hg, np.linalg.solve(A, g), rtol=1e-10, atol=1e-12)


def test_inexact_objective_matches_direct_at_tight_tolerance():
    p = wri_synth.custom_problem((9, 8, 7), nb=2, n_src=2, n_rec=6, seed=41, freqs=(7.0,))
    ex = oracle.objective_grad(p, return_fields=False)
    J, g, iters = oracle.inexact_objective_grad(p, p.m, rtol=1e-12)
    assert J == pytest.approx(ex["J"], rel=1e-8)
    assert np.allclose(g[0], ex["g"][0].reshape(-1), rtol=1e-6, atol=1e-8 * np.abs(g[0]).max())
    assert min(iters) > 0


def test_awri_outer_loop_behaviour():
    """Algorithm 2 with exact solves: the first trial moves by step0 * max|m|
    in the largest-gradient cell, accepted F never increases, and a rejection
    halves eps and re-evaluates at the same model."""
    p = wri_synth.custom_problem((10, 9, 8), nb=2, n_src=3, n_rec=12, seed=43, freqs=(6.0, 9.0))
    m0 = p.m[0].reshape(-1)
    out = oracle.awri(p, m0, gamma=1e-8, eps0=1e-3, n_outer=3, memory=3, eps_tv=1e-9, step0=0.02)
    h = out["history"]
    acc = [r["F"] for r in h if r["accepted"]]
    assert len(acc) >= 2
    assert all(b <= a * (1 + 1e-12) for a, b in zip(acc, acc[1:]))
    # the first trial, by hand: m - (step0 max|m| / max|g|) g with g = gradient of J + gamma TV
    o = oracle.objective_grad(p, return_fields=False)
    gfull = o["g"][0].reshape(-1) + 1e-8 * oracle.tv_grad(p.grids[0], m0, 1e-9)
    step = 0.02 * np.abs(m0).max() / np.abs(gfull).max() * gfull
    Ftrial = oracle.objective_grad(p, [(m0 - step).reshape(p.grids[0].shape)], return_fields=False)["J"] + \
        1e-8 * oracle.tv(p.grids[0], m0 - step, 1e-9)
    assert h[0]["F"] == pytest.approx(o["J"] + 1e-8 * oracle.tv(p.grids[0], m0, 1e-9), rel=1e-12)
    assert h[1]["F"] == pytest.approx(Ftrial, rel=1e-10)
    # every rejected trial is followed by a re-evaluation at half the tolerance
    for i, r in enumerate(h[:-1]):
        if not r["accepted"]:
            assert h[i + 1].get("reeval") and h[i + 1]["eps"] == pytest.approx(0.5 * r["eps"])


# --------------------------------------------------------------------------
# Reduced FWI baseline (eqs. FWI, PDEsolve, FWI2)
# --------------------------------------------------------------------------

def _fwi_problem(seed=31, mode=oracle.ESTIMATE):
    p = wri_synth.custom_problem((9, 8, 7), nb=2, n_src=2, n_rec=7, seed=seed, freqs=(6.0, 9.0),
                                 lam=0.0, mode=mode)
    return p


@pytest.mark.parametrize("mode", ["estimate", "known"])
def test_fwi_gradient_matches_central_differences(mode):
    """Central differences of the reduced FWI objective (direct solves) at a
    handful of cells, and a Taylor test: |f(m + t dm) - f(m) - t g.dm| = O(t^2).
    A wrong sign, a missing conjugate or a dropped omega^2 in the adjoint-state
    gradient fails it; in ESTIMATE mode so does a gradient that forgets that
    alpha moves with m."""
    p = _fwi_problem(mode=mode)
    out = oracle.fwi_objective_grad(p)
    g = out["g"][0].reshape(-1)
    m = p.m[0].reshape(-1)
    sh = p.grids[0].shape
    rng = _rng(32)
    cells = list(rng.choice(np.arange(m.size), 4, replace=False)) + [int(np.argmax(np.abs(g)))]
    for c in cells:
        step = 1e-4 * m[c]
        mp, mm = m.copy(), m.copy()
        mp[c] += step
        mm[c] -= step
        fd = (oracle.fwi_objective_grad(p, m_list=[mp.reshape(sh)])["f"] -
              oracle.fwi_objective_grad(p, m_list=[mm.reshape(sh)])["f"]) / (2 * step)
        assert abs(fd - g[c]) <= 1e-6 * np.abs(g).max(), (c, fd, g[c])
    dm = rng.standard_normal(m.size) * m * 0.01
    res = []
    for t in (1.0, 0.5, 0.25):
        ft = oracle.fwi_objective_grad(p, m_list=[(m + t * dm).reshape(sh)])["f"]
        res.append(abs(ft - out["f"] - t * g @ dm))
    assert 3.0 < res[0] / res[1] < 5.0 and 3.0 < res[1] / res[2] < 5.0


def test_fwi_source_estimate_is_the_misfit_minimiser():
    """ESTIMATE: the weight minimises 1/2 ||alpha P A^{-1} e - d||^2 (checked by
    brute perturbation in four directions), and KNOWN with that weight gives the
    same f and the same gradient (the alpha-derivative vanishes at the optimum)."""
    p = _fwi_problem(seed=33)
    est = oracle.fwi_objective_grad(p, mode=oracle.ESTIMATE)
    for k, s in enumerate(p.systems):
        A, P, e = oracle.system_operators(p, k)
        Pw = P @ oracle.plain_helmholtz_solution(A, e)
        f = lambda a: 0.5 * np.vdot(a * Pw - s.d, a * Pw - s.d).real
        a0 = est["alpha"][k]
        assert abs(f(a0) - est["f_sys"][k]) <= 1e-12 * f(a0)
        for da in (1e-3, -1e-3, 1e-3j, -1e-3j):
            assert f(a0 + da * abs(a0)) > f(a0)
    pk = dataclasses.replace(p, mode=oracle.KNOWN, systems=[dataclasses.replace(s, alpha=complex(a))
                                                            for s, a in zip(p.systems, est["alpha"])])
    kn = oracle.fwi_objective_grad(pk)
    assert abs(kn["f"] - est["f"]) <= 1e-12 * est["f"]
    assert np.abs(kn["g"][0] - est["g"][0]).max() <= 1e-10 * np.abs(est["g"][0]).max()


def test_fwi_is_the_small_lambda_limit_of_wri():
    """With a known weight, the WRI objective and gradient (eqs. VarObj2,
    VarG2, computed by the separate normal-equation route) divided by lam^2
    tend to 2 f and 2 df/dm of reduced FWI as lam -> 0 (the PDE becomes a hard
    constraint), with errors O(lam^2).  Pins the factor 1/2, the sign and the
    adjoint field of the FWI gradient against an independent computation."""
    p = _fwi_problem(seed=34, mode=oracle.KNOWN)
    fwi = oracle.fwi_objective_grad(p)
    ef, eg = [], []
    for lam in (3e-4, 3e-5):   # smaller lam: the gradient's PDE residual drowns in cancellation
        pl = dataclasses.replace(p, systems=[dataclasses.replace(s, lam=lam) for s in p.systems])
        w = oracle.objective_grad(pl, mode=oracle.KNOWN)
        ef.append(abs(w["J"] / lam ** 2 - 2.0 * fwi["f"]) / (2.0 * fwi["f"]))
        eg.append(np.abs(w["g"][0] / lam ** 2 - 2.0 * fwi["g"][0]).max() / np.abs(2.0 * fwi["g"][0]).max())
    assert ef[-1] < 1e-5 and eg[-1] < 1e-4, (ef, eg)
    assert 30 < ef[0] / ef[1] < 300 and 30 < eg[0] / eg[1] < 300, (ef, eg)


def test_fwi_zero_at_the_data_generating_model():
    """Noise-free data from the same model: f = 0, g = 0 and, estimating the
    weight, alpha = the true weight."""
    p = wri_synth.custom_problem((10, 9, 8), nb=2, n_src=2, n_rec=8, seed=35, data="none", lam=0.0)
    p.m_true = [m.copy() for m in p.m]
    p = p.with_data(oracle.observed_data(p, noise=0.0))
    out = oracle.fwi_objective_grad(p, mode=oracle.ESTIMATE)
    for k, s in enumerate(p.systems):
        assert abs(out["alpha"][k] - s.alpha) <= 1e-10 * abs(s.alpha)
    dn = sum(np.vdot(s.d, s.d).real for s in p.systems)
    assert out["f"] <= 1e-20 * dn
    gref = np.abs(oracle.fwi_objective_grad(p, m_list=[m * 1.05 for m in p.m])["g"][0]).max()
    assert np.abs(out["g"][0]).max() <= 1e-8 * gref


def test_receiver_source_solution_is_adjoint_of_sampling():
    """Reciprocity: for the complex-symmetric A, <P A^{-1} e_s, c> (plain
    transpose) equals <e_s, A^{-1} P^T c>, i.e. the field of receiver sources
    sampled at the source equals the source's field sampled at the receivers,
    weighted by c."""
    p = _fwi_problem(seed=36)
    rng = _rng(37)
    for k, s in enumerate(p.systems):
        A, P, e = oracle.system_operators(p, k)
        c = _crandn(rng, len(s.rec))
        z = oracle.receiver_source_solution(A, p.grids[0].n, s.rec, c)
        w = oracle.plain_helmholtz_solution(A, e)
        lhs = np.sum(w[np.asarray(s.rec)] * c)
        assert abs(z[s.src] - lhs) <= 1e-10 * abs(lhs)


# --------------------------------------------------------------------------
# One model grid, per-frequency simulation grids (trilinear resampling)
# --------------------------------------------------------------------------

def test_resample_matches_scipy_linear_interpolation():
    """R m equals scipy's RegularGridInterpolator (method 'linear') at the
    simulation nodes, for grids coarser and finer than the model grid."""
    from scipy.interpolate import RegularGridInterpolator
    rng = _rng(61)
    mg = Grid(9, 7, 6, 10.0, 0, 1500.0)
    m = rng.standard_normal(mg.shape)
    axes_m = [np.arange(n) * mg.h for n in mg.shape]  # (z, y, x)
    f = RegularGridInterpolator(axes_m, m, method="linear")
    for g in (Grid(5, 4, 3, 20.0, 0, 1500.0), Grid(13, 10, 8, 6.5, 0, 1500.0), Grid(9, 7, 6, 10.0, 0, 1500.0)):
        zz, yy, xx = np.meshgrid(*[np.arange(n) * g.h for n in g.shape], indexing="ij")
        ref = f(np.stack([zz.ravel(), yy.ravel(), xx.ravel()], axis=1))
        out = oracle.resample_matrix(mg, g) @ m.reshape(-1)
        assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()


def test_resample_affine_exact_and_partition_of_unity():
    mg = Grid(8, 9, 10, 12.0, 0, 1500.0)
    g = Grid(11, 13, 15, 7.7, 0, 1500.0)
    R = oracle.resample_matrix(mg, g)
    assert np.allclose(R @ np.ones(mg.n), 1.0, atol=1e-14, rtol=0)
    assert R.data.min() >= 0.0
    z, y, x = np.meshgrid(*[np.arange(n) * mg.h for n in mg.shape], indexing="ij")
    aff = lambda x, y, z: 0.3 + 2e-3 * x - 1e-3 * y + 4e-3 * z
    zg, yg, xg = np.meshgrid(*[np.arange(n) * g.h for n in g.shape], indexing="ij")
    assert np.abs(R @ aff(x, y, z).ravel() - aff(xg, yg, zg).ravel()).max() < 1e-13
    assert abs((oracle.resample_matrix(mg, mg) - sp.identity(mg.n)).max()) < 1e-15


def test_objective_on_the_model_grid_gradient_matches_central_differences():
    """Two simulation grids (different cell sizes) tied to one model grid:
    dJ/dm_model from sum_g R_g^T g_g agrees with central differences of
    J(R_g m_model) — pins the transpose in the chain rule."""
    mgrid = Grid(8, 7, 6, 10.0, 0, 1500.0)
    rng = _rng(62)
    m_model = (1.0 / rng.uniform(1800.0, 2400.0, mgrid.shape) ** 2)
    pa = wri_synth.custom_problem((8, 7, 6), h=10.0, nb=2, n_src=1, n_rec=5, seed=63, freqs=(9.0,), lam=0.03)
    pb = wri_synth.custom_problem((5, 5, 4), h=17.0, nb=1, n_src=1, n_rec=4, seed=64, freqs=(6.0,), lam=0.03)
    sb = [dataclasses.replace(s, grid=1) for s in pb.systems]
    p = dataclasses.replace(pa, grids=[pa.grids[0], pb.grids[0]], m=[pa.m[0], pb.m[0]],
                            m_true=[pa.m_true[0], pb.m_true[0]], systems=list(pa.systems) + sb)
    out = oracle.objective_grad_model(p, mgrid, m_model)
    g = out["g"].reshape(-1)
    mm = m_model.reshape(-1)
    for c in list(rng.choice(np.arange(mm.size), 4, replace=False)) + [int(np.argmax(np.abs(g)))]:
        step = 1e-4 * mm[c]
        mp, mn = mm.copy(), mm.copy()
        mp[c] += step
        mn[c] -= step
        fd = (oracle.objective_grad_model(p, mgrid, mp)["J"] - oracle.objective_grad_model(p, mgrid, mn)["J"]) / (2 * step)
        assert abs(fd - g[c]) <= 1e-6 * np.abs(g).max(), (c, fd, g[c])


# --------------------------------------------------------------------------
# Off-grid sources and receivers (trilinear e and P)
# --------------------------------------------------------------------------

def _offgrid_positions(p, rng, jitter=True):
    """Source and receiver coordinates [m]: the problem's cells, moved by up to
    half a cell when jitter is set; two receivers share a cell."""
    g = p.grids[0]
    def xyz(c):
        c = int(c)
        return np.array([c % g.nx, (c // g.nx) % g.ny, c // (g.nx * g.ny)], dtype=np.float64) * g.h
    src, rec = [], []
    for s in p.systems:
        sp_ = xyz(s.src) + (rng.uniform(-0.5, 0.5, 3) * g.h if jitter else 0.0)
        rr = np.array([xyz(c) for c in s.rec])
        if jitter:
            rr = rr + rng.uniform(-0.5, 0.5, rr.shape) * g.h
            rr[1] = rr[0] + 0.3 * g.h   # within one cell of receiver 0
        src.append(sp_)
        rec.append(rr)
    return src, rec


def test_trilinear_point_matches_scipy_interpolation():
    from scipy.interpolate import RegularGridInterpolator
    rng = _rng(81)
    g = Grid(7, 6, 5, 12.5, 0, 1500.0)
    u = rng.standard_normal(g.shape)
    f = RegularGridInterpolator([np.arange(n) * g.h for n in g.shape], u, method="linear")
    for _ in range(50):
        pt = rng.uniform(0, 1, 3) * np.array([(g.nx - 1), (g.ny - 1), (g.nz - 1)]) * g.h
        cells, w = oracle.trilinear_point(g, pt)
        assert abs(w.sum() - 1.0) < 1e-14 and len(set(cells)) == len(cells)
        assert abs(np.dot(w, u.reshape(-1)[cells]) - f([pt[::-1]])[0]) < 1e-12
    # a node gives one cell of weight one; a degenerate axis merges corners
    cells, w = oracle.trilinear_point(g, np.array([2, 3, 1]) * g.h)
    assert list(cells) == [(1 * g.ny + 3) * g.nx + 2] and np.allclose(w, [1.0])
    g1 = Grid(7, 1, 5, 12.5, 0, 1500.0)
    cells, w = oracle.trilinear_point(g1, (20.0, 0.0, 30.0))
    assert len(cells) == 4 and abs(w.sum() - 1.0) < 1e-14


def test_offgrid_at_nodes_equals_on_grid():
    """Positions on the nodes: the off-grid objective, gradient, wavefields and
    source weights equal the on-grid oracle's (independent e and P)."""
    p = wri_synth.custom_problem((9, 8, 7), nb=2, n_src=2, n_rec=6, seed=82, lam=0.05)
    src, rec = _offgrid_positions(p, _rng(83), jitter=False)
    for mode in ("estimate", "known"):
        a = oracle.objective_grad_offgrid(p, src, rec, mode=mode)
        b = oracle.objective_grad(p, mode=mode)
        assert abs(a["J"] - b["J"]) <= 1e-10 * b["J"]
        assert np.abs(a["g"][0] - b["g"][0]).max() <= 1e-9 * np.abs(b["g"][0]).max()
        for k in range(len(p.systems)):
            assert abs(a["alpha"][k] - b["alpha"][k]) <= 1e-10 * abs(b["alpha"][k])


def test_offgrid_estimate_routes_agree_and_alpha_stationary():
    p = wri_synth.custom_problem((9, 8, 7), nb=2, n_src=1, n_rec=6, seed=84, lam=0.05)
    src, rec = _offgrid_positions(p, _rng(85))
    g = p.grids[0]
    A = oracle.helmholtz(g, p.m[0], p.systems[0].omega)
    e, P = oracle.offgrid_operators(g, src[0], rec[0])
    d = p.systems[0].d
    u1, a1 = oracle.solve_estimate_general(A, P, p.systems[0].lam, e, d, route="varpro")
    u2, a2 = oracle.solve_estimate_general(A, P, p.systems[0].lam, e, d, route="augmented")
    assert np.linalg.norm(u1 - u2) <= 1e-10 * np.linalg.norm(u2) and abs(a1 - a2) <= 1e-10 * abs(a2)
    # at the optimum alpha = e^H A u / e^H e
    assert abs(np.vdot(e, A @ u1) / np.vdot(e, e) - a1) <= 1e-10 * abs(a1)


def test_offgrid_gradient_matches_central_differences():
    p = wri_synth.custom_problem((9, 8, 7), nb=2, n_src=2, n_rec=6, seed=86, lam=0.05, freqs=(7.0,))
    src, rec = _offgrid_positions(p, _rng(87))
    out = oracle.objective_grad_offgrid(p, src, rec)
    g = out["g"][0].reshape(-1)
    m = p.m[0].reshape(-1)
    rng = _rng(88)
    for c in list(rng.choice(np.arange(m.size), 3, replace=False)) + [int(np.argmax(np.abs(g)))]:
        step = 1e-4 * m[c]
        mp, mn = m.copy(), m.copy()
        mp[c] += step
        mn[c] -= step
        fd = (oracle.objective_grad_offgrid(p, src, rec, m_list=[mp.reshape(p.grids[0].shape)])["J"] -
              oracle.objective_grad_offgrid(p, src, rec, m_list=[mn.reshape(p.grids[0].shape)])["J"]) / (2 * step)
        assert abs(fd - g[c]) <= 1e-6 * np.abs(g).max(), (c, fd, g[c])


# --------------------------------------------------------------------------
# N^{-1} through the factors of A (Sherman-Morrison-Woodbury route)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("lam,n_rec", [(0.12, 9), (3.0, 1), (0.0, 6), (0.5, 0)])
def test_normal_inverse_through_factors_of_A(lam, n_rec):
    """NormalInverse.solve(y) against a dense solve with N = A^H A + lam^2 P^H P
    assembled from A (brute force on 7 x 6 x 5), for several receiver counts,
    lam = 0 (N = A^H A) and no receivers."""
    g = Grid(7, 6, 5, 10.0, 1, 1600.0)
    rng = _rng(11)
    m = rng.uniform(1 / 3000.0 ** 2, 1 / 1600.0 ** 2, g.n)
    A = oracle.helmholtz(g, m, 2 * np.pi * 11.0)
    rec = np.sort(rng.choice(g.n, size=n_rec, replace=False))
    P = oracle.restriction(g.n, rec)
    Ad, Pd = A.toarray(), P.toarray()
    N = Ad.conj().T @ Ad + lam ** 2 * Pd.conj().T @ Pd
    Y = _crandn(rng, g.n, 3)
    ref = np.linalg.solve(N, Y)
    inv = oracle.NormalInverse(A, P, lam)
    got = np.stack([inv.solve(Y[:, j]) for j in range(3)], axis=1)
    assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("mode", ["estimate", "known"])
def test_objective_grad_same_by_both_normal_solvers(mode):
    """The exact minimiser, J and g computed with a factor of N and with the
    factors of A (Woodbury) agree to rounding on a two-frequency problem."""
    p = wri_synth.custom_problem((11, 9, 8), nb=2, n_src=2, n_rec=7, seed=44, freqs=(6.0, 9.0))
    a = oracle.objective_grad(p, mode=mode)
    b = oracle.objective_grad(p, mode=mode, normal_solver="woodbury")
    assert b["J"] == pytest.approx(a["J"], rel=1e-10)
    for ua, ub in zip(a["u"], b["u"]):
        assert np.linalg.norm(ua - ub) <= 1e-10 * np.linalg.norm(ua)
    assert np.allclose(b["alpha"], a["alpha"], rtol=1e-10, atol=0)
    ga, gb = a["g"][0].reshape(-1), b["g"][0].reshape(-1)
    assert np.linalg.norm(ga - gb) <= 1e-9 * np.linalg.norm(ga)


# --------------------------------------------------------------------------
# Preconditioned CGLS: the complex-shifted-Laplacian V-cycle
# --------------------------------------------------------------------------

def test_csl_prolongation_is_trilinear_by_brute_force():
    """P of the V-cycle against weights written out cell by cell: along each
    axis coarse i sits on fine 2i+1 (weight 1) and its two fine neighbours
    take 1/2; the 3D weight is the product over the axes (x fastest)."""
    g = Grid(10, 9, 8, 10.0, 2, 1500.0)
    lev = oracle.csl_levels(g, np.full(g.n, 1 / 2000.0 ** 2))
    assert lev[1]["shape"] == (4, 4, 5) and lev[1]["h"] == 20.0
    Pm = lev[0]["P"].toarray()

    def w(f, i):
        return 1.0 if f == 2 * i + 1 else (0.5 if abs(f - (2 * i + 1)) == 1 else 0.0)
    ref = np.zeros((g.n, 4 * 4 * 5))
    for z in range(8):
        for y in range(9):
            for x in range(10):
                for cz in range(4):
                    for cy in range(4):
                        for cx in range(5):
                            ref[(z * 9 + y) * 10 + x, (cz * 4 + cy) * 5 + cx] = w(z, cz) * w(y, cy) * w(x, cx)
    assert np.array_equal(Pm, ref)
    # coarse m is the weighted mean: a constant model stays constant
    assert np.allclose(lev[1]["m"], 1 / 2000.0 ** 2, rtol=1e-14, atol=0)


def test_csl_vcycle_is_linear_and_complex_symmetric():
    """M is a fixed linear map with M^T = M (R = P^T / 8, the same Jacobi
    step before and after), so the adjoint cycle is the cycle on conj(A_beta):
    y^T (M x) = x^T (M y) and <M x, y> = <x, M^H y>."""
    g = Grid(20, 18, 16, 12.0, 3, 1600.0)
    rng = _rng(21)
    m = rng.uniform(1 / 3000.0 ** 2, 1 / 1600.0 ** 2, g.n)
    lev = oracle.csl_levels(g, m)
    assert len(lev) == 3
    om = 2 * np.pi * 9.0
    x, y = _crandn(rng, g.n), _crandn(rng, g.n)
    Mx, My = oracle.csl_vcycle(lev, om, x), oracle.csl_vcycle(lev, om, y)
    a, b = 1.5 - 0.5j, -0.25 + 2j
    assert np.allclose(oracle.csl_vcycle(lev, om, a * x + b * y), a * Mx + b * My, rtol=1e-12, atol=1e-12 * np.abs(Mx).max())
    assert abs(y @ Mx - x @ My) <= 1e-12 * abs(y @ Mx)
    MHy = oracle.csl_vcycle(lev, om, y, adjoint=True)
    assert abs(np.vdot(y, Mx) - np.vdot(MHy, x)) <= 1e-12 * abs(np.vdot(y, Mx))


def test_csl_vcycle_iteration_converges_to_the_shifted_solve():
    """Repeated cycles as a stationary iteration x <- x + M (f - A_beta x)
    converge to A_beta^{-1} f (sparse LU of the shifted operator assembled
    independently from the oracle's Helmholtz matrix), at a steady rate of
    about 0.67 per cycle (bound 0.75): M approximates the inverse of the
    shifted operator (a wrong shift sign, smoother or transfer would stall or
    diverge)."""
    g = Grid(24, 20, 18, 10.0, 4, 1500.0)
    rng = _rng(22)
    m = rng.uniform(1 / 3500.0 ** 2, 1 / 1500.0 ** 2, g.n)
    om = 2 * np.pi * 8.0
    Ab = oracle.helmholtz(g, m, om) - 1j * 0.5 * om ** 2 * sp.diags(m)
    f = _crandn(rng, g.n)
    ref = spl.spsolve(Ab.tocsc(), f)
    lev = oracle.csl_levels(g, m)
    x = np.zeros(g.n, complex)
    errs = []
    for _ in range(60):
        x = x + oracle.csl_vcycle(lev, om, f - Ab @ x)
        errs.append(np.linalg.norm(x - ref) / np.linalg.norm(ref))
    assert errs[-1] < 1e-10, errs[-1]
    assert max(b / a for a, b in zip(errs[4:], errs[5:])) < 0.75


@pytest.mark.parametrize("mode", ["estimate", "known"])
def test_pcgls_with_the_identity_is_cgls(mode):
    """With M = I the preconditioned recurrences are those of the plain CGLS:
    the same iterate after k steps."""
    p = wri_synth.custom_problem((9, 8, 7), nb=2, n_src=1, n_rec=6, seed=45, freqs=(7.0,))
    s = p.systems[0]
    A, P, e = oracle.system_operators(p, 0)
    ident = lambda v: v
    for k in (1, 3, 8):
        a = oracle.cgls(A, P, s.lam, s.src, mode, s.alpha, s.d, rtol=0.0, maxiter=k, alpha_scale=0.3)
        b = oracle.pcgls(A, P, s.lam, s.src, mode, s.alpha, s.d, 0.0, k, ident, ident, alpha_scale=0.3)
        assert np.allclose(b["u"], a["u"], rtol=1e-11, atol=1e-13 * np.abs(a["u"]).max())
        assert b["iters"] == a["iters"] == k


@pytest.mark.parametrize("mode", ["estimate", "known"])
def test_pcgls_reaches_the_exact_minimiser_in_fewer_iterations(mode):
    """The V-cycle-preconditioned CGLS at a tight tolerance reaches the exact
    minimiser (the preconditioner changes the iterates, not the solution);
    at rtol 1e-5 it takes well under half the plain CGLS's iterations."""
    p = wri_synth.custom_problem((24, 22, 20), nb=4, n_src=1, n_rec=9, seed=46, freqs=(9.0,))
    s = p.systems[0]
    A, P, e = oracle.system_operators(p, 0)
    ex = oracle.objective_grad(p, mode=mode)
    lev = oracle.csl_levels(p.grids[0], p.m[0])
    M = lambda v: oracle.csl_vcycle(lev, s.omega, v)
    MH = lambda v: oracle.csl_vcycle(lev, s.omega, v, adjoint=True)
    tight = oracle.pcgls(A, P, s.lam, s.src, mode, s.alpha, s.d, 1e-11, 5000, M, MH)
    assert tight["status"] == "converged"
    assert np.linalg.norm(tight["u"] - ex["u"][0]) <= 1e-7 * np.linalg.norm(ex["u"][0])
    if mode == "estimate":
        assert abs(tight["alpha"] - ex["alpha"][0]) <= 1e-7 * abs(ex["alpha"][0])
    plain = oracle.cgls(A, P, s.lam, s.src, mode, s.alpha, s.d, rtol=1e-5, maxiter=100000)
    pre = oracle.pcgls(A, P, s.lam, s.src, mode, s.alpha, s.d, 1e-5, 100000, M, MH)
    assert pre["iters"] < 0.5 * plain["iters"], (pre["iters"], plain["iters"])
