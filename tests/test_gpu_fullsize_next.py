"""Full-size checks of the paths beyond the augmented solve (reduced FWI, the
model grid, off-grid sources and receivers), in the configurations that
`bench.py --fwi / --model-grid / --offgrid` time.  The oracle cannot factor
these grids, so the checks are properties it evaluates in float64 without a
solve: objective values recomputed from the returned wavefields, the
stationarity of the source weights, true normal residuals, and the gradient
pull-back recomputed with the oracle's sparse interpolation matrices.
"""
import dataclasses
import sys

import numpy as np
import pytest
import scipy.sparse as sp
import torch

import oracle
import wri_synth
from wri_synth import Grid
from paper_2410_18429_amd import wri

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _np(t):
    return t.detach().cpu().numpy().astype(np.complex128)


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    torch.cuda.init()
    yield
    torch.cuda.synchronize()


def test_fwi_full_size_properties():
    """128^3, 48 systems, rtol 1e-4: f and the estimated weights from the
    returned wavefields, and the forward solves' true normal residual."""
    _say("fwi full size 128^3 x 48")
    p = wri_synth.make_config("differentiation", seed=0)
    b = wri.Batch(p, device=DEV)
    u = wri.alloc_wavefields(b)
    f, grads, res = wri.fwi_objective_grad(b, u_out=u)
    assert all(r["status_fwd"] == "converged" and r["status_adj"] == "converged" for r in res)
    assert torch.isfinite(grads[0]).all().item()
    ftot = 0.0
    for k, s in enumerate(p.systems):
        pu = _np(u[k])[np.asarray(s.rec)]
        rho = pu - s.d
        fk = 0.5 * float(np.vdot(rho, rho).real)
        ftot += fk
        assert abs(res[k]["f"] - fk) <= 1e-5 * fk, k
        # the weight minimises the misfit: (P u)^H (P u - d) = 0
        assert abs(np.vdot(pu, rho)) <= 1e-5 * np.linalg.norm(pu) * np.linalg.norm(rho), k
    assert abs(f - ftot) <= 1e-6 * ftot
    ops = {}
    for k in (0, 23, 47):
        s = p.systems[k]
        if s.freq not in ops:
            ops[s.freq] = oracle.system_operators(p, k)[:2]
        A, P = ops[s.freq]
        uk = _np(u[k])
        # u = alpha w with A w = e: the normal residual of A u = alpha e at the returned u
        tr = oracle.normal_residual(A, P, 0.0, s.src, "known", res[k]["alpha"], s.d, uk)
        _say(f"  sys {k}: forward true normal residual {tr:.2e}")
        assert tr <= 2e-4   # the recurred residual met rtol 1e-4; float32 drift stays within 2x


def _jitter(p, rng):
    g = p.grids[0]

    def xyz(c):
        return np.array([c % g.nx, (c // g.nx) % g.ny, c // (g.nx * g.ny)], dtype=np.float64) * g.h
    src = [xyz(int(s.src)) + rng.uniform(-0.5, 0.5, 3) * g.h for s in p.systems]
    rec = [np.array([xyz(int(c)) for c in s.rec]) + rng.uniform(-0.5, 0.5, (len(s.rec), 3)) * g.h
           for s in p.systems]
    return src, rec


def test_offgrid_full_size_properties():
    """64^3, 8 systems, positions moved up to half a cell, rtol 1e-4: J from
    the returned (u, alpha), alpha_ls = e^H A u / e^H e, and the true normal
    residual of the augmented system with the trilinear e and P."""
    _say("off-grid full size 64^3 x 8")
    p = wri_synth.make_config("medium", seed=0)
    src, rec = _jitter(p, np.random.default_rng(5))
    b = wri.Batch(p, device=DEV)
    u = wri.alloc_wavefields(b)
    J, grads, res = wri.objective_grad_offgrid(b, src, rec, u_out=u)
    assert all(r["status"] == "converged" for r in res)
    g = p.grids[0]
    c = np.sqrt(42.0) / g.h ** 2
    for k in (0, 3, 7):
        s = p.systems[k]
        A = oracle.helmholtz(g, p.m[0], s.omega)
        e, P = oracle.offgrid_operators(g, src[k], rec[k])
        uk = _np(u[k])
        a = res[k]["alpha"]
        r1 = a * e - A @ uk
        r2 = s.lam * (s.d - P @ uk)
        Jk = float(np.vdot(r1, r1).real + np.vdot(r2, r2).real)
        assert abs(res[k]["J"] - Jk) <= 1e-3 * Jk, k
        au = A @ uk
        als = np.vdot(e, au) / np.vdot(e, e)
        assert abs(res[k]["alpha_ls"] - als) <= 1e-5 * abs(als), k
        # normal residual of S = [[A, -c e], [lam P, 0]], b = [0; lam d]
        su = A.conj().T @ r1 + s.lam * (P.conj().T @ r2)
        sa = -c * np.vdot(e, r1)
        sb = s.lam * (s.lam * (P.conj().T @ s.d))
        tr = np.sqrt(np.vdot(su, su).real + abs(sa) ** 2) / np.linalg.norm(sb)
        _say(f"  sys {k}: J gpu {res[k]['J']:.6e} float64 {Jk:.6e}, true normal residual {tr:.2e}")
        assert tr <= 2e-4


def test_model_grid_full_size_pullback():
    """The uneven workload (96 systems on 48^3 / 64^3 / 96^3 grids) with a
    148^3 model grid: the model-grid gradient equals sum_g R_g^T grad_g
    computed with the oracle's sparse R_g from the per-grid gradients of the
    same models, and J is identical."""
    _say("model grid full size (uneven)")
    p = wri_synth.make_config("uneven", seed=0)
    h_m = 12.0
    ext = [max((getattr(g, a) - 1) * g.h for g in p.grids) for a in ("nx", "ny", "nz")]
    mgrid = Grid(*[int(np.ceil(e / h_m)) + 1 for e in ext], h=h_m, nb=0, v_ref=1500.0)
    rng = np.random.default_rng(7)
    m_model = torch.tensor((1.0 / rng.uniform(1800.0, 2400.0, mgrid.n) ** 2).astype(np.float32), device=DEV)
    b = wri.Batch(p, device=DEV)
    J, gm, res = wri.objective_grad_model(b, mgrid, m_model)
    b.set_m([wri.model_to_grid(mgrid, m_model, gr) for gr in p.grids])
    J2, grads, _ = wri.objective_grad(b)
    assert J2 == J
    ref = np.zeros(mgrid.n)
    for gr, gg in zip(p.grids, grads):
        ref += oracle.resample_matrix(mgrid, gr).T @ gg.cpu().numpy().astype(np.float64)
    got = gm.cpu().numpy().astype(np.float64)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    _say(f"  pull-back max deviation {err:.2e}")
    assert err <= 1e-5
