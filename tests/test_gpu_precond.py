"""GPU parity of the V-cycle-preconditioned CGLS (wri_objective_grad_precond)
against the oracle: its iterates after k steps against the oracle's pcgls with
the oracle's V-cycle (float32 storage: 1e-4), converged solves against the
exact minimiser (u, alpha, J 1e-4, g 1e-3), graph replay against eager
launches (bit for bit), edge cases, and the iteration count against the plain
batched solver."""
import dataclasses
import sys

import numpy as np
import pytest
import torch

import oracle
import wri_synth
from paper_2410_18429_amd import wri

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    b = np.asarray(b)
    return float(np.linalg.norm(np.asarray(a) - b) / max(np.linalg.norm(b), 1e-300))


def _np(t):
    return t.detach().cpu().numpy().astype(np.complex128)


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    torch.cuda.init()
    yield
    torch.cuda.synchronize()


def _oracle_pcgls(p, i, mode, rtol, maxiter):
    s = p.systems[i]
    g = p.grids[s.grid]
    m32 = np.asarray(p.m[s.grid], dtype=np.float32).astype(np.float64).reshape(-1)
    A, P, e = oracle.system_operators(p, i, m=m32)
    lev = oracle.csl_levels(g, m32)
    M = lambda v: oracle.csl_vcycle(lev, s.omega, v)
    MH = lambda v: oracle.csl_vcycle(lev, s.omega, v, adjoint=True)
    d = np.asarray(s.d).astype(np.complex64).astype(np.complex128)
    return oracle.pcgls(A, P, s.lam, s.src, mode, s.alpha, d, rtol, maxiter, M, MH), len(lev)


@pytest.mark.parametrize("mode", ["estimate", "known"])
@pytest.mark.parametrize("k", [1, 2, 5])
def test_precond_iterates_match_oracle(mode, k):
    """After k iterations (max_iter = k, rtol 0) on a grid with three V-cycle
    levels (24x22x20 -> 12x11x10 -> 6x5x5): the wavefield, the CGLS source
    unknown and the recurred residual against the oracle's preconditioned CGLS
    with the oracle's V-cycle on the same float32 inputs."""
    _say(f"precond iterates mode={mode} k={k}")
    p = wri_synth.custom_problem((24, 22, 20), nb=4, n_src=2, n_rec=9, seed=61, freqs=(9.0,), rtol=0.0)
    b = wri.Batch(p, device=DEV, mode=mode)
    u = wri.alloc_wavefields(b)
    _, _, res = wri.objective_grad_precond(b, max_iter=k, u_out=u, with_grad=False)
    for i in range(len(p.systems)):
        ref, nlev = _oracle_pcgls(p, i, mode, 0.0, k)
        assert nlev == 3
        eu = rel(_np(u[i]), ref["u"])
        _say(f"  sys {i}: u err {eu:.2e} relres {res[i]['relres']:.6e} oracle {ref['relres']:.6e}")
        assert res[i]["iters"] == k and res[i]["status"] == "max_iter"
        assert eu < 1e-4
        assert abs(res[i]["relres"] - ref["relres"]) <= 1e-4 * ref["relres"]
        if mode == "estimate":
            assert abs(res[i]["alpha"] - ref["alpha"]) <= 1e-4 * abs(ref["alpha"])


PC_SHAPES = [(24, 22, 20), (40, 18, 33), (16, 16, 16), (9, 3, 7)]


@pytest.mark.parametrize("mode", ["estimate", "known"])
@pytest.mark.parametrize("shape", PC_SHAPES)
def test_precond_solve_matches_exact_minimiser(shape, mode):
    """Converged at rtol 1e-7 (the parity tolerance of the plain solver):
    u, alpha and J per system within 1e-4 and the gradient within 1e-3 of the
    exact minimiser; the 9x3x7 grid is too thin to coarsen, so its cycle is
    four Jacobi steps on the grid itself."""
    _say(f"precond solve shape={shape} mode={mode}")
    p = wri_synth.custom_problem(shape, nb=min(6, min(shape) // 3), n_src=2, n_rec=10, seed=7, freqs=(6.0, 9.0),
                                 rtol=1e-7)
    ref = oracle.objective_grad(p, mode=mode)
    b = wri.Batch(p, device=DEV, mode=mode)
    u = wri.alloc_wavefields(b)
    J, grads, res = wri.objective_grad_precond(b, max_iter=60000, u_out=u)
    for i in range(len(p.systems)):
        eu = rel(_np(u[i]), ref["u"][i])
        eJ = abs(res[i]["J"] - ref["J_sys"][i]) / ref["J_sys"][i]
        _say(f"  sys {i}: iters {res[i]['iters']} u err {eu:.2e} J err {eJ:.2e}")
        assert res[i]["status"] == "converged", res[i]
        assert eu < 1e-4
        assert eJ < 1e-4
        if mode == "estimate":
            assert abs(res[i]["alpha_ls"] - ref["alpha"][i]) < 1e-4 * abs(ref["alpha"][i])
    assert abs(J - ref["J"]) < 1e-4 * ref["J"]
    g = grads[0].cpu().numpy().astype(np.float64)
    assert rel(g, ref["g"][0].reshape(-1)) < 1e-3


def test_precond_uneven_grids_one_call():
    """Three grids of different sizes in one call (each grid's systems iterate
    in lockstep with their own V-cycle hierarchy), per-system tolerances:
    every system converges, and each matches the same system solved alone
    bit for bit (the batch changes no arithmetic)."""
    _say("precond uneven grids")
    rng = np.random.default_rng(12)
    parts = [wri_synth.custom_problem(sh, h=h, nb=3, n_src=2, n_rec=8, seed=s, freqs=(f,), rtol=1e-6)
             for sh, h, s, f in (((16, 16, 16), 20.0, 1, 5.0), ((24, 20, 18), 14.0, 2, 8.0),
                                  ((33, 17, 9), 10.0, 3, 12.0))]
    grids, m, mt, systems = [], [], [], []
    for gi, q in enumerate(parts):
        grids += q.grids
        m += q.m
        mt += q.m_true
        for s in q.systems:
            s.grid = gi
            s.rtol = float(10.0 ** (-2 - 3 * rng.uniform()))
            systems.append(s)
    p = wri_synth.Problem("uneven-small", grids, m, mt, systems)
    b = wri.Batch(p, device=DEV)
    u = wri.alloc_wavefields(b)
    J, grads, res = wri.objective_grad_precond(b, u_out=u)
    for i in range(len(p.systems)):
        assert res[i]["status"] == "converged" and res[i]["relres"] <= p.systems[i].rtol, res[i]
        gi = p.systems[i].grid
        one = wri_synth.Problem("one", [p.grids[gi]], [p.m[gi]], [p.m_true[gi]],
                                [dataclasses.replace(p.systems[i], grid=0)])
        b1 = wri.Batch(one, device=DEV)
        u1 = wri.alloc_wavefields(b1)
        _, _, r1 = wri.objective_grad_precond(b1, u_out=u1)
        assert r1[0]["iters"] == res[i]["iters"], i
        assert torch.equal(u1[0], u[i]), i


def test_precond_graph_and_eager_agree():
    _say("precond graph vs eager")
    p = wri_synth.custom_problem((40, 20, 30), nb=3, n_src=2, n_rec=8, seed=10, freqs=(7.0,), rtol=1e-6)
    b = wri.Batch(p, device=DEV)
    ue = wri.alloc_wavefields(b)
    Je, ge, re_ = wri.objective_grad_precond(b, flags=wri.FLAG_NO_GRAPH, u_out=ue)
    for rep in range(2):
        ug = wri.alloc_wavefields(b)
        Jg, gg, rg = wri.objective_grad_precond(b, u_out=ug)
        torch.cuda.synchronize()
        _ = torch.randn(1 << 20, device=DEV).sum().item()
        assert Jg == Je
        assert torch.equal(gg[0], ge[0])
        for i in range(len(p.systems)):
            assert rg[i]["iters"] == re_[i]["iters"]
            assert torch.equal(ug[i], ue[i]), (rep, i)


def test_precond_edge_cases():
    _say("precond edge cases")
    p = wri_synth.custom_problem((20, 10, 8), nb=2, n_src=2, n_rec=5, seed=12)
    pz = p.with_data([np.zeros_like(s.d) for s in p.systems])
    b = wri.Batch(pz, device=DEV)
    u = wri.alloc_wavefields(b)
    J, g, res = wri.objective_grad_precond(b, u_out=u)
    for i in range(len(pz.systems)):
        assert res[i]["status"] == "zero_rhs" and res[i]["iters"] == 0
        assert not torch.any(u[i] != 0)
    assert J == 0.0 and not torch.any(g[0] != 0)
    b = wri.Batch(p, device=DEV)
    u = wri.alloc_wavefields(b)
    _, _, res = wri.objective_grad_precond(b, max_iter=0, u_out=u, with_grad=False)
    assert all(r["status"] == "max_iter" and r["iters"] == 0 for r in res)
    assert not any(torch.any(v != 0) for v in u)
    with pytest.raises(wri.WriError) as ei:
        wri.objective_grad_precond(b, flags=wri.FLAG_PLAIN)
    assert ei.value.code == wri.EINVAL


def test_precond_needs_far_fewer_iterations_than_the_plain_solver():
    """The 32^3 crop of the 128^3 workload (48 systems, rtol 1e-4): the
    preconditioned solver's iteration counts against the plain batched
    solver's, and the float64 true normal residual of its wavefields."""
    _say("precond vs plain iterations, crop32")
    p = wri_synth.make_config("crop32", seed=0).with_rtol(1e-4)
    b = wri.Batch(p, device=DEV)
    _, _, rp = wri.objective_grad(b)
    u = wri.alloc_wavefields(b)
    _, _, rq = wri.objective_grad_precond(b, u_out=u)
    ip = np.array([r["iters"] for r in rp])
    iq = np.array([r["iters"] for r in rq])
    _say(f"  plain mean {ip.mean():.0f} (max {ip.max()}), preconditioned mean {iq.mean():.0f} (max {iq.max()})")
    assert all(r["status"] == "converged" for r in rq)
    assert iq.mean() < 0.2 * ip.mean()
    for k in (0, 47):
        s = p.systems[k]
        A, P, e = oracle.system_operators(p, k)
        tr = oracle.normal_residual(A, P, s.lam, s.src, "estimate", 0, s.d, _np(u[k]), rq[k]["alpha"])
        _say(f"  sys {k}: true normal residual {tr:.2e}")
        assert tr <= 2e-4
