"""Benchmark: source-frequency augmented solves per second on one MI355X.

One step = one pass of the whole hot path over the batch: the batched
source-estimating CGLS solve of all systems, the source-weight estimate, the
objective and its gradient (wri_objective_grad).  Workload: the 128^3
differentiation configuration (h = 10 m, sponge 10 cells, 16 sources on a 4x4
surface grid x 5/7/9 Hz = 48 systems, 128 receivers in a vertical well,
lambda = 0.12, rtol 1e-4), synthetic layered + anomaly model, inputs resident
in HBM before the timed region.

Also reported: the plain form (one system at a time, unfused kernels, host
loop) on a sample of systems, per-kernel HBM roofline of the fused stencil
launches (HIP events around every launch in one extra timed step), and the
CPU oracle (complex128 CGLS) on a bounded sample.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-plain] [--no-cpu]
"""
import argparse
import dataclasses
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "src·freq augmented solves/s at 128³, rtol 1e-4: batched vs plain; stencil GB/s"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per (system, cell) of one fused launch (complex64 = 8 B, m = 4 B), as
# the library counts them for every timed launch:
#   forward k: read s, p_{k-1}, m; write p_k, t                          -> 36
#              + on even k >= 2: read x, p_{k-2}; write x               -> +24
#   adjoint k: read r_k, t, m; write r_{k+1}, s                         -> 36
# Tiles with pf >= 2 recompute t = S p_k in the adjoint pass: the forward pass writes no t
# (28, +24) and the adjoint pass reads p_k in its place (36).
def bytes_note(pf):
    if pf >= 2:
        return {"fwd": "28, +24 on even iterations (x update of two steps); t is not stored",
                "adj": "36 (reads p_k and recomputes t = S p_k)"}
    return {"fwd": "36, +24 on even iterations (x update of two steps)", "adj": "36"}


def kernel_label(dominant, pf):
    if dominant == "fwd":
        return "k_fwd_pf (fused forward CGLS stencil, t not stored)" if pf >= 2 else \
               "k_fwd / k_fwd_pf (fused forward CGLS stencil)"
    return "k_adj_rc (fused adjoint CGLS stencil, t recomputed)" if pf >= 2 else \
           "k_adj / k_adj_pf (fused adjoint CGLS stencil)"


# HBM traffic of one full-batch launch (48 systems x 128^3) from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch, median over the launches of a 20-iteration
# probe with the tile forced), each scaled by what the counter reads for a 1 GiB device copy
# (FETCH_SIZE x 2.000, WRITE_SIZE x 1.000).  "fwd_x" is the forward launch that also updates x
# (even iterations).  Valid only for the solver sources it was measured on (sha256 prefix of
# kernels.hip + capi.hip + wri_impl.hpp + stencil.hpp) and for the tile shape in the key;
# summary and commands: profiles/fused_cgls_kernels_128cube_48sys_hbm_traffic.md
TRAFFIC = {
    "sources_sha256": "1d0cda1bde45a0f6",
    "tiles": {
        "8,4,64,2,4": {"fwd_x": {"fetch_kib": 1802998.8, "write_kib": 1573197.4},
                       "fwd": {"fetch_kib": 974238.8, "write_kib": 786607.1},
                       "adj": {"fetch_kib": 928214.9, "write_kib": 1573033.0}},
        "8,4,64,2,2": {"fwd_x": {"fetch_kib": 1815348.9, "write_kib": 1573197.9},
                       "fwd": {"fetch_kib": 1032783.0, "write_kib": 786610.6},
                       "adj": {"fetch_kib": 976969.6, "write_kib": 1573040.8}},
    },
    "fetch_scale": 2.000, "write_scale": 1.000,
}


def _sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "capi.hip", "wri_impl.hpp", "stencil.hpp"):
        with open(os.path.join(ROOT, "paper_2410_18429_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]



def _cpu_worker(args):
    """Oracle CGLS (complex128, scipy CSR) on one system for a bounded time."""
    name, k, tlimit, scale = args
    import oracle
    import wri_synth
    p = wri_synth.make_config(name, seed=0)
    s = p.systems[k]
    A, P, e = oracle.system_operators(p, k)
    t0 = time.perf_counter()
    out = oracle.cgls(A, P, s.lam, s.src, "estimate", 0, s.d, rtol=s.rtol, maxiter=10 ** 9,
                      time_limit=tlimit, alpha_scale=scale)
    return out["iters"], out["seconds"], time.perf_counter() - t0


# Cores this job may use on the GPU machine: the box allots 16 host cores per GPU
# (more worker processes than that are killed), whatever os.cpu_count() says.
HOST_CORE_SHARE = 16


_THREAD_VARS = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")


def _single_threaded_pool(procs):
    """A spawn pool of `procs` workers that each run the oracle on one thread:
    the thread-count variables are set before the workers import numpy (a
    worker per core; the box exports OMP_NUM_THREADS = 16)."""
    saved = {k: os.environ.get(k) for k in _THREAD_VARS}
    for k in _THREAD_VARS:
        os.environ[k] = "1"
    try:
        return mp.get_context("spawn").Pool(procs)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def host_description():
    """CPU model, core counts and the library versions the CPU oracle runs on."""
    import scipy
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "affinity_cores": aff,
            "core_share": HOST_CORE_SHARE, "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS", ""),
            "numpy": np.__version__, "scipy": scipy.__version__}


def cpu_baseline(name, systems, mean_iters, seconds, h):
    host = host_description()
    procs = max(1, min(HOST_CORE_SHARE, host["affinity_cores"] or 1, len(systems)))
    scale = 42.0 ** 0.5 / h ** 2
    with _single_threaded_pool(procs) as pool:
        outs = pool.map(_cpu_worker, [(name, k, seconds, scale) for k in systems[:procs]])
    it_per_s = sum(it / max(sec, 1e-9) for it, sec, _ in outs)
    solves_per_s = it_per_s / mean_iters
    return {"value": solves_per_s, "unit": "solves/s", "cores": procs, "kind": "oracle",
            "sample": (f"oracle complex128 CGLS (scipy CSR mat-vecs) on {procs} of the {name} systems, one "
                       f"single-threaded process per core (the box's share of {HOST_CORE_SHARE} cores), "
                       f"{seconds:.0f} s each "
                       f"({sum(o[0] for o in outs)} iterations total, {it_per_s:.2f} it/s aggregate); "
                       f"solves/s = it/s / {mean_iters:.0f} (mean GPU iterations per solve at rtol 1e-4); "
                       f"completed CPU solves and the direct oracle: profiles/cpu_oracle_host_baseline.md"),
            "host": host,
            "direct_oracle_16cube_s": _direct_oracle_seconds("tiny")}


def _cpu_complete_worker(args):
    """One job of the CPU validation run: ("cgls", config, system) runs the
    oracle's complex128 CGLS to the system's rtol; ("direct", config, system,
    solver) the oracle's exact solve (objective and gradient) of one system."""
    import oracle
    import wri_synth
    kind, name, k = args[:3]
    if kind == "direct":
        p = wri_synth.make_config(name, seed=0, data="none" if name == "tiny" else "green")
        if name == "tiny":
            p = p.with_data(oracle.observed_data(p, seed=0))
        p = p.subset([k])
        t0 = time.perf_counter()
        oracle.objective_grad(p, return_fields=False, normal_solver=args[3])
        return {"kind": "direct", "config": name, "system": k, "solver": args[3], "cells": p.grids[0].n,
                "seconds": time.perf_counter() - t0}
    p = wri_synth.make_config(name, seed=0)
    s = p.systems[k]
    A, P, e = oracle.system_operators(p, k)
    t0 = time.perf_counter()
    out = oracle.cgls(A, P, s.lam, s.src, "estimate", 0, s.d, rtol=s.rtol, maxiter=10 ** 9,
                      alpha_scale=42.0 ** 0.5 / p.grids[s.grid].h ** 2)
    return {"kind": "cgls", "config": name, "system": k, "cells": p.grids[s.grid].n, "iters": out["iters"],
            "seconds": time.perf_counter() - t0, "rtol": s.rtol}


def cpu_validate(dev, big):
    """The CPU oracle on the host of the GPU machine, run to completion: complex128
    CGLS on every system of the medium workload (and on `big` systems of the
    128^3 workload), one process per job within the box's core share, next to
    the direct oracle (sparse LU) at 16^3 and 32^3; the GPU's iteration counts
    for the same systems (batched, complex64 with float64 reductions) for the
    it/s -> solves/s conversion of the default run's CPU baseline."""
    import torch
    import wri_synth
    from paper_2410_18429_amd import wri
    host = host_description()
    jobs = [("direct", "tiny", 0, "factor_N"), ("direct", "crop32", 0, "factor_N"),
            ("direct", "crop32", 0, "woodbury")]
    jobs += [("cgls", "medium", k) for k in range(8)]
    jobs += [("cgls", "differentiation", k) for k in (0, 23, 47)[:big]]
    t0 = time.perf_counter()
    outs = []
    with _single_threaded_pool(min(HOST_CORE_SHARE, len(jobs))) as pool:
        for o in pool.imap_unordered(_cpu_complete_worker, jobs):
            outs.append(o)
            print(f"[cpu-validate] {json.dumps(o)}", file=sys.stderr, flush=True)
    outs.sort(key=lambda o: (o["kind"], o["config"], o["system"], o.get("solver", "")))
    wall = time.perf_counter() - t0
    gpu = {}
    for name in sorted(set(o["config"] for o in outs if o["kind"] == "cgls")):
        ks = [o["system"] for o in outs if o["kind"] == "cgls" and o["config"] == name]
        prob = wri_synth.make_config(name, seed=0)
        b = wri.Batch(prob.subset(ks), device=dev)
        _, _, res = wri.objective_grad(b)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, _, res = wri.objective_grad(b)
        torch.cuda.synchronize()
        gpu[name] = {"systems": ks, "iters": [r["iters"] for r in res], "seconds": time.perf_counter() - t1}
    for o in outs:
        if o["kind"] == "cgls":
            g = gpu[o["config"]]
            o["gpu_iters"] = g["iters"][g["systems"].index(o["system"])]
    med = [o for o in outs if o["kind"] == "cgls" and o["config"] == "medium"]
    line = {"mode": "cpu_validate", "host": host, "pool_wall_s": round(wall, 1), "jobs": outs, "gpu": gpu,
            "medium_cpu_solves_per_s_all_jobs_parallel": len(med) / max(o["seconds"] for o in med),
            "medium_cpu_seconds_per_solve_mean": float(np.mean([o["seconds"] for o in med])),
            "medium_cpu_over_gpu_iters": float(np.mean([o["iters"] / o["gpu_iters"] for o in med]))}
    print(json.dumps(line), flush=True)


def _direct_oracle_seconds(name):
    """Wall time of the oracle's exact solve (SuperLU factor of the normal
    matrix, objective and gradient) of the first system of a small workload."""
    import oracle
    import wri_synth
    p = wri_synth.make_config(name, seed=0, data="none")
    p = p.with_data(oracle.observed_data(p, seed=0)).subset([0])
    t0 = time.perf_counter()
    oracle.objective_grad(p, return_fields=False)
    return round(time.perf_counter() - t0, 3)


def error_vs_fp64(prob, batch, dev, sample=(0, 23, 47)):
    """Errors of the GPU results against float64, computed by the oracle on
    the host after the timed region (one more GPU evaluation provides the
    wavefields):
      * true normal residual ||S^H (b - S x)|| / ||S^H b|| in float64 of the
        returned (u, alpha) of sampled systems (the solver stops on the
        recurred value at rtol 1e-4);
      * J of those systems recomputed in float64 from (u, alpha) against the
        GPU's recurred J;
      * alpha_ls = (A u)[src] in float64 against the GPU's;
      * the 32^3 crop of the same model (48 systems, rtol 1e-8) against the
        exact float64 minimiser of the golden file: wavefield-free J, alpha and
        gradient errors."""
    import torch
    import oracle
    import wri_synth
    from paper_2410_18429_amd import wri
    u = wri.alloc_wavefields(batch)
    J, grads, res = wri.objective_grad(batch, u_out=u)
    torch.cuda.synchronize()
    per = []
    ops = {}
    for k in sample:
        s = prob.systems[k]
        if s.freq not in ops:
            ops[s.freq] = oracle.system_operators(prob, k)[:2]
        A, P = ops[s.freq]
        e = oracle.unit_vector(A.shape[0], s.src)
        uk = u[k].cpu().numpy().astype(np.complex128)
        t1, t2 = oracle.objective_terms(A, P, s.lam, uk, res[k]["alpha"], e, s.d)
        tr = oracle.normal_residual(A, P, s.lam, s.src, "estimate", 0, s.d, uk, res[k]["alpha"])
        a64 = (A @ uk)[s.src]
        per.append({"system": k, "true_normal_residual": float(tr), "recurred_relres": res[k]["relres"],
                    "J_rel_err": abs(res[k]["J"] - (t1 + t2)) / (t1 + t2),
                    "alpha_ls_rel_err": abs(res[k]["alpha_ls"] - a64) / abs(a64)})
    del u
    gold = np.load(os.path.join(ROOT, "tests", "golden", "crop32_oracle.npz"))
    cp = wri_synth.make_config("crop32", seed=0)
    cb = wri.Batch(cp, device=dev)
    Jc, gc, rc = wri.objective_grad(cb)
    torch.cuda.synchronize()
    g = gc[0].cpu().numpy().astype(np.float64)
    gref = gold["g"].reshape(-1)
    alpha = np.array([r["alpha_ls"] for r in rc])
    crop = {"J_rel_err": abs(Jc - float(gold["J"])) / float(gold["J"]),
            "alpha_max_rel_err": float(np.max(np.abs(alpha - gold["alpha"]) / np.abs(gold["alpha"]))),
            "grad_rel_err": float(np.linalg.norm(g - gref) / np.linalg.norm(gref)),
            "systems": len(cp.systems), "rtol": 1e-8}
    return {"reference": "float64 oracle (host)", "sampled_128cube": per, "crop32_vs_exact_minimiser": crop}


def tail_probe(dev, tiles, k1=600, k2=800):
    """Steady-state kernel time per CGLS iteration (forward + adjoint, HIP events
    around every launch) against the number of systems still iterating, per
    tile: batches of n systems of the 128^3 workload (spread over its three
    frequencies) and of the large workload's 256 x 256 x 192 grid, rtol 0, timed
    over iterations k1..k2 as the difference of a run to k1 and one to k2
    iterations, after the wavefield has filled the grid (the first few hundred
    iterations of a solve run faster: the fields are still mostly zero)."""
    import torch
    import wri_synth
    from paper_2410_18429_amd import wri
    out = []
    for name, counts in (("differentiation", (1, 2, 4, 6, 8, 12, 16, 24, 32, 48)), ("large", (1, 2, 4, 8))):
        prob = wri_synth.make_config(name, seed=0)
        nsys = len(prob.systems)
        for tile in tiles:
            os.environ["WRI_TILE"] = tile
            for n in counts:
                pick = [int(round(i * nsys / n)) for i in range(n)]
                q = prob.subset(pick).with_rtol(0.0)
                b = wri.Batch(q, device=dev)
                t = {}
                for K in (k1, k2):
                    wri.objective_grad(b, max_iter=K, flags=wri.FLAG_TIMING)
                    torch.cuda.synchronize()
                    kt = wri.kernel_times()
                    t[K] = (kt["fwd_ms"] + kt["adj_ms"], kt["fwd_bytes"] + kt["adj_bytes"])
                ms = (t[k2][0] - t[k1][0]) / (k2 - k1)
                gbs = (t[k2][1] - t[k1][1]) / ((t[k2][0] - t[k1][0]) * 1e-3) / 1e9
                rec = {"workload": name, "tile": tile, "systems": n, "cells": n * q.grids[0].n,
                       "ms_per_iteration": round(ms, 4), "gbs": round(gbs, 1)}
                print(json.dumps(rec), file=sys.stderr, flush=True)
                out.append(rec)
                del b
        os.environ.pop("WRI_TILE", None)
    return out


def precond_bench(dev, steps, rtols=(1e-4, 1e-5), ref_rtol=1e-7, sample=(0, 16, 32, 47)):
    """The 128^3 workload (48 systems) solved by the plain batched CGLS (the
    headline method) and by the V-cycle-preconditioned CGLS (fewer iterations): seconds
    per objective-and-gradient evaluation, iteration counts, and the wavefield
    and source-weight errors of both against a tight preconditioned solve
    (rtol 1e-7, about what float32 storage resolves) of the same systems, on
    sampled systems."""
    import torch
    import wri_synth
    from paper_2410_18429_amd import wri
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    prob = wri_synth.make_config("differentiation", seed=0)
    nsys = len(prob.systems)
    b = wri.Batch(prob, device=dev)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            out = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, out

    def fields(fn):
        u = wri.alloc_wavefields(b)
        _, _, res = fn(u)
        torch.cuda.synchronize()
        return [u[k].cpu().numpy().astype(np.complex128) for k in sample], [res[k]["alpha_ls"] for k in sample], res

    b.set_rtol(ref_rtol)
    ref_u, ref_a, ref_res = fields(lambda u: wri.objective_grad_precond(b, u_out=u, max_iter=5000))
    log(f"[precond] reference: rtol {ref_rtol:g}, iterations {[ref_res[k]['iters'] for k in sample]}")

    def errs(us, als):
        return ([float(np.linalg.norm(u - r) / np.linalg.norm(r)) for u, r in zip(us, ref_u)],
                [float(abs(a - r) / abs(r)) for a, r in zip(als, ref_a)])

    out = {"mode": "precond", "workload": "differentiation: 128x128x128 h=10 m, 48 systems, ESTIMATE",
           "systems": nsys, "steps": steps, "reference_rtol": ref_rtol, "sample": list(sample),
           "reference_iters": [ref_res[k]["iters"] for k in sample], "runs": []}
    for rt in rtols:
        b.set_rtol(rt)
        for name, call in (("plain", lambda u=None: wri.objective_grad(b, u_out=u)),
                           ("precond", lambda u=None: wri.objective_grad_precond(b, u_out=u))):
            sec, (_, _, res) = timed(call)
            us, als, _ = fields(lambda u: call(u))
            eu, ea = errs(us, als)
            it = np.array([r["iters"] for r in res])
            rec = {"solver": name, "rtol": rt, "seconds_per_evaluation": round(sec, 4),
                   "solves_per_s": round(nsys / sec, 3), "iters_mean": float(it.mean()), "iters_max": int(it.max()),
                   "status": sorted(set(r["status"] for r in res)),
                   "u_rel_err_vs_reference": eu, "alpha_rel_err_vs_reference": ea}
            log(f"[precond] {json.dumps(rec)}")
            out["runs"].append(rec)
    print(json.dumps(out), flush=True)


def stream_ceilings(wri, dev, n=1 << 27, reps=5):
    """GB/s of the library's streaming probe for each access mix (copy, forward,
    forward with the x update, adjoint) over n complex64 elements per array, and
    of the forward mix in a tiled plane-by-plane order (64 x 16 x 32 tiles) over
    the 48 grids of 128^3 of the workload ("fwd_tiles")."""
    out = {mix: wri.stream_probe(mix, n, reps, device=dev) for mix in ("copy", "fwd", "fwd_x", "adj")}
    out["fwd_tiles"] = wri.tile_probe(128, 128, 128, 48, reps, device=dev)
    return out


def awri_bench(name, updates, dev):
    """Algorithm 2 on one workload, the four settings of the paper's comparison
    (fixed tight tolerance, fixed loose tolerance, adaptive, adaptive + TV) and
    two with warm-started solves, up to `updates` accepted model updates each
    from the same start model."""
    import torch
    import wri_synth
    from paper_2410_18429_amd import wri
    prob = wri_synth.make_config(name, seed=0)
    g = prob.grids[0]
    # Observed data consistent with the true model: this library's own solve of
    # A(m_true) u = alpha_true e (KNOWN mode, lambda = 0, i.e. min ||A u - q||),
    # sampled at the receivers, plus 1 % complex Gaussian noise.  (The
    # configuration's own data are free-space Green's functions of a
    # homogeneous medium, against which a model error means nothing.)
    sys_true = [dataclasses.replace(s, lam=0.0, alpha=complex(wri_synth.alpha_true(s.freq)), rtol=1e-7)
                for s in prob.systems]
    ptrue = dataclasses.replace(prob, m=prob.m_true, systems=sys_true)
    bt = wri.Batch(ptrue, device=dev, mode=wri.KNOWN)
    t0 = time.perf_counter()
    ut, rt_ = wri.solve(bt, mode=wri.KNOWN, max_iter=400000)
    rng = np.random.default_rng(1)
    dl = []
    for k, s in enumerate(prob.systems):
        d = ut[k][torch.as_tensor(np.asarray(s.rec, dtype=np.int64), device=dev)].cpu().numpy().astype(np.complex128)
        sig = 0.01 * np.linalg.norm(d) / np.sqrt(2 * d.size)
        dl.append(d + sig * (rng.standard_normal(d.size) + 1j * rng.standard_normal(d.size)))
    prob = prob.with_data(dl)
    print(f"[awri] data: true-model solves in {time.perf_counter() - t0:.1f} s, iterations "
          f"{[r['iters'] for r in rt_]}, status {sorted(set(r['status'] for r in rt_))}", file=sys.stderr, flush=True)
    m0 = torch.as_tensor(np.asarray(prob.m[0], dtype=np.float32).reshape(-1), device=dev)
    mt = np.asarray(prob.m_true[0], dtype=np.float64).reshape(-1)
    b = g.nb
    inner = np.zeros(g.shape, dtype=bool)
    inner[b:g.nz - b, b:g.ny - b, b:g.nx - b] = True
    inner = inner.reshape(-1)
    err = lambda m: float(np.linalg.norm((m - mt)[inner]) / np.linalg.norm(mt[inner]))
    batch = wri.Batch(prob, device=dev)
    # TV weight: 2 % of the starting objective
    J0, _, _ = wri.objective_grad(batch.__class__(prob.with_rtol(1e-6), device=dev))
    tv0 = wri.tv(g, m0, 1e-9)
    gamma_tv = 0.02 * J0 / tv0
    common = dict(step0=0.002, memory=5, max_step=0.005, m_min=1.0 / 5000.0 ** 2, m_max=1.0 / 1400.0 ** 2,
                  eps_tv=1e-9, mask_sponge=True, max_outer=updates)
    runs = [("WRI eps 1e-6", dict(eps0=1e-6, eps_min=1e-6, gamma=0.0)),
            ("WRI eps 4e-4", dict(eps0=4e-4, eps_min=4e-4, gamma=0.0)),
            ("AWRI eps0 4e-4", dict(eps0=4e-4, eps_min=1e-6, gamma=0.0)),
            ("AWRI-TV eps0 4e-4", dict(eps0=4e-4, eps_min=1e-6, gamma=gamma_tv)),
            ("AWRI-TV eps0 4e-4, warm start", dict(eps0=4e-4, eps_min=1e-6, gamma=gamma_tv, warm_start=True)),
            ("WRI eps 1e-6, warm start", dict(eps0=1e-6, eps_min=1e-6, gamma=0.0, warm_start=True))]
    # warm the solver (autotune, graphs) once
    wri.objective_grad(batch)
    out = []
    for label, kw in runs:
        batch.set_m([m0.clone()])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        code, recs = wri.awri(batch, **common, **kw)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        m = batch.m[0].cpu().numpy().astype(np.float64)
        acc = sum(r["kind"] == "accepted" for r in recs)
        out.append({"run": label, "seconds": round(secs, 3), "accepted_updates": acc,
                    "rejected_trials": sum(r["kind"] == "rejected" for r in recs),
                    "evaluations": len(recs), "cgls_iterations": int(sum(r["iters"] for r in recs)),
                    "final_eps": recs[-1]["eps"], "F_start": recs[0]["F"], "F_end":
                    [r["F"] for r in recs if r["kind"] != "rejected"][-1],
                    "model_error_start": round(err(m0.cpu().numpy().astype(np.float64)), 6),
                    "model_error_end": round(err(m), 6), "status": int(code)})
        print(f"[awri] {label}: {secs:.2f} s, {acc} updates, {out[-1]['cgls_iterations']} CGLS iterations, "
              f"eps {recs[-1]['eps']:.2e}, model error {out[-1]['model_error_start']:.4f} -> "
              f"{out[-1]['model_error_end']:.4f}", file=sys.stderr, flush=True)
    base = out[0]["seconds"]
    print(json.dumps({"metric": "Algorithm 2 outer loop: seconds per run of accepted l-BFGS updates",
                      "workload": f"{name}: {g.nx}x{g.ny}x{g.nz}, {len(prob.systems)} systems, ESTIMATE",
                      "updates": updates, "gamma_tv": gamma_tv,
                      "data": "synthetic: this library's solves of A(m_true) u = alpha_true e (lambda = 0) at the "
                              "receivers, + 1 % noise",
                      "runs": out, "speedup_vs_tight": {r["run"]: round(base / r["seconds"], 3) for r in out}}))


def fwi_bench(name, steps, dev):
    """Reduced FWI (eqs. FWI, PDEsolve, FWI2) against WRI on one workload: time
    and CGLS iterations per objective-and-gradient evaluation of all systems
    at the workload's tolerance (FWI: a forward and an adjoint Helmholtz solve
    per system; WRI: one augmented solve)."""
    import torch
    import wri_synth
    from paper_2410_18429_amd import wri
    prob = wri_synth.make_config(name, seed=0)
    g = prob.grids[0]
    batch = wri.Batch(prob, device=dev)
    out = {}
    for label, fn in (("fwi", lambda: wri.fwi_objective_grad(batch)), ("wri", lambda: wri.objective_grad(batch))):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            val, grads, res = fn()
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        if label == "fwi":
            it_f = [r["iters_fwd"] for r in res]
            it_a = [r["iters_adj"] for r in res]
            st = sorted(set(r["status_fwd"] for r in res) | set(r["status_adj"] for r in res))
            out[label] = {"seconds_per_eval": round(sec, 3), "f": val, "iters_fwd_mean": float(np.mean(it_f)),
                          "iters_adj_mean": float(np.mean(it_a)), "iters_total": int(sum(it_f) + sum(it_a)),
                          "status": st}
        else:
            it = [r["iters"] for r in res]
            out[label] = {"seconds_per_eval": round(sec, 3), "J": val, "iters_mean": float(np.mean(it)),
                          "iters_total": int(sum(it)), "status": sorted(set(r["status"] for r in res))}
        print(f"[fwi] {label}: {sec:.3f} s per evaluation, {out[label]}", file=sys.stderr, flush=True)
    wri.fwi_objective_grad(batch, flags=wri.FLAG_TIMING)
    torch.cuda.synchronize()
    kt = wri.kernel_times()
    out["adjoint_solve_kernels"] = {
        "fwd_gbs": round(kt["fwd_bytes"] / (kt["fwd_ms"] * 1e-3) / 1e9, 1),
        "adj_gbs": round(kt["adj_bytes"] / (kt["adj_ms"] * 1e-3) / 1e9, 1)}
    print(json.dumps({"metric": "objective-and-gradient evaluations: reduced FWI vs WRI",
                      "workload": f"{name}: {g.nx}x{g.ny}x{g.nz}, {len(prob.systems)} systems, ESTIMATE, "
                                  f"rtol {prob.systems[0].rtol:g}",
                      "steps": steps, **out,
                      "fwi_over_wri_time": round(out["fwi"]["seconds_per_eval"] / out["wri"]["seconds_per_eval"], 3)}))


def model_grid_bench(steps, dev):
    """The uneven workload (48^3, 64^3, 96^3 simulation grids at 8 points per
    wavelength for 5/8/12 Hz) with one model grid that covers all three: time
    of an objective-and-gradient evaluation with the model on the model grid
    against the same evaluation with per-grid models, and the resampling
    kernels on their own (HIP events on the current stream)."""
    import torch
    import wri_synth
    from wri_synth import Grid
    from paper_2410_18429_amd import wri
    prob = wri_synth.make_config("uneven", seed=0)
    h_m = 12.0
    ext = [max((getattr(g, a) - 1) * g.h for g in prob.grids) for a in ("nx", "ny", "nz")]
    mgrid = Grid(*[int(np.ceil(e / h_m)) + 1 for e in ext], h=h_m, nb=0, v_ref=1500.0)
    batch = wri.Batch(prob, device=dev)
    m_model = torch.full((mgrid.n,), 1.0 / 2000.0 ** 2, dtype=torch.float32, device=dev)
    batch.set_m([wri.model_to_grid(mgrid, m_model, g) for g in prob.grids])
    out = {}
    for label, fn in (("model_grid", lambda: wri.objective_grad_model(batch, mgrid, m_model)),
                      ("per_grid", lambda: wri.objective_grad(batch))):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            J, _, res = fn()
        torch.cuda.synchronize()
        out[label] = {"seconds_per_eval": round((time.perf_counter() - t0) / steps, 4), "J": J,
                      "iters_total": int(sum(r["iters"] for r in res))}
        print(f"[model-grid] {label}: {out[label]}", file=sys.stderr, flush=True)
    kern = []
    gvec = [torch.randn(g.n, dtype=torch.float32, device=dev) for g in prob.grids]
    gm = torch.empty(mgrid.n, dtype=torch.float32, device=dev)
    reps = 20
    for gi, g in enumerate(prob.grids):
        mg = torch.empty(g.n, dtype=torch.float32, device=dev)
        for name, fn, nbytes in (
                ("model_to_grid", lambda: wri.model_to_grid(mgrid, m_model, g, out=mg), 4 * (mgrid.n + g.n)),
                ("grid_to_model_adjoint", lambda: wri.grid_to_model_adjoint(mgrid, g, gvec[gi], out=gm),
                 4 * (mgrid.n + g.n))):
            fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            kern.append({"kernel": name, "grid": f"{g.nx}^3 h={g.h:g}", "ms": round(ms, 4),
                         "algorithmic_bytes": nbytes, "gbs": round(nbytes / (ms * 1e-3) / 1e9, 1)})
            print(f"[model-grid] {kern[-1]}", file=sys.stderr, flush=True)
    print(json.dumps({"metric": "objective-and-gradient evaluation with the model on one model grid",
                      "workload": f"uneven: 96 systems on 48^3/64^3/96^3 grids; model grid "
                                  f"{mgrid.nx}x{mgrid.ny}x{mgrid.nz} at {h_m:g} m",
                      "steps": steps, **out, "resample_kernels": kern,
                      "overhead": round(out["model_grid"]["seconds_per_eval"] / out["per_grid"]["seconds_per_eval"]
                                        - 1.0, 4)}))


def offgrid_bench(name, steps, dev):
    """Sources and receivers moved off the grid nodes (up to half a cell, seeded):
    time per objective-and-gradient evaluation of the off-grid path against the
    on-grid plain (one system at a time, unfused) and batched paths on the same
    workload."""
    import torch
    import wri_synth
    from paper_2410_18429_amd import wri
    prob = wri_synth.make_config(name, seed=0)
    g = prob.grids[0]
    rng = np.random.default_rng(5)
    def xyz(c):
        return np.array([c % g.nx, (c // g.nx) % g.ny, c // (g.nx * g.ny)], dtype=np.float64) * g.h
    src = [xyz(int(s.src)) + rng.uniform(-0.5, 0.5, 3) * g.h for s in prob.systems]
    rec = [np.array([xyz(int(c)) for c in s.rec]) + rng.uniform(-0.5, 0.5, (len(s.rec), 3)) * g.h
           for s in prob.systems]
    batch = wri.Batch(prob, device=dev)
    out = {}
    for label, fn in (("offgrid", lambda: wri.objective_grad_offgrid(batch, src, rec)),
                      ("plain_on_grid", lambda: wri.objective_grad(batch, flags=wri.FLAG_PLAIN)),
                      ("batched_on_grid", lambda: wri.objective_grad(batch))):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            J, _, res = fn()
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        it = int(sum(r["iters"] for r in res))
        out[label] = {"seconds_per_eval": round(sec, 4), "J": J, "iters_total": it,
                      "ms_per_iteration_per_system": round(1e3 * sec / max(it, 1) * 1.0, 4)}
        print(f"[offgrid] {label}: {out[label]}", file=sys.stderr, flush=True)
    print(json.dumps({"metric": "objective-and-gradient evaluations with off-grid sources and receivers",
                      "workload": f"{name}: {g.nx}x{g.ny}x{g.nz}, {len(prob.systems)} systems, ESTIMATE, "
                                  f"positions moved up to half a cell", "steps": steps, **out}))


def large_bench(freq, rtol, dev):
    """The large workload (256 x 256 x 192, 12.6 M cells per system) one
    frequency band at a time (64 systems, 45 GB of solver vectors): time of an
    objective-and-gradient evaluation and the fused kernels' rates (HIP events
    around every launch in a second, timed evaluation)."""
    import torch
    import wri_synth
    from paper_2410_18429_amd import wri
    p = wri_synth.make_config("large", seed=0)
    band = [k for k, s in enumerate(p.systems) if s.freq == freq]
    q = p.subset(band).with_rtol(rtol)
    g = q.grids[0]
    b = wri.Batch(q, device=dev)
    wri.objective_grad(b)   # warm-up: autotuner and graph capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, _, res = wri.objective_grad(b)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    it = [r["iters"] for r in res]
    wri.objective_grad(b, flags=wri.FLAG_TIMING)
    torch.cuda.synchronize()
    kt = wri.kernel_times()
    out = {"seconds_per_eval": round(sec, 3), "solves_per_s": round(len(band) / sec, 3),
           "iters_mean": float(np.mean(it)), "iters_max": int(max(it)),
           "status": sorted(set(r["status"] for r in res)),
           "fwd_gbs": round(kt["fwd_bytes"] / (kt["fwd_ms"] * 1e-3) / 1e9, 1),
           "adj_gbs": round(kt["adj_bytes"] / (kt["adj_ms"] * 1e-3) / 1e9, 1),
           "fwd_gbs_full_batch": round(kt["fwd_bytes_full"] / (kt["fwd_ms_full"] * 1e-3) / 1e9, 1),
           "adj_gbs_full_batch": round(kt["adj_bytes_full"] / (kt["adj_ms_full"] * 1e-3) / 1e9, 1),
           "tile": f"{kt['tile_w']},{kt['tile_ry']},{kt['tile_tz']},{kt['tile_pf']},{kt['tile_order']}"}
    print(f"[large] {out}", file=sys.stderr, flush=True)
    print(json.dumps({"metric": "large workload, one frequency band per call",
                      "workload": f"large: {g.nx}x{g.ny}x{g.nz}, {len(band)} systems at {freq:g} Hz, ESTIMATE, "
                                  f"rtol {rtol:g}", **out}))


def large_gd_step_size():
    import wri_synth
    p = wri_synth.make_config("large", seed=0)
    return 0.01 * float(np.abs(np.asarray(p.m[0], dtype=np.float32)).max())


def large_gd_model_step(m_in, g_in, m_out):
    """The protocol's model update on the host, for an iteration whose bands
    ran in several calls: g = the sum of the calls' band gradients (float32, in
    band order), m <- m - 0.01 max|m0| g / max|g|."""
    m = np.load(m_in).astype(np.float32)
    g = np.zeros_like(m)
    for f in g_in:
        g += np.load(f).astype(np.float32)
    m -= np.float32(large_gd_step_size()) * g / np.abs(g).max()
    np.save(m_out, m)
    print(json.dumps({"large_gd_step": {"m_in": m_in, "g_in": g_in, "m_out": m_out, "max_abs_g": float(np.abs(g).max())}}))


def large_gd_bench(n_iter, dev, start=0, m_in="", m_out="", warm=False, band_sel=None, g_out="", max_iter=20000):
    """The large workload's protocol: 10 outer gradient-descent iterations over
    all six frequency bands (64 systems each, one call per band), the solver
    tolerance tightened as rtol_k = 1e-2 (1e-3)^(k/9), each iteration the full
    objective, gradient and source-weight estimate of all 384 systems, then
    m <- m - 0.01 max|m0| g / max|g|.  Reports latency per iteration and the
    fused kernels' rates (HIP events around every launch).  With band_sel only
    those bands of one iteration run; their summed gradient goes to g_out and
    the model is not stepped (large_gd_model_step does it on the host)."""
    import torch
    import wri_synth
    from paper_2410_18429_amd import wri
    p = wri_synth.make_config("large", seed=0)
    freqs = sorted(set(s.freq for s in p.systems))
    bands = [[k for k, s in enumerate(p.systems) if s.freq == f] for f in freqs]
    if band_sel is not None:
        if n_iter != 1 or warm:
            raise SystemExit("--large-gd-bands runs one cold iteration (--large-gd 1)")
        bands = [bands[i] for i in band_sel]
    m0 = np.asarray(p.m[0], dtype=np.float32).reshape(-1)
    step = 0.01 * float(np.abs(m0).max())
    # a run may continue an earlier one (iterations start.. with its model)
    m = torch.tensor(np.load(m_in) if m_in else m0, device=dev)
    rows = []
    # warm: every system keeps its wavefield and source weight between outer
    # iterations and starts its next solve there (zeros at the first)
    keep_u = [[torch.zeros(p.grids[0].n, dtype=torch.complex64, device=dev) for _ in band] for band in bands] \
        if warm else None
    keep_a = [[0j for _ in band] for band in bands] if warm else None
    for it in range(start, start + n_iter):
        rtol = 1e-2 * (1e-3) ** (it / 9.0)
        t0 = time.perf_counter()
        J = 0.0
        g = torch.zeros_like(m)
        fb = fms = ab = ams = 0.0
        iters = []
        statuses = []
        for bi, band in enumerate(bands):
            b = wri.Batch(p.subset(band).with_rtol(rtol), device=dev, m=[m])
            if warm:
                b.set_alpha(keep_a[bi])
                Jb, gb, res = wri.objective_grad(b, flags=wri.FLAG_TIMING | wri.FLAG_WARM_START, u_out=keep_u[bi],
                                                 max_iter=max_iter)
                keep_a[bi] = [r["alpha"] for r in res]
            else:
                Jb, gb, res = wri.objective_grad(b, flags=wri.FLAG_TIMING, max_iter=max_iter)
            kt = wri.kernel_times()
            fb += kt["fwd_bytes"]; fms += kt["fwd_ms"]; ab += kt["adj_bytes"]; ams += kt["adj_ms"]
            J += Jb
            g += gb[0]
            iters += [r["iters"] for r in res]
            statuses += [r["status"] for r in res]
            del b, gb
            print(f"[large-gd] iteration {it} band {p.systems[band[0]].freq:g} Hz: "
                  f"{time.perf_counter() - t0:.1f} s so far, max iterations {max(r['iters'] for r in res)}",
                  file=sys.stderr, flush=True)
        if band_sel is None:
            m -= step * g / g.abs().max()
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        rows.append({"iteration": it, "rtol": float(f"{rtol:.3g}"), "seconds": round(sec, 2), "J": J,
                     "cgls_iterations_mean": round(float(np.mean(iters)), 1), "cgls_iterations_max": int(max(iters)),
                     "not_converged": int(sum(1 for x in statuses if x != "converged")),
                     "fwd_gbs": round(fb / (fms * 1e-3) / 1e9, 1), "adj_gbs": round(ab / (ams * 1e-3) / 1e9, 1)})
        if band_sel is not None:
            rows[-1]["bands_hz"] = [freqs[i] for i in band_sel]
        print(f"[large-gd] {rows[-1]}", file=sys.stderr, flush=True)
        if m_out and band_sel is None:
            np.save(m_out, m.cpu().numpy())
        if g_out:
            np.save(g_out, g.cpu().numpy())
    print(json.dumps({"metric": "large workload: latency per outer gradient-descent iteration",
                      "workload": "large: 256x256x192, 384 systems (64 sources x 6 frequencies, one call per band), "
                                  "ESTIMATE" + (", warm-started solves" if warm else ""), "iterations": rows,
                      "total_seconds": round(sum(r["seconds"] for r in rows), 2)}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="differentiation")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--plain-sample", type=int, default=3)
    ap.add_argument("--probe-iters", type=int, default=0,
                    help="counter runs: only run the batch for this many CGLS iterations and exit")
    ap.add_argument("--awri", action="store_true",
                    help="outer-loop measurement instead of the headline: Algorithm 2 (adaptive tolerance, "
                         "l-BFGS, TV) against fixed-tolerance WRI on --config (default medium)")
    ap.add_argument("--awri-updates", type=int, default=20)
    ap.add_argument("--model-grid", action="store_true",
                    help="model-grid measurement instead of the headline: the uneven workload with one model "
                         "grid tied to its three simulation grids")
    ap.add_argument("--offgrid", action="store_true",
                    help="off-grid source/receiver measurement instead of the headline (on --offgrid-config)")
    ap.add_argument("--offgrid-config", default="medium")
    ap.add_argument("--large-band", type=float, default=0.0,
                    help="large-workload measurement instead of the headline: the 64-system band at this "
                         "frequency (4, 6, ..., 14 Hz) at --large-rtol")
    ap.add_argument("--large-rtol", type=float, default=1e-3)
    ap.add_argument("--large-gd", type=int, default=0,
                    help="the large workload's gradient-descent protocol for this many outer iterations (10)")
    ap.add_argument("--large-gd-start", type=int, default=0,
                    help="first outer iteration (a continued run loads its model with --large-gd-m-in)")
    ap.add_argument("--large-gd-m-in", default="", help="model (.npy, float32) to continue from")
    ap.add_argument("--large-gd-m-out", default="", help="write the model after every outer iteration (.npy)")
    ap.add_argument("--large-gd-bands", default="",
                    help="with --large-gd 1: only these frequency bands (indices 0-5, comma-separated) of the "
                         "iteration; their summed gradient goes to --large-gd-g-out and the model is not stepped")
    ap.add_argument("--large-gd-g-out", default="", help="write the iteration's summed gradient (.npy)")
    ap.add_argument("--large-gd-max-iter", type=int, default=20000, help="CGLS iteration cap of the protocol's solves")
    ap.add_argument("--large-gd-step", default="",
                    help="host-only model update: 'M_IN;G1,G2,...;M_OUT' (gradients of one iteration's calls)")
    ap.add_argument("--large-gd-warm", action="store_true",
                    help="start every solve from the system's wavefield and weight of the previous outer iteration")
    ap.add_argument("--fwi", action="store_true",
                    help="reduced-FWI baseline measurement instead of the headline: objective-and-gradient "
                         "evaluations of FWI and WRI on --config")
    ap.add_argument("--cpu-validate", type=int, default=-1,
                    help="CPU oracle run to completion on the medium workload's systems (and this many 128^3 "
                         "systems), the direct oracle at 16^3 and 32^3, GPU iteration counts alongside")
    ap.add_argument("--tail-probe", default="",
                    help="steady-state time per iteration against the number of systems still iterating, for "
                         "these tiles (';'-separated, e.g. '4,4,32,2,4;4,4,32,1,4')")
    ap.add_argument("--precond", action="store_true",
                    help="the V-cycle-preconditioned solver against the plain one on the 128^3 workload "
                         "(time per evaluation, iterations, errors against a tight solve), one JSON line")
    ap.add_argument("--precond-evals", type=int, default=0,
                    help="profiling run: this many preconditioned objective-and-gradient evaluations of the 128^3 "
                         "workload at rtol 1e-4, one JSON line")
    ap.add_argument("--stream-probe", action="store_true",
                    help="only the streaming probe of every access mix (profiling run), one JSON line")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="counter calibration: copy a buffer of this many MiB three times and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the systems are independent: a batch would shard by system across GPUs).", file=sys.stderr)
        sys.exit(2)
    if args.large_gd_step:
        m_in, g_in, m_out = args.large_gd_step.split(";")
        large_gd_model_step(m_in, [f for f in g_in.split(",") if f], m_out)
        return

    import torch
    import wri_synth
    from paper_2410_18429_amd import wri

    dev = "cuda:0"
    if args.copy_probe_mb > 0:
        n = args.copy_probe_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n, "launches": 3}))
        return
    if args.tail_probe:
        print(json.dumps({"tail_probe": tail_probe(dev, args.tail_probe.split(";"))}), flush=True)
        return
    if args.precond:
        precond_bench(dev, args.steps)
        return
    if args.precond_evals > 0:
        prob = wri_synth.make_config("differentiation", seed=0)
        b = wri.Batch(prob, device=dev)
        recs = []
        for i in range(args.precond_evals):
            t0 = time.perf_counter()
            J, _, res = wri.objective_grad_precond(b)
            torch.cuda.synchronize()
            recs.append({"seconds": round(time.perf_counter() - t0, 4), "J": J,
                         "iters_mean": float(np.mean([r["iters"] for r in res]))})
            print(f"[precond] evaluation {i}: {json.dumps(recs[-1])}", file=sys.stderr, flush=True)
        print(json.dumps({"mode": "precond_evals", "evaluations": recs}), flush=True)
        return
    if args.stream_probe:
        print(json.dumps({"stream_ceiling_gbs": stream_ceilings(wri, dev)}), flush=True)
        return
    if args.cpu_validate >= 0:
        cpu_validate(dev, args.cpu_validate)
        return
    if args.awri:
        awri_bench("medium" if args.config == "differentiation" else args.config, args.awri_updates, dev)
        return
    if args.fwi:
        fwi_bench(args.config, args.steps, dev)
        return
    if args.model_grid:
        model_grid_bench(args.steps, dev)
        return
    if args.large_gd > 0:
        sel = [int(v) for v in args.large_gd_bands.split(",")] if args.large_gd_bands else None
        large_gd_bench(args.large_gd, dev, args.large_gd_start, args.large_gd_m_in, args.large_gd_m_out,
                       args.large_gd_warm, sel, args.large_gd_g_out, args.large_gd_max_iter)
        return
    if args.large_band > 0:
        large_bench(args.large_band, args.large_rtol, dev)
        return
    if args.offgrid:
        offgrid_bench(args.offgrid_config, args.steps, dev)
        return
    prob = wri_synth.make_config(args.config, seed=0)
    g = prob.grids[0]
    nsys = len(prob.systems)
    batch = wri.Batch(prob, device=dev)
    n_cells = sum(batch.grid_cells(s.grid) for s in prob.systems)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    log(f"[bench] {args.config}: {nsys} systems, grid {g.nx}x{g.ny}x{g.nz}")
    if args.probe_iters > 0:
        _, _, res = wri.objective_grad(batch, max_iter=args.probe_iters)
        torch.cuda.synchronize()
        print(json.dumps({"probe_iters": args.probe_iters, "systems": nsys, "cells_per_system": g.n,
                          "iters": [r["iters"] for r in res][:4]}))
        return

    for w in range(args.warmup):
        t0 = time.perf_counter()
        J, grads, res = wri.objective_grad(batch)
        torch.cuda.synchronize()
        log(f"[bench] warmup {w}: {time.perf_counter() - t0:.2f} s, iters mean "
            f"{np.mean([r['iters'] for r in res]):.0f}")

    torch.cuda.synchronize()
    times = []
    t_all = time.perf_counter()
    for k in range(args.steps):
        t0 = time.perf_counter()
        J, grads, res = wri.objective_grad(batch)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        log(f"[bench] step {k}: {times[-1]:.3f} s  J={J:.6e}")
    torch.cuda.synchronize()
    total = time.perf_counter() - t_all
    ms_step = 1000.0 * total / args.steps
    value = nsys / (total / args.steps)
    iters = np.array([r["iters"] for r in res])
    statuses = sorted(set(r["status"] for r in res))

    # per-kernel timing: one more step with an event pair around every fused launch
    wri.objective_grad(batch, flags=wri.FLAG_TIMING)
    torch.cuda.synchronize()
    kt = wri.kernel_times()
    fwd_gbs = kt["fwd_bytes"] / (kt["fwd_ms"] * 1e-3) / 1e9
    adj_gbs = kt["adj_bytes"] / (kt["adj_ms"] * 1e-3) / 1e9
    fwd_full_ms = kt["fwd_ms_full"] / max(1, kt["fwd_launches_full"])
    adj_full_ms = kt["adj_ms_full"] / max(1, kt["adj_launches_full"])
    fwd_full_bytes = kt["fwd_bytes_full"] / max(1, kt["fwd_launches_full"])
    adj_full_bytes = kt["adj_bytes_full"] / max(1, kt["adj_launches_full"])
    fwd_full_gbs = fwd_full_bytes / (fwd_full_ms * 1e-3) / 1e9
    adj_full_gbs = adj_full_bytes / (adj_full_ms * 1e-3) / 1e9
    log(f"[bench] kernels (all launches): fwd {kt['fwd_ms'] / kt['fwd_launches']:.3f} ms ({fwd_gbs:.0f} GB/s), "
        f"adj {kt['adj_ms'] / kt['adj_launches']:.3f} ms ({adj_gbs:.0f} GB/s); full batch: fwd "
        f"{fwd_full_ms:.3f} ms ({fwd_full_gbs:.0f} GB/s), adj {adj_full_ms:.3f} ms ({adj_full_gbs:.0f} GB/s)")
    dominant = "fwd" if kt["fwd_ms"] >= kt["adj_ms"] else "adj"
    ach = fwd_gbs if dominant == "fwd" else adj_gbs
    ach_full = fwd_full_gbs if dominant == "fwd" else adj_full_gbs
    tile = f"{kt['tile_w']},{kt['tile_ry']},{kt['tile_tz']},{kt['tile_pf']},{kt['tile_order']}"
    traffic = None
    tt = TRAFFIC["tiles"].get(tile)
    if tt is not None and args.config == "differentiation" and _sources_sha() == TRAFFIC["sources_sha256"]:
        per = lambda v: 1024.0 * (v["fetch_kib"] * TRAFFIC["fetch_scale"] + v["write_kib"] * TRAFFIC["write_scale"])
        # the forward launches alternate between the x-updating and the plain variant
        traffic = round(0.5 * (per(tt["fwd_x"]) + per(tt["fwd"]))) if dominant == "fwd" else round(per(tt["adj"]))
    roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
                "traffic_unit": "HBM bytes per full-batch launch",
                "algorithmic_bytes_full_launch": round(fwd_full_bytes if dominant == "fwd" else adj_full_bytes),
                "kernel": kernel_label(dominant, kt["tile_pf"]),
                "avg_launch_ms": round((kt["fwd_ms"] / kt["fwd_launches"]) if dominant == "fwd"
                                       else (kt["adj_ms"] / kt["adj_launches"]), 4),
                "achieved_full_batch": round(ach_full, 1),
                "frac_full_batch": round(ach_full / HBM_PEAK_GBS, 4),
                "avg_launch_ms_full_batch": round(fwd_full_ms if dominant == "fwd" else adj_full_ms, 4),
                "fwd_gbs": round(fwd_gbs, 1), "adj_gbs": round(adj_gbs, 1),
                "fwd_gbs_full_batch": round(fwd_full_gbs, 1), "adj_gbs_full_batch": round(adj_full_gbs, 1),
                "bytes_per_cell": bytes_note(kt["tile_pf"]), "tile": tile}

    # practical streaming ceilings on this device: a plain kernel with the access
    # mix of each fused launch and none of its arithmetic (wri_stream_probe, 2^27
    # complex64 elements per array, best of five launches per variant), and the
    # forward mix in a tiled plane-by-plane order like the fused kernels' (wri_tile_probe)
    ceil = stream_ceilings(wri, dev)
    pf = kt["tile_pf"]
    if dominant == "fwd":
        # forward launches alternate between the plain and the x-updating mix
        b0, b1 = (28.0, 52.0) if pf >= 2 else (36.0, 60.0)
        mix_ceiling = (b0 + b1) / (b0 / ceil["fwd"] + b1 / ceil["fwd_x"])
        if pf < 2:
            mix_ceiling = None   # the probe has no mix with a stored t
    else:
        mix_ceiling = ceil["adj"]
    roofline["stream_ceiling_gbs"] = {k: round(v, 1) for k, v in ceil.items()}
    roofline["copy_ceiling_gbs"] = round(ceil["copy"], 1)
    roofline["frac_of_copy_ceiling"] = round(ach / ceil["copy"], 4)
    roofline["mix_ceiling_gbs"] = round(mix_ceiling, 1) if mix_ceiling else None
    roofline["frac_of_mix_ceiling"] = round(ach / mix_ceiling, 4) if mix_ceiling else None
    roofline["adj_frac_of_mix_ceiling_full_batch"] = round(adj_full_gbs / ceil["adj"], 4)
    roofline["tile_order_ceiling_gbs"] = round(ceil["fwd_tiles"], 1)
    roofline["frac_of_tile_order_ceiling_full_batch"] = round(ach_full / ceil["fwd_tiles"], 4)
    roofline["adj_frac_of_tile_order_ceiling_full_batch"] = round(adj_full_gbs / ceil["fwd_tiles"], 4)
    log(f"[bench] stream ceilings {json.dumps(roofline['stream_ceiling_gbs'])}; dominant kernel at "
        f"{ach / ceil['copy']:.3f} of the copy, {roofline['frac_of_mix_ceiling']} of its own mix")

    plain = None
    if not args.no_plain and args.plain_sample > 0:
        freqs = sorted(set(s.freq for s in prob.systems))
        pick = [next(i for i, s in enumerate(prob.systems) if s.freq == f) for f in freqs][:args.plain_sample]
        pb = wri.Batch(prob.subset(pick), device=dev)
        wri.objective_grad(pb, flags=wri.FLAG_PLAIN)     # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, pres = wri.objective_grad(pb, flags=wri.FLAG_PLAIN)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        bt = wri.Batch(prob.subset(pick), device=dev)
        wri.objective_grad(bt)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, _, bres = wri.objective_grad(bt)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t1
        plain = {"value": len(pick) / tp, "unit": "solves/s", "systems": pick,
                 "iters": [r["iters"] for r in pres],
                 "same_systems_batched": len(pick) / tb,
                 "sample": f"systems {pick} (one per frequency), one at a time, unfused kernels, host loop"}
        log(f"[bench] plain: {plain['value']:.3f} solves/s on {pick}; batched same systems "
            f"{plain['same_systems_batched']:.3f}")

    cpu = None
    errors = None
    if not args.no_cpu:
        log("[bench] cpu baseline ...")
        cpu = cpu_baseline(args.config, list(range(0, nsys, max(1, nsys // 16))), float(iters.mean()),
                           args.cpu_seconds, g.h)
        log(f"[bench] cpu: {cpu['value']:.5f} solves/s on {cpu['cores']} cores")
        if args.config == "differentiation":
            log("[bench] error against float64 ...")
            errors = error_vs_fp64(prob, batch, dev)
            log(f"[bench] errors: {json.dumps(errors)}")

    line = {
        "metric": METRIC, "value": round(value, 4), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {g.nx}x{g.ny}x{g.nz} h={g.h:g} m, "
                               f"{nsys} systems (16 sources x 5/7/9 Hz), ESTIMATE, rtol 1e-4, "
                               f"solve + source estimate + J + gradient per step",
                   "systems": nsys, "cells_per_system": g.n, "reductions": "f64",
                   "iters_mean": float(iters.mean()), "iters_min": int(iters.min()), "iters_max": int(iters.max()),
                   "status": statuses, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "error_vs_fp64": errors,
        "plain": plain,
        "batched_vs_plain": round(value / plain["value"], 3) if plain else None,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
