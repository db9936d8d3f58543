"""Thin ctypes binding over libwri.so (include/wri.h).

Argument marshalling only: every step of the solve, the source estimate, the
objective and the gradient runs in the library's HIP kernels.  PyTorch is used
for device memory (workspace, wavefields, gradients) and for the current HIP
stream.  There is no CPU fallback: if libwri.so is missing the import of the
library raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_float, c_int, c_int32, c_size_t, c_void_p
from typing import List, Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# WRI_LIBRARY selects another build of the same library (the host-sanitized
# one of the CPU tests); the default is the in-tree libwri.so.
LIB_PATH = os.environ.get("WRI_LIBRARY") or os.path.join(_HERE, "libwri.so")

KNOWN = 0
ESTIMATE = 1
FLAG_PLAIN = 1
FLAG_NO_GRAPH = 2
FLAG_NO_AUTOTUNE = 4
FLAG_UNSCALED_ALPHA = 8
FLAG_TIMING = 16
FLAG_WARM_START = 32
FLAG_ADJOINT_SOURCE = 64


def alpha_scale(h: float) -> float:
    """Scale c of the source column (-c e) of S in ESTIMATE mode: sqrt(42)/h^2."""
    return 42.0 ** 0.5 / (h * h)

OK, NOT_CONVERGED = 0, 1
EINVAL, ERANGE, EDUP, ENOWS, EHIP, EBREAKDOWN = -1, -2, -3, -4, -5, -6
SYS_CONVERGED, SYS_MAX_ITER, SYS_BREAKDOWN, SYS_ZERO_RHS, SYS_DIVERGED = 0, 1, 2, 3, 4
STATUS_NAMES = {0: "converged", 1: "max_iter", 2: "breakdown", 3: "zero_rhs", 4: "diverged"}


class WriGrid(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("nz", c_int32), ("nb", c_int32),
                ("h", c_double), ("v_ref", c_double)]


class WriC32(ctypes.Structure):
    _fields_ = [("re", c_float), ("im", c_float)]


class WriC64(ctypes.Structure):
    _fields_ = [("re", c_double), ("im", c_double)]


class WriSystem(ctypes.Structure):
    _fields_ = [("grid", c_int32), ("src", c_int32), ("omega", c_double), ("lambda_", c_double),
                ("rtol", c_double), ("alpha", WriC64), ("n_rec", c_int32), ("_pad", c_int32),
                ("rec", POINTER(c_int32)), ("d", c_void_p)]


class WriResult(ctypes.Structure):
    _fields_ = [("iters", c_int32), ("status", c_int32), ("relres", c_double), ("J", c_double),
                ("alpha", WriC64), ("alpha_ls", WriC64)]


class WriTiming(ctypes.Structure):
    _fields_ = [("fwd_ms", c_double), ("adj_ms", c_double), ("fwd_launches", ctypes.c_int64),
                ("adj_launches", ctypes.c_int64), ("fwd_bytes", c_double), ("adj_bytes", c_double),
                ("fwd_ms_full", c_double), ("adj_ms_full", c_double), ("fwd_launches_full", ctypes.c_int64),
                ("adj_launches_full", ctypes.c_int64), ("fwd_bytes_full", c_double),
                ("adj_bytes_full", c_double), ("tile_w", ctypes.c_int32), ("tile_ry", ctypes.c_int32),
                ("tile_tz", ctypes.c_int32), ("tile_pf", ctypes.c_int32), ("tile_order", ctypes.c_int32),
                ("tail_switches", ctypes.c_int32)]


class WriAwriOptions(ctypes.Structure):
    _fields_ = [("gamma", c_double), ("eps_tv", c_double), ("eps0", c_double), ("eps_min", c_double),
                ("step0", c_double), ("max_step", c_double), ("m_min", c_double), ("m_max", c_double),
                ("max_outer", c_int32), ("memory", c_int32), ("max_iter", c_int32), ("flags", c_int32),
                ("mask_sponge", c_int32), ("warm_start", c_int32)]


class WriAwriRecord(ctypes.Structure):
    _fields_ = [("F", c_double), ("J", c_double), ("tv", c_double), ("eps", c_double), ("kind", c_int32),
                ("solver_iters", c_int32), ("seconds", c_double)]


AWRI_KINDS = {0: "eval", 1: "accepted", 2: "rejected"}


class WriFwiResult(ctypes.Structure):
    _fields_ = [("f", c_double), ("alpha", WriC64), ("iters_fwd", c_int32), ("iters_adj", c_int32),
                ("status_fwd", c_int32), ("status_adj", c_int32)]


class WriPositions(ctypes.Structure):
    _fields_ = [("src", c_double * 3), ("rec", POINTER(c_double))]


class WriError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"wri error {code}: {msg}")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """Load libwri.so (built in-tree by paper_2410_18429_amd._build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2410_18429_amd._build` "
                          f"(there is no fallback implementation)")
    L = ctypes.CDLL(LIB_PATH)
    vp, pp = c_void_p, POINTER(c_void_p)
    L.wri_workspace_bytes.argtypes = [POINTER(WriGrid), c_int32, POINTER(WriSystem), c_int32, c_int32, c_int32]
    L.wri_workspace_bytes.restype = c_size_t
    L.wri_validate.argtypes = [POINTER(WriGrid), c_int32, POINTER(WriSystem), c_int32, c_int32, c_int32]
    L.wri_validate.restype = c_int
    L.wri_solve.argtypes = [POINTER(WriGrid), c_int32, pp, POINTER(WriSystem), c_int32, c_int32, c_int32,
                            c_int32, pp, POINTER(WriResult), vp, c_size_t, vp]
    L.wri_solve.restype = c_int
    L.wri_solve_noalloc.argtypes = [POINTER(WriGrid), c_int32, pp, POINTER(WriSystem), c_int32, c_int32, c_int32,
                                    c_int32, pp, POINTER(WriResult), vp]
    L.wri_solve_noalloc.restype = c_int
    L.wri_objective_grad.argtypes = [POINTER(WriGrid), c_int32, pp, POINTER(WriSystem), c_int32, c_int32,
                                     c_int32, c_int32, POINTER(c_double), pp, pp, POINTER(WriResult), vp,
                                     c_size_t, vp]
    L.wri_objective_grad.restype = c_int
    L.estimate_source.argtypes = [POINTER(WriGrid), c_int32, pp, POINTER(WriSystem), c_int32, c_int32,
                                  c_int32, POINTER(WriC64), pp, POINTER(WriResult), vp, c_size_t, vp]
    L.estimate_source.restype = c_int
    L.wri_apply_helmholtz.argtypes = [POINTER(WriGrid), vp, c_double, vp, vp, c_int32, vp]
    L.wri_apply_helmholtz.restype = c_int
    L.wri_strerror.argtypes = [c_int]
    L.wri_strerror.restype = ctypes.c_char_p
    L.wri_last_error.argtypes = []
    L.wri_last_error.restype = ctypes.c_char_p
    L.wri_version.argtypes = []
    L.wri_version.restype = c_int
    L.wri_kernel_times.argtypes = [POINTER(WriTiming)]
    L.wri_kernel_times.restype = c_int
    L.wri_precond_workspace_bytes.argtypes = [POINTER(WriGrid), c_int32, POINTER(WriSystem), c_int32, c_int32]
    L.wri_precond_workspace_bytes.restype = c_size_t
    L.wri_objective_grad_precond.argtypes = [POINTER(WriGrid), c_int32, pp, POINTER(WriSystem), c_int32, c_int32,
                                             c_int32, c_int32, POINTER(c_double), pp, pp, POINTER(WriResult), vp,
                                             c_size_t, vp]
    L.wri_objective_grad_precond.restype = c_int
    L.wri_stream_probe_bytes.argtypes = [c_int32, ctypes.c_int64]
    L.wri_stream_probe_bytes.restype = c_size_t
    L.wri_stream_probe.argtypes = [c_int32, ctypes.c_int64, c_int32, vp, c_size_t, vp, POINTER(c_double)]
    L.wri_stream_probe.restype = c_int
    L.wri_tile_probe_bytes.argtypes = [c_int32, c_int32, c_int32, c_int32]
    L.wri_tile_probe_bytes.restype = c_size_t
    L.wri_tile_probe.argtypes = [c_int32, c_int32, c_int32, c_int32, c_int32, vp, c_size_t, vp, POINTER(c_double)]
    L.wri_tile_probe.restype = c_int
    L.wri_tv_workspace_bytes.argtypes = [POINTER(WriGrid)]
    L.wri_tv_workspace_bytes.restype = c_size_t
    L.wri_tv.argtypes = [POINTER(WriGrid), vp, c_double, c_double, POINTER(c_double), vp, vp, c_size_t, vp]
    L.wri_tv.restype = c_int
    L.wri_lbfgs_workspace_bytes.argtypes = [c_int32]
    L.wri_lbfgs_workspace_bytes.restype = c_size_t
    L.wri_lbfgs_direction.argtypes = [ctypes.c_int64, vp, vp, vp, c_int32, c_int32, c_int32, c_double, vp, vp,
                                      c_size_t, vp]
    L.wri_lbfgs_direction.restype = c_int
    L.wri_awri_workspace_bytes.argtypes = [POINTER(WriGrid), POINTER(WriSystem), c_int32, c_int32, c_int32,
                                           c_int32]
    L.wri_awri_workspace_bytes.restype = c_size_t
    L.wri_awri.argtypes = [POINTER(WriGrid), vp, POINTER(WriSystem), c_int32, c_int32, POINTER(WriAwriOptions),
                           POINTER(WriAwriRecord), c_int32, POINTER(c_int32), vp, c_size_t, vp]
    L.wri_awri.restype = c_int
    L.wri_fwi_workspace_bytes.argtypes = [POINTER(WriGrid), c_int32, POINTER(WriSystem), c_int32, c_int32,
                                          c_int32]
    L.wri_fwi_workspace_bytes.restype = c_size_t
    L.wri_fwi_objective_grad.argtypes = [POINTER(WriGrid), c_int32, pp, POINTER(WriSystem), c_int32, c_int32,
                                         c_int32, c_int32, POINTER(c_double), pp, pp, POINTER(WriFwiResult), vp,
                                         c_size_t, vp]
    L.wri_fwi_objective_grad.restype = c_int
    L.wri_model_to_grid.argtypes = [POINTER(WriGrid), vp, POINTER(WriGrid), vp, vp]
    L.wri_model_to_grid.restype = c_int
    L.wri_grid_to_model_adjoint.argtypes = [POINTER(WriGrid), POINTER(WriGrid), vp, vp, c_int32, vp]
    L.wri_grid_to_model_adjoint.restype = c_int
    L.wri_model_workspace_bytes.argtypes = [POINTER(WriGrid), POINTER(WriGrid), c_int32, POINTER(WriSystem),
                                            c_int32, c_int32, c_int32]
    L.wri_model_workspace_bytes.restype = c_size_t
    L.wri_objective_grad_model.argtypes = [POINTER(WriGrid), vp, POINTER(WriGrid), c_int32, POINTER(WriSystem),
                                           c_int32, c_int32, c_int32, c_int32, POINTER(c_double), vp, pp,
                                           POINTER(WriResult), vp, c_size_t, vp]
    L.wri_objective_grad_model.restype = c_int
    L.wri_offgrid_workspace_bytes.argtypes = [POINTER(WriGrid), c_int32, POINTER(WriSystem), c_int32,
                                              POINTER(WriPositions)]
    L.wri_offgrid_workspace_bytes.restype = c_size_t
    L.wri_objective_grad_offgrid.argtypes = [POINTER(WriGrid), c_int32, pp, POINTER(WriSystem), c_int32,
                                             POINTER(WriPositions), c_int32, c_int32, c_int32, POINTER(c_double), pp,
                                             pp, POINTER(WriResult), vp, c_size_t, vp]
    L.wri_objective_grad_offgrid.restype = c_int
    _lib = L
    return L


EXPORTED = ("wri_workspace_bytes", "wri_validate", "wri_solve", "wri_solve_noalloc", "wri_precond_workspace_bytes",
            "wri_objective_grad_precond", "wri_stream_probe_bytes",
            "wri_stream_probe", "wri_tile_probe_bytes", "wri_tile_probe", "wri_objective_grad", "estimate_source",
            "wri_apply_helmholtz", "wri_kernel_times", "wri_strerror", "wri_last_error", "wri_version",
            "wri_tv_workspace_bytes", "wri_tv", "wri_lbfgs_workspace_bytes", "wri_lbfgs_direction",
            "wri_awri_workspace_bytes", "wri_awri", "wri_fwi_workspace_bytes", "wri_fwi_objective_grad",
            "wri_model_to_grid", "wri_grid_to_model_adjoint", "wri_model_workspace_bytes",
            "wri_objective_grad_model", "wri_offgrid_workspace_bytes", "wri_objective_grad_offgrid")


def kernel_times() -> dict:
    """Totals of the last FLAG_TIMING call on this thread."""
    t = WriTiming()
    _check(lib().wri_kernel_times(ctypes.byref(t)))
    return {name: getattr(t, name) for name, _ in WriTiming._fields_}


STREAM_MIXES = {"copy": 0, "fwd": 1, "fwd_x": 2, "adj": 3}


def stream_probe(mix: str, n: int, reps: int = 5, device="cuda") -> float:
    """wri_stream_probe: GB/s of a plain streaming kernel with the access mix
    of a fused launch (see STREAM_MIXES) over n complex64 elements per array."""
    code = STREAM_MIXES[mix]
    nbytes = lib().wri_stream_probe_bytes(code, int(n))
    if nbytes == 0:
        raise WriError(EINVAL, "bad stream probe size")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    out = c_double(0.0)
    _check(lib().wri_stream_probe(code, int(n), int(reps), c_void_p(ws.data_ptr()), nbytes,
                                  _stream(torch.device(device)), ctypes.byref(out)))
    del ws
    return out.value


def tile_probe(nx: int, ny: int, nz: int, n_sys: int, reps: int = 5, device="cuda") -> float:
    """wri_tile_probe: GB/s of a plain streaming kernel with the forward pass's
    byte mix in a tiled plane-by-plane order like the fused kernels' (64 x 16 x 32
    tiles) over n_sys grids of nx x ny x nz."""
    nbytes = lib().wri_tile_probe_bytes(int(nx), int(ny), int(nz), int(n_sys))
    if nbytes == 0:
        raise WriError(EINVAL, "bad tile probe shape")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    out = c_double(0.0)
    _check(lib().wri_tile_probe(int(nx), int(ny), int(nz), int(n_sys), int(reps), c_void_p(ws.data_ptr()), nbytes,
                                _stream(torch.device(device)), ctypes.byref(out)))
    del ws
    return out.value


def last_error() -> str:
    return lib().wri_last_error().decode()


def _check(code: int, allow_not_converged=True) -> int:
    if code < 0 or (code == NOT_CONVERGED and not allow_not_converged):
        raise WriError(code, last_error() or lib().wri_strerror(code).decode())
    return code


def _stream(device) -> c_void_p:
    return c_void_p(torch.cuda.current_stream(device).cuda_stream)


def make_grid(g) -> WriGrid:
    return WriGrid(int(g.nx), int(g.ny), int(g.nz), int(g.nb), float(g.h), float(g.v_ref))


class Batch:
    """Device-side copy of a set of systems (a wri_synth.Problem or any object
    with .grids, .m and .systems), plus a cached workspace.

    m: per grid float32 device tensors (defaults to problem.m); d: complex64
    device tensors per system; receiver indices stay on the host."""

    def __init__(self, problem, device="cuda", m=None, mode=None):
        self.device = torch.device(device)
        self.problem = problem
        mode = problem.mode if mode is None else mode
        self.mode = {"known": KNOWN, "estimate": ESTIMATE}.get(mode, mode)
        self.grids_py = list(problem.grids)
        self.cgrids = (WriGrid * max(1, len(self.grids_py)))(*[make_grid(g) for g in self.grids_py])
        src_m = problem.m if m is None else m
        self.m = [torch.as_tensor(np.asarray(mm) if not torch.is_tensor(mm) else mm)
                  .to(self.device, torch.float32).contiguous().reshape(-1) for mm in src_m]
        self.rec = [np.ascontiguousarray(np.asarray(s.rec, dtype=np.int32)) for s in problem.systems]
        self.d = [torch.as_tensor(np.asarray(s.d, dtype=np.complex64)).to(self.device).contiguous()
                  for s in problem.systems]
        systems = []
        for k, s in enumerate(problem.systems):
            a = complex(s.alpha)
            systems.append(WriSystem(
                int(s.grid), int(s.src), float(s.omega), float(s.lam), float(s.rtol), WriC64(a.real, a.imag),
                int(self.rec[k].size), 0,
                self.rec[k].ctypes.data_as(POINTER(c_int32)) if self.rec[k].size else None,
                c_void_p(self.d[k].data_ptr()) if self.rec[k].size else None))
        self.nsys = len(systems)
        self.csys = (WriSystem * max(1, self.nsys))(*systems)
        self._ws = {}

    def set_m(self, m_list):
        self.m = [mm.to(self.device, torch.float32).contiguous().reshape(-1) for mm in m_list]

    def set_alpha(self, alphas):
        """Per-system source weights: the known weight (KNOWN mode) or the
        initial guess of a warm start (ESTIMATE mode)."""
        for k, a in enumerate(alphas):
            self.csys[k].alpha = WriC64(float(np.real(a)), float(np.imag(a)))

    def set_rtol(self, rtol):
        r = [rtol] * self.nsys if np.isscalar(rtol) else list(rtol)
        for k in range(self.nsys):
            self.csys[k].rtol = float(r[k])

    def m_ptrs(self):
        return (c_void_p * max(1, len(self.m)))(*[c_void_p(t.data_ptr()) for t in self.m])

    def workspace(self, mode, flags):
        nbytes = lib().wri_workspace_bytes(self.cgrids, len(self.grids_py), self.csys, self.nsys, mode, flags)
        if nbytes == 0:
            raise WriError(EINVAL, last_error())
        key = (mode, flags & FLAG_PLAIN)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < nbytes:
            ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self._ws[key] = ws
        return ws

    def fwi_workspace(self, mode, flags):
        nbytes = lib().wri_fwi_workspace_bytes(self.cgrids, len(self.grids_py), self.csys, self.nsys, mode, flags)
        if nbytes == 0:
            raise WriError(EINVAL, last_error())
        key = ("fwi", mode, flags & FLAG_PLAIN)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < nbytes:
            ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self._ws[key] = ws
        return ws

    def grid_cells(self, g):
        gg = self.grids_py[g]
        return gg.nx * gg.ny * gg.nz


def _results(res, n):
    return [dict(iters=res[k].iters, status=STATUS_NAMES.get(res[k].status, res[k].status),
                 relres=res[k].relres, J=res[k].J, alpha=complex(res[k].alpha.re, res[k].alpha.im),
                 alpha_ls=complex(res[k].alpha_ls.re, res[k].alpha_ls.im)) for k in range(n)]


def _u_ptrs(batch: Batch, u_out):
    if u_out is None:
        return None
    return (c_void_p * max(1, batch.nsys))(*[c_void_p(u.data_ptr()) if u is not None else None for u in u_out])


def alloc_wavefields(batch: Batch) -> List[torch.Tensor]:
    return [torch.empty(batch.grid_cells(s.grid), dtype=torch.complex64, device=batch.device)
            for s in batch.problem.systems]


def solve(batch: Batch, mode=None, max_iter=20000, flags=0, u_out=None, return_u=True):
    """Batched augmented solve. Returns (u list or None, results list)."""
    mode = batch.mode if mode is None else mode
    if return_u and u_out is None:
        u_out = alloc_wavefields(batch)
    ws = batch.workspace(mode, flags)
    res = (WriResult * max(1, batch.nsys))()
    code = lib().wri_solve(batch.cgrids, len(batch.grids_py), batch.m_ptrs(), batch.csys, batch.nsys, mode,
                           int(max_iter), int(flags), _u_ptrs(batch, u_out), res, c_void_p(ws.data_ptr()),
                           ws.numel(), _stream(batch.device))
    _check(code)
    return u_out, _results(res, batch.nsys)


def objective_grad_precond(batch: Batch, mode=None, max_iter=20000, flags=0, u_out=None, grad_out=None,
                           with_grad=True):
    """wri_objective_grad_precond: the V-cycle-preconditioned CGLS.  Returns
    (J or None, per-grid gradients or None, results); u_out as in solve()."""
    mode = batch.mode if mode is None else mode
    grads = None
    gptr = None
    if with_grad:
        grads = grad_out or [torch.empty(batch.grid_cells(g), dtype=torch.float32, device=batch.device)
                             for g in range(len(batch.grids_py))]
        gptr = (c_void_p * max(1, len(grads)))(*[c_void_p(g.data_ptr()) for g in grads])
    nbytes = lib().wri_precond_workspace_bytes(batch.cgrids, len(batch.grids_py), batch.csys, batch.nsys, mode)
    if nbytes == 0:
        raise WriError(EINVAL, last_error())
    key = ("precond", mode)
    ws = batch._ws.get(key)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=batch.device)
        batch._ws[key] = ws
    res = (WriResult * max(1, batch.nsys))()
    J = c_double(0.0)
    code = lib().wri_objective_grad_precond(batch.cgrids, len(batch.grids_py), batch.m_ptrs(), batch.csys,
                                            batch.nsys, mode, int(max_iter), int(flags),
                                            ctypes.byref(J) if with_grad else None, gptr, _u_ptrs(batch, u_out),
                                            res, c_void_p(ws.data_ptr()), ws.numel(), _stream(batch.device))
    _check(code)
    return (J.value if with_grad else None), grads, _results(res, batch.nsys)


NOALLOC_SCRATCH_BYTES = 64 << 20   # WRI_NOALLOC_SCRATCH_BYTES


def solve_noalloc(batch: Batch, mode=None, max_iter=20000, flags=0, u_out=None):
    """wri_solve_noalloc: the batched solve on the library's fixed device
    scratch (no workspace, no device allocation inside the call).  u_out
    (one tensor per system) is allocated here when not given.  Returns
    (u list, results list)."""
    mode = batch.mode if mode is None else mode
    if u_out is None:
        u_out = alloc_wavefields(batch)
    res = (WriResult * max(1, batch.nsys))()
    code = lib().wri_solve_noalloc(batch.cgrids, len(batch.grids_py), batch.m_ptrs(), batch.csys, batch.nsys,
                                   mode, int(max_iter), int(flags), _u_ptrs(batch, u_out), res,
                                   _stream(batch.device))
    _check(code)
    return u_out, _results(res, batch.nsys)


def objective_grad(batch: Batch, mode=None, max_iter=20000, flags=0, u_out=None, grad_out=None):
    """J (float), per-grid gradients (float32 device tensors), results."""
    mode = batch.mode if mode is None else mode
    grads = grad_out or [torch.empty(batch.grid_cells(g), dtype=torch.float32, device=batch.device)
                         for g in range(len(batch.grids_py))]
    gptr = (c_void_p * max(1, len(grads)))(*[c_void_p(g.data_ptr()) for g in grads])
    ws = batch.workspace(mode, flags)
    res = (WriResult * max(1, batch.nsys))()
    J = c_double(0.0)
    code = lib().wri_objective_grad(batch.cgrids, len(batch.grids_py), batch.m_ptrs(), batch.csys, batch.nsys,
                                    mode, int(max_iter), int(flags), ctypes.byref(J), gptr,
                                    _u_ptrs(batch, u_out), res, c_void_p(ws.data_ptr()), ws.numel(),
                                    _stream(batch.device))
    _check(code)
    return J.value, grads, _results(res, batch.nsys)


def fwi_objective_grad(batch: Batch, mode=None, max_iter=20000, flags=0, u_out=None, grad_out=None,
                       with_grad=True):
    """Reduced FWI baseline (eqs. FWI, PDEsolve, FWI2): f (float), per-grid
    gradients (float32 device tensors, or None), per-system results
    (f, alpha, iterations and statuses of the forward and adjoint solves)."""
    mode = batch.mode if mode is None else mode
    grads = None
    gptr = None
    if with_grad:
        grads = grad_out or [torch.empty(batch.grid_cells(g), dtype=torch.float32, device=batch.device)
                             for g in range(len(batch.grids_py))]
        gptr = (c_void_p * max(1, len(grads)))(*[c_void_p(g.data_ptr()) for g in grads])
    ws = batch.fwi_workspace(mode, flags)
    res = (WriFwiResult * max(1, batch.nsys))()
    f = c_double(0.0)
    code = lib().wri_fwi_objective_grad(batch.cgrids, len(batch.grids_py), batch.m_ptrs(), batch.csys, batch.nsys,
                                        mode, int(max_iter), int(flags), ctypes.byref(f), gptr,
                                        _u_ptrs(batch, u_out), res, c_void_p(ws.data_ptr()), ws.numel(),
                                        _stream(batch.device))
    _check(code)
    out = [dict(f=res[k].f, alpha=complex(res[k].alpha.re, res[k].alpha.im), iters_fwd=res[k].iters_fwd,
                iters_adj=res[k].iters_adj, status_fwd=STATUS_NAMES.get(res[k].status_fwd, res[k].status_fwd),
                status_adj=STATUS_NAMES.get(res[k].status_adj, res[k].status_adj)) for k in range(batch.nsys)]
    return f.value, grads, out


def model_to_grid(model_grid, m_model: torch.Tensor, grid, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Trilinear resampling of a model (float32 device tensor on model_grid)
    onto `grid` (common origin at cell 0)."""
    mg = make_grid(model_grid)
    gg = make_grid(grid)
    m_model = m_model.contiguous()
    out = out if out is not None else torch.empty(grid.nx * grid.ny * grid.nz, dtype=torch.float32,
                                                  device=m_model.device)
    _check(lib().wri_model_to_grid(ctypes.byref(mg), c_void_p(m_model.data_ptr()), ctypes.byref(gg),
                                   c_void_p(out.data_ptr()), _stream(m_model.device)))
    return out


def grid_to_model_adjoint(model_grid, grid, g_grid: torch.Tensor, out: Optional[torch.Tensor] = None,
                          accumulate=False) -> torch.Tensor:
    """Transpose of model_to_grid applied to g_grid (float32 device tensor on `grid`)."""
    mg = make_grid(model_grid)
    gg = make_grid(grid)
    g_grid = g_grid.contiguous()
    if out is None:
        out = torch.empty(model_grid.nx * model_grid.ny * model_grid.nz, dtype=torch.float32, device=g_grid.device)
    _check(lib().wri_grid_to_model_adjoint(ctypes.byref(mg), ctypes.byref(gg), c_void_p(g_grid.data_ptr()),
                                           c_void_p(out.data_ptr()), int(bool(accumulate)), _stream(g_grid.device)))
    return out


def objective_grad_model(batch: Batch, model_grid, m_model: torch.Tensor, mode=None, max_iter=20000, flags=0,
                         u_out=None, with_grad=True):
    """J, dJ/dm on the model grid (float32 device tensor, or None), results:
    every simulation grid of the batch takes its model by trilinear resampling
    of m_model."""
    mode = batch.mode if mode is None else mode
    mg = make_grid(model_grid)
    nbytes = lib().wri_model_workspace_bytes(ctypes.byref(mg), batch.cgrids, len(batch.grids_py), batch.csys,
                                             batch.nsys, mode, flags)
    if nbytes == 0:
        raise WriError(EINVAL, last_error())
    key = ("model", mode, flags & FLAG_PLAIN)
    ws = batch._ws.get(key)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=batch.device)
        batch._ws[key] = ws
    m_model = m_model.to(batch.device, torch.float32).contiguous().reshape(-1)
    grad = torch.empty_like(m_model) if with_grad else None
    res = (WriResult * max(1, batch.nsys))()
    J = c_double(0.0)
    code = lib().wri_objective_grad_model(ctypes.byref(mg), c_void_p(m_model.data_ptr()), batch.cgrids,
                                          len(batch.grids_py), batch.csys, batch.nsys, mode, int(max_iter),
                                          int(flags), ctypes.byref(J),
                                          c_void_p(grad.data_ptr()) if grad is not None else None,
                                          _u_ptrs(batch, u_out), res, c_void_p(ws.data_ptr()), ws.numel(),
                                          _stream(batch.device))
    _check(code)
    return J.value, grad, _results(res, batch.nsys)


def objective_grad_offgrid(batch: Batch, src_xyz, rec_xyz, mode=None, max_iter=20000, flags=0, u_out=None,
                           with_grad=True):
    """Objective, per-grid gradients (or None) and results with sources and
    receivers at arbitrary points: src_xyz[k] (3 floats, metres) and rec_xyz[k]
    (n_rec x 3) replace system k's source and receiver cells (trilinear
    weights; cell (i, j, k) at (i h, j h, k h))."""
    mode = batch.mode if mode is None else mode
    recs = [np.ascontiguousarray(np.asarray(r, dtype=np.float64).reshape(-1, 3)) for r in rec_xyz]
    for k, r in enumerate(recs):
        if r.shape[0] != batch.csys[k].n_rec:
            raise ValueError(f"system {k}: {r.shape[0]} receiver positions for {batch.csys[k].n_rec} data")
    pos = (WriPositions * max(1, batch.nsys))(
        *[WriPositions((c_double * 3)(*[float(v) for v in src_xyz[k]]),
                       recs[k].ctypes.data_as(POINTER(c_double)) if recs[k].size else None)
          for k in range(batch.nsys)])
    nbytes = lib().wri_offgrid_workspace_bytes(batch.cgrids, len(batch.grids_py), batch.csys, batch.nsys, pos)
    if nbytes == 0:
        raise WriError(EINVAL, last_error())
    key = ("offgrid",)
    ws = batch._ws.get(key)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=batch.device)
        batch._ws[key] = ws
    grads, gptr = None, None
    if with_grad:
        grads = [torch.empty(batch.grid_cells(g), dtype=torch.float32, device=batch.device)
                 for g in range(len(batch.grids_py))]
        gptr = (c_void_p * max(1, len(grads)))(*[c_void_p(g.data_ptr()) for g in grads])
    res = (WriResult * max(1, batch.nsys))()
    J = c_double(0.0)
    code = lib().wri_objective_grad_offgrid(batch.cgrids, len(batch.grids_py), batch.m_ptrs(), batch.csys,
                                            batch.nsys, pos, mode, int(max_iter), int(flags), ctypes.byref(J), gptr,
                                            _u_ptrs(batch, u_out), res, c_void_p(ws.data_ptr()), ws.numel(),
                                            _stream(batch.device))
    _check(code)
    return J.value, grads, _results(res, batch.nsys)


def estimate_source(batch: Batch, max_iter=20000, flags=0, u_out=None):
    """On-the-fly source weights (complex128 numpy array) and results."""
    ws = batch.workspace(ESTIMATE, flags)
    res = (WriResult * max(1, batch.nsys))()
    alpha = (WriC64 * max(1, batch.nsys))()
    code = lib().estimate_source(batch.cgrids, len(batch.grids_py), batch.m_ptrs(), batch.csys, batch.nsys,
                                 int(max_iter), int(flags), alpha, _u_ptrs(batch, u_out), res,
                                 c_void_p(ws.data_ptr()), ws.numel(), _stream(batch.device))
    _check(code)
    return np.array([complex(alpha[k].re, alpha[k].im) for k in range(batch.nsys)]), _results(res, batch.nsys)


def apply_helmholtz(grid, m: torch.Tensor, omega: float, x: torch.Tensor, adjoint=False) -> torch.Tensor:
    """y = A x (or A^H x) on one grid; x complex64 device tensor of n cells."""
    cg = make_grid(grid)
    x = x.contiguous()
    m = m.to(torch.float32).contiguous()
    y = torch.empty_like(x)
    code = lib().wri_apply_helmholtz(ctypes.byref(cg), c_void_p(m.data_ptr()), float(omega),
                                     c_void_p(x.data_ptr()), c_void_p(y.data_ptr()), 1 if adjoint else 0,
                                     _stream(x.device))
    _check(code)
    return y


class WRIObjective(torch.autograd.Function):
    """J(m) of the batch at model(s) m, differentiable in m.

    forward runs wri_objective_grad (one batched solve); backward returns
    grad_output * dJ/dm with no further solve (the envelope theorem: the
    wavefield and source weight minimise J for fixed m)."""

    @staticmethod
    def forward(ctx, batch: Batch, mode, max_iter, flags, *ms):
        batch.set_m(ms)
        J, grads, res = objective_grad(batch, mode=mode, max_iter=max_iter, flags=flags)
        ctx.save_for_backward(*grads)
        ctx.shapes = [m.shape for m in ms]
        ctx.results = res
        batch.last_results = res
        return torch.tensor(J, dtype=torch.float64, device=ms[0].device)

    @staticmethod
    def backward(ctx, gJ):
        grads = ctx.saved_tensors
        out = [(gJ.to(torch.float32) * g).reshape(s) for g, s in zip(grads, ctx.shapes)]
        return (None, None, None, None, *out)


def wri_objective(batch: Batch, *ms, mode=None, max_iter=20000, flags=0):
    """Functional form of WRIObjective."""
    return WRIObjective.apply(batch, batch.mode if mode is None else mode, max_iter, flags, *ms)


class FWIObjective(torch.autograd.Function):
    """Reduced FWI objective f(m) (eq. FWI2) of the batch, differentiable in
    m: forward runs wri_fwi_objective_grad (forward and adjoint solves);
    backward returns grad_output * df/dm."""

    @staticmethod
    def forward(ctx, batch: Batch, mode, max_iter, flags, *ms):
        batch.set_m(ms)
        f, grads, res = fwi_objective_grad(batch, mode=mode, max_iter=max_iter, flags=flags)
        ctx.save_for_backward(*grads)
        ctx.shapes = [m.shape for m in ms]
        batch.last_results = res
        return torch.tensor(f, dtype=torch.float64, device=ms[0].device)

    @staticmethod
    def backward(ctx, gf):
        grads = ctx.saved_tensors
        out = [(gf.to(torch.float32) * g).reshape(s) for g, s in zip(grads, ctx.shapes)]
        return (None, None, None, None, *out)


def fwi_objective(batch: Batch, *ms, mode=None, max_iter=20000, flags=0):
    """Functional form of FWIObjective."""
    return FWIObjective.apply(batch, batch.mode if mode is None else mode, max_iter, flags, *ms)


class ModelGridObjective(torch.autograd.Function):
    """J(m_model) with every simulation grid's model resampled from one model
    grid, differentiable in m_model (wri_objective_grad_model)."""

    @staticmethod
    def forward(ctx, batch: Batch, model_grid, mode, max_iter, flags, m_model):
        J, g, res = objective_grad_model(batch, model_grid, m_model, mode=mode, max_iter=max_iter, flags=flags)
        ctx.save_for_backward(g)
        ctx.shape = m_model.shape
        batch.last_results = res
        return torch.tensor(J, dtype=torch.float64, device=m_model.device)

    @staticmethod
    def backward(ctx, gJ):
        (g,) = ctx.saved_tensors
        return (None, None, None, None, None, (gJ.to(torch.float32) * g).reshape(ctx.shape))


def model_grid_objective(batch: Batch, model_grid, m_model: torch.Tensor, mode=None, max_iter=20000, flags=0):
    """Functional form of ModelGridObjective."""
    return ModelGridObjective.apply(batch, model_grid, batch.mode if mode is None else mode, max_iter, flags,
                                    m_model)


# --------------------------------------------------------------------------
# outer loop: TV, l-BFGS direction, Algorithm 2 (adaptive tolerance)
# --------------------------------------------------------------------------

def tv(grid, m: torch.Tensor, eps: float, gamma: float = 0.0, grad: Optional[torch.Tensor] = None) -> float:
    """Smoothed TV of m (device float32) on `grid` (a wri_synth.Grid);
    grad (device float32) += gamma * dTV/dm when given."""
    cg = make_grid(grid)
    nbytes = lib().wri_tv_workspace_bytes(ctypes.byref(cg))
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=m.device)
    v = c_double(0.0)
    _check(lib().wri_tv(ctypes.byref(cg), c_void_p(m.data_ptr()), float(eps), float(gamma), ctypes.byref(v),
                        c_void_p(grad.data_ptr()) if grad is not None else None, c_void_p(ws.data_ptr()),
                        ws.numel(), _stream(m.device)))
    return v.value


def lbfgs_direction(g: torch.Tensor, S: torch.Tensor, Y: torch.Tensor, count: int, newest: int,
                    h0: float) -> torch.Tensor:
    """-H g from the curvature-pair rings S, Y (device float32, [capacity, n])."""
    cap = int(S.shape[0]) if S is not None else 0
    nbytes = lib().wri_lbfgs_workspace_bytes(cap)
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=g.device)
    d = torch.empty_like(g)
    _check(lib().wri_lbfgs_direction(g.numel(), c_void_p(g.data_ptr()),
                                     c_void_p(S.data_ptr()) if cap else None, c_void_p(Y.data_ptr()) if cap else None,
                                     cap, int(count), int(newest), float(h0), c_void_p(d.data_ptr()),
                                     c_void_p(ws.data_ptr()), ws.numel(), _stream(g.device)))
    return d


def awri(batch: Batch, gamma=0.0, eps_tv=1e-9, eps0=1e-3, eps_min=1e-8, step0=0.01, max_step=0.0,
         m_min=0.0, m_max=0.0, max_outer=10, memory=5, max_iter=20000, flags=0, mask_sponge=True,
         warm_start=False, mode=None, history_cap=4096):
    """Algorithm 2 on the batch's single grid.  The batch's model tensor is
    updated in place.  Returns (status code, list of evaluation records)."""
    if len(batch.grids_py) != 1:
        raise WriError(EINVAL, "the outer loop runs on one grid")
    mode = batch.mode if mode is None else mode
    o = WriAwriOptions(float(gamma), float(eps_tv), float(eps0), float(eps_min), float(step0), float(max_step),
                       float(m_min), float(m_max), int(max_outer), int(memory), int(max_iter), int(flags),
                       int(bool(mask_sponge)), int(bool(warm_start)))
    qflags = int(flags) | (FLAG_WARM_START if warm_start else 0)
    nbytes = lib().wri_awri_workspace_bytes(batch.cgrids, batch.csys, batch.nsys, mode, qflags, int(memory))
    if nbytes == 0:
        raise WriError(EINVAL, last_error())
    ws = torch.empty(nbytes, dtype=torch.uint8, device=batch.device)
    hist = (WriAwriRecord * max(1, history_cap))()
    nrec = c_int32(0)
    code = lib().wri_awri(batch.cgrids, c_void_p(batch.m[0].data_ptr()), batch.csys, batch.nsys, mode,
                          ctypes.byref(o), hist, int(history_cap), ctypes.byref(nrec), c_void_p(ws.data_ptr()),
                          ws.numel(), _stream(batch.device))
    if code < 0:
        _check(code)
    recs = [dict(F=hist[i].F, J=hist[i].J, TV=hist[i].tv, eps=hist[i].eps, kind=AWRI_KINDS[hist[i].kind],
                 iters=hist[i].solver_iters, seconds=hist[i].seconds) for i in range(min(nrec.value, history_cap))]
    return code, recs
