"""Host-only checks of the C ABI (no device calls): the library loads, exports
every function declared in include/wri.h, its struct layout matches the header,
and argument validation / workspace sizing behave as documented."""
import ctypes
import os
import re
import subprocess
import sys
import tempfile

import numpy as np
import pytest

from paper_2410_18429_amd import wri

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wri.h")


def _header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       txt, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_library_exports_every_header_function():
    L = wri.lib()
    names = _header_functions()
    assert set(names) == set(wri.EXPORTED), names
    for n in names:
        assert hasattr(L, n), n
    assert L.wri_version() >= 100


def test_struct_layout_matches_header():
    src = r"""
    #include <stdio.h>
    #include <stddef.h>
    #include "wri.h"
    int main(void) {
      printf("%zu %zu %zu\n", sizeof(wri_grid), sizeof(wri_system), sizeof(wri_result));
      printf("%zu %zu %zu %zu %zu %zu %zu %zu\n", offsetof(wri_system, omega), offsetof(wri_system, lambda),
             offsetof(wri_system, rtol), offsetof(wri_system, alpha), offsetof(wri_system, n_rec),
             offsetof(wri_system, rec), offsetof(wri_system, d), offsetof(wri_grid, h));
      printf("%zu %zu %zu %zu\n", offsetof(wri_result, relres), offsetof(wri_result, J),
             offsetof(wri_result, alpha), offsetof(wri_result, alpha_ls));
      printf("%zu %zu %zu %zu\n", sizeof(wri_timing), offsetof(wri_timing, fwd_ms_full),
             offsetof(wri_timing, adj_bytes_full), offsetof(wri_timing, tile_order));
      printf("%zu %zu %zu %zu %zu %zu\n", sizeof(wri_awri_options), offsetof(wri_awri_options, max_outer),
             offsetof(wri_awri_options, mask_sponge), sizeof(wri_awri_record), offsetof(wri_awri_record, kind),
             offsetof(wri_awri_record, seconds));
      printf("%zu %zu %zu %zu\n", sizeof(wri_fwi_result), offsetof(wri_fwi_result, alpha),
             offsetof(wri_fwi_result, iters_adj), offsetof(wri_fwi_result, status_adj));
      return 0;
    }
    """
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.check_output([exe]).decode().split()
    vals = list(map(int, out))
    S, G, R = wri.WriSystem, wri.WriGrid, wri.WriResult
    assert vals[:3] == [ctypes.sizeof(G), ctypes.sizeof(S), ctypes.sizeof(R)]
    assert vals[3:11] == [S.omega.offset, S.lambda_.offset, S.rtol.offset, S.alpha.offset, S.n_rec.offset,
                          S.rec.offset, S.d.offset, G.h.offset]
    assert vals[11:15] == [R.relres.offset, R.J.offset, R.alpha.offset, R.alpha_ls.offset]
    Tm = wri.WriTiming
    assert vals[15:19] == [ctypes.sizeof(Tm), Tm.fwd_ms_full.offset, Tm.adj_bytes_full.offset, Tm.tile_order.offset]
    O, Rr = wri.WriAwriOptions, wri.WriAwriRecord
    assert vals[19:25] == [ctypes.sizeof(O), O.max_outer.offset, O.mask_sponge.offset, ctypes.sizeof(Rr),
                           Rr.kind.offset, Rr.seconds.offset]
    F = wri.WriFwiResult
    assert vals[25:] == [ctypes.sizeof(F), F.alpha.offset, F.iters_adj.offset, F.status_adj.offset]


def _mk(n_rec=4, dup=False, src=5, rec_bad=False, grid=0, lam=0.1, omega=30.0, rtol=1e-6, nb=2, v_ref=1500.0):
    g = (wri.WriGrid * 1)(wri.WriGrid(10, 9, 8, nb, 10.0, v_ref))
    rec = np.arange(n_rec, dtype=np.int32) * 7
    if dup and n_rec > 1:
        rec[1] = rec[0]
    if rec_bad:
        rec[-1] = 10 * 9 * 8
    fake_d = ctypes.c_void_p(0x1000)  # never dereferenced by host-only calls
    s = (wri.WriSystem * 1)(wri.WriSystem(grid, src, omega, lam, rtol, wri.WriC64(1.0, 0.0), n_rec, 0,
                                          rec.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), fake_d))
    return g, s, rec


@pytest.mark.parametrize("kw,code", [
    ({}, wri.OK),
    (dict(dup=True), wri.EDUP),
    (dict(rec_bad=True), wri.ERANGE),
    (dict(src=-1), wri.ERANGE),
    (dict(src=720), wri.ERANGE),
    (dict(grid=1), wri.EINVAL),
    (dict(lam=-1.0), wri.EINVAL),
    (dict(omega=float("nan")), wri.EINVAL),
    (dict(rtol=-1e-3), wri.EINVAL),
    (dict(v_ref=0.0), wri.EINVAL),
    (dict(v_ref=0.0, nb=0), wri.OK),
    (dict(n_rec=0), wri.OK),
])
def test_validate_codes(kw, code):
    g, s, rec = _mk(**kw)
    assert wri.lib().wri_validate(g, 1, s, 1, wri.ESTIMATE, 100) == code
    if code != wri.OK:
        assert wri.last_error() != ""


def test_validate_mode_and_iters():
    g, s, rec = _mk()
    L = wri.lib()
    assert L.wri_validate(g, 1, s, 1, 7, 100) == wri.EINVAL
    assert L.wri_validate(g, 1, s, 1, wri.KNOWN, -1) == wri.EINVAL
    bad = (wri.WriGrid * 1)(wri.WriGrid(0, 9, 8, 0, 10.0, 1500.0))
    assert L.wri_validate(bad, 1, s, 1, wri.KNOWN, 1) == wri.EINVAL
    huge = (wri.WriGrid * 1)(wri.WriGrid(2048, 2048, 512, 0, 10.0, 1500.0))
    assert L.wri_validate(huge, 1, None, 0, wri.KNOWN, 1) == wri.EINVAL
    wide = (wri.WriGrid * 1)(wri.WriGrid(2000, 2000, 10, 0, 10.0, 1500.0))   # 4e6 cells in one plane
    assert L.wri_validate(wide, 1, None, 0, wri.KNOWN, 1) == wri.EINVAL
    assert "plane" in wri.last_error()
    ok = (wri.WriGrid * 1)(wri.WriGrid(1930, 1930, 10, 0, 10.0, 1500.0))
    assert L.wri_validate(ok, 1, None, 0, wri.KNOWN, 1) == wri.OK


def test_workspace_bytes_and_dedup():
    L = wri.lib()
    g, s, rec = _mk()
    one = L.wri_workspace_bytes(g, 1, s, 1, wri.ESTIMATE, 0)
    assert one > 7 * 8 * 720
    two = (wri.WriSystem * 2)(s[0], s[0])
    both = L.wri_workspace_bytes(g, 1, two, 2, wri.ESTIMATE, 0)
    assert one < both < 2 * one + 4096
    plain = L.wri_workspace_bytes(g, 1, two, 2, wri.ESTIMATE, wri.FLAG_PLAIN)
    assert plain < both
    gb, sb, _ = _mk(dup=True)
    assert L.wri_workspace_bytes(gb, 1, sb, 1, wri.ESTIMATE, 0) == 0


def test_solve_rejects_small_workspace_before_any_device_call():
    L = wri.lib()
    g, s, rec = _mk()
    res = (wri.WriResult * 1)()
    m = (ctypes.c_void_p * 1)(ctypes.c_void_p(0x2000))
    code = L.wri_solve(g, 1, m, s, 1, wri.ESTIMATE, 10, 0, None, res, ctypes.c_void_p(0x3000), 16, None)
    assert code == wri.ENOWS
    assert "workspace" in wri.last_error()
    code = L.wri_solve(g, 1, m, s, 1, wri.ESTIMATE, 10, 0, None, None, ctypes.c_void_p(0x3000), 1 << 40, None)
    assert code == wri.EINVAL
    g2, s2, _ = _mk(dup=True)
    code = L.wri_solve(g2, 1, m, s2, 1, wri.ESTIMATE, 10, 0, None, res, ctypes.c_void_p(0x3000), 1 << 40, None)
    assert code == wri.EDUP


def test_strerror():
    L = wri.lib()
    for c in (0, 1, -1, -2, -3, -4, -5, -6):
        assert len(L.wri_strerror(c)) > 0


def test_outer_loop_entry_points_validate_before_device_work():
    L = wri.lib()
    g = (wri.WriGrid * 1)(wri.WriGrid(10, 9, 8, 2, 10.0, 1500.0))
    v = ctypes.c_double(0.0)
    assert L.wri_tv(None, ctypes.c_void_p(0x1000), 1e-9, 0.0, ctypes.byref(v), None, None, 0, None) == wri.EINVAL
    assert L.wri_tv(g, ctypes.c_void_p(0x1000), -1.0, 0.0, ctypes.byref(v), None, None, 0, None) == wri.EINVAL
    assert L.wri_tv(g, ctypes.c_void_p(0x1000), 1e-9, 0.0, ctypes.byref(v), None, ctypes.c_void_p(0x2000), 8,
                    None) == wri.ENOWS
    assert L.wri_tv_workspace_bytes(g) >= 3 * 8 * 720
    # l-BFGS ring checks
    p = ctypes.c_void_p(0x1000)
    assert L.wri_lbfgs_direction(100, p, p, p, 4, 5, 0, 1.0, p, p, 1 << 20, None) == wri.EINVAL
    assert L.wri_lbfgs_direction(100, p, p, p, 4, 2, 4, 1.0, p, p, 1 << 20, None) == wri.EINVAL
    assert L.wri_lbfgs_direction(100, p, None, None, 0, 0, 0, 0.0, p, p, 1 << 20, None) == wri.EINVAL
    assert L.wri_lbfgs_direction(100, p, p, p, 4, 2, 1, 1.0, p, p, 8, None) == wri.ENOWS
    # driver options
    gg, s, rec = _mk()
    o = wri.WriAwriOptions(0.0, 1e-9, 1e-3, 1e-2, 0.01, 0.0, 0.0, 0.0, 3, 2, 100, 0, 1, 0)   # eps_min > eps0
    n = ctypes.c_int32(0)
    assert L.wri_awri(gg, p, s, 1, wri.ESTIMATE, ctypes.byref(o), None, 0, ctypes.byref(n), p, 1 << 40,
                      None) == wri.EINVAL
    o.eps_min = 1e-6
    o.m_min, o.m_max = 2e-7, 1e-7
    assert L.wri_awri(gg, p, s, 1, wri.ESTIMATE, ctypes.byref(o), None, 0, ctypes.byref(n), p, 1 << 40,
                      None) == wri.EINVAL
    o.m_min, o.m_max = 0.0, 0.0
    need = L.wri_awri_workspace_bytes(gg, s, 1, wri.ESTIMATE, 0, 2)
    assert need > L.wri_workspace_bytes(gg, 1, s, 1, wri.ESTIMATE, 0) + 7 * 4 * 720
    need_warm = L.wri_awri_workspace_bytes(gg, s, 1, wri.ESTIMATE, wri.FLAG_WARM_START, 2)
    assert need_warm >= need + 2 * 8 * 720
    o.warm_start = 1
    assert L.wri_awri(gg, p, s, 1, wri.ESTIMATE, ctypes.byref(o), None, 0, ctypes.byref(n), p, need_warm - 1,
                      None) == wri.ENOWS
    o.warm_start = 0
    assert L.wri_awri(gg, p, s, 1, wri.ESTIMATE, ctypes.byref(o), None, 0, ctypes.byref(n), p, need - 1,
                      None) == wri.ENOWS


def test_warm_start_flag_validation():
    L = wri.lib()
    g, s, rec = _mk()
    res = (wri.WriResult * 1)()
    m = (ctypes.c_void_p * 1)(ctypes.c_void_p(0x2000))
    ws = ctypes.c_void_p(0x3000)
    code = L.wri_solve(g, 1, m, s, 1, wri.ESTIMATE, 10, wri.FLAG_WARM_START, None, res, ws, 1 << 40, None)
    assert code == wri.EINVAL and "u_out" in wri.last_error()
    u = (ctypes.c_void_p * 1)(None)
    code = L.wri_solve(g, 1, m, s, 1, wri.ESTIMATE, 10, wri.FLAG_WARM_START, u, res, ws, 1 << 40, None)
    assert code == wri.EINVAL
    u = (ctypes.c_void_p * 1)(ctypes.c_void_p(0x4000))
    code = L.wri_solve(g, 1, m, s, 1, wri.ESTIMATE, 10, wri.FLAG_WARM_START | wri.FLAG_PLAIN, u, res, ws, 1 << 40,
                       None)
    assert code == wri.EINVAL and "batched" in wri.last_error()


def test_adjoint_source_flag_validation():
    """Receiver-source solves: KNOWN mode, lambda = 0, no warm start; rejected
    before any device call."""
    L = wri.lib()
    res = (wri.WriResult * 1)()
    m = (ctypes.c_void_p * 1)(ctypes.c_void_p(0x2000))
    ws = ctypes.c_void_p(0x3000)
    g, s, rec = _mk(lam=0.0)
    code = L.wri_solve(g, 1, m, s, 1, wri.ESTIMATE, 10, wri.FLAG_ADJOINT_SOURCE, None, res, ws, 1 << 40, None)
    assert code == wri.EINVAL and "WRI_KNOWN" in wri.last_error()
    u = (ctypes.c_void_p * 1)(ctypes.c_void_p(0x4000))
    code = L.wri_solve(g, 1, m, s, 1, wri.KNOWN, 10, wri.FLAG_ADJOINT_SOURCE | wri.FLAG_WARM_START, u, res, ws,
                       1 << 40, None)
    assert code == wri.EINVAL
    g, s, rec = _mk(lam=0.1)
    code = L.wri_solve(g, 1, m, s, 1, wri.KNOWN, 10, wri.FLAG_ADJOINT_SOURCE, None, res, ws, 1 << 40, None)
    assert code == wri.EINVAL and "lambda" in wri.last_error()


def test_fwi_entry_point_validates_before_device_work():
    L = wri.lib()
    g, s, rec = _mk(lam=0.3)   # lambda is not used by the FWI baseline
    res = (wri.WriFwiResult * 1)()
    m = (ctypes.c_void_p * 1)(ctypes.c_void_p(0x2000))
    f = ctypes.c_double(0.0)
    need = L.wri_fwi_workspace_bytes(g, 1, s, 1, wri.ESTIMATE, 0)
    solver = L.wri_workspace_bytes(g, 1, s, 1, wri.KNOWN, 0)
    assert need > solver + 2 * 720 * 8
    assert L.wri_fwi_workspace_bytes(g, 1, s, 1, 7, 0) == 0
    code = L.wri_fwi_objective_grad(g, 1, m, s, 1, wri.ESTIMATE, 10, 0, f, None, None, res,
                                    ctypes.c_void_p(0x3000), need - 1, None)
    assert code == wri.ENOWS
    code = L.wri_fwi_objective_grad(g, 1, m, s, 1, wri.ESTIMATE, 10, 0, None, None, None, res,
                                    ctypes.c_void_p(0x3000), need, None)
    assert code == wri.EINVAL and "f_out" in wri.last_error()
    code = L.wri_fwi_objective_grad(g, 1, m, s, 1, wri.ESTIMATE, 10, wri.FLAG_WARM_START, f, None, None, res,
                                    ctypes.c_void_p(0x3000), need, None)
    assert code == wri.EINVAL
    code = L.wri_fwi_objective_grad(g, 1, m, s, 1, wri.ESTIMATE, 10, wri.FLAG_ADJOINT_SOURCE, f, None, None, res,
                                    ctypes.c_void_p(0x3000), need, None)
    assert code == wri.EINVAL
    gbad = (ctypes.c_void_p * 1)(None)
    code = L.wri_fwi_objective_grad(g, 1, m, s, 1, wri.ESTIMATE, 10, 0, f, gbad, None, res,
                                    ctypes.c_void_p(0x3000), need, None)
    assert code == wri.EINVAL and "grad" in wri.last_error()
    g2, s2, _ = _mk(dup=True)
    assert L.wri_fwi_objective_grad(g2, 1, m, s2, 1, wri.ESTIMATE, 10, 0, f, None, None, res,
                                    ctypes.c_void_p(0x3000), need, None) == wri.EDUP


def test_resampling_entry_points_validate_before_device_work():
    L = wri.lib()
    model = wri.WriGrid(10, 9, 8, 0, 10.0, 1500.0)
    ok = wri.WriGrid(5, 4, 4, 0, 20.0, 1500.0)        # (n-1) h = 80, 60, 60 <= 90, 80, 70
    beyond = wri.WriGrid(6, 4, 4, 0, 20.0, 1500.0)    # 100 > 90 along x
    fine = wri.WriGrid(81, 72, 64, 0, 1.0, 1500.0)   # 10x finer than the model
    p = ctypes.c_void_p(0x1000)
    assert L.wri_model_to_grid(ctypes.byref(model), p, ctypes.byref(beyond), p, None) == wri.EINVAL
    assert "beyond" in wri.last_error()
    assert L.wri_model_to_grid(ctypes.byref(model), p, ctypes.byref(fine), p, None) == wri.EINVAL
    assert "finer" in wri.last_error()
    assert L.wri_model_to_grid(ctypes.byref(model), None, ctypes.byref(ok), p, None) == wri.EINVAL
    assert L.wri_grid_to_model_adjoint(ctypes.byref(model), ctypes.byref(ok), p, None, 0, None) == wri.EINVAL
    g, s, rec = _mk()
    gg = (wri.WriGrid * 1)(wri.WriGrid(10, 9, 8, 2, 10.0, 1500.0))
    need = L.wri_model_workspace_bytes(ctypes.byref(model), gg, 1, s, 1, wri.ESTIMATE, 0)
    assert need > L.wri_workspace_bytes(gg, 1, s, 1, wri.ESTIMATE, 0) + 2 * 720 * 4
    res = (wri.WriResult * 1)()
    J = ctypes.c_double(0.0)
    code = L.wri_objective_grad_model(ctypes.byref(model), p, gg, 1, s, 1, wri.ESTIMATE, 10, 0, J, p, None, res,
                                      p, need - 1, None)
    assert code == wri.ENOWS
    gb = (wri.WriGrid * 1)(wri.WriGrid(11, 9, 8, 2, 10.0, 1500.0))   # beyond the model grid
    assert L.wri_model_workspace_bytes(ctypes.byref(model), gb, 1, s, 1, wri.ESTIMATE, 0) == 0


def test_offgrid_entry_point_validates_before_device_work():
    L = wri.lib()
    g, s, rec = _mk()
    rxyz = np.zeros((4, 3))
    pos = (wri.WriPositions * 1)(wri.WriPositions((ctypes.c_double * 3)(5.0, 5.0, 5.0),
                                                  rxyz.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    need = L.wri_offgrid_workspace_bytes(g, 1, s, 1, pos)
    assert need > 5 * 720 * 8
    res = (wri.WriResult * 1)()
    m = (ctypes.c_void_p * 1)(ctypes.c_void_p(0x2000))
    J = ctypes.c_double(0.0)
    ws = ctypes.c_void_p(0x3000)
    assert L.wri_objective_grad_offgrid(g, 1, m, s, 1, pos, wri.ESTIMATE, 10, 0, J, None, None, res, ws, need - 1,
                                        None) == wri.ENOWS
    assert L.wri_objective_grad_offgrid(g, 1, m, s, 1, pos, wri.ESTIMATE, 10, wri.FLAG_WARM_START, J, None, None, res,
                                        ws, need, None) == wri.EINVAL
    rxyz[2, 1] = float("nan")
    assert L.wri_offgrid_workspace_bytes(g, 1, s, 1, pos) == 0
    assert L.wri_objective_grad_offgrid(g, 1, m, s, 1, pos, wri.ESTIMATE, 10, 0, J, None, None, res, ws, need,
                                        None) == wri.EINVAL
    assert "position" in wri.last_error()
    assert ctypes.sizeof(wri.WriPositions) == 32


def test_noalloc_rejects_systems_beyond_the_scratch_before_any_device_call():
    """wri_solve_noalloc checks the workspace its systems need against the
    fixed scratch (WRI_NOALLOC_SCRATCH_BYTES) before any device call, and
    validates its arguments like wri_solve."""
    txt = open(HEADER).read()
    assert re.search(r"#define\s+WRI_NOALLOC_SCRATCH_BYTES\s+\(\(size_t\)64 << 20\)", txt)
    assert wri.NOALLOC_SCRATCH_BYTES == 64 << 20
    L = wri.lib()
    rec = np.arange(4, dtype=np.int32)
    g = (wri.WriGrid * 1)(wri.WriGrid(128, 128, 128, 10, 10.0, 1500.0))
    s = (wri.WriSystem * 1)(wri.WriSystem(0, 5, 30.0, 0.1, 1e-4, wri.WriC64(1.0, 0.0), 4, 0,
                                          rec.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                          ctypes.c_void_p(0x1000)))
    assert L.wri_workspace_bytes(g, 1, s, 1, wri.ESTIMATE, 0) > wri.NOALLOC_SCRATCH_BYTES
    res = (wri.WriResult * 1)()
    m = (ctypes.c_void_p * 1)(ctypes.c_void_p(0x2000))
    assert L.wri_solve_noalloc(g, 1, m, s, 1, wri.ESTIMATE, 10, 0, None, res, None) == wri.ENOWS
    assert "scratch" in wri.last_error()
    g2, s2, _ = _mk()
    assert L.wri_solve_noalloc(g2, 1, m, s2, 1, wri.ESTIMATE, 10, wri.FLAG_TIMING, None, res, None) == wri.EINVAL
    g3, s3, _ = _mk(dup=True)
    assert L.wri_solve_noalloc(g3, 1, m, s3, 1, wri.ESTIMATE, 10, 0, None, res, None) == wri.EDUP
    g4, s4, _ = _mk(src=720)
    assert L.wri_solve_noalloc(g4, 1, m, s4, 1, wri.ESTIMATE, 10, 0, None, res, None) == wri.ERANGE


def test_host_code_under_address_and_undefined_behaviour_sanitizers():
    """The host-only cases of this file again, in a subprocess against the
    library built with AddressSanitizer and UndefinedBehaviorSanitizer on its
    host code (`python -m paper_2410_18429_amd._build --host-sanitized`, also
    done by the package build), the ASan runtime preloaded: an out-of-bounds
    access, a use after free or undefined behaviour in argument validation,
    the planner, the workspace layout or the receiver maps aborts the run."""
    san = os.path.join(ROOT, "paper_2410_18429_amd", "libwri_hostsan.so")
    if not os.path.exists(san):
        pytest.skip("host-sanitized library not built")
    syms = subprocess.check_output(["nm", "-D", san]).decode()
    assert "__asan_report" in syms and "__ubsan_handle" in syms
    rt = subprocess.check_output(["/opt/rocm/llvm/bin/clang", "-print-file-name=libclang_rt.asan-x86_64.so"])
    rt = rt.decode().strip()
    assert os.path.exists(rt), rt
    env = dict(os.environ, LD_PRELOAD=rt, WRI_LIBRARY=san,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    proc = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", __file__,
                           "-k", "not sanitizers"], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    tail = (proc.stdout + proc.stderr)[-3000:]
    assert proc.returncode == 0, tail
    assert "passed" in proc.stdout and "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail


def test_probe_entry_points_validate_before_device_work():
    """The streaming probes size and check their arguments on the host: bad
    mixes, odd or non-positive sizes, tile shapes that are not multiples of
    64 x 16 x 32, missing workspace and a NULL result pointer are rejected
    before any launch."""
    L = wri.lib()
    assert L.wri_stream_probe_bytes(4, 1 << 10) == 0
    assert L.wri_stream_probe_bytes(0, 1023) == 0
    assert L.wri_stream_probe_bytes(1, 1 << 10) > 0
    assert L.wri_tile_probe_bytes(128, 128, 128, 48) > 48 * 128 ** 3 * 8 * 3
    for shape in ((100, 128, 128, 1), (128, 24, 128, 1), (128, 128, 40, 1), (128, 128, 128, 0), (0, 16, 32, 1)):
        assert L.wri_tile_probe_bytes(*shape) == 0, shape
    out = ctypes.c_double(0.0)
    assert L.wri_tile_probe(100, 128, 128, 1, 3, None, 0, None, ctypes.byref(out)) == wri.EINVAL
    assert L.wri_tile_probe(128, 128, 128, 1, 0, None, 0, None, ctypes.byref(out)) == wri.EINVAL
    assert L.wri_tile_probe(128, 128, 128, 1, 3, None, 0, None, None) == wri.EINVAL
    assert L.wri_tile_probe(128, 128, 128, 1, 3, None, 0, None, ctypes.byref(out)) == wri.ENOWS
    assert L.wri_tile_probe(4096, 4096, 256, 64, 3, None, 0, None, ctypes.byref(out)) == wri.EINVAL
    assert L.wri_stream_probe(5, 1 << 10, 3, None, 0, None, ctypes.byref(out)) == wri.EINVAL
    assert L.wri_stream_probe(1, 1 << 10, 3, None, 0, None, ctypes.byref(out)) == wri.ENOWS
    assert out.value == 0.0
