"""The seeded input generator: deterministic, in-bounds, distinct receivers."""
import numpy as np
import pytest

import wri_synth


@pytest.mark.parametrize("name", ["tiny", "medium", "uneven", "differentiation", "crop32", "large"])
def test_configs_are_valid_and_deterministic(name):
    p = wri_synth.make_config(name, seed=0)
    q = wri_synth.make_config(name, seed=0)
    expect = {"tiny": 1, "medium": 8, "uneven": 96, "differentiation": 48, "crop32": 48, "large": 384}
    assert len(p.systems) == expect[name]
    for s, t in zip(p.systems, q.systems):
        g = p.grids[s.grid]
        assert 0 <= s.src < g.n
        assert s.rec.dtype == np.int32 and s.rec.size > 0
        assert np.all((s.rec >= 0) & (s.rec < g.n))
        assert np.unique(s.rec).size == s.rec.size
        assert np.array_equal(s.d, t.d) and s.rtol == t.rtol
        assert np.all(np.isfinite(s.d)) and np.abs(s.d).max() > 0
    for m, g in zip(p.m, p.grids):
        assert m.shape == g.shape and np.all(m > 0)
        v = 1 / np.sqrt(m)
        assert v.min() >= 1500.0 - 1e-9 and v.max() <= 4500.0 * 1.1 + 1e-6


def test_uneven_tolerances_and_grids():
    p = wri_synth.make_config("uneven")
    r = np.array([s.rtol for s in p.systems])
    assert r.min() >= 1e-5 and r.max() <= 1e-2
    assert [g.nx for g in p.grids] == [48, 64, 96]
    for g, f in zip(p.grids, (5.0, 8.0, 12.0)):
        assert abs(g.h * 8 * f - 1500.0) < 1e-9        # 8 points per wavelength at 1500 m/s


def test_noise_level():
    rng = np.random.default_rng(0)
    d = np.ones(10000, complex)
    dn = wri_synth.add_noise(d, rng)
    assert abs(np.linalg.norm(dn - d) / np.linalg.norm(d) - 0.01) < 5e-4
