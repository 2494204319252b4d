"""Parity of the HIP library (through its C ABI) with the FP64 oracle.

Both sides start from the same FP32 inputs (the oracle widens them to
FP64). The bar for fields is the stated one: max |q_gpu - q_oracle| /
max |q_oracle| <= 1e-5 after the run. Integer-exact properties (TE/TM
zeros, determinism, step splitting) are compared bit for bit.
"""
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2301_13601_amd import scenes

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def qla():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_13601_amd import qla as q
    q.lib()
    return q


def gpu_run(qla, n, q, delta, steps, mode="eq28", beta="phys", chunks=None):
    n32 = np.ascontiguousarray(n, dtype=np.float32)
    q32 = np.ascontiguousarray(q, dtype=np.float32)
    sim = qla.Simulation(n32, q32, delta, mode, beta)
    for k in (chunks or [steps]):
        sim.step(k)
    out = sim.fields("Q")
    sim.close()
    return out


def oracle_run(n, q, delta, steps, mode="eq28", beta="phys"):
    n32 = np.asarray(n, dtype=np.float32).astype(np.float64)
    q32 = np.asarray(q, dtype=np.float32).astype(np.float64)
    return O.run(n32, q32, delta, steps, mode, beta)


def rel_err(got, want):
    return float(np.abs(got.astype(np.float64) - want).max() / np.abs(want).max())


def _case(tag):
    print(f"[parity] {tag}", flush=True)


# --------------------------------------------------------------------------
# The 256 x 256 scattering run, in full.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("pol", ["Ez", "Ey"])
def test_single_instance_full_run(qla, pol):
    sc = scenes.config_single()
    q0 = sc.q if pol == "Ez" else scenes.gaussian_pulse(256, 256, "Ey", 48, 20)
    _case(f"single 256x256 {pol} 500 steps")
    got = gpu_run(qla, sc.n, q0, sc.delta, sc.steps, "eq28")
    want = oracle_run(sc.n, q0, sc.delta, sc.steps, "eq28")
    err = rel_err(got, want)
    e0 = O.energy(q0.astype(np.float32))
    drift_gpu = O.energy(got) / e0 - 1
    drift_orc = O.energy(want) / e0 - 1
    print(f"  max rel field err {err:.3e}; energy drift gpu {drift_gpu:+.6e} oracle {drift_orc:+.6e}")
    assert err <= TOL
    assert abs(drift_gpu - drift_orc) < 1e-5 * max(1.0, abs(drift_orc))


# --------------------------------------------------------------------------
# Small, odd and ragged lattices; both potential placements and scalings.
# --------------------------------------------------------------------------

SHAPES = [(1, 1), (3, 5), (7, 1), (1, 9), (2, 2), (17, 13), (120, 7), (121, 33),
          (250, 19), (300, 70), (64, 200)]


@pytest.mark.parametrize("nx,ny", SHAPES)
@pytest.mark.parametrize("mode", ["eq23", "eq28"])
def test_small_lattices_smooth_medium(qla, nx, ny, mode):
    seed = 31 * nx + ny
    n = scenes.smooth_random_profile(nx, ny, seed, 1.0, 3.0)
    q = scenes.random_state(nx, ny, seed + 1)
    _case(f"smooth {nx}x{ny} {mode}")
    got = gpu_run(qla, n, q, 0.3, 9, mode)
    want = oracle_run(n, q, 0.3, 9, mode)
    assert rel_err(got, want) <= TOL


@pytest.mark.parametrize("nx,ny", [(5, 3), (40, 24), (130, 66)])
@pytest.mark.parametrize("mode", ["eq23", "eq28"])
@pytest.mark.parametrize("beta", ["phys", "lattice", "off"])
def test_rough_medium_wide_angles(qla, nx, ny, mode, beta):
    # n drawn per site: potential angles beyond the short-series range
    seed = 7 * nx + ny
    n = scenes.random_profile(nx, ny, seed, 1.0, 3.0)
    q = scenes.random_state(nx, ny, seed + 2)
    _case(f"rough {nx}x{ny} {mode} {beta}")
    got = gpu_run(qla, n, q, 0.3, 6, mode, beta)
    want = oracle_run(n, q, 0.3, 6, mode, beta)
    assert rel_err(got, want) <= TOL


@pytest.mark.parametrize("delta", [0.05, 0.3, 1.0])
def test_delta_range(qla, delta):
    n = scenes.smooth_random_profile(96, 40, 5, 1.0, 2.5)
    q = scenes.random_state(96, 40, 6)
    _case(f"delta {delta}")
    got = gpu_run(qla, n, q, delta, 8)
    want = oracle_run(n, q, delta, 8)
    assert rel_err(got, want) <= TOL


# --------------------------------------------------------------------------
# Exact properties.
# --------------------------------------------------------------------------

def test_step_splitting_and_determinism_are_bitwise(qla):
    n = scenes.smooth_random_profile(130, 50, 9, 1.0, 3.0)
    q = scenes.random_state(130, 50, 10)
    _case("split/determinism")
    a = gpu_run(qla, n, q, 0.3, 7)
    b = gpu_run(qla, n, q, 0.3, 7, chunks=[3, 4])
    c = gpu_run(qla, n, q, 0.3, 7, chunks=[1, 1, 5])
    assert np.array_equal(a, b) and np.array_equal(a, c)


@pytest.mark.parametrize("pol,zero", [("Ez", (0, 1, 5)), ("Ey", (2, 3, 4))])
def test_te_tm_blocks_stay_exactly_zero(qla, pol, zero):
    n = scenes.object_profile(200, 90, "ellipse", (30, 20), (1.5, 2.0, 3.0), 6.0)
    q = scenes.gaussian_pulse(200, 90, pol, x0=40, width=10)
    _case(f"te/tm {pol}")
    got = gpu_run(qla, n, q, 0.3, 40)
    for c in zero:
        assert np.all(got[c] == 0.0), c


def test_zero_steps_returns_input(qla):
    n = scenes.smooth_random_profile(33, 17, 3)
    q = scenes.random_state(33, 17, 4).astype(np.float32)
    got = gpu_run(qla, n, q, 0.3, 0)
    assert np.array_equal(got, q)


# --------------------------------------------------------------------------
# Diagnostics and field export.
# --------------------------------------------------------------------------

def test_diagnostics_match_plain_definitions(qla):
    nx, ny = 150, 77
    n = scenes.smooth_random_profile(nx, ny, 12, 1.0, 3.0)
    q = scenes.random_state(nx, ny, 13)
    sim = qla.Simulation(n, q, 0.3)
    sim.step(5)
    d = sim.diagnostics()
    qs = sim.fields("Q")
    sim.close()
    ref = O.diagnostics(qs, n.astype(np.float32))
    assert d["step"] == 5
    for k in ("energy", "divB_max", "divB_l2", "B_max", "B_l2", "divD_max", "divD_l2", "D_max"):
        assert abs(d[k] - ref[k]) <= 1e-11 * abs(ref[k]), (k, d[k], ref[k])


def test_fields_export_e_and_b(qla):
    nx, ny = 64, 31
    n = scenes.smooth_random_profile(nx, ny, 14, 1.0, 3.0).astype(np.float32)
    q = scenes.random_state(nx, ny, 15).astype(np.float32)
    sim = qla.Simulation(n, q, 0.3)
    sim.step(2)
    qs = sim.fields("Q")
    eb = sim.fields("EB")
    again = sim.fields("Q")
    sim.close()
    assert np.array_equal(eb[:3], qs[:3] / n)     # IEEE FP32 division on both sides
    assert np.array_equal(eb[3:], qs[3:])
    assert np.array_equal(again, qs)              # exporting leaves the state alone


def test_init_rejects_nonpositive_index(qla):
    import torch
    n = np.ones((3, 8, 8), dtype=np.float32)
    n[1, 3, 4] = 0.0
    with pytest.raises(qla.QlaError) as ei:
        qla.Simulation(n, np.zeros((6, 8, 8), np.float32), 0.3)
    assert ei.value.status == qla.QLA_EINVAL
    n[1, 3, 4] = np.nan
    with pytest.raises(qla.QlaError):
        qla.Simulation(n, np.zeros((6, 8, 8), np.float32), 0.3)


# --------------------------------------------------------------------------
# Full-size lattice in the benchmark's launch configuration: sampled windows.
# --------------------------------------------------------------------------

def _window_oracle(n, q, delta, steps, y, x, h, w):
    """Exact oracle values of the h x w window at (y, x) after ``steps`` steps:
    one step's support is +-4 cells, so a patch with a margin of 4*steps + 2
    around the window, run periodically on its own, is exact in the window."""
    m = 4 * steps + 2
    ny, nx = n.shape[1:]
    ys = np.arange(y - m, y + h + m) % ny
    xs = np.arange(x - m, x + w + m) % nx
    npatch = n[:, ys][:, :, xs]
    qpatch = q[:, ys][:, :, xs]
    out = oracle_run(npatch, qpatch, delta, steps)
    return out[:, m:m + h, m:m + w]


def test_full_size_cylinder_sampled(qla):
    # the cylinder profile of the 4096 x 4096 run with a random state, so that
    # every sampled window carries signal
    sc = scenes.config_scale(seed=2, N=4096, steps=12)
    n32 = np.ascontiguousarray(sc.n, dtype=np.float32)
    rng = np.random.default_rng(77)
    q32 = rng.standard_normal((6, 4096, 4096), dtype=np.float32)
    _case("cylinder 4096x4096, random state, 12 steps, sampled windows")
    got = gpu_run(qla, n32, q32, sc.delta, sc.steps)
    N = 4096
    c = N // 2
    windows = [(0, 0), (N - 16, N - 16), (0, N - 8), (c - 8, c - 400 - 8), (c + 300, c + 250),
               (c - 8, N // 4 - 8), (1000, 3000), (2047, 4090)]
    for (y, x) in windows:
        want = _window_oracle(n32, q32, sc.delta, sc.steps, y, x, 16, 16)
        ys = np.arange(y, y + 16) % N
        xs = np.arange(x, x + 16) % N
        g = got[:, ys][:, :, xs]
        assert np.abs(g - want).max() / np.abs(want).max() <= TOL, (y, x)
