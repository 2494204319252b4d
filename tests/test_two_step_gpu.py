"""The two-step launch (temporal blocking: each wave runs the step twice in
one march) against the one-step launch, bit for bit, and against the
oracle, through the C ABI."""
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


def _case(tag):
    print(f"[two-step] {tag}", flush=True)


def run(qla, n, q, delta, steps, spp, mode="eq28", beta="phys", pol="both", form="printed", chunks=None,
        graph_steps=0, seg_rows=0):
    sim = qla.Simulation(np.ascontiguousarray(n, dtype=np.float32), np.ascontiguousarray(q, dtype=np.float32),
                         delta, mode, beta, polarisation=pol, v_form=form)
    sim.set_launch(seg_rows=seg_rows, graph_steps=graph_steps, steps_per_pass=spp)
    assert sim.launch()["steps_per_pass"] == spp
    for k in (chunks or [steps]):
        sim.step(k)
    out = sim.fields("Q")
    sim.close()
    return out


def oracle_run(n, q, delta, steps, mode="eq28", beta="phys", form="printed"):
    n64 = np.asarray(n, dtype=np.float32).astype(np.float64)
    q64 = np.asarray(q, dtype=np.float32).astype(np.float64)
    return O.run(n64, q64, delta, steps, mode, beta, v_form=form)


def rel_err(got, want):
    return float(np.abs(got.astype(np.float64) - want).max() / np.abs(want).max())


SHAPES = [(1, 1), (3, 5), (7, 1), (1, 9), (17, 13), (112, 9), (113, 40), (121, 33), (250, 19), (300, 70)]


@pytest.mark.parametrize("nx,ny", SHAPES)
@pytest.mark.parametrize("mode", ["eq23", "eq28"])
def test_two_step_equals_one_step_smooth(qla, nx, ny, mode):
    seed = 13 * nx + ny
    n = scenes.smooth_random_profile(nx, ny, seed, 1.0, 3.0)
    q = scenes.random_state(nx, ny, seed + 1)
    _case(f"smooth {nx}x{ny} {mode}")
    one = run(qla, n, q, 0.3, 9, 1, mode)
    two = run(qla, n, q, 0.3, 9, 2, mode)
    assert np.array_equal(one, two)
    assert rel_err(two, oracle_run(n, q, 0.3, 9, mode)) <= TOL


@pytest.mark.parametrize("nx,ny", [(5, 3), (40, 24), (130, 66)])
@pytest.mark.parametrize("mode", ["eq23", "eq28"])
@pytest.mark.parametrize("beta", ["phys", "lattice", "off"])
@pytest.mark.parametrize("form", ["printed", "skew"])
def test_two_step_equals_one_step_rough(qla, nx, ny, mode, beta, form):
    seed = 5 * nx + ny
    n = scenes.random_profile(nx, ny, seed, 1.0, 3.0)          # wide angles
    q = scenes.random_state(nx, ny, seed + 2)
    _case(f"rough {nx}x{ny} {mode} {beta} {form}")
    one = run(qla, n, q, 0.3, 8, 1, mode, beta, form=form)
    two = run(qla, n, q, 0.3, 8, 2, mode, beta, form=form)
    assert np.array_equal(one, two)
    assert rel_err(two, oracle_run(n, q, 0.3, 8, mode, beta, form)) <= TOL


@pytest.mark.parametrize("pol,dead", [("tm", (0, 1, 5)), ("te", (2, 3, 4))])
@pytest.mark.parametrize("mode", ["eq23", "eq28"])
def test_two_step_polarised(qla, pol, dead, mode):
    n = scenes.object_profile(256, 96, "ellipse", (30, 20), (1.5, 2.0, 3.0), 3.0)
    q = scenes.random_state(256, 96, 4).astype(np.float32)
    for c in dead:
        q[c] = 0.0
    _case(f"polarised {pol} {mode}")
    one = run(qla, n, q, 0.3, 11, 1, mode)
    two = run(qla, n, q, 0.3, 11, 2, mode, pol=pol)
    assert np.array_equal(one, two)


@pytest.mark.parametrize("seg_rows", [4, 8, 36, 200])
def test_two_step_segment_heights(qla, seg_rows):
    n = scenes.smooth_random_profile(200, 150, 21, 1.0, 3.0)
    q = scenes.random_state(200, 150, 22)
    _case(f"segments of {seg_rows} rows")
    one = run(qla, n, q, 0.3, 6, 1)
    two = run(qla, n, q, 0.3, 6, 2, seg_rows=seg_rows)
    assert np.array_equal(one, two)


def test_two_step_graph_replays_and_splits(qla):
    n = scenes.smooth_random_profile(130, 50, 9, 1.0, 3.0)
    q = scenes.random_state(130, 50, 10)
    _case("graph replays, odd splits")
    eager = run(qla, n, q, 0.3, 45, 1, graph_steps=1)
    g = run(qla, n, q, 0.3, 45, 2, graph_steps=8, chunks=[16, 3, 13, 8, 5])
    assert np.array_equal(eager, g)


def test_two_step_batch(qla):
    specs = [(200, 120), (130, 66), (64, 250), (7, 5), (512, 40)]
    ns, qs, ds = [], [], []
    for i, (nx, ny) in enumerate(specs):
        ns.append(scenes.smooth_random_profile(nx, ny, 60 + i, 1.0, 3.0).astype(np.float32))
        qs.append(scenes.random_state(nx, ny, 70 + i).astype(np.float32))
        ds.append(0.3 if i % 2 == 0 else 0.2)
    _case("batch")
    b = qla.Batch(ns, qs, ds)
    b.set_launch(steps_per_pass=2, graph_steps=4)
    b.step(10)
    b.step(3)
    outs = b.fields("Q")
    b.close()
    for i in range(len(specs)):
        assert np.array_equal(outs[i], run(qla, ns[i], qs[i], ds[i], 13, 1)), i


def test_two_step_full_size_bitwise(qla):
    sc = scenes.config_scale(seed=2, N=4096, steps=10)
    rng = np.random.default_rng(5)
    q = rng.standard_normal((6, 4096, 4096), dtype=np.float32)
    _case("4096x4096 cylinder, random state, 10 steps, one-step vs two-step launches")
    one = run(qla, sc.n, q, sc.delta, 10, 1)
    two = run(qla, sc.n, q, sc.delta, 10, 2)
    assert np.array_equal(one, two)


def test_steps_per_pass_is_validated(qla):
    n = scenes.uniform_profile(16, 8, (1.5, 2.0, 3.0))
    q = np.zeros((6, 8, 16), np.float32)
    sim = qla.Simulation(n, q, 0.3)
    assert sim.launch()["steps_per_pass"] in (1, 2)
    with pytest.raises(qla.QlaError):
        sim.set_launch(steps_per_pass=3)
    sim.close()


@pytest.mark.parametrize("spp", [1, 2])
@pytest.mark.parametrize("mode", ["eq23", "eq28"])
def test_state_load_cache_policy_is_bitwise(qla, spp, mode):
    """Non-temporal and default state loads give the same bits; single
    lattices and batches default to the default policy, and a TM context
    always uses it."""
    n = scenes.smooth_random_profile(300, 210, 41, 1.0, 3.0).astype(np.float32)
    q = scenes.random_state(300, 210, 42).astype(np.float32)
    _case(f"state-load cache policy, {spp} step(s) per launch, {mode}")
    outs = []
    for pol in (1, 2):
        sim = qla.Simulation(n, q, 0.3, mode)
        assert sim.launch()["stream_loads"] == 2
        sim.set_launch(steps_per_pass=spp, stream_loads=pol)
        assert sim.launch()["stream_loads"] == pol
        sim.step(11)
        outs.append(sim.fields("Q"))
        sim.close()
    assert np.array_equal(outs[0], outs[1])
    b = qla.Batch([n, n], [q, q], [0.3, 0.3], mode)
    assert b.launch()["stream_loads"] == 2
    b.set_launch(steps_per_pass=spp, stream_loads=1)
    b.step(11)
    for f in b.fields("Q"):
        assert np.array_equal(f, outs[0])
    b.close()
    tm = qla.Simulation(n, q, 0.3, mode, polarisation="tm")
    tm.set_launch(stream_loads=1)
    assert tm.launch()["stream_loads"] == 2
    tm.close()
