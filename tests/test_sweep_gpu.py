"""The surrogate-accelerated sweep: QLA checks, fallback, and what a briefly
trained network gains (or not) over plain QLA, on the GPU through the C
ABIs of both libraries."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_13601_amd import qla, scenes, surrogate
    qla.lib()
    return torch, scenes, surrogate


def _lattices(scenes, count, L, seed):
    specs = scenes.batch_instance_specs(count, seed=seed, sides=(L,))
    scs = [scenes.scene_from_spec(sp, steps=0) for sp in specs]
    return [s.n.astype(np.float32) for s in scs], [s.q.astype(np.float32) for s in scs], scs[0].delta


def _case(tag):
    print(f"[sweep] {tag}", flush=True)


def test_sweep_falls_back_at_first_check_and_matches_plain_qla(env):
    torch, scenes, S = env
    ns, qs, delta = _lattices(scenes, 3, 256, 41)
    net = S.UNet(seed=3)                      # untrained: fails any check
    _case("untrained network, tol 1e-3")
    res, finals = S.sweep(net, ns, qs, delta, total_steps=1024, K=256, check_every=4, tol=1e-3)
    assert res.checks == 1 and res.rejected == 1 and res.fell_back and res.unchecked == 0
    secs, plain = S.plain(ns, qs, delta, 1024, stream=net.stream)
    for a, b in zip(finals, plain):
        assert np.array_equal(a, b)


def test_sweep_without_checks_uses_every_jump(env):
    torch, scenes, S = env
    ns, qs, delta = _lattices(scenes, 2, 256, 42)
    net = S.UNet(seed=4)
    _case("no checks")
    res, finals = S.sweep(net, ns, qs, delta, total_steps=1000, K=256, check_every=0)
    # 3 jumps of 256, then the remaining 232 steps by QLA
    assert res.jumps == 3 and res.unchecked == 3 and res.checks == 0 and not res.fell_back
    secs, plain = S.plain(ns, qs, delta, 1000, stream=net.stream)
    assert not np.array_equal(finals[0], plain[0])


def test_trained_network_error_and_sweep_gain(env):
    torch, scenes, S = env
    _case("train 600 steps on 256 runs, evaluate on 32 held-out runs and a 4-lattice sweep")
    data = S.generate(256, seed=11, L=256, K=256, snaps=5)
    held = S.generate(32, seed=999, L=256, K=256, snaps=5)
    net = S.UNet(seed=0)
    S.train(net, data, steps=600, batch=16, lr=1e-3, seed=1, log_every=0)
    err = S.evaluate(net, held)
    # the identity map (Q(t + K) = Q(t)) misses by more than the field itself
    ident = []
    for r in range(held.runs):
        for s in range(held.snaps - 1):
            a = held.q[r * held.snaps + s].double()
            b = held.q[r * held.snaps + s + 1].double()
            ident.append(float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)))
    print(f"  held-out relative error: network median {np.median(err):.3f}, identity median {np.median(ident):.3f}")
    assert np.median(err) < 0.5 * np.median(ident)
    ns, qs, delta = _lattices(scenes, 4, 256, 43)
    res, finals = S.sweep(net, ns, qs, delta, total_steps=2048, K=256, check_every=4, tol=1e-3)
    secs, plain = S.plain(ns, qs, delta, 2048, stream=net.stream)
    print(f"  sweep at tol 1e-3: {res.jumps} jumps, {res.rejected} rejected, fell back {res.fell_back}, "
          f"first check error {res.max_check_error:.3e}; {secs / res.seconds:.2f}x plain QLA")
    # a network this far from the 1e-3 bar must be caught at its first check
    if res.max_check_error > 1e-3:
        assert res.fell_back and res.unchecked == 0
        for a, b in zip(finals, plain):
            assert np.array_equal(a, b)
