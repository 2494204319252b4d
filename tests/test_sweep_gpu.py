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
    # the BF16 floor: the GPU network against the same weights run exactly
    # (FP64 oracle network, no rounding) on two held-out inputs
    from oracle import nn_oracle as N
    pairs = held.pairs()[:2]
    idx = torch.as_tensor(pairs.T.copy()).cuda()
    L = held.L
    net.pack(2, L, L, held.q, idx[0], held.n, idx[1])
    y = net.forward_packed(2, L, L, fused=True).cpu().numpy().reshape(2, L, L, S.OUT_LD)[..., :6].astype(np.float64)
    x = net.act["x"].float().cpu().numpy().astype(np.float64).reshape(2, L, L, S.IN_CH)
    exact, _ = N.unet_forward(net.p.cpu().numpy().astype(np.float64), x, bf16=False)
    exact = exact[..., :6]
    floor = float(np.linalg.norm(y - exact) / np.linalg.norm(exact))
    print(f"  BF16 network vs the same network in exact arithmetic: relative L2 {floor:.3e}")
    assert floor < np.median(err)
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


def _by_hand(torch, qla, net, ns, qs, delta, plan):
    """The sweep's composition built directly: plan is a list of ("qla", k)
    and ("jump",) items applied in order to a QLA batch."""
    B, (_, H, W) = len(ns), ns[0].shape
    b = qla.Batch(ns, qs, [delta] * B, "eq28", "phys", stream=net.stream)
    cur = torch.empty((B, 6, H, W), dtype=torch.float32, device="cuda")
    pred = torch.empty_like(cur)
    n_dev = torch.stack([t.view(3, H, W) for t in b.n])
    for item in plan:
        if item[0] == "qla":
            b.step(item[1])
            continue
        for k in range(B):
            qla.qla_fields_at(b.ctx, k, cur[k].data_ptr(), 0, False)
        net.predict(cur, n_dev, pred)
        for k in range(B):
            qla.qla_load_at(b.ctx, k, pred[k].data_ptr(), False)
    out = b.fields("Q")
    b.close()
    return out


def test_sweep_correction_windows_step_accounting(env):
    """Jumps of 256 steps with 100-step QLA windows over 1000 steps and no
    checks: jump, window, jump, window, jump, then a 32-step window; bit for
    bit the same composition built by hand."""
    torch, scenes, S = env
    from paper_2301_13601_amd import qla
    ns, qs, delta = _lattices(scenes, 2, 256, 44)
    net = S.UNet(seed=6)
    _case("windows of 100 steps, no checks")
    res, finals = S.sweep(net, ns, qs, delta, total_steps=1000, K=256, window=100, check_every=0)
    assert (res.jumps, res.unchecked, res.checks, res.windows, res.window_steps) == (3, 3, 0, 3, 232)
    want = _by_hand(torch, qla, net, ns, qs, delta,
                    [("jump",), ("qla", 100), ("jump",), ("qla", 100), ("jump",), ("qla", 32)])
    for a, b in zip(finals, want):
        assert np.array_equal(a, b)


def test_sweep_correction_windows_with_passing_checks(env):
    """Checks at jumps 1 and 2 (the QLA result is kept), window 50: QLA for
    256 + 50 + 256 + 50 steps, one surrogate jump, a window of 50 and 82
    plain steps to reach 1000; bit for bit the composition built by hand."""
    torch, scenes, S = env
    from paper_2301_13601_amd import qla
    ns, qs, delta = _lattices(scenes, 2, 256, 46)
    net = S.UNet(seed=8)
    _case("windows of 50 steps, checks every 2nd jump, tolerance that passes")
    res, finals = S.sweep(net, ns, qs, delta, total_steps=1000, K=256, window=50, check_every=2, tol=1e30)
    assert (res.jumps, res.checks, res.unchecked, res.rejected, res.windows, res.window_steps) == (3, 2, 1, 0, 3, 150)
    assert not res.fell_back
    want = _by_hand(torch, qla, net, ns, qs, delta, [("qla", 612), ("jump",), ("qla", 132)])
    for a, b in zip(finals, want):
        assert np.array_equal(a, b)


def test_sweep_correction_windows_fall_back_to_plain_qla(env):
    """An untrained network fails its first check; with windows configured
    the rest is plain QLA and the result is plain QLA bit for bit."""
    torch, scenes, S = env
    ns, qs, delta = _lattices(scenes, 2, 256, 45)
    net = S.UNet(seed=7)
    _case("windows of 64 steps, untrained network, tol 1e-3")
    res, finals = S.sweep(net, ns, qs, delta, total_steps=1100, K=256, window=64, check_every=1, tol=1e-3)
    assert res.fell_back and res.checks == 1 and res.rejected == 1 and res.unchecked == 0 and res.windows == 0
    secs, plain = S.plain(ns, qs, delta, 1100, stream=net.stream)
    for a, b in zip(finals, plain):
        assert np.array_equal(a, b)
