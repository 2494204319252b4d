"""The surrogate network at the size the inference benchmark runs it
(lattices of 1024 x 1024, 16 lattices per pass): against the FP64 oracle
network on one lattice, and, for the whole 16-lattice batch, the
translation property that holds at any size. Also the convolution kernels
next to the 31-bit element-offset limit, each against a kernel with its
own indexing."""
import numpy as np
import pytest

from oracle import nn_oracle as N

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_13601_amd import scenes, surrogate as S
    return torch, scenes, S


def _lattices(torch, scenes, count, L, seed):
    specs = scenes.batch_instance_specs(count, seed=seed, sides=(L,))
    scs = [scenes.scene_from_spec(sp, steps=0) for sp in specs]
    q = torch.as_tensor(np.stack([s.q.astype(np.float32) for s in scs])).cuda()
    n = torch.as_tensor(np.stack([s.n.astype(np.float32) for s in scs])).cuda()
    return q, n


def _case(tag):
    print(f"[nn full size] {tag}", flush=True)


def test_network_1024_matches_oracle(env):
    """One 1024 x 1024 lattice through the inference path (packing, fused
    decoder, FP32 output) against the FP64 oracle network fed the same
    packed BF16 input, with the weights rounded to BF16 as the GPU uses
    them; the same relative L2 bar as the 32 x 32 whole-network test."""
    torch, scenes, S = env
    _case("1 lattice of 1024x1024 vs the FP64 oracle network")
    q, n = _lattices(torch, scenes, 1, 1024, 61)
    net = S.UNet(seed=7)
    L = 1024
    net.pack(1, L, L, q, None, n, None)
    out = net.forward_packed(1, L, L, fused=True)
    got = out.cpu().numpy().reshape(1, L, L, S.OUT_LD)[..., :6].astype(np.float64)
    xr = net.act["x"].float().cpu().numpy().astype(np.float64).reshape(1, L, L, 48)
    p = net.p.cpu().numpy().astype(np.float64)
    pr = p.copy()
    off = 0
    for name, ci, co, _, _ in N.unet_layers():
        pr[off:off + co * 9 * ci] = N.bf16_round(p[off:off + co * 9 * ci].astype(np.float32))
        off += co * 9 * ci + co
    ref, _ = N.unet_forward(pr, xr, bf16=True)
    ref = ref[..., :6]
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"  relative L2 difference {err:.2e}")
    assert err <= 2e-2


def test_network_translation_equivariance_16x1024(env):
    """The map is periodic-translation equivariant for shifts that are
    multiples of 16 cells (the four 2 x 2 poolings then stay aligned), and
    every output is computed with the same arithmetic wherever its tile
    lies: rolling the 16 input lattices rolls the predictions bitwise."""
    torch, scenes, S = env
    _case("16 lattices of 1024x1024, predictions of rolled inputs")
    q, n = _lattices(torch, scenes, 16, 1024, 62)
    net = S.UNet(seed=8)
    a = torch.empty_like(q)
    net.predict(q, n, a)
    qs = torch.roll(q, shifts=(48, 96), dims=(2, 3)).contiguous()
    ns = torch.roll(n, shifts=(48, 96), dims=(2, 3)).contiguous()
    b = torch.empty_like(q)
    net.predict(qs, ns, b)
    torch.cuda.synchronize()
    assert torch.equal(torch.roll(a, shifts=(48, 96), dims=(2, 3)), b)


def test_predict_2048_in_chunks(env):
    """Lattices of 2048 x 2048, the sweep's size: 8 of them take two chunks
    (7 + 1, the offset limit of the upsampled 64-channel level-1 output).
    Chunked prediction equals one-lattice-at-a-time prediction bitwise (each
    lattice is scaled and computed on its own), and rolling the inputs by
    multiples of 16 cells rolls the predictions bitwise."""
    torch, scenes, S = env
    L, B = 2048, 8
    assert S.default_chunk(L, L) == 7
    _case(f"{B} lattices of {L}x{L}, chunked vs single predictions")
    q, n = _lattices(torch, scenes, B, L, 63)
    net = S.UNet(seed=9)
    a = torch.empty_like(q)
    net.predict(q, n, a)
    one = torch.empty_like(q)
    net.predict(q, n, one, chunk=1)
    torch.cuda.synchronize()
    assert torch.equal(a, one)
    assert torch.isfinite(a).all() and float(a.abs().max()) > 0
    del one
    qs = torch.roll(q[5:], shifts=(32, 2000), dims=(2, 3)).contiguous()
    ns = torch.roll(n[5:], shifts=(32, 2000), dims=(2, 3)).contiguous()
    b = torch.empty_like(qs)
    net.predict(qs, ns, b)
    torch.cuda.synchronize()
    assert torch.equal(torch.roll(a[5:], shifts=(32, 2000), dims=(2, 3)), b)


def _bf16_randn(torch, shape, scale, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    return (torch.randn(shape, generator=g, device="cuda") * scale).to(torch.bfloat16)


def test_resident_weight_kernels_at_the_offset_limit(env):
    """32 lattices of 1024 x 1024 x 32 channels (2^30 elements, the largest
    power of two under the limit): the resident-weight convolution, its
    pooled form and its scaled-planes form, bitwise against the pipelined
    kernel (the fused entry point with neither upsampling nor skip), the
    separate pooling and the separate unpacking."""
    torch, _, _ = env
    from paper_2301_13601_amd import qnn
    B, H, W, C = 32, 1024, 1024, 32
    _case(f"resident-weight conv and pool, {B}x{H}x{W}x{C}")
    x = _bf16_randn(torch, (B, H, W, C), 0.5, 70)
    w = _bf16_randn(torch, (C, 9, C), 1 / np.sqrt(9 * C), 71)
    bias = torch.randn(C, device="cuda")
    y_pipe = torch.empty((B, H, W, C), dtype=torch.bfloat16, device="cuda")
    qnn.qnn_conv3x3_fwd_fused(B, H, W, x, C, 0, w, bias, C, 1, None, y_pipe, C)
    y = torch.empty_like(y_pipe)
    pool = torch.empty((B, H // 2, W // 2, C), dtype=torch.bfloat16, device="cuda")
    qnn.qnn_conv3x3_fwd_pool(B, H, W, x, C, w, bias, C, 1, y, pool)
    assert torch.equal(y.view(torch.int16), y_pipe.view(torch.int16))
    del y
    want = torch.empty_like(pool)
    qnn.qnn_avgpool2(B, H, W, C, y_pipe, want)
    assert torch.equal(pool.view(torch.int16), want.view(torch.int16))
    del pool, want, y_pipe
    # the output layer's planes against the FP32 result and the separate
    # unpacking (whose indexing is its own)
    scale = torch.rand(B, device="cuda") + 0.5
    yf = torch.empty((B, H, W, 8), dtype=torch.float32, device="cuda")
    qnn.qnn_conv3x3_fwd(B, H, W, x, C, w, bias, C, 0, yf, 1, 8, 6)
    want_q = torch.empty((B, 6, H, W), dtype=torch.float32, device="cuda")
    qnn.qnn_unpack_output(B, H, W, yf, 8, scale, want_q)
    del yf
    got_q = torch.empty_like(want_q)
    qnn.qnn_conv3x3_fwd_planes(B, H, W, x, C, w, bias, C, 0, scale, 6, got_q)
    assert torch.equal(got_q.view(torch.int32), want_q.view(torch.int32))


def test_window_kernel_at_the_offset_limit(env):
    """16 lattices of 1024 x 1024, 64 -> 32 channels from a half-resolution
    input plus a skip input (the upsampled input has 2^30 elements, the
    limit's largest power of two): the window kernel bitwise against the
    separate upsampling, pipelined convolution and addition."""
    torch, _, _ = env
    from paper_2301_13601_amd import qnn
    B, H, W, ci, co = 16, 1024, 1024, 64, 32
    _case(f"window conv, {B}x{H}x{W}, {ci}->{co} upsampled + skip")
    x = _bf16_randn(torch, (B, H // 2, W // 2, ci), 0.5, 72)
    w = _bf16_randn(torch, (co, 9, ci), 1 / np.sqrt(9 * ci), 73)
    e = _bf16_randn(torch, (B, H, W, co), 1.0, 74)
    bias = torch.randn(co, device="cuda")
    got = torch.empty((B, H, W, co), dtype=torch.bfloat16, device="cuda")
    qnn.qnn_conv3x3_fwd_fused(B, H, W, x, ci, 1, w, bias, co, 1, e, got, co)
    u = torch.empty((B, H, W, ci), dtype=torch.bfloat16, device="cuda")
    qnn.qnn_upsample2(B, H // 2, W // 2, ci, x, u)
    d = torch.empty_like(got)
    qnn.qnn_conv3x3_fwd(B, H, W, u, ci, w, bias, co, 1, d, 0, co, co)
    del u
    want = torch.empty_like(got)
    qnn.qnn_add(d.numel(), d, e, want)
    assert torch.equal(got.view(torch.int16), want.view(torch.int16))
