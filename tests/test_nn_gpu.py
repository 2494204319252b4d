"""Surrogate kernels (C ABI of include/qla_nn.h) against the FP64 reference
in oracle/nn_oracle.py.

Inputs are BF16-representable, so the reference sees exactly the values the
kernels read; what remains is FP32 accumulation (tolerances below) and, for
BF16 outputs, one rounding.
"""
import numpy as np
import pytest

from oracle import nn_oracle as N

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_13601_amd import qnn
    return torch, qnn


def bf(torch, a):
    """Device BF16 tensor of a (rounded), and the FP64 values it holds."""
    t = torch.tensor(np.asarray(a, np.float32)).to(torch.bfloat16).cuda()
    return t, t.float().cpu().numpy().astype(np.float64)


def rnd(seed, shape, scale=1.0):
    return np.random.default_rng(seed).standard_normal(shape) * scale


@pytest.mark.parametrize("B,H,W,ci,co", [(2, 16, 32, 16, 32), (1, 8, 24, 32, 64), (2, 6, 10, 64, 128),
                                         (1, 2, 2, 128, 128), (3, 5, 7, 16, 96),
                                         # pipelined kernel (W in {16, 32} or a multiple of 64):
                                         # tiles taller than the image and partial last tiles,
                                         # several tiles per block, 1 to 8 channel chunks, and
                                         # the four tile shapes (128 or 256 pixels x 32 or 64
                                         # channels)
                                         (64, 15, 64, 48, 32), (600, 7, 16, 32, 128), (2, 256, 128, 128, 128),
                                         (512, 3, 32, 64, 64), (600, 1, 16, 16, 32), (2, 168, 192, 32, 96),
                                         (16, 32, 32, 128, 128), (3, 20, 64, 16, 64),
                                         # resident-weight kernel (32 or 48 -> 32 channels, W a
                                         # multiple of 16): 32- and 16-wide tiles, partial and
                                         # over-tall tiles, more tiles than resident blocks
                                         (64, 64, 64, 32, 32), (48, 64, 64, 48, 32), (3, 20, 48, 32, 32),
                                         (2, 5, 96, 48, 32),
                                         # and for 64 output channels (256 tiles or more): two
                                         # 32-channel blocks a tile, or one 64-channel block
                                         (24, 48, 64, 32, 64), (16, 64, 80, 64, 64)])
@pytest.mark.parametrize("act", [0, 1])
def test_conv_forward(env, B, H, W, ci, co, act):
    torch, qnn = env
    x, xr = bf(torch, rnd(1, (B, H, W, ci)))
    w, wr = bf(torch, rnd(2, (co, 9, ci), 1 / np.sqrt(9 * ci)))
    bias = torch.tensor(rnd(3, co).astype(np.float32)).cuda()
    ref = N.conv3x3(xr, wr, bias.cpu().numpy().astype(np.float64))
    if act:
        ref = N.leaky(ref)
    y = torch.empty((B, H, W, co), dtype=torch.float32, device="cuda")
    qnn.qnn_conv3x3_fwd(B, H, W, x, ci, w, bias, co, act, y, 1, co, co)
    got = y.cpu().numpy()
    assert np.abs(got - ref).max() <= 2e-6 * np.abs(ref).max() + 1e-6
    yb = torch.empty((B, H, W, co), dtype=torch.bfloat16, device="cuda")
    qnn.qnn_conv3x3_fwd(B, H, W, x, ci, w, bias, co, act, yb, 0, co, co)
    gotb = yb.float().cpu().numpy()
    assert np.all(np.abs(gotb - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-6)


@pytest.mark.parametrize("W", [16, 24])
def test_conv_forward_partial_store(env, W):
    torch, qnn = env
    B, H, ci, co = 1, 8, 32, 32
    x, xr = bf(torch, rnd(4, (B, H, W, ci)))
    w, wr = bf(torch, rnd(5, (co, 9, ci), 0.1))
    ref = N.conv3x3(xr, wr)
    y = torch.full((B, H, W, co), 7.0, dtype=torch.float32, device="cuda")
    qnn.qnn_conv3x3_fwd(B, H, W, x, ci, w, None, co, 0, y, 1, co, 6)
    got = y.cpu().numpy()
    assert np.abs(got[..., :6] - ref[..., :6]).max() <= 2e-6 * np.abs(ref).max()
    assert np.all(got[..., 6:] == 7.0)
    # BF16 results for part of the channels, in rows of 8 (y_ld = 8)
    yb = torch.full((B, H, W, 8), 7.0, dtype=torch.bfloat16, device="cuda")
    qnn.qnn_conv3x3_fwd(B, H, W, x, ci, w, None, co, 0, yb, 0, 8, 6)
    gotb = yb.float().cpu().numpy()
    assert np.all(np.abs(gotb[..., :6] - ref[..., :6]) <= 2.0 ** -8 * np.abs(ref[..., :6]) + 1e-6)
    assert np.all(gotb[..., 6:] == 7.0)


@pytest.mark.parametrize("B,H,W,ci,co", [(2, 32, 64, 64, 32), (3, 16, 16, 128, 128), (2, 20, 32, 32, 64),
                                         (16, 64, 128, 128, 64),
                                         # the separate convolution on the resident-weight kernel,
                                         # the fused one on the pipelined kernel
                                         (4, 24, 64, 32, 32), (2, 40, 32, 48, 32), (40, 32, 64, 32, 32),
                                         # 64 -> 32 channels upsampled: the half-resolution window
                                         # kernel (window taller than the input, more tiles than
                                         # resident blocks)
                                         (3, 6, 32, 64, 32), (5, 2, 16, 64, 32), (24, 64, 128, 64, 32),
                                         # 64 output channels: resident-weight kernel vs pipelined
                                         (24, 48, 64, 32, 64), (16, 64, 64, 64, 64),
                                         # 128 -> 64 upsampled on 2^20 pixels: the window kernel
                                         (16, 256, 256, 128, 64)])
@pytest.mark.parametrize("up", [0, 1])
@pytest.mark.parametrize("with_add", [False, True])
def test_conv_fused_is_bitwise_the_separate_steps(env, B, H, W, ci, co, up, with_add):
    torch, qnn = env
    h, w_ = (H // 2, W // 2) if up else (H, W)
    x, _ = bf(torch, rnd(30, (B, h, w_, ci)))
    w, _ = bf(torch, rnd(31, (co, 9, ci), 1 / np.sqrt(9 * ci)))
    bias = torch.tensor(rnd(32, co).astype(np.float32)).cuda()
    e, _ = bf(torch, rnd(33, (B, H, W, co))) if with_add else (None, None)
    # the separate steps
    xin = x
    if up:
        xin = torch.empty((B, H, W, ci), dtype=torch.bfloat16, device="cuda")
        qnn.qnn_upsample2(B, h, w_, ci, x, xin)
    d = torch.empty((B, H, W, co), dtype=torch.bfloat16, device="cuda")
    qnn.qnn_conv3x3_fwd(B, H, W, xin, ci, w, bias, co, 1, d, 0, co, co)
    want = d
    if with_add:
        want = torch.empty_like(d)
        qnn.qnn_add(d.numel(), d, e, want)
    got = torch.full((B, H, W, co), 3.0, dtype=torch.bfloat16, device="cuda")
    qnn.qnn_conv3x3_fwd_fused(B, H, W, x, ci, up, w, bias, co, 1, e, got, co)
    assert torch.equal(got.view(torch.int16), want.view(torch.int16))


@pytest.mark.parametrize("B,H,W,ci,co", [(2, 16, 32, 32, 32), (3, 20, 48, 48, 32), (2, 6, 64, 32, 32),
                                         (40, 32, 64, 32, 32), (16, 64, 64, 64, 64), (24, 48, 64, 32, 64),
                                         (2, 16, 16, 128, 128), (3, 10, 24, 32, 32)])
@pytest.mark.parametrize("act", [0, 1])
def test_conv_pool_is_bitwise_conv_then_pool(env, B, H, W, ci, co, act):
    """Convolution with the 2x2 pooling of its result: bitwise
    qnn_conv3x3_fwd then qnn_avgpool2, pooled in the resident-weight epilogue
    (32- and 16-wide tiles, partial and over-tall tiles, 64 channels as one
    or two blocks) or by the two calls (128 channels, W not a multiple of
    16)."""
    torch, qnn = env
    x, _ = bf(torch, rnd(60, (B, H, W, ci)))
    w, _ = bf(torch, rnd(61, (co, 9, ci), 1 / np.sqrt(9 * ci)))
    bias = torch.tensor(rnd(62, co).astype(np.float32)).cuda()
    y0 = torch.empty((B, H, W, co), dtype=torch.bfloat16, device="cuda")
    qnn.qnn_conv3x3_fwd(B, H, W, x, ci, w, bias, co, act, y0, 0, co, co)
    p0 = torch.empty((B, H // 2, W // 2, co), dtype=torch.bfloat16, device="cuda")
    qnn.qnn_avgpool2(B, H, W, co, y0, p0)
    y1 = torch.full_like(y0, 3.0)
    p1 = torch.full_like(p0, 3.0)
    qnn.qnn_conv3x3_fwd_pool(B, H, W, x, ci, w, bias, co, act, y1, p1)
    assert torch.equal(y1.view(torch.int16), y0.view(torch.int16))
    assert torch.equal(p1.view(torch.int16), p0.view(torch.int16))


@pytest.mark.parametrize("B,H,W,ci", [(2, 16, 32, 32), (3, 20, 48, 48), (2, 5, 64, 32), (40, 32, 64, 32)])
@pytest.mark.parametrize("act", [0, 1])
def test_conv_planes_is_bitwise_conv_then_unpack(env, B, H, W, ci, act):
    """The output layer writing scaled planes: bitwise the FP32 convolution
    followed by qnn_unpack_output (6 planes), and the plain product for all
    32 (16- and 32-wide tiles, a tile taller than the image, many tiles)."""
    torch, qnn = env
    x, _ = bf(torch, rnd(50, (B, H, W, ci)))
    w, _ = bf(torch, rnd(51, (32, 9, ci), 1 / np.sqrt(9 * ci)))
    bias = torch.tensor(rnd(52, 32).astype(np.float32)).cuda()
    scale = torch.tensor((0.5 + np.abs(rnd(53, B))).astype(np.float32)).cuda()
    y = torch.empty((B, H, W, 8), dtype=torch.float32, device="cuda")
    qnn.qnn_conv3x3_fwd(B, H, W, x, ci, w, bias, 32, act, y, 1, 8, 6)
    want = torch.empty((B, 6, H, W), dtype=torch.float32, device="cuda")
    qnn.qnn_unpack_output(B, H, W, y, 8, scale, want)
    got = torch.full((B, 6, H, W), 3.0, dtype=torch.float32, device="cuda")
    qnn.qnn_conv3x3_fwd_planes(B, H, W, x, ci, w, bias, 32, act, scale, 6, got)
    assert torch.equal(got.view(torch.int32), want.view(torch.int32))
    y32 = torch.empty((B, H, W, 32), dtype=torch.float32, device="cuda")
    qnn.qnn_conv3x3_fwd(B, H, W, x, ci, w, bias, 32, act, y32, 1, 32, 32)
    want32 = y32.permute(0, 3, 1, 2).contiguous() * scale[:, None, None, None]
    got32 = torch.empty((B, 32, H, W), dtype=torch.float32, device="cuda")
    qnn.qnn_conv3x3_fwd_planes(B, H, W, x, ci, w, bias, 32, act, scale, 32, got32)
    assert torch.equal(got32.view(torch.int32), want32.view(torch.int32))


@pytest.mark.parametrize("B,H,W,ci,co", [(2, 16, 16, 16, 32), (1, 6, 10, 64, 32), (2, 2, 2, 128, 128),
                                         (4, 32, 64, 32, 64)])
def test_conv_data_gradient(env, B, H, W, ci, co):
    torch, qnn = env
    dy, dyr = bf(torch, rnd(6, (B, H, W, co)))
    w, wr = bf(torch, rnd(7, (co, 9, ci), 0.1))
    wt = torch.empty_like(w)
    qnn.qnn_conv3x3_flip(w, co, ci, wt)
    if ci % 32 == 0:      # the data gradient runs the forward kernel with c_out = ci
        dx = torch.empty((B, H, W, ci), dtype=torch.float32, device="cuda")
        qnn.qnn_conv3x3_fwd(B, H, W, dy, co, wt, None, ci, 0, dx, 1, ci, ci)
        ref = N.conv3x3_dgrad(dyr, wr)
        assert np.abs(dx.cpu().numpy() - ref).max() <= 2e-6 * np.abs(ref).max()
    # the flip itself, entry by entry
    wt_np = wt.float().cpu().numpy().reshape(ci, 9, co)
    for t in range(9):
        np.testing.assert_array_equal(wt_np[:, 8 - t, :], wr[:, t, :].T)


@pytest.mark.parametrize("B,H,W,ci,co", [(2, 16, 32, 16, 32), (1, 32, 32, 32, 64), (2, 4, 4, 128, 128),
                                         (1, 2, 2, 128, 128), (3, 7, 5, 16, 32),
                                         # staged kernel: W = 24 (groups advance over several rows
                                         # per chunk), 720 pixels (a partial last chunk), many
                                         # pixel ranges, c_out = 96 (one 32-channel tile per block)
                                         (3, 10, 24, 48, 32), (4, 64, 64, 32, 64), (2, 16, 32, 16, 96)])
def test_conv_weight_gradient(env, B, H, W, ci, co):
    torch, qnn = env
    x, xr = bf(torch, rnd(8, (B, H, W, ci)))
    dy, dyr = bf(torch, rnd(9, (B, H, W, co)))
    dw = torch.empty(co * 9 * ci, dtype=torch.float32, device="cuda")
    db = torch.empty(co, dtype=torch.float32, device="cuda")
    work = torch.empty(qnn.qnn_wgrad_work_floats(B, H, W, ci, co), dtype=torch.float32, device="cuda")
    qnn.qnn_conv3x3_wgrad(B, H, W, x, ci, dy, co, dw, db, work)
    rdw, rdb = N.conv3x3_wgrad(xr, dyr)
    got = dw.cpu().numpy().reshape(co, 9, ci)
    P = B * H * W
    assert np.abs(got - rdw).max() <= 1e-6 * np.sqrt(P) * np.abs(rdw).max() + 1e-5
    assert np.abs(db.cpu().numpy() - rdb).max() <= 1e-6 * np.sqrt(P) * np.abs(rdb).max() + 1e-5
    again = torch.empty_like(dw)
    qnn.qnn_conv3x3_wgrad(B, H, W, x, ci, dy, co, again, None, work)
    assert torch.equal(dw, again)       # deterministic reduction order


@pytest.mark.parametrize("B,H,W,ci,co", [(2, 16, 32, 16, 32), (3, 7, 5, 32, 64)])
def test_conv_weight_gradient_unaligned_views(env, B, H, W, ci, co):
    """x and dy one element into their buffers (not 16-byte aligned): the
    pixel-list weight-gradient kernel, which reads 2-byte elements."""
    torch, qnn = env
    xa, xr = bf(torch, rnd(10, B * H * W * ci + 1))
    da, dr = bf(torch, rnd(11, B * H * W * co + 1))
    x, dy = xa[1:], da[1:]
    xr = xr[1:].reshape(B, H, W, ci)
    dyr = dr[1:].reshape(B, H, W, co)
    dw = torch.empty(co * 9 * ci, dtype=torch.float32, device="cuda")
    db = torch.empty(co, dtype=torch.float32, device="cuda")
    work = torch.empty(qnn.qnn_wgrad_work_floats(B, H, W, ci, co), dtype=torch.float32, device="cuda")
    qnn.qnn_conv3x3_wgrad(B, H, W, x, ci, dy, co, dw, db, work)
    rdw, rdb = N.conv3x3_wgrad(xr, dyr)
    P = B * H * W
    got = dw.cpu().numpy().reshape(co, 9, ci)
    assert np.abs(got - rdw).max() <= 1e-6 * np.sqrt(P) * np.abs(rdw).max() + 1e-5
    assert np.abs(db.cpu().numpy() - rdb).max() <= 1e-6 * np.sqrt(P) * np.abs(rdb).max() + 1e-5

@pytest.mark.parametrize("C", [32, 48, 12])
def test_elementwise_kernels_bit_exact(env, C):
    """C % 8 == 0 runs the 16-byte vector kernels, C = 12 the scalar ones."""
    torch, qnn = env
    B, H, W = 2, 8, 12
    x, xr = bf(torch, rnd(10, (B, H, W, C)))
    y, yr = bf(torch, rnd(11, (B, H, W, C)))
    n = B * H * W * C
    out = torch.empty_like(x)
    qnn.qnn_add(n, x, y, out)
    np.testing.assert_array_equal(out.float().cpu().numpy(), N.bf16_round(xr + yr))
    qnn.qnn_leaky_bwd(n, x, y, out)
    np.testing.assert_array_equal(out.float().cpu().numpy(), N.bf16_round(N.leaky_bwd(xr, yr)))
    p = torch.empty((B, H // 2, W // 2, C), dtype=torch.bfloat16, device="cuda")
    qnn.qnn_avgpool2(B, H, W, C, x, p)
    np.testing.assert_array_equal(p.float().cpu().numpy(), N.bf16_round(N.avgpool2(xr)))
    pr = p.float().cpu().numpy().astype(np.float64)
    g = torch.empty_like(x)
    qnn.qnn_avgpool2_bwd(B, H, W, C, p, g, 0)
    np.testing.assert_array_equal(g.float().cpu().numpy(), N.bf16_round(N.avgpool2_bwd(pr)))
    g2 = y.clone()
    qnn.qnn_avgpool2_bwd(B, H, W, C, p, g2, 1)
    np.testing.assert_array_equal(g2.float().cpu().numpy(), N.bf16_round(yr + N.avgpool2_bwd(pr)))
    u = torch.empty((B, 2 * H, 2 * W, C), dtype=torch.bfloat16, device="cuda")
    qnn.qnn_upsample2(B, H, W, C, x, u)
    np.testing.assert_array_equal(u.float().cpu().numpy(), N.upsample2(xr))
    d = torch.empty_like(x)
    qnn.qnn_upsample2_bwd(B, H, W, C, u, d)
    np.testing.assert_array_equal(d.float().cpu().numpy(), N.bf16_round(N.upsample2_bwd(N.upsample2(xr))))


def test_elementwise_unaligned_views(env):
    """Views that start 2 bytes into a buffer take the scalar kernels."""
    torch, qnn = env
    n = 8 * 1000
    xa, xr = bf(torch, rnd(30, n + 1))
    ya, yr = bf(torch, rnd(31, n + 1))
    out = torch.empty(n + 1, dtype=torch.bfloat16, device="cuda")
    qnn.qnn_add(n, xa[1:], ya[1:], out[1:])
    np.testing.assert_array_equal(out[1:].float().cpu().numpy(), N.bf16_round(xr[1:] + yr[1:]))
    qnn.qnn_leaky_bwd(n, xa[1:], ya[1:], out[1:])
    np.testing.assert_array_equal(out[1:].float().cpu().numpy(), N.bf16_round(N.leaky_bwd(xr[1:], yr[1:])))


def test_pack_absmax_unpack(env):
    torch, qnn = env
    Nq, Bn, H, W = 5, 3, 16, 32
    q = torch.tensor(rnd(12, (Nq, 6, H, W)).astype(np.float32)).cuda()
    nn = torch.tensor((2 + rnd(13, (Bn, 3, H, W))).astype(np.float32)).cuda()
    idx_q = torch.tensor([4, 0, 2, 2], dtype=torch.int32).cuda()
    idx_n = torch.tensor([1, 0, 2, 1], dtype=torch.int32).cuda()
    B = 4
    scale = torch.empty(B, dtype=torch.float32, device="cuda")
    qnn.qnn_absmax(B, H, W, q, idx_q, scale)
    qn = q.cpu().numpy()
    want_scale = np.abs(qn[[4, 0, 2, 2]]).reshape(B, -1).max(axis=1)
    np.testing.assert_array_equal(scale.cpu().numpy(), want_scale.astype(np.float32))
    x = torch.empty((B, H, W, 48), dtype=torch.bfloat16, device="cuda")
    nnp = nn.cpu().numpy()
    # displacements within the lattice, negative, and longer than both sides
    for d in (5, -3, 37):
        qnn.qnn_pack_input(B, H, W, q, idx_q, nn, idx_n, scale, 2.0, 1.0, d, x)
        xs = x.float().cpu().numpy()
        check_pack(xs, qn, nnp, want_scale, d)
    y = torch.tensor(rnd(14, (B, H, W, 32)).astype(np.float32)).cuda()
    out = torch.empty((B, 6, H, W), dtype=torch.float32, device="cuda")
    qnn.qnn_unpack_output(B, H, W, y, 32, scale, out)
    want = y.cpu().numpy()[..., :6].transpose(0, 3, 1, 2) * scale.cpu().numpy()[:, None, None, None]
    np.testing.assert_array_equal(out.cpu().numpy(), want.astype(np.float32))


def test_pack_input_ragged_and_large(env):
    """A pixel count that leaves a partial run of 256, and a batch large
    enough that blocks pack several runs (rows sampled)."""
    torch, qnn = env
    for B, H, W, d, rows in ((3, 7, 45, 4, None), (5, 1024, 1024, 77, (0, 1, 76, 77, 500, 947, 1023))):
        qn = rnd(40, (B, 6, H, W)).astype(np.float32)
        nnp = (2 + rnd(41, (B, 3, H, W))).astype(np.float32)
        q, nn = torch.tensor(qn).cuda(), torch.tensor(nnp).cuda()
        scale = torch.empty(B, dtype=torch.float32, device="cuda")
        qnn.qnn_absmax(B, H, W, q, None, scale)
        x = torch.empty((B, H, W, 48), dtype=torch.bfloat16, device="cuda")
        qnn.qnn_pack_input(B, H, W, q, None, nn, None, scale, 2.0, 1.0, d, x)
        sc = scale.cpu().numpy()
        sel = slice(None) if rows is None else list(rows)
        xs = x[:, sel].float().cpu().numpy()
        for b in range(B):
            f = (qn[b] / np.float32(sc[b])).transpose(1, 2, 0)
            want = np.concatenate([f, (nnp[b] - np.float32(2.0)).transpose(1, 2, 0), np.roll(f, d, axis=1),
                                   np.roll(f, -d, axis=1), np.roll(f, d, axis=0), np.roll(f, -d, axis=0),
                                   np.zeros((H, W, 15), np.float32)], axis=2)
            np.testing.assert_array_equal(xs[b], N.bf16_round(want[sel]))


def check_pack(xs, qn, nnp, want_scale, d):
    for b, (iq, inn) in enumerate(zip([4, 0, 2, 2], [1, 0, 2, 1])):
        f = (qn[iq] / np.float32(want_scale[b])).transpose(1, 2, 0)          # (H, W, 6)
        np.testing.assert_array_equal(xs[b, :, :, :6], N.bf16_round(f))
        np.testing.assert_array_equal(xs[b, :, :, 6:9], N.bf16_round((nnp[inn] - np.float32(2.0)).transpose(1, 2, 0)))
        np.testing.assert_array_equal(xs[b, :, :, 9:15], N.bf16_round(np.roll(f, d, axis=1)))    # Q(y, x - d)
        np.testing.assert_array_equal(xs[b, :, :, 15:21], N.bf16_round(np.roll(f, -d, axis=1)))  # Q(y, x + d)
        np.testing.assert_array_equal(xs[b, :, :, 21:27], N.bf16_round(np.roll(f, d, axis=0)))   # Q(y - d, x)
        np.testing.assert_array_equal(xs[b, :, :, 27:33], N.bf16_round(np.roll(f, -d, axis=0)))  # Q(y + d, x)
        assert np.all(xs[b, :, :, 33:] == 0)


def test_absmax_large_and_zero_samples(env):
    torch, qnn = env
    B, H, W = 3, 512, 384
    q = torch.tensor(rnd(21, (B, 6, H, W)).astype(np.float32)).cuda()
    q[1].zero_()
    q[2, 5, 511, 383] = -7.5
    scale = torch.full((B,), 123.0, dtype=torch.float32, device="cuda")
    qnn.qnn_absmax(B, H, W, q, None, scale)
    want = np.abs(q.cpu().numpy()).reshape(B, -1).max(axis=1)
    want[1] = 1.0
    np.testing.assert_array_equal(scale.cpu().numpy(), want.astype(np.float32))
    # an odd pixel count (6 H W not a multiple of 4) and an unaligned view:
    # the 4-byte-load form
    for B, H, W, off in ((3, 7, 9, 0), (2, 8, 8, 1)):
        buf = torch.tensor(rnd(22, B * 6 * H * W + off).astype(np.float32)).cuda()
        q = buf[off:].view(B, 6, H, W)
        scale = torch.empty(B, dtype=torch.float32, device="cuda")
        qnn.qnn_absmax(B, H, W, q, None, scale)
        want = np.abs(q.cpu().numpy()).reshape(B, -1).max(axis=1)
        np.testing.assert_array_equal(scale.cpu().numpy(), want.astype(np.float32))


@pytest.mark.parametrize("pred_ld,d_ld", [(32, 32), (8, 32), (8, 6)])
def test_relative_l2_loss_and_gradient(env, pred_ld, d_ld):
    torch, qnn = env
    B, H, W = 3, 16, 16
    pred = torch.tensor(rnd(15, (B, H, W, pred_ld)).astype(np.float32)).cuda()
    tgt = torch.tensor(rnd(16, (4, 6, H, W)).astype(np.float32)).cuda()
    idx = torch.tensor([3, 1, 0], dtype=torch.int32).cuda()
    scale = torch.tensor([2.0, 0.5, 1.0], dtype=torch.float32).cuda()
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    per = torch.zeros(B, dtype=torch.float64, device="cuda")
    work = torch.zeros(64 * B, dtype=torch.float64, device="cuda")
    d = torch.full((B, H, W, d_ld), 5.0, dtype=torch.bfloat16, device="cuda")
    qnn.qnn_rel_l2(B, H, W, pred, pred_ld, tgt, idx, scale, d, d_ld, loss, per, work)
    p = pred.cpu().numpy().astype(np.float64)[..., :6]
    t = (tgt.cpu().numpy().astype(np.float64)[[3, 1, 0]] / np.array([2.0, 0.5, 1.0])[:, None, None, None])
    t = t.transpose(0, 2, 3, 1)
    rl, rper, rg = N.rel_l2(p, t)
    assert abs(loss.item() - rl) <= 1e-12 * rl
    np.testing.assert_allclose(per.cpu().numpy(), rper, rtol=1e-12)
    dg = d.float().cpu().numpy()
    assert np.all(np.abs(dg[..., :6] - rg) <= 2.0 ** -8 * np.abs(rg) + 1e-30)
    assert np.all(dg[..., 6:] == 0)


def test_adam_step(env):
    torch, qnn = env
    n = 1000
    r = np.random.default_rng(17)
    p0, m0, v0, g0 = (r.standard_normal(n).astype(np.float32) for _ in range(4))
    v0 = np.abs(v0)
    p, m, v, g = (torch.tensor(a).cuda() for a in (p0, m0, v0, g0))
    pb = torch.empty(n, dtype=torch.bfloat16, device="cuda")
    qnn.qnn_adam(n, p, m, v, g, pb, 1e-3, 0.9, 0.999, 1e-8, 3)
    b1, b2, lr, eps, t = 0.9, 0.999, 1e-3, 1e-8, 3
    m1 = b1 * m0.astype(np.float64) + (1 - b1) * g0
    v1 = b2 * v0.astype(np.float64) + (1 - b2) * g0.astype(np.float64) ** 2
    p1 = p0 - lr * (m1 / (1 - b1 ** t)) / (np.sqrt(v1 / (1 - b2 ** t)) + eps)
    np.testing.assert_allclose(p.cpu().numpy(), p1, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(m.cpu().numpy(), m1, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(v.cpu().numpy(), v1, rtol=1e-6, atol=1e-7)
    np.testing.assert_array_equal(pb.float().cpu().numpy(), N.bf16_round(p.cpu().numpy()))


@pytest.mark.parametrize("m", [1, 1000, 300001])
def test_compare(env, m):
    torch, qnn = env
    a = torch.tensor(rnd(18, (3, m)).astype(np.float32)).cuda()
    b = torch.tensor(rnd(19, (3, m)).astype(np.float32)).cuda()
    rel = torch.empty(3, dtype=torch.float64, device="cuda")
    en = torch.empty(3, dtype=torch.float64, device="cuda")
    work = torch.empty(qnn.qnn_compare_work_doubles(3), dtype=torch.float64, device="cuda")
    qnn.qnn_compare(3, m, a, b, rel, en, work)
    A, Bn = a.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(rel.cpu().numpy(), np.linalg.norm(A - Bn, axis=1) / np.linalg.norm(Bn, axis=1), rtol=1e-12)
    np.testing.assert_allclose(en.cpu().numpy(), np.abs((A ** 2).sum(1) - (Bn ** 2).sum(1)) / (Bn ** 2).sum(1), rtol=1e-10)


@pytest.mark.parametrize("H,W", [(64, 128), (32, 64)])
def test_network_forward_fused_is_bitwise_unfused(env, H, W):
    """Inference folds each decoder level's upsampling and skip addition
    into its first convolution where the tile widths fit (at W = 64 the
    8-wide level stays unfused)."""
    torch, qnn = env
    from paper_2301_13601_amd import surrogate as S

    net = S.UNet(seed=5)
    B = 2
    net._buffers(B, H, W)
    xin = rnd(24, (B, H, W, 48))
    xin[..., 33:] = 0
    xt, _ = bf(torch, xin)
    net.act["x"].copy_(xt.view(-1))
    a = net.forward_packed(B, H, W).clone()
    b = net.forward_packed(B, H, W, fused=True).clone()
    assert torch.equal(a, b)


def test_whole_network_forward_and_gradients(env):
    """GPU U-net (BF16 storage, FP32 accumulation) against the FP64 oracle
    network. Forward: the oracle rounds to BF16 where the GPU stores BF16.
    Every activation the GPU saves for its backward pass is checked against
    the oracle's. Backward: the oracle runs on the GPU's saved activations
    (so both use the same leaky-ReLU masks: a pre-activation within rounding
    of zero can otherwise land on either side) and rounds stored activation
    gradients to BF16 as the GPU does; per-layer weight and bias gradients
    then agree to a few parts in a thousand; on the oracle's own activations
    the whole gradient agrees to a few percent. Also reports the forward's
    distance from the same network in exact arithmetic (the BF16 floor)."""
    torch, qnn = env
    from paper_2301_13601_amd import surrogate as S

    net = S.UNet(seed=21)
    B, H, W = 2, 32, 32
    net._buffers(B, H, W, train=True)
    xin = rnd(22, (B, H, W, 48))
    xin[..., 33:] = 0
    xt, xr = bf(torch, xin)
    net.act["x"].copy_(xt.view(-1))
    out = net.forward_packed(B, H, W)
    got = out.cpu().numpy().reshape(B, H, W, S.OUT_LD)[..., :6]
    p = net.p.cpu().numpy().astype(np.float64)
    # weights as the GPU uses them (BF16), biases FP32
    pr = p.copy()
    off = 0
    for name, ci, co, _, _ in N.unet_layers():
        pr[off:off + co * 9 * ci] = N.bf16_round(p[off:off + co * 9 * ci].astype(np.float32))
        off += co * 9 * ci + co
    ref, act = N.unet_forward(pr, xr, bf16=True)
    assert np.linalg.norm(got - ref[..., :6]) <= 2e-2 * np.linalg.norm(ref[..., :6])

    gpu_act = {}
    for name, r in act.items():
        if name in net.act and name != "out":
            gpu_act[name] = net.act[name].float().cpu().numpy().astype(np.float64).reshape(r.shape)
            # the buffers the backward pass reads hold this forward's values
            assert np.linalg.norm(gpu_act[name] - r) <= 2e-2 * np.linalg.norm(r), name
    # the BF16 floor of this network: the same weights and input in exact
    # arithmetic (no BF16 rounding anywhere)
    exact, _ = N.unet_forward(p, xr, bf16=False)
    floor = np.linalg.norm(got - exact[..., :6]) / np.linalg.norm(exact[..., :6])
    print(f"  forward vs exact FP64 network: relative L2 {floor:.3e}")
    assert floor <= 5e-2
    dout = rnd(23, (B, H, W, 32)) * 0.1
    dout[..., 6:] = 0
    dt, dr = bf(torch, dout)
    net.backward(B, H, W, dt.view(-1))
    g = net.g.cpu().numpy().astype(np.float64)
    rg = N.unet_backward(pr, gpu_act, dr, bf16=True)
    # and on the oracle's own activations: the leaky-ReLU masks may differ
    # where a pre-activation is within rounding of zero, so the bar is looser
    rg_own = N.unet_backward(pr, act, dr, bf16=True)
    assert np.linalg.norm(g - rg_own) <= 5e-2 * np.linalg.norm(rg_own)
    off = 0
    for name, ci, co, _, _ in N.unet_layers():
        n_w = co * 9 * ci
        for a, b in ((g[off:off + n_w], rg[off:off + n_w]), (g[off + n_w:off + n_w + co], rg[off + n_w:off + n_w + co])):
            assert np.linalg.norm(a - b) <= 1e-2 * np.linalg.norm(b), name
        off += n_w + co
