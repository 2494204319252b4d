"""Convolutional surrogate of K whole QLA steps, trained on the library's own
runs, with plain QLA as its check and fallback.

The network maps (Q(t), n) -> Q(t + K) on a periodic lattice (K = 256 by
default). QLA is linear in Q for fixed n, so each sample is divided by its
largest |q| on the way in and multiplied back on the way out. Architecture:
a four-level U-net with additive skips,

  level l (l = 0..3, resolution /2^l): two 3x3 convs to C_l = 32, 64, 128, 128
  bottleneck (resolution /16): four 3x3 convs at 128 channels
  decoder level l: 2x upsample, 3x3 conv to C_l, add the level-l encoder
                   output, 3x3 conv
  output: 3x3 conv to 6 channels (FP32), no activation

The input carries, besides Q(t) and n, four copies of Q(t) displaced by the
distance a vacuum wave covers in one jump (delta*K cells) along +x, -x, +y
and -y, so that the skip paths see detail where waves moving along an axis
end up. Circular padding everywhere (the lattice is periodic), leaky ReLU
(slope 1/8), BF16 activations and weights, FP32 accumulation, FP32 master
weights and Adam. Its receptive field is about +-125 cells, beyond the
~77 cells a vacuum pulse travels in 256 steps at delta = 0.3. Every
arithmetic step runs in the HIP kernels of include/qla_nn.h; torch only
holds device memory.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import qla, qnn, scenes

LEVELS = (32, 64, 128, 128)
BOTTLENECK = 4
IN_CH = 48            # 6 field + 3 index + 4x6 displaced field channels, padded to 48
LIVE_IN = 33          # channels that carry data
OUT_CH = 32           # output conv width (6 stored)
OUT_LD = 8            # row length of the FP32 network output (6 used)
N_SHIFT, N_SCALE = 2.0, 1.0


@dataclasses.dataclass
class Conv:
    name: str
    c_in: int
    c_out: int
    act: int
    level: int
    w_off: int = 0    # offsets into the flat parameter buffer
    b_off: int = 0

    @property
    def n_w(self) -> int:
        return self.c_out * 9 * self.c_in


def widest_per_pixel() -> int:
    """Most elements per full-resolution pixel that one convolution reads
    or writes at its own level: the packed input, and every layer's input
    (for a decoder's first convolution, its 2x-upsampled input) and output,
    divided by the 4^level pixels they are spread over. 64 for this network:
    the level-1 output that decoder level 0 reads upsampled to full size."""
    widest = IN_CH
    for s in layer_specs():
        widest = max(widest, -(-max(s.c_in, s.c_out) // 4 ** s.level))
    return widest


def default_chunk(H: int, W: int) -> int:
    """Lattices per inference chunk: as many as the kernels' 31-bit element
    offsets allow for the widest tensor of any layer, at most 16, at least
    1."""
    return max(1, min(16, ((1 << 31) - 1) // (widest_per_pixel() * H * W)))


def layer_specs() -> List[Conv]:
    L = qnn.QNN_ACT_LEAKY
    specs = [Conv("e0a", IN_CH, LEVELS[0], L, 0), Conv("e0", LEVELS[0], LEVELS[0], L, 0)]
    for l in range(1, 4):
        specs += [Conv(f"e{l}a", LEVELS[l - 1], LEVELS[l], L, l), Conv(f"e{l}", LEVELS[l], LEVELS[l], L, l)]
    for k in range(BOTTLENECK):
        specs.append(Conv(f"b{k}", LEVELS[3], LEVELS[3], L, 4))
    up_in = LEVELS[3]
    for l in (3, 2, 1, 0):
        specs += [Conv(f"d{l}a", up_in, LEVELS[l], L, l), Conv(f"d{l}", LEVELS[l], LEVELS[l], L, l)]
        up_in = LEVELS[l]
    specs.append(Conv("out", LEVELS[0], OUT_CH, qnn.QNN_ACT_NONE, 0))
    off = 0
    for s in specs:
        s.w_off = off
        off += s.n_w
        s.b_off = off
        off += s.c_out
    return specs


def macs_per_pixel() -> float:
    """Multiply-accumulates of one forward pass per full-resolution pixel."""
    return sum(s.n_w / 4 ** s.level for s in layer_specs())


class UNet:
    """Parameters, Adam state and activation buffers of the surrogate."""

    def __init__(self, device="cuda:0", seed: int = 0, stream=None, shift: int = 77):
        import torch

        # displacement of the shifted input copies: the distance (cells) a
        # vacuum wave travels over one jump, delta * K (0.3 * 256 = 76.8)
        self.shift = int(shift)
        self.torch = torch
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.specs = layer_specs()
        self.by_name = {s.name: s for s in self.specs}
        self.n_params = self.specs[-1].b_off + self.specs[-1].c_out
        rng = np.random.default_rng(seed)
        p = np.zeros(self.n_params, dtype=np.float32)
        for s in self.specs:
            fan_in = 9 * (LIVE_IN if s.name == "e0a" else s.c_in)
            std = math.sqrt(2.0 / fan_in) * (0.1 if s.name == "out" else 1.0)
            w = rng.standard_normal((s.c_out, 9, s.c_in)).astype(np.float32) * std
            if s.name == "e0a":
                w[:, :, LIVE_IN:] = 0.0
            p[s.w_off:s.w_off + s.n_w] = w.ravel()
        f32 = dict(dtype=torch.float32, device=self.device)
        self.p = torch.as_tensor(p).to(self.device)
        self.m = torch.zeros(self.n_params, **f32)
        self.v = torch.zeros(self.n_params, **f32)
        self.g = torch.zeros(self.n_params, **f32)
        self.pb = torch.empty(self.n_params, dtype=torch.bfloat16, device=self.device)
        self.flipped = {s.name: torch.empty(s.n_w, dtype=torch.bfloat16, device=self.device)
                        for s in self.specs}
        qnn.qnn_to_bf16(self.n_params, self.p, self.pb, self.stream)
        self.t = 0
        self.geom = None
        self.trainable = False

    # -- parameter views ----------------------------------------------------
    def w(self, s: Conv):
        return self.pb[s.w_off:s.w_off + s.n_w]

    def b(self, s: Conv):
        return self.p[s.b_off:s.b_off + s.c_out]

    def dw(self, s: Conv):
        return self.g[s.w_off:s.w_off + s.n_w]

    def db(self, s: Conv):
        return self.g[s.b_off:s.b_off + s.c_out]

    def state(self) -> Dict[str, np.ndarray]:
        return {"p": self.p.cpu().numpy(), "m": self.m.cpu().numpy(), "v": self.v.cpu().numpy(),
                "t": np.array(self.t)}

    def load(self, st: Dict[str, np.ndarray]) -> None:
        torch = self.torch
        self.p.copy_(torch.as_tensor(st["p"]))
        self.m.copy_(torch.as_tensor(st["m"]))
        self.v.copy_(torch.as_tensor(st["v"]))
        self.t = int(st["t"])
        qnn.qnn_to_bf16(self.n_params, self.p, self.pb, self.stream)

    # -- buffers ---------------------------------------------------------------
    def _buffers(self, B: int, H: int, W: int, train: bool = False) -> None:
        if self.geom == (B, H, W) and (self.trainable or not train):
            return
        self.trainable = train
        if H % 16 or W % 16:
            raise ValueError("lattice sides must be multiples of 16")
        torch = self.torch
        bf = dict(dtype=torch.bfloat16, device=self.device)
        self.geom = (B, H, W)
        self.act, self.grad = {}, {}

        def px(level):
            return B * (H >> level) * (W >> level)

        self.act["x"] = torch.empty(px(0) * IN_CH, **bf)
        for s in self.specs:
            if s.name == "out":
                self.act["out"] = torch.empty(px(0) * OUT_LD, dtype=torch.float32, device=self.device)
            else:
                self.act[s.name] = torch.empty(px(s.level) * s.c_out, **bf)
        for l in range(1, 5):
            self.act[f"p{l}"] = torch.empty(px(l) * LEVELS[l - 1], **bf)
        up_c = LEVELS[3]
        for l in (3, 2, 1, 0):
            self.act[f"u{l}"] = torch.empty(px(l) * up_c, **bf)
            self.act[f"h{l}"] = torch.empty(px(l) * LEVELS[l], **bf)
            up_c = LEVELS[l]
        if train:
            # gradients of every activation, and the activation-gradient
            # product of each leaky ReLU
            for name, t in self.act.items():
                if name not in ("x", "out"):
                    self.grad[name] = torch.empty_like(t)
            self.grad["out"] = torch.empty(px(0) * OUT_CH, **bf)
            self.dz = {s.name: torch.empty(px(s.level) * s.c_out, **bf) for s in self.specs}
            wk = max(qnn.qnn_wgrad_work_floats(B, H >> s.level, W >> s.level, s.c_in, s.c_out)
                     for s in self.specs)
            self.wwork = torch.empty(wk, dtype=torch.float32, device=self.device)
        self.scale = torch.empty(B, dtype=torch.float32, device=self.device)
        self.loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        self.per_sample = torch.zeros(B, dtype=torch.float64, device=self.device)
        self.lwork = torch.zeros(64 * B, dtype=torch.float64, device=self.device)

    # -- forward -----------------------------------------------------------------
    def _conv(self, s: Conv, x, B, H, W, y=None, fp32=False):
        h, w = H >> s.level, W >> s.level
        y = self.act[s.name] if y is None else y
        if fp32:
            qnn.qnn_conv3x3_fwd(B, h, w, x, s.c_in, self.w(s), self.b(s), s.c_out, s.act, y, 1, OUT_LD, 6,
                                self.stream)
        else:
            qnn.qnn_conv3x3_fwd(B, h, w, x, s.c_in, self.w(s), self.b(s), s.c_out, s.act, y, 0, s.c_out,
                                s.c_out, self.stream)
        return y

    def forward_packed(self, B: int, H: int, W: int, fused: bool = False, planes=None):
        """Run the network on self.act["x"]; returns the FP32 output [P][8]
        (6 channels used). fused: each decoder level's upsampling and skip
        addition run inside its first convolution (qnn_conv3x3_fwd_fused,
        bitwise the same result) wherever that kernel's tile widths fit; the
        upsampled and pre-addition tensors are then not stored, so training,
        whose backward pass reads them, runs unfused. planes: an FP32 tensor
        [B][6][H][W] that receives the unpacked, rescaled output directly
        (qnn_conv3x3_fwd_planes, bitwise the FP32 output then
        qnn_unpack_output); None is returned then."""
        A, S = self.act, self.by_name
        st = self.stream
        x = A["x"]
        for l in range(4):
            x = self._conv(S[f"e{l}a"], x, B, H, W)
            s = S[f"e{l}"]
            if fused:
                # the level's pooled output from the convolution's own tiles
                # where they allow it (qnn_conv3x3_fwd_pool, bitwise the two
                # calls below)
                qnn.qnn_conv3x3_fwd_pool(B, H >> l, W >> l, x, s.c_in, self.w(s), self.b(s), s.c_out, s.act,
                                         A[s.name], A[f"p{l + 1}"], st)
            else:
                self._conv(s, x, B, H, W)
                qnn.qnn_avgpool2(B, H >> l, W >> l, LEVELS[l], A[s.name], A[f"p{l + 1}"], st)
            x = A[f"p{l + 1}"]
        for k in range(BOTTLENECK):
            x = self._conv(S[f"b{k}"], x, B, H, W)
        up_c = LEVELS[3]
        for l in (3, 2, 1, 0):
            s, w_l = S[f"d{l}a"], W >> l
            if fused and (w_l in (16, 32) or w_l % 64 == 0):
                qnn.qnn_conv3x3_fwd_fused(B, H >> l, w_l, x, s.c_in, 1, self.w(s), self.b(s), s.c_out, s.act,
                                          A[f"e{l}"], A[f"h{l}"], s.c_out, st)
            else:
                qnn.qnn_upsample2(B, H >> (l + 1), W >> (l + 1), up_c, x, A[f"u{l}"], st)
                d = self._conv(s, A[f"u{l}"], B, H, W)
                n = B * (H >> l) * (W >> l) * LEVELS[l]
                qnn.qnn_add(n, d, A[f"e{l}"], A[f"h{l}"], st)
            x = self._conv(S[f"d{l}"], A[f"h{l}"], B, H, W)
            up_c = LEVELS[l]
        if planes is not None:
            s = S["out"]
            qnn.qnn_conv3x3_fwd_planes(B, H, W, x, s.c_in, self.w(s), self.b(s), s.c_out, s.act, self.scale, 6,
                                       planes, st)
            return None
        return self._conv(S["out"], x, B, H, W, fp32=True)

    def pack(self, B, H, W, q, idx_q, n, idx_n, train=False):
        """Input tensor from lattice fields (q [N][6][H][W], n [M][3][H][W],
        int32 index tensors or None); sets the per-sample scales."""
        self._buffers(B, H, W, train)
        qnn.qnn_absmax(B, H, W, q, idx_q, self.scale, self.stream)
        qnn.qnn_pack_input(B, H, W, q, idx_q, n, idx_n, self.scale, N_SHIFT, N_SCALE, self.shift,
                           self.act["x"], self.stream)

    def predict(self, q, n, out_q, chunk: int = 0):
        """out_q[b] = network(q[b], n[b]) for lattices q [B][6][H][W] (FP32),
        in chunks of at most ``chunk`` lattices (0: as many as the kernels'
        31-bit element offsets allow for the widest layer tensor, at most 16;
        fewer, smaller launches leave the deep layers' grids short)."""
        B, _, H, W = q.shape
        if chunk <= 0:
            chunk = default_chunk(H, W)
        for c0 in range(0, B, chunk):
            c1 = min(B, c0 + chunk)
            self.pack(c1 - c0, H, W, q[c0:c1], None, n[c0:c1], None)
            self.forward_packed(c1 - c0, H, W, fused=True, planes=out_q[c0:c1])

    # -- backward ----------------------------------------------------------------
    def _conv_bwd(self, s: Conv, x_in, dy, B, H, W, dx=None):
        """Gradients of y = act(conv(x_in)) given dL/dy; returns dL/dx_in
        (written to dx) unless dx is None."""
        h, w = H >> s.level, W >> s.level
        st = self.stream
        if s.act == qnn.QNN_ACT_LEAKY:
            dz = self.dz[s.name]
            qnn.qnn_leaky_bwd(B * h * w * s.c_out, self.act[s.name], dy, dz, st)
        else:
            dz = dy
        qnn.qnn_conv3x3_wgrad(B, h, w, x_in, s.c_in, dz, s.c_out, self.dw(s), self.db(s), self.wwork, st)
        if dx is not None:
            qnn.qnn_conv3x3_fwd(B, h, w, dz, s.c_out, self.flipped[s.name], None, s.c_in, qnn.QNN_ACT_NONE,
                                dx, 0, s.c_in, s.c_in, st)
        return dx

    def backward(self, B: int, H: int, W: int, dout) -> None:
        A, G, S = self.act, self.grad, self.by_name
        st = self.stream
        for s in self.specs:
            qnn.qnn_conv3x3_flip(self.w(s), s.c_out, s.c_in, self.flipped[s.name], st)
        # decoder, top down
        g = self._conv_bwd(S["out"], A["d0"], dout, B, H, W, G["d0"])
        for l in (0, 1, 2, 3):
            # d_l = conv(h_l); h_l = d_la + e_l; d_la = conv(u_l); u_l = up(prev)
            self._conv_bwd(S[f"d{l}"], A[f"h{l}"], g, B, H, W, G[f"h{l}"])
            prev = "b3" if l == 3 else f"d{l + 1}"
            up_c = LEVELS[3] if l == 3 else LEVELS[l + 1]
            self._conv_bwd(S[f"d{l}a"], A[f"u{l}"], G[f"h{l}"], B, H, W, G[f"u{l}"])
            qnn.qnn_upsample2_bwd(B, H >> (l + 1), W >> (l + 1), up_c, G[f"u{l}"], G[prev], st)
            g = G[prev]
        # bottleneck
        for k in range(BOTTLENECK - 1, -1, -1):
            x_in = A["p4"] if k == 0 else A[f"b{k - 1}"]
            dx = G["p4"] if k == 0 else G[f"b{k - 1}"]
            self._conv_bwd(S[f"b{k}"], x_in, g, B, H, W, dx)
            g = dx
        # encoder, bottom up: e_l's gradient is dL/dh_l (from the skip) plus
        # the pooled path, accumulated into G[h_l]
        for l in (3, 2, 1, 0):
            qnn.qnn_avgpool2_bwd(B, H >> l, W >> l, LEVELS[l], g, G[f"h{l}"], 1, st)
            self._conv_bwd(S[f"e{l}"], A[f"e{l}a"], G[f"h{l}"], B, H, W, G[f"e{l}a"])
            x_in = A["x"] if l == 0 else A[f"p{l}"]
            dx = None if l == 0 else G[f"p{l}"]
            self._conv_bwd(S[f"e{l}a"], x_in, G[f"e{l}a"], B, H, W, dx)
            g = dx

    def adam(self, lr: float, b1=0.9, b2=0.999, eps=1e-8) -> None:
        self.t += 1
        qnn.qnn_adam(self.n_params, self.p, self.m, self.v, self.g, self.pb, lr, b1, b2, eps, self.t, self.stream)

    def train_step(self, q, idx_q, n, idx_n, target, idx_t, B, H, W, lr) -> None:
        """One optimisation step on B pairs (input q[idx_q], n[idx_n], target
        target[idx_t]). The loss stays on the device in self.loss."""
        self.pack(B, H, W, q, idx_q, n, idx_n, train=True)
        y = self.forward_packed(B, H, W)
        qnn.qnn_rel_l2(B, H, W, y, OUT_LD, target, idx_t, self.scale, self.grad["out"], OUT_CH, self.loss,
                       self.per_sample, self.lwork, self.stream)
        self.backward(B, H, W, self.grad["out"])
        self.adam(lr)

    def eval_error(self, q, idx_q, n, idx_n, target, idx_t, B, H, W):
        """Per-sample relative field errors |pred - target| / |target|."""
        self.pack(B, H, W, q, idx_q, n, idx_n)
        y = self.forward_packed(B, H, W, fused=True)
        qnn.qnn_rel_l2(B, H, W, y, OUT_LD, target, idx_t, self.scale, None, OUT_CH, self.loss, self.per_sample,
                       self.lwork, self.stream)
        return self.per_sample.cpu().numpy().copy()


# ---------------------------------------------------------------------------
# Training data: QLA runs generated by the library itself.
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Dataset:
    q: object            # device FP32 [runs * snaps][6][L][L]
    n: object            # device FP32 [runs][3][L][L]
    runs: int
    snaps: int
    L: int
    K: int
    seconds: float

    def pairs(self) -> np.ndarray:
        """(input index, index-profile index, target index) of every pair."""
        out = []
        for r in range(self.runs):
            for s in range(self.snaps - 1):
                out.append((r * self.snaps + s, r, r * self.snaps + s + 1))
        return np.asarray(out, dtype=np.int32)


def generate(runs: int, seed: int, L: int = 256, K: int = 256, snaps: int = 9, chunk: int = 128,
             device: str = "cuda:0", stream=None) -> Dataset:
    """QLA runs of the batched scattering family at L x L (objects, tensors,
    pulses drawn as in scenes.batch_instance_specs), with the state recorded
    every K steps (snaps snapshots per run)."""
    import torch

    dev = torch.device(device)
    stream = stream if stream is not None else torch.cuda.current_stream(dev)
    specs = scenes.batch_instance_specs(runs, seed=seed, sides=(L,))
    qall = torch.empty((runs * snaps, 6, L, L), dtype=torch.float32, device=dev)
    nall = torch.empty((runs, 3, L, L), dtype=torch.float32, device=dev)
    t0 = time.perf_counter()
    for c0 in range(0, runs, chunk):
        sub = specs[c0:c0 + chunk]
        scs = [scenes.scene_from_spec(sp, steps=K * (snaps - 1)) for sp in sub]
        batch = qla.Batch([s.n for s in scs], [s.q for s in scs], [s.delta for s in scs], "eq28", "phys",
                          device=device, stream=stream)
        for k, s in enumerate(scs):
            nall[c0 + k].copy_(batch.n[k].view(3, L, L))
        for sn in range(snaps):
            if sn:
                batch.step(K)
            for k in range(len(scs)):
                dst = qall[(c0 + k) * snaps + sn]
                qla.qla_fields_at(batch.ctx, k, dst.data_ptr(), 0, False)
        batch.close()
    torch.cuda.synchronize(dev)
    return Dataset(qall, nall, runs, snaps, L, K, time.perf_counter() - t0)


def train(net: UNet, data: Dataset, steps: int, batch: int = 16, lr: float = 1e-3, seed: int = 0,
          log_every: int = 100, log=None, guard_every: int = 500) -> List[Dict]:
    """Adam on random pairs of ``data`` with a cosine learning-rate decay.

    Every ``guard_every`` steps the batch loss is read back: if it is not
    finite or has jumped above 20 times the lowest loss seen at these
    reads, the parameters and Adam moments return to the last good read
    and the learning rate is halved from then on (a divergence guard)."""
    import torch

    rng = np.random.default_rng(seed)
    pairs = data.pairs()
    hist = []
    dev = net.device
    good = None
    best = math.inf
    scale = 1.0
    for it in range(steps):
        sel = pairs[rng.integers(0, len(pairs), batch)]
        idx = torch.as_tensor(sel.T.copy()).to(dev)
        rate = lr * scale * 0.5 * (1.0 + math.cos(math.pi * it / max(steps, 1)))
        net.train_step(data.q, idx[0], data.n, idx[1], data.q, idx[2], batch, data.L, data.L,
                       max(rate, lr * scale * 0.02))
        if guard_every and (it + 1) % guard_every == 0:
            loss = float(net.loss.item())
            if not math.isfinite(loss) or loss > 20.0 * best:
                if good is not None:
                    for dst, src in zip((net.p, net.m, net.v), good[:3]):
                        dst.copy_(src)
                    net.t = good[3]
                    qnn.qnn_to_bf16(net.n_params, net.p, net.pb, net.stream)
                scale *= 0.5
                rec = {"step": it, "loss": loss, "rolled_back": True, "lr_scale": scale}
                hist.append(rec)
                if log:
                    log(rec)
            else:
                best = min(best, loss)
                good = (net.p.clone(), net.m.clone(), net.v.clone(), net.t)
        if log_every and (it % log_every == 0 or it == steps - 1):
            rec = {"step": it, "loss": float(net.loss.item()), "lr": rate}
            hist.append(rec)
            if log:
                log(rec)
    return hist


def evaluate(net: UNet, data: Dataset, batch: int = 16) -> np.ndarray:
    """Relative field error of the network on every pair of ``data``."""
    import torch

    pairs = data.pairs()
    errs = []
    for c0 in range(0, len(pairs), batch):
        sel = pairs[c0:c0 + batch]
        idx = torch.as_tensor(sel.T.copy()).to(net.device)
        errs.append(net.eval_error(data.q, idx[0], data.n, idx[1], data.q, idx[2], len(sel), data.L, data.L))
    return np.concatenate(errs)


# ---------------------------------------------------------------------------
# Surrogate-accelerated sweep with QLA checks and fallback.
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class SweepResult:
    steps: int
    jumps: int
    unchecked: int       # jumps taken from the surrogate
    checks: int          # jumps also run by QLA (the QLA result is kept)
    rejected: int        # checks whose surrogate error exceeded the tolerance
    fell_back: bool
    seconds: float
    max_check_error: float
    max_check_energy: float
    windows: int = 0     # QLA correction windows run
    window_steps: int = 0
    energy_change: float = 0.0   # max over lattices of |E(end)/E(0) - 1| (Eq. (27))


def _shape(a) -> Tuple[int, ...]:
    return tuple(int(v) for v in a.shape)


def _export(batch, dst) -> None:
    for k in range(batch.count):
        qla.qla_fields_at(batch.ctx, k, dst[k].data_ptr(), 0, False)


def _stacked(ts):
    """ts as one [B][...] tensor: the tensor they are consecutive views of,
    if they are (no copy of a large batch), else a stacked copy."""
    import torch
    base = ts[0]._base
    if (base is not None and base.dim() == ts[0].dim() + 1 and base.shape[0] == len(ts) and base.is_contiguous()
            and all(x.data_ptr() == base[k].data_ptr() and x.shape == base.shape[1:] for k, x in enumerate(ts))):
        return base
    return torch.stack(ts)


def _energies(batch) -> np.ndarray:
    return np.array([d["energy"] for d in batch.diagnostics()])


def sweep(net: UNet, n_list: Sequence, q_list: Sequence, delta: float, total_steps: int, K: int = 256,
          window: int = 0, check_every: int = 4, tol: float = 1e-3, max_rejects: int = 1,
          device: str = "cuda:0", v_form: str = "printed", energy_tol: Optional[float] = None,
          out=None, progress=None) -> Tuple[SweepResult, Optional[List[np.ndarray]]]:
    """Advance lattices (all the same size, sides multiples of 16; numpy
    arrays or device tensors) by ``total_steps`` QLA steps, replacing runs of
    K steps by surrogate jumps.

    The first jump and then every ``check_every``-th jump is also run by
    plain QLA from the saved pre-jump state: the QLA result is kept, and if
    the surrogate's relative field error or relative energy error against it
    exceeds ``tol`` on any lattice the check counts as rejected; after
    ``max_rejects`` rejections the sweep falls back to plain QLA for the
    rest of the run. Other jumps take the surrogate's prediction
    (``check_every`` <= 0: no checks at all). ``window`` plain QLA steps
    follow each jump. A check measures the error of one jump from the
    current state; it does not bound the error earlier unchecked jumps have
    left in that state. ``energy_tol``: a check also fails when some
    lattice's energy (Eq. (27)) has moved from its initial value by more
    than this fraction -- a test for the energy-conserving skew potentials
    (``v_form="skew"``); the printed potentials change the energy by design.
    ``out``: a device tensor [B][6][H][W] that receives the final states
    instead of a host copy (None is then returned in their place).
    ``progress``: called with the step count after every jump and every
    chunk of at most 5000 plain steps."""
    import torch

    dev = torch.device(device)
    stream = net.stream
    B = len(n_list)
    _, H, W = _shape(n_list[0])
    batch = qla.Batch(list(n_list), list(q_list), [delta] * B, "eq28", "phys", device=device, stream=stream,
                      v_form=v_form)
    cur = torch.empty((B, 6, H, W), dtype=torch.float32, device=dev)
    pred = torch.empty_like(cur)
    ref = torch.empty_like(cur) if check_every > 0 else None
    n_dev = _stacked([t.view(3, H, W) for t in batch.n])
    rel = torch.empty(B, dtype=torch.float64, device=dev)
    en = torch.empty(B, dtype=torch.float64, device=dev)
    cmp_work = torch.empty(qnn.qnn_compare_work_doubles(B), dtype=torch.float64, device=dev)
    e0 = _energies(batch)

    jumps = unchecked = checks = rejected = windows = window_steps = 0
    max_err = max_en = 0.0
    fell_back = False
    t = 0
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    while t < total_steps:
        if fell_back or t + K > total_steps:
            while t < total_steps:
                k = min(5000, total_steps - t)
                batch.step(k)
                t += k
                if progress is not None:
                    torch.cuda.synchronize(dev)    # report steps done, not steps enqueued
                    progress(t)
            break
        _export(batch, cur)
        net.predict(cur, n_dev, pred)
        jumps += 1
        if check_every > 0 and (jumps == 1 or jumps % check_every == 0):
            checks += 1
            batch.step(K)                        # QLA from the saved pre-jump state
            _export(batch, ref)
            qnn.qnn_compare(B, 6 * H * W, pred, ref, rel, en, cmp_work, stream)
            r, e = rel.cpu().numpy(), en.cpu().numpy()
            max_err, max_en = max(max_err, float(r.max())), max(max_en, float(e.max()))
            bad = float(r.max()) > tol or float(e.max()) > tol
            if energy_tol is not None:
                bad = bad or float(np.abs(_energies(batch) / e0 - 1.0).max()) > energy_tol
            if bad:
                rejected += 1
                fell_back = rejected >= max_rejects
        else:
            unchecked += 1
            for k in range(B):
                qla.qla_load_at(batch.ctx, k, pred[k].data_ptr(), False)
        t += K
        if window and not fell_back and t < total_steps:
            w = min(window, total_steps - t)
            batch.step(w)
            t += w
            windows += 1
            window_steps += w
        if progress is not None:
            torch.cuda.synchronize(dev)
            progress(t)
    torch.cuda.synchronize(dev)
    secs = time.perf_counter() - t0
    change = float(np.abs(_energies(batch) / e0 - 1.0).max())
    if out is not None:
        _export(batch, out)
        torch.cuda.synchronize(dev)
        finals = None
    else:
        finals = batch.fields("Q")
    batch.close()
    res = SweepResult(total_steps, jumps, unchecked, checks, rejected, fell_back, secs, max_err, max_en, windows,
                      window_steps, change)
    return res, finals


def plain(n_list: Sequence, q_list: Sequence, delta: float, total_steps: int, device: str = "cuda:0",
          stream=None, v_form: str = "printed", out=None, progress=None) -> Tuple[float, Optional[List[np.ndarray]]]:
    """Plain QLA for the same lattices: (seconds, final states; None when
    ``out``, a device tensor [B][6][H][W], receives them). ``progress``:
    called with the step count after every chunk of at most 5000 steps."""
    import torch

    dev = torch.device(device)
    batch = qla.Batch(list(n_list), list(q_list), [delta] * len(n_list), "eq28", "phys", device=device,
                      stream=stream, v_form=v_form)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    done = 0
    while done < total_steps:
        k = min(5000, total_steps - done)
        batch.step(k)
        done += k
        if progress is not None:
            torch.cuda.synchronize(dev)
            progress(done)
    torch.cuda.synchronize(dev)
    secs = time.perf_counter() - t0
    if out is not None:
        _export(batch, out)
        torch.cuda.synchronize(dev)
        finals = None
    else:
        finals = batch.fields("Q")
    batch.close()
    return secs, finals
