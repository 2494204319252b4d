"""Seeded synthetic inputs for the qubit lattice algorithm (QLA).

This module builds the two inputs of one scattering run and nothing else:

* a refractive-index profile ``n`` of shape ``(3, ny, nx)`` holding the
  diagonal tensor components (n_x, n_y, n_z) of a localized dielectric
  object in vacuum (paper Sec. 4, the object of Fig. 2 is described there
  only in words, so the shapes here are synthetic stand-ins), and
* an initial state ``q`` of shape ``(6, ny, nx)`` holding the Dyson-mapped
  field Q = (n_x E_x, n_y E_y, n_z E_z, B_x, B_y, B_z) of Eq. (15), here a
  1D Gaussian pulse travelling in +x (Sec. 4) or random states for tests.

It holds none of the method's arithmetic (no collision, streaming or
potential operator, no angle): both the HIP library and the FP64 oracle
consume these arrays, and the two share nothing else.

Layout convention for every array: component-major planes, then rows (y),
then columns (x), x fastest. Lattice cell (i, j) has coordinates x = i,
y = j in cell units; the lattice is periodic in both directions.

All generators are deterministic in their ``seed`` (numpy ``default_rng``).
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

# Pulse polarisations (Sec. 4.1 and 4.2).
EZ = "Ez"
EY = "Ey"

SHAPES = ("ellipse", "disk", "rectangle", "two_disk")


@dataclasses.dataclass
class Scene:
    """One scattering run: index profile, initial state and run parameters."""

    name: str
    n: np.ndarray          # (3, ny, nx) float64, n_x, n_y, n_z
    q: np.ndarray          # (6, ny, nx) float64, initial Q
    delta: float           # the paper's perturbation parameter
    steps: int
    pot_mode: str = "eq28"
    meta: Dict = dataclasses.field(default_factory=dict)

    @property
    def nx(self) -> int:
        return self.n.shape[2]

    @property
    def ny(self) -> int:
        return self.n.shape[1]

    def as_f32(self) -> Tuple[np.ndarray, np.ndarray]:
        """The FP32 arrays handed to the GPU library (and, widened back to
        FP64, to the oracle, so that both start from identical values)."""
        return (np.ascontiguousarray(self.n, dtype=np.float32),
                np.ascontiguousarray(self.q, dtype=np.float32))


# ----------------------------------------------------------------------------
# Object profiles.
# ----------------------------------------------------------------------------

def _grid(nx: int, ny: int, cx: float, cy: float) -> Tuple[np.ndarray, np.ndarray]:
    x = np.arange(nx, dtype=np.float64) - cx
    y = np.arange(ny, dtype=np.float64) - cy
    return np.meshgrid(x, y, indexing="xy")  # each (ny, nx)


def signed_distance(nx: int, ny: int, shape: str, size: Sequence[float],
                    center: Optional[Tuple[float, float]] = None) -> np.ndarray:
    """Approximate signed distance (cells) to the boundary of ``shape``,
    negative inside.

    ellipse:   size = (a, b) semi-axes along x and y; first-order distance
               (r - 1)/|grad r| of the implicit r = sqrt((x/a)^2 + (y/b)^2).
    disk:      size = (radius,).
    rectangle: size = (hx, hy) half-sides; max-norm box distance.
    two_disk:  size = (r1, r2, sep); disks centred at +-sep along y.
    """
    if center is None:
        center = (nx / 2.0, ny / 2.0)
    X, Y = _grid(nx, ny, *center)
    if shape == "ellipse":
        a, b = float(size[0]), float(size[1])
        r = np.sqrt((X / a) ** 2 + (Y / b) ** 2)
        gx = X / (a * a)
        gy = Y / (b * b)
        with np.errstate(divide="ignore", invalid="ignore"):
            grad = np.sqrt(gx * gx + gy * gy) / r
        grad = np.where(r > 0, grad, 1.0 / max(a, b))
        return (r - 1.0) / grad
    if shape == "disk":
        R = float(size[0])
        return np.sqrt(X * X + Y * Y) - R
    if shape == "rectangle":
        hx, hy = float(size[0]), float(size[1])
        return np.maximum(np.abs(X) - hx, np.abs(Y) - hy)
    if shape == "two_disk":
        r1, r2, sep = float(size[0]), float(size[1]), float(size[2])
        d1 = np.sqrt(X * X + (Y - sep) ** 2) - r1
        d2 = np.sqrt(X * X + (Y + sep) ** 2) - r2
        return np.minimum(d1, d2)
    raise ValueError(f"unknown shape {shape!r}")


def object_profile(nx: int, ny: int, shape: str, size: Sequence[float],
                   n_obj: Sequence[float], edge_width: float = 6.0,
                   center: Optional[Tuple[float, float]] = None,
                   n_vac: float = 1.0) -> np.ndarray:
    """Diagonal index tensor of a localized object in vacuum (Sec. 4):
    n_c = n_vac + (n_obj_c - n_vac) * (1 - tanh(s / w)) / 2, with s the
    signed distance to the object's boundary and w the tanh edge width."""
    s = signed_distance(nx, ny, shape, size, center)
    prof = 0.5 * (1.0 - np.tanh(s / float(edge_width)))
    n = np.empty((3, ny, nx), dtype=np.float64)
    for c in range(3):
        n[c] = n_vac + (float(n_obj[c]) - n_vac) * prof
    return n


def uniform_profile(nx: int, ny: int, n_c: Sequence[float]) -> np.ndarray:
    n = np.empty((3, ny, nx), dtype=np.float64)
    for c in range(3):
        n[c] = float(n_c[c])
    return n


def smooth_random_profile(nx: int, ny: int, seed: int, lo: float = 1.0,
                          hi: float = 3.0, modes: int = 3) -> np.ndarray:
    """A smooth periodic random index field in [lo, hi] (sum of a few
    low Fourier modes per component). Used by parity and pin tests."""
    rng = np.random.default_rng(seed)
    X, Y = _grid(nx, ny, 0.0, 0.0)
    n = np.empty((3, ny, nx), dtype=np.float64)
    for c in range(3):
        f = np.zeros((ny, nx))
        for _ in range(modes):
            kx = rng.integers(0, 3)
            ky = rng.integers(0, 3)
            ph = rng.uniform(0, 2 * np.pi)
            f += rng.uniform(0.5, 1.0) * np.cos(2 * np.pi * (kx * X / nx + ky * Y / ny) + ph)
        f -= f.min()
        if f.max() > 0:
            f /= f.max()
        n[c] = lo + (hi - lo) * f
    return n


# ----------------------------------------------------------------------------
# Initial states.
# ----------------------------------------------------------------------------

def gaussian_pulse(nx: int, ny: int, polarisation: str, x0: float, width: float,
                   amplitude: float = 1.0, axis: str = "x") -> np.ndarray:
    """A 1D Gaussian pulse g = A exp(-((s - s0)/w)^2), uniform across the
    other axis, set up to travel in the +axis direction in vacuum.

    The partner component follows from the curl equations of Eq. (16) for a
    wave f(x - t): for propagation along +x, E_z polarisation has
    B_y = -E_z (q4 = -q2) and E_y polarisation has B_z = +E_y (q5 = +q1).
    Along +y: E_z polarisation has B_x = +E_z (q3 = +q2) and E_x
    polarisation has B_z = -E_x (q5 = -q0)."""
    q = np.zeros((6, ny, nx), dtype=np.float64)
    if axis == "x":
        s = np.arange(nx, dtype=np.float64)
        g = amplitude * np.exp(-(((s - x0) / width) ** 2))
        g2 = np.broadcast_to(g[None, :], (ny, nx))
        if polarisation == EZ:
            q[2] = g2
            q[4] = -g2
        elif polarisation == EY:
            q[1] = g2
            q[5] = g2
        else:
            raise ValueError("x-travelling pulse: polarisation must be Ez or Ey")
    elif axis == "y":
        s = np.arange(ny, dtype=np.float64)
        g = amplitude * np.exp(-(((s - x0) / width) ** 2))
        g2 = np.broadcast_to(g[:, None], (ny, nx))
        if polarisation == EZ:
            q[2] = g2
            q[3] = g2
        elif polarisation == "Ex":
            q[0] = g2
            q[5] = -g2
        else:
            raise ValueError("y-travelling pulse: polarisation must be Ez or Ex")
    else:
        raise ValueError("axis must be 'x' or 'y'")
    return q


def random_state(nx: int, ny: int, seed: int, comps: Sequence[int] = range(6)) -> np.ndarray:
    """Standard-normal Q on the listed components, zero elsewhere."""
    rng = np.random.default_rng(seed)
    q = np.zeros((6, ny, nx), dtype=np.float64)
    for c in comps:
        q[c] = rng.standard_normal((ny, nx))
    return q


def random_profile(nx: int, ny: int, seed: int, lo: float = 1.0, hi: float = 3.0) -> np.ndarray:
    """Index drawn independently per site and component, U[lo, hi]: the
    roughest input the method accepts (large potential angles)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(3, ny, nx))


# ----------------------------------------------------------------------------
# The scattering workloads.
# ----------------------------------------------------------------------------

def config_single(seed: int = 1) -> Scene:
    """256 x 256 periodic lattice, delta = 0.3, 500 steps, Eq. (28) potentials;
    E_z pulse of width 20 cells starting at x0 = 48 moving in +x; centred
    elliptic object, semi-axes 30 (x) by 20 (y) cells, tanh edge width 6,
    n = (1.5, 2.0, 3.0) inside and 1 outside. (``seed`` is unused: the
    scene is fully specified.)"""
    N = 256
    n = object_profile(N, N, "ellipse", (30.0, 20.0), (1.5, 2.0, 3.0), 6.0)
    q = gaussian_pulse(N, N, EZ, x0=48.0, width=20.0)
    return Scene("single_256", n, q, delta=0.3, steps=500, pot_mode="eq28",
                 meta={"shape": "ellipse", "size": [30, 20], "n_obj": [1.5, 2.0, 3.0],
                       "edge_width": 6, "pulse": EZ, "width": 20, "x0": 48})


def config_scale(seed: int = 2, N: int = 4096, steps: int = 20000) -> Scene:
    """4096 x 4096 single instance, delta = 0.3, 20000 steps; E_z pulse of
    width 160 cells at x0 = N/4; centred cylinder (disk) of radius 400 cells,
    tanh edge width 6, with n_x, n_y, n_z drawn U[1.2, 3.0] from ``seed``."""
    rng = np.random.default_rng(seed)
    n_obj = rng.uniform(1.2, 3.0, size=3)
    radius = 400.0 * N / 4096.0
    n = object_profile(N, N, "disk", (radius,), n_obj, 6.0)
    q = gaussian_pulse(N, N, EZ, x0=N / 4.0, width=160.0 * N / 4096.0)
    return Scene(f"cylinder_{N}", n, q, delta=0.3, steps=steps, pot_mode="eq28",
                 meta={"seed": seed, "shape": "disk", "radius": radius,
                       "n_obj": [float(v) for v in n_obj], "edge_width": 6,
                       "pulse": EZ, "width": 160.0 * N / 4096.0, "x0": N / 4.0})


BATCH_SIDES = (512, 768, 1024, 1536, 2048)


def batch_instance_specs(count: int = 64, seed: int = 3,
                         sides: Sequence[int] = BATCH_SIDES) -> List[Dict]:
    """Per-instance draws for a batch of scattering runs of uneven size:
    side L ~ U{sides}, n_c ~ U[1.1, 3.5], shape ~ U{ellipse, rectangle,
    two-disk} with sizes scaled to L, polarisation ~ U{E_y, E_z}, pulse
    width 20 placed 50 cells left of the object, delta = 0.3."""
    rng = np.random.default_rng(seed)
    specs = []
    for k in range(count):
        L = int(rng.choice(np.asarray(sides)))
        n_obj = rng.uniform(1.1, 3.5, size=3)
        shape = ("ellipse", "rectangle", "two_disk")[int(rng.integers(0, 3))]
        if shape in ("ellipse", "rectangle"):
            size = tuple(rng.uniform(L / 16.0, L / 8.0, size=2))
            half_x = size[0]
        else:
            r = rng.uniform(L / 32.0, L / 16.0, size=2)
            size = (r[0], r[1], L / 8.0)
            half_x = max(r)
        pol = (EY, EZ)[int(rng.integers(0, 2))]
        specs.append({"index": k, "L": L, "n_obj": [float(v) for v in n_obj],
                      "shape": shape, "size": [float(v) for v in size],
                      "polarisation": pol, "width": 20.0,
                      "x0": float(L / 2.0 - half_x - 50.0), "delta": 0.3})
    return specs


def scene_from_spec(spec: Dict, steps: int = 5000) -> Scene:
    L = int(spec["L"])
    n = object_profile(L, L, spec["shape"], spec["size"], spec["n_obj"], 6.0)
    q = gaussian_pulse(L, L, spec["polarisation"], x0=spec["x0"], width=spec["width"])
    return Scene(f"batch_{spec['index']}_{L}", n, q, delta=float(spec["delta"]),
                 steps=steps, pot_mode="eq28", meta=dict(spec))
