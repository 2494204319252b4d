"""Python face of the FP64 QLA oracle (arXiv:2301.13601).

TEST INFRASTRUCTURE. Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import this module. It loads the plain C
oracle in ``qla_oracle.c`` (compiled with gcc; OpenMP when available) and
adds the diagnostics of the paper written as plain numpy definitions. It
imports nothing from the HIP library's package.

Arrays: ``n`` is (3, ny, nx) = (n_x, n_y, n_z); ``q`` is (6, ny, nx) =
Q of Eq. (15); x is the last (fastest) axis; the lattice is periodic.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qla_oracle.c")
_LIB = os.path.join(_HERE, "libqla_oracle.so")

POT_MODES = {"eq23": 0, "eq28": 1}
BETA_SCALES = {"phys": 0, "lattice": 1, "off": 2}
V_FORMS = {"printed": 0, "skew": 1}

_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle into ``oracle/libqla_oracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.qla_oracle_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                       ctypes.c_int, dp, dp, ctypes.c_int64, ctypes.c_int]
        lib.qla_oracle_run.restype = ctypes.c_int
        lib.qla_oracle_run_form.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                            ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_int64,
                                            ctypes.c_int]
        lib.qla_oracle_run_form.restype = ctypes.c_int
        lib.qla_oracle_potential.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                             ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, dp]
        lib.qla_oracle_potential.restype = ctypes.c_int
        lib.qla_oracle_angles.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                          dp, dp, dp]
        lib.qla_oracle_angles.restype = ctypes.c_int
        lib.qla_oracle_threads.argtypes = [ctypes.c_int]
        lib.qla_oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def threads(nthreads: int = 0) -> int:
    """Threads the oracle's parallel loops use (``nthreads`` <= 0: default)."""
    return int(_load().qla_oracle_threads(int(nthreads)))


def run(n: np.ndarray, q: np.ndarray, delta: float, steps: int, pot_mode: str = "eq28",
        beta_scale: str = "phys", nthreads: int = 0, v_form: str = "printed") -> np.ndarray:
    """Return Q after ``steps`` full QLA steps (Eq. (23) or Eq. (28)),
    computed in FP64, with the potentials of Eq. (21)/(22) as printed
    (``v_form="printed"``) or their skew-symmetric variant (``"skew"``).
    The inputs are not modified."""
    n64 = np.ascontiguousarray(n, dtype=np.float64)
    q64 = np.array(q, dtype=np.float64, order="C", copy=True)
    if n64.ndim != 3 or n64.shape[0] != 3 or q64.shape != (6,) + n64.shape[1:]:
        raise ValueError("expected n of shape (3, ny, nx) and q of shape (6, ny, nx)")
    ny, nx = n64.shape[1:]
    rc = _load().qla_oracle_run_form(int(nx), int(ny), float(delta), POT_MODES[pot_mode],
                                     BETA_SCALES[beta_scale], V_FORMS[v_form], _dptr(n64),
                                     _dptr(q64), int(steps), int(nthreads))
    if rc != 0:
        raise ValueError(f"oracle rejected its arguments (status {rc})")
    return q64


def potential(n: np.ndarray, q: np.ndarray, delta: float, axis: str, frac: float = 1.0,
              beta_scale: str = "phys", v_form: str = "printed") -> np.ndarray:
    """V_X (``axis="x"``, Eq. (21)) or V_Y (``"y"``, Eq. (22)) alone, with
    the angles of Eq. (25) scaled by ``frac``, applied to a copy of q."""
    n64 = np.ascontiguousarray(n, dtype=np.float64)
    q64 = np.array(q, dtype=np.float64, order="C", copy=True)
    ny, nx = n64.shape[1:]
    rc = _load().qla_oracle_potential(int(nx), int(ny), float(delta), BETA_SCALES[beta_scale],
                                      V_FORMS[v_form], {"x": 0, "y": 1}[axis], float(frac),
                                      _dptr(n64), _dptr(q64))
    if rc != 0:
        raise ValueError(f"oracle rejected its arguments (status {rc})")
    return q64


def angles(n: np.ndarray, delta: float, beta_scale: str = "phys"):
    """(theta, beta) as the oracle computes them: theta (3, ny, nx) per
    Eq. (24); beta (4, ny, nx) per Eq. (25)."""
    n64 = np.ascontiguousarray(n, dtype=np.float64)
    ny, nx = n64.shape[1:]
    theta = np.empty((3, ny, nx))
    beta = np.empty((4, ny, nx))
    rc = _load().qla_oracle_angles(int(nx), int(ny), float(delta), BETA_SCALES[beta_scale],
                                   _dptr(n64), _dptr(theta), _dptr(beta))
    if rc != 0:
        raise ValueError(f"oracle rejected its arguments (status {rc})")
    return theta, beta


# ----------------------------------------------------------------------------
# Diagnostics (plain definitions, FP64).
# ----------------------------------------------------------------------------

def energy(q: np.ndarray) -> float:
    """Eq. (27): (1/L^2) * integral of Q.Q, i.e. the lattice mean of
    sum_c q_c^2."""
    q64 = np.asarray(q, dtype=np.float64)
    return float(np.sum(q64 * q64) / (q64.shape[1] * q64.shape[2]))


def _dx(f: np.ndarray) -> np.ndarray:
    return 0.5 * (np.roll(f, -1, axis=-1) - np.roll(f, 1, axis=-1))


def _dy(f: np.ndarray) -> np.ndarray:
    return 0.5 * (np.roll(f, -1, axis=-2) - np.roll(f, 1, axis=-2))


def div_b(q: np.ndarray) -> np.ndarray:
    """div B = d_x B_x + d_y B_y in cell units (periodic central differences);
    B = (q3, q4, q5) with mu_0 = 1 (Eq. (15)); the fields are 2D so d_z = 0."""
    q64 = np.asarray(q, dtype=np.float64)
    return _dx(q64[3]) + _dy(q64[4])


def div_d(q: np.ndarray, n: np.ndarray) -> np.ndarray:
    """div D with D_c = eps_c E_c = n_c^2 E_c = n_c q_c (c = x, y)."""
    q64 = np.asarray(q, dtype=np.float64)
    n64 = np.asarray(n, dtype=np.float64)
    return _dx(n64[0] * q64[0]) + _dy(n64[1] * q64[1])


def fields(q: np.ndarray, n: np.ndarray) -> np.ndarray:
    """(E, B) from Q: E_c = q_c / n_c (Eq. (15)), B = (q3, q4, q5)."""
    q64 = np.asarray(q, dtype=np.float64)
    n64 = np.asarray(n, dtype=np.float64)
    out = q64.copy()
    out[:3] = q64[:3] / n64
    return out


def diagnostics(q: np.ndarray, n: np.ndarray) -> Dict[str, float]:
    """Energy, |div B| and |div D| (max and L2) with the field magnitudes they
    are reported against."""
    q64 = np.asarray(q, dtype=np.float64)
    n64 = np.asarray(n, dtype=np.float64)
    db = div_b(q64)
    dd = div_d(q64, n64)
    bmag = np.sqrt(q64[3] ** 2 + q64[4] ** 2 + q64[5] ** 2)
    d = n64 * q64[:3]
    dmag = np.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
    return {
        "energy": energy(q64),
        "divB_max": float(np.max(np.abs(db))),
        "divB_l2": float(np.sqrt(np.sum(db * db))),
        "B_max": float(np.max(bmag)),
        "B_l2": float(np.sqrt(np.sum(bmag * bmag))),
        "divD_max": float(np.max(np.abs(dd))),
        "divD_l2": float(np.sqrt(np.sum(dd * dd))),
        "D_max": float(np.max(dmag)),
    }
