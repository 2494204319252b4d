"""Dense brute-force form of the QLA step on tiny lattices (test helper).

Builds every operator of Sec. 3 of arXiv:2301.13601 as an explicit
(6 N) x (6 N) matrix over the whole lattice, N = nx * ny, directly from the
matrices and printed products in ``tests/golden/operators.txt``, and
multiplies them in the printed order. It is a second, structurally
different construction of the same step that the oracle computes pass by
pass: a transposed matrix, a wrong component, a misordered factor or a
shift in the wrong direction in either one shows up as a mismatch.

State vector index: (c * ny + y) * nx + x.
Streaming reading: S^{+x}_{ab} sets q_a(x, y) to the old q_a(x + 1, y)
(and S^{-x} to the old value at x - 1), periodic; likewise along y.
"""
from __future__ import annotations

import os
import re
from typing import Dict, List, Tuple

import numpy as np
import scipy.sparse as sp

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "operators.txt")


def load_golden(path: str = GOLDEN) -> Tuple[Dict[str, List[List[str]]], Dict[str, List[str]]]:
    matrices: Dict[str, List[List[str]]] = {}
    sequences: Dict[str, List[str]] = {}
    cur = None
    with open(path) as f:
        for raw in f:
            line = raw.split("#", 1)[0].strip()
            if not line:
                continue
            if line.startswith("matrix "):
                cur = line.split()[1]
                matrices[cur] = []
            elif line == "end":
                assert len(matrices[cur]) == 6, cur
                cur = None
            elif line.startswith("sequence "):
                name, rhs = line[len("sequence "):].split("=", 1)
                sequences[name.strip()] = rhs.split()
            else:
                row = line.split()
                assert cur is not None and len(row) == 6, line
                matrices[cur].append(row)
    return matrices, sequences


def angles(n: np.ndarray, delta: float, kappa: float):
    """theta_k = delta / (4 n_k), Eq. (24) (k = 0, 1, 2 -> n_x, n_y, n_z);
    beta per Eq. (25) with the periodic central difference in cells times
    kappa. Returns dicts of (ny, nx) arrays."""
    th = {k: delta / (4.0 * n[k]) for k in range(3)}

    def dx(f):
        return 0.5 * (np.roll(f, -1, axis=1) - np.roll(f, 1, axis=1))

    def dy(f):
        return 0.5 * (np.roll(f, -1, axis=0) - np.roll(f, 1, axis=0))

    be = {0: kappa * dx(n[1]) / n[1] ** 2,
          1: kappa * dy(n[0]) / n[0] ** 2,
          2: kappa * dx(n[2]) / n[2] ** 2,
          3: kappa * dy(n[2]) / n[2] ** 2}
    return th, be


_SYM = re.compile(r"^(-?)(cb|sb|c|s)(\d)$")


def _entry(tok: str, th, be, frac: float, nsites: int) -> np.ndarray:
    if tok in ("0", "1"):
        return np.full(nsites, float(tok))
    m = _SYM.match(tok)
    assert m, tok
    neg, kind, k = m.group(1), m.group(2), int(m.group(3))
    if kind in ("c", "s"):
        ang = th[k].ravel()
    else:
        ang = frac * be[k].ravel()
    val = np.cos(ang) if kind in ("c", "cb") else np.sin(ang)
    return -val if neg else val


def site_matrix(sym: List[List[str]], th, be, nx: int, ny: int, frac: float = 1.0,
                adjoint: bool = False) -> sp.csr_matrix:
    N = nx * ny
    rows, cols, vals = [], [], []
    idx = np.arange(N)
    for i in range(6):
        for j in range(6):
            v = _entry(sym[i][j], th, be, frac, N)
            if not np.any(v):
                continue
            r, c = (j, i) if adjoint else (i, j)
            rows.append(r * N + idx)
            cols.append(c * N + idx)
            vals.append(v)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(6 * N, 6 * N))


def stream_matrix(comps: Tuple[int, int], sign: int, axis: str, nx: int, ny: int) -> sp.csr_matrix:
    N = nx * ny
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    dst = (Y * nx + X).ravel()
    if axis == "x":
        src = (Y * nx + (X + sign) % nx).ravel()
    else:
        src = (((Y + sign) % ny) * nx + X).ravel()
    rows, cols = [], []
    for c in range(6):
        rows.append(c * N + dst)
        cols.append(c * N + (src if c in comps else dst))
    r = np.concatenate(rows)
    return sp.csr_matrix((np.ones(r.size), (r, np.concatenate(cols))), shape=(6 * N, 6 * N))


_STREAM = re.compile(r"^S([+-])([xy])(\d)(\d)$")


def build_operator(name: str, n: np.ndarray, delta: float, kappa: float,
                   golden=None) -> sp.csr_matrix:
    """The (6N x 6N) matrix of a matrix or sequence named in the golden file."""
    matrices, sequences = golden if golden is not None else load_golden()
    ny, nx = n.shape[1:]
    th, be = angles(n, delta, kappa)

    def token(tok: str) -> sp.csr_matrix:
        m = _STREAM.match(tok)
        if m:
            sign = 1 if m.group(1) == "+" else -1
            return stream_matrix((int(m.group(3)), int(m.group(4))), sign, m.group(2), nx, ny)
        adjoint = tok.endswith("^")
        half = tok.endswith("'")
        base = tok.rstrip("^'")
        if base in matrices:
            return site_matrix(matrices[base], th, be, nx, ny, 0.5 if half else 1.0, adjoint)
        if base in sequences:
            return product(sequences[base])
        raise KeyError(tok)

    def product(tokens: List[str]) -> sp.csr_matrix:
        M = sp.identity(6 * nx * ny, format="csr")
        for tok in tokens:          # left to right: M = M @ factor
            M = M @ token(tok)
        return M.tocsr()

    return token(name)


def apply(M: sp.csr_matrix, q: np.ndarray) -> np.ndarray:
    return (M @ q.reshape(-1)).reshape(q.shape)
