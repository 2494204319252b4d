"""Pins of the oracle's diagnostics to closed forms.

The diagnostics of the paper are the energy of Eq. (27), the divergence of
B (Sec. 4.1, whose smallness the paper reports for the E_z runs) and the
divergence of D (Sec. 4.2, E_y runs), with E and B recovered from Q by
Eq. (15). The oracle computes them with periodic central differences in
cells, D f(i) = (f(i+1) - f(i-1)) / 2, and D_c = eps_c E_c = n_c q_c.

Every check here uses lattice fields whose sums and differences have exact
trigonometric closed forms:

* on an N-point periodic lattice, the mean of sin^2(2 pi m i / N) is 1/2
  whenever 2m is not a multiple of N, and mixed products average to 0;
* the central difference of sin(a i) is sin(a) cos(a i), exactly.

The last test plants the slips a reading of the formulas could make (axes
swapped, a sign flipped, the factor n dropped, the wrong normalisation) in
copies of the oracle's functions and shows that each one fails a check.
"""
import math

import numpy as np

from oracle import oracle as O

NX, NY = 48, 40          # unequal, so a wrong normalisation or a swapped axis shows


def _grid():
    x = np.arange(NX, dtype=np.float64)[None, :]
    y = np.arange(NY, dtype=np.float64)[:, None]
    return np.broadcast_to(x, (NY, NX)), np.broadcast_to(y, (NY, NX))


def _state(**planes):
    q = np.zeros((6, NY, NX))
    for k, v in planes.items():
        q[int(k[1:])] = v
    return q


# ---------------------------------------------------------------------------
# The checks, each a function of the diagnostic it judges.
# ---------------------------------------------------------------------------

def check_energy(energy) -> bool:
    """Eq. (27): lattice mean of Q.Q. The state below has mean square
    1 + 4/2 + 9/2 + 0.25 + 1/2 + 2.25 = 10.5."""
    X, Y = _grid()
    q = _state(q0=np.ones((NY, NX)),
               q1=2.0 * np.sin(2 * math.pi * 3 * X / NX),
               q2=3.0 * np.cos(2 * math.pi * 2 * Y / NY),
               q3=0.5 * np.ones((NY, NX)),
               q4=np.sin(2 * math.pi * (X / NX + Y / NY)),
               q5=-1.5 * np.ones((NY, NX)))
    return abs(energy(q) - 10.5) < 1e-13


def _div_b_case():
    X, Y = _grid()
    a, b = 2 * math.pi * 2 / NX, 2 * math.pi * 3 / NY
    rng = np.random.default_rng(5)
    q = rng.standard_normal((6, NY, NX))        # q0, q1, q2 must not enter div B
    q[3] = 1.5 * np.sin(a * X)                  # B_x varies along x only
    q[4] = 0.75 * np.sin(b * Y)                 # B_y varies along y only
    q[5] = 0.4 * np.cos(2 * math.pi * (X / NX - 2 * Y / NY))   # B_z: no d/dz in 2D
    want = 1.5 * math.sin(a) * np.cos(a * X) + 0.75 * math.sin(b) * np.cos(b * Y)
    return q, want


def check_div_b(div_b) -> bool:
    """div B = D_x B_x + D_y B_y with B_x = 1.5 sin(a x), B_y = 0.75 sin(b y):
    exactly 1.5 sin(a) cos(a x) + 0.75 sin(b) cos(b y)."""
    q, want = _div_b_case()
    return np.abs(div_b(q) - want).max() < 1e-14


def _div_d_case():
    X, Y = _grid()
    n = np.empty((3, NY, NX))
    n[0] = 2.0 + 0.5 * np.sin(2 * math.pi * X / NX)       # n_x varies along x
    n[1] = 1.5 + 0.3 * np.cos(2 * math.pi * Y / NY)       # n_y varies along y
    n[2] = np.random.default_rng(6).uniform(1.0, 3.0, (NY, NX))
    a, b = 2 * math.pi * 2 / NX, 2 * math.pi * 2 / NY
    rng = np.random.default_rng(7)
    q = rng.standard_normal((6, NY, NX))        # B and q2 must not enter div D
    q[0] = np.sin(a * X) / n[0]                 # D_x = n_x q0 = sin(a x)
    q[1] = 2.0 * np.sin(b * Y) / n[1]           # D_y = n_y q1 = 2 sin(b y)
    want = math.sin(a) * np.cos(a * X) + 2.0 * math.sin(b) * np.cos(b * Y)
    return q, n, want


def check_div_d(div_d) -> bool:
    """div D with D_c = n_c q_c (Eq. (15): q_c = n_c E_c, D_c = n_c^2 E_c),
    D_x = sin(a x), D_y = 2 sin(b y): exactly sin(a) cos(a x) + 2 sin(b) cos(b y)."""
    q, n, want = _div_d_case()
    return np.abs(div_d(q, n) - want).max() < 1e-13


def check_fields(fields) -> bool:
    """Eq. (15): E_c = q_c / n_c, B = (q3, q4, q5) unchanged."""
    rng = np.random.default_rng(8)
    n = rng.uniform(1.0, 3.0, (3, NY, NX))
    E = rng.standard_normal((3, NY, NX))
    B = rng.standard_normal((3, NY, NX))
    q = np.concatenate([n * E, B])
    out = fields(q, n)
    return (np.abs(out[:3] - E).max() <= 1e-15 * np.abs(E).max() * 4
            and np.array_equal(out[3:], B))


# ---------------------------------------------------------------------------
# The oracle passes every check.
# ---------------------------------------------------------------------------

def test_energy_is_the_lattice_mean_of_q_dot_q():
    assert check_energy(O.energy)


def test_div_b_closed_form():
    assert check_div_b(O.div_b)


def test_div_d_closed_form():
    assert check_div_d(O.div_d)


def test_fields_recover_e_and_b():
    assert check_fields(O.fields)


def test_diagnostics_closed_forms():
    """Every reported value of oracle.diagnostics on states whose maxima and
    sums are known: maxima sit at sites where every sine is 1 (or every
    cosine of a divergence is 1), sums follow from the mean-square rule."""
    a, b = 2 * math.pi * 2 / NX, 2 * math.pi * 2 / NY   # sin(a x) = 1 at x = 6, sin(b y) = 1 at y = 5
    X, Y = _grid()
    # B: B_x = 1.5 sin(a x), B_y = 0.75 sin(b y), B_z = 0.4
    q, n, wdd = _div_d_case()
    q[2] = 0.5 / n[2]                           # D_z = 0.5
    q[3] = 1.5 * np.sin(a * X)
    q[4] = 0.75 * np.sin(b * Y)
    q[5] = 0.4
    d = O.diagnostics(q, n)
    sites = NX * NY
    # the energy has its own closed-form pin above; here it is the same function
    assert d["energy"] == O.energy(q)
    assert abs(d["divB_max"] - (1.5 * math.sin(a) + 0.75 * math.sin(b))) < 1e-14
    assert abs(d["divB_l2"] - math.sqrt(sites * (1.5 ** 2 * math.sin(a) ** 2 / 2
                                                 + 0.75 ** 2 * math.sin(b) ** 2 / 2))) < 1e-12
    assert abs(d["B_max"] - math.sqrt(1.5 ** 2 + 0.75 ** 2 + 0.4 ** 2)) < 1e-14
    assert abs(d["B_l2"] - math.sqrt(sites * (1.5 ** 2 / 2 + 0.75 ** 2 / 2 + 0.4 ** 2))) < 1e-11
    assert abs(d["divD_max"] - (math.sin(a) + 2.0 * math.sin(b))) < 1e-13
    assert abs(d["divD_l2"] - math.sqrt(sites * (math.sin(a) ** 2 / 2 + 4 * math.sin(b) ** 2 / 2))) < 1e-11
    assert abs(d["D_max"] - math.sqrt(1.0 + 4.0 + 0.25)) < 1e-14


def test_energy_pin_of_a_step_state_uses_eq27_scale():
    # a unit plane wave in one component: mean square 1/2 whatever the lattice
    X, _ = _grid()
    q = _state(q2=np.cos(2 * math.pi * 5 * X / NX))
    assert abs(O.energy(q) - 0.5) < 1e-15


# ---------------------------------------------------------------------------
# Planted slips fail the checks.
# ---------------------------------------------------------------------------

def _dx(f):
    return 0.5 * (np.roll(f, -1, axis=-1) - np.roll(f, 1, axis=-1))


def _dy(f):
    return 0.5 * (np.roll(f, -1, axis=-2) - np.roll(f, 1, axis=-2))


def test_planted_slips_fail_the_checks():
    slips_div_b = {
        "axes swapped": lambda q: _dy(q[3]) + _dx(q[4]),
        "sign of one term": lambda q: _dx(q[3]) - _dy(q[4]),
        "one-sided difference": lambda q: (np.roll(q[3], -1, -1) - q[3]) + (np.roll(q[4], -1, -2) - q[4]),
        "missing 1/2": lambda q: 2 * (_dx(q[3]) + _dy(q[4])),
        "wrong components": lambda q: _dx(q[4]) + _dy(q[5]),
    }
    for name, fn in slips_div_b.items():
        assert not check_div_b(fn), name
    slips_div_d = {
        "on q, not n q": lambda q, n: _dx(q[0]) + _dy(q[1]),
        "on n^2 q": lambda q, n: _dx(n[0] ** 2 * q[0]) + _dy(n[1] ** 2 * q[1]),
        "index planes swapped": lambda q, n: _dx(n[1] * q[0]) + _dy(n[0] * q[1]),
        "axes swapped": lambda q, n: _dy(n[0] * q[0]) + _dx(n[1] * q[1]),
    }
    for name, fn in slips_div_d.items():
        assert not check_div_d(fn), name
    slips_energy = {
        "1/Nx^2": lambda q: float(np.sum(q * q) / (q.shape[2] ** 2)),
        "1/Ny^2": lambda q: float(np.sum(q * q) / (q.shape[1] ** 2)),
        "mean over components too": lambda q: float(np.mean(q * q)),
        "B left out": lambda q: float(np.sum(q[:3] * q[:3]) / (q.shape[1] * q.shape[2])),
    }
    for name, fn in slips_energy.items():
        assert not check_energy(fn), name
    slips_fields = {
        "divided by n^2": lambda q, n: np.concatenate([q[:3] / n ** 2, q[3:]]),
        "times n": lambda q, n: np.concatenate([q[:3] * n, q[3:]]),
        "index planes rotated": lambda q, n: np.concatenate([q[:3] / np.roll(n, 1, axis=0), q[3:]]),
    }
    for name, fn in slips_fields.items():
        assert not check_fields(fn), name
