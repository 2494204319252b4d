"""Pins of the oracle's skew-symmetric potential variant (no GPU).

The paper names a fully unitary potential as future work without giving
one. The variant here replaces V_X, V_Y (Eq. (21), (22)) by the exponential
of the antisymmetric part of their first-order generator. These tests tie
it to things other than its own code:

* per site it equals expm(b (G - G^T)/2), with G measured from the printed
  operator (itself pinned by the printed matrices);
* it conserves the energy of Eq. (27) exactly in an inhomogeneous medium;
* it keeps the TE and TM triples apart;
* in a smooth 1D dielectric slab it converges at second order to Maxwell's
  equations, solved independently here by a Fourier method of lines with
  RK4 -- while the printed potentials converge to something else (an
  O(1) discrepancy that does not shrink with delta).
"""
from __future__ import annotations

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import oracle as O
from paper_2301_13601_amd import scenes


def _site_matrices(n, delta, axis, frac, form):
    """The 6x6 matrix of V at every site: column c is V applied to the
    state with q_c = 1 everywhere (the potentials are site-local)."""
    ny, nx = n.shape[1:]
    M = np.empty((ny, nx, 6, 6))
    for c in range(6):
        e = np.zeros((6, ny, nx))
        e[c] = 1.0
        M[:, :, :, c] = np.moveaxis(O.potential(n, e, delta, axis, frac, "phys", form), 0, -1)
    return M


@pytest.mark.parametrize("axis", ["x", "y"])
def test_skew_potential_is_exp_of_antisymmetric_generator(axis):
    n = scenes.random_profile(12, 10, 5, 1.0, 3.5)
    delta = 0.4
    h = 1e-6
    # generator of the printed operator, by central differences in the angle
    G = (_site_matrices(n, delta, axis, h, "printed") - _site_matrices(n, delta, axis, -h, "printed")) / (2 * h)
    assert np.abs(G).max() > 1e-2          # the profile has real gradients
    S = _site_matrices(n, delta, axis, 1.0, "skew")
    worst = 0.0
    for j in range(n.shape[1]):
        for i in range(n.shape[2]):
            g = G[j, i]
            want = sla.expm(0.5 * (g - g.T))
            worst = max(worst, np.abs(S[j, i] - want).max())
            # orthogonal to rounding
            assert np.abs(S[j, i] @ S[j, i].T - np.eye(6)).max() < 1e-14
    assert worst < 1e-8, worst


@pytest.mark.parametrize("mode", ["eq23", "eq28"])
def test_skew_conserves_energy_in_inhomogeneous_medium(mode):
    n = scenes.random_profile(24, 20, 12, 1.0, 3.5)
    q = scenes.random_state(24, 20, 13)
    out = O.run(n, q, 0.3, 100, mode, "phys", v_form="skew")
    assert abs(O.energy(out) / O.energy(q) - 1) < 1e-12
    # the printed potentials do not (same scene)
    out_p = O.run(n, q, 0.3, 20, mode, "phys")
    assert abs(O.energy(out_p) / O.energy(q) - 1) > 1e-4


@pytest.mark.parametrize("pol,zero", [("Ez", (0, 1, 5)), ("Ey", (2, 3, 4))])
def test_skew_keeps_te_tm_blocks_apart(pol, zero):
    n = scenes.object_profile(64, 48, "ellipse", (12, 8), (1.5, 2.0, 3.0), 3.0)
    q = scenes.gaussian_pulse(64, 48, pol, x0=12, width=5)
    out = O.run(n, q, 0.3, 60, "eq28", "phys", v_form="skew")
    for c in zero:
        assert np.all(out[c] == 0.0), c


# ---------------------------------------------------------------------------
# Convergence to Maxwell's equations in a 1D slab.
# ---------------------------------------------------------------------------
# For propagation along x, E_z polarisation couples (q2, q4) = (n E_z, B_y),
# E_y polarisation couples (q1, q5) = (n E_y, B_z), with n the matching index
# component. Maxwell's equations (eps = n^2, mu = 1, c = 1) then read
#     a_t = s (1/n) d_x b,   b_t = s d_x(a / n)
# with (a, b, s) = (q2, q4, +1) for E_z and (q1, q5, -1) for E_y (the sign
# that makes the pulses of the scene generator move towards +x).

_LP, _T, _X0, _W = 51.2, 10.0, 8.0, 2.0


def _slab(X, a=12.0, b=20.0, w=2.0, n_in=3.0):
    h = 0.5 * (n_in - 1)
    return 1 + h * (np.tanh((X - a) / w) - np.tanh((X - b) / w))


def _maxwell_1d(N, n, a0, b0, s, T, dt=0.005):
    """Fourier method of lines on the periodic interval of length _LP,
    classical RK4 in time (time error ~1e-10 at this dt)."""
    k = 2 * np.pi * np.fft.rfftfreq(N, d=_LP / N)

    def D(f):
        return np.fft.irfft(1j * k * np.fft.rfft(f), n=N)

    def rhs(y):
        return np.array([s * D(y[1]) / n, s * D(y[0] / n)])

    y = np.array([a0, b0])
    for _ in range(int(round(T / dt))):
        k1 = rhs(y)
        k2 = rhs(y + 0.5 * dt * k1)
        k3 = rhs(y + 0.5 * dt * k2)
        k4 = rhs(y + dt * k3)
        y = y + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return y


_POL = {"Ez": (2, 4, 2, 1.0), "Ey": (1, 5, 1, -1.0)}   # a, b, index component, s


def _errors_vs_maxwell(pol, form, mode):
    ia, ib, ic, s = _POL[pol]
    Nr = 1024
    Xr = np.arange(Nr) * _LP / Nr
    qr = scenes.gaussian_pulse(Nr, 1, pol, x0=_X0 * Nr / _LP, width=_W * Nr / _LP)
    ref = _maxwell_1d(Nr, _slab(Xr), qr[ia, 0], qr[ib, 0], s, _T)
    errs = []
    for d in (0.2, 0.1, 0.05):
        N = int(round(_LP / d))
        X = np.arange(N) * d
        n = np.ones((3, 1, N))
        n[ic, 0] = _slab(X)
        q = scenes.gaussian_pulse(N, 1, pol, x0=_X0 / d, width=_W / d)
        out = O.run(n, q, d, int(round(_T / d ** 2)), mode, "phys", v_form=form)
        st = Nr // N
        errs.append(max(np.abs(out[ia, 0] - ref[0][::st]).max(), np.abs(out[ib, 0] - ref[1][::st]).max()))
    return errs


@pytest.mark.parametrize("pol", ["Ez", "Ey"])
@pytest.mark.parametrize("mode", ["eq23", "eq28"])
def test_skew_converges_to_maxwell_at_second_order(pol, mode):
    e = _errors_vs_maxwell(pol, "skew", mode)
    assert 3.5 < e[0] / e[1] < 4.6 and 3.5 < e[1] / e[2] < 4.6, e
    assert e[2] < 2e-2, e


@pytest.mark.parametrize("pol", ["Ez", "Ey"])
def test_printed_potentials_do_not_converge_to_maxwell(pol):
    """The finding the variant answers: with site-local collision angles
    the printed V leaves an O(1) difference from Maxwell in this slab."""
    e = _errors_vs_maxwell(pol, "printed", "eq28")
    assert min(e) > 0.5 and e[1] / e[2] < 1.2, e
