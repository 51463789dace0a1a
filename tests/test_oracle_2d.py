"""Pins of the two-dimensional oracle (d = 2, the paper's 2D example) against what the
mathematics fixes: brute-force bilinear deposit and gather with minimum-image distances,
mass conservation of the deposit, exact spectral derivatives of Fourier modes, exact decay
of a Fourier mode of m under the implicit solve, the closed-form particle mass for a uniform
w, the ECM decay for uniform m, and the Wiener increment statistics of the push."""
import math

import numpy as np
import pytest

from oracle import pic, spectral
from oracle import step as S


def _min_image(d, L):
    return d - L * np.round(d / L)


def test_deposit_and_gather_brute_force():
    N, L = 4, 1.0
    h = L / N
    rng = np.random.default_rng(0)
    X = rng.random((7, 2))
    a = rng.random(7) + 0.1
    u = pic.deposit(X, a, N, L)
    assert u.shape == (N, N)
    ref = np.zeros((N, N))
    f = rng.random((N, N))
    g_ref = np.zeros(7)
    for q1 in range(N):
        for q2 in range(N):
            d1 = np.abs(_min_image(X[:, 0] - q1 * h, L)) / h
            d2 = np.abs(_min_image(X[:, 1] - q2 * h, L)) / h
            K = np.maximum(1 - d1, 0) * np.maximum(1 - d2, 0)
            ref[q1, q2] = np.sum(a * K) / h ** 2
            g_ref += K * f[q1, q2]
    np.testing.assert_allclose(u, ref, rtol=1e-13)
    np.testing.assert_allclose(pic.gather([f], X, N, L)[0], g_ref, rtol=1e-13)
    assert math.isclose(h * h * u.sum(), a.sum(), rel_tol=1e-13)


def test_gradient_of_fourier_modes():
    N, L = 16, 2.0
    x = np.arange(N) * (L / N)
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    for q in [(1, 0), (2, -3), (0, 5), (7, 1)]:
        ph = 2 * np.pi * (q[0] * X1 + q[1] * X2) / L
        g = spectral.gradient(np.cos(ph), L)
        assert len(g) == 2
        for j in range(2):
            np.testing.assert_allclose(g[j], -(2 * np.pi * q[j] / L) * np.sin(ph), atol=1e-12)


def _state(N, P, L, rng, m=None, v=None, w=None):
    X = rng.random((P, 2)) * L
    a = np.full(P, 1.0 / max(P, 1))
    one = np.ones((N, N))
    return S.State(X, a, one.copy() if v is None else v, np.zeros((N, N)) if m is None else m,
                   one.copy() if w is None else w, 0)


def test_fourier_mode_of_m_decays_exactly():
    N, L, dt = 16, 1.0, 1e-2
    x = np.arange(N) * (L / N)
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    q = (2, 3)
    m0 = np.cos(2 * np.pi * (q[0] * X1 + q[1] * X2) / L)
    st = _state(N, 0, L, np.random.default_rng(1), m=m0)
    prm = S.Params(N=N, dt=dt, L=L, D_m=0.3, beta=0.7)
    out = S.run(st, prm, 5)
    k2 = (2 * np.pi / L) ** 2 * (q[0] ** 2 + q[1] ** 2)
    np.testing.assert_allclose(out.m, m0 * (1 + dt * (0.7 + 0.3 * k2)) ** -5, atol=1e-13)


def test_mass_for_uniform_w_and_ecm_decay():
    N, L, dt, n = 8, 1.0, 1e-2, 7
    w0 = np.full((N, N), 0.6)
    m0 = np.full((N, N), 0.4)
    st = _state(N, 50, L, np.random.default_rng(2), m=m0, w=w0.copy())
    prm = S.Params(N=N, dt=dt, L=L, freeze_w=True, freeze_m=True, alpha=3.0)
    out = S.run(st, prm, n)
    rho = 2 * 0.6 / 1.6
    np.testing.assert_allclose(out.a, st.a * np.exp(n * dt * (rho - 1)), rtol=1e-13)
    np.testing.assert_allclose(out.v, np.exp(-3.0 * dt * 0.4 * n), rtol=1e-13)


def test_wiener_increments():
    N, L, dt, Du = 8, 1.0, 1e-3, 0.05
    P = 20000
    st = _state(N, P, L, np.random.default_rng(3))
    st.X[:] = 0.5
    prm = S.Params(N=N, dt=dt, L=L, D_u=Du, chi=0.0, seed=4)
    out = S.step(st, prm)
    dX = out.X - 0.5
    assert out.X.shape == (P, 2)
    sd = math.sqrt(2 * Du * dt)
    assert abs(dX.mean()) < 4 * sd / math.sqrt(2 * P)
    assert dX.var() == pytest.approx(sd * sd, rel=0.03)
    assert abs(np.corrcoef(dX[:, 0], dX[:, 1])[0, 1]) < 0.03


def test_two_and_three_dimensional_multipliers_agree_on_planes():
    """The d = 3 multiplier restricted to q3 = 0 is the d = 2 one."""
    N, L, dt = 8, 1.0, 0.1
    m3 = spectral.implicit_multiplier(N, L, dt, 0.2, 0.5, d=3)[:, :, 0]
    m2 = spectral.implicit_multiplier(N, L, dt, 0.2, 0.5, d=2)
    np.testing.assert_array_equal(m2, m3)
    a3 = spectral.aliased_multiplier(N, L, dt, 0.2, 0.5, d=3)
    a2 = spectral.aliased_multiplier(N, L, dt, 0.2, 0.5, d=2)
    # a3 = e s(q1) s(q2) s(q3) and a2 = e s(q1) s(q2): the q3 = 0 plane is a2 times s(0)
    np.testing.assert_allclose(a3[:, :, 0], a2 * (a3[0, 0, 0] / a2[0, 0]), rtol=1e-14)
