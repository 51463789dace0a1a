"""Pins of the oracle's spectral operators (eq. gradv, eq. k_q_tilde_update, Lemma kernel).

* the spectral gradient differentiates trigonometric modes exactly on the nodes and returns
  zero for the Nyquist mode (the reading used for |q_j| = N/2);
* a naive O(N^6) evaluation of eq. gradv at N = 4 (explicit Fourier sums, no FFT library);
* Poisson summation: the inverse DFT of the aliased multiplier equals h^3 times the periodised
  heat kernel (4 pi D tau)^{-3/2} exp(-|x|^2 / (4 D tau)) e^{-R tau} at the nodes, hence is
  positive, and stays within the Lemma kernel bound of the plain multiplier;
* the low-pass filter equals convolution with a Gaussian of variance L^2 / H0^2 per axis.
"""
import itertools

import numpy as np
import pytest

from oracle import spectral


def _nodes(N, L):
    x = np.arange(N) * (L / N)
    return np.meshgrid(x, x, x, indexing="ij")


@pytest.mark.parametrize("N,L", [(8, 1.0), (16, 6.0)])
def test_gradient_of_modes_exact(N, L):
    X1, X2, X3 = _nodes(N, L)
    rng = np.random.default_rng(N)
    for _ in range(5):
        q = rng.integers(-(N // 2) + 1, N // 2, size=3)
        ph = rng.uniform(0, 2 * np.pi)
        arg = 2 * np.pi * (q[0] * X1 + q[1] * X2 + q[2] * X3) / L + ph
        g = spectral.gradient(np.cos(arg), L)
        for j in range(3):
            np.testing.assert_allclose(g[j], -(2 * np.pi * q[j] / L) * np.sin(arg),
                                       atol=1e-12 * (1 + abs(q[j])) * N)


def test_gradient_nyquist_zero():
    N, L = 8, 1.0
    i = np.arange(N)
    v = ((-1.0) ** i)[:, None, None] * np.ones((N, N, N))
    g = spectral.gradient(v, L)
    for j in range(3):
        assert np.abs(g[j]).max() < 1e-12


def test_gradient_naive_dft_sums():
    """eq. gradv with explicit sums; the differentiated axis skips its Nyquist frequency."""
    N, L = 4, 1.0
    rng = np.random.default_rng(0)
    v = rng.standard_normal((N, N, N))
    idx = list(itertools.product(range(N), repeat=3))
    qs = list(itertools.product(range(-N // 2, N // 2), repeat=3))
    # Fourier coefficients k_q = N^-3 sum_x v(x) e^{-2 pi i q.x/L}
    kq = {}
    for q in qs:
        s = 0j
        for p in idx:
            s += v[p] * np.exp(-2j * np.pi * np.dot(q, p) / N)
        kq[q] = s / N ** 3
    got = spectral.gradient(v, L)
    for j in range(3):
        ref = np.zeros((N, N, N))
        for p in idx:
            s = 0j
            for q in qs:
                if q[j] == -N // 2:
                    continue
                s += (2j * np.pi * q[j] / L) * kq[q] * np.exp(2j * np.pi * np.dot(q, p) / N)
            ref[p] = s.real
        np.testing.assert_allclose(got[j], ref, atol=1e-12)


def test_implicit_multiplier_values():
    N, L, dt, D, R = 8, 2.0, 0.01, 0.3, 0.7
    mult = spectral.implicit_multiplier(N, L, dt, D, R)
    assert mult[0, 0, 0] == pytest.approx(1.0 / (1.0 + dt * R), rel=1e-15)
    # q = (1, -4, 2): index 4 is the Nyquist -4
    q2 = 1 + 16 + 4
    assert mult[1, 4, 2] == pytest.approx(1.0 / (1 + dt * (R + D * (2 * np.pi / L) ** 2 * q2)),
                                          rel=1e-14)


@pytest.mark.parametrize("N,L,Dt", [(8, 1.0, 2e-3), (16, 1.0, 1e-3), (16, 6.0, 0.05)])
def test_aliased_kernel_is_periodised_heat_kernel(N, L, Dt):
    D, dt, R = 1.0, Dt, 0.4
    Khat = spectral.aliased_multiplier(N, L, dt, D, R)
    g = np.real(np.fft.ifftn(Khat))
    X1, X2, X3 = _nodes(N, L)
    G = np.zeros((N, N, N))
    nimg = 4
    for n in itertools.product(range(-nimg, nimg + 1), repeat=3):
        r2 = (X1 + n[0] * L) ** 2 + (X2 + n[1] * L) ** 2 + (X3 + n[2] * L) ** 2
        G += np.exp(-r2 / (4 * D * dt))
    G *= (4 * np.pi * D * dt) ** -1.5 * np.exp(-R * dt) * (L / N) ** 3
    np.testing.assert_allclose(g, G, rtol=1e-10, atol=1e-14 * G.max())
    # positive up to FFT roundoff (the exact values G are all > 0)
    assert G.min() > 0 and g.min() > -1e-15 * g.max()
    K = spectral.exp_multiplier(N, L, dt, D, R)
    assert np.abs(Khat - K).max() < 4 * np.exp(-np.pi ** 2 * D * dt * N ** 2 / L ** 2)


def test_implicit_kernel_has_negative_lobes():
    """The reading that m, w positivity is only soft with the implicit multiplier."""
    mult = spectral.implicit_multiplier(16, 1.0, 1e-3, 1e-3, 0.5)
    g = np.real(np.fft.ifftn(mult))
    assert g.min() < -1e-5 * g.max()


def test_lowpass_is_gaussian_convolution():
    N, L, H0 = 16, 1.0, 6.0
    g = np.real(np.fft.ifftn(spectral.lowpass(N, H0)))
    s2 = L ** 2 / H0 ** 2
    X1, X2, X3 = _nodes(N, L)
    G = np.zeros((N, N, N))
    for n in itertools.product(range(-3, 4), repeat=3):
        r2 = (X1 + n[0] * L) ** 2 + (X2 + n[1] * L) ** 2 + (X3 + n[2] * L) ** 2
        G += np.exp(-r2 / (2 * s2))
    G *= (2 * np.pi * s2) ** -1.5 * (L / N) ** 3
    np.testing.assert_allclose(g, G, rtol=1e-9, atol=1e-13)
