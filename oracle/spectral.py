"""Spectral operators on the periodic N^d grid, d = 3 or 2 (oracle side; test infrastructure
only).

Fourier convention: numpy's fftn / ifftn (forward sum with e^{-2 pi i q.x / L}, inverse with
the 1/N^3 factor), integer frequencies q_j in standard DFT order {0, 1, ..., N/2-1, -N/2, ...,
-1}.  The paper's index set U_H = {-H/2, ..., H/2}^3 lists H+1 values per axis; with N nodes
only N frequencies exist, and the Nyquist frequency -N/2 is used as is in |q|^2.

* Implicit diffusion-decay multiplier (eq. k_q_tilde_update; the m-solve in the proof of the
  concentration lemma):  1 / (1 + tau (R + D (2 pi / L)^2 |q|^2)).
* Exponential multiplier K_tau (eq. k_q_update): exp(-tau (R + D (2 pi / L)^2 |q|^2)).
* Aliased multiplier (proof of Lemma kernel): the sum of K_tau over q + n N, n in Z^3, whose
  inverse DFT is the periodised Gaussian and hence positive.  The Gaussian factorises over
  axes, so the lattice sum is a product of three 1D sums.
* Low-pass filter (Alg. p2g text, Alg. sipf-pic): exp(-2 pi^2 |q|^2 / H0^2).
* Spectral gradient (eq. gradv): d_j v = IFFT(i (2 pi / L) q_j FFT(v)), with the Nyquist
  frequency of the differentiated axis set to zero so that the derivative of a real field is
  real.

Pinned by tests/test_oracle_spectral.py (exact Fourier-mode decay, exact derivatives of
trigonometric modes, naive DFT sums of eq. gradv at N = 4, positivity of the aliased kernel).
"""
import numpy as np


def freqs(N):
    """Integer frequencies in DFT order as float64: 0..N/2-1, -N/2..-1."""
    return np.fft.fftfreq(N, d=1.0 / N)


def _q2(N, d):
    """|q|^2 on the full (N,)*d frequency grid."""
    q = freqs(N) ** 2
    out = np.zeros((N,) * d)
    for j in range(d):
        shape = [1] * d
        shape[j] = N
        out = out + q.reshape(shape)
    return out


def k_squared(N, L, d=3):
    """(2 pi / L)^2 |q|^2 on the full (N,)*d frequency grid."""
    return (2.0 * np.pi / L) ** 2 * _q2(N, d)


def implicit_multiplier(N, L, dt, D, decay, d=3):
    return 1.0 / (1.0 + dt * (decay + D * k_squared(N, L, d)))


def exp_multiplier(N, L, dt, D, decay, d=3):
    return np.exp(-dt * (decay + D * k_squared(N, L, d)))


def aliased_multiplier(N, L, dt, D, decay, nmax=None, d=3):
    """sum_{n in Z^d} exp(-tau (decay + D (2 pi/L)^2 |q + n N|^2)), truncated at |n_j| <= nmax."""
    q = freqs(N)
    c = dt * D * (2.0 * np.pi / L) ** 2
    if nmax is None:
        # terms beyond |n| where c (|n| N - N/2)^2 > 745 underflow to zero in float64
        nmax = 1
        while c * ((nmax + 1) * N - N / 2) ** 2 < 745.0 and nmax < 100000:
            nmax += 1
    n = np.arange(-nmax, nmax + 1, dtype=np.float64)
    s1 = np.exp(-c * (q[:, None] + n[None, :] * N) ** 2).sum(axis=1)
    out = np.exp(-dt * decay) * np.ones((N,) * d)
    for j in range(d):
        shape = [1] * d
        shape[j] = N
        out = out * s1.reshape(shape)
    return out


def lowpass(N, H0, d=3):
    return np.exp(-2.0 * np.pi ** 2 * _q2(N, d) / H0 ** 2)


def apply_multiplier(f, mult):
    """Real part of IFFT(mult * FFT(f))."""
    return np.real(np.fft.ifftn(np.fft.fftn(f) * mult))


def derivative_freqs(N, L):
    """i (2 pi / L) q_j per axis with the Nyquist entry zeroed (1D array over q_j)."""
    q = freqs(N).copy()
    q[N // 2] = 0.0
    return 1j * (2.0 * np.pi / L) * q


def gradient(v, L, mult=None):
    """(d_1 v, .., d_d v) on the nodes via eq. gradv; optional extra spectral multiplier."""
    N, d = v.shape[0], v.ndim
    V = np.fft.fftn(v)
    if mult is not None:
        V = V * mult
    ik = derivative_freqs(N, L)
    out = []
    for j in range(d):
        shape = [1] * d
        shape[j] = N
        out.append(np.real(np.fft.ifftn(V * ik.reshape(shape))))
    return out
