"""Pins of the oracle's particle-in-cell transfers (Alg. p2g, Alg. g2p, R_h, R_h^(4)).

Brute force: R_h evaluated from its defining formula at every node of a tiny grid with
minimum-image distances (no cell index arithmetic), compared with the oracle's stencil code.
Closed forms: a particle on a node / at a cell centre; mass conservation (partition of unity);
exact reproduction of constants and linear functions by the trilinear gather; vanishing
moments of degree 1..3 of the fourth-order assignment; O(h^2) gather error (Thm pic_error).
"""
import itertools

import numpy as np
import pytest

from oracle import pic


def _min_image(d, L):
    d = np.abs(d)
    return np.minimum(d, L - d)


def _brute_R(X, N, L):
    """h^3 R_h(X_p, qh) for every node q: shape (P, N, N, N), straight from the formula."""
    h = L / N
    q = np.arange(N) * h
    P = X.shape[0]
    out = np.ones((P, N, N, N))
    for j, shape in enumerate([(1, N, 1, 1), (1, 1, N, 1), (1, 1, 1, N)]):
        d = _min_image(X[:, j][:, None] - q[None, :], L) / h
        out = out * np.maximum(1.0 - d, 0.0).reshape((P,) + shape[1:])
    return out


def _brute_R4(X, N, L):
    h = L / N
    q = np.arange(N) * h
    P = X.shape[0]
    d = [(_min_image(X[:, j][:, None] - q[None, :], L) / h) for j in range(3)]
    D1 = d[0][:, :, None, None] * np.ones((1, 1, N, N))
    D2 = d[1][:, None, :, None] * np.ones((1, N, 1, N))
    D3 = d[2][:, None, None, :] * np.ones((1, N, N, 1))
    return pic.r4_weight(D1, D2, D3)


@pytest.mark.parametrize("N", [4, 8])
def test_deposit_matches_bruteforce(N):
    rng = np.random.default_rng(N)
    L = 1.0
    P = 16
    X = rng.uniform(0, L, (P, 3))
    X[0] = [0.0, 0.0, 0.0]                  # on a node at the origin
    X[1] = [L - 1e-13, 0.5, L - 1e-13]      # straddles the periodic boundary
    a = rng.uniform(0.5, 2.0, P)
    u = pic.deposit(X, a, N, L)
    ref = np.einsum("p,pijk->ijk", a, _brute_R(X, N, L)) / (L / N) ** 3
    np.testing.assert_allclose(u, ref, rtol=1e-13, atol=1e-13 * ref.max())


def test_deposit4_matches_bruteforce():
    rng = np.random.default_rng(4)
    N, L, P = 8, 1.0, 12
    X = rng.uniform(0, L, (P, 3))
    X[0] = [0.999999, 0.0, 0.5]
    a = rng.uniform(0.5, 2.0, P)
    u = pic.deposit(X, a, N, L, order=4)
    ref = np.einsum("p,pijk->ijk", a, _brute_R4(X, N, L)) / (L / N) ** 3
    np.testing.assert_allclose(u, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_particle_on_node_and_cell_centre():
    N, L = 8, 1.0
    h = L / N
    u = pic.deposit(np.array([[2 * h, 1 * h, 3 * h]]), np.array([0.7]), N, L)
    assert u[2, 1, 3] == pytest.approx(0.7 / h ** 3, rel=1e-15)
    assert np.count_nonzero(u) == 1
    u = pic.deposit(np.array([[2.5 * h, 7.5 * h, 0.5 * h]]), np.array([0.8]), N, L)
    nz = np.argwhere(u != 0)
    assert len(nz) == 8
    assert {tuple(x) for x in nz} == {(i, j, k) for i in (2, 3) for j in (7, 0) for k in (0, 1)}
    np.testing.assert_allclose(u[u != 0], 0.8 / (8 * h ** 3), rtol=1e-14)


@pytest.mark.parametrize("order", [2, 4])
def test_mass_conservation(order):
    rng = np.random.default_rng(order)
    N, L, P = 16, 1.0, 5000
    X = rng.uniform(0, L, (P, 3))
    a = rng.uniform(0.1, 1.0, P)
    u = pic.deposit(X, a, N, L, order=order)
    assert (L / N) ** 3 * u.sum() == pytest.approx(a.sum(), rel=1e-13)
    if order == 2:
        assert u.min() >= 0.0


def test_gather_bruteforce_and_constants():
    rng = np.random.default_rng(7)
    N, L, P = 4, 1.0, 32
    X = rng.uniform(0, L, (P, 3))
    f = rng.standard_normal((N, N, N))
    got = pic.gather([f, np.full((N, N, N), 3.25)], X, N, L)
    ref = np.einsum("pijk,ijk->p", _brute_R(X, N, L), f)
    np.testing.assert_allclose(got[0], ref, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(got[1], 3.25, rtol=1e-15)


def test_gather_linear_exact_inside():
    N, L = 16, 1.0
    h = L / N
    rng = np.random.default_rng(3)
    X = rng.uniform(0.1, 0.85, (100, 3))   # stencils never wrap
    q = np.arange(N) * h
    f = 2.0 * q[:, None, None] - 3.0 * q[None, :, None] + 0.5 * q[None, None, :] + 1.0
    got = pic.gather([f], X, N, L)[0]
    np.testing.assert_allclose(got, 2 * X[:, 0] - 3 * X[:, 1] + 0.5 * X[:, 2] + 1.0,
                               rtol=1e-13, atol=1e-14)


def test_r4_partition_of_unity_and_moments():
    rng = np.random.default_rng(11)
    N, L = 8, 1.0
    X = rng.uniform(0, L, (50, 3))
    idx, w = pic.r4_weights(X, N, L)
    np.testing.assert_allclose(w.sum(axis=0), 1.0, rtol=0, atol=1e-14)
    s = X / (L / N)
    i0 = np.floor(s).astype(np.int64)
    offs = list(itertools.product((-1, 0, 1, 2), repeat=3))
    for e in itertools.product(range(4), repeat=3):
        if 0 < sum(e) <= 3:
            mom = np.zeros(X.shape[0])
            for c, o in enumerate(offs):
                d = (i0 + np.array(o)) - s
                mom += w[c] * np.prod(d ** np.array(e), axis=1)
            assert np.abs(mom).max() < 1e-13, e
    # outer weights are negative, inner non-negative
    assert w.min() < 0


def test_gather_second_order_rate():
    """Thm pic_error: |w_H - w| <= K_2 h^2 for a smooth field; slope of log err vs log N."""
    rng = np.random.default_rng(5)
    L = 1.0
    X = rng.uniform(0, L, (4000, 3))
    kvec = np.array([1, 2, -1])
    exact = np.cos(2 * np.pi * X @ kvec)
    errs, Ns = [], [8, 16, 32, 64]
    for N in Ns:
        q = np.arange(N) * (L / N)
        Q = np.stack(np.meshgrid(q, q, q, indexing="ij"), axis=-1)
        f = np.cos(2 * np.pi * Q @ kvec)
        errs.append(np.abs(pic.gather([f], X, N, L)[0] - exact).max())
    slope = np.polyfit(np.log(Ns), np.log(errs), 1)[0]
    assert slope < -1.8, (slope, errs)
