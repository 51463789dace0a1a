"""Particle-in-cell transfers (oracle side; test infrastructure only).

Grid: N nodes per axis on the periodic cube [0, L)^d (d = 3, or d = 2 for the
two-dimensional example), node q = (q1, .., qd) at position q*h, h = L/N.  Grid arrays are
indexed [q1, .., qd] (q1 slowest).  Particle positions X have shape (P, d).

* Multilinear assignment (Sec. 2.2.1): R_h(x, qh) = h^-d prod_j max(1 - |x_j - q_j h| / h, 0);
  nonzero only on the 2^d vertices of the cell that contains x (trilinear for d = 3,
  bilinear for d = 2).
* Particle-to-grid (Alg. p2g): ubar(qh) = sum_p a_p R_h(X_p, qh).  The density factor that
  appears in eq. def_u_overline is read as a typesetting slip: the algorithm adds a_p R_h.
* Grid-to-particle (Alg. g2p, eq. g2p): f(X) = sum_q K_h(X, qh) f(qh) with K_h = h^3 R_h,
  so the weights sum to one.
* Fourth-order assignment R_h^(4) (Sec. 2.2.1): with p_j = |x_j - q_j h| / h, an inner weight
  on the 8 cell vertices and a negative outer weight on the 24 nodes one further step along a
  single axis; zero elsewhere.

Pinned by tests/test_oracle_pic.py (brute force over every node with minimum-image distances,
partition of unity, mass conservation, single-particle closed forms, O(h^2) gather rate).
"""
import numpy as np


def _cell_and_frac(X, N, L):
    """Lower node index (unwrapped) and grid coordinates s = x/h of every particle."""
    h = L / N
    s = np.asarray(X, dtype=np.float64) / h
    i0 = np.floor(s).astype(np.int64)
    return i0, s


def _flat(qw, N):
    """Row-major flat index of wrapped node coordinates qw (P, d)."""
    f = qw[:, 0].copy()
    for j in range(1, qw.shape[1]):
        f = f * N + qw[:, j]
    return f


def cic_weights(X, N, L):
    """Multilinear stencil of every particle (d = X.shape[1]).

    Returns (idx, wgt): idx (2^d, P) flat node indices (periodically wrapped), wgt (2^d, P)
    the interaction weights K_h = h^d R_h = prod_j max(1 - |s_j - q_j|, 0).
    """
    i0, s = _cell_and_frac(X, N, L)
    P, d = s.shape[0], s.shape[1]
    idx = np.empty((2 ** d, P), dtype=np.int64)
    wgt = np.empty((2 ** d, P), dtype=np.float64)
    for c, corner in enumerate(np.ndindex(*([2] * d))):
        q = i0 + np.array(corner, dtype=np.int64)
        w = np.ones(P)
        for j in range(d):
            w = w * np.maximum(1.0 - np.abs(s[:, j] - q[:, j]), 0.0)
        idx[c] = _flat(q % N, N)
        wgt[c] = w
    return idx, wgt


def _r4_1d_inner(p):
    return 1.0 - p


def r4_weight(p1, p2, p3):
    """h^3 R_h^(4) as a function of the per-axis distances in grid units (Sec. 2.2.1)."""
    p = [np.asarray(p1, dtype=np.float64), np.asarray(p2, dtype=np.float64),
         np.asarray(p3, dtype=np.float64)]
    inner = [pj <= 1.0 for pj in p]
    outer = [(pj > 1.0) & (pj <= 2.0) for pj in p]
    out = np.zeros(np.broadcast(*p).shape)
    all_inner = inner[0] & inner[1] & inner[2]
    w_in = ((1.0 - p[0]) * (1.0 - p[1]) * (1.0 - p[2])
            * (1.0 + sum(pj * (1.0 - pj) / 2.0 for pj in p)))
    out = np.where(all_inner, w_in, out)
    for j in range(3):
        k, l = [a for a in range(3) if a != j]
        mask = outer[j] & inner[k] & inner[l]
        w_out = -(1.0 / 6.0) * (1.0 - p[k]) * (1.0 - p[l]) \
            * (p[j] - 1.0) * (2.0 - p[j]) * (3.0 - p[j])
        out = np.where(mask, w_out, out)
    return out


def r4_weights(X, N, L):
    """Fourth-order stencil: the 4x4x4 nodes i0-1 .. i0+2 per axis (zero weight off support).

    Returns (idx, wgt) of shape (64, P); wgt is h^3 R_h^(4).
    """
    i0, s = _cell_and_frac(X, N, L)
    P = s.shape[0]
    idx = np.empty((64, P), dtype=np.int64)
    wgt = np.empty((64, P), dtype=np.float64)
    c = 0
    for o1 in (-1, 0, 1, 2):
        for o2 in (-1, 0, 1, 2):
            for o3 in (-1, 0, 1, 2):
                q = i0 + np.array([o1, o2, o3], dtype=np.int64)
                d = np.abs(s - q)
                wgt[c] = r4_weight(d[:, 0], d[:, 1], d[:, 2])
                qw = q % N
                idx[c] = (qw[:, 0] * N + qw[:, 1]) * N + qw[:, 2]
                c += 1
    return idx, wgt


def deposit(X, a, N, L, order=2):
    """Alg. p2g: ubar(qh) = sum_p a_p R_h(X_p, qh); returns an (N,)*d float64 array."""
    h = L / N
    d = np.asarray(X).shape[1]
    if order == 4 and d != 3:
        raise ValueError("the fourth-order assignment is stated for d = 3")
    if order == 2:
        idx, wgt = cic_weights(X, N, L)
    elif order == 4:
        idx, wgt = r4_weights(X, N, L)
    else:
        raise ValueError("deposit order must be 2 or 4")
    a = np.asarray(a, dtype=np.float64)
    u = np.zeros(N ** d)
    for c in range(idx.shape[0]):
        u += np.bincount(idx[c], weights=a * wgt[c], minlength=N ** d)
    return (u / h ** d).reshape((N,) * d)


def gather(fields, X, N, L):
    """Alg. g2p with K_h = h^d R_h (multilinear): values of each grid field at the particles.

    fields: sequence of (N,)*d arrays.  Returns an array of shape (len(fields), P).
    """
    idx, wgt = cic_weights(X, N, L)
    out = np.zeros((len(fields), idx.shape[1]))
    for f, field in enumerate(fields):
        flat = np.asarray(field, dtype=np.float64).reshape(-1)
        for c in range(idx.shape[0]):
            out[f] += wgt[c] * flat[idx[c]]
    return out
