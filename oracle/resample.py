"""Residual resampling, Alg. res_res (Sec. 2.3, resampling for long-term simulation).

TEST INFRASTRUCTURE ONLY (part of the oracle; see the package header).

The algorithm replaces P weighted particles by P particles of equal mass a0 = (1/P) sum_p a_p:
particle p is copied k_p = floor(a_p / a0) times, and the N_stoch = P - sum_p k_p remaining
particles are drawn from {1..P} with probabilities proportional to the residuals
r_p = a_p - k_p a0.  The paper leaves the arithmetic and the random source open; the reading
used here (shared with the GPU library so that both produce the same particle list) is:

* a0 = S / P with S the correctly rounded sum of the masses (math.fsum) and one IEEE division;
* q_p = a_p / a0 (one IEEE division), k_p = floor(q_p), and the residual is carried as the
  integer R_p = floor((q_p - k_p) 2^32), i.e. r_p / a0 in 32-bit fixed point (q_p - k_p is
  exact in float64), so that its prefix sums are exact and independent of summation order;
* draw j (j = 0 .. N_stoch - 1) takes the first two words (r0, r1) of Philox4x32-10 at counter
  (j, n, sim_lo, sim_hi | 2^31), key (seed_lo, seed_hi), forms u = r0 + 2^32 r1 and the target
  t = floor(u R_tot / 2^64) with R_tot = sum_p R_p, and selects the p whose interval
  [C_{p-1}, C_p) of the inclusive prefix sums C contains t (inverse CDF);
* the output list holds the deterministic copies in particle order, then the drawn particles
  in draw order, every one with mass a0;
* degenerate cases: if R_tot = 0 while N_stoch > 0 the draws are uniform over {0..P-1}
  (p = floor(u P / 2^64)); if rounding makes sum_p k_p exceed P the list is cut at P.

Pinned by tests/test_oracle_resample.py: exact cases with integer multiples of the mean, the
mass of the output, the copy counts, residual-free particles never drawn, the frequencies of
the draws against r_p / sum r (chi-square over many independent draws), the exactness of the
mean against rational arithmetic, and the Philox words against the generator's pin.
"""
import math

import numpy as np

from .philox import philox4x32_10

DOMAIN_BIT = 1 << 31   # set in counter word 3: resampling draws, never a step's noise


def mean_mass(a):
    """a0 = fl(fl(sum a) / P) with the sum correctly rounded."""
    a = np.asarray(a, dtype=np.float64)
    return math.fsum(a.tolist()) / a.shape[0]


def split(a, a0):
    """Deterministic copy counts k_p and fixed-point residuals R_p (Alg. res_res, first loop)."""
    q = np.asarray(a, dtype=np.float64) / a0
    k = np.floor(q)
    R = np.floor((q - k) * 2.0 ** 32)
    return k.astype(np.int64), R.astype(np.uint64)


def draws(nstoch, n, sim_id, seed):
    """64-bit uniform integers of the resampling stream (as Python ints)."""
    j = np.arange(nstoch, dtype=np.uint64)
    sim_id, seed = int(sim_id), int(seed)
    r0, r1, _, _ = philox4x32_10(j, np.uint64(n & 0xFFFFFFFF),
                                 np.uint64(sim_id & 0xFFFFFFFF),
                                 np.uint64((sim_id >> 32) | DOMAIN_BIT),
                                 np.uint64(seed & 0xFFFFFFFF), np.uint64(seed >> 32))
    return [int(x) | (int(y) << 32) for x, y in zip(r0, r1)]


def residual_resample(X, a, n, sim_id, seed):
    """Alg. res_res.  X: (P, 3) positions, a: (P,) masses, n: step index of the state.

    Returns (X_new, a_new, info) with info = dict(a0, k, R, n_det, n_stoch, src) where src is
    the source particle of every output particle.
    """
    X = np.asarray(X, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)
    P = a.shape[0]
    if P == 0:
        return X.copy(), a.copy(), dict(a0=0.0, k=np.zeros(0, np.int64),
                                        R=np.zeros(0, np.uint64), n_det=0, n_stoch=0,
                                        src=np.zeros(0, np.int64))
    a0 = mean_mass(a)
    k, R = split(a, a0)
    # deterministic splitting: k_p copies of particle p, in particle order
    det = np.repeat(np.arange(P, dtype=np.int64), k)[:P]
    n_stoch = P - det.shape[0]
    picked = np.zeros(0, dtype=np.int64)
    if n_stoch > 0:
        u = draws(n_stoch, n, sim_id, seed)
        R_tot = sum(int(x) for x in R)
        if R_tot > 0:
            C = np.cumsum(R.astype(np.uint64))          # exact: R_tot < 2^64
            t = np.array([(x * R_tot) >> 64 for x in u], dtype=np.uint64)
            picked = np.searchsorted(C, t, side="right").astype(np.int64)
        else:
            picked = np.array([(x * P) >> 64 for x in u], dtype=np.int64)
    src = np.concatenate([det, picked])
    info = dict(a0=a0, k=k, R=R, n_det=int(det.shape[0]), n_stoch=int(n_stoch), src=src)
    return X[src].copy(), np.full(P, a0), info
