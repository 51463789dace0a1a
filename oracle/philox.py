"""Philox4x32-10 and Box-Muller normals (oracle side; test infrastructure only).

The paper only states that the Wiener increments are independent N(0, 2 D_u tau I_3) draws
(eq. u_hat_update and the sampling step of Alg. sipf-pic).  To make a GPU run and this oracle
draw the *same* increments, both sides implement the counter-based generator Philox4x32-10
from its published definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC'11):

* state: a 128-bit counter (c0, c1, c2, c3) and a 64-bit key (k0, k1), all 32-bit words;
* one round multiplies c0 and c2 by the two Philox multipliers, giving 64-bit products
  (hi, lo), and forms the new counter (hi(c2*M1) ^ c1 ^ k0, lo(c2*M1), hi(c0*M0) ^ c3 ^ k1,
  lo(c0*M0));
* between rounds the key is advanced by the two Weyl constants (golden ratio and sqrt(3)-1
  in 32-bit fixed point); 10 rounds in total.

Stream assignment used by the step: counter = (p, n, sim_id_lo, sim_id_hi) with p the particle
index and n the absolute index of the step being taken, key = (seed_lo, seed_hi).

Uniforms: u_i = (r_i + 1/2) 2^-32, exact in FP64 and strictly inside (0, 1).
Normals (Box-Muller): z1 = sqrt(-2 ln u0) cos(2 pi u1), z2 = sqrt(-2 ln u0) sin(2 pi u1),
z3 = sqrt(-2 ln u2) cos(2 pi u3).

Pinned by tests/test_oracle_philox.py against the independent Philox engine that ships as a
header with PyTorch, and by distribution tests of the normals.
"""
import numpy as np

_MASK32 = np.uint64(0xFFFFFFFF)
# Philox4x32 round multipliers and Weyl key increments (Salmon et al., SC'11).
PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
PHILOX_W0 = np.uint64(0x9E3779B9)
PHILOX_W1 = np.uint64(0xBB67AE85)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox4x32 rounds on vectors of counters.

    All arguments are integer arrays (or scalars) holding 32-bit values; they broadcast.
    Returns four uint32 arrays (r0, r1, r2, r3).
    """
    c0 = np.asarray(c0, dtype=np.uint64) & _MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & _MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & _MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & _MASK32
    k0 = np.asarray(k0, dtype=np.uint64) & _MASK32
    k1 = np.asarray(k1, dtype=np.uint64) & _MASK32
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + PHILOX_W0) & _MASK32
            k1 = (k1 + PHILOX_W1) & _MASK32
        prod0 = PHILOX_M0 * c0          # < 2^64, exact in uint64
        prod1 = PHILOX_M1 * c2
        hi0, lo0 = prod0 >> np.uint64(32), prod0 & _MASK32
        hi1, lo1 = prod1 >> np.uint64(32), prod1 & _MASK32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return (c0.astype(np.uint32), c1.astype(np.uint32),
            c2.astype(np.uint32), c3.astype(np.uint32))


def uniforms(r):
    """Map uint32 words to (0,1): u = (r + 1/2) / 2^32, exact in float64."""
    return (np.asarray(r, dtype=np.float64) + 0.5) * (2.0 ** -32)


def step_normals(p, n, sim_id, seed):
    """Three standard normals per particle for step n (shape (len(p), 3)).

    p: particle indices (array), n: absolute step index, sim_id/seed: 64-bit integers.
    """
    p = np.asarray(p, dtype=np.uint64)
    sim_id = int(sim_id)
    seed = int(seed)
    r0, r1, r2, r3 = philox4x32_10(p, np.uint64(n & 0xFFFFFFFF),
                                   np.uint64(sim_id & 0xFFFFFFFF), np.uint64(sim_id >> 32),
                                   np.uint64(seed & 0xFFFFFFFF), np.uint64(seed >> 32))
    u0, u1, u2, u3 = uniforms(r0), uniforms(r1), uniforms(r2), uniforms(r3)
    rad01 = np.sqrt(-2.0 * np.log(u0))
    rad23 = np.sqrt(-2.0 * np.log(u2))
    z = np.empty((p.shape[0], 3), dtype=np.float64)
    z[:, 0] = rad01 * np.cos(2.0 * np.pi * u1)
    z[:, 1] = rad01 * np.sin(2.0 * np.pi * u1)
    z[:, 2] = rad23 * np.cos(2.0 * np.pi * u3)
    return z
