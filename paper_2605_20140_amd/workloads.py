"""Seeded synthetic workloads for the SIPF-W step (inputs only).

This module builds initial states and parameter sets; it contains none of the method's
arithmetic and is the only code that both the GPU path's callers and the FP64 oracle's tests
use.  All randomness here comes from numpy's Philox bit generator with a stated seed, so every
workload is reproducible.

Initial data follow the paper's recipe (Alg. sipf-pic initialisation: particles sampled i.i.d.
from u(., 0) with equal masses M0 / P; concentrations sampled at the nodes), with Gaussian-blob
cell densities on the periodic unit cube:

* g_b(x) = exp(-d(x, c_b)^2 / (2 sigma_b^2)), d the minimum-image distance on the torus;
  G = sum_b g_b / max_nodes(sum_b g_b), so the peak is 1;
* particles: particle p belongs to blob p mod B and sits at c_b + sigma_b Z (wrapped), Z a
  standard normal 3-vector; masses a_p = 1 / P (total mass 1);
* v0 = 1 - 0.5 G, m0 = 0.5 G, w0 = 1 (or the random-mode ECM field of the 64^3 workload).
"""
import math
import numpy as np

# Shared physical parameters of every workload (unit cube).
BASE_PARAMS = dict(L=1.0, D_u=1e-3, chi=5e-3, D_m=1e-3, D_w=5e-3, alpha=10.0, beta=0.5,
                   gamma=0.5)


def _rng(seed):
    return np.random.Generator(np.random.Philox(int(seed)))


def _wrap_unit(X, L):
    Y = np.mod(X, L)
    Y[Y >= L] = 0.0
    return Y


def blob_field(N, L, centres, sigmas):
    """Peak-normalised sum of periodic Gaussian blobs sampled at the nodes, shape (N, N, N)."""
    x = np.arange(N) * (L / N)
    G = np.zeros((N, N, N))
    for c, s in zip(centres, sigmas):
        d2 = np.zeros((N, N, N))
        for j, shape in enumerate([(N, 1, 1), (1, N, 1), (1, 1, N)]):
            dj = np.abs(x - c[j])
            dj = np.minimum(dj, L - dj)
            d2 = d2 + (dj ** 2).reshape(shape)
        G += np.exp(-d2 / (2.0 * s * s))
    return G / G.max()


def blob_particles(P, L, centres, sigmas, rng):
    """P positions, particle p drawn from blob p mod B; returns (P, 3) float64 in [0, L)."""
    B = len(centres)
    centres = np.asarray(centres, dtype=np.float64)
    sigmas = np.asarray(sigmas, dtype=np.float64)
    b = np.arange(P) % B
    Z = rng.standard_normal((P, 3))
    return _wrap_unit(centres[b] + sigmas[b][:, None] * Z, L)


def random_mode_field(N, L, nmodes=32, qmax=4, seed=1, floor=0.05):
    """v0 = max(1 + 0.1 sum_j A_j cos(2 pi q_j.x / L + phi_j), floor).

    q_j uniform over the integer vectors with 0 < |q| <= qmax, A_j ~ N(0,1), phi_j ~ U[0, 2pi).
    """
    rng = _rng(seed)
    r = np.arange(-qmax, qmax + 1)
    Q = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 3)
    n2 = (Q ** 2).sum(axis=1)
    Q = Q[(n2 > 0) & (n2 <= qmax * qmax)]
    sel = Q[rng.integers(0, Q.shape[0], size=nmodes)]
    A = rng.standard_normal(nmodes)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=nmodes)
    x = np.arange(N) * (L / N)
    X1, X2, X3 = np.meshgrid(x, x, x, indexing="ij")
    s = np.zeros((N, N, N))
    for q, amp, ph in zip(sel, A, phi):
        s += amp * np.cos(2.0 * np.pi * (q[0] * X1 + q[1] * X2 + q[2] * X3) / L + ph)
    return np.maximum(1.0 + 0.1 * s, floor)


def random_blobs(nblobs, rng, smin=0.05, smax=0.12):
    centres = rng.uniform(0.0, 1.0, size=(nblobs, 3))
    sigmas = rng.uniform(smin, smax, size=nblobs)
    return centres, sigmas


# name: (N, P, steps, dt, noise seed, IC recipe)
WORKLOADS = {
    # single blob, the small FP64 case
    "blob16": dict(N=16, P=4096, steps=100, dt=1e-3, seed=0, ic="blob1", ic_seed=0),
    # FP64 vs FP32 comparison case with a random-mode ECM field
    "modes64": dict(N=64, P=1 << 20, steps=500, dt=1e-3, seed=2, ic="modes", ic_seed=1),
    # headline scale: 4 random blobs
    "blobs128": dict(N=128, P=1 << 23, steps=1000, dt=5e-4, seed=3, ic="blobs", nblobs=4,
                     ic_seed=3),
    # largest single-GPU case: 16 random blobs
    "blobs256": dict(N=256, P=1 << 25, steps=200, dt=2.5e-4, seed=5, ic="blobs", nblobs=16,
                     ic_seed=5),
}


def make_params(name, **over):
    """Parameter dict of a named workload (physical constants + sizes), with overrides."""
    w = dict(WORKLOADS[name])
    w.update(over)
    prm = dict(BASE_PARAMS)
    for k in ("L", "D_u", "chi", "D_m", "D_w", "alpha", "beta", "gamma"):
        if k in over:
            prm[k] = over[k]
    prm.update(N=w["N"], P=w["P"], dt=w["dt"], seed=w["seed"], steps=w["steps"])
    return prm


def weighted_masses(P, spread, rng):
    """Log-normal particle masses exp(spread Z), scaled to total mass 1: the unequal weights a
    long run accumulates (Lemma mass), for resampling inputs."""
    a = np.exp(spread * rng.standard_normal(P))
    return a / a.sum()


def make_initial_state(name, **over):
    """Initial state of a named workload: dict with X0 (P,3), a0 (P,), v0, m0, w0 (N,N,N).

    Overrides may change N, P, dt, steps, seed, ic_seed and the physical constants;
    mass_spread > 0 draws unequal (log-normal) particle masses instead of equal ones.
    """
    w = dict(WORKLOADS[name])
    w.update(over)
    prm = make_params(name, **over)
    N, P, L = prm["N"], prm["P"], prm["L"]
    rng = _rng(w["ic_seed"])
    if w["ic"] in ("blob1", "modes"):
        centres, sigmas = [(0.5, 0.5, 0.5)], [0.1]
    else:
        centres, sigmas = random_blobs(w["nblobs"], rng)
    G = blob_field(N, L, centres, sigmas)
    X0 = blob_particles(P, L, centres, sigmas, rng)
    a0 = np.full(P, 1.0 / P) if P > 0 else np.zeros(0)
    if w.get("mass_spread") and P > 0:
        a0 = weighted_masses(P, w["mass_spread"], rng)
    if w["ic"] == "modes":
        v0 = random_mode_field(N, L, seed=w["ic_seed"])
    else:
        v0 = 1.0 - 0.5 * G
    m0 = 0.5 * G
    w0 = np.ones((N, N, N))
    return dict(params=prm, X0=X0, a0=a0, v0=v0, m0=m0, w0=w0)


def served_mix(nreq=256, rate=None, steps=200, dt=1e-3, seed=4, sizes=(32, 64, 128),
               logp=(16, 22), chi_range=(1e-3, 1e-2)):
    """Request list of the served workload: arrival times (Poisson), grid, particles, chi.

    Each request is a dict with keys t_arrive, N, P, chi, steps, dt, ic_seed, seed, sim_id.
    rate: arrivals per second (None: all arrive at t = 0).
    """
    rng = _rng(seed)
    t = 0.0
    out = []
    for i in range(nreq):
        if rate:
            t += rng.exponential(1.0 / rate)
        N = int(rng.choice(sizes))
        P = int(round(2.0 ** rng.uniform(*logp)))
        chi = float(10.0 ** rng.uniform(math.log10(chi_range[0]), math.log10(chi_range[1])))
        out.append(dict(t_arrive=t, N=N, P=P, chi=chi, steps=steps, dt=dt,
                        ic_seed=1000 + i, seed=1000 + i, sim_id=i))
    return out


def served_initial_state(req, nblobs=4):
    """Initial state of one served request (random blobs, as the headline workload)."""
    N, P, L = req["N"], req["P"], BASE_PARAMS["L"]
    rng = _rng(req["ic_seed"])
    centres, sigmas = random_blobs(nblobs, rng)
    G = blob_field(N, L, centres, sigmas)
    X0 = blob_particles(P, L, centres, sigmas, rng)
    prm = dict(BASE_PARAMS)
    prm.update(N=N, P=P, dt=req["dt"], chi=req["chi"], seed=req["seed"], steps=req["steps"])
    return dict(params=prm, X0=X0, a0=np.full(P, 1.0 / P), v0=1.0 - 0.5 * G, m0=0.5 * G,
                w0=np.ones((N, N, N)))


# ---- the paper's three-dimensional example (Sec. numerical experiments, 3D simulation) ----
# Periodic cube [0, 6]^3; u0 = 3 on the ball |x - (3,3,3)| <= sqrt(0.3), m0 = u0,
# v0 = 0.05 cos(5 pi x1^2 / 18) sin(13 pi x2^2 / 72) cos(pi x3^2 / 12) + 0.3, w0 = 4 v0;
# chi = 0.4, D_u = D_m = D_w = 0.01, alpha = 5, beta = 0.01, gamma = 5; tau = 1e-3 to T = 6
# (6000 steps); P = 2^22 particles.
PAPER3D_PARAMS = dict(L=6.0, D_u=0.01, chi=0.4, D_m=0.01, D_w=0.01, alpha=5.0, beta=0.01,
                      gamma=5.0, dt=1e-3, steps=6000, seed=21)
PAPER3D_BALL = dict(centre=(3.0, 3.0, 3.0), radius=math.sqrt(0.3), height=3.0)


def paper3d_initial_state(N, P=1 << 22, ic_seed=21, **over):
    """Initial state of the paper's 3D example on an N^3 grid: particles i.i.d. uniform in the
    ball (the normalised u0), equal masses 3 |ball| / P; fields sampled at the nodes."""
    prm = dict(PAPER3D_PARAMS)
    prm.update(over)
    prm.update(N=N, P=P)
    L = prm["L"]
    c = np.asarray(PAPER3D_BALL["centre"])
    r0 = PAPER3D_BALL["radius"]
    rng = _rng(ic_seed)
    d = rng.standard_normal((P, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    r = r0 * rng.random(P) ** (1.0 / 3.0)
    X0 = _wrap_unit(c + r[:, None] * d, L)
    mass = PAPER3D_BALL["height"] * 4.0 / 3.0 * math.pi * r0 ** 3
    a0 = np.full(P, mass / P) if P > 0 else np.zeros(0)
    x = np.arange(N) * (L / N)
    X1, X2, X3 = np.meshgrid(x, x, x, indexing="ij")
    inside = (X1 - c[0]) ** 2 + (X2 - c[1]) ** 2 + (X3 - c[2]) ** 2 <= r0 * r0
    m0 = np.where(inside, PAPER3D_BALL["height"], 0.0)
    v0 = (0.05 * np.cos(5.0 * math.pi * X1 ** 2 / 18.0) * np.sin(13.0 * math.pi * X2 ** 2 / 72.0)
          * np.cos(math.pi * X3 ** 2 / 12.0) + 0.3)
    return dict(params=prm, X0=X0, a0=a0, v0=v0, m0=m0, w0=4.0 * v0)


# ---- two-dimensional inputs (Sec. numerical experiments, 2D simulation) -------------------
def blob2d_initial_state(N=32, P=4096, seed=0, ic_seed=0, dt=1e-3, sigma=0.1, **over):
    """2D counterpart of the single-blob workload on the unit square: G = exp(-d^2/(2 s^2))
    (peak 1), particles c + s Z (wrapped), masses 1/P, v0 = 1 - 0.5 G, m0 = 0.5 G, w0 = 1."""
    prm = dict(BASE_PARAMS)
    prm.update(over)
    prm.update(N=N, P=P, dt=dt, seed=seed, steps=100, dim=2)
    L = prm["L"]
    rng = _rng(ic_seed)
    c = np.array([0.5, 0.5])
    x = np.arange(N) * (L / N)
    d2 = np.zeros((N, N))
    for j, shape in enumerate([(N, 1), (1, N)]):
        dj = np.abs(x - c[j])
        dj = np.minimum(dj, L - dj)
        d2 = d2 + (dj ** 2).reshape(shape)
    G = np.exp(-d2 / (2.0 * sigma * sigma))
    X0 = _wrap_unit(c + sigma * rng.standard_normal((P, 2)), L)
    a0 = np.full(P, 1.0 / P) if P > 0 else np.zeros(0)
    if over.get("mass_spread") and P > 0:
        a0 = weighted_masses(P, over["mass_spread"], rng)
    return dict(params=prm, X0=X0, a0=a0, v0=1.0 - 0.5 * G, m0=0.5 * G, w0=np.ones((N, N)))


# The paper's 2D example: periodic square [0, 6]^2; u0 = 5 max(r0^2 - |x - (3,3)|^2, 0) with
# r0 = sqrt(0.3), m0 = u0, v0 = 0.05 cos(5 pi x1^2 / 18) sin(13 pi x2^2 / 72) + 0.3, w0 = 4 v0;
# the same constants as the 3D example; tau = 1e-3 to T = 6; P = 2^22.
def paper2d_initial_state(N, P=1 << 22, ic_seed=22, **over):
    """Particles i.i.d. from the normalised u0 (radius r with r^2 = r0^2 (1 - sqrt(1 - U)),
    uniform angle), equal masses; fields sampled at the nodes."""
    prm = dict(PAPER3D_PARAMS)
    prm.update(over)
    prm.update(N=N, P=P, dim=2, seed=22)
    L = prm["L"]
    c = np.array([3.0, 3.0])
    r0sq = 0.3
    rng = _rng(ic_seed)
    r = np.sqrt(r0sq * (1.0 - np.sqrt(1.0 - rng.random(P))))
    th = 2.0 * math.pi * rng.random(P)
    X0 = _wrap_unit(c + np.stack([r * np.cos(th), r * np.sin(th)], axis=1), L)
    mass = 5.0 * math.pi * r0sq * r0sq / 2.0
    a0 = np.full(P, mass / P) if P > 0 else np.zeros(0)
    x = np.arange(N) * (L / N)
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    m0 = 5.0 * np.maximum(r0sq - (X1 - c[0]) ** 2 - (X2 - c[1]) ** 2, 0.0)
    v0 = 0.05 * np.cos(5.0 * math.pi * X1 ** 2 / 18.0) * np.sin(13.0 * math.pi * X2 ** 2 / 72.0) + 0.3
    return dict(params=prm, X0=X0, a0=a0, v0=v0, m0=m0, w0=4.0 * v0)
