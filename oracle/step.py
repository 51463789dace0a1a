"""One SIPF-W time step, Alg. sipf-pic, in float64 (oracle side; test infrastructure only).

State at step n: particles (X_p, a_p), X_p in [0, L)^d, a_p > 0; nodal fields v, m, w on the
N^d grid (nodes at q h, h = L / N); the absolute step index n.  d = 3, or d = 2 for the
paper's two-dimensional example (the method is stated for general d; the 2D step uses the
bilinear assignment and the first two normals of the Philox block).

One step n -> n+1, every right-hand side taken at time n (explicit operator splitting,
eq. g_hat_phy; Euler-Maruyama, eq. u_hat_update):

1. ubar = P2G(X, a) (Alg. p2g; trilinear, or the fourth-order assignment on request).
2. grad v = spectral gradient of v (eq. gradv), optionally low-pass filtered.
3. (grad v)_p, w_p = G2P at X_p (Alg. g2p, trilinear K_h = h^3 R_h).
4. Explicit reaction R_tau (eq. g_hat_phy with S of eq. g_t):
   m* = m + tau ubar;  w* = w + tau (gamma v - eta(ubar) w),  eta(u) = 2u / (1 + u);
   v^{n+1} = v exp(-alpha tau m)   (exact flow of v_t = -alpha m v at frozen m; the paper's
   implicit form v / (1 + alpha tau m) of the positivity section is available as a flag).
5. Diffusion and linear decay in Fourier space (eq. k_q_tilde_update):
   m^{n+1} = IFFT(FFT(m*) / (1 + tau (beta + D_m k^2))),
   w^{n+1} = IFFT(FFT(w*) / (1 + tau (1 + D_w k^2))),
   or the exponential / aliased multipliers of eq. k_q_update and Lemma kernel on request,
   times the low-pass filter exp(-2 pi^2 |q|^2 / H0^2) when H0 > 0.
6. Push: X^{n+1} = wrap(X + chi tau (grad v)_p + sqrt(2 D_u tau) Z_p), Z_p from Philox with
   counter (p, n, sim_id) (see oracle.philox);
   a^{n+1} = a exp(tau (rho(w_p) - 1)), rho(w) = 2w / (1 + w)  (exact flow of
   d(log a) = rho - 1 of eq. SDE at frozen w_p; the linear Euler form a (1 + tau rho - tau) of
   eq. u_hat_update is available as a flag).
7. n <- n + 1.

Wrap: X <- X - L floor(X / L); a result equal to L (rounding of a tiny negative X) is set to 0.
"""
from dataclasses import dataclass, replace
import numpy as np

from . import pic, philox, spectral


@dataclass
class Params:
    N: int
    dt: float
    L: float = 1.0
    D_u: float = 1e-3
    chi: float = 5e-3
    D_m: float = 1e-3
    D_w: float = 5e-3
    alpha: float = 10.0
    beta: float = 0.5
    gamma: float = 0.5
    seed: int = 0
    sim_id: int = 0
    deposit_order: int = 2
    H0: float = 0.0                 # 0: no low-pass filter
    diffusion: str = "implicit"     # "implicit" | "exp" | "aliased"
    freeze_w: bool = False
    freeze_v: bool = False
    freeze_m: bool = False
    no_noise: bool = False
    linear_mass: bool = False
    implicit_v: bool = False


@dataclass
class State:
    X: np.ndarray      # (P, 3)
    a: np.ndarray      # (P,)
    v: np.ndarray      # (N, N, N)
    m: np.ndarray
    w: np.ndarray
    n: int = 0

    def copy(self):
        return State(self.X.copy(), self.a.copy(), self.v.copy(), self.m.copy(),
                     self.w.copy(), self.n)


def rho(w):
    """Proliferation rate rho(w) = 2w / (1 + w) (eq. haptotaxis-system)."""
    return 2.0 * w / (1.0 + w)


def eta(u):
    """Oxygen consumption eta(u) = 2u / (1 + u) (eq. haptotaxis-system)."""
    return 2.0 * u / (1.0 + u)


def diffusion_multiplier(prm, D, decay, d=3):
    if prm.diffusion == "implicit":
        mult = spectral.implicit_multiplier(prm.N, prm.L, prm.dt, D, decay, d=d)
    elif prm.diffusion == "exp":
        mult = spectral.exp_multiplier(prm.N, prm.L, prm.dt, D, decay, d=d)
    elif prm.diffusion == "aliased":
        mult = spectral.aliased_multiplier(prm.N, prm.L, prm.dt, D, decay, d=d)
    else:
        raise ValueError(prm.diffusion)
    if prm.H0 > 0:
        mult = mult * spectral.lowpass(prm.N, prm.H0, d=d)
    return mult


def wrap(X, L):
    Y = X - L * np.floor(X / L)
    Y[Y >= L] = 0.0
    return Y


def field_update(ubar, v, m, w, prm):
    """Steps 4 and 5 on the grid: explicit reaction on the time-n fields, then the diffusion
    and decay solves.  Returns (v^{n+1}, m^{n+1}, w^{n+1})."""
    d, dt = v.ndim, prm.dt
    m_star = m + dt * ubar
    w_star = w + dt * (prm.gamma * v - eta(ubar) * w)
    if prm.implicit_v:
        v_new = v / (1.0 + prm.alpha * dt * m)
    else:
        v_new = v * np.exp(-prm.alpha * dt * m)
    m_new = spectral.apply_multiplier(m_star, diffusion_multiplier(prm, prm.D_m, prm.beta, d))
    w_new = spectral.apply_multiplier(w_star, diffusion_multiplier(prm, prm.D_w, 1.0, d))
    if prm.freeze_v:
        v_new = v.copy()
    if prm.freeze_m:
        m_new = m.copy()
    if prm.freeze_w:
        w_new = w.copy()
    return v_new, m_new, w_new


def particle_update(X, a, ids, g, n, prm):
    """Step 6 for the particles with indices ids (rows of X and a, in the same order): g holds
    their gathered values ((grad v)_p rows, then w_p), n the step index that keys the noise.
    Returns (X^{n+1}, a^{n+1}) of those particles."""
    P, d = X.shape[0], X.shape[1]
    dt = prm.dt
    if prm.no_noise or P == 0:
        z = np.zeros((P, d))
    else:
        z = philox.step_normals(np.asarray(ids), n, prm.sim_id, prm.seed)[:, :d]
    X_new = wrap(X + prm.chi * dt * g[:d].T + np.sqrt(2.0 * prm.D_u * dt) * z, prm.L)
    w_p = g[d]
    if prm.linear_mass:
        a_new = a * (1.0 + dt * rho(w_p) - dt)
    else:
        a_new = a * np.exp(dt * (rho(w_p) - 1.0))
    return X_new, a_new, z


def step(state, prm, return_aux=False):
    """Advance one step; returns the new State (and a dict of intermediates if asked)."""
    N, L = prm.N, prm.L
    X, a, v, m, w = state.X, state.a, state.v, state.m, state.w
    P, d = X.shape[0], v.ndim

    # 1. particle-to-grid
    ubar = pic.deposit(X, a, N, L, order=prm.deposit_order)
    # 2. spectral gradient of the old v
    grad = spectral.gradient(v, L, mult=spectral.lowpass(N, prm.H0, d=d) if prm.H0 > 0 else None)
    # 3. grid-to-particle at the old positions
    g = pic.gather(list(grad) + [w], X, N, L)
    # 4. explicit reaction on the old fields, 5. diffusion + linear decay
    v_new, m_new, w_new = field_update(ubar, v, m, w, prm)
    # 6. Euler-Maruyama push and mass update
    X_new, a_new, z = particle_update(X, a, np.arange(P), g, state.n, prm)
    new = State(X_new, a_new, v_new, m_new, w_new, state.n + 1)
    if return_aux:
        return new, dict(ubar=ubar, grad=grad, g=g, z=z)
    return new


def run(state, prm, nsteps):
    s = state
    for _ in range(nsteps):
        s = step(s, prm)
    return s


def diagnostics(state, prm):
    """Mass sums and positivity figures of a state (Lemma mass, Corollary mass, positivity)."""
    N, L = prm.N, prm.L
    h3 = (L / N) ** state.v.ndim   # cell volume h^d
    ubar = pic.deposit(state.X, state.a, N, L, order=prm.deposit_order)
    return dict(
        mass_particles=float(np.sum(state.a)),
        mass_grid=float(h3 * np.sum(ubar)),
        mass_m=float(h3 * np.sum(state.m)),
        min_v=float(state.v.min()), min_m=float(state.m.min()), min_w=float(state.w.min()),
        max_m=float(state.m.max()), max_w=float(state.w.max()),
        min_a=float(state.a.min()) if state.a.size else 0.0,
        max_a=float(state.a.max()) if state.a.size else 0.0,
        min_u=float(ubar.min()),
        n_nan=int(np.isnan(state.X).sum() + np.isnan(state.a).sum() + np.isnan(state.v).sum()
                  + np.isnan(state.m).sum() + np.isnan(state.w).sum()),
        n_neg_m=int((state.m < 0).sum()), n_neg_w=int((state.w < 0).sum()),
        step=state.n,
    )


def with_(prm, **kw):
    return replace(prm, **kw)
