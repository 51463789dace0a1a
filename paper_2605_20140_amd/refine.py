"""Grid-refinement studies of the paper's examples (Sec. numerical experiments): the
three-dimensional example run to T = 6 at H = N = 2^4 .. 2^8, and the two-dimensional one at
H = 2^6 .. 2^10, each with the same particles and the same Wiener increments at every
resolution; each run's cell density at T is compared with the finest run's.  The
convergence order is the slope of log2 E against log2 N.

Error measure (the paper's, stated for its 2D example and used in 3D by analogy): every
density is downsampled by Fourier truncation to a 16^d grid and
    E = ||u_1 - u_2||_2 / max(||u_1||_2, ||u_2||_2),  ||u||_2 = (L / 16)^(d/2) (sum u^2)^(1/2).
The density of a run is its particle-to-grid deposit ubar on its own grid.  The truncation
keeps the integer frequencies |q_j| <= 7 (the 16-point Nyquist mode is dropped so the result
stays real).

Readings the paper leaves open in 3D, selectable here: the error measure (the 2D one above,
or the final particles deposited onto a 32^3 grid, the grid the paper's 3D density plots use:
--measure p2g32), whether every resolution shares the Wiener increments (default) or draws
its own (--noise independent), whether it shares the initial particles (default) or samples
its own (--ic independent), and the assignment order of the deposit (--order 4).

    python -m paper_2605_20140_amd.refine [--dim 3|2] [--steps 6000] [--particles 4194304]
                                          [--grids 16,32,64,128,256] [--fp32]
                                          [--measure fourier16|p2g32] [--noise shared|independent]
                                          [--ic shared|independent] [--order 2|4]
"""
import argparse
import json
import math
import sys
import time

import numpy as np

from . import sipf
from . import workloads as W

COARSE = 16


def downsample(u, n=COARSE):
    """Fourier truncation of an (N,)*d periodic grid field to (n,)*d, keeping values."""
    N, d = u.shape[0], u.ndim
    F = np.fft.fftn(u)
    h = n // 2
    src = np.r_[0:h, N - h + 1:N]
    dst = np.r_[0:h, n - h + 1:n]
    G = np.zeros((n,) * d, dtype=complex)
    G[np.ix_(*([dst] * d))] = F[np.ix_(*([src] * d))]
    return np.real(np.fft.ifftn(G)) * (n / N) ** d


def norm(u, L):
    return (L / u.shape[0]) ** (u.ndim / 2.0) * math.sqrt(float((u * u).sum()))


def rel_error(u1, u2, L):
    return norm(u1 - u2, L) / max(norm(u1, L), norm(u2, L))


def deposit_on(N, X, a, L, dim):
    """Particle-to-grid deposit of (X, a) onto an N^d grid, by the library (Alg. p2g)."""
    P = a.size
    p = sipf.make_params(N=N, P=P, dt=1e-3, L=L, dim=dim)
    g = np.ones((N,) * dim)
    sim = sipf.Simulation(p, X, a, g, 0.0 * g, g)
    u, _ = sim.aux()
    sim.close()
    return u


def run_one(N, P, steps, precision, log=None, dim=3, measure="fourier16", noise="shared",
            ic_mode="shared", order=2):
    ic_seed = dict(ic_seed=(21 if dim == 3 else 22) + (N if ic_mode == "independent" else 0))
    ic = (W.paper3d_initial_state if dim == 3 else W.paper2d_initial_state)(N, P=P, **ic_seed)
    prm = dict(ic["params"])
    if noise == "independent":
        prm["seed"] = prm["seed"] + 1000 * N
    prm["deposit_order"] = order
    p = sipf.make_params(precision=precision, **prm)  # prm carries dim
    t0 = time.perf_counter()
    sim = sipf.Simulation(p, ic["X0"], ic["a0"], ic["v0"], ic["m0"], ic["w0"])
    del ic
    t1 = time.perf_counter()
    done = 0
    while done < steps:   # chunks, so that progress is visible on long runs
        k = min(1000, steps - done)
        sim.step(k)
        done += k
        out = sim.fields(particles=False)
        if log:
            log(f"N={N} step {done}/{steps} mass {out['diag']['mass_particles']:.6f}")
    t2 = time.perf_counter()
    diag = out["diag"]
    if measure == "p2g32":
        fin = sim.fields()
        sim.close()
        return (deposit_on(32, fin["X"], fin["a"], prm["L"], dim), diag,
                dict(init_s=t1 - t0, run_s=t2 - t1))
    u, _ = sim.aux()
    sim.close()
    return downsample(u), diag, dict(init_s=t1 - t0, run_s=t2 - t1)


GRIDS = {3: (16, 32, 64, 128, 256), 2: (64, 128, 256, 512, 1024)}


def study(Ns=None, P=1 << 22, steps=6000, precision=0, log=None, dim=3, measure="fourier16",
          noise="shared", ic_mode="shared", order=2):
    L = W.PAPER3D_PARAMS["L"]
    Ns = GRIDS[dim] if Ns is None else Ns
    dens, info = {}, {}
    for N in Ns:
        dens[N], diag, tm = run_one(N, P, steps, precision, log, dim, measure, noise, ic_mode,
                                    order)
        info[N] = dict(mass_particles=diag["mass_particles"], min_v=diag["min_v"],
                       n_nan=diag["n_nan"], **tm)
    ref = max(Ns)
    errs = {N: rel_error(dens[N], dens[ref], L) for N in Ns if N != ref}
    xs = np.log2([N for N in errs])
    ys = np.log2([errs[N] for N in errs])
    slope = float(np.polyfit(xs, ys, 1)[0]) if len(xs) >= 2 else None
    return dict(dim=dim, errors={int(k): v for k, v in errs.items()}, slope=slope,
                reference_N=ref, measure=measure, noise=noise, ic=ic_mode, order=order,
                runs={int(k): v for k, v in info.items()}, steps=steps, particles=P,
                precision="f32" if precision else "f64")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--steps", type=int, default=W.PAPER3D_PARAMS["steps"])
    ap.add_argument("--particles", type=int, default=1 << 22)
    ap.add_argument("--grids", type=str, default=None, help="default: 16..256 (3D), 64..1024 (2D)")
    ap.add_argument("--dim", type=int, default=3, choices=(2, 3))
    ap.add_argument("--fp32", action="store_true")
    ap.add_argument("--measure", choices=("fourier16", "p2g32"), default="fourier16")
    ap.add_argument("--noise", choices=("shared", "independent"), default="shared")
    ap.add_argument("--ic", choices=("shared", "independent"), default="shared")
    ap.add_argument("--order", type=int, choices=(2, 4), default=2)
    a = ap.parse_args(argv)
    Ns = tuple(int(x) for x in a.grids.split(",")) if a.grids else None
    res = study(Ns, a.particles, a.steps, 1 if a.fp32 else 0,
                log=lambda s: print(s, file=sys.stderr, flush=True), dim=a.dim,
                measure=a.measure, noise=a.noise, ic_mode=a.ic, order=a.order)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
