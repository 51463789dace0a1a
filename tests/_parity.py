"""Helpers shared by the parity tests: run the oracle and the HIP path on the same seeded
inputs and compare them field by field."""
import numpy as np

from oracle import step as S
from paper_2605_20140_amd import workloads as W

FLAG_BITS = dict(freeze_w=0x01, freeze_v=0x02, freeze_m=0x04, no_noise=0x08,
                 linear_mass=0x10, implicit_v=0x20)


def oracle_params(prm, **kw):
    o = S.Params(N=prm["N"], dt=prm["dt"], L=prm["L"], D_u=prm["D_u"], chi=prm["chi"],
                 D_m=prm["D_m"], D_w=prm["D_w"], alpha=prm["alpha"], beta=prm["beta"],
                 gamma=prm["gamma"], seed=prm["seed"], sim_id=prm.get("sim_id", 0))
    return S.with_(o, **kw)


def flags_of(**kw):
    f = 0
    for k, bit in FLAG_BITS.items():
        if kw.get(k):
            f |= bit
    if kw.get("diffusion") == "exp":
        f |= 0x80
    if kw.get("diffusion") == "aliased":
        f |= 0x100
    return f


def oracle_state(ic, step0=0):
    return S.State(ic["X0"].copy(), ic["a0"].copy(), ic["v0"].copy(), ic["m0"].copy(),
                   ic["w0"].copy(), step0)


def gpu_sim(ic, precision=0, flags=0, sim_id=0, step0=0, **over):
    from paper_2605_20140_amd import sipf
    prm = dict(ic["params"])
    prm.update(over)
    p = sipf.make_params(precision=precision, flags=flags, sim_id=sim_id, step0=step0, **prm)
    return sipf.Simulation(p, ic["X0"], ic["a0"], ic["v0"], ic["m0"], ic["w0"])


def rel_errors(got, ref):
    d = got - ref
    l2 = np.linalg.norm(d) / max(np.linalg.norm(ref), 1e-300)
    mx = np.abs(d).max() / max(np.abs(ref).max(), 1e-300)
    return l2, mx


def min_image(d, L=1.0):
    return d - L * np.round(d / L)


def compare_state(out, ref, tol, L=1.0, fields=("v", "m", "w")):
    """Return a dict of errors and assert all are within tol."""
    errs = {}
    for f in fields:
        assert np.all(np.isfinite(out[f])) and np.all(np.isfinite(getattr(ref, f))), f
        errs[f] = rel_errors(out[f], getattr(ref, f))
    if ref.X.shape[0]:
        assert np.all(np.isfinite(out["X"])) and np.all(np.isfinite(out["a"]))
        assert np.all(np.isfinite(ref.X)) and np.all(np.isfinite(ref.a))
        errs["X"] = np.abs(min_image(out["X"] - ref.X, L)).max() / L
        errs["a"] = np.abs(out["a"] / ref.a - 1.0).max()
    bad = {k: v for k, v in errs.items() if (max(v) if isinstance(v, tuple) else v) > tol}
    assert not bad, f"errors above {tol}: {bad}"
    return errs


def gradient_tolerance(v, grad, L, precision):
    """Tolerance of the spectral gradient, an intermediate the state tolerances do not cover.
    Rounding in the working precision (unit u = 2^-24 or 2^-53: the stored v and the
    transforms, whose rms error grows like sqrt(log2 N^d)) is white across the spectrum, and
    the derivative multiplies each frequency by (2 pi / L) |q_j|, whose rms over the grid is
    (2 pi / L) N / (2 sqrt 3); relative to |grad v| that noise is
    u sqrt(log2 N^d) (2 pi / L) N / (2 sqrt 3) |v| / |grad v|.  Twice that, and never below
    the state tolerance (1e-4 float32, 1e-10 float64), is the bound: it grows linearly with N
    (float32 at 512^3: 1.3e-3)."""
    N, d = v.shape[0], v.ndim
    u = 2.0 ** -24 if precision else 2.0 ** -53
    amp = (2.0 * np.pi / L) * N / (2.0 * np.sqrt(3.0))
    ratio = np.linalg.norm(v) / np.linalg.norm(np.stack(grad))
    return max(1e-4 if precision else 1e-10,
               2.0 * u * np.sqrt(np.log2(float(N) ** d)) * amp * ratio)
