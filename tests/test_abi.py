"""The C ABI library loads, exports every symbol include/sipf.h declares, and rejects
invalid parameters and inputs before touching a device (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2605_20140_amd import sipf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sipf.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(sipf_\w+)\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    L = sipf.lib()
    names = _declared()
    assert set(names) == set(sipf.EXPORTS), names
    for n in names:
        assert hasattr(L, n), n


def test_struct_sizes_match_header():
    # sipf_params: 8+4+4+8+8+7*8+3*8+4*4+8 = 136; sipf_diag: 11 doubles + 4 int64 = 120
    assert ctypes.sizeof(sipf.Params) == 136
    assert ctypes.sizeof(sipf.Diag) == 120


def _p(**kw):
    base = dict(N=16, P=1000, dt=1e-3)
    base.update(kw)
    return sipf.make_params(**base)


@pytest.mark.parametrize("bad", [dict(N=12), dict(N=2), dict(N=1024), dict(P=-1),
                                 dict(P=1 << 32), dict(dt=0.0), dict(dt=0.6),
                                 dict(L=-1.0), dict(D_u=-1e-3), dict(chi=float("nan")),
                                 dict(precision=2), dict(deposit_order=3),
                                 dict(flags=0x80 | 0x100), dict(flags=0x4000),
                                 dict(H0=-1.0), dict(flags=0x100), dict(dim=1), dict(dim=4),
                                 dict(dim=2, N=2048, precision=1),
                                 dict(dim=2, deposit_order=4)])
def test_state_bytes_rejects_invalid_params(bad):
    with pytest.raises(sipf.SipfError) as e:
        sipf.state_bytes(_p(**bad))
    assert e.value.code == -1


def test_state_bytes_scales():
    b64 = sipf.state_bytes(_p(N=64, P=1 << 20))
    b32 = sipf.state_bytes(_p(N=64, P=1 << 20, precision=1))
    assert b32 < b64
    # particles: two sets of (3 s + 8 + 4) bytes + an 8-byte binning key; grid: s N^3 times
    # (2 ubar buffers + v, m, w + 2 four-component gather arrays) real + 5 half spectra
    N, P = 64, 1 << 20
    expect64 = P * (2 * (24 + 12) + 8) + N ** 3 * 13 * 8 + 5 * (N // 2 + 1) * N * N * 16
    assert expect64 <= b64 < expect64 + 64 * 1024
    assert sipf.state_bytes(_p(P=0)) > 0


def _init(params, X0, a0, v0, m0, w0, nbytes=None, ws=256):
    L = sipf.lib()
    h = ctypes.c_void_p()
    if nbytes is None:
        nbytes = sipf.state_bytes(params)
    dp = sipf._dptr
    return L.sipf_init(ctypes.byref(params), ctypes.c_void_p(ws), nbytes, None,
                       dp(X0), dp(a0), dp(v0), dp(m0), dp(w0), ctypes.byref(h))


def _inputs(N=8, P=10):
    rng = np.random.default_rng(0)
    X0 = np.ascontiguousarray(rng.uniform(0, 1, (3, P)))
    return (X0, np.full(P, 1.0 / P), np.ones(N ** 3), np.zeros(N ** 3), np.ones(N ** 3))


@pytest.mark.parametrize("what", ["X_nan", "a_zero", "a_neg", "v_neg", "m_nan", "w_nan"])
def test_init_rejects_invalid_inputs(what):
    N, P = 8, 10
    X0, a0, v0, m0, w0 = _inputs(N, P)
    if what == "X_nan":
        X0[1, 3] = np.nan
    elif what == "a_zero":
        a0[2] = 0.0
    elif what == "a_neg":
        a0[2] = -1.0
    elif what == "v_neg":
        v0[5] = -1e-3
    elif what == "m_nan":
        m0[0] = np.inf
    elif what == "w_nan":
        w0[7] = np.nan
    rc = _init(_p(N=N, P=P), X0, a0, v0, m0, w0)
    assert rc == -1, sipf.lib().sipf_last_error()


def test_init_rejects_small_or_misaligned_workspace():
    N, P = 8, 10
    X0, a0, v0, m0, w0 = _inputs(N, P)
    prm = _p(N=N, P=P)
    need = sipf.state_bytes(prm)
    assert _init(prm, X0, a0, v0, m0, w0, nbytes=need - 1) == -2
    assert b"needs" in sipf.lib().sipf_last_error()
    assert _init(prm, X0, a0, v0, m0, w0, ws=128) == -1


def test_null_handles():
    L = sipf.lib()
    assert L.sipf_step(None, 1) == -1
    assert L.sipf_fields(None, None, None, None, None, None, None) == -1
    L.sipf_destroy(None)
    arr = (ctypes.c_void_p * 1)(None)
    assert L.sipf_step_batch(arr, 1, 1) == -1
    assert L.sipf_step_batch(arr, 0, 1) == -1


def test_two_dimensional_state_bytes():
    """dim = 2: N^2 grids and two coordinates per particle; N up to 1024."""
    b2 = sipf.state_bytes(_p(N=64, P=1 << 16, dim=2))
    b3 = sipf.state_bytes(_p(N=64, P=1 << 16))
    assert b2 < b3
    N, P = 64, 1 << 16
    expect = P * (2 * (16 + 12) + 8) + N ** 2 * 13 * 8 + 5 * (N // 2 + 1) * N * 16
    assert expect <= b2 < expect + 64 * 1024
    assert sipf.state_bytes(_p(N=1024, P=100, dim=2)) > 0
    assert sipf.state_bytes(_p(N=512, P=100, dim=3)) == sipf.state_bytes(_p(N=512, P=100, dim=0))


def test_noalloc_batch_rejects_more_than_64_simulations():
    L = sipf.lib()
    arr = (ctypes.c_void_p * 65)()
    assert L.sipf_step_batch_noalloc(arr, 65, 1) == -1
    assert b"at most 64" in L.sipf_last_error()
    assert L.sipf_step_batch_noalloc(arr, 0, 1) == -1
