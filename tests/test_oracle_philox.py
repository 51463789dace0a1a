"""Pins of the oracle's Philox4x32-10 and Box-Muller normals.

* bit-exact agreement with the independent Philox engine that ships as a C++ header with
  PyTorch (at::philox_engine: key = seed, counter = (offset_lo, offset_hi, subsequence_lo,
  subsequence_hi)), compiled here with g++;
* the uniforms lie strictly in (0, 1); the normals have mean 0, variance 1 and Gaussian tails.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import philox

_SRC = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
int main() {
  unsigned long long seed, sub, off;
  while (scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
    at::philox_engine e(seed, sub, off);
    unsigned a = e(), b = e(), c = e(), d = e();
    printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
"""


def _torch_include():
    import torch
    return os.path.join(os.path.dirname(torch.__file__), "include")


@pytest.fixture(scope="module")
def torch_philox():
    gxx = shutil.which("g++")
    inc = _torch_include()
    if gxx is None or not os.path.exists(os.path.join(inc, "ATen/core/PhiloxRNGEngine.h")):
        pytest.skip("g++ or torch's Philox header not available")
    d = tempfile.mkdtemp()
    src = os.path.join(d, "ph.cpp")
    exe = os.path.join(d, "ph")
    with open(src, "w") as f:
        f.write(_SRC)
    subprocess.run([gxx, "-std=c++17", "-O1", "-I" + inc, src, "-o", exe], check=True)

    def run(triples):
        inp = "\n".join(f"{s} {b} {o}" for s, b, o in triples) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True)
        return np.array([[int(t) for t in line.split()] for line in out.stdout.splitlines()],
                        dtype=np.uint64)
    yield run
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_library_engine(torch_philox):
    rng = np.random.default_rng(123)
    triples = [(0, 0, 0), (2**64 - 1, 2**64 - 1, 2**64 - 1), (5, 7, 12345678901)]
    for _ in range(200):
        triples.append((int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2)),
                        int(rng.integers(0, 2**63)), int(rng.integers(0, 2**63))))
    ref = torch_philox(triples)
    for (seed, sub, off), r in zip(triples, ref):
        got = philox.philox4x32_10(off & 0xFFFFFFFF, off >> 32, sub & 0xFFFFFFFF, sub >> 32,
                                   seed & 0xFFFFFFFF, seed >> 32)
        assert [int(g) for g in got] == [int(x) for x in r], (seed, sub, off)


def test_philox_vectorised_equals_scalar():
    p = np.arange(1000, dtype=np.uint64)
    vec = philox.philox4x32_10(p, 17, 3, 0, 99, 1)
    for i in (0, 1, 500, 999):
        sc = philox.philox4x32_10(i, 17, 3, 0, 99, 1)
        assert all(int(vec[k][i]) == int(sc[k]) for k in range(4))


def test_uniforms_open_interval():
    u = philox.uniforms(np.array([0, 2**32 - 1], dtype=np.uint64))
    assert u[0] > 0.0 and u[1] < 1.0
    assert u[0] == 2.0 ** -33 and u[1] == 1.0 - 2.0 ** -33


def test_normals_statistics():
    P = 1 << 20
    z = philox.step_normals(np.arange(P), 3, 0, 7)
    assert z.shape == (P, 3)
    for j in range(3):
        assert abs(z[:, j].mean()) < 5.0 / np.sqrt(P)
        assert abs(z[:, j].var() - 1.0) < 5.0 * np.sqrt(2.0 / P)
        # P(|Z| > 3) = 0.0026998
        frac = np.mean(np.abs(z[:, j]) > 3.0)
        assert abs(frac - 0.0026998) < 5.0 * np.sqrt(0.0027 / P)
    # independent streams: different steps and sims are uncorrelated
    z2 = philox.step_normals(np.arange(P), 4, 0, 7)
    z3 = philox.step_normals(np.arange(P), 3, 1, 7)
    assert abs(np.mean(z[:, 0] * z2[:, 0])) < 5.0 / np.sqrt(P)
    assert abs(np.mean(z[:, 0] * z3[:, 0])) < 5.0 / np.sqrt(P)
    assert abs(np.mean(z[:, 0] * z[:, 1])) < 5.0 / np.sqrt(P)
