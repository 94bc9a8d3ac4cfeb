"""Pins of oracle.normals: Philox words, elementary functions, normal law."""

import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

from oracle import normals as nm

HERE = os.path.dirname(os.path.abspath(__file__))


def _rocrand_words(rows):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("hipcc / rocRAND headers not available")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "philox_ref")
        subprocess.run([hipcc, "-O1", "-o", exe, os.path.join(HERE, "philox_ref.cpp")],
                       check=True, capture_output=True, timeout=300)
        inp = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True, timeout=60)
    return np.array([[int(v) for v in line.split()] for line in out.stdout.strip().splitlines()],
                    dtype=np.uint64)


def test_philox_matches_rocrand_engine():
    rng = np.random.default_rng(7)
    rows = rng.integers(0, 2 ** 32, size=(300, 6), dtype=np.uint64)
    rows[0] = 0
    rows[1] = 2 ** 32 - 1
    rows[2, :4] = [5, 0, 0, 0]
    ref = _rocrand_words(rows)
    got = np.stack(nm.philox4x32_10(*[rows[:, i] for i in range(6)]), axis=1)
    np.testing.assert_array_equal(got, ref)


def _ulp_err(got, ref):
    return np.abs(got - ref) / np.spacing(np.maximum(np.abs(ref), np.finfo(float).tiny))


def test_ln_within_few_ulp():
    rng = np.random.default_rng(4)
    u = np.concatenate([rng.uniform(0, 1, 200000), 2.0 ** -np.arange(0, 54),
                        1 - 2.0 ** -np.arange(1, 54), np.array([1.0, 0.5, 0.7071067811865476])])
    u = u[u > 0]
    assert _ulp_err(nm.ln(u), np.log(u)).max() <= 4
    assert nm.ln(np.array([1.0]))[0] == 0.0


def test_sqrt_within_few_ulp():
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.uniform(0, 80, 200000), 2.0 ** np.arange(-60, 8), [0.0, 1.0, 4.0]])
    got = nm.sqrt(x)
    ref = np.sqrt(x)
    nz = x > 0
    assert _ulp_err(got[nz], ref[nz]).max() <= 2
    assert got[x == 0][0] == 0.0


def test_sincos_within_few_ulp_of_unit_scale():
    rng = np.random.default_rng(6)
    u = np.concatenate([rng.uniform(0, 1, 200000), np.arange(0, 64) / 64.0, [1 - 2.0 ** -53]])
    c, s = nm.sincos_2pi(u)
    # absolute error in units of the spacing at 1 (the relevant scale of cos/sin values)
    assert np.max(np.abs(c - np.cos(2 * np.pi * u))) <= 4 * np.spacing(1.0)
    assert np.max(np.abs(s - np.sin(2 * np.pi * u))) <= 4 * np.spacing(1.0)
    q = np.arange(0, 4) / 4.0
    cq, sq = nm.sincos_2pi(q)
    np.testing.assert_array_equal(cq, [1.0, 0.0, -1.0, 0.0])
    np.testing.assert_array_equal(sq, [0.0, 1.0, 0.0, -1.0])


def test_uniform_ranges():
    z = np.zeros(1, dtype=np.uint64)
    f = np.full(1, 0xFFFFFFFF, dtype=np.uint64)
    u1, u2 = nm.uniforms(z, z, z, z)
    assert u1[0] == 2.0 ** -53 and u2[0] == 0.0
    u1, u2 = nm.uniforms(f, f, f, f)
    assert u1[0] == 1.0 and u2[0] == 1.0 - 2.0 ** -53


def test_normal_law():
    e = np.arange(200000, dtype=np.uint64)
    g0, g1 = nm.normals(seed=12345, q=3, stream=1, e=e)
    for g in (g0, g1):
        assert abs(g.mean()) < 5 / np.sqrt(e.size)
        assert abs(g.var() - 1) < 5 * np.sqrt(2.0 / e.size)
        assert stats.kstest(g, "norm").pvalue > 1e-4
    assert abs(np.corrcoef(g0, g1)[0, 1]) < 5 / np.sqrt(e.size)
    # different counters give unrelated streams
    h0, _ = nm.normals(seed=12345, q=4, stream=1, e=e)
    assert abs(np.corrcoef(g0, h0)[0, 1]) < 5 / np.sqrt(e.size)
