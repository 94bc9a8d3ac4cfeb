"""Host build of the library's K_nu routine (paper_2306_13493_amd/csrc/
besselk.hpp, used by the device covariance kernel) against independent
values: mpmath's besselk at 40 digits and the closed forms of K_nu for
half-integer nu (Matern nu = 1/2, 3/2, 5/2)."""

import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2306_13493_amd", "csrc")


@pytest.fixture(scope="module")
def besselk(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("besselk")
    src = d / "bk.cpp"
    src.write_text('#include "besselk.hpp"\nextern "C" double bk(double nu, double x) '
                   '{ return ces::bessel_k(nu, x); }\n')
    lib = d / "libbk.so"
    subprocess.run([gxx, "-O2", "-shared", "-fPIC", "-I" + CSRC, str(src), "-o", str(lib)], check=True)
    h = ctypes.CDLL(str(lib))
    h.bk.restype = ctypes.c_double
    h.bk.argtypes = [ctypes.c_double, ctypes.c_double]
    return h.bk


XS = np.logspace(-8, np.log10(700.0), 120)


@pytest.mark.parametrize("nu", [0.2, 0.5, 1.0, 1.5, 2.0, 2.5, 3.7, 5.0])
def test_against_mpmath(besselk, nu):
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    worst = 0.0
    for x in XS[::2]:
        ref = mpmath.besselk(nu, x)
        worst = max(worst, float(abs(mpmath.mpf(besselk(nu, float(x))) - ref) / ref))
    assert worst <= 5e-15, worst


@pytest.mark.parametrize("nu,poly", [(0.5, lambda x: 1.0), (1.5, lambda x: 1.0 + 1.0 / x),
                                     (2.5, lambda x: 1.0 + 3.0 / x + 3.0 / x ** 2)])
def test_half_integer_closed_forms(besselk, nu, poly):
    for x in XS:
        ref = np.sqrt(np.pi / (2 * x)) * np.exp(-x) * poly(x)
        assert abs(besselk(nu, x) - ref) <= 5e-15 * ref, x


def test_small_argument_limit(besselk):
    # x^nu K_nu(x) -> 2^(nu-1) Gamma(nu) as x -> 0 (the Matern C(0) = sigma^2)
    from math import gamma
    for nu in (0.5, 1.0, 1.5, 2.3):
        x = 1e-9
        assert abs(x ** nu * besselk(nu, x) / (2 ** (nu - 1) * gamma(nu)) - 1) < 1e-8
