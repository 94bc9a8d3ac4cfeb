"""CPU checks of the quasi-Monte Carlo host code in the library: the CBC
generating vector of ces_lattice_cbc equals the oracle's bit for bit (an
integer decision taken on exactly summed, truncated terms on both sides),
and the lattice entry points reject bad arguments without a device."""

import ctypes
import os

import numpy as np
import pytest

from oracle import qmc as oqmc


@pytest.fixture(scope="module")
def lib():
    from paper_2306_13493_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2306_13493_amd import build
        build.build()
    return _lib.load()


def cbc(lib, p, gamma):
    g = np.ascontiguousarray(gamma, dtype=np.float64)
    z = np.zeros(g.size, dtype=np.uint32)
    rc = lib.ces_lattice_cbc(p, g.size, g.ctypes.data_as(ctypes.c_void_p), z.ctypes.data_as(ctypes.c_void_p))
    return rc, [int(v) for v in z]


@pytest.mark.parametrize("p,gamma", [
    (0, [1.0]), (1, [0.5, 0.5]), (4, [1.0, 0.5, 0.25]),
    (7, list(0.9 ** np.arange(12))),
    (10, list(1.0 / (1.0 + np.arange(24)) ** 2)),
    # eigenvalue-like weights scaled to sum one, with exact ties
    (9, list(np.repeat([0.2, 0.1, 0.05, 0.025], 4) / 1.5)),
])
def test_cbc_matches_oracle(lib, p, gamma):
    rc, z = cbc(lib, p, gamma)
    assert rc == 0
    assert z == oqmc.cbc(p, gamma)


def test_cbc_rejects_bad_arguments(lib):
    assert cbc(lib, 21, [1.0])[0] == -1
    assert cbc(lib, -1, [1.0])[0] == -1
    assert cbc(lib, 4, [-0.1])[0] == -1
    assert cbc(lib, 4, [float("nan")])[0] == -1
    assert cbc(lib, 4, [40.0, 30.0])[0] == -1
    assert lib.ces_lattice_cbc(4, 0, None, None) == -1


def test_lattice_entry_points_reject_bad_arguments(lib):
    from paper_2306_13493_amd import _lib
    assert ctypes.sizeof(_lib.MlqmcOpts) == 56
    o = _lib.MlqmcOpts()
    lib.ces_mlqmc_opts_default(ctypes.byref(o))
    assert o.struct_size == 56 and o.n_pilot == 1 and o.theta == 0.5 and o.l_start == 2
    r = _lib.MlmcResult()
    assert lib.ces_mlqmc_run(None, None, None, 1, ctypes.byref(o), None, ctypes.byref(r)) == -1
    assert lib.ces_plan_set_lattice(None, 1, None, None, 4) == -1
    assert lib.ces_plan_set_lattice_default(None, 1, 4, 4) == -1
    assert lib.ces_plan_lattice_order(None, 1, None, None) == -1
