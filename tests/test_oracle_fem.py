"""Pins of oracle.fem and oracle.qoi (Sections 3.1-3.2, 4)."""

import math

import numpy as np
import pytest
from scipy.fft import dstn, idstn

from oracle import fem, qoi


def test_constant_coefficient_is_textbook_five_point_laplacian():
    m = 6
    A, b = fem.assemble(np.full((m + 1) ** 2, 2.5), m)
    A = A.toarray()
    w = m + 1
    for j in range(1, m):
        for i in range(1, m):
            p = i + w * j
            row = np.zeros(w * w)
            row[p] = 4.0
            for q in (p - 1, p + 1, p - w, p + w):
                row[q] = -1.0
            np.testing.assert_allclose(A[p], 2.5 * row, atol=1e-14)
    np.testing.assert_allclose(A, A.T, atol=1e-15)
    np.testing.assert_allclose(A.sum(axis=1), 0, atol=1e-13)
    h = 1.0 / m
    np.testing.assert_allclose(b.reshape(w, w)[1:-1, 1:-1], h * h, rtol=1e-14)
    assert abs(b.sum() - 1.0) < 1e-14


def test_variable_coefficient_five_point_form():
    # nodal quadrature on the right-diagonal mesh: only axis-aligned couplings,
    # conductance of edge (i,j)-(i+1,j) = (2k_ij + 2k_i+1,j + k_i+1,j+1 + k_i,j-1)/6
    m = 5
    rng = np.random.default_rng(0)
    k = rng.uniform(0.5, 2.0, (m + 1) ** 2)
    A = fem.assemble(k, m)[0].toarray()
    K = k.reshape(m + 1, m + 1)  # [j, i]
    w = m + 1
    for j in range(1, m):
        for i in range(1, m - 1):
            cx = (2 * K[j, i] + 2 * K[j, i + 1] + K[j + 1, i + 1] + K[j - 1, i]) / 6
            assert abs(A[i + w * j, i + 1 + w * j] + cx) < 1e-14
    for j in range(1, m - 1):
        for i in range(1, m):
            cy = (2 * K[j, i] + 2 * K[j + 1, i] + K[j + 1, i + 1] + K[j, i - 1]) / 6
            assert abs(A[i + w * j, i + w * (j + 1)] + cy) < 1e-14
            assert abs(A[i + w * j, i + 1 + w * (j + 1)]) < 1e-15


def test_poisson_solution_equals_discrete_sine_transform_solve():
    m = 16
    u, _, _ = fem.solve(np.ones((m + 1) ** 2), m)
    h = 1.0 / m
    b = np.full((m - 1, m - 1), h * h)
    kk = np.arange(1, m)
    lam = 4 - 2 * np.cos(np.pi * kk / m)[None, :] - 2 * np.cos(np.pi * kk / m)[:, None]
    ref = idstn(dstn(b, type=1) / lam, type=1)
    np.testing.assert_allclose(u[1:-1, 1:-1], ref, rtol=1e-12)


def test_integral_of_poisson_solution_converges_at_h2():
    # int u for -Lap u = 1 on the unit square: sum over odd j,k of 64/(pi^6 j^2 k^2 (j^2+k^2))
    J = np.arange(1, 4001, 2, dtype=float)
    exact = float((64 / math.pi ** 6) * np.sum(1.0 / (J[:, None] ** 2 * J[None, :] ** 2
                                                     * (J[:, None] ** 2 + J[None, :] ** 2))))
    assert abs(exact - 0.035144253736) < 1e-9
    errs = []
    for m in (16, 32, 64):
        u, _, _ = fem.solve(np.ones((m + 1) ** 2), m)
        errs.append(abs(qoi.integral(u, m) - exact))
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_manufactured_solution_second_order():
    # u* = sin(pi x) sin(pi y), k = 1 + x y^2, f = -div(k grad u*)
    def data(m):
        h = 1.0 / m
        x, y = np.meshgrid(np.arange(m + 1) * h, np.arange(m + 1) * h, indexing="xy")
        k = 1 + x * y * y
        ux = math.pi * np.cos(math.pi * x) * np.sin(math.pi * y)
        uy = math.pi * np.sin(math.pi * x) * np.cos(math.pi * y)
        lap = -2 * math.pi ** 2 * np.sin(math.pi * x) * np.sin(math.pi * y)
        f = -(y * y * ux + 2 * x * y * uy + k * lap)
        return k.ravel(), f.ravel(), (np.sin(math.pi * x) * np.sin(math.pi * y))
    errs = []
    for m in (16, 32, 64):
        k, f, ue = data(m)
        u, _, _ = fem.solve(k, m, fem.DIRICHLET0, f)
        errs.append(np.abs(u - ue).max())
    assert 3.3 < errs[0] / errs[1] < 4.7 and 3.3 < errs[1] / errs[2] < 4.7


def test_dense_solve_tiny_mesh():
    m = 4
    rng = np.random.default_rng(1)
    k = np.exp(rng.normal(size=(m + 1) ** 2))
    for bc in (fem.DIRICHLET0, fem.FLOWCELL):
        u, A, b = fem.solve(k, m, bc)
        fixed, val = fem.dirichlet_nodes(m, bc)
        M = A.toarray()
        rhs = b.copy()
        M[fixed] = 0
        M[fixed, np.flatnonzero(fixed)] = 1
        rhs[fixed] = val[fixed]
        np.testing.assert_allclose(u.ravel(), np.linalg.solve(M, rhs), rtol=1e-12, atol=1e-14)


def test_flowcell_flux_balance():
    m = 32
    rng = np.random.default_rng(2)
    k = np.exp(rng.normal(size=(m + 1) ** 2))
    u, A, b = fem.solve(k, m, fem.FLOWCELL, 1.0)
    res = b - A @ u.ravel()
    i = np.arange((m + 1) ** 2) % (m + 1)
    inflow = -res[i == 0].sum()
    out = qoi.outflux(u, m, A, b)
    assert abs(out - (inflow + 1.0)) < 1e-10


def test_qoi_exact_on_linear_data():
    m = 8
    h = 1.0 / m
    x, y = np.meshgrid(np.arange(m + 1) * h, np.arange(m + 1) * h, indexing="xy")
    assert abs(qoi.integral(np.ones((m + 1, m + 1)), m) - 1.0) < 1e-14
    assert abs(qoi.l2(np.ones((m + 1, m + 1)), m) - 1.0) < 1e-14
    assert abs(qoi.integral(x, m) - 0.5) < 1e-14
    assert abs(qoi.l2(x, m) - math.sqrt(1.0 / 3.0)) < 1e-14
    lin = 0.3 + 2 * x - 0.7 * y
    for px, py in ((7 / 15, 7 / 15), (0.1, 0.93), (1.0, 1.0), (0.0, 0.0)):
        assert abs(qoi.point(lin, m, px, py) - (0.3 + 2 * px - 0.7 * py)) < 1e-14
