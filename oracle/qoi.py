"""Quantities of interest (oracle; test infrastructure only).

Section 3.1 names the pressure at a point and the L2 norm of u; Section 4
uses Q = u(7/15, 7/15) and Q = ||u||_{L2}; the benchmark configurations
also use the integral of u and the outflow through x1 = 1.  All are
evaluated on the P1 finite element function u_h:

* INTEGRAL: int u_h = sum_p u_p int phi_p (exact for P1).
* POINT: u_h(x*) by linear interpolation in the triangle containing x*.
* L2: sqrt(u^T M u) with the exact P1 mass matrix (|T|/12 [2 1 1; 1 2 1;
  1 1 2] per triangle).
* OUTFLUX: sum over the vertices on x1 = 1 of (b - A u)_p, the consistent
  (Galerkin) value of the outward flux -int k du/dx1 along x1 = 1.

Pins (tests/test_oracle_fem.py): integral and L2 of constant and linear
nodal data, exact interpolation of linear data at the point, flux balance.
"""

import numpy as np
import scipy.sparse as sp

from .fem import triangles, _geometry

INTEGRAL = 0
POINT = 1
L2 = 2
OUTFLUX = 3


def integral(u, m):
    tri = triangles(m)
    area, _ = _geometry(m, tri)
    w = np.zeros((m + 1) ** 2)
    np.add.at(w, tri.ravel(), np.repeat(area / 3.0, 3))
    return float(np.dot(w, np.asarray(u).reshape(-1)))


def mass_matrix(m):
    tri = triangles(m)
    area, _ = _geometry(m, tri)
    loc = np.array([[2.0, 1.0, 1.0], [1.0, 2.0, 1.0], [1.0, 1.0, 2.0]]) / 12.0
    vals = (area[:, None, None] * loc[None, :, :]).ravel()
    rows = np.repeat(tri, 3, axis=1).ravel()
    cols = np.tile(tri, (1, 3)).ravel()
    N = (m + 1) ** 2
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, N))


def l2(u, m):
    uu = np.asarray(u).reshape(-1)
    return float(np.sqrt(uu @ (mass_matrix(m) @ uu)))


def point(u, m, x, y):
    """P1 interpolation at (x, y) on the mesh of triangles()."""
    u = np.asarray(u).reshape(m + 1, m + 1)
    h = 1.0 / m
    i = min(int(np.floor(x / h)), m - 1)
    j = min(int(np.floor(y / h)), m - 1)
    sx = x / h - i
    sy = y / h - j
    if sx >= sy:  # triangle (i,j), (i+1,j), (i+1,j+1)
        return float((1 - sx) * u[j, i] + (sx - sy) * u[j, i + 1] + sy * u[j + 1, i + 1])
    # triangle (i,j), (i+1,j+1), (i,j+1)
    return float((1 - sy) * u[j, i] + sx * u[j + 1, i + 1] + (sy - sx) * u[j + 1, i])


def outflux(u, m, A, b):
    uu = np.asarray(u).reshape(-1)
    res = b - A @ uu
    i = np.arange((m + 1) ** 2) % (m + 1)
    return float(res[i == m].sum())


def evaluate(kind, u, m, A=None, b=None, x=7.0 / 15.0, y=7.0 / 15.0):
    if kind == INTEGRAL:
        return integral(u, m)
    if kind == POINT:
        return point(u, m, x, y)
    if kind == L2:
        return l2(u, m)
    if kind == OUTFLUX:
        return outflux(u, m, A, b)
    raise ValueError("unknown QoI")
