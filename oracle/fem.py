"""P1 finite elements for -div(k grad u) = f on (0,1)^2 (oracle; test only).

Section 3.1 (the Darcy model and its boundary conditions) and Section 3.2
(piecewise-linear elements; the system is assembled with a nodal
quadrature rule so that u_h depends on k only through its grid values).

Readings of the paper taken here:
* mesh: the (m+1)^2 vertex grid, each square split along the diagonal
  (i, j)-(i+1, j+1);
* quadrature: trapezoidal (vertex) rule on each triangle, so a triangle's
  stiffness is its P1 stiffness times the mean of k over its 3 vertices and
  the load of a vertex is f |T|/3 summed over its triangles;
* DIRICHLET0: u = 0 on the whole boundary (the analysis setting);
  FLOWCELL: u = 1 at x1 = 0, u = 0 at x1 = 1, natural (zero Neumann)
  condition at x2 = 0 and x2 = 1.

Assembly is element by element from the vertex coordinates and the
barycentric gradients; the solve is scipy's sparse direct solver.

Pins (tests/test_oracle_fem.py): constant k gives the textbook 5-point
Laplacian, solved exactly by the discrete sine transform; the integral of
u for -Lap u = 1 converges at O(h^2) to the Fourier-series value; a
manufactured smooth solution converges at O(h^2); dense solve on tiny
meshes; flow-cell flux balance (outflow = inflow + integral of f);
symmetric matrix with zero row sums.
"""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

DIRICHLET0 = 0
FLOWCELL = 1


def triangles(m):
    """Vertex index triples (x index fastest: p = i + (m+1) j) of the mesh."""
    i, j = np.meshgrid(np.arange(m), np.arange(m), indexing="xy")
    i = i.ravel()
    j = j.ravel()
    w = m + 1
    p00 = i + w * j
    p10 = (i + 1) + w * j
    p11 = (i + 1) + w * (j + 1)
    p01 = i + w * (j + 1)
    t1 = np.stack([p00, p10, p11], axis=1)
    t2 = np.stack([p00, p11, p01], axis=1)
    return np.concatenate([t1, t2], axis=0)


def _geometry(m, tri):
    h = 1.0 / m
    w = m + 1
    x = (tri % w) * h
    y = (tri // w) * h
    b11 = x[:, 1] - x[:, 0]
    b12 = x[:, 2] - x[:, 0]
    b21 = y[:, 1] - y[:, 0]
    b22 = y[:, 2] - y[:, 0]
    det = b11 * b22 - b12 * b21
    area = 0.5 * np.abs(det)
    # rows of B^{-T}: gradients of barycentric coordinates 1 and 2
    g1 = np.stack([b22, -b12], axis=1) / det[:, None]
    g2 = np.stack([-b21, b11], axis=1) / det[:, None]
    g0 = -g1 - g2
    grads = np.stack([g0, g1, g2], axis=1)  # (ntri, 3, 2)
    return area, grads


def assemble(k, m, f=1.0):
    """Full stiffness matrix A (CSR, all (m+1)^2 vertices) and load b.

    f is a constant or an array of nodal values."""
    k = np.asarray(k, dtype=np.float64).reshape(-1)
    tri = triangles(m)
    area, grads = _geometry(m, tri)
    kbar = k[tri].mean(axis=1)
    loc = np.einsum("tad,tbd->tab", grads, grads) * (area * kbar)[:, None, None]
    rows = np.repeat(tri, 3, axis=1).ravel()
    cols = np.tile(tri, (1, 3)).ravel()
    N = (m + 1) ** 2
    A = sp.csr_matrix((loc.ravel(), (rows, cols)), shape=(N, N))
    # load: trapezoidal rule on each triangle, int_T f phi_p ~ |T|/3 f(p)
    fv = np.broadcast_to(np.asarray(f, dtype=np.float64).reshape(-1), (N,)) \
        if np.ndim(f) else np.full(N, float(f))
    b = np.zeros(N)
    np.add.at(b, tri.ravel(), np.repeat(area / 3.0, 3) * fv[tri.ravel()])
    return A, b


def dirichlet_nodes(m, bc):
    """(fixed-node mask, prescribed values) on the full vertex grid."""
    i, j = np.meshgrid(np.arange(m + 1), np.arange(m + 1), indexing="xy")
    i = i.ravel()
    j = j.ravel()
    if bc == DIRICHLET0:
        fixed = (i == 0) | (i == m) | (j == 0) | (j == m)
        val = np.zeros(fixed.shape)
    elif bc == FLOWCELL:
        fixed = (i == 0) | (i == m)
        val = np.where(i == 0, 1.0, 0.0)
    else:
        raise ValueError("unknown boundary condition")
    return fixed, val


def solve(k, m, bc=DIRICHLET0, f=1.0):
    """Nodal solution u (shape (m+1, m+1), [j, i]) and (A, b)."""
    A, b = assemble(k, m, f)
    fixed, val = dirichlet_nodes(m, bc)
    free = ~fixed
    u = np.where(fixed, val, 0.0)
    rhs = b[free] - A[free][:, fixed] @ val[fixed]
    Aii = A[free][:, free].tocsc()
    u[free] = spla.spsolve(Aii, rhs)
    return u.reshape(m + 1, m + 1), A, b
