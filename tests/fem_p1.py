"""Independent P1 finite-element assembly on triangles, used only to pin the
oracle's operator (App. A.1 of the paper: P1 elements on a uniform
rectangular grid split into triangles, nodal quadrature for the mass and
boundary terms).

This is element-by-element assembly from barycentric gradients, a different
computation from the oracle's edge-coupling (five-point) form.  The two agree
only if the paper's statement that S is the five-point Laplacian holds and the
oracle's weights are right.
"""
import numpy as np
import scipy.sparse as sp


def _triangles(nx, nz, diagonal):
    """Split each cell into two right triangles along '/' or '\\'."""
    tris = []
    for j in range(nz - 1):
        for i in range(nx - 1):
            a = j * nx + i          # (i, j)
            b = a + 1               # (i+1, j)
            c = a + nx              # (i, j+1)
            d = c + 1               # (i+1, j+1)
            if diagonal == "/":
                tris += [(a, b, d), (a, d, c)]
            else:
                tris += [(a, b, c), (b, d, c)]
    return tris


def assemble(nx, nz, hx, hz, diagonal="/"):
    """Return (S, mass, bnd): stiffness (sparse), lumped-mass weights d_k and
    boundary weights b_k, all from element and boundary-edge loops."""
    N = nx * nz
    xy = np.array([[(k % nx) * hx, (k // nx) * hz] for k in range(N)])
    rows, cols, vals = [], [], []
    mass = np.zeros(N)
    for t in _triangles(nx, nz, diagonal):
        P = xy[list(t)]
        J = np.array([P[1] - P[0], P[2] - P[0]]).T          # 2x2
        area = 0.5 * abs(np.linalg.det(J))
        # gradients of the barycentric coordinates
        Ginv = np.linalg.inv(J)
        grads = np.vstack([-Ginv.sum(axis=0), Ginv[0], Ginv[1]])   # 3 x 2
        K = area * grads @ grads.T
        for p in range(3):
            mass[t[p]] += area / 3.0       # vertex (nodal) quadrature of int phi_p
            for q in range(3):
                rows.append(t[p]); cols.append(t[q]); vals.append(K[p, q])
    S = sp.csr_matrix((vals, (rows, cols)), shape=(N, N))
    S.sum_duplicates()
    bnd = np.zeros(N)
    edges = []
    for i in range(nx - 1):
        edges.append((i, i + 1, hx))                                   # top
        edges.append(((nz - 1) * nx + i, (nz - 1) * nx + i + 1, hx))   # bottom
    for j in range(nz - 1):
        edges.append((j * nx, (j + 1) * nx, hz))                       # left
        edges.append((j * nx + nx - 1, (j + 1) * nx + nx - 1, hz))    # right
    for a, b, L in edges:
        bnd[a] += L / 2.0          # nodal quadrature on the boundary edge
        bnd[b] += L / 2.0
    return S, mass, bnd


def operator(nx, nz, hx, hz, m, omega):
    """A = S - w^2 diag(d m) - i w diag(b sqrt m), with d the mean of the two
    triangulation directions' lumped masses (the corner reading)."""
    S1, d1, b1 = assemble(nx, nz, hx, hz, "/")
    S2, d2, b2 = assemble(nx, nz, hx, hz, "\\")
    d = 0.5 * (d1 + d2)
    return (S1.astype(complex) - sp.diags(omega ** 2 * d * m + 1j * omega * b1 * np.sqrt(m))).tocsr(), S1, S2, d, b1


def boundary_edges(nx, nz, hx, hz):
    """(node_a, node_b, length, outward normal) of every boundary edge."""
    out = []
    for i in range(nx - 1):
        out.append((i, i + 1, hx, (0.0, -1.0)))
        out.append(((nz - 1) * nx + i, (nz - 1) * nx + i + 1, hx, (0.0, 1.0)))
    for j in range(nz - 1):
        out.append((j * nx, (j + 1) * nx, hz, (-1.0, 0.0)))
        out.append((j * nx + nx - 1, (j + 1) * nx + nx - 1, hz, (1.0, 0.0)))
    return out
