"""Linear elasticity on a structured hexahedral mesh: the 27-point, 3-dof
symmetric positive definite stencil of the L D L^T workload.

Trilinear (Q1) unit-cube elements, isotropic material with Poisson ratio nu
and per-element Young modulus E_e ~ lognormal(0, sigma), element stiffness
integrated with the 2x2x2 Gauss rule.  The mesh has n nodes per side
((n-1)^3 elements); the outer layer of nodes is clamped (removed), leaving
(n-2)^3 free nodes and 3 (n-2)^3 unknowns, numbered node by node
(x fastest, then y, then z) and component by component (u_x, u_y, u_z).
Only input construction lives here: the element integral, the draws and the
assembly into CSC.
"""
from __future__ import annotations

import numpy as np

from .stencils import Problem, _coo_to_csc


def material_matrix(nu: float = 0.3, E: float = 1.0) -> np.ndarray:
    """6x6 isotropic stress-strain matrix in Voigt order (xx, yy, zz, yz, xz,
    xy) with engineering shear strains."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[[0, 1, 2], [0, 1, 2]] = lam + 2.0 * mu
    D[[3, 4, 5], [3, 4, 5]] = mu
    return D


def _corner(a: int):
    return a & 1, (a >> 1) & 1, (a >> 2) & 1


def strain_matrix(xi: float, eta: float, zeta: float) -> np.ndarray:
    """6x24 strain-displacement matrix of the unit-cube Q1 element at a point
    of [0, 1]^3; local node a sits at corner (a & 1, (a >> 1) & 1, a >> 2)."""
    p = (xi, eta, zeta)
    B = np.zeros((6, 24))
    for a in range(8):
        c = _corner(a)
        f = [p[d] if c[d] else 1.0 - p[d] for d in range(3)]
        df = [1.0 if c[d] else -1.0 for d in range(3)]
        gx, gy, gz = df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2]
        k = 3 * a
        B[0, k] = gx
        B[1, k + 1] = gy
        B[2, k + 2] = gz
        B[3, k + 1], B[3, k + 2] = gz, gy
        B[4, k], B[4, k + 2] = gz, gx
        B[5, k], B[5, k + 1] = gy, gx
    return B


def element_stiffness(nu: float = 0.3) -> np.ndarray:
    """24x24 stiffness of the unit-cube Q1 element with E = 1 (2x2x2 Gauss)."""
    D = material_matrix(nu)
    g = (0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0))
    K = np.zeros((24, 24))
    for x in g:
        for y in g:
            for z in g:
                B = strain_matrix(x, y, z)
                K += 0.125 * B.T @ D @ B
    return 0.5 * (K + K.T)


def elasticity3d(n: int, seed: int, sigma: float = 0.5, nu: float = 0.3) -> Problem:
    """Clamped Q1 elasticity matrix on an n^3-node mesh (n >= 3): element
    moduli drawn in element order (x fastest) from lognormal(0, sigma)."""
    n = int(n)
    if n < 3:
        raise ValueError("need at least 3 nodes per side")
    rng = np.random.default_rng(seed)
    ne1 = n - 1
    E = rng.lognormal(0.0, sigma, ne1 ** 3)
    Ke = element_stiffness(nu)
    # free-node numbering: interior nodes only, x fastest
    coord = np.arange(n)
    inner = (coord > 0) & (coord < n - 1)
    free = -np.ones((n, n, n), dtype=np.int64)   # [z, y, x]
    m = n - 2
    free[np.ix_(inner, inner, inner)] = np.arange(m ** 3).reshape(m, m, m)
    ez, ey, ex = np.meshgrid(np.arange(ne1), np.arange(ne1), np.arange(ne1), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()   # element order: x fastest
    dof = np.empty((ne1 ** 3, 24), dtype=np.int64)
    for a in range(8):
        cx, cy, cz = _corner(a)
        node = free[ez + cz, ey + cy, ex + cx]
        for comp in range(3):
            dof[:, 3 * a + comp] = np.where(node >= 0, 3 * node + comp, -1)
    rows = np.broadcast_to(dof[:, :, None], (len(E), 24, 24))
    cols = np.broadcast_to(dof[:, None, :], (len(E), 24, 24))
    vals = E[:, None, None] * Ke[None, :, :]
    keep = (rows >= 0) & (cols >= 0)
    N = 3 * m ** 3
    colptr, rowind, values = _coo_to_csc(N, rows[keep], cols[keep], vals[keep])
    return Problem(N, colptr, rowind, values, name="elasticity3d_q1_%d^3" % m,
                   meta={"nodes": n, "free_nodes": m ** 3, "sigma": sigma, "nu": nu, "seed": seed})
