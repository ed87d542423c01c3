"""Finite-element layer of the oracle (test infrastructure only).

SIMP stiffness law (Sec. 1, Eq. 1), bilinear Q4 plane-stress and trilinear
Hex8 element matrices on unit elements by full Gauss quadrature, the global
system K u = f (Sec. 2, Eq. 2) with clamped DOFs removed and solved by a sparse
direct factorisation, the compliance c = f^T u and its gradient
dc/drho_e = -p rho_e^(p-1) (E0 - Emin) u_e^T K0_e u_e (self-adjoint compliance).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# two-point Gauss rule on [0, 1]: points 1/2 -+ 1/(2 sqrt 3), weights 1/2
_G = (0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0))
_W = (0.5, 0.5)


def simp_modulus(rho, p, E0, Emin):
    """Sec. 1, Eq. (1): E = Emin + rho^p (E0 - Emin)."""
    rho = np.asarray(rho, dtype=np.float64)
    return Emin + rho ** p * (E0 - Emin)


def material_matrix(dim, nu, E=1.0):
    """Hooke matrix: plane stress in 2D (strain order xx, yy, xy), isotropic
    3D (xx, yy, zz, yz, xz, xy), engineering shear strains."""
    if dim == 2:
        c = E / (1.0 - nu * nu)
        return c * np.array([[1.0, nu, 0.0], [nu, 1.0, 0.0], [0.0, 0.0, 0.5 * (1.0 - nu)]])
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[:3, :3] += 2.0 * mu * np.eye(3)
    D[3:, 3:] = mu * np.eye(3)
    return D


def corner_offsets(dim):
    """Element corners in local lexicographic order, x fastest."""
    return [tuple(reversed(c)) for c in itertools.product((0, 1), repeat=dim)]


def _shape_gradients(xi, dim):
    """d N_a / d x_d for the (bi/tri)linear shape functions of the unit element."""
    offs = corner_offsets(dim)
    g = np.zeros((len(offs), dim))
    for a, o in enumerate(offs):
        for d in range(dim):
            val = 1.0 if o[d] == 1 else -1.0
            for d2 in range(dim):
                if d2 != d:
                    val *= xi[d2] if o[d2] == 1 else (1.0 - xi[d2])
            g[a, d] = val
    return g


def strain_matrix(xi, dim):
    g = _shape_gradients(xi, dim)
    n = g.shape[0]
    if dim == 2:
        B = np.zeros((3, 2 * n))
        for a in range(n):
            B[0, 2 * a] = g[a, 0]
            B[1, 2 * a + 1] = g[a, 1]
            B[2, 2 * a] = g[a, 1]
            B[2, 2 * a + 1] = g[a, 0]
        return B
    B = np.zeros((6, 3 * n))
    for a in range(n):
        dx, dy, dz = g[a]
        B[0, 3 * a] = dx
        B[1, 3 * a + 1] = dy
        B[2, 3 * a + 2] = dz
        B[3, 3 * a + 1] = dz
        B[3, 3 * a + 2] = dy
        B[4, 3 * a] = dz
        B[4, 3 * a + 2] = dx
        B[5, 3 * a] = dy
        B[5, 3 * a + 1] = dx
    return B


def element_stiffness(dim, nu):
    """Unit-modulus element matrix K0 = sum_gp w B^T D B over the full Gauss rule."""
    D = material_matrix(dim, nu)
    n = dim * 2 ** dim
    K = np.zeros((n, n))
    for pt in itertools.product(range(2), repeat=dim):
        xi = [_G[i] for i in pt]
        w = np.prod([_W[i] for i in pt])
        B = strain_matrix(xi, dim)
        K += w * B.T @ D @ B
    return K


def node_shape(nel):
    return tuple(n + 1 for n in nel)


def element_nodes(nel):
    """[n_el, 2^dim] global node numbers of every element, elements and corners
    both lexicographic (x fastest)."""
    dim = len(nel)
    nn = node_shape(nel)
    strides = [int(np.prod(nn[:d])) for d in range(dim)]
    grids = np.meshgrid(*[np.arange(n) for n in nel[::-1]], indexing="ij")
    base = np.zeros(grids[0].shape, dtype=np.int64)
    for d in range(dim):
        base += grids[dim - 1 - d] * strides[d]
    base = base.ravel()
    offs = corner_offsets(dim)
    out = np.empty((base.size, len(offs)), dtype=np.int64)
    for a, o in enumerate(offs):
        out[:, a] = base + sum(o[d] * strides[d] for d in range(dim))
    return out


def element_dofs(nel):
    dim = len(nel)
    en = element_nodes(nel)
    return (dim * en[:, :, None] + np.arange(dim)[None, None, :]).reshape(en.shape[0], -1)


def assemble_global(nel, nu, E):
    """Sec. 2, Eq. (2): K = sum_e E_e K0 scattered by element DOFs (scipy CSR)."""
    dim = len(nel)
    K0 = element_stiffness(dim, nu)
    ed = element_dofs(nel)
    n = dim * int(np.prod(node_shape(nel)))
    rows = np.repeat(ed, ed.shape[1], axis=1).ravel()
    cols = np.tile(ed, (1, ed.shape[1])).ravel()
    vals = (np.asarray(E)[:, None] * K0.ravel()[None, :]).ravel()
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def direct_solve(K, f, fixed):
    """Solve K u = f with u = 0 on the clamped DOFs by sparse LU of the free block."""
    n = K.shape[0]
    free = np.setdiff1d(np.arange(n), fixed)
    Kff = K[free][:, free].tocsc()
    u = np.zeros(n)
    u[free] = spla.splu(Kff).solve(f[free])
    return u


def solve_problem(prob):
    """Global direct solution u* of a workloads.Problem."""
    E = simp_modulus(prob.rho, prob.p, prob.E0, prob.Emin)
    K = assemble_global(prob.nel, prob.nu, E)
    return direct_solve(K, prob.load(), prob.fixed_dofs())


def compliance(f, u):
    return float(np.dot(f, u))


def compliance_gradient(prob, u):
    """dc/drho_e = -p rho_e^(p-1) (E0 - Emin) u_e^T K0 u_e."""
    K0 = element_stiffness(prob.dim, prob.nu)
    ue = u[element_dofs(prob.nel)]
    energy = np.einsum("ei,ij,ej->e", ue, K0, ue)
    return -prob.p * prob.rho ** (prob.p - 1.0) * (prob.E0 - prob.Emin) * energy
