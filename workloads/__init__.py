"""Seeded synthetic inputs for the FETI workloads.

This module is shared by the oracle and by the HIP path. It holds no solver
arithmetic: only grid sizes, subdomain cuts, element densities drawn from a
seeded ``numpy.random.default_rng``, the clamped-DOF list and the load vector.

Conventions (shared interface, like a file format):

* nodes are numbered lexicographically, x fastest:
  ``node = ix + (nx+1)*(iy + (ny+1)*iz)``;
* DOFs are interleaved per node: ``dof = dpn*node + component``;
* elements are numbered lexicographically, x fastest: ``e = ex + nx*(ey + ny*ez)``;
* all elements are unit squares (unit cubes), thickness 1;
* the face x = 0 is clamped (every DOF of every node with ix = 0);
* one unit point load acts in -y at node (nx, ny//2[, nz//2]).

The workloads stand in for the paper's academic problems and modular
topology-optimisation snapshots (Sec. 4), whose density fields and material
contrasts the paper does not give.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np


@dataclass
class Problem:
    """One SIMP elasticity problem on a structured grid with a tensor-product partition."""

    dim: int
    nel: tuple                      # elements per axis
    cuts: tuple                     # per axis: increasing element indices, cuts[a][0]=0, cuts[a][-1]=nel[a]
    rho: np.ndarray                 # [n_el] densities in [0, 1]
    nu: float = 0.3
    E0: float = 1.0
    Emin: float = 1e-6
    p: float = 3.0
    name: str = ""
    groups: Optional[tuple] = None  # S-FETI direction groups: subdomain blocks per axis (None = one per subdomain)
    traction: Optional[tuple] = None  # uniform traction (tx, ty) on the edge x = nx instead of the point load

    @property
    def dpn(self) -> int:
        return self.dim

    @property
    def nsub(self) -> tuple:
        return tuple(len(c) - 1 for c in self.cuts)

    @property
    def n_sub(self) -> int:
        return int(np.prod(self.nsub))

    @property
    def n_el(self) -> int:
        return int(np.prod(self.nel))

    @property
    def n_nodes(self) -> int:
        return int(np.prod([n + 1 for n in self.nel]))

    @property
    def n_dof(self) -> int:
        return self.dpn * self.n_nodes

    def fixed_dofs(self) -> np.ndarray:
        return clamped_dofs(self.dim, self.nel)

    def load(self) -> np.ndarray:
        if self.traction is not None:
            return edge_traction(self.nel, self.traction)
        return point_load(self.dim, self.nel)


def uniform_cuts(n: int, parts: int) -> List[int]:
    if n % parts:
        raise ValueError("uniform partition needs nel divisible by nsub")
    return [i * (n // parts) for i in range(parts + 1)]


def clamped_dofs(dim: int, nel: Sequence[int]) -> np.ndarray:
    """Every DOF of every node on the face x = 0, increasing."""
    shape = [n + 1 for n in nel]
    idx = np.arange(int(np.prod(shape))).reshape(shape[::-1])  # [.., iy, ix]
    nodes = np.sort(idx[..., 0].ravel())
    return (dim * nodes[:, None] + np.arange(dim)[None, :]).ravel().astype(np.int64)


def point_load(dim: int, nel: Sequence[int]) -> np.ndarray:
    """Unit load in -y at node (nx, ny//2[, nz//2])."""
    nn = [n + 1 for n in nel]
    ix, iy = nel[0], nel[1] // 2
    node = ix + nn[0] * iy
    if dim == 3:
        node += nn[0] * nn[1] * (nel[2] // 2)
    f = np.zeros(dim * int(np.prod(nn)))
    f[dim * node + 1] = -1.0
    return f


def edge_traction(nel: Sequence[int], t: Sequence[float]) -> np.ndarray:
    """2D: nodal forces of a uniform traction t = (tx, ty) per unit length on the edge x = nx
    (unit element edges: end nodes carry half an edge, the others a whole one)."""
    nn = [n + 1 for n in nel]
    f = np.zeros(2 * nn[0] * nn[1])
    for iy in range(nn[1]):
        node = nel[0] + nn[0] * iy
        w = 0.5 if iy in (0, nel[1]) else 1.0
        f[2 * node] = w * t[0]
        f[2 * node + 1] = w * t[1]
    return f


def _module_rho(rng, nsub, m, dim, solid_fraction=0.5):
    """Modular 0/1 design: every subdomain (module of m^dim elements) gets exactly
    round(solid_fraction * m^dim) solid elements chosen by a seeded permutation."""
    nel = tuple(s * m for s in nsub)
    rho = np.zeros(nel[::-1])
    n_mod = m ** dim
    n_solid = int(round(solid_fraction * n_mod))
    for sidx in np.ndindex(*nsub[::-1]):          # z, y, x order -> subdomains x fastest
        pat = np.zeros(n_mod)
        pat[rng.permutation(n_mod)[:n_solid]] = 1.0
        pat = pat.reshape((m,) * dim)
        sl = tuple(slice(k * m, (k + 1) * m) for k in sidx)
        rho[sl] = pat
    return rho.ravel()


def modular_types_2d(seed: int = 0, nsub=(8, 4), m: int = 16, n_types: int = 4, Emin: float = 1e-6) -> Problem:
    """2D modular design built from n_types module types (Sec. 1: a modular structure repeats a few
    module designs): every type is a seeded 0/1 pattern at solid fraction 0.5, and every subdomain
    takes a seeded type."""
    rng = np.random.default_rng(seed)
    n_mod = m * m
    types = []
    for _ in range(n_types):
        pat = np.zeros(n_mod)
        pat[rng.permutation(n_mod)[:n_mod // 2]] = 1.0
        types.append(pat.reshape(m, m))
    rho = np.zeros((nsub[1] * m, nsub[0] * m))
    for sy in range(nsub[1]):
        for sx in range(nsub[0]):
            rho[sy * m:(sy + 1) * m, sx * m:(sx + 1) * m] = types[int(rng.integers(n_types))]
    nel = (nsub[0] * m, nsub[1] * m)
    return Problem(2, nel, tuple(uniform_cuts(n, s) for n, s in zip(nel, nsub)), rho.ravel(), Emin=Emin,
                   name=f"modular_types2d_{nsub[0]}x{nsub[1]}_of_{m}_{n_types}types")


def cantilever_tfeti(seed: int = 0, nsub=(4, 2), m: int = 8) -> Problem:
    """2D Q4 cantilever, 4x2 subdomains of 8x8 elements, rho ~ U(0,1) i.i.d., Emin 1e-6."""
    rng = np.random.default_rng(seed)
    nel = (nsub[0] * m, nsub[1] * m)
    rho = rng.uniform(0.0, 1.0, nel[0] * nel[1])
    return Problem(2, nel, tuple(uniform_cuts(n, s) for n, s in zip(nel, nsub)), rho,
                   Emin=1e-6, name=f"cantilever2d_{nsub[0]}x{nsub[1]}_of_{m}")


def modular_2d(seed: int = 0, nsub=(8, 4), m: int = 32, Emin: float = 1e-6) -> Problem:
    """2D Q4 modular design: each 32x32 module a seeded 0/1 pattern at solid fraction 0.5."""
    rng = np.random.default_rng(seed)
    rho = _module_rho(rng, nsub, m, 2)
    nel = (nsub[0] * m, nsub[1] * m)
    return Problem(2, nel, tuple(uniform_cuts(n, s) for n, s in zip(nel, nsub)), rho,
                   Emin=Emin, name=f"modular2d_{nsub[0]}x{nsub[1]}_of_{m}")


def beta_2d(seed: int = 0, nsub=(16, 16), m: int = 64, n_dirs: int = 64, Emin: float = 1e-9) -> Problem:
    """2D Q4, rho ~ Beta(0.3, 0.3) per element, contrast 1e-9; S-FETI groups of
    2x2 subdomains for 64 directions or 4x2 for 32 (x-major)."""
    rng = np.random.default_rng(seed)
    nel = (nsub[0] * m, nsub[1] * m)
    rho = rng.beta(0.3, 0.3, nel[0] * nel[1])
    groups = group_shape(nsub, n_dirs)
    return Problem(2, nel, tuple(uniform_cuts(n, s) for n, s in zip(nel, nsub)), rho,
                   Emin=Emin, name=f"beta2d_{nsub[0]}x{nsub[1]}_of_{m}", groups=groups)


def beta_2d_block(seed: int = 0, bs: int = 4, nsub=(16, 16), m: int = 64, Emin: float = 1e-9) -> Problem:
    """The lower-left bs x bs block of subdomains of beta_2d(seed): the same 64x64-element
    subdomains and the same density values, clamped at its own x = 0 edge and loaded at its own
    right-mid node; 2x2 subdomain groups. A bounded sample of that workload for timing CPU code."""
    full = beta_2d(seed, nsub, m, Emin=Emin)
    rho = full.rho.reshape(full.nel[1], full.nel[0])[: bs * m, : bs * m].ravel().copy()
    return Problem(2, (bs * m, bs * m), tuple(uniform_cuts(bs * m, bs) for _ in range(2)), rho,
                   Emin=Emin, name=f"beta2d_block{bs}x{bs}_of_{m}", groups=(2, 2))


def modular_3d(seed: int = 0, nsub=(4, 4, 4), m: int = 12, Emin: float = 1e-6) -> Problem:
    """3D Hex8 modular design: each 12^3 module a seeded 0/1 pattern at solid fraction 0.5."""
    rng = np.random.default_rng(seed)
    rho = _module_rho(rng, nsub, m, 3)
    nel = tuple(s * m for s in nsub)
    return Problem(3, nel, tuple(uniform_cuts(n, s) for n, s in zip(nel, nsub)), rho,
                   Emin=Emin, name=f"modular3d_{nsub[0]}x{nsub[1]}x{nsub[2]}_of_{m}")


def uneven_design(seed: int, d: int, g=(4, 8), w=(16, 48)) -> Problem:
    """One design of the batched workload: gx, gy ~ U{g0..g1} subdomains per axis (4..8),
    per-column widths and per-row heights ~ U{w0..w1} elements (16..48), modular 0/1 rho."""
    rng = np.random.default_rng([seed, d])
    gx, gy = int(rng.integers(g[0], g[1] + 1)), int(rng.integers(g[0], g[1] + 1))
    wx = rng.integers(w[0], w[1] + 1, gx)
    wy = rng.integers(w[0], w[1] + 1, gy)
    cx = [0] + list(np.cumsum(wx).astype(int))
    cy = [0] + list(np.cumsum(wy).astype(int))
    nel = (cx[-1], cy[-1])
    rho = np.zeros((nel[1], nel[0]))
    for jy in range(gy):
        for jx in range(gx):
            h, w = int(wy[jy]), int(wx[jx])
            n_mod = h * w
            pat = np.zeros(n_mod)
            pat[rng.permutation(n_mod)[:int(round(0.5 * n_mod))]] = 1.0
            rho[cy[jy]:cy[jy + 1], cx[jx]:cx[jx + 1]] = pat.reshape(h, w)
    return Problem(2, nel, (tuple(cx), tuple(cy)), rho.ravel(), Emin=1e-6,
                   name=f"uneven2d_seed{seed}_d{d}")


# ---- academic problems (Sec. 4.1): two materials, stiff (rho = 1, E0) and compliant (rho = 0,
# Emin), clamped on the left edge, uniform tensile and tangential traction (1, -1) on the right
# edge. The paper gives neither the material contrast nor the layer geometry beyond its figure
# captions; the contrast here is Emin / E0 = 1e-4, with 14 x 14 (layers) or 16 x 16 (inclusion)
# elements per subdomain.

def _layers(m: int, n_layers: int, horizontal: bool) -> np.ndarray:
    """m x m module of n_layers alternating layers (stiff first), rows y, columns x."""
    if m % n_layers:
        raise ValueError("the module size must be a multiple of the layer count")
    k = (np.arange(m) // (m // n_layers)) % 2 == 0
    return np.tile(k[:, None], (1, m)).astype(float) if horizontal else np.tile(k[None, :], (m, 1)).astype(float)


def laminated_beam(nsub: int = 9, m: int = 14, n_layers: int = 7, Emin: float = 1e-4) -> Problem:
    """Laminated beam: a row of nsub square subdomains, each of n_layers horizontal layers
    alternating stiff and compliant, continuous from one subdomain to the next (no cross-points)."""
    mod = _layers(m, n_layers, True)
    rho = np.tile(mod, (1, nsub))
    nel = (nsub * m, m)
    return Problem(2, nel, (tuple(uniform_cuts(nel[0], nsub)), (0, m)), rho.ravel(), Emin=Emin,
                   name=f"laminated_beam_{nsub}_of_{m}", traction=(1.0, -1.0))


def layered_grid(nsub=(3, 3), m: int = 14, n_layers: int = 7, Emin: float = 1e-4) -> Problem:
    """Grid of layered subdomains (n_layers alternating layers each) whose layer direction
    alternates in a checkerboard (horizontal where sx + sy is even, vertical otherwise), so the
    stiffness met at interface nodes and cross-points differs from one subdomain to the next."""
    rho = np.zeros((nsub[1] * m, nsub[0] * m))
    for sy in range(nsub[1]):
        for sx in range(nsub[0]):
            rho[sy * m:(sy + 1) * m, sx * m:(sx + 1) * m] = _layers(m, n_layers, (sx + sy) % 2 == 0)
    nel = (nsub[0] * m, nsub[1] * m)
    return Problem(2, nel, tuple(uniform_cuts(n, s) for n, s in zip(nel, nsub)), rho.ravel(), Emin=Emin,
                   name=f"layered_grid_{nsub[0]}x{nsub[1]}_of_{m}", traction=(1.0, -1.0))


def inclusion_grid(nsub=(4, 4), m: int = 16, Emin: float = 1e-4) -> Problem:
    """Grid of compliant subdomains, each with one stiff square inclusion of m/2 x m/2 elements at
    its centre: the material on every interface is the compliant one."""
    mod = np.zeros((m, m))
    a = m // 4
    mod[a:m - a, a:m - a] = 1.0
    rho = np.tile(mod, (nsub[1], nsub[0]))
    nel = (nsub[0] * m, nsub[1] * m)
    return Problem(2, nel, tuple(uniform_cuts(n, s) for n, s in zip(nel, nsub)), rho.ravel(), Emin=Emin,
                   name=f"inclusion_grid_{nsub[0]}x{nsub[1]}_of_{m}", traction=(1.0, -1.0))


ACADEMIC = {"laminated_beam": laminated_beam, "layered_grid": layered_grid, "inclusion_grid": inclusion_grid}


def group_shape(nsub, n_dirs):
    """Subdomain block shape giving n_dirs S-FETI direction groups (x-major blocks)."""
    n_sub = int(np.prod(nsub))
    if n_dirs >= n_sub:
        return None
    if len(nsub) == 2 and n_sub // n_dirs == 4 and nsub[0] % 2 == 0 and nsub[1] % 2 == 0:
        return (2, 2)
    if len(nsub) == 2 and n_sub // n_dirs == 8 and nsub[0] % 4 == 0 and nsub[1] % 2 == 0:
        return (4, 2)
    raise ValueError(f"no group shape for {nsub} subdomains and {n_dirs} directions")


def group_of_subdomains(nsub, groups) -> np.ndarray:
    """Column index g(s) of every subdomain s (subdomains numbered x fastest);
    groups are blocks of the subdomain grid numbered x fastest."""
    n_sub = int(np.prod(nsub))
    if groups is None:
        return np.arange(n_sub, dtype=np.int64)
    nb = [n // g for n, g in zip(nsub, groups)]
    out = np.empty(n_sub, dtype=np.int64)
    for s in range(n_sub):
        idx, rem = [], s
        for n in nsub:
            idx.append(rem % n)
            rem //= n
        bidx = [i // g for i, g in zip(idx, groups)]
        gid, stride = 0, 1
        for b, n in zip(bidx, nb):
            gid += b * stride
            stride *= n
        out[s] = gid
    return out


CONFIGS = {
    "c1": cantilever_tfeti,
    "c2": modular_2d,
    "c3": beta_2d,
    "c5": modular_3d,
}
