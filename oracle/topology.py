"""Decomposition layer of the oracle (test infrastructure only).

* Partition of the structured grid into N_s boxes of elements (Sec. 2).
* Total FETI constraints B u = c (Sec. 2.1, Eq. 4): pairwise gluing rows at every
  free DOF shared by m >= 2 subdomains (all m(m-1)/2 pairs, redundant at
  cross-points, as k-scaling assumes in Sec. 3.1) and one Dirichlet row for every
  subdomain copy of a clamped DOF (c = 0 for homogeneous clamps). No gluing rows
  are written at clamped DOFs.
* FETI-DP split (Sec. 2.2, Eqs. 8-10): corner nodes are the subdomain vertices
  shared by at least two subdomains that carry a free DOF; their free DOFs are the
  primal set c. Clamped DOFs are eliminated. All other free DOFs of nodes shared
  by >= 2 subdomains are dual and glued pairwise by B_r.
* Rigid-body modes R^s of every subdomain (Sec. 2.1), orthonormalised.
* Scaling of B (Sec. 3.1): multiplicity 1/m, or k-scaling Eq. (15), for which the
  weight of subdomain s on its row with partner q is K^q_jj / sum over all
  subdomains t sharing the node of K^t_jj, with K^t_jj the diagonal entry of
  subdomain t's assembled stiffness at that DOF; one-sided Dirichlet rows get 1.

Row order (an interface convention shared with the GPU library): rows are
emitted node by node in increasing global node number, then component, then
Dirichlet rows by subdomain or gluing pairs (a, b) with a < b lexicographic. In a
gluing row the lower-numbered subdomain carries +1, the other -1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from . import fem


@dataclass
class Subdomain:
    index: int
    lo: tuple            # first element per axis
    hi: tuple            # one past the last element per axis
    nodes: np.ndarray    # global node of every local node (local lexicographic, x fastest)
    dofs: np.ndarray     # global DOF of every local DOF (interleaved)
    elems: np.ndarray    # global element numbers, local lexicographic order
    elem_ldofs: np.ndarray  # [n_el_s, dpn*2^dim] local DOFs of every element

    @property
    def n_loc(self):
        return self.dofs.size


@dataclass
class Decomposition:
    prob: object
    subs: list
    node_subs: dict      # global node -> tuple of subdomains containing it (only nodes with m >= 2)
    fixed: np.ndarray    # bool [n_dof]
    corner_node: np.ndarray  # bool [n_nodes]
    g2l: list            # per subdomain: dict global DOF -> local DOF
    fixed_node_subs: dict  # global node with a clamped DOF -> subdomains containing it


def subdomain_grid_index(prob, s):
    idx = []
    for n in prob.nsub:
        idx.append(s % n)
        s //= n
    return idx


def adaptive_primal_nodes(prob, theta=0.2, cap=3):
    """Adaptive choice of further primal nodes for FETI-DP (the paper's Sec. 6, item i: nodes
    other than the corners whose compatibility is enforced in primal variables). 2D only (3D: no
    further nodes). A node's stiffness is the sum of the Young moduli E_e = Emin + rho_e^p (E0 -
    Emin) of the elements containing it, taken in lexicographic element order. Along every edge
    shared by two subdomains (its end vertices excluded), the nodes whose stiffness is at least
    theta times the edge's largest form runs of consecutive nodes; the cap runs of largest total
    stiffness (earlier run first on ties) each contribute their middle node ((first + last) // 2),
    unless that node carries no free DOF. Returns the sorted global node numbers."""
    if prob.dim != 2:
        return np.zeros(0, dtype=np.int64)
    nx, ny = prob.nel
    # libm pow per element, so that the threshold decisions are taken on the same values as in any
    # other implementation that calls it
    E = [prob.Emin + math.pow(float(r), prob.p) * (prob.E0 - prob.Emin) for r in prob.rho]

    def stiffness(x, y):
        k = 0.0
        for ey in (y - 1, y):
            for ex in (x - 1, x):
                if 0 <= ex < nx and 0 <= ey < ny:
                    k += E[ex + nx * ey]
        return k

    fixed = np.zeros(prob.n_dof, dtype=bool)
    fixed[prob.fixed_dofs()] = True
    cx, cy = prob.cuts
    edges = []
    for i in range(1, len(cx) - 1):
        for j in range(len(cy) - 1):
            edges.append([(cx[i], y) for y in range(cy[j] + 1, cy[j + 1])])
    for j in range(1, len(cy) - 1):
        for i in range(len(cx) - 1):
            edges.append([(x, cy[j]) for x in range(cx[i] + 1, cx[i + 1])])
    out = set()
    for e in edges:
        if not e:
            continue
        k = [stiffness(x, y) for (x, y) in e]
        kmax = max(k)
        if not kmax > 0.0:
            continue
        runs, a = [], None
        for t in range(len(e) + 1):
            stiff = t < len(e) and k[t] >= theta * kmax
            if stiff and a is None:
                a = t
            elif not stiff and a is not None:
                runs.append((a, t - 1, sum(k[a:t])))
                a = None
        runs.sort(key=lambda r: (-r[2], r[0]))
        for a, b, _ in runs[:cap]:
            x, y = e[(a + b) // 2]
            nd = x + (nx + 1) * y
            if not (fixed[2 * nd] and fixed[2 * nd + 1]):
                out.add(nd)
    return np.array(sorted(out), dtype=np.int64)


def decompose(prob, primal_nodes=None) -> Decomposition:
    dim, nel, cuts = prob.dim, prob.nel, prob.cuts
    nn = fem.node_shape(nel)
    strides = [int(np.prod(nn[:d])) for d in range(dim)]
    subs = []
    g2l = []
    for s in range(prob.n_sub):
        gi = subdomain_grid_index(prob, s)
        lo = tuple(cuts[a][gi[a]] for a in range(dim))
        hi = tuple(cuts[a][gi[a] + 1] for a in range(dim))
        loc_nn = [hi[a] - lo[a] + 1 for a in range(dim)]
        grids = np.meshgrid(*[np.arange(lo[a], hi[a] + 1) for a in reversed(range(dim))], indexing="ij")
        nodes = np.zeros(grids[0].shape, dtype=np.int64)
        for a in range(dim):
            nodes += grids[dim - 1 - a] * strides[a]
        nodes = nodes.ravel()
        dofs = (dim * nodes[:, None] + np.arange(dim)[None, :]).ravel()
        eg = np.meshgrid(*[np.arange(lo[a], hi[a]) for a in reversed(range(dim))], indexing="ij")
        elems = np.zeros(eg[0].shape, dtype=np.int64)
        est = [int(np.prod(nel[:d])) for d in range(dim)]
        for a in range(dim):
            elems += eg[dim - 1 - a] * est[a]
        elems = elems.ravel()
        loc_el = tuple(hi[a] - lo[a] for a in range(dim))
        elem_ldofs = fem.element_dofs(loc_el)
        subs.append(Subdomain(s, lo, hi, nodes, dofs, elems, elem_ldofs))
        g2l.append({int(g): l for l, g in enumerate(dofs)})

    # nodes shared by >= 2 subdomains
    counts = {}
    for sd in subs:
        for nd in sd.nodes:
            counts.setdefault(int(nd), []).append(sd.index)
    node_subs = {nd: tuple(sorted(v)) for nd, v in counts.items() if len(v) >= 2}

    fixed = np.zeros(prob.n_dof, dtype=bool)
    fixed[prob.fixed_dofs()] = True
    fixed_nodes = np.nonzero(fixed.reshape(-1, dim).any(axis=1))[0]
    fixed_node_subs = {int(nd): tuple(sorted(counts[int(nd)])) for nd in fixed_nodes}

    cut_sets = [set(c) for c in cuts]
    corner = np.zeros(prob.n_nodes, dtype=bool)
    for nd in node_subs:
        coord, rem = [], nd
        for a in range(dim):
            coord.append(rem % nn[a])
            rem //= nn[a]
        if all(coord[a] in cut_sets[a] for a in range(dim)):
            if not all(fixed[dim * nd + c] for c in range(dim)):
                corner[nd] = True
    # further primal nodes (FETI-DP with an enlarged primal set): shared, with a free DOF
    for nd in ([] if primal_nodes is None else primal_nodes):
        nd = int(nd)
        if nd not in node_subs or all(fixed[dim * nd + c] for c in range(dim)):
            raise ValueError(f"primal node {nd} is not a shared node with a free DOF")
        corner[nd] = True
    return Decomposition(prob, subs, node_subs, fixed, corner, g2l, fixed_node_subs)


# ----------------------------------------------------------------------------- TFETI


@dataclass
class Constraints:
    """Signed Boolean constraint matrix split per subdomain.

    rows[k] = list of (s, local_dof, sign); B^s is n_rows x n_loc^s.
    """
    n_rows: int
    rows: list
    B: list              # per subdomain scipy CSR [n_rows, n_loc_s] (or n_r_s for FETI-DP)
    bset: list           # per subdomain: sorted local DOF indices (into the column space of B) touched by B
    Bb: list             # per subdomain: B restricted to bset columns (CSR [n_rows, n_b])


def _assemble_constraints(rows, ncols):
    n = len(rows)
    per = [[] for _ in ncols]
    for k, row in enumerate(rows):
        for (s, j, sg) in row:
            per[s].append((k, j, sg))
    B, bset, Bb = [], [], []
    for s, nc in enumerate(ncols):
        if per[s]:
            r, c, v = zip(*per[s])
        else:
            r, c, v = (), (), ()
        Bs = sp.csr_matrix((np.array(v, float), (np.array(r, int), np.array(c, int))), shape=(n, nc))
        bs = np.array(sorted(set(c)), dtype=np.int64)
        B.append(Bs)
        bset.append(bs)
        Bb.append(Bs[:, bs].tocsr())
    return Constraints(n, rows, B, bset, Bb)


def tfeti_constraints(dec: Decomposition) -> Constraints:
    """Sec. 2.1, Eq. (4): gluing rows plus Dirichlet rows, columns = all local DOFs."""
    dim = dec.prob.dim
    rows = []
    node_list = sorted(set(dec.node_subs) | set(dec.fixed_node_subs))
    for nd in node_list:
        subs = dec.node_subs.get(nd) or dec.fixed_node_subs[nd]
        for c in range(dim):
            g = dim * nd + c
            if dec.fixed[g]:
                for s in subs:
                    rows.append([(s, dec.g2l[s][g], 1.0)])
            elif len(subs) >= 2:
                for ia in range(len(subs)):
                    for ib in range(ia + 1, len(subs)):
                        a, b = subs[ia], subs[ib]
                        rows.append([(a, dec.g2l[a][g], 1.0), (b, dec.g2l[b][g], -1.0)])
    return _assemble_constraints(rows, [sd.n_loc for sd in dec.subs])


# ----------------------------------------------------------------------------- FETI-DP


@dataclass
class DPSplit:
    """Per-subdomain index sets in local DOF numbering (all sorted increasing)."""
    r: list              # remainder local DOFs (free, not corner)
    c: list              # corner local DOFs
    corner_dofs: np.ndarray   # global DOFs of the primal vector u_c, increasing
    Bc: list             # per subdomain CSR [n_c_s, n_cg]: u_c^s = B_c^s u_c (Eq. 9)


def fetidp_split(dec: Decomposition):
    dim = dec.prob.dim
    corner_dofs = []
    for nd in np.nonzero(dec.corner_node)[0]:
        for c in range(dim):
            g = dim * nd + c
            if not dec.fixed[g]:
                corner_dofs.append(g)
    corner_dofs = np.array(corner_dofs, dtype=np.int64)
    cg_index = {int(g): k for k, g in enumerate(corner_dofs)}
    r_sets, c_sets, Bc = [], [], []
    for sd in dec.subs:
        is_c = np.array([int(g) in cg_index for g in sd.dofs])
        is_fix = dec.fixed[sd.dofs]
        c_loc = np.nonzero(is_c)[0]
        r_loc = np.nonzero(~is_c & ~is_fix)[0]
        cols = np.array([cg_index[int(sd.dofs[j])] for j in c_loc], dtype=np.int64)
        Bc.append(sp.csr_matrix((np.ones(c_loc.size), (np.arange(c_loc.size), cols)),
                                shape=(c_loc.size, corner_dofs.size)))
        r_sets.append(r_loc)
        c_sets.append(c_loc)
    split = DPSplit(r_sets, c_sets, corner_dofs, Bc)

    # B_r (Eq. 10): columns are positions in the remainder set r of each subdomain
    rows = []
    rpos = [{int(l): k for k, l in enumerate(r)} for r in r_sets]
    for nd in sorted(dec.node_subs):
        if dec.corner_node[nd]:
            continue
        subs = dec.node_subs[nd]
        for c in range(dim):
            g = dim * nd + c
            if dec.fixed[g]:
                continue
            for ia in range(len(subs)):
                for ib in range(ia + 1, len(subs)):
                    a, b = subs[ia], subs[ib]
                    rows.append([(a, rpos[a][dec.g2l[a][g]], 1.0), (b, rpos[b][dec.g2l[b][g]], -1.0)])
    cons = _assemble_constraints(rows, [r.size for r in r_sets])
    return split, cons


# ----------------------------------------------------------------------------- kernels of K^s


def rigid_body_modes(prob, sd: Subdomain):
    """Columns spanning the null space of a floating subdomain's stiffness:
    translations and infinitesimal rotations about the subdomain centre,
    orthonormalised (Sec. 2.1: three modes in 2D, six in 3D)."""
    dim = prob.dim
    nn = fem.node_shape(prob.nel)
    coords = np.zeros((sd.nodes.size, dim))
    rem = sd.nodes.copy()
    for a in range(dim):
        coords[:, a] = rem % nn[a]
        rem //= nn[a]
    x = coords - coords.mean(axis=0)
    n = sd.nodes.size
    if dim == 2:
        R = np.zeros((2 * n, 3))
        R[0::2, 0] = 1.0
        R[1::2, 1] = 1.0
        R[0::2, 2] = -x[:, 1]
        R[1::2, 2] = x[:, 0]
    else:
        R = np.zeros((3 * n, 6))
        for a in range(3):
            R[a::3, a] = 1.0
        # rotation about z: (-y, x, 0); about x: (0, -z, y); about y: (z, 0, -x)
        R[0::3, 3] = -x[:, 1]
        R[1::3, 3] = x[:, 0]
        R[1::3, 4] = -x[:, 2]
        R[2::3, 4] = x[:, 1]
        R[0::3, 5] = x[:, 2]
        R[2::3, 5] = -x[:, 0]
    Q, _ = np.linalg.qr(R)
    return Q


# ----------------------------------------------------------------------------- scaling


def scaling_weights(cons: Constraints, diag_of, kind: str):
    """Per subdomain a vector w^s over the rows (zero where the row does not touch s)
    defining B~^s = W^s B^s (Sec. 3.1).

    diag_of(s, col) returns K^s_jj for column `col` of B^s. Rows with one side
    (Dirichlet rows) get weight 1. For pairwise rows the node's full set of
    sharing subdomains is recovered from all rows on the same (node, component):
    rows are grouped by the set of (s, col) entries that share a DOF.
    """
    n_sub = len(cons.B)
    w = [np.zeros(cons.n_rows) for _ in range(n_sub)]
    # group pairwise rows by DOF: two rows belong to the same DOF iff they share an (s, col) entry
    parent = list(range(cons.n_rows))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    seen = {}
    for k, row in enumerate(cons.rows):
        for (s, j, _) in row:
            key = (s, j)
            if key in seen:
                ra, rb = find(seen[key]), find(k)
                if ra != rb:
                    parent[rb] = ra
            else:
                seen[key] = k
    members = {}
    for k, row in enumerate(cons.rows):
        if len(row) == 2:
            g = find(k)
            for (s, j, _) in row:
                members.setdefault(g, {})[s] = j
    for k, row in enumerate(cons.rows):
        if len(row) == 1:
            s, j, _ = row[0]
            w[s][k] = 1.0
            continue
        mem = members[find(k)]
        if kind == "mult":
            m = len(mem)
            for (s, j, _) in row:
                w[s][k] = 1.0 / m
        elif kind == "k":
            tot = sum(diag_of(t, jt) for t, jt in mem.items())
            (a, ja, _), (b, jb, _) = row
            w[a][k] = diag_of(b, jb) / tot
            w[b][k] = diag_of(a, ja) / tot
        else:
            raise ValueError(kind)
    return w
