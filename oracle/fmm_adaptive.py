"""Adaptive Lagrange FMM written out plainly in numpy FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 3 describes the first of the FMM's five steps as partitioning the
region recursively until every leaf cell holds a small number of segments.
On clustered dislocation ensembles that makes a tree whose leaves sit on
different levels.  This module is the plain version of the FMM on such a
tree, with the four lists of the adaptive FMM spelled out by their
definitions (brute force over all cells), and the transfers of Alg. lagrange
(P2M, M2M, M2L with each level's operator of Eq. m2l, L2L, L2P) unchanged:

  * A cell is split while it lies above level Dmax and holds more than
    ``leaf_max`` points; cells of levels 0 and 1 are always split (the M2L
    starts at level 2).  Only children that hold points exist.
  * Two cells are adjacent when their closed boxes touch (any level).
  * U(B), for a leaf B: the leaves adjacent to B (B included).  Direct sum.
  * V(B), for every cell B of level >= 2: the cells of B's level that are
    not adjacent to B and whose parents are adjacent.  M2L.
  * W(B), for a leaf B: the cells A finer than B, not adjacent to B, whose
    parent is adjacent to B.  A's multipole weights act on B's points as
    point sources at A's nodes (in the Lagrange FMM the weights W_m are the
    strengths of sources at the nodes: sigma(x) ~ sum_m K(x - y_m) W_m).
  * X(B): the leaves A with B in W(A).  A's points act on B's nodes, whose
    values are B's local expansion (the stress at the nodes).

Every pair of points is then counted exactly once (``coverage`` checks it
combinatorially), and with a kernel that is a polynomial of degree p-1 in
each coordinate every far transfer is exact, so the FMM equals the direct
sum: the pins of this module.  Optionally (``direct_max``) a W or X pair
whose finer cell holds few points is summed directly instead, which keeps
both properties.
"""
from __future__ import annotations

import numpy as np

from . import assemble_forces, points
from .fmm import _direct, _kern, lagrange_basis


class AdaptiveTree:
    """Cells of the adaptive octree and their lists (by definition)."""

    def __init__(self, y, Dmax, box_lo, box_size, leaf_max):
        self.Dmax, self.lo, self.size = Dmax, np.asarray(box_lo, dtype=np.float64), float(box_size)
        n = 2 ** Dmax
        cf = np.floor((y - self.lo) / (self.size / n)).astype(np.int64)
        self.cf = np.clip(cf, 0, n - 1)  # finest-level coordinates of every point
        self.level, self.ijk, self.parent, self.pts, self.children, self.leaf = [], [], [], [], [], []
        self._make(0, np.zeros(3, dtype=np.int64), -1, np.arange(y.shape[0]), leaf_max)
        self.level = np.asarray(self.level)
        self.ijk = np.asarray(self.ijk)
        self.leaf = np.asarray(self.leaf)
        self.n = len(self.level)
        self.by_level = {l: [c for c in range(self.n) if self.level[c] == l] for l in range(Dmax + 1)}
        self._lists()

    def _make(self, level, ijk, parent, idx, leaf_max):
        c = len(self.level)
        self.level.append(level)
        self.ijk.append(ijk)
        self.parent.append(parent)
        self.pts.append(idx)
        self.children.append([])
        split = level < self.Dmax and (level < 2 or len(idx) > leaf_max)
        self.leaf.append(not split)
        if split:
            sub = self.cf[idx] >> (self.Dmax - level - 1)  # coordinates at level + 1
            for cc in np.unique(sub, axis=0):
                sel = idx[np.all(sub == cc, axis=1)]
                self.children[c].append(self._make(level + 1, cc, c, sel, leaf_max))
        return c

    def box(self, c):
        """Closed box of cell c in units of the finest cells."""
        w = 2 ** (self.Dmax - self.level[c])
        return self.ijk[c] * w, self.ijk[c] * w + w

    def adjacent(self, a, b):
        la, ha = self.box(a)
        lb, hb = self.box(b)
        return bool(np.all(np.maximum(la, lb) <= np.minimum(ha, hb)))

    def ancestors(self, c):
        out = []
        while c >= 0:
            out.append(c)
            c = self.parent[c]
        return out  # c itself first, root last

    def _lists(self):
        n, lvl, par, leaf = self.n, self.level, self.parent, self.leaf
        adj = np.array([[self.adjacent(a, b) for b in range(n)] for a in range(n)], dtype=bool)
        self.adj = adj
        self.U = {b: [a for a in range(n) if leaf[a] and adj[a, b]] for b in range(n) if leaf[b]}
        self.V = {b: [a for a in self.by_level[lvl[b]] if not adj[a, b] and adj[par[a], par[b]]]
                  for b in range(n) if lvl[b] >= 2}
        self.W = {b: [a for a in range(n) if lvl[a] > lvl[b] and not adj[a, b] and adj[par[a], b]]
                  for b in range(n) if leaf[b]}
        self.X = {b: [] for b in range(n)}
        for b, ws in self.W.items():
            for a in ws:
                self.X[a].append(b)

    def coverage(self):
        """For every ordered pair of leaves (target B, source A), how many of
        the list interactions carry A's points to B's points: U directly, V
        between ancestors of equal level, W from an ancestor of A to B, X from
        A to an ancestor of B.  Must be 1 everywhere."""
        leaves = [c for c in range(self.n) if self.leaf[c]]
        anc = {c: self.ancestors(c) for c in leaves}
        cnt = {}
        for b in leaves:
            for a in leaves:
                k = int(a in self.U[b])
                for bb in anc[b]:
                    for aa in anc[a]:
                        if self.level[bb] == self.level[aa] and self.level[bb] >= 2 and aa in self.V[bb]:
                            k += 1
                k += sum(1 for aa in anc[a] if aa in self.W[b])
                k += sum(1 for bb in anc[b] if a in self.X[bb])
                cnt[(b, a)] = k
        return cnt

    def nodes(self, c, p):
        """Node positions of cell c [p^3, 3], node (a, b, c) in C order."""
        s = self.size / 2 ** self.level[c]
        g = np.arange(p) / (p - 1)
        G = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
        return self.lo + s * (self.ijk[c] + G)

    def stats(self):
        leaves = [c for c in range(self.n) if self.leaf[c]]
        return {"cells": self.n, "leaves": len(leaves),
                "leaf_levels": sorted(set(int(self.level[c]) for c in leaves)),
                "u_pairs": sum(len(v) for v in self.U.values()), "v_pairs": sum(len(v) for v in self.V.values()),
                "w_pairs": sum(len(v) for v in self.W.values()), "x_pairs": sum(len(v) for v in self.X.values())}


def _subtree_points(T, c):
    """Indices of the points below cell c (its leaves' points)."""
    if T.leaf[c]:
        return T.pts[c]
    return np.concatenate([_subtree_points(T, ch) for ch in T.children[c]])


def fmm_stress_adaptive(y, q, kernel, p, Dmax, box_lo, box_size, leaf_max, return_parts=False, tree=None,
                        direct_max=None):
    """Stress at every point y[N,3] from all points (y, q[N,9]) by the
    adaptive Lagrange FMM on the tree that ``leaf_max`` and ``Dmax`` define.
    kernel: packed medium or callable x[n,3] -> K[n,6,9].  Returns
    sigma[N,6]; with return_parts also the far part (L2P and W lists) and
    the near part (U lists, and the W/X pairs evaluated directly).

    direct_max = m: a W or X pair whose finer cell A holds at most m points
    is summed directly between the points of A and of the leaf (exact; a
    pair through A's nodes costs p^3 evaluations per point of the leaf)."""
    y = np.asarray(y, dtype=np.float64).reshape(-1, 3)
    q = np.asarray(q, dtype=np.float64).reshape(-1, 9)
    N = y.shape[0]
    T = tree if tree is not None else AdaptiveTree(y, Dmax, box_lo, box_size, leaf_max)
    lo = T.lo
    xi = np.arange(p) / (p - 1)
    S = [lagrange_basis(p, (b + xi) / 2.0).T for b in (0, 1)]  # [i_parent, m_child]

    def cell_lo(c):
        return lo + T.ijk[c] * (box_size / 2 ** T.level[c])

    def bases(c, idx):
        s = box_size / 2 ** T.level[c]
        t = (y[idx] - cell_lo(c)) / s
        return [lagrange_basis(p, t[:, d]) for d in range(3)]

    # -- upward pass: P2M at the leaves (any level), M2M for the other cells
    W = {}
    for l in range(Dmax, 1, -1):
        for c in T.by_level[l]:
            if T.leaf[c]:
                L1, L2, L3 = bases(c, T.pts[c])
                W[c] = np.einsum("nw,na,nb,nc->wabc", q[T.pts[c]], L1, L2, L3)
            else:
                acc = np.zeros((9, p, p, p))
                for ch in T.children[c]:
                    b = T.ijk[ch] % 2
                    acc += np.einsum("im,jn,ko,wmno->wijk", S[b[0]], S[b[1]], S[b[2]], W[ch])
                W[c] = acc
    # -- V lists: M2L with each level's operators (dense, Eq. m2l)
    s = {c: np.zeros((6, p, p, p)) for c in range(T.n) if T.level[c] >= 2}
    g = np.arange(p)
    for l in range(2, Dmax + 1):
        sl = box_size / 2 ** l
        h = sl / (p - 1)
        R = 4 * (p - 1)
        ax = np.arange(-R, R + 1)
        lat = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), axis=-1).reshape(-1, 3) * h
        Klat = _kern(kernel, lat).reshape(2 * R + 1, 2 * R + 1, 2 * R + 1, 6, 9)
        ops = {}
        for b in T.by_level[l]:
            for a in T.V[b]:
                o = tuple(T.ijk[b] - T.ijk[a])
                if o not in ops:
                    dd = [o[d] * (p - 1) + g[:, None] - g[None, :] + R for d in range(3)]
                    ops[o] = Klat[dd[0][:, None, None, :, None, None],
                                  dd[1][None, :, None, None, :, None],
                                  dd[2][None, None, :, None, None, :]]  # [l1,l2,l3,m1,m2,m3,6,9]
                s[b] += np.einsum("abcdefxw,wdef->xabc", ops[o], W[a])
    def direct_pair(a):
        return direct_max is not None and len(_subtree_points(T, a)) <= direct_max

    # -- X lists: the source leaf's points straight onto the target's nodes
    # (or, for a small target cell, onto the points below it)
    sig_x = np.zeros((N, 6))
    for b in range(T.n):
        if T.level[b] >= 2 and T.X[b]:
            src = np.sort(np.concatenate([T.pts[a] for a in T.X[b]]))
            if direct_pair(b):
                tgt = np.sort(_subtree_points(T, b))
                sig_x[tgt] += _direct(kernel, y[tgt], y[src], q[src])
            else:
                s[b] += _direct(kernel, T.nodes(b, p), y[src], q[src]).T.reshape(6, p, p, p)
    # -- downward pass: L2L into every cell of level >= 3
    for l in range(3, Dmax + 1):
        for c in T.by_level[l]:
            b = T.ijk[c] % 2
            s[c] += np.einsum("im,jn,ko,xijk->xmno", S[b[0]], S[b[1]], S[b[2]], s[T.parent[c]])
    # -- leaves: L2P, W lists (node sources), U lists (direct)
    sig_far = np.zeros((N, 6))
    sig_near = np.zeros((N, 6))
    for c in range(T.n):
        if not T.leaf[c]:
            continue
        idx = T.pts[c]
        L1, L2, L3 = bases(c, idx)
        sig_far[idx] = np.einsum("xabc,na,nb,nc->nx", s[c], L1, L2, L3)
        for a in T.W[c]:
            if direct_pair(a):
                sa = np.sort(_subtree_points(T, a))
                sig_near[idx] += _direct(kernel, y[idx], y[sa], q[sa])
            else:
                sig_far[idx] += _direct(kernel, y[idx], T.nodes(a, p), W[a].reshape(9, -1).T)
        src = np.sort(np.concatenate([T.pts[a] for a in T.U[c]]))
        sig_near[idx] += _direct(kernel, y[idx], y[src], q[src])
    sig_near += sig_x
    if return_parts:
        return sig_far + sig_near, sig_far, sig_near
    return sig_far + sig_near


def fmm_forces_adaptive(seg, burg, kernel, p, Dmax, box_lo, box_size, leaf_max, nq=3, return_parts=False,
                        direct_max=None):
    """End-point forces f[N_s, 2, 3] with the stress from ``fmm_stress_adaptive``."""
    seg = np.asarray(seg, dtype=np.float64).reshape(-1, 2, 3)
    y, q = points(seg, burg, nq)
    out = fmm_stress_adaptive(y, q, kernel, p, Dmax, box_lo, box_size, leaf_max, return_parts=return_parts,
                              direct_max=direct_max)
    tgt = np.arange(seg.shape[0])
    if return_parts:
        return tuple(assemble_forces(seg, burg, tgt, o, nq) for o in out)
    return assemble_forces(seg, burg, tgt, out, nq)
