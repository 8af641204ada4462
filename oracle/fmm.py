"""Lagrange FMM (Sec. 4, Alg. lagrange) written out plainly in numpy FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions, each a reading of the paper where it is silent:
  * p is the number of interpolation nodes per dimension (Eq. interpolant
    uses p^3 nodes per cell and the operator has (2p-1)^3 distinct entries,
    Theorem 1), so the 1D polynomials have degree p-1.
  * Nodes are equally spaced in each cell including its faces:
    x_l = lo + s (l / (p-1)), l = 0..p-1 (Sec. 4.1).
  * Root cube = level 0; leaves at level D (2^D cells per side).  M2L runs on
    levels 2..D.  Free space, no periodic images.
  * Every quadrature point is binned by its own position into half-open
    cells [lo, lo+s); points on the upper face of the root are clamped in.
  * Neighbours N(I): cells of the same level at Chebyshev distance <= 1
    (self included).  Interaction list I(I): children of the neighbours of
    I's parent that are not neighbours of I.
  * L2L and L2P interpolate with the coarser (resp. leaf) basis evaluated at
    the finer nodes (resp. the points); M2M is the transpose (anterpolation).
"""
from __future__ import annotations

import numpy as np

from . import assemble_forces, kernel_batch, points, stress


def lagrange_basis(p: int, t: np.ndarray) -> np.ndarray:
    """ell_i(t) for nodes i/(p-1), i = 0..p-1 (footnote to Eq. interpolant).

    t: array of normalised coordinates; returns [len(t), p]."""
    t = np.asarray(t, dtype=np.float64).reshape(-1)
    xi = np.arange(p, dtype=np.float64) / (p - 1)
    out = np.ones((t.shape[0], p))
    for i in range(p):
        for k in range(p):
            if k != i:
                out[:, i] *= (t - xi[k]) / (xi[i] - xi[k])
    return out


def lsq_projector(p, d):
    """Stabilised interpolation on the p equispaced nodes (Sec. 4.3, the
    remark after Alg. fast_sum): the least-squares polynomial of degree d
    fitted to the node values.  Its values at the nodes are P f with
    P = V (V^T V)^{-1} V^T, V[m, k] = phi_k(x_m) for a basis phi_0..phi_d of
    the polynomials of degree <= d (Legendre on [-1, 1] here; P does not
    depend on the basis).  As the fit has degree <= p-1 it is reproduced by
    the Lagrange interpolant through the nodes, so the fitted function is
    sum_m ell_m(x) (P f)_m: the least-squares basis is the Lagrange basis
    times P.  d = p - 1 gives P = I."""
    x = np.linspace(-1.0, 1.0, p)
    V = np.polynomial.legendre.legvander(x, d)  # [p, d+1]
    return V @ np.linalg.solve(V.T @ V, V.T)


def _project(P, a):
    """Apply P to each of the three node axes of a[..., p, p, p]."""
    return np.einsum("ai,bj,ck,...ijk->...abc", P, P, P, a)


def _kern(kernel, x):
    """Kernel values [n, 6, 9] at displacements x[n, 3]."""
    if callable(kernel):
        return np.asarray(kernel(np.asarray(x, dtype=np.float64).reshape(-1, 3)), dtype=np.float64)
    return kernel_batch(x, kernel)


def _direct(kernel, xt, ys, q):
    if callable(kernel):
        d = xt[:, None, :] - ys[None, :, :]
        K = _kern(kernel, d.reshape(-1, 3)).reshape(xt.shape[0], ys.shape[0], 6, 9)
        return np.einsum("tsak,sk->ta", K, q)
    return stress(xt, ys, q, kernel)


def fmm_stress(y, q, kernel, p, D, box_lo, box_size, return_parts=False, lsq_degree=None):
    """Stress at every point y[N,3] from all points (y, q[N,9]) by Alg. lagrange.

    kernel is a packed medium (numpy array, see ``oracle.medium``) or a
    callable x[n,3] -> K[n,6,9].  Returns sigma[N,6] (Voigt order).

    lsq_degree = d switches the interpolant to the least-squares polynomial
    of degree d on the same nodes (``lsq_projector``): the multipole weights
    enter the M2L as P W (P on every axis), and the local values of every
    cell are replaced by P s before they are passed to the children (L2L)
    or to the points (L2P).  The upward pass keeps the Lagrange weights,
    whose parent transfer is exact (M2M)."""
    y = np.asarray(y, dtype=np.float64).reshape(-1, 3)
    q = np.asarray(q, dtype=np.float64).reshape(-1, 9)
    N = y.shape[0]
    lo = np.asarray(box_lo, dtype=np.float64)
    nside = 2 ** D
    sD = box_size / nside
    # -- partition: leaf coordinates of every point (half-open, clamped)
    c = np.floor((y - lo) / sD).astype(np.int64)
    c = np.clip(c, 0, nside - 1)

    def key(cc, lvl):
        n = 2 ** lvl
        return (cc[..., 0] * n + cc[..., 1]) * n + cc[..., 2]

    # occupied cells per level: coords and point/child membership
    cells = {}
    leaf_keys, pt_cell = np.unique(key(c, D), return_inverse=True)
    n = nside
    leaf_coords = np.stack([leaf_keys // (n * n), (leaf_keys // n) % n, leaf_keys % n], axis=1)
    cells[D] = leaf_coords
    for lvl in range(D - 1, 1, -1):
        pc = np.unique(cells[lvl + 1] // 2, axis=0)
        cells[lvl] = pc
    index = {lvl: {tuple(cc): i for i, cc in enumerate(cells[lvl])} for lvl in cells}

    # 1D transfer matrices between a parent and its child octant bit b:
    # S[b][i, m] = ell_i of the parent at the child's node m.
    xi = np.arange(p) / (p - 1)
    S = [lagrange_basis(p, (b + xi) / 2.0).T for b in (0, 1)]  # [i_parent, m_child]

    # -- P2M (Alg. lagrange step 1.a)
    W = {D: np.zeros((len(cells[D]), 9, p, p, p))}
    for ic, cc in enumerate(cells[D]):
        sel = np.nonzero(pt_cell == ic)[0]
        t = (y[sel] - (lo + cc * sD)) / sD
        L1, L2, L3 = (lagrange_basis(p, t[:, d]) for d in range(3))
        W[D][ic] = np.einsum("nw,na,nb,nc->wabc", q[sel], L1, L2, L3)
    # -- M2M (step 1.b)
    for lvl in range(D - 1, 1, -1):
        W[lvl] = np.zeros((len(cells[lvl]), 9, p, p, p))
        for ic, cc in enumerate(cells[lvl + 1]):
            ip = index[lvl][tuple(cc // 2)]
            b = cc % 2
            W[lvl][ip] += np.einsum("im,jn,ko,wmno->wijk", S[b[0]], S[b[1]], S[b[2]], W[lvl + 1][ic])
    Pm = None if lsq_degree is None else lsq_projector(p, lsq_degree)
    Win = W if Pm is None else {lvl: _project(Pm, W[lvl]) for lvl in W}
    # -- M2L (step 2), dense sum over nodes (Eq. m2l)
    s = {lvl: np.zeros((len(cells[lvl]), 6, p, p, p)) for lvl in cells}
    g = np.arange(p)
    for lvl in range(2, D + 1):
        sl = box_size / 2 ** lvl
        h = sl / (p - 1)
        R = 4 * (p - 1)
        ax = np.arange(-R, R + 1)
        lat = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), axis=-1).reshape(-1, 3) * h
        Klat = _kern(kernel, lat).reshape(2 * R + 1, 2 * R + 1, 2 * R + 1, 6, 9)
        ops = {}
        pairs = {}
        for it, tc in enumerate(cells[lvl]):
            ptc = tc // 2
            # candidates: the children of the parent's 27 neighbours
            for d in np.ndindex(6, 6, 6):
                jc = 2 * (ptc - 1) + np.array(d)
                jt = index[lvl].get(tuple(jc))
                if jt is None or np.max(np.abs(jc - tc)) <= 1:
                    continue
                o = tuple(tc - jc)
                pairs.setdefault(o, []).append((it, jt))
        for o, pl in pairs.items():
            if o not in ops:
                # displacement index o(p-1) + l - m per dimension, shifted by R
                dd = [np.asarray(o[d]) * (p - 1) + g[:, None] - g[None, :] + R for d in range(3)]
                op = Klat[dd[0][:, None, None, :, None, None],
                          dd[1][None, :, None, None, :, None],
                          dd[2][None, None, :, None, None, :]]  # [l1,l2,l3,m1,m2,m3,6,9]
                ops[o] = op
            pl = np.asarray(pl)
            contrib = np.einsum("abcdefxw,nwdef->nxabc", ops[o], Win[lvl][pl[:, 1]])
            np.add.at(s[lvl], pl[:, 0], contrib)
    # -- L2L (step 3.a)
    if Pm is not None:
        s[2] = _project(Pm, s[2])
    for lvl in range(3, D + 1):
        for ic, cc in enumerate(cells[lvl]):
            ip = index[lvl - 1][tuple(cc // 2)]
            b = cc % 2
            s[lvl][ic] += np.einsum("im,jn,ko,xijk->xmno", S[b[0]], S[b[1]], S[b[2]], s[lvl - 1][ip])
        if Pm is not None:
            s[lvl] = _project(Pm, s[lvl])
    # -- L2P (step 3.b, far part) and the near field over N(I)
    sig_far = np.zeros((N, 6))
    sig_near = np.zeros((N, 6))
    for ic, cc in enumerate(cells[D]):
        sel = np.nonzero(pt_cell == ic)[0]
        t = (y[sel] - (lo + cc * sD)) / sD
        L1, L2, L3 = (lagrange_basis(p, t[:, d]) for d in range(3))
        sig_far[sel] = np.einsum("xabc,na,nb,nc->nx", s[D][ic], L1, L2, L3)
        srcs = []
        for d in np.ndindex(3, 3, 3):
            k = tuple(cc + np.array(d) - 1)
            if k in index[D]:
                srcs.append(np.nonzero(pt_cell == index[D][k])[0])
        src = np.sort(np.concatenate(srcs))
        sig_near[sel] = _direct(kernel, y[sel], y[src], q[src])
    if return_parts:
        return sig_far + sig_near, sig_far, sig_near
    return sig_far + sig_near


def fmm_forces(seg, burg, kernel, p, D, box_lo, box_size, nq=3, return_parts=False, lsq_degree=None):
    """End-point forces f[N_s, 2, 3] with the stress from ``fmm_stress``."""
    seg = np.asarray(seg, dtype=np.float64).reshape(-1, 2, 3)
    y, q = points(seg, burg, nq)
    out = fmm_stress(y, q, kernel, p, D, box_lo, box_size, return_parts=return_parts, lsq_degree=lsq_degree)
    tgt = np.arange(seg.shape[0])
    if return_parts:
        sig, sf, sn = out
        return (assemble_forces(seg, burg, tgt, sig, nq),
                assemble_forces(seg, burg, tgt, sf, nq),
                assemble_forces(seg, burg, tgt, sn, nq))
    return assemble_forces(seg, burg, tgt, out, nq)
