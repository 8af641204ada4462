"""Pins of the oracle's adaptive Lagrange FMM (Sec. 3's partition until every
leaf holds few segments; the four lists of the adaptive FMM)."""
import numpy as np
import pytest

import oracle
import synth
from oracle.fmm_adaptive import AdaptiveTree, fmm_forces_adaptive, fmm_stress_adaptive
from test_oracle_fmm import direct_numpy, poly_kernel

BOX_LO, BOX = synth.loops.BOX_LO, synth.loops.BOX_SIZE


def clustered(n_big=4, n_small=3, seed=26):
    """A few loops spread over the cube and a tight cluster of small ones
    (each moved next to one centre): leaves of the adaptive tree then sit on
    three or more levels, and the W/X lists are not empty."""
    seg1, b1 = synth.make_loops(n_big, 0.04, 0.1, seed)
    seg2, b2 = synth.make_loops(n_small, 0.01, 0.03, seed + 100)
    rng = np.random.default_rng(seed + 200)
    for k in range(n_small):
        s = seg2[40 * k:40 * k + 40]
        seg2[40 * k:40 * k + 40] = s - s.reshape(-1, 3).mean(axis=0) + 0.3 + rng.uniform(-0.03, 0.03, size=3)
    return np.concatenate([seg1, seg2]), np.concatenate([b1, b2])


@pytest.fixture(scope="module")
def case():
    seg, b = clustered()
    y, q = oracle.points(seg, b)
    T = AdaptiveTree(y, 4, BOX_LO, BOX, 40)
    return seg, b, y, q, T


def test_tree_has_leaves_on_several_levels(case):
    _, _, y, _, T = case
    st = T.stats()
    assert st["leaf_levels"] == [2, 3, 4] and st["w_pairs"] > 0 and st["x_pairs"] == st["w_pairs"]
    # the leaves partition the points
    leaves = [c for c in range(T.n) if T.leaf[c]]
    allp = np.sort(np.concatenate([T.pts[c] for c in leaves]))
    assert np.array_equal(allp, np.arange(y.shape[0]))
    # every leaf above the deepest level holds at most leaf_max points
    assert all(len(T.pts[c]) <= 40 for c in leaves if T.level[c] < 4)


def test_every_pair_of_leaves_is_covered_once(case):
    """U, V (between ancestors), W (from an ancestor of the source) and X
    (to an ancestor of the target) together carry every ordered pair of
    leaves exactly once."""
    _, _, _, _, T = case
    cov = T.coverage()
    assert len(cov) == T.stats()["leaves"] ** 2 and set(cov.values()) == {1}


def test_exact_for_polynomial_kernels(case):
    """With a kernel that is a polynomial of degree p-1 in each coordinate,
    M2L, M2P (W) and P2L (X) are exact, so the adaptive FMM is the direct
    sum (the dropped-list cases below show that the check has teeth)."""
    _, _, y, q, T = case
    p = 3
    K = poly_kernel(p, 5)
    ref = direct_numpy(K, y, q)
    s = fmm_stress_adaptive(y, q, K, p, 4, BOX_LO, BOX, 40, tree=T)
    assert np.abs(s - ref).max() <= 1e-10 * np.abs(ref).max()


def test_direct_small_pairs_keep_exactness(case):
    """W/X pairs whose finer cell holds at most p^3 points summed directly:
    still exact for polynomial kernels, and with direct_max 0 the plain
    adaptive FMM."""
    _, _, y, q, T = case
    p = 3
    K = poly_kernel(p, 5)
    ref = direct_numpy(K, y, q)
    s_d = fmm_stress_adaptive(y, q, K, p, 4, BOX_LO, BOX, 40, tree=T, direct_max=p ** 3)
    assert np.abs(s_d - ref).max() <= 1e-10 * np.abs(ref).max()
    med = oracle.medium(*synth.loops.ISO, 1e-3)
    s0 = fmm_stress_adaptive(y, q, med, p, 4, BOX_LO, BOX, 40, tree=T)
    s00 = fmm_stress_adaptive(y, q, med, p, 4, BOX_LO, BOX, 40, tree=T, direct_max=0)
    assert np.array_equal(s0, s00)


@pytest.mark.parametrize("drop", ["W", "X"])
def test_a_dropped_list_breaks_exactness(case, drop):
    """The exactness pin has teeth: without the W (or X) interactions the
    polynomial kernel's sum is wrong."""
    _, _, y, q, T0 = case
    T = AdaptiveTree(y, 4, BOX_LO, BOX, 40)
    for k in getattr(T, drop):
        getattr(T, drop)[k] = []
    K = poly_kernel(3, 5)
    ref = direct_numpy(K, y, q)
    s = fmm_stress_adaptive(y, q, K, 3, 4, BOX_LO, BOX, 40, tree=T)
    assert np.abs(s - ref).max() > 1e-4 * np.abs(ref).max()


def test_full_split_is_the_uniform_fmm():
    """leaf_max = 0 splits every cell down to Dmax: the uniform tree, no W or
    X lists, and the result of the plain uniform FMM."""
    seg, b = synth.make_loops(8, 0.01, 0.05, 4)
    y, q = oracle.points(seg, b)
    med = oracle.medium(*synth.loops.ISO, 1e-3)
    T = AdaptiveTree(y, 3, BOX_LO, BOX, 0)
    assert T.stats()["w_pairs"] == 0 and T.stats()["leaf_levels"] == [3]
    s_a = fmm_stress_adaptive(y, q, med, 4, 3, BOX_LO, BOX, 0, tree=T)
    s_u = oracle.fmm_stress(y, q, med, 4, 3, BOX_LO, BOX)
    assert np.abs(s_a - s_u).max() <= 1e-12 * np.abs(s_u).max()


def test_adaptive_forces_converge_to_direct():
    seg, b = clustered(3, 2, 23)
    med = oracle.medium(*synth.loops.CUBIC_A25, 1e-3)
    ref = oracle.direct_forces(seg, b, med)
    errs = [oracle.rel_err(fmm_forces_adaptive(seg, b, med, p, 4, BOX_LO, BOX, 40), ref) for p in (3, 4, 5)]
    assert errs[1] < errs[0] / 2 and errs[2] < errs[1] / 2 and errs[2] < 1e-3
