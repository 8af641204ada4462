"""Pins of the oracle's plain Lagrange FMM (Alg. lagrange) and of the loop generator."""
import numpy as np
import pytest

import oracle
import synth

BOX_LO, BOX = synth.loops.BOX_LO, synth.loops.BOX_SIZE


def poly_kernel(p, seed):
    """A 54-component kernel that is a polynomial of degree p-1 in each coordinate."""
    rng = np.random.default_rng(seed)
    coef = rng.normal(size=(p, p, p, 54))

    def K(x):
        out = np.zeros((x.shape[0], 54))
        for i in range(p):
            for j in range(p):
                for k in range(p):
                    out += (x[:, 0:1] ** i) * (x[:, 1:2] ** j) * (x[:, 2:3] ** k) * coef[i, j, k]
        return out.reshape(-1, 6, 9)

    return K


def direct_numpy(kernel, y, q):
    d = y[:, None, :] - y[None, :, :]
    K = kernel(d.reshape(-1, 3)).reshape(y.shape[0], y.shape[0], 6, 9)
    return np.einsum("tsak,sk->ta", K, q)


@pytest.mark.parametrize("p,D", [(3, 3), (4, 3), (2, 4)])
def test_fmm_exact_for_polynomial_kernels(p, D):
    """Interpolation of degree p-1 reproduces such kernels exactly, so every
    transfer (P2M, M2M, M2L, L2L, L2P) must reproduce the direct sum."""
    seg, b = synth.make_loops(6, 0.05, 0.15, 21)
    y, q = oracle.points(seg, b)
    K = poly_kernel(p, 5)
    ref = direct_numpy(K, y, q)
    s = oracle.fmm_stress(y, q, K, p, D, BOX_LO, BOX)
    assert np.abs(s - ref).max() <= 1e-10 * np.abs(ref).max()
    # a kernel of one degree higher is not reproduced: the test has teeth
    K2 = poly_kernel(p + 1, 6)
    s2 = oracle.fmm_stress(y, q, K2, p, D, BOX_LO, BOX)
    ref2 = direct_numpy(K2, y, q)
    assert np.abs(s2 - ref2).max() > 1e-6 * np.abs(ref2).max()


@pytest.mark.parametrize("p,d,D", [(4, 2, 3), (4, 1, 3), (3, 1, 4)])
def test_lsq_fmm_exact_for_polynomial_kernels_of_its_degree(p, d, D):
    """The least-squares interpolant of degree d (the stabilised scheme of
    Sec. 4.3) reproduces polynomials of degree <= d from their node values,
    so with such a kernel every transfer is exact and the FMM equals the
    direct sum; a kernel of degree d + 1 is not reproduced (while the plain
    Lagrange FMM with the same p, of degree p - 1 > d, still reproduces it)."""
    seg, b = synth.make_loops(4, 0.05, 0.15, 21)
    y, q = oracle.points(seg, b)
    K = poly_kernel(d + 1, 7)  # degree d in each coordinate
    ref = direct_numpy(K, y, q)
    s = oracle.fmm_stress(y, q, K, p, D, BOX_LO, BOX, lsq_degree=d)
    assert np.abs(s - ref).max() <= 1e-10 * np.abs(ref).max()
    K2 = poly_kernel(d + 2, 8)  # degree d + 1
    ref2 = direct_numpy(K2, y, q)
    s2 = oracle.fmm_stress(y, q, K2, p, D, BOX_LO, BOX, lsq_degree=d)
    assert np.abs(s2 - ref2).max() > 1e-6 * np.abs(ref2).max()
    s3 = oracle.fmm_stress(y, q, K2, p, D, BOX_LO, BOX)
    assert np.abs(s3 - ref2).max() <= 1e-10 * np.abs(ref2).max()


def test_lsq_of_full_degree_is_the_lagrange_fmm():
    """d = p - 1: the least-squares fit through p nodes is the interpolant."""
    seg, b = synth.make_loops(8, 0.01, 0.05, 4)
    med = oracle.medium(*synth.loops.ISO, 1e-3)
    f_lag = oracle.fmm_forces(seg, b, med, 4, 3, BOX_LO, BOX)
    f_lsq = oracle.fmm_forces(seg, b, med, 4, 3, BOX_LO, BOX, lsq_degree=3)
    assert oracle.rel_err(f_lsq, f_lag) <= 1e-13
    P = oracle.fmm.lsq_projector(6, 3)
    assert np.allclose(P @ P, P, atol=1e-13) and np.allclose(P, P.T, atol=1e-14)


def test_fmm_all_near_equals_direct():
    # every point within the 2x2x2 centre leaves at depth 2: no M2L pair exists
    seg, b = synth.make_loops(5, 0.02, 0.05, 3)
    seg = 0.5 + 0.35 * (seg - seg.mean(axis=(0, 1)))
    assert seg.min() > 0.275 and seg.max() < 0.825
    med = oracle.medium(*synth.loops.ISO, 1e-3)
    f = oracle.fmm_forces(seg, b, med, 4, 2, BOX_LO, BOX)
    ref = oracle.direct_forces(seg, b, med)
    assert oracle.rel_err(f, ref) <= 1e-13


def test_fmm_converges_with_order():
    seg, b = synth.make_loops(25, 0.01, 0.05, 1)
    med = oracle.medium(*synth.loops.ISO, 1e-3)
    ref = oracle.direct_forces(seg, b, med)
    errs = [oracle.rel_err(oracle.fmm_forces(seg, b, med, p, 3, BOX_LO, BOX), ref) for p in (3, 4, 5, 6)]
    for e0, e1 in zip(errs, errs[1:]):
        assert e1 < e0 / 2.0
    assert errs[-1] < 3e-5


def test_fmm_anisotropic_close_to_direct():
    seg, b = synth.make_loops(10, 0.01, 0.05, 9)
    med = oracle.medium(1.0, 0.6, 0.5, 1e-3)
    ref = oracle.direct_forces(seg, b, med)
    f = oracle.fmm_forces(seg, b, med, 5, 3, BOX_LO, BOX)
    assert oracle.rel_err(f, ref) < 1e-3


# --------------------------------------------------------------- generator
def test_generator_properties():
    seg, b = synth.make_loops(30, 0.01, 0.05, 4)
    seg2, b2 = synth.make_loops(30, 0.01, 0.05, 4)
    assert np.array_equal(seg, seg2) and np.array_equal(b, b2)
    assert seg.shape == (30 * 40, 2, 3) and b.shape == (30 * 40, 3)
    lo = np.array(BOX_LO)
    assert np.all(seg > lo) and np.all(seg < lo + BOX)
    assert np.allclose(np.linalg.norm(b, axis=1), 1.0)
    assert np.allclose(np.abs(b) * np.sqrt(3), 1.0)  # unit <111>
    for il in range(30):
        s = seg[40 * il:40 * il + 40]
        dS = s[:, 1] - s[:, 0]
        assert np.abs(dS.sum(axis=0)).max() < 1e-15  # closed
        assert np.allclose(s[1:, 0], s[:-1, 1]) and np.allclose(s[0, 0], s[-1, 1])
        n = np.cross(dS[0], dS[10])
        n /= np.linalg.norm(n)
        assert np.abs(dS @ n).max() < 1e-14  # planar
        assert abs(b[40 * il] @ n) < 1e-12  # glide loop: b in the plane
        assert sorted(np.abs(n * np.sqrt(2)).round(6)) == [0.0, 1.0, 1.0]  # {110}


def test_workloads_sizes():
    for name, n in (("iso2k", 2000), ("cubic100k", 100000)):
        w = synth.WORKLOADS[name]
        assert w["n_loops"] * 40 == n
