"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: library
quadrature rules, finite differences, textbook closed forms (Kelvin's solution,
Hirth-Lothe infinite-line stresses), symmetries, invariants and brute-force
integration.  None of them needs a GPU.
"""
import numpy as np
import pytest
from scipy import integrate

import oracle
import synth

MU, NU = 1.0, 0.3
LAM = 2 * MU * NU / (1 - 2 * NU)
ISO = (LAM + 2 * MU, LAM, MU)
RNG = np.random.default_rng(1234)


def iso_med(a=0.0):
    return oracle.medium(*ISO, a)


# ---------------------------------------------------------------- quadrature
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 12])
def test_gauss_legendre_matches_library_and_is_exact(n):
    u, w = oracle.gauss_legendre(n)
    ul, wl = np.polynomial.legendre.leggauss(n)
    assert np.allclose(u, ul, atol=1e-14) and np.allclose(w, wl, atol=1e-14)
    for k in range(2 * n):  # exact up to degree 2n-1
        exact = (1 - (-1) ** (k + 1)) / (k + 1)
        assert abs(np.dot(w, u ** k) - exact) < 1e-13


# ------------------------------------------------------- isotropic kernel
def kelvin(x, mu, nu):
    r = np.linalg.norm(x)
    T = x / r
    return ((3 - 4 * nu) * np.eye(3) + np.outer(T, T)) / (16 * np.pi * mu * (1 - nu) * r)


def test_G_iso_is_kelvin_solution():
    for _ in range(5):
        x = RNG.normal(size=3)
        assert np.allclose(oracle.G_iso(x, MU, NU, 0.0), kelvin(x, MU, NU), rtol=1e-13, atol=0)


@pytest.mark.parametrize("a", [0.0, 1e-3, 0.3])
def test_dG_iso_is_derivative_of_G_iso(a):
    h = 1e-5
    for _ in range(4):
        x = RNG.normal(size=3)
        D = oracle.dG_iso(x, MU, NU, a)
        for q in range(3):
            e = np.zeros(3)
            e[q] = h
            fd = (oracle.G_iso(x + e, MU, NU, a) - oracle.G_iso(x - e, MU, NU, a)) / (2 * h)
            assert np.abs(D[:, :, q] - fd).max() <= 1e-8 * np.abs(D).max()


def test_dG_iso_regular_at_origin_and_symmetric():
    assert np.all(oracle.dG_iso(np.zeros(3), MU, NU, 1e-3) == 0.0)
    x = RNG.normal(size=3)
    D = oracle.dG_iso(x, MU, NU, 1e-3)
    assert np.allclose(D, D.transpose(1, 0, 2), atol=0)
    assert np.allclose(oracle.dG_iso(-x, MU, NU, 1e-3), -D, rtol=1e-14)


# ----------------------------------------------------- anisotropic kernel
def test_circle_G_and_dG_reduce_to_isotropic_closed_form():
    C = oracle.stiffness(*ISO)
    for _ in range(5):
        x = RNG.normal(size=3)
        assert np.allclose(oracle.G_circle(x, C, 64), oracle.G_iso(x, MU, NU, 0.0), rtol=1e-13, atol=1e-16)
        D0 = oracle.dG_iso(x, MU, NU, 0.0)
        assert np.abs(oracle.dG_circle(x, C, 64) - D0).max() <= 1e-13 * np.abs(D0).max()
    # the isotropic crystal given through other constants (Zener ratio 1)
    C = oracle.stiffness(1.0, 0.6, 0.2)
    mu, nu = 0.2, 0.6 / (2 * (0.6 + 0.2))
    x = RNG.normal(size=3)
    D0 = oracle.dG_iso(x, mu, nu, 0.0)
    assert np.abs(oracle.dG_circle(x, C, 64) - D0).max() <= 1e-13 * np.abs(D0).max()


@pytest.mark.parametrize("cub", [(1.0, 0.6, 0.5), (1.0, 0.6, 2.0), (1.0, 0.6, 0.02)])
def test_circle_dG_is_derivative_of_circle_G(cub):
    C = oracle.stiffness(*cub)
    h = 1e-5
    for _ in range(3):
        x = RNG.normal(size=3)
        D = oracle.dG_circle(x, C, 256)
        for q in range(3):
            e = np.zeros(3)
            e[q] = h
            fd = (oracle.G_circle(x + e, C, 256) - oracle.G_circle(x - e, C, 256)) / (2 * h)
            assert np.abs(D[:, :, q] - fd).max() <= 1e-7 * np.abs(D).max()


def test_circle_quadrature_converges_in_nphi():
    C = oracle.stiffness(1.0, 0.6, 0.5)  # Zener ratio 2.5
    x = RNG.normal(size=3)
    ref = oracle.dG_circle(x, C, 512)
    assert np.abs(oracle.dG_circle(x, C, 64) - ref).max() <= 1e-11 * np.abs(ref).max()
    assert np.abs(oracle.dG_circle(x, C, 16) - ref).max() > 1e-9 * np.abs(ref).max()


def test_circle_dG_symmetries():
    C = oracle.stiffness(1.0, 0.6, 0.5)
    x = RNG.normal(size=3)
    D = oracle.dG_circle(x, C, 64)
    assert np.abs(D - D.transpose(1, 0, 2)).max() <= 1e-14 * np.abs(D).max()
    assert np.abs(oracle.dG_circle(-x, C, 64) + D).max() <= 1e-14 * np.abs(D).max()
    assert np.abs(oracle.dG_circle(3.0 * x, C, 64) - D / 9.0).max() <= 1e-14 * np.abs(D).max()
    # cubic symmetry: a 90 degree rotation about z maps the medium to itself
    Rz = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1.0]])
    Dr = oracle.dG_circle(Rz @ x, C, 64)
    Dt = np.einsum("ai,bj,ck,ijk->abc", Rz, Rz, Rz, D)
    assert np.abs(Dr - Dt).max() <= 1e-13 * np.abs(D).max()


def test_regularised_anisotropic_kernel_limits():
    a = 1e-3
    cub = oracle.medium(1.0, 0.6, 0.5, a)
    C = oracle.stiffness(1.0, 0.6, 0.5)
    # R >> a: the singular anisotropic derivative
    x = RNG.normal(size=3)
    x *= 0.5 / np.linalg.norm(x)
    D = oracle.dG_medium(x, cub)
    Ds = oracle.dG_circle(x, C, 64)
    assert np.abs(D - Ds).max() <= 1e-5 * np.abs(Ds).max()
    # bounded at the core and zero at the origin
    assert np.all(oracle.dG_medium(np.zeros(3), cub) == 0.0)
    for r in (1e-6, 1e-4, 1e-3, 3e-3):
        xr = x / np.linalg.norm(x) * r
        assert np.abs(oracle.dG_medium(xr, cub)).max() < 10.0 / a ** 2
    # continuity across the isotropic switch: a medium whose Zener ratio is 1 + 1e-9
    eps = 1e-9
    near = oracle.medium(ISO[0], ISO[1], ISO[2] * (1 + eps), a)
    for r in (2e-4, 1e-3, 0.1):
        xr = x / np.linalg.norm(x) * r
        Di = oracle.dG_iso(xr, MU, NU, a)
        assert np.abs(oracle.dG_medium(xr, near) - Di).max() <= 1e-7 * np.abs(Di).max()


# ------------------------------------------------ straight dislocations
def graded_line(M, L, b, fine=0.05):
    u = np.linspace(-1, 1, M + 1)
    z = np.sinh(u * np.arcsinh(L / fine)) * fine
    seg = np.zeros((M, 2, 3))
    seg[:, 0, 2] = z[:-1]
    seg[:, 1, 2] = z[1:]
    return seg, np.tile(np.asarray(b, float), (M, 1))


def test_screw_stress_matches_hirth_lothe():
    seg, bb = graded_line(600, 1e4, [0, 0, 1.0])
    y, q = oracle.points(seg, bb)
    pts = np.array([[1.0, 0, 0], [0, 1.0, 0], [0.6, -0.8, 0.0]])
    sig = oracle.stress(pts, y, q, iso_med())
    for (X, Y, _), s in zip(pts, sig):
        r2 = X * X + Y * Y
        ref = np.array([0, 0, 0, MU * X / (2 * np.pi * r2), -MU * Y / (2 * np.pi * r2), 0])
        assert np.abs(s - ref).max() <= 1e-7 * MU / (2 * np.pi)


def test_edge_stress_matches_hirth_lothe():
    seg, bb = graded_line(1200, 1e4, [1.0, 0, 0])
    y, q = oracle.points(seg, bb)
    pts = np.array([[0.7, 0.4, 0.0], [-0.3, 0.9, 0.0], [1.1, -0.5, 0.0]])
    sig = oracle.stress(pts, y, q, iso_med())
    Dd = MU / (2 * np.pi * (1 - NU))
    for (X, Y, _), s in zip(pts, sig):
        r2 = X * X + Y * Y
        sxx = -Dd * Y * (3 * X * X + Y * Y) / r2 ** 2
        syy = Dd * Y * (X * X - Y * Y) / r2 ** 2
        sxy = Dd * X * (X * X - Y * Y) / r2 ** 2
        ref = np.array([sxx, syy, NU * (sxx + syy), 0, 0, sxy])
        assert np.abs(s - ref).max() <= 1e-6 * Dd


def _pair_force(b1, b2, d, M=400, L=2e3):
    """Force per unit length on line 2 (through (d,0,0)) from line 1 (through 0)."""
    s1, bb1 = graded_line(M, L, b1)
    s2, bb2 = graded_line(M, L, b2)
    s2[:, :, 0] += d
    seg = np.concatenate([s1, s2])
    bb = np.concatenate([bb1, bb2])
    mid = M + M // 2  # a segment of line 2 at z ~ 0
    f = oracle.direct_forces(seg, bb, iso_med(), targets=[mid])[0]
    # subtract the self-stress of line 2 by computing with line 1 only
    f_self = oracle.direct_forces(s2, bb2, iso_med(), targets=[M // 2])[0]
    length = s2[M // 2, 1, 2] - s2[M // 2, 0, 2]
    return (f - f_self).sum(axis=0) / length


def test_like_screws_repel_with_textbook_magnitude():
    fx, fy, fz = _pair_force([0, 0, 1.0], [0, 0, 1.0], 1.0)
    assert fx > 0  # away from the other line
    assert abs(fx - MU / (2 * np.pi)) <= 1e-5 and abs(fy) < 1e-9 and abs(fz) < 1e-9
    fx2, _, _ = _pair_force([0, 0, 1.0], [0, 0, -1.0], 1.0)
    assert fx2 < 0  # opposite screws attract


def test_parallel_edges_glide_force():
    X = 1.0
    fx, fy, fz = _pair_force([1.0, 0, 0], [1.0, 0, 0], X)
    # F_x = D b^2 x (x^2 - y^2) / r^4 on the plane y = 0
    Dd = MU / (2 * np.pi * (1 - NU))
    assert abs(fx - Dd / X) <= 1e-5


# ----------------------------------------------------------- force assembly
def test_force_assembly_shape_functions_exact_for_linear_stress():
    seg = np.array([[[0.1, 0.2, 0.3], [0.5, -0.1, 0.9]]])
    b = np.array([[0.3, -0.7, 0.2]])
    u, w = oracle.gauss_legendre(3)
    s = 0.5 * (1 + u)
    s0 = RNG.normal(size=6)
    s1 = RNG.normal(size=6)
    sig = np.stack([s0 + sk * s1 for sk in s])

    def pk(sv):
        S = np.array([[sv[0], sv[5], sv[4]], [sv[5], sv[1], sv[3]], [sv[4], sv[3], sv[2]]])
        return np.cross(S @ b[0], seg[0, 1] - seg[0, 0])

    f = oracle.assemble_forces(seg, b, [0], sig)[0]
    # int_0^1 (1-s)(s0 + s s1) ds = s0/2 + s1/6 ; int_0^1 s(s0 + s s1) ds = s0/2 + s1/3
    assert np.allclose(f[0], pk(s0 / 2 + s1 / 6), rtol=1e-13, atol=1e-15)
    assert np.allclose(f[1], pk(s0 / 2 + s1 / 3), rtol=1e-13, atol=1e-15)


def test_quadrature_sum_converges_to_line_integral():
    """Brute force: the n-point sum of Eq. stress_discrete tends to the line
    integral of Eq. stress evaluated by adaptive quadrature."""
    x1, x2 = np.array([0.0, 0.0, 0.0]), np.array([0.3, 0.1, 0.2])
    b = np.array([0.5, -0.5, 0.7071067811865476])
    xt = np.array([[0.4, -0.2, 0.5]])
    for med in (iso_med(1e-3), oracle.medium(1.0, 0.6, 0.5, 1e-3)):
        dS = x2 - x1

        def integrand(t, ab):
            K = oracle.kernel_batch((xt[0] - (x1 + t * dS))[None], med)[0]
            return K[ab] @ np.outer(b, dS).reshape(9)

        ref = np.array([integrate.quad(integrand, 0, 1, args=(ab,), epsabs=1e-14, epsrel=1e-12)[0]
                        for ab in range(6)])
        for nq, tol in ((3, 2e-2), (8, 1e-6), (16, 1e-11)):
            y, q = oracle.points(np.array([[x1, x2]]), b[None], nq)
            s = oracle.stress(xt, y, q, med)[0]
            assert np.abs(s - ref).max() <= tol * np.abs(ref).max(), (nq, np.abs(s - ref).max())


# ------------------------------------------------------- whole-sum pins
def _loops(n, seed, r=(0.01, 0.05)):
    return synth.make_loops(n, r[0], r[1], seed)


@pytest.mark.parametrize("cub", [ISO, (1.0, 0.6, 0.5)])
def test_closed_loop_net_force_and_action_reaction(cub):
    seg, b = _loops(2, 7, r=(0.05, 0.08))
    nq = 6
    med = oracle.medium(*cub, 1e-3)
    f = oracle.direct_forces(seg, b, med, nq=nq)
    scale = np.abs(f).sum()
    fA = f[:40].sum(axis=(0, 1))
    fB = f[40:].sum(axis=(0, 1))
    # self-force of each loop and the pair force: computed separately
    fAA = oracle.direct_forces(seg[:40], b[:40], med, nq=nq).sum(axis=(0, 1))
    fBB = oracle.direct_forces(seg[40:], b[40:], med, nq=nq).sum(axis=(0, 1))
    assert np.abs(fAA).max() < 1e-3 * scale and np.abs(fBB).max() < 1e-3 * scale
    fAB, fBA = fA - fAA, fB - fBB
    assert np.abs(fAB + fBA).max() < 1e-3 * np.abs(fAB).max()


def test_scaling_rotation_linearity():
    seg, b = _loops(3, 11)
    med = iso_med(1e-3)
    tgt = [0, 17, 55, 101]
    f = oracle.direct_forces(seg, b, med, targets=tgt)
    # x -> 3x, a -> 3a: forces unchanged
    f3 = oracle.direct_forces(3 * seg, b, oracle.medium(*ISO, 3e-3), targets=tgt)
    assert np.allclose(f3, f, rtol=1e-10, atol=1e-12 * np.abs(f).max())
    # linear in b, proportional to the moduli
    assert np.allclose(oracle.direct_forces(seg, 2 * b, med, targets=tgt), 4 * f, rtol=1e-12,
                       atol=1e-14 * np.abs(f).max())
    med2 = oracle.medium(*(2 * np.array(ISO)), 1e-3)
    assert np.allclose(oracle.direct_forces(seg, b, med2, targets=tgt), 2 * f, rtol=1e-12,
                       atol=1e-14 * np.abs(f).max())
    # any rotation (isotropic)
    Q, _ = np.linalg.qr(RNG.normal(size=(3, 3)))
    fr = oracle.direct_forces(seg @ Q.T, b @ Q.T, med, targets=tgt)
    assert np.allclose(fr, f @ Q.T, rtol=1e-9, atol=1e-11 * np.abs(f).max())
    # cubic medium: a cube symmetry (90 degrees about x)
    cub = oracle.medium(1.0, 0.6, 0.5, 1e-3)
    Rx = np.array([[1, 0, 0], [0, 0, -1], [0, 1, 0.0]])
    fc = oracle.direct_forces(seg, b, cub, targets=tgt)
    fcr = oracle.direct_forces(seg @ Rx.T, b @ Rx.T, cub, targets=tgt)
    assert np.allclose(fcr, fc @ Rx.T, rtol=1e-9, atol=1e-11 * np.abs(fc).max())


# ------------------------------------------- cube symmetry of the kernel
@pytest.mark.parametrize("C,a", [((1.0, 0.6, 0.5), 1e-3), (ISO, 0.0), (ISO, 2e-2)])
def test_kernel_transforms_under_the_cube_group(C, a):
    """The reading behind the symmetry-reduced M2L store (Sec. 6): for every
    signed permutation R of the axes (48 elements, which leave a cubic or
    isotropic stiffness unchanged), K(R x) = det(R) R.R.R.R K(x) on the
    kernel's four indices (the det from the Levi-Civita symbol in Eq.
    kernel).  Checked on the oracle's kernel at random points, and shown to
    fail without the det for the improper elements."""
    import itertools

    VA, VB = (0, 1, 2, 1, 0, 0), (0, 1, 2, 2, 2, 1)

    def full(K6):
        F = np.zeros((3, 3, 3, 3))
        for ab in range(6):
            F[VA[ab], VB[ab]] = K6[ab]
            F[VB[ab], VA[ab]] = K6[ab]
        return F

    med = oracle.medium(*C, a)
    rng = np.random.default_rng(8)
    for x in rng.normal(size=(3, 3)) * 0.05:
        K = full(oracle.kernel_batch(x[None], med)[0].reshape(6, 3, 3))
        scale = np.abs(K).max()
        for perm in itertools.permutations(range(3)):
            for sg in itertools.product((1, -1), repeat=3):
                R = np.zeros((3, 3))
                for i in range(3):
                    R[i, perm[i]] = sg[i]
                d = round(np.linalg.det(R))
                KR = full(oracle.kernel_batch((R @ x)[None], med)[0].reshape(6, 3, 3))
                T = np.einsum("ai,bj,wk,rl,ijkl->abwr", R, R, R, R, K)
                assert np.abs(KR - d * T).max() <= 1e-12 * scale
                if d < 0:
                    assert np.abs(KR - T).max() > 1e-3 * scale


# ------------------------------------------- the core reading R1 against R2
def dG_spread(x, C, a, n_u=600, n_phi=256):
    """d_q G_vp of the Green's function with the delta of the plane-wave form
    spread as rho_a(s) = (3/4) a^4 (s^2 + a^2)^(-5/2) (the non-singular
    spreading the paper cites for the isotropic case, written for any C):
    G_a(x) = 1/(8 pi^2) int_{S^2} (kCk)^{-1} rho_a(k.x) dk, so
    d_q G_a = 1/(8 pi^2) int (kCk)^{-1} k_q rho_a'(k.x) dk.  Product
    Gauss-Legendre in u = k.x/|x| times the trapezoid rule in the angle
    about x.  Test-only reference for the regularisation reading."""
    x = np.asarray(x, dtype=np.float64)
    R = np.linalg.norm(x)
    xh = x / R
    t = np.array([1.0, 0.0, 0.0]) if abs(xh[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(xh, t)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(xh, e1)
    u, wu = np.polynomial.legendre.leggauss(n_u)
    phi = 2 * np.pi * np.arange(n_phi) / n_phi
    st = np.sqrt(1 - u ** 2)
    k = u[:, None, None] * xh + st[:, None, None] * (np.cos(phi)[None, :, None] * e1 + np.sin(phi)[None, :, None] * e2)
    M = np.linalg.inv(np.einsum("ijkl,abj,abl->abik", C, k, k))
    s = R * u
    drho = -(15.0 / 4.0) * a ** 4 * s * (s * s + a * a) ** -3.5
    return np.einsum("a,abvp,abq,a->vpq", wu, M, k, drho) * (2 * np.pi / n_phi) / (8 * np.pi ** 2)


def test_spread_core_reduces_to_the_isotropic_closed_form():
    """The spread-core reference with an isotropic C equals the closed-form
    dG with R -> R_a (independent formulas), at R = a, 3a, 10a."""
    a, mu, nu = 1e-3, 1.0, 0.3
    lam = 2 * mu * nu / (1 - 2 * nu)
    C = oracle.stiffness(lam + 2 * mu, lam, mu)
    d = np.array([0.3, -0.5, 0.81])
    d /= np.linalg.norm(d)
    for f in (1.0, 3.0, 10.0):
        Di = oracle.dG_iso(f * a * d, mu, nu, a)
        assert np.abs(dG_spread(f * a * d, C, a) - Di).max() <= 1e-12 * np.abs(Di).max()


def test_r1_core_against_the_spread_core():
    """The R1 reading of the cubic core (isotropic Voigt core plus the damped
    anisotropic difference) against the spread core R2, Zener ratio 2.5.
    They differ by up to ~30% of the kernel for R <~ a; the difference then
    falls like (a/R)^2 with the singular kernel's own, ~2% at 10a and ~0.2%
    at 30a, so R1 changes only near-coincident pairs."""
    a = 1e-3
    C = oracle.stiffness(1.0, 0.6, 0.5)
    med = oracle.medium(1.0, 0.6, 0.5, a)
    rng = np.random.default_rng(1)
    for trial in range(2):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        diffs = []
        for f in (1.0, 2.0, 3.0, 5.0, 10.0, 30.0):
            D2 = dG_spread(f * a * d, C, a)
            D1 = oracle.dG_medium(f * a * d, med)
            diffs.append(np.abs(D1 - D2).max() / np.abs(D2).max())
        print("R1 vs R2 at R/a = 1, 2, 3, 5, 10, 30:", ["%.2e" % v for v in diffs])
        assert all(d1 < d0 for d0, d1 in zip(diffs[1:], diffs[2:]))
        assert diffs[0] < 0.4 and diffs[4] < 3e-2 and diffs[5] < 5e-3
