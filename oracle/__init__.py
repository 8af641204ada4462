"""FP64 CPU oracle for dislocation stress and Peach-Koehler forces.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are its only users.  The GPU library never imports, links or
calls it, and it shares no code with the GPU library; the only common module is
the seeded loop generator in ``synth``.

Two references live here:
  * ``direct_forces`` -- the plain O(N^2) sum of Eq. stress3 over all
    quadrature points (C, FP64, Neumaier-compensated), then the end-point
    force quadrature.  This is the definition the FMM approximates.
  * ``fmm_forces`` -- the Lagrange FMM of Sec. 4 (Alg. lagrange) written out
    step by step in numpy FP64, with the M2L step evaluated as the plain dense
    sum over interpolation nodes (Eq. m2l), no FFT.  The GPU FMM must agree
    with it to rounding; it must agree with ``direct_forces`` to the
    interpolation error.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dfmm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (OpenMP) into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        d = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        L = _lib
        L.or_gauss_legendre.argtypes = [ctypes.c_int, d, d]
        L.or_stiffness.argtypes = [ctypes.c_double] * 3 + [d]
        L.or_G_iso.argtypes = [d, ctypes.c_double, ctypes.c_double, ctypes.c_double, d]
        L.or_dG_iso.argtypes = [d, ctypes.c_double, ctypes.c_double, ctypes.c_double, d]
        L.or_G_circle.argtypes = [d, d, ctypes.c_int, d]
        L.or_dG_circle.argtypes = [d, d, ctypes.c_int, d]
        L.or_dG_medium.argtypes = [d, d, d]
        L.or_kernel54.argtypes = [d, d, d]
        L.or_kernel_batch.argtypes = [i64, d, d, d]
        L.or_stress.argtypes = [i64, d, i64, d, d, d, d]
        L.or_points.argtypes = [i64, d, d, ctypes.c_int, d, d]
        L.or_assemble_forces.argtypes = [i64, ctypes.POINTER(ctypes.c_int64), d, d, ctypes.c_int, d, d]
        L.or_forces.argtypes = [i64, d, d, d, ctypes.c_int, i64, ctypes.POINTER(ctypes.c_int64), d]
        L.or_forces.restype = ctypes.c_int
        L.or_num_threads.restype = ctypes.c_int
        L.or_set_threads.argtypes = [ctypes.c_int]
        L.or_voigt.argtypes = [d, d, d]
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _pi(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def num_threads() -> int:
    return lib().or_num_threads()


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


# --------------------------------------------------------------------------
# Medium helpers
def medium(c11, c12, c44, a, nphi=64):
    """Packed medium description [c11, c12, c44, a, nphi]."""
    return np.array([c11, c12, c44, a, float(nphi)], dtype=np.float64)


def medium_from_params(prm, nphi=64):
    return medium(prm["c11"], prm["c12"], prm["c44"], prm["core_a"], nphi)


def gauss_legendre(n):
    u = np.empty(n)
    w = np.empty(n)
    lib().or_gauss_legendre(n, _p(u), _p(w))
    return u, w


def stiffness(c11, c12, c44):
    C = np.empty(81)
    lib().or_stiffness(c11, c12, c44, _p(C))
    return C.reshape(3, 3, 3, 3)


def voigt(med):
    mu = ctypes.c_double()
    nu = ctypes.c_double()
    lib().or_voigt(_p(_f64(med)), ctypes.byref(mu), ctypes.byref(nu))
    return mu.value, nu.value


def G_iso(x, mu, nu, a):
    G = np.empty(9)
    lib().or_G_iso(_p(_f64(x)), mu, nu, a, _p(G))
    return G.reshape(3, 3)


def dG_iso(x, mu, nu, a):
    D = np.empty(27)
    lib().or_dG_iso(_p(_f64(x)), mu, nu, a, _p(D))
    return D.reshape(3, 3, 3)


def G_circle(x, C, nphi):
    G = np.empty(9)
    lib().or_G_circle(_p(_f64(x)), _p(_f64(C)), nphi, _p(G))
    return G.reshape(3, 3)


def dG_circle(x, C, nphi):
    D = np.empty(27)
    lib().or_dG_circle(_p(_f64(x)), _p(_f64(C)), nphi, _p(D))
    return D.reshape(3, 3, 3)


def dG_medium(x, med):
    D = np.empty(27)
    lib().or_dG_medium(_p(_f64(x)), _p(_f64(med)), _p(D))
    return D.reshape(3, 3, 3)


def kernel54(D, C):
    K = np.empty(54)
    lib().or_kernel54(_p(_f64(D)), _p(_f64(C)), _p(K))
    return K.reshape(6, 3, 3)


def kernel_batch(x, med):
    """K(x) for x[n,3]; returns [n, 6, 9] (Voigt ab, w*3+r)."""
    x = _f64(x).reshape(-1, 3)
    K = np.empty((x.shape[0], 54))
    lib().or_kernel_batch(x.shape[0], _p(x), _p(_f64(med)), _p(K))
    return K.reshape(-1, 6, 9)


def stress(xt, ys, q, med):
    """Eq. stress3: sigma[i] (Voigt) at targets xt from sources (ys, q[j, 9])."""
    xt = _f64(xt).reshape(-1, 3)
    ys = _f64(ys).reshape(-1, 3)
    q = _f64(q).reshape(-1, 9)
    sig = np.empty((xt.shape[0], 6))
    lib().or_stress(xt.shape[0], _p(xt), ys.shape[0], _p(ys), _p(q), _p(_f64(med)), _p(sig))
    return sig


def points(seg, burg, nq=3):
    """Quadrature points y[N,3] and strengths q[N,9] (Eq. stress_discrete)."""
    seg = _f64(seg).reshape(-1, 2, 3)
    burg = _f64(burg).reshape(-1, 3)
    n = seg.shape[0]
    y = np.empty((n * nq, 3))
    q = np.empty((n * nq, 9))
    lib().or_points(n, _p(seg), _p(burg), nq, _p(y), _p(q))
    return y, q


def assemble_forces(seg, burg, tgt, sig_t, nq=3):
    seg = _f64(seg).reshape(-1, 2, 3)
    burg = _f64(burg).reshape(-1, 3)
    tgt = np.ascontiguousarray(tgt, dtype=np.int64)
    sig_t = _f64(sig_t).reshape(-1, 6)
    f = np.empty((tgt.shape[0], 2, 3))
    lib().or_assemble_forces(tgt.shape[0], _pi(tgt), _p(seg), _p(burg), nq, _p(sig_t), _p(f))
    return f


def direct_forces(seg, burg, med, targets=None, nq=3):
    """Direct O(N^2) end-point forces f[t, 2, 3] on the target segments."""
    seg = _f64(seg).reshape(-1, 2, 3)
    burg = _f64(burg).reshape(-1, 3)
    n = seg.shape[0]
    tgt = np.arange(n, dtype=np.int64) if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    f = np.empty((tgt.shape[0], 2, 3))
    rc = lib().or_forces(n, _p(seg), _p(burg), _p(_f64(med)), nq, tgt.shape[0], _pi(tgt), _p(f))
    if rc != 0:
        raise MemoryError("oracle: allocation failed")
    return f


def rel_err(f, ref):
    """Global relative L2 error over all end-point force components."""
    f = np.asarray(f, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(f - ref) / np.linalg.norm(ref))


from .fmm import fmm_forces, fmm_stress  # noqa: E402,F401
