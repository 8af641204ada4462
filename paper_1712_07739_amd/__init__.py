"""Python binding of libdfmm (the gfx950 Lagrange-FMM library for dislocation forces).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in include/dfmm.h.  Device memory comes from
torch tensors (float64, on the current HIP device); the current torch stream is
passed as the HIP stream.  The library must have been built
(``python -m paper_1712_07739_amd.build`` or ``__graft_entry__.build()``);
there is no fallback of any kind.
"""
from __future__ import annotations

import ctypes
import json
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdfmm.so")

DFMM_FP64 = 0
DFMM_MIXED = 1
DFMM_MIXED_F16 = 2
DFMM_M2L_FFT = 0
DFMM_M2L_FFT_SYM = 1
DFMM_KERNEL_EXACT = 0
DFMM_KERNEL_SURROGATE = 1
DFMM_LSQ_AUTO = -1
N_STAGES = 8
STAGES = ("points+P2M", "M2M", "DFT", "M2L-Hadamard", "IDFT", "L2L", "near+L2P", "forces")

ENTRY_POINTS = (
    "dfmm_default_params", "dfmm_fmm_setup", "dfmm_build_tree", "dfmm_fmm_forces",
    "dfmm_direct_forces", "dfmm_tree_set_timing", "dfmm_tree_stage_times", "dfmm_plan_info",
    "dfmm_tree_info", "dfmm_tree_destroy", "dfmm_plan_destroy", "dfmm_status_string",
    "dfmm_last_error", "dfmm_surrogate_default_cfg", "dfmm_surrogate_train", "dfmm_surrogate_use",
    "dfmm_surrogate_info", "dfmm_surrogate_get_params", "dfmm_surrogate_set_params",
    "dfmm_surrogate_loss_grad", "dfmm_surrogate_forward", "dfmm_batch_create", "dfmm_batch_run",
    "dfmm_batch_latencies", "dfmm_batch_destroy", "dfmm_autotune_depth",
    "dfmm_direct_forces_noalloc", "dfmm_direct_noalloc_bytes", "dfmm_surrogate_get_gate",
    "dfmm_surrogate_save", "dfmm_surrogate_load", "dfmm_forces_batched", "dfmm_autotune_batch_lanes",
    "dfmm_tree_check_positions",
)
NOALLOC_SCRATCH_BYTES = 64 << 20


class Params(ctypes.Structure):
    """Mirror of dfmm_params."""

    _fields_ = [
        ("order", ctypes.c_int), ("depth", ctypes.c_int),
        ("c11", ctypes.c_double), ("c12", ctypes.c_double), ("c44", ctypes.c_double),
        ("core_a", ctypes.c_double), ("box_lo", ctypes.c_double * 3), ("box_size", ctypes.c_double),
        ("n_quad", ctypes.c_int), ("n_circle", ctypes.c_int), ("precision", ctypes.c_int),
        ("m2l_mode", ctypes.c_int), ("aniso_kernel", ctypes.c_int), ("lsq_degree", ctypes.c_int),
        ("leaf_max", ctypes.c_int), ("freq_chunks", ctypes.c_int),
    ]


class SurrogateCfg(ctypes.Structure):
    """Mirror of dfmm_surrogate_cfg."""

    _fields_ = [
        ("hidden", ctypes.c_int), ("epochs", ctypes.c_int), ("batch", ctypes.c_int), ("bins", ctypes.c_int),
        ("n_samples", ctypes.c_int64), ("lr", ctypes.c_double), ("tol", ctypes.c_double),
        ("seed", ctypes.c_uint64),
    ]


class DfmmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("dfmm status %d: %s" % (status, msg))
        self.status = status


_lib = None


def lib():
    """Load libdfmm.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libdfmm.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    pp = ctypes.POINTER(ctypes.c_void_p)
    L.dfmm_default_params.argtypes = [ctypes.POINTER(Params)]
    L.dfmm_fmm_setup.argtypes = [ctypes.POINTER(Params), vp, pp]
    L.dfmm_build_tree.argtypes = [vp, vp, i64, vp, pp]
    L.dfmm_fmm_forces.argtypes = [vp, vp, vp, vp, vp, vp]
    L.dfmm_direct_forces.argtypes = [vp, vp, vp, i64, vp, i64, vp, i32, vp]
    L.dfmm_direct_forces_noalloc.argtypes = [vp, vp, vp, i64, vp, i64, vp, i32, vp]
    L.dfmm_direct_noalloc_bytes.argtypes = [vp, i64, i64]
    L.dfmm_direct_noalloc_bytes.restype = ctypes.c_size_t
    L.dfmm_tree_set_timing.argtypes = [vp, i32]
    L.dfmm_tree_stage_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32)]
    L.dfmm_plan_info.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
    L.dfmm_tree_info.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
    L.dfmm_tree_check_positions.argtypes = [vp, vp, vp, vp]
    L.dfmm_tree_destroy.argtypes = [vp]
    L.dfmm_plan_destroy.argtypes = [vp]
    L.dfmm_status_string.argtypes = [i32]
    L.dfmm_status_string.restype = ctypes.c_char_p
    L.dfmm_last_error.restype = ctypes.c_char_p
    L.dfmm_surrogate_default_cfg.argtypes = [ctypes.POINTER(SurrogateCfg)]
    L.dfmm_surrogate_train.argtypes = [vp, ctypes.POINTER(SurrogateCfg), vp]
    L.dfmm_surrogate_use.argtypes = [vp, i32, vp]
    L.dfmm_surrogate_info.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
    L.dfmm_surrogate_get_params.argtypes = [vp, vp, i64, ctypes.POINTER(i64)]
    L.dfmm_surrogate_set_params.argtypes = [vp, vp, i64]
    L.dfmm_surrogate_loss_grad.argtypes = [vp, vp, vp, i64, vp, ctypes.POINTER(ctypes.c_double), vp]
    L.dfmm_surrogate_forward.argtypes = [vp, vp, i64, vp, vp]
    L.dfmm_surrogate_get_gate.argtypes = [vp, vp, i64, ctypes.POINTER(i32)]
    L.dfmm_surrogate_save.argtypes = [vp, ctypes.c_char_p]
    L.dfmm_surrogate_load.argtypes = [vp, ctypes.c_char_p, vp]
    L.dfmm_batch_create.argtypes = [vp, vp, vp, vp, vp, i32, i32, vp, pp]
    L.dfmm_batch_run.argtypes = [vp, vp]
    L.dfmm_batch_latencies.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i32]
    L.dfmm_batch_destroy.argtypes = [vp]
    L.dfmm_forces_batched.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int, vp]
    L.dfmm_autotune_batch_lanes.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int, ctypes.c_int, vp,
                                            ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
    L.dfmm_autotune_depth.argtypes = [ctypes.POINTER(Params), vp, vp, i64, i32, i32, vp, ctypes.POINTER(i32),
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    for name in ENTRY_POINTS:
        getattr(L, name)
    _lib = L
    return L


def _check(rc):
    if rc != 0:
        L = lib()
        raise DfmmError(rc, "%s (%s)" % (L.dfmm_status_string(rc).decode(), L.dfmm_last_error().decode()))


def _stream(stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f64(t, shape, name):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError("%s must be a float64 tensor on the GPU" % name)
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    return t.contiguous()


def default_params():
    p = Params()
    lib().dfmm_default_params(ctypes.byref(p))
    return p


def make_params(order, depth, c11, c12, c44, core_a, box_lo, box_size, n_quad=3, n_circle=64,
                precision=DFMM_FP64, m2l_mode=DFMM_M2L_FFT, aniso_kernel=DFMM_KERNEL_EXACT, lsq_degree=0, leaf_max=0, freq_chunks=0):
    p = default_params()
    p.m2l_mode, p.aniso_kernel, p.lsq_degree = int(m2l_mode), int(aniso_kernel), int(lsq_degree)
    p.leaf_max, p.freq_chunks = int(leaf_max), int(freq_chunks)
    p.order, p.depth = int(order), int(depth)
    p.c11, p.c12, p.c44, p.core_a = float(c11), float(c12), float(c44), float(core_a)
    for i in range(3):
        p.box_lo[i] = float(box_lo[i])
    p.box_size = float(box_size)
    p.n_quad, p.n_circle, p.precision = int(n_quad), int(n_circle), int(precision)
    return p


class Plan:
    """dfmm_fmm_setup: per-level M2L operator spectra for one medium/order/depth."""

    def __init__(self, params: Params, stream=None):
        self.params = params
        self._h = ctypes.c_void_p()
        _check(lib().dfmm_fmm_setup(ctypes.byref(params), _stream(stream), ctypes.byref(self._h)))

    @property
    def handle(self):
        return self._h

    def info(self):
        buf = ctypes.create_string_buffer(4096)
        _check(lib().dfmm_plan_info(self._h, buf, 4096))
        return json.loads(buf.value.decode())

    # ---- learned surrogate of the anisotropic kernel
    def surrogate_train(self, stream=None, **cfg):
        c = SurrogateCfg()
        lib().dfmm_surrogate_default_cfg(ctypes.byref(c))
        for k, v in cfg.items():
            setattr(c, k, v)
        _check(lib().dfmm_surrogate_train(self._h, ctypes.byref(c), _stream(stream)))
        return self.surrogate_info()

    def surrogate_use(self, on: bool, stream=None):
        _check(lib().dfmm_surrogate_use(self._h, 1 if on else 0, _stream(stream)))

    def surrogate_info(self):
        buf = ctypes.create_string_buffer(1 << 16)
        _check(lib().dfmm_surrogate_info(self._h, buf, 1 << 16))
        return json.loads(buf.value.decode())

    def surrogate_params(self):
        import numpy as np

        n = ctypes.c_int64()
        _check(lib().dfmm_surrogate_get_params(self._h, None, 0, ctypes.byref(n)))
        out = np.empty(n.value, dtype=np.float32)
        _check(lib().dfmm_surrogate_get_params(self._h, ctypes.c_void_p(out.ctypes.data), n.value, ctypes.byref(n)))
        return out

    def surrogate_set_params(self, params):
        import numpy as np

        a = np.ascontiguousarray(params, dtype=np.float32)
        _check(lib().dfmm_surrogate_set_params(self._h, ctypes.c_void_p(a.ctypes.data), a.size))

    def surrogate_loss_grad(self, X, Y, stream=None):
        """Loss and gradient for device float32 rows X [n,6], Y [n,18]."""
        import torch

        n = int(X.shape[0])
        g = torch.empty(int(self.surrogate_params().size), dtype=torch.float32, device=X.device)
        loss = ctypes.c_double()
        _check(lib().dfmm_surrogate_loss_grad(self._h, ctypes.c_void_p(X.contiguous().data_ptr()),
                                              ctypes.c_void_p(Y.contiguous().data_ptr()), n,
                                              ctypes.c_void_p(g.data_ptr()), ctypes.byref(loss), _stream(stream)))
        return loss.value, g

    def surrogate_gate(self):
        """The residual gate: uint8 array [6, bins, bins], 1 where the network is used."""
        import numpy as np

        bins = ctypes.c_int()
        _check(lib().dfmm_surrogate_get_gate(self._h, None, 0, ctypes.byref(bins)))
        out = np.empty((6, bins.value, bins.value), dtype=np.uint8)
        _check(lib().dfmm_surrogate_get_gate(self._h, ctypes.c_void_p(out.ctypes.data), out.size, ctypes.byref(bins)))
        return out

    def surrogate_save(self, path):
        _check(lib().dfmm_surrogate_save(self._h, os.fsencode(path)))

    def surrogate_load(self, path, stream=None):
        _check(lib().dfmm_surrogate_load(self._h, os.fsencode(path), _stream(stream)))

    def surrogate_forward(self, X, stream=None):
        import torch

        n = int(X.shape[0])
        Y = torch.empty((n, 18), dtype=torch.float32, device=X.device)
        _check(lib().dfmm_surrogate_forward(self._h, ctypes.c_void_p(X.contiguous().data_ptr()), n,
                                            ctypes.c_void_p(Y.data_ptr()), _stream(stream)))
        return Y

    def close(self):
        if self._h:
            lib().dfmm_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tree:
    """dfmm_build_tree: octree + workspaces for one set of segment positions."""

    def __init__(self, plan: Plan, seg, stream=None):
        self.plan = plan
        self.n_seg = int(seg.shape[0])
        self._seg = _dev_f64(seg, (self.n_seg, 2, 3), "seg")
        self._h = ctypes.c_void_p()
        _check(lib().dfmm_build_tree(plan.handle, ctypes.c_void_p(self._seg.data_ptr()), self.n_seg,
                                     _stream(stream), ctypes.byref(self._h)))

    @property
    def handle(self):
        return self._h

    def info(self):
        buf = ctypes.create_string_buffer(1 << 16)
        _check(lib().dfmm_tree_info(self._h, buf, 1 << 16))
        return json.loads(buf.value.decode())

    def set_timing(self, on: bool):
        _check(lib().dfmm_tree_set_timing(self._h, 1 if on else 0))

    def stage_times(self):
        ms = (ctypes.c_double * N_STAGES)()
        n = ctypes.c_int()
        _check(lib().dfmm_tree_stage_times(self._h, ms, ctypes.byref(n)))
        return list(ms), n.value

    def close(self):
        if self._h:
            lib().dfmm_tree_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fmm_forces(plan: Plan, tree: Tree, seg, burgers, out=None, stream=None):
    """Lagrange-FMM end-point forces [n_seg, 2, 3] (float64, on the GPU)."""
    import torch

    n = tree.n_seg
    seg = _dev_f64(seg, (n, 2, 3), "seg")
    burgers = _dev_f64(burgers, (n, 3), "burgers")
    if out is None:
        out = torch.empty((n, 2, 3), dtype=torch.float64, device=seg.device)
    else:
        out = _dev_f64(out, (n, 2, 3), "out")
    _check(lib().dfmm_fmm_forces(plan.handle, tree.handle, ctypes.c_void_p(seg.data_ptr()),
                                 ctypes.c_void_p(burgers.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                 _stream(stream)))
    return out


def tree_check_positions(plan: Plan, tree: Tree, seg, stream=None):
    """Raise DfmmError (DFMM_E_STATE) unless `seg` holds, bit for bit, the
    positions `tree` was built from (synchronises the stream)."""
    seg = _dev_f64(seg, (tree.n_seg, 2, 3), "seg")
    _check(lib().dfmm_tree_check_positions(plan.handle, tree.handle, ctypes.c_void_p(seg.data_ptr()),
                                           _stream(stream)))


def direct_forces(plan: Plan, seg, burgers, targets=None, fp32=False, out=None, stream=None, noalloc=False):
    """Direct O(N^2) end-point forces on `targets` (int64 GPU tensor, or all).

    noalloc=True calls dfmm_direct_forces_noalloc (scratch in the library's
    fixed per-GPU array; `out` should then be given by the caller)."""
    import torch

    n = int(seg.shape[0])
    seg = _dev_f64(seg, (n, 2, 3), "seg")
    burgers = _dev_f64(burgers, (n, 3), "burgers")
    if targets is None:
        nt, tptr = n, ctypes.c_void_p(0)
    else:
        if not targets.is_cuda or targets.dtype != torch.int64:
            raise TypeError("targets must be an int64 tensor on the GPU")
        targets = targets.contiguous()
        nt, tptr = int(targets.numel()), ctypes.c_void_p(targets.data_ptr())
    if out is None:
        out = torch.empty((nt, 2, 3), dtype=torch.float64, device=seg.device)
    fn = lib().dfmm_direct_forces_noalloc if noalloc else lib().dfmm_direct_forces
    _check(fn(plan.handle, ctypes.c_void_p(seg.data_ptr()), ctypes.c_void_p(burgers.data_ptr()), n, tptr, nt,
              ctypes.c_void_p(out.data_ptr()), 1 if fp32 else 0, _stream(stream)))
    return out


def direct_noalloc_bytes(plan: Plan, n_seg, n_targets):
    """Scratch bytes dfmm_direct_forces_noalloc needs for these sizes."""
    return int(lib().dfmm_direct_noalloc_bytes(plan.handle, int(n_seg), int(n_targets)))


class Batch:
    """dfmm_batch_create: the force evaluations of many (plan, tree, seg,
    burgers, forces) configurations captured into one HIP graph."""

    def __init__(self, plans, trees, segs, burgers, forces, lanes=4, stream=None):
        n = len(plans)
        assert len(trees) == len(segs) == len(burgers) == len(forces) == n
        self._keep = (plans, trees, segs, burgers, forces)
        P = ctypes.c_void_p * n
        self._args = (P(*[p.handle for p in plans]), P(*[t.handle for t in trees]),
                      P(*[s.data_ptr() for s in segs]), P(*[b.data_ptr() for b in burgers]),
                      P(*[f.data_ptr() for f in forces]))
        self.n = n
        self._h = ctypes.c_void_p()
        _check(lib().dfmm_batch_create(*[ctypes.cast(a, ctypes.c_void_p) for a in self._args], n, lanes,
                                       _stream(stream), ctypes.byref(self._h)))

    def run(self, stream=None):
        _check(lib().dfmm_batch_run(self._h, _stream(stream)))

    def latencies_ms(self):
        ms = (ctypes.c_double * self.n)()
        _check(lib().dfmm_batch_latencies(self._h, ms, self.n))
        return list(ms)

    def close(self):
        if self._h:
            lib().dfmm_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def forces_batched(plans, trees, segs, burgers, forces, stream=None):
    """dfmm_forces_batched: the force evaluations of many configurations in
    one graph launch, returned when all are written (forces: caller tensors)."""
    n = len(plans)
    assert len(trees) == len(segs) == len(burgers) == len(forces) == n
    P = ctypes.c_void_p * n
    args = (P(*[p.handle for p in plans]), P(*[t.handle for t in trees]), P(*[x.data_ptr() for x in segs]),
            P(*[x.data_ptr() for x in burgers]), P(*[x.data_ptr() for x in forces]))
    _check(lib().dfmm_forces_batched(*[ctypes.cast(a, ctypes.c_void_p) for a in args], n, _stream(stream)))
    return forces


def autotune_batch_lanes(plans, trees, segs, burgers, forces, reps=3, stream=None):
    """dfmm_autotune_batch_lanes: the batch graph's branch count with the
    smallest mean replay time; returns (best, {branches: ms})."""
    n = len(plans)
    P = ctypes.c_void_p * n
    args = (P(*[p.handle for p in plans]), P(*[t.handle for t in trees]), P(*[x.data_ptr() for x in segs]),
            P(*[x.data_ptr() for x in burgers]), P(*[x.data_ptr() for x in forces]))
    best = ctypes.c_int()
    ms = (ctypes.c_double * 4)()
    _check(lib().dfmm_autotune_batch_lanes(*[ctypes.cast(a, ctypes.c_void_p) for a in args], n, reps,
                                           _stream(stream), ctypes.byref(best), ms))
    return best.value, {b: ms[k] for k, b in enumerate((1, 2, 4, 8)) if ms[k] > 0}


def autotune_depth(params: Params, seg, burgers, d_min=3, d_max=7, stream=None):
    """dfmm_autotune_depth: the App. B cost model's fastest depth and its
    neighbours are timed; returns (best depth, predicted ms per depth,
    measured ms per timed depth)."""
    n = int(seg.shape[0])
    seg = _dev_f64(seg, (n, 2, 3), "seg")
    burgers = _dev_f64(burgers, (n, 3), "burgers")
    best = ctypes.c_int()
    k = d_max - d_min + 1
    pred = (ctypes.c_double * k)()
    meas = (ctypes.c_double * k)()
    _check(lib().dfmm_autotune_depth(ctypes.byref(params), ctypes.c_void_p(seg.data_ptr()),
                                     ctypes.c_void_p(burgers.data_ptr()), n, d_min, d_max, _stream(stream),
                                     ctypes.byref(best), pred, meas))
    return (best.value, {d_min + i: pred[i] for i in range(k)},
            {d_min + i: meas[i] for i in range(k) if meas[i] > 0})
