"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars: direct sum FP64 <= 1e-12 and FP32 <= 1e-6 relative (global L2 over all
end-point force components); GPU FMM vs the oracle's plain FMM (same
approximation, dense M2L) <= 1e-10 in FP64; mixed precision <= 2e-5 of the
FP64 FMM; FMM vs the direct sum <= 1e-4 at the orders the workloads use.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BOX_LO, BOX = synth.loops.BOX_LO, synth.loops.BOX_SIZE
ISO = synth.loops.ISO
CUB = synth.loops.CUBIC_A25


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_1712_07739_amd as pk

    assert torch.cuda.is_available()
    pk.lib()
    return torch, pk, torch.device("cuda:0")


def run_fmm(env, seg, b, C, p, D, precision=0, a=1e-3):
    torch, pk, dev = env
    prm = pk.make_params(p, D, C[0], C[1], C[2], a, BOX_LO, BOX, precision=precision)
    plan = pk.Plan(prm)
    ts = torch.tensor(seg, device=dev)
    tb = torch.tensor(b, device=dev)
    tree = pk.Tree(plan, ts)
    f = pk.fmm_forces(plan, tree, ts, tb).cpu().numpy()
    return f, plan, tree


def run_direct(env, seg, b, C, fp32=False, targets=None, a=1e-3):
    torch, pk, dev = env
    prm = pk.make_params(4, 3, C[0], C[1], C[2], a, BOX_LO, BOX)
    plan = pk.Plan(prm)
    ts = torch.tensor(seg, device=dev)
    tb = torch.tensor(b, device=dev)
    tt = None if targets is None else torch.tensor(np.asarray(targets, dtype=np.int64), device=dev)
    return pk.direct_forces(plan, ts, tb, targets=tt, fp32=fp32).cpu().numpy()


# ------------------------------------------------------------- direct sum
@pytest.mark.parametrize("C,nloops", [(ISO, 50), (CUB, 8)])
def test_direct_matches_oracle(env, C, nloops):
    seg, b = synth.make_loops(nloops, 0.01, 0.05, 1)
    med = oracle.medium(*C, 1e-3)
    tgt = synth.segment_subset(len(seg), 150, 3)
    ref = oracle.direct_forces(seg, b, med, targets=tgt)
    f64 = run_direct(env, seg, b, C)
    assert oracle.rel_err(f64[tgt], ref) <= 1e-12
    f32 = run_direct(env, seg, b, C, fp32=True)
    assert oracle.rel_err(f32[tgt], ref) <= 1e-6
    # the target-list path gives the same rows as the all-targets path
    fs = run_direct(env, seg, b, C, targets=tgt)
    assert np.array_equal(fs, f64[tgt])


def test_direct_rejects_bad_targets(env):
    torch, pk, dev = env
    seg, b = synth.make_loops(2, 0.01, 0.05, 1)
    with pytest.raises(pk.DfmmError) as e:
        run_direct(env, seg, b, ISO, targets=[0, len(seg)])
    assert e.value.status == -1


# ------------------------------------------------------------------- FMM
@pytest.mark.parametrize("name,C,nloops,p,D", [
    ("iso2k", ISO, 50, 4, 3),
    ("iso-p5-D4", ISO, 30, 5, 4),
    ("iso-p2-D2", ISO, 12, 2, 2),
    ("iso-p3-D5", ISO, 20, 3, 5),
    ("cubic-p4-D3", CUB, 10, 4, 3),
    ("cubic-p6-D2", CUB, 6, 6, 2),
    # the order the 1M-segment benchmark runs (p = 7) and the largest order a
    # plan accepts (p = 8): every order-specialised kernel (DFTs, M2M, L2L,
    # L2P) at those orders against the oracle's dense M2L
    ("iso-p7-D3", ISO, 10, 7, 3),
    ("cubic-p7-D3", CUB, 6, 7, 3),
    ("iso-p8-D3", ISO, 8, 8, 3),
    ("cubic-p8-D3", CUB, 5, 8, 3),
])
def test_fmm_fp64_matches_oracle_fmm(env, name, C, nloops, p, D):
    seg, b = synth.make_loops(nloops, 0.01, 0.05, 1 if name == "iso2k" else 17)
    med = oracle.medium(*C, 1e-3)
    ref_fmm = oracle.fmm_forces(seg, b, med, p, D, BOX_LO, BOX)
    f, plan, tree = run_fmm(env, seg, b, C, p, D)
    assert oracle.rel_err(f, ref_fmm) <= 1e-10, name
    # mixed precision against the same approximation
    fm, _, _ = run_fmm(env, seg, b, C, p, D, precision=1)
    assert oracle.rel_err(fm, ref_fmm) <= 2e-5, name


def test_fmm_error_vs_direct_decreases_with_order(env):
    seg, b = synth.make_loops(50, 0.01, 0.05, 1)
    med = oracle.medium(*ISO, 1e-3)
    ref = oracle.direct_forces(seg, b, med)
    errs = [oracle.rel_err(run_fmm(env, seg, b, ISO, p, 3)[0], ref) for p in (3, 4, 5, 6, 7)]
    for e0, e1 in zip(errs, errs[1:]):
        assert e1 < e0 / 2
    assert errs[2] <= 1e-4 and errs[-1] <= 5e-6


def test_fmm_all_near_equals_direct(env):
    seg, b = synth.make_loops(5, 0.02, 0.05, 3)
    seg = 0.5 + 0.35 * (seg - seg.mean(axis=(0, 1)))
    f, _, tree = run_fmm(env, seg, b, ISO, 4, 2)
    assert tree.info()["m2l_pairs"] == 0
    ref = run_direct(env, seg, b, ISO)
    assert oracle.rel_err(f, ref) <= 1e-13


@pytest.mark.parametrize("C", [ISO, CUB])
def test_single_precision_path_with_close_pairs_only(env, C):
    """One loop of radius 2e-4: every pair of its 120 points is closer than
    2a = 2e-3, so the single-precision path's near field is entirely the
    double-precision close-pair kernel and must equal the FP64 direct sum."""
    seg, b = synth.make_loops(1, 2e-4, 2e-4, 11)
    seg = seg - seg.mean(axis=(0, 1)) + 0.5
    f, _, tree = run_fmm(env, seg, b, C, 4, 2, precision=1)
    assert tree.info()["m2l_pairs"] == 0
    ref = oracle.direct_forces(seg, b, oracle.medium(*C, 1e-3))
    assert oracle.rel_err(f, ref) <= 1e-11


def test_dense_cluster_of_close_pairs(env):
    """20 tiny loops packed into a 3e-3 cube (about a thousand close partners
    per point): the close-pair buffer fills and is evaluated many times per
    wave.  All pairs are near; single vs FP64 path vs the oracle."""
    rng = np.random.default_rng(12)
    segs, bs = [], []
    for k in range(20):
        s1, b1 = synth.make_loops(1, 1e-4, 4e-4, 100 + k)
        segs.append(s1 - s1.mean(axis=(0, 1)) + 0.5 + rng.uniform(-1.5e-3, 1.5e-3, size=3))
        bs.append(b1)
    seg, b = np.concatenate(segs), np.concatenate(bs)
    ref = oracle.direct_forces(seg, b, oracle.medium(*CUB, 1e-3))
    f64, _, tree = run_fmm(env, seg, b, CUB, 4, 4, precision=0)
    assert tree.info()["m2l_pairs"] == 0
    f32, _, _ = run_fmm(env, seg, b, CUB, 4, 4, precision=1)
    assert oracle.rel_err(f64, ref) <= 1e-12
    assert oracle.rel_err(f32, ref) <= 2e-5


def test_symmetric_near_field_small_and_large_leaves(env):
    """Cubic near field with one kernel evaluation per unordered pair, in
    single and in double precision: a shallow tree puts whole loops in one
    leaf (more than 64 points: the launch for large leaves) beside small
    leaves (64 or fewer), and both paths must match the oracle's FMM."""
    seg, b = synth.make_loops(12, 0.01, 0.04, 23)
    med = oracle.medium(*CUB, 1e-3)
    f32, _, tree = run_fmm(env, seg, b, CUB, 4, 3, precision=1)
    info = tree.info()
    assert 64 < info["max_leaf_points"] <= 1024
    ref = oracle.fmm_forces(seg, b, med, 4, 3, BOX_LO, BOX)
    assert oracle.rel_err(f32, ref) <= 2e-5
    f64, _, tree64 = run_fmm(env, seg, b, CUB, 4, 3, precision=0)
    assert tree.info()["symmetric_near"] == 1 and tree64.info()["symmetric_near"] == 1
    assert oracle.rel_err(f64, ref) <= 1e-10
    assert oracle.rel_err(f32, f64) <= 2e-5


@pytest.mark.parametrize("nloops,symmetric", [(7, 1), (9, 0)])
def test_near_field_leaves_around_the_symmetric_limit(env, nloops, symmetric):
    """One leaf of 840 points (seven loops shrunk into it) or 1080 points
    (nine) beside small leaves.  Up to 1024 points both precisions take the
    symmetric near field, its large-leaf launch included; beyond, the
    one-sided near field.  Both must match the oracle's FMM."""
    s1, b1 = synth.make_loops(nloops, 0.01, 0.04, 31)
    s1 = 0.635 + 0.2 * (s1 - s1.reshape(-1, 3).mean(axis=0))
    s2, b2 = synth.make_loops(6, 0.01, 0.04, 32)
    seg, b = np.concatenate([s1, s2]), np.concatenate([b1, b2])
    med = oracle.medium(*CUB, 1e-3)
    ref = oracle.fmm_forces(seg, b, med, 4, 2, BOX_LO, BOX)
    f64, _, tree = run_fmm(env, seg, b, CUB, 4, 2, precision=0)
    info = tree.info()
    assert (768 < info["max_leaf_points"] <= 1024) if symmetric else info["max_leaf_points"] > 1024
    assert info["symmetric_near"] == symmetric
    assert oracle.rel_err(f64, ref) <= 1e-10
    f32, _, tree32 = run_fmm(env, seg, b, CUB, 4, 2, precision=1)
    assert tree32.info()["symmetric_near"] == symmetric
    assert oracle.rel_err(f32, ref) <= 2e-5


# ------------------------------------------------------------ edge cases
def test_single_segment_and_degenerate_inputs(env):
    torch, pk, dev = env
    seg = np.array([[[0.3, 0.3, 0.3], [0.31, 0.305, 0.3]]])
    b = np.array([[1.0, 0.0, 0.0]]) / 1.0
    f, _, _ = run_fmm(env, seg, b, ISO, 4, 3)
    ref = oracle.direct_forces(seg, b, oracle.medium(*ISO, 1e-3))
    assert np.allclose(f, ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())
    # a zero-length segment contributes nothing and feels no force
    seg2, b2 = synth.make_loops(3, 0.01, 0.05, 5)
    seg2 = np.concatenate([seg2, [[[0.5, 0.5, 0.5], [0.5, 0.5, 0.5]]]])
    b2 = np.concatenate([b2, [[0.0, 0.0, 1.0]]])
    f2, _, _ = run_fmm(env, seg2, b2, ISO, 4, 3)
    f1, _, _ = run_fmm(env, seg2[:-1], b2[:-1], ISO, 4, 3)
    assert np.all(f2[-1] == 0.0)
    assert oracle.rel_err(f2[:-1], f1) <= 1e-13
    # points on the upper faces of the root cube
    hi = BOX_LO[0] + BOX
    seg3 = np.array([[[hi, hi, hi], [hi, hi - 0.01, hi]], [[BOX_LO[0], 0.2, 0.3], [BOX_LO[0], 0.21, 0.3]],
                     [[0.4, 0.4, 0.4], [0.42, 0.4, 0.4]]])
    b3 = np.array([[0, 0, 1.0], [0, 1.0, 0], [1.0, 0, 0]])
    f3, _, _ = run_fmm(env, seg3, b3, ISO, 4, 3)
    ref3 = oracle.fmm_forces(seg3, b3, oracle.medium(*ISO, 1e-3), 4, 3, BOX_LO, BOX)
    assert oracle.rel_err(f3, ref3) <= 1e-10


def test_errors_for_bad_coordinates(env):
    torch, pk, dev = env
    prm = pk.make_params(4, 3, *ISO, 1e-3, BOX_LO, BOX)
    plan = pk.Plan(prm)
    seg = np.array([[[0.3, 0.3, 0.3], [0.31, 0.305, 0.3]], [[1.2, 0.3, 0.3], [1.21, 0.3, 0.3]]])
    with pytest.raises(pk.DfmmError) as e:
        pk.Tree(plan, torch.tensor(seg, device=dev))
    assert e.value.status == -4
    seg[1] = [[0.3, np.nan, 0.3], [0.31, 0.3, 0.3]]
    with pytest.raises(pk.DfmmError) as e:
        pk.Tree(plan, torch.tensor(seg, device=dev))
    assert e.value.status == -5
    # a tree used with another plan
    plan2 = pk.Plan(prm)
    seg[1] = [[0.3, 0.3, 0.35], [0.31, 0.3, 0.35]]
    ts = torch.tensor(seg, device=dev)
    tree = pk.Tree(plan, ts)
    with pytest.raises(pk.DfmmError) as e:
        pk.fmm_forces(plan2, tree, ts, torch.zeros((2, 3), dtype=torch.float64, device=dev))
    assert e.value.status == -6
    # no segments at all: rejected before any work
    with pytest.raises(pk.DfmmError) as e:
        pk.Tree(plan, torch.zeros((0, 2, 3), dtype=torch.float64, device=dev))
    assert e.value.status == -1


@pytest.mark.parametrize("precision,leaf_max", [(0, 0), (2, 0), (1, 8)])
def test_tree_check_positions(env, precision, leaf_max):
    """dfmm_tree_check_positions accepts the segments a tree was built from
    and rejects, with the first segment named, endpoints moved by 1e-9 in one
    coordinate (uniform and adaptive trees, FP64 and single)."""
    torch, pk, dev = env
    seg, b = synth.loops.make_loops(12, 0.01, 0.05, seed=31)
    prm = pk.make_params(4, 4, *CUB, 1e-3, BOX_LO, BOX, precision=precision, leaf_max=leaf_max)
    plan = pk.Plan(prm)
    ts = torch.tensor(seg, device=dev)
    tree = pk.Tree(plan, ts)
    pk.tree_check_positions(plan, tree, ts)
    moved = seg.copy()
    moved[37, 0, 2] += 1e-9
    moved[200, 1, 0] -= 1e-9
    with pytest.raises(pk.DfmmError) as e:
        pk.tree_check_positions(plan, tree, torch.tensor(moved, device=dev))
    assert e.value.status == -6 and "first at segment 37" in str(e.value)
    pk.tree_check_positions(plan, tree, ts)  # the counters start again at zero
    pk.fmm_forces(plan, tree, ts, torch.tensor(b, device=dev))
    pk.tree_check_positions(plan, tree, ts)  # a force call leaves the build's copy alone
    with pytest.raises(pk.DfmmError) as e:
        pk.tree_check_positions(pk.Plan(prm), tree, ts)
    assert e.value.status == -6


def test_maximum_depth(env):
    """Depth 10, the deepest the 30-bit Morton keys allow (2^30 leaves in
    the key space), on a small input: against the oracle's FMM."""
    seg, b = synth.make_loops(4, 0.01, 0.03, 41)
    ref = oracle.fmm_forces(seg, b, oracle.medium(*ISO, 1e-3), 3, 10, BOX_LO, BOX)
    f, plan, tree = run_fmm(env, seg, b, ISO, 3, 10)
    assert tree.info()["depth"] == 10
    assert oracle.rel_err(f, ref) <= 1e-10


def test_determinism_and_stage_timing(env):
    torch, pk, dev = env
    seg, b = synth.make_loops(40, 0.01, 0.05, 8)
    for prec in (0, 1):
        f, plan, tree = run_fmm(env, seg, b, ISO, 5, 4, precision=prec)
        ts = torch.tensor(seg, device=dev)
        tb = torch.tensor(b, device=dev)
        tree.set_timing(True)
        g = pk.fmm_forces(plan, tree, ts, tb).cpu().numpy()
        ms, n = tree.stage_times()
        assert np.array_equal(f, g)
        assert n == 1 and all(x >= 0 for x in ms) and ms[3] > 0 and ms[6] > 0


# -------------------------------------------------- full-size workloads
def _golden(name):
    path = os.path.join(ROOT, "tests", "golden", "oracle_samples_%s.json" % name)
    if not os.path.exists(path):
        pytest.skip("golden file missing: " + path)
    return json.load(open(path))


# Orders that meet the 1e-4 bar on these ensembles.  At the orders the
# workloads are defined with (p = 5, 5, 6) the method's own interpolation
# error measured here is 1.7e-4, 1.2e-4 and 1.2e-4 (identical in FP64 and
# mixed precision and equal to the oracle FMM's), consistent with the
# ~3^-p decay of the Lagrange FMM; one more order brings it below 1e-4.
BAR_ORDER = {"iso200k": 6, "cubic100k": 6, "cubic1m": 7}


@pytest.mark.parametrize("name,precision", [("iso200k", 0), ("iso200k", 1), ("cubic100k", 0), ("cubic100k", 1),
                                            ("cubic1m", 0), ("cubic1m", 1)])
def test_full_size_fmm_vs_oracle_samples(env, name, precision):
    """The launch configuration the benchmark times, at the full size, against
    the oracle's direct sum on sampled segments (values written by
    tests/golden/make_golden.py from the oracle only)."""
    torch, pk, dev = env
    g = _golden(name)
    seg, b, prm = synth.make_workload(name)
    assert seg.shape[0] == g["n_seg"]
    C = (prm["c11"], prm["c12"], prm["c44"])
    tgt = np.asarray(g["targets"])
    ref = np.asarray(g["forces"])
    f, plan, tree = run_fmm(env, seg, b, C, BAR_ORDER[name], prm["depth"], precision=precision)
    err = oracle.rel_err(f[tgt], ref)
    print("%s p=%d precision=%d: rel err vs oracle on %d segments = %.3e"
          % (name, BAR_ORDER[name], precision, len(tgt), err))
    assert err <= 1e-4
    del tree, plan
    # the workload's own order: error of the method, 3^-p-like, above the bar
    f, plan, tree = run_fmm(env, seg, b, C, prm["order"], prm["depth"], precision=precision)
    err_p = oracle.rel_err(f[tgt], ref)
    print("%s p=%d precision=%d: rel err = %.3e" % (name, prm["order"], precision, err_p))
    assert err < err_p <= 3e-4


# ----------------------------------------- symmetry-reduced operator store
@pytest.mark.parametrize("name,C,nloops,p,D", [
    ("iso-p4-D3", ISO, 20, 4, 3),
    ("cubic-p5-D3", CUB, 10, 5, 3),
    ("cubic-p7-D3", CUB, 6, 7, 3),
    ("iso-p3-D5", ISO, 20, 3, 5),
])
def test_symmetry_reduced_operators_match_oracle_fmm(env, name, C, nloops, p, D):
    """DFMM_M2L_FFT_SYM stores the spectra of the 16 class representatives
    only and expands them in the Hadamard product (class, signed permutation
    and det of each offset); the result is the same approximation as the
    158-offset store and the oracle's dense M2L."""
    torch, pk, dev = env
    seg, b = synth.make_loops(nloops, 0.01, 0.05, 17)
    ref_fmm = oracle.fmm_forces(seg, b, oracle.medium(*C, 1e-3), p, D, BOX_LO, BOX)
    ts, tb = torch.tensor(seg, device=dev), torch.tensor(b, device=dev)
    out = {}
    for mode in (0, 1):
        for prec in (0, 1):
            prm = pk.make_params(p, D, *C, 1e-3, BOX_LO, BOX, precision=prec, m2l_mode=mode)
            plan = pk.Plan(prm)
            tree = pk.Tree(plan, ts)
            out[mode, prec] = pk.fmm_forces(plan, tree, ts, tb).cpu().numpy()
            info = plan.info()
            assert info["m2l_mode"] == mode and info["stored_offsets"] == (16 if mode else 158)
    assert oracle.rel_err(out[1, 0], ref_fmm) <= 1e-10, name
    assert oracle.rel_err(out[1, 1], ref_fmm) <= 2e-5, name
    # the same operators up to rounding: FP64 stores agree far below the bar
    assert oracle.rel_err(out[1, 0], out[0, 0]) <= 1e-13, name
    assert oracle.rel_err(out[1, 1], out[0, 1]) <= 2e-6, name


def test_operator_memory_against_the_paper(env):
    """Eq. mem_unif at p = 7 (the paper prints about 300 MB per level) and the
    16-operator store's reduction by 316/16 (about 20x, Sec. 6), from the
    plan's own accounting of the FP64 generators behind its spectra."""
    torch, pk, dev = env
    pn = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_numbers.json")))
    D = 3
    infos = {}
    for mode in (0, 1):
        plan = pk.Plan(pk.make_params(7, D, *CUB, 1e-3, BOX_LO, BOX, precision=0, m2l_mode=mode))
        infos[mode] = plan.info()
    mem = infos[0]["mem_unif_fp64_bytes_per_level"] / 1e6
    assert abs(mem - pn["mem_unif_p7_MB"]["value"]) <= pn["mem_unif_p7_MB"]["rel_tol"] * pn["mem_unif_p7_MB"]["value"]
    # the plan keeps one of each pair (o, -o): half of the 316 generators
    assert infos[0]["generator_fp64_bytes_per_level"] * 2 == infos[0]["mem_unif_fp64_bytes_per_level"]
    assert infos[1]["stored_offsets"] == pn["m2l_operators_with_symmetry"]["value"]
    factor = infos[0]["mem_unif_fp64_bytes_per_level"] / infos[1]["generator_fp64_bytes_per_level"]
    f = pn["symmetry_memory_factor"]
    assert abs(factor - f["value"]) <= f["rel_tol"] * f["value"], factor
    # the spectra actually held (half spectrum, complex): 158 -> 16 offsets (the
    # 158-offset FP64 store keeps each offset in the product's slot order, 55
    # entries with one pad; the class store 54)
    assert infos[0]["spectra_bytes"] * 16 * 54 == infos[1]["spectra_bytes"] * 158 * 55
    print("operator memory per level at p=7: Eq. mem_unif %.1f MB, 16-class generators %.1f MB (x%.2f); "
          "spectra held %.1f MB -> %.1f MB for %d levels"
          % (mem, infos[1]["generator_fp64_bytes_per_level"] / 1e6, factor, infos[0]["spectra_bytes"] / 1e6,
             infos[1]["spectra_bytes"] / 1e6, D - 1))


def test_dense_tree_lists_have_the_paper_counts(env):
    """All 8^l cells occupied (a point in every leaf): every cell's
    interaction list is counted by brute force in the test, and interior
    cells have the paper's 189 far cells and 27 neighbours (App. B)."""
    torch, pk, dev = env
    pn = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_numbers.json")))
    D = 4
    n = 2 ** D
    h = BOX / n
    c = (np.arange(n) + 0.5) * h + BOX_LO[0]
    P = np.stack(np.meshgrid(c, c, c, indexing="ij"), -1).reshape(-1, 3)
    seg = np.stack([P - 0.1 * h, P + 0.1 * h], axis=1)  # 3 points per leaf
    prm = pk.make_params(3, D, *ISO, 1e-3, BOX_LO, BOX)
    plan = pk.Plan(prm)
    tree = pk.Tree(plan, torch.tensor(seg, device=dev))
    info = tree.info()
    for lv in info["levels"]:
        l = lv["level"]
        m = 2 ** l
        idx = np.arange(m)
        # per axis, the number of cells j with |i - j| >= 2 and |i/2 - j/2| <= 1
        cnt = np.array([[1 if abs(i - j) >= 2 and abs(i // 2 - j // 2) <= 1 else 0 for j in idx] for i in idx])
        near = np.array([[1 if abs(i - j) <= 1 else 0 for j in idx] for i in idx])
        cand = np.array([[1 if abs(i // 2 - j // 2) <= 1 else 0 for j in idx] for i in idx])
        # far = (parent neighbours' children) minus (own neighbours), in 3D
        c1, nr = cand.sum(1), near.sum(1)
        far = (np.einsum("i,j,k->ijk", c1, c1, c1) - np.einsum("i,j,k->ijk", nr, nr, nr))
        assert lv["cells"] == m ** 3
        assert lv["m2l_pairs"] == int(far.sum()), l
        if m >= 8:  # interior cells
            assert far[3, 3, 3] == pn["far_cells"]["value"]
            assert nr[3] ** 3 == pn["near_cells"]["value"]
    assert info["near_pairs"] == sum(
        int(np.prod([min(i + 1, n - 1) - max(i - 1, 0) + 1 for i in cc])) * 3 * 3
        for cc in np.ndindex(n, n, n))


# ------------------------------------------------- f16 operands in the M2L
F16_U = 2.0 ** -11  # unit roundoff of IEEE half precision


@pytest.mark.parametrize("name,C,nloops,p,D,mode", [
    ("iso-p4-D3", ISO, 50, 4, 3, 0),
    ("cubic-p5-D3", CUB, 10, 5, 3, 1),
    ("cubic-p7-D3", CUB, 6, 7, 3, 1),
    ("iso-p6-D4", ISO, 30, 6, 4, 0),
])
def test_fmm_f16_m2l_matches_oracle_fmm(env, name, C, nloops, p, D, mode):
    """DFMM_MIXED_F16: the Hadamard product takes f16 operator and source
    spectra (f32 accumulation).  Each f16 operand carries a relative
    rounding error of at most 2^-11, so every product term at most 2^-10:
    the far field is off by at most about 2^-10 of itself, and the forces by
    that times the far field's share, which the oracle's FMM reports.  The
    bar adds that to the f32 path's 2e-5."""
    torch, pk, dev = env
    seg, b = synth.make_loops(nloops, 0.01, 0.05, 1 if name == "iso-p4-D3" else 17)
    med = oracle.medium(*C, 1e-3)
    ref, ref_far, _ = oracle.fmm_forces(seg, b, med, p, D, BOX_LO, BOX, return_parts=True)
    share = float(np.linalg.norm(ref_far) / np.linalg.norm(ref))
    ts, tb = torch.tensor(seg, device=dev), torch.tensor(b, device=dev)
    prm = pk.make_params(p, D, *C, 1e-3, BOX_LO, BOX, precision=2, m2l_mode=mode)
    plan = pk.Plan(prm)
    tree = pk.Tree(plan, ts)
    f16 = pk.fmm_forces(plan, tree, ts, tb).cpu().numpy()
    err = oracle.rel_err(f16, ref)
    bar = 2e-5 + 2 * F16_U * share
    print("%s: f16 M2L vs oracle FMM %.2e (far-field share %.3f, bar %.2e)" % (name, err, share, bar))
    assert err <= bar, name
    # repeated calls are bit-identical (the scales are recomputed each call)
    assert np.array_equal(f16, pk.fmm_forces(plan, tree, ts, tb).cpu().numpy())


@pytest.mark.parametrize("name,C,nloops,seed", [("iso", ISO, 10, 17), ("cubic", CUB, 6, 19)])
def test_single_precision_dfts_on_levels_of_both_parities(env, name, C, nloops, seed):
    """In single precision the forward and inverse DFTs take two consecutive
    cells per block, so on a level with an odd number of cells the last block
    holds one.  These trees (p = 7, depth 3) have levels of both parities
    (checked), and the f32 and f16 paths match the oracle's FMM on them at the
    bars of the tests above."""
    seg, b = synth.make_loops(nloops, 0.01, 0.05, seed)
    med = oracle.medium(*C, 1e-3)
    ref, ref_far, _ = oracle.fmm_forces(seg, b, med, 7, 3, BOX_LO, BOX, return_parts=True)
    share = float(np.linalg.norm(ref_far) / np.linalg.norm(ref))
    f32, _, tree = run_fmm(env, seg, b, C, 7, 3, precision=1)
    cells = [lv["cells"] for lv in tree.info()["levels"]]
    assert {n % 2 for n in cells} == {0, 1}, cells
    assert oracle.rel_err(f32, ref) <= 2e-5, name
    f16, _, _ = run_fmm(env, seg, b, C, 7, 3, precision=2)
    assert oracle.rel_err(f16, ref) <= 2e-5 + 2 * F16_U * share, name


def test_full_size_f16_m2l_vs_oracle_samples(env):
    """The 1M-segment cubic workload with f16 operands in the M2L at p = 7:
    the force error against the oracle's direct sum on the 64 golden
    segments stays within the 1e-4 bar."""
    torch, pk, dev = env
    g = _golden("cubic1m")
    seg, b, prm = synth.make_workload("cubic1m")
    C = (prm["c11"], prm["c12"], prm["c44"])
    tgt = np.asarray(g["targets"])
    ref = np.asarray(g["forces"])
    f, plan, tree = run_fmm(env, seg, b, C, 7, prm["depth"], precision=2)
    err = oracle.rel_err(f[tgt], ref)
    print("cubic1m p=7 f16 M2L: rel err vs oracle on %d segments = %.3e" % (len(tgt), err))
    assert err <= 1e-4


# ------------------------------------------- stabilised interpolation (LS)
def lsq_auto(p):
    """The degree DFMM_LSQ_AUTO picks: the largest d < 2 sqrt(p), the bound
    Sec. 4.3 gives for a stable least-squares fit on p equispaced nodes, at
    most p - 1 (which is the interpolant itself: the plan reports 0)."""
    d = 0
    while (d + 1) ** 2 < 4 * p:
        d += 1
    d = min(d, p - 1)
    return 0 if d == p - 1 else d


@pytest.mark.parametrize("name,C,nloops,p,D,d,mode", [
    ("iso-p4-D3-d2", ISO, 40, 4, 3, 2, 0),
    ("cubic-p6-D3-auto", CUB, 10, 6, 3, -1, 1),
    ("iso-p7-D3-d4", ISO, 6, 7, 3, 4, 1),
    ("cubic-p6-D4-d3", CUB, 8, 6, 4, 3, 0),
])
def test_lsq_fmm_matches_oracle_lsq_fmm(env, name, C, nloops, p, D, d, mode):
    """Least-squares interpolation of degree d on the p equispaced nodes
    (Sec. 4.3): the GPU FMM against the oracle's FMM with the same
    projector, in FP64 (<= 1e-10), single precision (<= 2e-5) and with f16
    M2L operands (the f16 bar of the Lagrange path)."""
    torch, pk, dev = env
    seg, b = synth.make_loops(nloops, 0.01, 0.05, 23)
    med = oracle.medium(*C, 1e-3)
    deg = lsq_auto(p) if d < 0 else d
    assert deg > 0
    ref, ref_far, _ = oracle.fmm_forces(seg, b, med, p, D, BOX_LO, BOX, return_parts=True, lsq_degree=deg)
    share = float(np.linalg.norm(ref_far) / np.linalg.norm(ref))
    ts, tb = torch.tensor(seg, device=dev), torch.tensor(b, device=dev)
    bars = {0: 1e-10, 1: 2e-5, 2: 2e-5 + 2 * F16_U * share}
    for prec, bar in bars.items():
        plan = pk.Plan(pk.make_params(p, D, *C, 1e-3, BOX_LO, BOX, precision=prec, m2l_mode=mode, lsq_degree=d))
        assert plan.info()["lsq_degree"] == deg
        tree = pk.Tree(plan, ts)
        f = pk.fmm_forces(plan, tree, ts, tb).cpu().numpy()
        err = oracle.rel_err(f, ref)
        print("%s precision %d: LS FMM vs oracle LS FMM %.2e (bar %.2e)" % (name, prec, err, bar))
        assert err <= bar, (name, prec)


def test_lsq_of_full_degree_is_the_lagrange_path(env):
    """d = p - 1 is interpolation: the plan runs the Lagrange path and the
    forces are bit-identical to it."""
    torch, pk, dev = env
    seg, b = synth.make_loops(20, 0.01, 0.05, 5)
    ts, tb = torch.tensor(seg, device=dev), torch.tensor(b, device=dev)
    out = []
    for d in (0, 4):
        plan = pk.Plan(pk.make_params(5, 3, *CUB, 1e-3, BOX_LO, BOX, precision=1, lsq_degree=d))
        assert plan.info()["lsq_degree"] == 0
        tree = pk.Tree(plan, ts)
        out.append(pk.fmm_forces(plan, tree, ts, tb).cpu().numpy())
    assert np.array_equal(out[0], out[1])


def test_lsq_error_vs_direct(env):
    """Accuracy of the stabilised FMM against the FP64 direct sum, next to
    the Lagrange FMM of the same order: printed for each order, and the
    least-squares error still falls with the order (orders below 6 have
    no degree d < 2 sqrt(p) under p - 1 and run the Lagrange path)."""
    seg, b = synth.make_loops(50, 0.01, 0.05, 1)
    ref = oracle.direct_forces(seg, b, oracle.medium(*ISO, 1e-3))
    torch, pk, dev = env
    ts, tb = torch.tensor(seg, device=dev), torch.tensor(b, device=dev)
    errs = []
    for p in (4, 5, 6, 7, 8):
        row = []
        for d in (0, -1):
            plan = pk.Plan(pk.make_params(p, 3, *ISO, 1e-3, BOX_LO, BOX, precision=0, lsq_degree=d))
            tree = pk.Tree(plan, ts)
            row.append(oracle.rel_err(pk.fmm_forces(plan, tree, ts, tb).cpu().numpy(), ref))
        print("p=%d: Lagrange %.3e, least squares (d=%d) %.3e" % (p, row[0], lsq_auto(p), row[1]))
        errs.append(row[1])
    assert errs[-1] < errs[0] / 4


# ------------------------------------------------ spectra in frequency chunks
@pytest.mark.parametrize("chunks,expect", [(2, 2), (3, 3), (4, 3), (9, 9)])
def test_frequency_chunks_match_the_whole_spectrum(env, chunks, expect):
    """The M2L spectra taken in chunks of first frequency indices (the
    forward transform per chunk, the inverse transforms summed) give the
    whole-spectrum result: FP64 to 1e-13 and against the oracle's FMM to
    1e-10, single precision and f16 operands to 1e-6 (only the summation
    order of the inverse transform changes)."""
    torch, pk, dev = env
    seg, b = synth.make_loops(25, 0.01, 0.05, 31)
    ts, tb = torch.tensor(seg, device=dev), torch.tensor(b, device=dev)
    ref_o = oracle.fmm_forces(seg, b, oracle.medium(*CUB, 1e-3), 5, 4, BOX_LO, BOX)
    for prec, bar in ((0, 1e-13), (1, 1e-6), (2, 1e-6)):
        out = {}
        for c in (1, chunks):
            plan = pk.Plan(pk.make_params(5, 4, *CUB, 1e-3, BOX_LO, BOX, precision=prec, m2l_mode=1, freq_chunks=c))
            tree = pk.Tree(plan, ts)
            assert tree.info()["freq_chunks"] == (1 if c == 1 else expect)
            out[c] = pk.fmm_forces(plan, tree, ts, tb).cpu().numpy()
        assert oracle.rel_err(out[chunks], out[1]) <= bar, prec
        if prec == 0:
            assert oracle.rel_err(out[chunks], ref_o) <= 1e-10
