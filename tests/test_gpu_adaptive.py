"""GPU parity of the adaptive tree (Sec. 3's partition until every leaf holds
few points): lists bit-exact against the oracle's tree, forces against the
oracle's adaptive FMM, and the 1M-segment workload against the oracle's
direct sum on the golden samples."""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from oracle.fmm_adaptive import AdaptiveTree, fmm_forces_adaptive
from test_oracle_adaptive import clustered

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BOX_LO, BOX = synth.loops.BOX_LO, synth.loops.BOX_SIZE
ISO = synth.loops.ISO
CUB = synth.loops.CUBIC_A25
F16_U = 2.0 ** -11


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_1712_07739_amd as pk

    assert torch.cuda.is_available()
    pk.lib()
    return torch, pk, torch.device("cuda:0")


def run(env, seg, b, C, p, D, leaf_max, precision=0, m2l_mode=0):
    torch, pk, dev = env
    plan = pk.Plan(pk.make_params(p, D, *C, 1e-3, BOX_LO, BOX, precision=precision, m2l_mode=m2l_mode,
                                  leaf_max=leaf_max))
    ts, tb = torch.tensor(seg, device=dev), torch.tensor(b, device=dev)
    tree = pk.Tree(plan, ts)
    f = pk.fmm_forces(plan, tree, ts, tb).cpu().numpy()
    return f, tree.info(), (plan, tree, ts, tb)


@pytest.mark.parametrize("D,leaf_max", [(4, 40), (5, 20), (4, 8)])
def test_lists_equal_the_oracle_tree(env, D, leaf_max):
    """Cells, leaves and the U, V (M2L), W and X pair counts of the GPU's
    adaptive tree equal those of the oracle's tree built by the definitions."""
    seg, b = clustered()
    y, _ = oracle.points(seg, b)
    T = AdaptiveTree(y, D, BOX_LO, BOX, leaf_max)
    st = T.stats()
    _, info, _ = run(env, seg, b, ISO, 3, D, leaf_max)
    print("oracle", st, "gpu", {k: info[k] for k in ("leaves", "u_pairs", "w_pairs", "x_pairs", "m2l_pairs")})
    assert info["adaptive"] == 1
    assert info["leaves"] == st["leaves"]
    assert sum(lv["cells"] for lv in info["levels"]) == sum(1 for c in range(T.n) if T.level[c] >= 2)
    assert info["u_pairs"] == st["u_pairs"] and info["m2l_pairs"] == st["v_pairs"]
    assert info["w_pairs"] == st["w_pairs"] and info["x_pairs"] == st["x_pairs"]
    levels = sorted(lv["level"] for lv in info["levels"] if lv["leaves"] > 0)
    assert levels == st["leaf_levels"]


@pytest.mark.parametrize("name,C,p,D,leaf_max,mode", [
    ("iso-p4-D4", ISO, 4, 4, 40, 0),
    ("cubic-p4-D4", CUB, 4, 4, 40, 1),
    ("cubic-p5-D5", CUB, 5, 5, 20, 0),
])
def test_forces_match_oracle_adaptive_fmm(env, name, C, p, D, leaf_max, mode):
    """FP64 <= 1e-10, single precision <= 2e-5 and f16 M2L operands within
    the f16 bar, each against the oracle's adaptive FMM on the same tree
    (with the same rule for direct W/X pairs)."""
    seg, b = clustered()
    med = oracle.medium(*C, 1e-3)
    # the GPU sums a W or X pair directly when its finer cell holds at most p^3 points
    ref, ref_far, _ = fmm_forces_adaptive(seg, b, med, p, D, BOX_LO, BOX, leaf_max, return_parts=True,
                                          direct_max=p ** 3)
    share = float(np.linalg.norm(ref_far) / np.linalg.norm(ref))
    bars = {0: 1e-10, 1: 2e-5, 2: 2e-5 + 2 * F16_U * share}
    for prec, bar in bars.items():
        f, info, _ = run(env, seg, b, C, p, D, leaf_max, precision=prec, m2l_mode=mode)
        err = oracle.rel_err(f, ref)
        print("%s precision %d: adaptive GPU vs oracle adaptive FMM %.2e (bar %.2e, w pairs %d)"
              % (name, prec, err, bar, info["w_pairs"]))
        assert err <= bar, (name, prec)


def test_one_level_of_leaves_is_the_uniform_tree(env):
    """leaf_max larger than every cell: all level-2 cells are leaves, the
    tree is the uniform depth-2 tree, and the forces equal the uniform path's."""
    seg, b = clustered()
    f_a, info, _ = run(env, seg, b, CUB, 4, 5, 10 ** 9)
    assert info["depth"] == 2 and info["w_pairs"] == 0
    torch, pk, dev = env
    plan = pk.Plan(pk.make_params(4, 2, *CUB, 1e-3, BOX_LO, BOX, precision=0))
    ts, tb = torch.tensor(seg, device=dev), torch.tensor(b, device=dev)
    tree = pk.Tree(plan, ts)
    f_u = pk.fmm_forces(plan, tree, ts, tb).cpu().numpy()
    assert oracle.rel_err(f_a, f_u) <= 1e-12


def test_single_segment_and_repeated_calls(env):
    seg = np.array([[[0.40, 0.40, 0.40], [0.41, 0.405, 0.40]]])
    b = np.array([[1.0, 1.0, 1.0]]) / np.sqrt(3)
    f, info, (plan, tree, ts, tb) = run(env, seg, b, CUB, 4, 6, 2, precision=0)
    ref = oracle.direct_forces(seg, b, oracle.medium(*CUB, 1e-3))
    # three points, all in adjacent leaves: the direct sum
    assert info["m2l_pairs"] == 0 and info["w_pairs"] == 0
    assert oracle.rel_err(f, ref) <= 1e-12
    torch, pk, dev = env
    assert np.array_equal(f, pk.fmm_forces(plan, tree, ts, tb).cpu().numpy())


def _golden(name):
    with open(os.path.join(ROOT, "tests", "golden", "oracle_samples_%s.json" % name)) as fh:
        return json.load(fh)


def test_full_size_adaptive_vs_oracle_samples(env):
    """The 1M-segment cubic workload on an adaptive tree (depth up to 8,
    leaves of at most 64 points, p = 7, f16 M2L operands): the force error
    against the oracle's direct sum on the golden segments stays within 1e-4."""
    torch, pk, dev = env
    g = _golden("cubic1m")
    seg, b, prm = synth.make_workload("cubic1m")
    C = (prm["c11"], prm["c12"], prm["c44"])
    tgt = np.asarray(g["targets"])
    f, info, _ = run(env, seg, b, C, 7, 8, 64, precision=2, m2l_mode=1)
    err = oracle.rel_err(f[tgt], np.asarray(g["forces"]))
    print("cubic1m adaptive: %d leaves on levels %s, u/w/x pairs %d/%d/%d, error %.3e"
          % (info["leaves"], [lv["level"] for lv in info["levels"] if lv["leaves"] > 0], info["u_pairs"],
             info["w_pairs"], info["x_pairs"], err))
    assert err <= 1e-4


def test_deep_cells_below_the_core_size(env):
    """Leaves down to level 10, whose cells (1.1e-3) are narrower than 2a:
    W/X pairs summed directly then contain near-coincident pairs, which the
    single-precision path must hand to its FP64 close-pair pass like the U
    pairs'.  Against the oracle's adaptive FMM (FP64 throughout)."""
    seg, b = clustered()
    med = oracle.medium(*CUB, 1e-3)
    # leaves of at most 3 points: levels 4..10, with 8 near-coincident point
    # pairs among the W pairs summed directly
    ref = fmm_forces_adaptive(seg, b, med, 3, 10, BOX_LO, BOX, 3, direct_max=27)
    for prec, bar in ((0, 1e-10), (1, 2e-5)):
        f, info, _ = run(env, seg, b, CUB, 3, 10, 3, precision=prec)
        assert info["depth"] == 10 and info["w_pairs"] > 0
        err = oracle.rel_err(f, ref)
        print("deep adaptive tree, precision %d: %.2e vs oracle" % (prec, err))
        assert err <= bar, prec


def test_uniform_tree_lists_equal_a_brute_force_tree(env):
    """The uniform tree's lists, an integer result, against the oracle's tree
    built by definition with every cell split down to the depth (leaf_max 0):
    M2L pairs per level and near-field point pairs, exactly."""
    seg, b = synth.make_loops(30, 0.01, 0.05, 61)
    y, _ = oracle.points(seg, b)
    D = 4
    T = AdaptiveTree(y, D, BOX_LO, BOX, 0)
    v_per_level = {l: sum(len(T.V[c]) for c in T.by_level[l]) for l in range(2, D + 1)}
    near = sum(len(T.pts[c]) * sum(len(T.pts[a]) for a in T.U[c]) for c in range(T.n) if T.leaf[c])
    _, info, _ = run(env, seg, b, ISO, 3, D, 0)
    assert info["adaptive"] == 0
    assert {lv["level"]: lv["m2l_pairs"] for lv in info["levels"]} == v_per_level
    assert {lv["level"]: lv["cells"] for lv in info["levels"]} == {l: len(T.by_level[l]) for l in range(2, D + 1)}
    assert info["near_pairs"] == near


def test_adaptive_tree_with_spectrum_chunks(env):
    """The adaptive tree's M2L in frequency chunks equals its whole-spectrum
    result (FP64 1e-13, f16 operands 1e-6)."""
    torch, pk, dev = env
    seg, b = clustered()
    ts, tb = torch.tensor(seg, device=dev), torch.tensor(b, device=dev)
    for prec, bar in ((0, 1e-13), (2, 1e-6)):
        out = []
        for c in (1, 4):
            plan = pk.Plan(pk.make_params(4, 5, *CUB, 1e-3, BOX_LO, BOX, precision=prec, m2l_mode=1, leaf_max=20,
                                          freq_chunks=c))
            tree = pk.Tree(plan, ts)
            assert tree.info()["freq_chunks"] == (1 if c == 1 else 4) and tree.info()["adaptive"] == 1
            out.append(pk.fmm_forces(plan, tree, ts, tb).cpu().numpy())
        assert oracle.rel_err(out[1], out[0]) <= bar, prec
