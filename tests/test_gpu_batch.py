"""GPU tests of the batched graph launch and of the depth autotuner."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

BOX_LO, BOX = synth.loops.BOX_LO, synth.loops.BOX_SIZE
ISO = synth.loops.ISO


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_1712_07739_amd as pk

    assert torch.cuda.is_available()
    return torch, pk, torch.device("cuda:0")


def test_batched_graph_equals_individual_calls_on_every_replay(env):
    torch, pk, dev = env
    sizes = [10, 3, 25, 7, 1, 14]  # loops per configuration (ragged sizes)
    depths = [3, 2, 4, 3, 2, 4]
    plans = {d: pk.Plan(pk.make_params(4, d, *ISO, 1e-3, BOX_LO, BOX, precision=1)) for d in set(depths)}
    cfg = []
    for i, (nl, d) in enumerate(zip(sizes, depths)):
        seg, b = synth.make_loops(nl, 0.01, 0.05, 900 + i)
        ts, tb = torch.tensor(seg, device=dev), torch.tensor(b, device=dev)
        tree = pk.Tree(plans[d], ts)
        ref = pk.fmm_forces(plans[d], tree, ts, tb).cpu().numpy()
        out = torch.zeros((len(seg), 2, 3), dtype=torch.float64, device=dev)
        cfg.append((plans[d], tree, ts, tb, out, ref, seg, b))
    batch = pk.Batch([c[0] for c in cfg], [c[1] for c in cfg], [c[2] for c in cfg], [c[3] for c in cfg],
                     [c[4] for c in cfg], lanes=3)
    for rep in range(3):
        for c in cfg:
            c[4].zero_()  # eager work between replays
        torch.cuda.synchronize()
        batch.run()
        lat = batch.latencies_ms()
        for c in cfg:
            assert np.array_equal(c[4].cpu().numpy(), c[5]), rep
        assert all(x > 0 for x in lat)
    # and the batch agrees with the oracle's FMM
    p, tree, ts, tb, out, ref, seg, b = cfg[2]
    ref_o = oracle.fmm_forces(seg, b, oracle.medium(*ISO, 1e-3), 4, 4, BOX_LO, BOX)
    assert oracle.rel_err(out.cpu().numpy(), ref_o) <= 2e-5
    # The batch's streams go with it; the trees it captured stay usable and
    # are destroyed afterwards without touching those streams.
    batch.close()
    again = pk.fmm_forces(p, tree, ts, tb).cpu().numpy()
    assert np.array_equal(again, ref)
    for c in cfg:
        c[1].info()
        c[1].close()


def _measured_ms(pk, torch, prm_args, d, ts, tb, reps=3):
    import time

    plan = pk.Plan(pk.make_params(*prm_args[:1], d, *prm_args[1:], precision=1))
    tree = pk.Tree(plan, ts)
    out = torch.empty((ts.shape[0], 2, 3), dtype=torch.float64, device=ts.device)
    pk.fmm_forces(plan, tree, ts, tb, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        pk.fmm_forces(plan, tree, ts, tb, out=out)
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / reps


def test_depth_autotuner(env):
    """App. B model: the prediction's minimum is the model's pick; the returned
    depth (the fastest of the timed candidates) is within 25% of the fastest
    depth measured independently over the whole range."""
    torch, pk, dev = env
    for nl in (40, 800):
        seg, b = synth.make_loops(nl, 0.01, 0.05, 77)
        ts, tb = torch.tensor(seg, device=dev), torch.tensor(b, device=dev)
        prm = pk.make_params(5, 4, *ISO, 1e-3, BOX_LO, BOX, precision=1)
        d, pred, meas = pk.autotune_depth(prm, ts, tb, 2, 6)
        print("segments %d: depth %d, predicted ms %s, measured ms %s" % (
            nl * 40, d, {k: round(v, 3) for k, v in pred.items()}, {k: round(v, 3) for k, v in meas.items()}))
        assert 2 <= d <= 6 and all(v > 0 for v in pred.values())
        pick = min(pred, key=pred.get)
        assert set(meas) <= {pick - 1, pick, pick + 1} and pick in meas and d in meas
        assert meas[d] == min(meas.values())
        truth = {k: _measured_ms(pk, torch, (5, *ISO, 1e-3, BOX_LO, BOX), k, ts, tb) for k in range(2, 7)}
        print("  independent timing:", {k: round(v, 3) for k, v in truth.items()})
        assert truth[d] <= 1.25 * min(truth.values()) + 0.05


def test_forces_batched_one_shot_equals_individual_calls(env):
    """dfmm_forces_batched (create, run, destroy in one call) writes the same
    forces as individual dfmm_fmm_forces calls."""
    torch, pk, dev = env
    plan = pk.Plan(pk.make_params(4, 3, *ISO, 1e-3, BOX_LO, BOX, precision=1))
    cfg = []
    for i, nl in enumerate([4, 9, 2]):
        seg, b = synth.make_loops(nl, 0.01, 0.05, 950 + i)
        ts, tb = torch.tensor(seg, device=dev), torch.tensor(b, device=dev)
        tree = pk.Tree(plan, ts)
        ref = pk.fmm_forces(plan, tree, ts, tb).cpu().numpy()
        cfg.append((tree, ts, tb, torch.zeros((len(seg), 2, 3), dtype=torch.float64, device=dev), ref))
    pk.forces_batched([plan] * 3, [c[0] for c in cfg], [c[1] for c in cfg], [c[2] for c in cfg],
                      [c[3] for c in cfg])
    for c in cfg:
        assert np.array_equal(c[3].cpu().numpy(), c[4])


def test_batch_branch_autotuner(env):
    """The launch-shape autotuner times the batch graph at 1, 2, 4 and 8
    branches, returns the fastest measured count, and every replay writes the
    individual calls' forces."""
    torch, pk, dev = env
    plan = pk.Plan(pk.make_params(4, 3, *ISO, 1e-3, BOX_LO, BOX, precision=1))
    cfg = []
    for i, nl in enumerate([6, 2, 11, 4, 8]):
        seg, b = synth.make_loops(nl, 0.01, 0.05, 970 + i)
        ts, tb = torch.tensor(seg, device=dev), torch.tensor(b, device=dev)
        tree = pk.Tree(plan, ts)
        ref = pk.fmm_forces(plan, tree, ts, tb).cpu().numpy()
        cfg.append((tree, ts, tb, torch.zeros((len(seg), 2, 3), dtype=torch.float64, device=dev), ref))
    best, ms = pk.autotune_batch_lanes([plan] * 5, [c[0] for c in cfg], [c[1] for c in cfg], [c[2] for c in cfg],
                                       [c[3] for c in cfg], reps=2)
    print("batch branches -> ms per replay:", ms, "best", best)
    assert sorted(ms) == [1, 2, 4] and best in ms and ms[best] == min(ms.values())
    for c in cfg:
        assert np.array_equal(c[3].cpu().numpy(), c[4])
