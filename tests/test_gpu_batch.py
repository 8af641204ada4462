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
    batch.close()


def test_depth_autotuner(env):
    torch, pk, dev = env
    best = {}
    for nl in (40, 800):
        seg, b = synth.make_loops(nl, 0.01, 0.05, 77)
        prm = pk.make_params(5, 4, *ISO, 1e-3, BOX_LO, BOX, precision=1)
        d, pred = pk.autotune_depth(prm, torch.tensor(seg, device=dev), torch.tensor(b, device=dev), 2, 6)
        print("segments %d: depth %d, predicted ms %s" % (nl * 40, d, {k: round(v, 3) for k, v in pred.items()}))
        assert 2 <= d <= 6 and all(v > 0 for v in pred.values())
        assert pred[d] == min(pred.values())
        best[nl] = d
    assert best[800] >= best[40]  # more segments, finer leaves (App. B: N_c grows with N_s)
