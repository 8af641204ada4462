"""dfmm_direct_forces_noalloc (scratch in the library's fixed per-GPU array)
against dfmm_direct_forces (scratch allocated per call), through the C ABI:
two calls in a row on one stream, the second with a smaller input, so the
second reuses the array the first left behind.  The same chunking is used by
both entry points at these sizes, so the forces are bit-identical; the bar
is the direct sum's FP64 parity bar, 1e-12."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def test_noalloc_direct_matches_allocating_direct_twice():
    import torch

    import paper_1712_07739_amd as pk

    dev = torch.device("cuda:0")
    C = synth.loops.CUBIC_A25
    prm = pk.make_params(4, 3, *C, 1e-3, synth.loops.BOX_LO, synth.loops.BOX_SIZE)
    plan = pk.Plan(prm)
    cases = [(60, None, 0), (25, 120, 1), (10, 40, 0)]  # (loops, targets, fp32): sizes shrink call to call
    for nl, ntg, fp32 in cases:
        seg, b = synth.make_loops(nl, 0.01, 0.05, 40 + nl)
        ts, tb = torch.tensor(seg, device=dev), torch.tensor(b, device=dev)
        tgt = None if ntg is None else torch.tensor(synth.segment_subset(len(seg), ntg, 7), device=dev)
        nt = len(seg) if tgt is None else ntg
        need = pk.direct_noalloc_bytes(plan, len(seg), nt)
        assert 0 < need <= pk.NOALLOC_SCRATCH_BYTES
        print("case loops=%d targets=%s fp32=%d scratch=%d bytes" % (nl, ntg, fp32, need), flush=True)
        ref = pk.direct_forces(plan, ts, tb, targets=tgt, fp32=bool(fp32)).cpu().numpy()
        out = torch.full((nt, 2, 3), np.nan, dtype=torch.float64, device=dev)
        f = pk.direct_forces(plan, ts, tb, targets=tgt, fp32=bool(fp32), out=out, noalloc=True).cpu().numpy()
        assert np.isfinite(f).all()
        assert oracle.rel_err(f, ref) <= 1e-12
        assert np.array_equal(f, ref)


def test_noalloc_direct_rejects_sizes_beyond_its_scratch():
    import torch

    import paper_1712_07739_amd as pk

    dev = torch.device("cuda:0")
    prm = pk.make_params(4, 3, *synth.loops.ISO, 1e-3, synth.loops.BOX_LO, synth.loops.BOX_SIZE)
    plan = pk.Plan(prm)
    n = 120000  # 360k points: 26 MB of points plus 69 MB of partial stresses for all targets
    assert pk.direct_noalloc_bytes(plan, n, n) > pk.NOALLOC_SCRATCH_BYTES
    seg = torch.zeros((n, 2, 3), dtype=torch.float64, device=dev)
    b = torch.zeros((n, 3), dtype=torch.float64, device=dev)
    out = torch.empty((n, 2, 3), dtype=torch.float64, device=dev)
    with pytest.raises(pk.DfmmError) as e:
        pk.direct_forces(plan, seg, b, out=out, noalloc=True)
    assert e.value.status == -1
