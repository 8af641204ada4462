"""GPU tests of the learned anisotropic-kernel surrogate.

* forward pass and loss gradient of the library's kernels against a plain
  numpy FP64 implementation of the same network (textbook back-propagation);
* training lowers the loss; the residual gate reports per-bin errors;
* a gate that passes no bin gives results bit-identical to the exact kernel;
* with the surrogate in use the FMM still matches the oracle;
* the near-field time with and without the surrogate is measured and printed.
"""
import time

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

BOX_LO, BOX = synth.loops.BOX_LO, synth.loops.BOX_SIZE
CUB = synth.loops.CUBIC_A25
DIMS = (6, 128, 128, 128, 128, 18)


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_1712_07739_amd as pk

    assert torch.cuda.is_available()
    return torch, pk, torch.device("cuda:0")


def unpack(params):
    layers, off = [], 0
    for l in range(5):
        din, dout = DIMS[l], DIMS[l + 1]
        W = params[off:off + din * dout].reshape(dout, din)
        off += din * dout
        b = params[off:off + dout]
        off += dout
        layers.append((W, b))
    assert off == params.size
    return layers


def np_forward(params, X):
    layers = unpack(params)
    A, Z = [X], []
    for l, (W, b) in enumerate(layers):
        z = A[-1] @ W.T + b
        Z.append(z)
        A.append(z / (1.0 + np.exp(-z)) if l < 4 else z)
    return A, Z, layers


def np_loss_grad(params, X, Y):
    A, Z, layers = np_forward(params, X)
    n = Y.size
    d = A[-1] - Y
    loss = float((d ** 2).sum() / n)
    dZ = 2.0 * d / n
    grads = [None] * 5
    for l in range(4, -1, -1):
        W, b = layers[l]
        grads[l] = (dZ.T @ A[l], dZ.sum(0))
        if l > 0:
            dA = dZ @ W
            z = Z[l - 1]
            s = 1.0 / (1.0 + np.exp(-z))
            dZ = dA * s * (1.0 + z * (1.0 - s))
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


def cubic_plan(pk, p=4, D=3, precision=1):
    return pk.Plan(pk.make_params(p, D, *CUB, 1e-3, BOX_LO, BOX, precision=precision))


def test_forward_and_gradient_match_cpu_reference(env):
    torch, pk, dev = env
    plan = cubic_plan(pk)
    rng = np.random.default_rng(3)
    n_par = sum(DIMS[l] * DIMS[l + 1] + DIMS[l + 1] for l in range(5))
    params = (rng.normal(size=n_par) * 0.15).astype(np.float32)
    plan.surrogate_set_params(params)
    assert np.array_equal(plan.surrogate_params(), params)
    X = rng.normal(size=(333, 6)).astype(np.float32)
    Y = rng.normal(size=(333, 18)).astype(np.float32)
    p64 = params.astype(np.float64)
    A, _, _ = np_forward(p64, X.astype(np.float64))
    yg = plan.surrogate_forward(torch.tensor(X, device=dev)).cpu().numpy()
    assert np.abs(yg - A[-1]).max() <= 1e-4 * np.abs(A[-1]).max()
    loss_g, grad_g = plan.surrogate_loss_grad(torch.tensor(X, device=dev), torch.tensor(Y, device=dev))
    loss_c, grad_c = np_loss_grad(p64, X.astype(np.float64), Y.astype(np.float64))
    assert abs(loss_g - loss_c) <= 1e-5 * abs(loss_c)
    grad_g = grad_g.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(grad_g - grad_c) <= 1e-4 * np.linalg.norm(grad_c)
    # the check has teeth: a perturbed weight changes the gradient measurably
    params2 = params.copy()
    params2[100] += 0.5
    plan.surrogate_set_params(params2)
    _, grad_p = plan.surrogate_loss_grad(torch.tensor(X, device=dev), torch.tensor(Y, device=dev))
    assert np.linalg.norm(grad_p.cpu().numpy() - grad_c) > 1e-3 * np.linalg.norm(grad_c)


def test_training_lowers_loss_and_gate_reports(env):
    torch, pk, dev = env
    plan = cubic_plan(pk)
    info = plan.surrogate_train(n_samples=1 << 18, epochs=6, batch=2048, bins=8, tol=1e-3, seed=7)
    loss = info["loss"]
    print("surrogate training:", info)
    assert len(loss) == 6 and loss[-1] < 0.05 * loss[0]
    assert info["trained"] == 1 and 0.0 <= info["pass_frac"] <= 1.0
    assert info["max_bin_err"] >= info["median_bin_err"] > 0
    # a tolerance above every bin error gates everything in
    info2 = plan.surrogate_train(n_samples=1 << 16, epochs=1, batch=1024, bins=4, tol=10.0, seed=7)
    assert info2["pass_frac"] == 1.0


def _forces(env, plan, seg, b):
    torch, pk, dev = env
    ts = torch.tensor(seg, device=dev)
    tb = torch.tensor(b, device=dev)
    tree = pk.Tree(plan, ts)
    f = pk.fmm_forces(plan, tree, ts, tb).cpu().numpy()
    return f, tree, ts, tb


def test_gate_closed_is_bit_identical_to_exact(env):
    torch, pk, dev = env
    seg, b = synth.make_loops(12, 0.01, 0.05, 31)
    plan = cubic_plan(pk)
    f_exact, _, _, _ = _forces(env, plan, seg, b)
    info = plan.surrogate_train(n_samples=1 << 16, epochs=1, batch=1024, bins=8, tol=0.0, seed=3)
    assert info["pass_frac"] == 0.0
    plan.surrogate_use(True)
    f_sur, _, _, _ = _forces(env, plan, seg, b)
    assert np.array_equal(f_sur, f_exact)


def test_surrogate_in_use_matches_oracle_and_gain_is_measured(env):
    torch, pk, dev = env
    seg, b = synth.make_loops(12, 0.01, 0.05, 31)
    med = oracle.medium(*CUB, 1e-3)
    ref = oracle.fmm_forces(seg, b, med, 4, 3, BOX_LO, BOX)
    plan = cubic_plan(pk)
    info = plan.surrogate_train(n_samples=1 << 20, epochs=8, batch=4096, bins=16, tol=1e-4, seed=11)
    print("surrogate gate:", {k: info[k] for k in ("pass_frac", "max_bin_err", "median_bin_err", "train_ms")})
    f_exact, tree, ts, tb = _forces(env, plan, seg, b)
    plan.surrogate_use(True)
    f_sur, tree2, _, _ = _forces(env, plan, seg, b)
    assert oracle.rel_err(f_exact, ref) <= 2e-5
    # bins gated in at tolerance 1e-4 keep the kernel within 1e-4 of the exact one
    assert oracle.rel_err(f_sur, ref) <= 2e-4
    # near-field time with and without the network (the gain, or loss, it brings)
    res = {}
    for name, on, tr in (("exact", False, tree), ("surrogate", True, tree2)):
        plan.surrogate_use(on)
        tr.set_timing(True)
        for _ in range(3):
            pk.fmm_forces(plan, tr, ts, tb)
        ms, n = tr.stage_times()
        res[name] = ms[6] / n
        tr.set_timing(False)
    print("near-field ms per call: exact %.3f, surrogate %.3f (pass_frac %.3f)"
          % (res["exact"], res["surrogate"], info["pass_frac"]))
    assert res["exact"] > 0 and res["surrogate"] > 0
