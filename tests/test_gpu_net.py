"""GPU parity of the learned-initial-guess network against the FP64 oracle
(oracle/net.py), and the gain of a trained network over U_0 = 0.

The GPU network computes in FP32; tolerances: forward rel L2 <= 2e-5, loss rel
<= 2e-5, gradient rel L2 <= 2e-4 (FP32 accumulation over up to 65k pixels per
weight), Adam parameters rel L2 <= 1e-6.
"""

import numpy as np
import pytest
import torch

import synth
from oracle import net as onet
from paper_2502_03611_amd.learned_guess import (Net, cubic_solver, evaluate, generate_pairs,
                                                initial_guess, train)

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def inputs(B, H, W, seed):
    rng = np.random.default_rng(seed)
    f = 30.0 * rng.standard_normal((B, H, W))
    v = rng.standard_normal((B, H, W))
    target = rng.standard_normal((B, H, W))
    return f, v, target


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("B,H,W", [(2, 20, 37), (1, 33, 65), (3, 7, 5), (1, 1, 1)])
def test_forward_parity(B, H, W):
    print(f"net forward {B}x{H}x{W}", flush=True)
    theta = onet.he_init(7).astype(np.float32).astype(np.float64)
    f, v, _ = inputs(B, H, W, 1)
    net = Net(H, W, max_batch=4)
    net.set_params(theta)
    out = net.forward(dev(f), dev(v)).cpu().numpy()
    g_ref, _ = onet.forward(theta, onet.features(f, v))
    assert rel(f - out, g_ref) <= 2e-5


@pytest.mark.parametrize("B,H,W", [(2, 20, 37), (1, 33, 65), (3, 7, 5), (1, 1, 1), (1, 255, 255)])
def test_fused_fp16_forward_parity(B, H, W):
    """The fused FP16 inference kernel against the FP64 oracle.  FP16 rounds
    every weight and every stored activation to 2^-11 relative (five layers,
    FP32 accumulation over at most 288 products): a few 1e-3 relative in g,
    bound 1e-2; ragged tiles (W = 37, 65, 5, 255), one-pixel images and
    batches cover the halo recomputation and the zero padding."""
    print(f"net fused fp16 {B}x{H}x{W}", flush=True)
    theta = onet.he_init(7).astype(np.float32).astype(np.float64)
    f, v, _ = inputs(B, H, W, 1)
    net = Net(H, W, max_batch=4)
    net.set_params(theta)
    net.set_inference("fp16")
    out = net.forward(dev(f), dev(v)).cpu().numpy()
    g_ref, _ = onet.forward(theta, onet.features(f, v))
    err = rel(f - out, g_ref)
    print(f"  rel L2 of g vs oracle {err:.2e}", flush=True)
    assert err <= 1e-2
    net.set_inference("fp32")
    out32 = net.forward(dev(f), dev(v)).cpu().numpy()
    assert rel(f - out32, g_ref) <= 2e-5


def test_fused_fp16_forward_trained_weights_on_solver_inputs():
    """The committed trained weights on the workload's inputs (255^2 random
    field sources and their A_h^-1 f): g within 1e-2 of the oracle's."""
    from paper_2502_03611_amd import learned_guess as lg
    theta = np.load(lg.WEIGHTS, allow_pickle=False).astype(np.float64)
    n = 255
    s = cubic_solver(n)
    f = np.stack([synth.learned_guess_rhs(10000 + i, n) for i in range(2)])
    F = dev(f)
    V = torch.empty_like(F)
    for i in range(2):
        s.fdm_solve(F[i:i + 1], 1.0, 0.0, X=V[i:i + 1])
    net = Net(n, n, max_batch=2)
    net.set_params(theta)
    net.set_inference("fp16")
    out = net.forward(F, V).cpu().numpy()
    g_ref, _ = onet.forward(theta, onet.features(f, V.cpu().numpy()))
    err = rel(f - out, g_ref)
    print(f"  trained weights: rel L2 of g vs oracle {err:.2e}", flush=True)
    assert err <= 1e-2


def test_forward_batch_matches_single_images_bitwise():
    """Per-pixel arithmetic does not depend on the batch: a batch of two 255^2
    images (130050 pixels, so the output layer walks its grid-stride loop)
    returns the bits of the two images run one at a time."""
    H = W = 255
    theta = onet.he_init(9).astype(np.float32).astype(np.float64)
    f, v, _ = inputs(2, H, W, 5)
    net = Net(H, W, max_batch=2)
    net.set_params(theta)
    both = net.forward(dev(f), dev(v))
    for b in range(2):
        one = net.forward(dev(f[b:b + 1]), dev(v[b:b + 1]))
        assert torch.equal(both[b:b + 1], one), b


@pytest.mark.parametrize("B,H,W", [(2, 20, 37), (1, 17, 40)])
def test_loss_and_gradient_parity(B, H, W):
    print(f"net grad {B}x{H}x{W}", flush=True)
    theta = onet.he_init(11).astype(np.float32).astype(np.float64)
    f, v, target = inputs(B, H, W, 2)
    net = Net(H, W, max_batch=4)
    net.set_params(theta)
    loss = net.loss_grad(dev(f), dev(v), dev(target))
    g = net.get_grads()
    ref_loss, ref_g = onet.loss_and_grad(theta, onet.features(f, v), target)
    assert loss == pytest.approx(ref_loss, rel=2e-5)
    assert rel(g, ref_g) <= 2e-4
    # every layer's block separately (weights and biases)
    o = 0
    for ws, bs in onet.layer_shapes():
        for sz in (int(np.prod(ws)), int(np.prod(bs))):
            assert rel(g[o:o + sz], ref_g[o:o + sz]) <= 5e-4, (o, sz)
            o += sz


def test_adam_steps_match_oracle_and_are_deterministic():
    H, W = 12, 34
    theta = onet.he_init(5).astype(np.float32).astype(np.float64)
    f, vin, target = inputs(2, H, W, 3)
    ft, vt, tt = dev(f), dev(vin), dev(target)
    net = Net(H, W, max_batch=2)
    net.set_params(theta)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    th = theta.copy()
    for t in (1, 2):
        net.loss_grad(ft, vt, tt)
        g = net.get_grads().astype(np.float64)
        net.adam_step(1e-3)
        th, m, v = onet.adam_step(th, g, m, v, t, lr=1e-3)
        assert rel(net.get_params(), th) <= 1e-6
    net2 = Net(H, W, max_batch=2)
    net2.set_params(theta)
    for _ in (1, 2):
        net2.loss_grad(ft, vt, tt)
        net2.adam_step(1e-3)
    assert np.array_equal(net.get_params(), net2.get_params())


def test_fallback_to_zero_on_bad_network():
    n = 31
    net = Net(n, n, max_batch=1)
    theta = np.zeros(net.nparam, dtype=np.float32)
    theta[-1] = 1e20  # output bias: g = 1e20 everywhere, a useless guess
    net.set_params(theta)
    solver = cubic_solver(n)
    f = torch.from_numpy(synth.learned_guess_rhs(3, n)).cuda()
    u0, used = initial_guess(net, solver, f)
    assert int(used.item()) == 0 and float(u0.abs().max()) == 0.0


@pytest.mark.parametrize("red,keep", [((1.0, 0, 0, 2.0), True), ((2.0, 0, 0, 2.0), False),
                                      ((3.0, 0, 0, 2.0), False),
                                      ((float("nan"), 0, 0, 2.0), False),
                                      ((float("inf"), 0, 0, 2.0), False)])
def test_guess_fallback_decision(red, keep):
    """The device-side choice keeps the guess only when sum R^2 < sum F^2."""
    H, W = 19, 23
    net = Net(H, W, max_batch=1)
    u0 = dev(np.random.default_rng(4).standard_normal((1, H, W)))
    ref = u0.clone()
    used = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    net.guess_fallback(dev(np.array(red, np.float64)), u0, used)
    assert int(used.item()) == int(keep)
    assert torch.equal(u0, ref) if keep else float(u0.abs().max()) == 0.0
    net.guess_fallback(dev(np.array(red, np.float64)), u0)  # used is optional


def test_trained_network_saves_iterations():
    """Train on solver-generated pairs (small grid, short schedule) and compare
    iterations to 1e-10 on held-out seeds from U_0 = 0 and from the network."""
    print("net training gain", flush=True)
    n = 63
    F, V, G, _ = generate_pairs(range(0, 256), n=n)
    net = Net(n, n, max_batch=16)
    hist = train(net, F, V, G, epochs=30, batch=16, lr=1e-3, seed=0)
    assert hist[-1] < 0.2 * hist[0]
    rows = evaluate(net, range(10000, 10024), n=n)
    zero = np.mean([r["iters_zero"] for r in rows])
    learned = np.mean([r["iters_net"] for r in rows])
    print(f"  mean iterations: U0=0 {zero:.2f}, learned {learned:.2f}", flush=True)
    assert all(r["status"] == (0, 0) for r in rows)
    assert all(r["rel_diff"] <= 1e-8 for r in rows)  # same solution either way
    # v0 alone is the first quasi-Newton iterate (saves exactly 1); the trained
    # network must do better than that on average
    assert learned <= zero - 1.25
