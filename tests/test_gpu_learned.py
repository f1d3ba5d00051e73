"""Learned warm start of the measurement BP, through the C ABI: the device's
forward and backward kernels against the float64 oracle of the network
(oracle/mlp.py, same BF16-rounded weights and inputs), the Adam step, the
feature rows against the messages the handle reports, and a trained network
that reaches the same fixed points as uniform-start BP in fewer sweeps on a
run whose field h was held out of the training data."""

import numpy as np
import pytest

from oracle import mlp
from paper_2606_30985_amd import inputs
from tests.gpu_util import load_hpt

pytestmark = pytest.mark.gpu
F, H = 16, 128


def _params(seed, scale=0.3):
    g = inputs.rng(seed)
    return (g.standard_normal(mlp.n_params(F, H)) * scale).astype(np.float32)


def test_forward_and_backward_match_the_oracle():
    hpt = load_hpt()
    import torch
    theta = _params(1)
    g = inputs.rng(2)
    X = g.standard_normal((1531, F)).astype(np.float32)
    t = (0.1 * g.standard_normal(1531)).astype(np.float32)
    P = torch.from_numpy(theta).cuda()
    Xd = torch.from_numpy(X).cuda()
    td = torch.from_numpy(t).cuda()
    y = hpt.learn_forward(P, Xd)
    grad, loss = hpt.learn_backward(P, Xd, y, td)
    torch.cuda.synchronize()
    yr, _ = mlp.forward(theta.astype(np.float64), X, F, H)
    assert np.max(np.abs(y.cpu().numpy() - yr)) <= 2e-5 * (1 + np.max(np.abs(yr)))
    Lr, gr = mlp.loss_and_grad(theta.astype(np.float64), X, t, F, H)
    assert abs(loss.item() - Lr) <= 1e-5 * Lr
    gg = grad.cpu().numpy()
    assert np.max(np.abs(gg - gr)) <= 1e-4 * np.max(np.abs(gr))
    # the gradient is taken in a fixed order: the same call gives the same bits
    grad2, _ = hpt.learn_backward(P, Xd, y, td)
    assert torch.equal(grad, grad2)


def test_adam_step_matches_the_oracle():
    hpt = load_hpt()
    import torch
    theta = _params(3)
    gr = _params(4, 1.0)
    P = torch.from_numpy(theta).cuda()
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    G = torch.from_numpy(np.append(gr, 0.0).astype(np.float32)).cuda()
    th, mr, vr = theta.astype(np.float64), np.zeros(theta.size), np.zeros(theta.size)
    for step in (1, 2, 3):
        hpt.learn_adam(P, m, v, G, step, 1e-3)
        th, mr, vr = mlp.adam_step(th, mr, vr, gr.astype(np.float64), step, 1e-3)
    torch.cuda.synchronize()
    assert np.max(np.abs(P.cpu().numpy() - th)) <= 1e-6


def _norm(m):
    m = np.asarray(m, dtype=np.float64)
    s = np.sum(m)
    sg = 1.0 if s > 0 else (-1.0 if s < 0 else (1.0 if m[np.argmax(np.abs(m))] >= 0 else -1.0))
    return sg * m / np.linalg.norm(m)


def test_feature_rows_follow_the_messages():
    hpt = load_hpt()
    sim = hpt.Simulator(Lx=3, Ly=3, chi_max=8, bp_tol=1e-10)
    sim.step(3)
    sim.measure()
    prev = {(b, d): sim.get_meas_message(b, d) for b in range(sim.n_bonds) for d in range(2)}
    chi_prev = {b: sim.chi(b) for b in range(sim.n_bonds)}
    sim.step(1)
    X, base = sim.meas_features()
    X, base = X.cpu().numpy(), base.cpu().numpy()
    # the previous messages are left in place
    for (b, d), m in prev.items():
        if sim.chi(b) == chi_prev[b]:
            assert np.array_equal(sim.get_meas_message(b, d), m)
    row = 0
    for b in range(sim.n_bonds):
        c = sim.chi(b)
        lam = sim.spectrum(b)
        for d in range(2):
            r = slice(row, row + c)
            one = X[r, 1].astype(np.float64)
            assert abs(np.linalg.norm(one) - 1.0) < 1e-6 and np.sum(one) >= -1e-7
            cp = chi_prev[b]
            pn = _norm(prev[(b, d)])
            k = min(c, cp)
            assert np.max(np.abs(X[row: row + k, 2] - pn[:k])) < 1e-6
            assert np.all(X[row: row + k, 3] == 1.0) and np.all(X[row + k: row + c, 3] == 0.0)
            assert np.array_equal(base[r], np.where(X[r, 3] == 1.0, X[r, 2], X[r, 1]))
            assert np.max(np.abs(X[r, 4] - lam * np.sqrt(c))) < 1e-5 * np.sqrt(c)
            assert np.allclose(X[r, 5], np.arange(c) / c)
            row += c
    assert row == X.shape[0]
    m = sim.measure()
    import torch
    T = sim.meas_targets(torch.from_numpy(base).cuda()).cpu().numpy()
    row = 0
    for b in range(sim.n_bonds):
        c = sim.chi(b)
        for d in range(2):
            conv = _norm(sim.get_meas_message(b, d))
            assert np.max(np.abs(T[row: row + c] + base[row: row + c] - conv)) < 1e-6
            row += c
    assert np.isfinite(m["C"])
    sim.close()


def _collect(hpt, runs, layers):
    import torch
    Xs, Ts = [], []
    for cfg in runs:
        sim = hpt.Simulator(**cfg)
        sim.measure()
        for _ in range(layers):
            sim.step(1)
            X, base = sim.meas_features()
            sim.measure()
            Xs.append(X)
            Ts.append(sim.meas_targets(base))
        sim.close()
    return torch.cat(Xs), torch.cat(Ts)


def _train(hpt, X, T, steps, lr=2e-3, seed=5, batch=4096):
    import torch
    P = torch.from_numpy(_params(seed, 0.05)).cuda()
    P[-1] = 0.0
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    g = torch.Generator(device="cuda").manual_seed(seed)
    losses = []
    for step in range(1, steps + 1):
        idx = torch.randint(0, X.shape[0], (min(batch, X.shape[0]),), generator=g, device="cuda")
        Xb, Tb = X[idx].contiguous(), T[idx].contiguous()
        y = hpt.learn_forward(P, Xb)
        grad, loss = hpt.learn_backward(P, Xb, y, Tb)
        hpt.learn_adam(P, m, v, torch.cat([grad, loss]), step, lr)
        losses.append(loss.item())
    return P, losses


def test_trained_warm_start_saves_sweeps_on_a_held_out_field():
    hpt = load_hpt()
    import torch
    base = dict(Lx=4, Ly=4, chi_max=12, dt=0.05, bp_tol=1e-10, meas_tol=1e-10, meas_max_sweeps=400)
    train = [dict(base, h=h) for h in (0.6, 1.4, 2.2)] + [dict(base, Lx=3, Ly=3, h=h) for h in (0.8, 1.8)]
    X, T = _collect(hpt, train, 16)
    P, losses = _train(hpt, X, T, 400)
    assert np.mean(losses[-20:]) < np.mean(losses[:20])
    held = dict(base, h=1.0)
    uni = hpt.Simulator(**held)
    lrn = hpt.Simulator(meas_init="learned", **held)
    lrn.set_meas_model(P)
    su, sl = [], []
    for _ in range(16):
        uni.step(1)
        lrn.step(1)
        mu, ml = uni.measure(), lrn.measure()
        # the same fixed point: the Bethe estimate agrees to the BP tolerance
        assert abs(mu["C"] - ml["C"]) <= 1e-8, (mu["step"], mu["C"], ml["C"])
        su.append(mu["meas_sweeps"])
        sl.append(ml["meas_sweeps"])
    print("uniform sweeps", su, "learned sweeps (incl. the feature sweep)", sl)
    assert sum(sl) < sum(su)
    uni.close()
    lrn.close()
