"""GPU: the learned warm start's kernels against the CPU oracle.

* features and targets of a running state (oracle: the same definitions in
  FP64 on the oracle's own state, gradients from the oracle);
* bf16 matrix-core inference against the oracle's bf16 emulation, rows not
  a multiple of the 16-row tile;
* FP32 training kernels: loss and gradient against the FP64 oracle, one and
  three Adam steps against the oracle's update from its own gradient;
* the Grad-type initial distribution and the Maxwellian fallback against the
  oracle's construction from the same network outputs.
"""

import numpy as np
import pytest

import ugks_cases as uc
from oracle import Oracle
from oracle import learned as L
from paper_2606_15720_amd import ugks as U
from paper_2606_15720_amd import warmstart as WS

pytestmark = pytest.mark.gpu


def _states(case, steps):
    o = Oracle(case)
    s = U.Solver(case)
    o.step(steps)
    s.step(steps)
    return o, s


@pytest.mark.parametrize("which", ["cavity2d", "sod3d"])
def test_features_and_targets_match_oracle(which):
    if which == "cavity2d":
        case, steps = uc.cavity2d(n=8, nv=16, kn=0.1), 25
    else:
        case, steps = uc.sod3d_tets(n=3, nv=12), 6
    o, s = _states(case, steps)
    Fg, Tg = U.ugks_snapshot(s.h, case.mesh.n_cells)
    Wo, ho, bo, _ = o.state()
    Fo = L.features(Wo, o.grad_W(), case.gas)
    To = L.targets(Wo, ho, bo, case.vel, case.gas.R)
    print(which, "feature scale", np.abs(Fo).max(axis=0), flush=True)
    print(which, "target scale", np.abs(To).max(axis=0), flush=True)
    # stored as float: relative 2^-24 of each column's scale, plus the FP64 state difference
    fs = np.abs(Fo).max(axis=0) + 1e-12
    ts = np.abs(To).max(axis=0) + 1e-12
    assert np.all(np.abs(Fg - Fo).max(axis=0) <= 1e-6 * fs), np.abs(Fg - Fo).max(axis=0) / fs
    assert np.all(np.abs(Tg - To).max(axis=0) <= 1e-6 * ts), np.abs(Tg - To).max(axis=0) / ts
    assert np.abs(Fo).max() > 1e-4  # the state is not uniform
    s.close()


def _net(seed=1):
    rng = np.random.default_rng(seed)
    p = (WS.init_params(seed) + rng.normal(0, 0.05, WS.NPARAM)).astype(np.float32)
    si = rng.uniform(0.5, 2.0, 9).astype(np.float32)
    so = rng.uniform(0.5, 2.0, 9).astype(np.float32)
    return p, si, so


def test_mlp_inference_matches_oracle_bf16():
    p, si, so = _net(1)
    net = U.MLP(p, si, so)
    rng = np.random.default_rng(2)
    x = rng.normal(0.0, 1.0, (1000, 9)).astype(np.float32)  # 62.5 tiles of 16 rows
    y = net.forward(x)
    xs = (x * si).astype(np.float32)
    yb = L.forward_bf16(p, xs) * so
    y64 = L.forward(p, xs.astype(np.float64))[0] * so
    scale = np.abs(yb).max()
    err = np.abs(y - yb)
    print("bf16 inference: max", err.max() / scale, "mean", err.mean() / scale,
          "vs FP64 network", np.abs(y - y64).max() / scale, flush=True)
    # same roundings on both sides; a hidden activation whose bf16 rounding
    # flips on an accumulation-order difference moves an output by ~2^-8 |w|.
    # Such flips need a pre-activation within an FP32 rounding of a bf16
    # rounding boundary, so almost every row agrees to FP32 accumulation
    # error and the few that do not stay within the flip bound.
    rows_ok = np.mean(err.max(axis=1) <= 1e-5 * scale)
    print("rows within 1e-5 of the emulation:", rows_ok, flush=True)
    assert rows_ok >= 0.99
    assert err.max() <= 1e-2 * scale and err.mean() <= 1e-3 * scale
    assert np.abs(y - y64).max() <= 5e-2 * scale
    # empty and single-row calls
    assert net.forward(np.zeros((0, 9), np.float32)).shape == (0, 9)
    np.testing.assert_allclose(net.forward(x[:1]), y[:1], rtol=0, atol=0)
    net.close()


def test_mlp_gradient_and_adam_match_oracle():
    p, si, so = _net(3)
    net = U.MLP(p, si, so)
    rng = np.random.default_rng(4)
    n = 700
    x = rng.normal(0.0, 1.0, (n, 9)).astype(np.float32)
    t = rng.normal(0.0, 1.0, (n, 9)).astype(np.float32)
    xs = (x * si).astype(np.float64)
    ts = (t / so).astype(np.float64)
    loss_g, g_g = net.loss_grad(x, t)
    loss_o, g_o = L.loss_grad(p.astype(np.float64), xs, ts)
    rel = np.abs(g_g - g_o).max() / np.abs(g_o).max()
    print("loss", loss_g, loss_o, "grad rel err", rel, flush=True)
    assert loss_g == pytest.approx(loss_o, rel=1e-5)
    assert rel <= 1e-4
    # Adam from the oracle's own gradients, three full-batch steps
    lr = 1e-3
    po, m, v = p.astype(np.float64), np.zeros(WS.NPARAM), np.zeros(WS.NPARAM)
    for step in range(1, 4):
        g = L.loss_grad(po, xs, ts)[1]
        po, m, v = L.adam(po, m, v, g, step, lr)
    net.train(x, t, batch=n, steps=3, lr=lr)
    pg = net.params()
    # each step moves a parameter by about lr; gradients that are tiny next
    # to FP32 noise may go either way
    big = np.abs(g_o) > 1e-3 * np.abs(g_o).max()
    d = np.abs(pg - po)
    print("adam max dev (big grads)", d[big].max(), "all", d.max(), flush=True)
    assert d[big].max() <= 0.02 * lr * 3
    assert d.max() <= 2.0 * lr * 3
    net.close()


def test_training_reduces_the_loss():
    # a Chapman-Enskog-like target: linear in the features plus a mild nonlinearity
    rng = np.random.default_rng(6)
    x = rng.normal(0.0, 1.0, (4096, 9)).astype(np.float32)
    A = rng.normal(0.0, 1.0, (9, 9))
    t = (x @ A.T + 0.3 * np.tanh(x[:, :1]) * x[:, 1:2]).astype(np.float32)
    net, losses = WS.train(x, t, seed=0, steps=800, batch=512, lr=3e-3, lr_final=3e-4)
    print("loss first/last", losses[0], losses[-1], flush=True)
    assert losses[-1] < 0.05 * losses[0]
    net.close()


@pytest.mark.parametrize("which", ["couette2d", "sod3d"])
def test_warm_start_matches_oracle_grad_distribution(which):
    if which == "couette2d":
        case, steps = uc.couette2d(n=8, nv=16, kn=0.2), 30
    else:
        case, steps = uc.sod3d_tets(n=3, nv=12), 6
    s = U.Solver(case)
    s.step(steps)
    F, T = U.ugks_snapshot(s.h, case.mesh.n_cells)
    p, si, so = _net(5)
    so = (so * 0.02).astype(np.float32)  # outputs of the size of a real closure
    net = U.MLP(p, si, so)
    # a box that leaves the cells with the largest value of the most varied
    # feature out: they keep the Maxwellian
    lo, hi = F.min(axis=0), F.max(axis=0).copy()
    col = int(np.argmax(F.std(axis=0)))
    hi[col] = np.unique(F[:, col])[-2]
    net.set_box(lo, hi)
    W = s.W()
    out = net.forward(F)
    use = L.inside_box(F, lo, hi)
    nfall = U.ugks_warm_start(s.h, net)
    assert nfall == int(np.sum(~use)) and 0 < nfall < case.mesh.n_cells
    _, hg, bg = s.state()
    ho, bo = L.grad_distribution(W, out.astype(np.float64), case.vel, use=use)
    err = np.abs(hg - ho).max() / np.abs(ho).max()
    print(which, "fallback cells", nfall, "h err", err, flush=True)
    assert err <= 1e-13
    if case.mesh.dim == 2:
        assert np.abs(bg - bo).max() / np.abs(bo).max() <= 1e-13
    # the new state steps on as the oracle does from the same f
    o = Oracle(case)
    o.set_state(W, hg, bg)
    s.step(2)
    o.step(2)
    Wo = o.state(with_h=False)[0]
    Wg = s.W()
    assert np.abs(Wg - Wo).max() / np.abs(Wo).max() <= 1e-12
    net.close()
    s.close()


def test_trained_network_beats_the_maxwellian_start():
    """What the trained network gains: a rarefied cavity (Kn = 0.1) restarted
    on a fine velocity set from a coarse-velocity solution converges faster
    from the network's Grad-type f than from the Maxwellian of the same W.
    The network is trained here, on the GPU, on snapshots of other runs."""
    F, T = WS.build_training_set(4)
    net, losses = WS.train(F, T, seed=4, steps=4000, batch=1024)
    assert losses[-1] < 0.2 * losses[0]
    fine = uc.cavity2d(n=24, nv=28, kn=0.1, lid=0.5)
    coarse = uc.cavity2d(n=24, nv=12, kn=0.1, lid=0.5)
    p = U.Solver(coarse)
    _, r, ok = WS.run_to_residual(p, 1e-6, 20000, 500)
    assert ok
    Wp = p.W()
    p.close()
    hist = {}
    for warm in (False, True):
        case = uc.Case(fine.name, fine.mesh, fine.vel, fine.gas, fine.bcs, Wp, 0, fine.meta)
        s = U.Solver(case)
        if warm:
            assert U.ugks_warm_start(s.h, net) == 0  # every cell inside the training box
        rs = []
        for n in (400, 400, 800):
            rs.append(s.step(n)[1])
        hist[warm] = rs
        s.close()
    print("residual after 400/800/1600 steps: maxwell", hist[False], "learned", hist[True], flush=True)
    assert hist[True][0] < 0.5 * hist[False][0]
    assert hist[True][2] < 0.5 * hist[False][2]
    net.close()
