"""The Newton guess network on the GPU against the oracle (oracle/mlp.c).

Bars: evaluation with bfloat16 weights and binary32 sums within 1e-5 (relative
to the largest output) of the oracle's binary64 evaluation of the same
bfloat16-rounded weights; the training gradient and loss of one batch within
1e-5 of the oracle's; a short training run tracking the oracle's loss curve;
recorded samples equal to the history the diagnostics report; the in-step
guess equal to the host's reconstruction from those samples.
"""
import numpy as np
import pytest

import oracle
from paper_2603_24010_amd import workloads as W

pytestmark = pytest.mark.gpu

rng = np.random.default_rng(77)


def _gs():
    from paper_2603_24010_amd import gapsim
    return gapsim


def _theta(scale=0.12):
    th = rng.normal(0.0, scale, oracle.MLP_NPARAM).astype(np.float32)
    return th


def _unit_norm():
    return np.concatenate([np.zeros(48), np.ones(48), np.zeros(3), np.ones(3)])


def _small_sim(n_cells=256, n0=20000, beam=200, seed=3):
    gs = _gs()
    cfg = W.config2(n_cells=n_cells, beam_per_step=beam)
    sim = gs.GapSim(cfg, particle_fp=32, capacity=(200_000, 200_000))
    for sp, (x, v) in W.load_config2(n=n0, seed=seed).items():
        sim.inject(0, sp, x, v)
    return sim, cfg


def test_forward_matches_oracle_bf16():
    import torch
    sim, _ = _small_sim()
    theta = _theta()
    sim.mlp_set_weights(theta, _unit_norm())
    x = rng.normal(0, 1.5, (300, 48)).astype(np.float32)
    y = sim.mlp_forward(torch.from_numpy(x).cuda()).cpu().numpy()
    th_bf = oracle.round_bf16(theta).astype(np.float64)
    yo = oracle.mlp_forward(th_bf, x.astype(np.float64))
    err = np.abs(y - yo).max() / np.abs(yo).max()
    print(f"bf16 forward, binary32 sums vs binary64: {err:.2e}")
    assert err <= 1e-5
    # against the unrounded binary32 weights the bfloat16 rounding shows
    y32 = oracle.mlp_forward(theta.astype(np.float64), x.astype(np.float64))
    print(f"bf16 weights vs binary32 weights: {np.abs(y - y32).max() / np.abs(y32).max():.2e}")
    sim.close()


def _train_data(n):
    x = rng.normal(0, 1, (n, 48)).astype(np.float32)
    # a smooth target the network can fit
    t = np.stack([np.tanh(x[:, 0] - 0.5 * x[:, 7]), 0.3 * x[:, 3] * x[:, 12], np.sin(x[:, 20])],
                 axis=1).astype(np.float32)
    return x, t


def test_training_gradient_and_adam_match_oracle():
    import torch
    gs = _gs()
    n, B = 2048, 512
    x, t = _train_data(n)
    order = rng.permutation(n).astype(np.int32)[:B]
    theta0 = _theta(0.1)
    th = torch.from_numpy(theta0.copy()).cuda()
    m = torch.zeros_like(th)
    v = torch.zeros_like(th)
    lr = 1e-3
    loss, grad = gs.mlp_train(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda(),
                              torch.from_numpy(order).cuda(), B, th, m, v, step0=0, lr=lr, want_grad=True)
    lo, go = oracle.mlp_loss_grad(theta0.astype(np.float64), x[order].astype(np.float64),
                                  t[order].astype(np.float64))
    g = grad.cpu().numpy().astype(np.float64)
    gerr = np.abs(g - go).max() / np.abs(go).max()
    print(f"gradient vs oracle: {gerr:.2e}; loss {loss.item():.6e} vs {lo:.6e}")
    assert gerr <= 1e-5
    assert abs(loss.item() - lo) <= 1e-5 * lo
    # Adam from the GPU's own gradient, applied by the oracle
    th_o = theta0.astype(np.float64).copy()
    mo = np.zeros_like(th_o)
    vo = np.zeros_like(th_o)
    oracle.adam_step(th_o, mo, vo, 1, g, lr)
    np.testing.assert_allclose(th.cpu().numpy(), th_o, rtol=0, atol=1e-6 * lr + 1e-7)


def test_training_run_tracks_oracle():
    import torch
    gs = _gs()
    n, B, steps = 1024, 128, 25
    x, t = _train_data(n)
    order = np.concatenate([rng.permutation(n) for _ in range(4)]).astype(np.int32)[:B * steps]
    theta0 = _theta(0.1)
    th = torch.from_numpy(theta0.copy()).cuda()
    m, v = torch.zeros_like(th), torch.zeros_like(th)
    loss, _ = gs.mlp_train(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda(), torch.from_numpy(order).cuda(),
                           B, th, m, v, lr=3e-3)
    loss = loss.cpu().numpy()
    th_o = theta0.astype(np.float64).copy()
    mo, vo = np.zeros_like(th_o), np.zeros_like(th_o)
    lo = []
    for k in range(steps):
        idx = order[k * B:(k + 1) * B]
        l, gk = oracle.mlp_loss_grad(th_o, x[idx].astype(np.float64), t[idx].astype(np.float64))
        lo.append(l)
        oracle.adam_step(th_o, mo, vo, k + 1, gk, 3e-3)
    lo = np.array(lo)
    print("GPU loss", loss[[0, 5, 10, 24]], "oracle", lo[[0, 5, 10, 24]])
    assert loss[-1] < 0.7 * loss[0]
    np.testing.assert_allclose(loss, lo, rtol=2e-3)


def _qabs_qem(cfg, d):
    s = cfg.area * cfg.weight * cfg.q_unit
    qabs = s * (cfg.Z[1] * d["abs_step"][1][0] + cfg.Z[0] * d["abs_step"][0][0])
    qem = s * cfg.Z[0] * d["emit_step"][0]
    return qabs, qem


def test_recorded_samples_match_history():
    import torch
    sim, cfg = _small_sim()
    gs = _gs()
    n = 30
    xr = torch.zeros((n, 48), dtype=torch.float32, device="cuda")
    yr = torch.zeros((n, 3), dtype=torch.float32, device="cuda")
    sim.mlp_record(xr, yr)
    ds = []
    for _ in range(n):
        sim.step_strict(1, gs.GUESS_EXTRAP)
        ds.append(sim.diag(0))
    sim.mlp_record()
    xr, yr = xr.cpu().numpy(), yr.cpu().numpy()
    # level m: its (V, I_0, I_1, sigma) and the charge of the push after it,
    # which the diagnostics read right after level m report as the last push's
    hist = []
    for d in ds:
        qa, qe = _qabs_qem(cfg, d)
        hist.append([d["phi0"], d["I"][0], d["I"][1], d["sigma"], qa, qe])
    hist = np.array(hist)
    u = hist[:, :3]
    for lv in range(12, n):
        want = np.concatenate([hist[lv - kk] for kk in range(1, 9)])
        np.testing.assert_allclose(xr[lv], want.astype(np.float32), rtol=2e-7, atol=0)
        ue = 3 * u[lv - 1] - 3 * u[lv - 2] + u[lv - 3]
        np.testing.assert_allclose(yr[lv], (u[lv] - ue).astype(np.float32), rtol=1e-6,
                                   atol=1e-6 * np.abs(u[lv] - ue).max())
    sim.close()


def test_guess_from_network_in_strict_step():
    import torch
    sim, cfg = _small_sim()
    gs = _gs()
    n_warm, n_mlp = 20, 12
    xr = torch.zeros((n_warm + n_mlp, 48), dtype=torch.float32, device="cuda")
    yr = torch.zeros((n_warm + n_mlp, 3), dtype=torch.float32, device="cuda")
    sim.mlp_record(xr, yr)
    ds = []
    for _ in range(n_warm):
        sim.step_strict(1, gs.GUESS_EXTRAP)
        ds.append(sim.diag(0))
    # normalisation from the recorded history, a small random network
    # (scales kept above 1% of each feature's magnitude, so that the binary32
    # record of a feature pins its normalised value to about 1e-5)
    xh = xr[12:n_warm].cpu().numpy().astype(np.float64)
    mu, sd = xh.mean(0), np.maximum(xh.std(0), 1e-2 * np.abs(xh).max(0))
    sd[sd == 0.0] = 1.0
    yh = yr[12:n_warm].cpu().numpy().astype(np.float64)
    ymu, ysd = yh.mean(0), np.maximum(yh.std(0), 1e-2 * np.abs(yh).max(0))
    ysd[ysd == 0.0] = 1.0
    norm = np.concatenate([mu, sd, ymu, ysd])
    theta = _theta(0.05)
    sim.mlp_set_weights(theta, norm)
    th_bf = oracle.round_bf16(theta).astype(np.float64)
    for _ in range(n_mlp):
        sim.step_strict(1, gs.GUESS_MLP)
        ds.append(sim.diag(0))
    xr = xr.cpu().numpy().astype(np.float64)
    u = np.array([[d["phi0"], d["I"][0], d["I"][1]] for d in ds])
    for lv in range(n_warm, n_warm + n_mlp):
        d = ds[lv]
        assert d["newton_last"] >= 0 and d["newton_resid"] <= 1e-10
        ue = 3 * u[lv - 1] - 3 * u[lv - 2] + u[lv - 3]
        y = oracle.mlp_forward(th_bf, ((xr[lv] - mu) / sd)[None, :])[0]
        prop = ue + ymu + ysd * y
        scale = np.abs(ue) + ysd
        assert np.all(np.abs(d["mlp_proposal"] - prop) <= 1e-4 * scale), (lv, d["mlp_proposal"], prop)
        # the iteration starts from the proposal unless it was worse than the
        # extrapolation (then from the extrapolation)
        start = d["mlp_proposal"] if not d["newton_fallback_last"] else ue
        np.testing.assert_allclose(d["newton_guess"], start, rtol=1e-12, atol=1e-12 * scale.max())
    sim.close()


def test_mlp_guess_needs_weights_and_two_meshes():
    gs = _gs()
    sim, _ = _small_sim()
    with pytest.raises(gs.GapsimError) as e:
        sim.step_strict(1, gs.GUESS_MLP)
    assert e.value.status == gs.GS_ESTATE
    sim.close()
    cfg = W.config1(n_cells=32)  # one mesh
    sim = gs.GapSim(cfg, particle_fp=64, capacity=(64, 64))
    sim.mlp_set_weights(_theta(), _unit_norm())
    with pytest.raises(gs.GapsimError) as e:
        sim.step_strict(1, gs.GUESS_MLP)
    assert e.value.status == gs.GS_EINVAL
    sim.close()


def test_trained_network_against_plain_extrapolation():
    """What the trained network gains: record samples from a small ensemble,
    train on the GPU, then run held-out gaps with the plain extrapolated guess
    and with the network.  The network's start is never worse than the
    extrapolation (worse proposals fall back), so it can only save updates;
    training must beat the untrained network on held-out samples.  The gain
    itself is printed, not asserted: these inputs may hold little of what the
    correction depends on."""
    import torch
    import bench
    gs = _gs()
    G, steps, skip = 16, 240, 11
    sim, _, _ = bench.make_batched(G, 256, 0, steps, np_lo=5000, np_hi=20000)
    xr = torch.zeros((G * steps, 48), dtype=torch.float32, device="cuda")
    yr = torch.zeros((G * steps, 3), dtype=torch.float32, device="cuda")
    sim.mlp_record(xr, yr)
    sim.step_strict(steps, gs.GUESS_DIRECT)
    sim.mlp_record()
    sim.close()
    x, y = xr[skip * G:].double(), yr[skip * G:].double()
    xm, xs = x.mean(0), x.std(0)
    xs[xs == 0] = 1.0
    ym, ys = y.mean(0), y.std(0)
    ys[ys == 0] = 1.0
    norm = torch.cat([xm, xs, ym, ys]).cpu().numpy()
    xn, yn = ((x - xm) / xs).float(), ((y - ym) / ys).float()
    n = xn.shape[0]
    perm = torch.from_numpy(rng.permutation(n)).cuda()
    val, trn = perm[: n // 5], perm[n // 5:]
    theta0 = _theta(0.05)
    th = torch.from_numpy(theta0.copy()).cuda()
    m, v = torch.zeros_like(th), torch.zeros_like(th)
    order = torch.from_numpy(np.concatenate([rng.permutation(len(trn)) for _ in range(30)]).astype(np.int32)).cuda()
    gs.mlp_train(xn[trn].contiguous(), yn[trn].contiguous(), order, 64, th, m, v, lr=1e-3)
    theta = th.cpu().numpy()
    probe, _, _ = bench.make_batched(1, 64, 0, 1, np_lo=100, np_hi=100)
    mse = {}
    for name, w in (("trained", theta), ("untrained", theta0)):
        probe.mlp_set_weights(w, norm)
        mse[name] = float(((probe.mlp_forward(xn[val].contiguous()) - yn[val]) ** 2).mean())
    probe.close()
    mse["zero"] = float((yn[val] ** 2).mean())
    print("validation MSE (normalised):", mse)
    assert mse["trained"] < mse["untrained"]

    def run(guess, weights):
        s, _, _ = bench.make_batched(G, 256, 100, 80, np_lo=5000, np_hi=20000)
        if weights is not None:
            s.mlp_set_weights(weights, norm)
        s.step_strict(80, guess)
        ds = [s.diag(g) for g in range(G)]
        s.close()
        assert all(d["newton_converged"] for d in ds)
        return (sum(d["newton_total"] for d in ds) / sum(d["newton_levels"] for d in ds),
                sum(d["newton_fallbacks"] for d in ds))

    plain, _ = run(gs.GUESS_EXTRAP, None)
    net, fb = run(gs.GUESS_MLP, theta)
    print(f"Newton updates per level: plain {plain:.4f}, trained network {net:.4f} "
          f"(fallbacks to the extrapolation: {fb} of {G * 80} levels)")
    assert net <= plain + 0.02
