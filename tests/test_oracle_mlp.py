"""Pins of the oracle's guess network (oracle/mlp.c) against things other than itself.

- GELU and its derivative against torch's exact-form GELU and autograd (float64,
  CPU), and against finite differences;
- the forward pass and the gradient of the mean squared error against the same
  network built from torch.nn layers and differentiated by torch autograd;
- the gradient against central differences of the oracle's own loss;
- Adam against torch.optim.Adam over several steps;
- bfloat16 rounding against torch's float32 -> bfloat16 conversion, ties and
  special values included.
torch runs on the CPU here, as an independent library reference only.
"""
import numpy as np
import torch

import oracle

rng = np.random.default_rng(1234)


def _torch_net(theta):
    """The 48-128-128-128-3 GELU network as torch layers, loaded from theta."""
    layers = []
    dims = [(48, 128), (128, 128), (128, 128), (128, 3)]
    for k, (ni, no) in enumerate(dims):
        lin = torch.nn.Linear(ni, no, dtype=torch.float64)
        layers.append(lin)
        if k < 3:
            layers.append(torch.nn.GELU(approximate="none"))
    net = torch.nn.Sequential(*layers)
    lay = {n: (o, s) for n, o, s in oracle.MLP_LAYOUT}
    with torch.no_grad():
        for k in range(4):
            o, s = lay[f"W{k + 1}"]
            net[2 * k].weight.copy_(torch.from_numpy(theta[o:o + int(np.prod(s))].reshape(s)))
            o, s = lay[f"b{k + 1}"]
            net[2 * k].bias.copy_(torch.from_numpy(theta[o:o + s[0]]))
    return net


def _flat_grad(net):
    parts = []
    for k in range(4):
        parts.append(net[2 * k].weight.grad.numpy().ravel())
        parts.append(net[2 * k].bias.grad.numpy().ravel())
    return np.concatenate(parts)


def _theta(scale=0.15):
    return rng.normal(0.0, scale, oracle.MLP_NPARAM)


def test_layout_size():
    sizes = {n: int(np.prod(s)) for n, _, s in oracle.MLP_LAYOUT}
    assert sum(sizes.values()) == oracle.MLP_NPARAM == 39683


def test_gelu_against_torch_and_differences():
    z = np.concatenate([np.linspace(-8, 8, 161), rng.normal(0, 3, 200)])
    zt = torch.tensor(z, dtype=torch.float64, requires_grad=True)
    gt = torch.nn.functional.gelu(zt, approximate="none")
    gt.sum().backward()
    g = np.array([oracle.gelu(v) for v in z])
    dg = np.array([oracle.gelu_grad(v) for v in z])
    np.testing.assert_allclose(g, gt.detach().numpy(), rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(dg, zt.grad.numpy(), rtol=1e-13, atol=1e-14)
    h = 1e-5
    fd = np.array([(oracle.gelu(v + h) - oracle.gelu(v - h)) / (2 * h) for v in z])
    np.testing.assert_allclose(dg, fd, rtol=1e-8, atol=1e-9)
    # special values: GELU(0) = 0, GELU'(0) = 1/2, GELU(z) -> z and -> 0 in the tails
    assert oracle.gelu(0.0) == 0.0 and oracle.gelu_grad(0.0) == 0.5
    assert abs(oracle.gelu(10.0) - 10.0) < 1e-20 and abs(oracle.gelu(-10.0)) < 1e-20


def test_forward_and_gradient_against_torch_autograd():
    theta = _theta()
    x = rng.normal(0, 1, (37, 48))
    t = rng.normal(0, 1, (37, 3))
    net = _torch_net(theta)
    xt = torch.from_numpy(x)
    y_t = net(xt)
    np.testing.assert_allclose(oracle.mlp_forward(theta, x), y_t.detach().numpy(), rtol=1e-12, atol=1e-13)
    loss_t = torch.mean((y_t - torch.from_numpy(t)) ** 2)
    loss_t.backward()
    loss, g = oracle.mlp_loss_grad(theta, x, t)
    assert abs(loss - loss_t.item()) <= 1e-13 * loss_t.item()
    gt = _flat_grad(net)
    assert np.abs(g - gt).max() <= 1e-12 * np.abs(gt).max()


def test_gradient_against_central_differences():
    theta = _theta()
    x = rng.normal(0, 1, (9, 48))
    t = rng.normal(0, 1, (9, 3))
    _, g = oracle.mlp_loss_grad(theta, x, t)
    # components from every parameter block
    idx = []
    for _, o, s in oracle.MLP_LAYOUT:
        n = int(np.prod(s))
        idx += list(o + rng.choice(n, size=min(n, 6), replace=False))

    def central(i, h):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        return (oracle.mlp_loss_grad(tp, x, t)[0] - oracle.mlp_loss_grad(tm, x, t)[0]) / (2 * h)

    for i in idx:
        # Richardson-extrapolated central differences: truncation O(h^4), so a
        # step large enough to keep rounding near 1e-13 is still exact enough
        h = 1e-3
        fd = (4.0 * central(i, h / 2) - central(i, h)) / 3.0
        assert abs(g[i] - fd) <= 1e-7 * max(abs(fd), 1e-3 * np.abs(g).max()), (i, g[i], fd)


def test_output_bias_only_network():
    """Closed form: with every weight zero the output is b4; the loss gradient
    is 2 (b4 - mean t) / 3 on b4 and zero on every other parameter (all
    outgoing weights are zero and GELU(0) = 0)."""
    theta = np.zeros(oracle.MLP_NPARAM)
    lay = {n: (o, s) for n, o, s in oracle.MLP_LAYOUT}
    ob4 = lay["b4"][0]
    theta[ob4:ob4 + 3] = [0.5, -1.0, 2.0]
    x = rng.normal(0, 1, (11, 48))
    t = rng.normal(0, 1, (11, 3))
    y = oracle.mlp_forward(theta, x)
    np.testing.assert_array_equal(y, np.tile([0.5, -1.0, 2.0], (11, 1)))
    loss, g = oracle.mlp_loss_grad(theta, x, t)
    np.testing.assert_allclose(g[ob4:ob4 + 3], 2.0 * (np.array([0.5, -1.0, 2.0]) - t.mean(0)) / 3.0,
                               rtol=1e-14)
    assert np.all(g[:ob4] == 0.0)


def test_adam_against_torch():
    n = 1000
    theta0 = rng.normal(0, 1, n)
    grads = [rng.normal(0, 1, n) * 10.0 ** rng.uniform(-3, 1, n) for _ in range(6)]
    lr, b1, b2, eps = 3e-3, 0.9, 0.999, 1e-8
    th = theta0.copy()
    m = np.zeros(n)
    v = np.zeros(n)
    for k, g in enumerate(grads):
        oracle.adam_step(th, m, v, k + 1, g, lr, b1, b2, eps)
    p = torch.nn.Parameter(torch.from_numpy(theta0.copy()))
    opt = torch.optim.Adam([p], lr=lr, betas=(b1, b2), eps=eps)
    for g in grads:
        p.grad = torch.from_numpy(g.copy())
        opt.step()
    np.testing.assert_allclose(th, p.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_bf16_rounding_against_torch():
    vals = np.concatenate([
        rng.normal(0, 1, 5000).astype(np.float32),
        (rng.normal(0, 1, 2000) * 10.0 ** rng.uniform(-30, 30, 2000)).astype(np.float32),
        # exact ties (bit 15 set, lower bits clear) with even and odd bfloat16 mantissas
        np.array([1.00390625, 1.01171875, -1.00390625, -1.01171875, 3.0, 0.0, -0.0,
                  np.float32(3.4e38), np.float32(1e-40), np.inf, -np.inf], dtype=np.float32),
    ])
    got = oracle.round_bf16(vals)
    ref = torch.from_numpy(vals).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(got.view(np.uint32), ref.view(np.uint32))
    assert np.isnan(oracle.round_bf16(np.array([np.nan], dtype=np.float32))[0])
