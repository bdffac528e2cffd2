"""Pins of the optimiser oracle (oracle/adam.py) against facts that do not come from it:
torch.optim.Adam (an independent implementation of the same algorithm) on the raw
variables and, through autograd, on the log-scale / logit-opacity variables; closed forms
of Adam under a constant gradient; special cases (zero gradient, the opacity bound)."""
import math

import numpy as np
import pytest
import torch

from oracle import adam as A


def _params(rng, n, K):
    return dict(means=rng.standard_normal((n, 3)), scales=np.exp(rng.uniform(-5, -1, (n, 3))),
                quats=rng.standard_normal((n, 4)), opacities=rng.uniform(0.05, 0.95, n),
                sh=rng.standard_normal((n, K, 3)) * 0.3)


def test_raw_groups_match_torch_adam():
    rng = np.random.default_rng(0)
    n, K, T = 37, 16, 6
    p = _params(rng, n, K)
    hp = dict(A.DEFAULTS, eps=1e-8)
    m, v = A.zeros_like(p), A.zeros_like(p)
    tm = torch.tensor(p["means"], requires_grad=True)
    tq = torch.tensor(p["quats"], requires_grad=True)
    tdc = torch.tensor(p["sh"][:, :1], requires_grad=True)
    trest = torch.tensor(p["sh"][:, 1:], requires_grad=True)
    opt = torch.optim.Adam([dict(params=[tm], lr=hp["lr_means"]), dict(params=[tq], lr=hp["lr_quats"]),
                            dict(params=[tdc], lr=hp["lr_sh_dc"]), dict(params=[trest], lr=hp["lr_sh_rest"])],
                           betas=(hp["beta1"], hp["beta2"]), eps=hp["eps"])
    for t in range(1, T + 1):
        g = {k: rng.standard_normal(np.shape(p[k])) * 10.0 ** rng.uniform(-6, 0) for k in A.GROUPS}
        g["means"][3] = 0.0                     # a row without gradient keeps its momentum
        p, m, v = A.step(p, g, m, v, t, hp)
        tm.grad, tq.grad = torch.tensor(g["means"]), torch.tensor(g["quats"])
        tdc.grad, trest.grad = torch.tensor(g["sh"][:, :1]), torch.tensor(g["sh"][:, 1:])
        opt.step()
        np.testing.assert_allclose(p["means"], tm.detach().numpy(), rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(p["quats"], tq.detach().numpy(), rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(p["sh"][:, :1], tdc.detach().numpy(), rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(p["sh"][:, 1:], trest.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_activated_groups_match_torch_autograd_adam():
    # torch optimises the variables u = log s and w = logit o of a loss written on the
    # activated values; the oracle receives dL/ds and dL/do and must follow the same path
    rng = np.random.default_rng(1)
    n, T = 29, 8
    p = _params(rng, n, 1)
    hp = dict(A.DEFAULTS)
    s_star, o_star = np.exp(rng.uniform(-5, -1, (n, 3))), rng.uniform(0.05, 0.95, n)
    u = torch.tensor(np.log(p["scales"]), requires_grad=True)
    w = torch.tensor(np.log(p["opacities"] / (1 - p["opacities"])), requires_grad=True)
    opt = torch.optim.Adam([dict(params=[u], lr=hp["lr_scales"]), dict(params=[w], lr=hp["lr_opacities"])],
                           betas=(hp["beta1"], hp["beta2"]), eps=hp["eps"])
    m, v = A.zeros_like(p), A.zeros_like(p)
    for t in range(1, T + 1):
        # loss on the activated values; its gradient with respect to them for the oracle
        s_t = torch.tensor(p["scales"], requires_grad=True)
        o_t = torch.tensor(p["opacities"], requires_grad=True)
        L = ((s_t - torch.tensor(s_star)) ** 2 * 1e3).sum() + ((o_t - torch.tensor(o_star)) ** 3).sum()
        L.backward()
        g = {k: np.zeros(np.shape(p[k])) for k in A.GROUPS}
        g["scales"], g["opacities"] = s_t.grad.numpy(), o_t.grad.numpy()
        p, m, v = A.step(p, g, m, v, t, hp)
        opt.zero_grad()
        Lu = ((torch.exp(u) - torch.tensor(s_star)) ** 2 * 1e3).sum() + ((torch.sigmoid(w) - torch.tensor(o_star)) ** 3).sum()
        Lu.backward()
        opt.step()
        np.testing.assert_allclose(p["scales"], torch.exp(u).detach().numpy(), rtol=1e-10)
        np.testing.assert_allclose(p["opacities"], torch.sigmoid(w).detach().numpy(), rtol=1e-10)


def test_constant_gradient_closed_form():
    # with a constant gradient the bias-corrected moments are exactly g and g^2, so every
    # step moves x by lr * g / (|g| + eps)
    g = np.array([3.0, -1e-3, 2.5e-7, 0.0])
    x0 = np.array([1.0, -2.0, 0.5, 4.0])
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-15
    x, m, v = x0, np.zeros(4), np.zeros(4)
    for t in range(1, 41):
        x, m, v = A.adam_update(x, g, m, v, t, lr, b1, b2, eps)
        np.testing.assert_allclose(m, (1 - b1 ** t) * g, rtol=1e-13, atol=0)
        np.testing.assert_allclose(v, (1 - b2 ** t) * g * g, rtol=1e-13, atol=0)
    np.testing.assert_allclose(x, x0 - 40 * lr * g / (np.abs(g) + eps), rtol=1e-13, atol=1e-15)


def test_zero_gradient_and_momentum():
    x, m, v = A.adam_update([1.0], [0.0], [0.0], [0.0], 1, 0.1, 0.9, 0.999, 1e-15)
    assert x[0] == 1.0 and m[0] == 0.0 and v[0] == 0.0
    # after one step with gradient g, a zero gradient decays the moments geometrically and
    # x keeps moving: m2 = 0.9 * 0.1 g, v2 = 0.999 * 0.001 g^2
    g = 2.0
    x1, m1, v1 = A.adam_update([0.0], [g], [0.0], [0.0], 1, 0.1, 0.9, 0.999, 0.0)
    x2, m2, v2 = A.adam_update(x1, [0.0], m1, v1, 2, 0.1, 0.9, 0.999, 0.0)
    assert m2[0] == pytest.approx(0.09 * g, rel=1e-15) and v2[0] == pytest.approx(0.999e-3 * g * g, rel=1e-15)
    step2 = 0.1 * (m2[0] / (1 - 0.81)) / math.sqrt(v2[0] / (1 - 0.999 ** 2))
    assert x2[0] == pytest.approx(x1[0] - step2, rel=1e-14)


def test_first_step_moves_each_variable_by_its_rate():
    # step 1: x1 = x0 - lr sign(g) (|g| >> eps); DC and higher SH coefficients use their rates
    rng = np.random.default_rng(2)
    n, K = 11, 9
    p = _params(rng, n, K)
    g = {k: rng.choice([-1.0, 1.0], np.shape(p[k])) * rng.uniform(1e-3, 1, np.shape(p[k])) for k in A.GROUPS}
    q, _, _ = A.step(p, g, A.zeros_like(p), A.zeros_like(p), 1)
    d = A.DEFAULTS
    np.testing.assert_allclose(q["means"], p["means"] - d["lr_means"] * np.sign(g["means"]), rtol=1e-12)
    np.testing.assert_allclose(q["quats"], p["quats"] - d["lr_quats"] * np.sign(g["quats"]), rtol=1e-12)
    np.testing.assert_allclose(q["sh"][:, 0], p["sh"][:, 0] - d["lr_sh_dc"] * np.sign(g["sh"][:, 0]), rtol=1e-12)
    np.testing.assert_allclose(q["sh"][:, 1:], p["sh"][:, 1:] - d["lr_sh_rest"] * np.sign(g["sh"][:, 1:]),
                               rtol=1e-12)
    # log-scale: s1 = s0 exp(-lr sign(g)) since dL/du = s dL/ds has the sign of dL/ds
    np.testing.assert_allclose(q["scales"], p["scales"] * np.exp(-d["lr_scales"] * np.sign(g["scales"])),
                               rtol=1e-12)
    w0 = np.log(p["opacities"] / (1 - p["opacities"]))
    np.testing.assert_allclose(q["opacities"], 1 / (1 + np.exp(-(w0 - d["lr_opacities"] * np.sign(g["opacities"])))),
                               rtol=1e-12)


def test_opacity_stays_inside_its_bounds():
    p = dict(means=np.zeros((3, 3)), scales=np.ones((3, 3)), quats=np.ones((3, 4)),
             opacities=np.array([1 - 2.0 ** -24, 2.0 ** -24, 0.5]), sh=np.zeros((3, 1, 3)))
    g = {k: np.zeros(np.shape(p[k])) for k in A.GROUPS}
    g["opacities"] = np.array([-1.0, 1.0, 0.0])       # push towards 1 and towards 0
    q, _, _ = A.step(p, g, A.zeros_like(p), A.zeros_like(p), 1, dict(lr_opacities=50.0))
    assert q["opacities"][0] == A.OPACITY_MAX and q["opacities"][1] == A.OPACITY_MIN
    assert q["opacities"][2] == 0.5
    assert np.isfinite(np.log(q["opacities"] / (1 - q["opacities"]))).all()
