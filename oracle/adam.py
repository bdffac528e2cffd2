"""Plain FP64 oracle of the optimiser step over the Gaussian parameters (GSFusion Sec. III-B-3).

TEST INFRASTRUCTURE ONLY: the product library never imports or calls anything here.
It shares no code with the HIP path.

The paper optimises the Gaussian parameters directly by gradient descent on the loss of
Eq. 12, with every gradient derived explicitly, but does not name the optimiser.  The
reading taken here is the one of the 3D Gaussian splatting method whose tile rasterizer
the paper adopts: Adam (Kingma and Ba, 2015, Algorithm 1), per element x with gradient g
at step t = 1, 2, ...

    m <- beta1 m + (1 - beta1) g
    v <- beta2 v + (1 - beta2) g^2
    x <- x - lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps)

Readings where the paper is silent (each is a setting or stated here):

* the optimised variables are the means, the logarithms of the scales, the (unnormalised)
  quaternions, the logits of the opacities and the SH coefficients; the parameters are
  stored activated (scale s = exp(u), opacity o = 1 / (1 + exp(-w))), so a step maps
  the stored value to its variable (u = log s, w = log(o / (1 - o))), takes the
  gradient through the activation (dL/du = s dL/ds, dL/dw = o (1 - o) dL/do), updates
  the variable and stores the activated result;
* the opacity is kept in [2^-24, 1 - 2^-24] after the step, so that its logit stays
  finite in binary32;
* learning rates per group (the 3D Gaussian splatting defaults): means 1.6e-4,
  log-scales 5e-3, quaternions 1e-3, opacity logits 0.05, SH DC coefficients 2.5e-3
  and the other SH coefficients 2.5e-3 / 20; beta1 0.9, beta2 0.999, eps 1e-15;
* every row is updated at every step (dense Adam: an element whose gradient is zero
  still moves by its momentum).
"""
from __future__ import annotations

import math

import numpy as np

GROUPS = ("means", "scales", "quats", "opacities", "sh")
OPACITY_MIN = 2.0 ** -24
OPACITY_MAX = 1.0 - 2.0 ** -24

DEFAULTS = dict(lr_means=1.6e-4, lr_scales=5e-3, lr_quats=1e-3, lr_opacities=0.05, lr_sh_dc=2.5e-3,
                lr_sh_rest=2.5e-3 / 20, beta1=0.9, beta2=0.999, eps=1e-15)


def adam_update(x, g, m, v, t, lr, beta1, beta2, eps):
    """Algorithm 1 of Kingma and Ba for one step t >= 1; lr may be an array broadcast
    against x.  Returns (x, m, v) as new float64 arrays."""
    x, g, m, v = (np.asarray(a, np.float64) for a in (x, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return x - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def _sh_rates(shape, lr_dc, lr_rest):
    """Learning rate of every SH coefficient [n, K, 3]: the DC row (k = 0) and the rest."""
    lr = np.full(shape, float(lr_rest))
    lr[:, 0, :] = lr_dc
    return lr


def step(params: dict, grads: dict, m: dict, v: dict, t: int, hp: dict | None = None):
    """One Adam step of every group at step number t (>= 1).

    params: activated parameters (means [n,3], scales [n,3], quats [n,4], opacities [n],
    sh [n,K,3]); grads: dL/d(params) in the same layouts; m, v: the moments of the
    optimised variables, same layouts.  Returns (params, m, v) as new float64 dicts."""
    hp = dict(DEFAULTS, **(hp or {}))
    b1, b2, eps = hp["beta1"], hp["beta2"], hp["eps"]
    out_p, out_m, out_v = {}, {}, {}
    for name in GROUPS:
        p = np.asarray(params[name], np.float64)
        g = np.asarray(grads[name], np.float64)
        if name == "scales":
            var, gvar, lr = np.log(p), g * p, hp["lr_scales"]
        elif name == "opacities":
            var, gvar, lr = np.log(p / (1.0 - p)), g * p * (1.0 - p), hp["lr_opacities"]
        elif name == "sh":
            var, gvar, lr = p, g, _sh_rates(p.shape, hp["lr_sh_dc"], hp["lr_sh_rest"])
        else:
            var, gvar, lr = p, g, hp["lr_" + name]
        nv, out_m[name], out_v[name] = adam_update(var, gvar, m[name], v[name], t, lr, b1, b2, eps)
        if name == "scales":
            nv = np.exp(nv)
        elif name == "opacities":
            nv = np.clip(1.0 / (1.0 + np.exp(-nv)), OPACITY_MIN, OPACITY_MAX)
        out_p[name] = nv
    return out_p, out_m, out_v


def zeros_like(params: dict) -> dict:
    return {k: np.zeros(np.shape(params[k])) for k in GROUPS}


def bias_corrections(t: int, beta1: float, beta2: float):
    """(1 - beta1^t, 1 - beta2^t)."""
    return 1.0 - math.pow(beta1, t), 1.0 - math.pow(beta2, t)
