"""FP64 oracle of the learned star-formation closure (test infrastructure only: only tests,
the smoke check and the benchmark's CPU baseline use this package).

The paper proposes learned sub-grid models trained by differentiating through the simulator
(Sec. 4, the discussion of machine-learned refinements and neural sub-grid models).  Here a
small multilayer perceptron stands in for the deterministic part of the per-cell source update
of Sec. 2.4.  With the paper's physics (no cooling term) that part is the star-formation
probability of the relaxed model,

    pi0 = (1 - exp(-(eps_sf / t_ff) dt)) * s(y1) * s(y2),
    y1 = (Delta - Delta_c) / (w_rho Delta_c),   y2 = (T_c - T) / (w_T T_c),

and the network predicts its two factors that do not depend on the step length:

    o0 = ln(eps_sf / t_ff)                      the log star-formation rate per unit time,
    o1 = max(ln s(y1) + ln s(y2), -30)          the log threshold gate, clipped where nil,

so that pi0 = (1 - exp(-exp(o0) dt)) exp(min(o1, 0)).  The stochastic draw, the supernova
energy and the star field stay those of the plain source term.

Network: inputs x = ((ln Delta - 4.6) / 5, (ln T - 10.4) / 5, (ln a + 3) / 1.5,
eps_sf / 0.02 - 1, Delta_c / 100 - 1), centred on the default thresholds so that bfloat16
inputs resolve the gates finely; three hidden layers of 64 with SiLU; a linear output layer
whose result is multiplied by 10.  Parameters form one flat vector in the order W1[64][5], b1[64], W2[64][64],
b2[64], W3[64][64], b3[64], W4[2][64], b4[2] (8834 values, W[out][in]).

Training objective: the mean over samples of the summed squared output errors,
sum_k (o_k - t_k)^2, with t the targets above.
"""

import math

import numpy as np
import torch

from . import subgrid

N_IN, N_HID, N_OUT = 5, 64, 2
SHAPES = [(N_HID, N_IN), (N_HID,), (N_HID, N_HID), (N_HID,), (N_HID, N_HID), (N_HID,),
          (N_OUT, N_HID), (N_OUT,)]
FAN_IN = [N_IN, N_IN, N_HID, N_HID, N_HID, N_HID, N_HID, N_HID]
N_PARAMS = sum(int(np.prod(s)) for s in SHAPES)
OUT_SCALE = 10.0
GATE_CLIP = -30.0


def unpack(theta):
    """Split the flat parameter vector into the eight weight and bias tensors."""
    out, k = [], 0
    for s in SHAPES:
        m = int(np.prod(s))
        out.append(theta[k:k + m].reshape(s))
        k += m
    return out


def silu(z):
    return z * torch.sigmoid(z)


def _to_bf16(t):
    return t.detach().to(torch.bfloat16).to(torch.float64)


class _Bf16Round(torch.autograd.Function):
    """Rounding to bfloat16 whose backward passes the gradient unchanged (a cast's own
    backward would round the gradient too)."""

    @staticmethod
    def forward(ctx, t):
        return _to_bf16(t)

    @staticmethod
    def backward(ctx, g):
        return g


def bf16_round(t):
    """Round to the nearest bfloat16 value (ties to even), returned in float64.  Autograd
    passes gradients through the rounding unchanged."""
    return _Bf16Round.apply(t) if t.requires_grad else _to_bf16(t)


class _RoundGrad(torch.autograd.Function):
    """Identity whose backward rounds the incoming gradient to bfloat16."""

    @staticmethod
    def forward(ctx, t):
        return t.view_as(t)

    @staticmethod
    def backward(ctx, g):
        return _to_bf16(g)


class _SiluBf16Grad(torch.autograd.Function):
    """SiLU whose backward multiplies by the derivative rounded to bfloat16."""

    @staticmethod
    def forward(ctx, z):
        ctx.save_for_backward(z)
        return silu(z)

    @staticmethod
    def backward(ctx, g):
        z, = ctx.saved_tensors
        s = torch.sigmoid(z)
        return g * _to_bf16(s * (1.0 + z * (1.0 - s)))


def forward(theta, x, bf16=False):
    """Network outputs [2, ...] for inputs x [5, ...].

    With bf16, the arithmetic is that of a matrix-core evaluation: every operand of the four
    matrix products is rounded to bfloat16 (weights, inputs, hidden activations), and so are
    the operands of the products of the backward pass (the gradient with respect to each
    layer's pre-activation, the SiLU derivative it is formed with, and the gradient of the
    output layer's sum); sums, biases and activations stay in float64."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(theta)
    shape = x.shape[1:]
    if not bf16:
        h = x.reshape(N_IN, -1)
        for W, b in ((W1, b1), (W2, b2), (W3, b3)):
            h = silu(W @ h + b[:, None])
        o = OUT_SCALE * (W4 @ h + b4[:, None])
        return o.reshape((N_OUT,) + shape)
    r = bf16_round
    h = r(x.reshape(N_IN, -1))
    for W, b in ((W1, b1), (W2, b2), (W3, b3)):
        h = r(_SiluBf16Grad.apply(_RoundGrad.apply(r(W) @ h + b[:, None])))
    o = OUT_SCALE * _RoundGrad.apply(r(W4) @ h + b4[:, None])
    return o.reshape((N_OUT,) + shape)


def features(delta, temp, a, eps_sf, delta_c):
    """Normalised network inputs from gas overdensity, temperature [K], scale factor and the
    two star-formation parameters (scalars or tensors broadcastable to delta)."""
    z = torch.zeros_like(delta)
    return torch.stack([(torch.log(delta) - 4.6) / 5.0, (torch.log(temp) - 10.4) / 5.0,
                        (torch.log(torch.as_tensor(a, dtype=delta.dtype)) + 3.0) / 1.5 + z,
                        torch.as_tensor(eps_sf, dtype=delta.dtype) / 0.02 - 1.0 + z,
                        torch.as_tensor(delta_c, dtype=delta.dtype) / 100.0 - 1.0 + z])


def decode_features(x):
    """Inverse of features: (Delta, T, a, eps_sf, Delta_c)."""
    return (torch.exp(5.0 * x[0] + 4.6), torch.exp(5.0 * x[1] + 10.4),
            torch.exp(1.5 * x[2] - 3.0), 0.02 * (x[3] + 1.0), 100.0 * (x[4] + 1.0))


def targets(delta, temp, a, eps_sf, delta_c, *, omega_b, t_c, w_rho, w_t):
    """The two factors of pi0 of the plain relaxed source term (module docstring)."""
    tff = subgrid.free_fall_time(delta, a, omega_b)
    o0 = torch.log(eps_sf / tff)
    y1 = (delta - delta_c) / (w_rho * delta_c)
    y2 = (t_c - temp) / (w_t * t_c)
    o1 = torch.clamp(torch.nn.functional.logsigmoid(y1) + torch.nn.functional.logsigmoid(y2),
                     min=GATE_CLIP)
    return torch.stack([o0, o1])


def probability(o, dt):
    """pi0 from the two outputs and the step length."""
    return -torch.expm1(-torch.exp(o[0]) * dt) * torch.exp(torch.clamp(o[1], max=0.0))


def loss(theta, x, t, bf16=False):
    """Training objective: mean over samples of sum_k (o_k - t_k)^2."""
    o = forward(theta, x, bf16=bf16)
    return ((o - t) ** 2).sum(0).mean()


def closure_inputs(q, a, *, rho_mean_gas, gamma, e_floor, t_per_e, eps_sf, delta_c):
    """Network inputs of every cell of the gas state q (5, ...)."""
    delta = q[0] / rho_mean_gas
    temp = subgrid.temperature(q, a, gamma, e_floor, t_per_e)
    return features(delta, temp, a, eps_sf, delta_c)


def apply_with_outputs(q, star, a, dt, u, o, *, e0_code, tau, mode, with_draw=False,
                       smooth=False, gamma=None):
    """Source update of Sec. 2.4 with pi0 taken from network outputs o (returns Q, star, and
    the draw z with_draw); smooth: the supernova energy spread as subgrid.smooth_injection.
    A six-component (dual-energy) state also takes the injected energy into its entropy, as
    the plain source term does (subgrid.apply_source)."""
    pi0 = probability(o, dt)
    z = subgrid.draw(pi0, u, tau, mode)
    inj = a * a * q[0] * z * e0_code
    add = subgrid.smooth_injection(inj) if smooth else inj
    extra = [q[5] + add * q[0] ** (1.0 - gamma)] if q.shape[0] > 5 else []
    out = (torch.stack([q[0], q[1], q[2], q[3], q[4] + add] + extra), star + z)
    return out + (z,) if with_draw else out


def apply_closure(q, star, a, dt, u, theta, *, rho_mean_gas, gamma, e_floor, t_per_e, e0_code,
                  eps_sf, delta_c, tau, mode=subgrid.MODE_RELAXED, bf16=False, with_draw=False,
                  smooth=False):
    """The source term with pi0 from the network (returns Q, star, and z with_draw)."""
    x = closure_inputs(q, a, rho_mean_gas=rho_mean_gas, gamma=gamma, e_floor=e_floor,
                       t_per_e=t_per_e, eps_sf=eps_sf, delta_c=delta_c)
    o = forward(theta, x, bf16=bf16)
    return apply_with_outputs(q, star, a, dt, u, o, e0_code=e0_code, tau=tau, mode=mode,
                              with_draw=with_draw, smooth=smooth, gamma=gamma)


def init_params(seed):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) parameters, float64."""
    rng = np.random.default_rng(seed)
    parts = []
    for s, f in zip(SHAPES, FAN_IN):
        bound = 1.0 / math.sqrt(f)
        parts.append(rng.uniform(-bound, bound, size=int(np.prod(s))))
    return np.concatenate(parts)
