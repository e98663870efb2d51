"""FP64 oracle of one learned flow-map jump -- TEST INFRASTRUCTURE.

Only tests/, the smoke check and the bench's CPU-baseline leg may import it.

The learned form (not in the paper: one of the three forms the project adds to
the method) replaces 16 plain RK4 steps of size h by one network evaluation,
guarded by a residual test, with plain RK4 as the fallback:

    d(x)  = network displacement at x                      (mlp.forward)
    Y     = x + d(x)                                       the jumped position
    kind 1 ("one big step"):   r = | Y - Psi_{16h}(x) |_inf
    kind 0 ("commutation"):    r = | (Psi_h(x) + d(Psi_h(x))) - Psi_h(Y) |_inf
            where Psi_s is one classical RK4 step of size s (Sec. 3.1.2's update);
            if Psi_h(x) cannot be taken, x stands in for it
    accept iff r <= tol and Y is finite:  x <- Y, 16 steps counted
    else   16 plain RK4 steps of size h from x (or fewer, if the particle
           terminates on the way: the plain rules of Sec. 3.1.2 apply).
A residual whose own reference step cannot be taken is +inf (rejected).

Kind 0 measures whether the jump commutes with one plain step, which the
exact 16-step map does; so does the identity map, so a network that predicts
no motion at all passes kind 0 (pinned in tests/test_surrogate_oracle.py).
Kind 1 measures the jump against one RK4 step of 16h, whose own truncation
error is part of r.

The network is evaluated in FP64 on the weights and inputs the matrix cores
use: weights rounded to BF16 by the caller, the normalised input and every
hidden activation rounded to BF16 (round to nearest even), biases and sigma
as given -- so that the accept decision is taken at the kernel's precision,
with FP64 arithmetic between those rounding points.
"""
from __future__ import annotations

import numpy as np

from . import ACTIVE, EXIT, MAX_STEPS
from . import mlp as omlp

JUMP = 16


def bf16_weights(params):
    """Network parameters as the matrix cores hold them: W rounded to BF16, b as given."""
    return [(omlp.round_bf16(np.asarray(W, np.float64)), np.asarray(b, np.float64)) for W, b in params]


class Network:
    """d(x) on BF16 weights with BF16 input and hidden activations (FP64 in between)."""

    def __init__(self, params_bf16, sigma, period):
        self.params = params_bf16
        self.sigma = np.asarray(sigma, np.float64)
        self.period = float(period)

    def __call__(self, x):
        x = np.asarray(x, np.float64).reshape(-1, 3)
        xhat = omlp.round_bf16(omlp.normalise(x, self.period))
        out, _ = omlp.forward(self.params, xhat, self.sigma, round_act=omlp.round_bf16)
        return out


def residual(field, net, x, h, kind, eps=0.0, jump=JUMP):
    """Residual r and jumped position Y = x + d(x) for each row of x (FP64)."""
    x = np.asarray(x, np.float64).reshape(-1, 3)
    Y = x + net(x)
    r = np.full(len(x), np.inf)
    if kind == 1:
        ref, st = field.step(x, jump * h, eps=eps)
        ok = st == ACTIVE
        r[ok] = np.abs(Y[ok] - ref[ok]).max(axis=1)
    elif kind == 0:
        xh, st0 = field.step(x, h, eps=eps)
        xh = np.where((st0 == ACTIVE)[:, None], xh, x)
        lhs = xh + net(xh)
        ref, st = field.step(Y, h, eps=eps)
        ok = st == ACTIVE
        r[ok] = np.abs(lhs[ok] - ref[ok]).max(axis=1)
    else:
        raise ValueError("kind must be 0 or 1")
    return r, Y


def jump(field, net, x, h, tol, kind, eps=0.0, jump=JUMP):
    """One jump from each row of x.  Returns dict(residual, accept, next_pos, steps, code):
    the accepted rows move to Y with `jump` steps counted (EXIT if Y leaves the owned
    bounds of a non-periodic block); the rejected ones take up to `jump` plain steps
    (the oracle's trajectory rules, so they may terminate early).  Whether the step
    limit is reached is the caller's business (it knows the step count)."""
    x = np.asarray(x, np.float64).reshape(-1, 3)
    r, Y = residual(field, net, x, h, kind, eps=eps, jump=jump)
    accept = (r <= tol) & np.isfinite(Y).all(axis=1)
    nxt = Y.copy()
    steps = np.full(len(x), jump, np.int32)
    code = np.full(len(x), ACTIVE, np.int32)
    if not field.periodic:  # an accepted jump that leaves the owned bounds is an exit
        lo = np.array(field.b.lo[:], np.float64)
        hi = np.array(field.b.hi[:], np.float64)
        code[accept & ~np.all((Y >= lo) & (Y < hi), axis=1)] = EXIT
    rej = ~accept
    if rej.any():
        tr = field.trace(x[rej], h, jump, eps=eps, keep_verts=False)
        nxt[rej] = tr["final_pos"]
        steps[rej] = tr["steps"]
        # a particle that takes all `jump` steps goes on (the trace stops it at its limit)
        go_on = (tr["code"] == MAX_STEPS) & (tr["steps"] == jump)
        code[rej] = np.where(go_on, ACTIVE, tr["code"])
    return dict(residual=r, accept=accept, next_pos=nxt, steps=steps, code=code)
