"""Arithmetic on encrypted Z_t values built from the bootstrap and affine
maps (Sec. "Application of Functional Bootstrapping"):

* ``maximum(x, y) = max(x - y, 0) + y``: one bootstrap per pair;
* ``multiply(x, y) = q(x + y) - q(x - y)`` with ``q(s) = floor(s^2 / 4)``
  taken on the integer lift of s: exact, since x + y and x - y have the
  same parity.  Two bootstraps per pair, issued as one batch.

Every step runs in the library's kernels (``fdfb_affine``,
``fdfb_bootstrap_batch``); this module only builds the integer weight
matrices and tables.  Both need x, y in [0, t/2) (t = 2^log2_t): then
x - y is read correctly as a two's-complement value of Z_t and x + y < t;
the product is returned mod t.  The Chinese-remainder
plaintext extension the same section describes needs pairwise coprime
moduli, which t | 2^32 excludes at q = 2^32.
"""
from __future__ import annotations

import numpy as np

from . import affine


def _stack_weights(B: int, sign: int):
    """[I | sign*I] as int32 [B][2B]."""
    W = np.zeros((B, 2 * B), np.int32)
    W[np.arange(B), np.arange(B)] = 1
    W[np.arange(B), B + np.arange(B)] = sign
    return W


def relu_table(t: int) -> np.ndarray:
    """max(d, 0) for d in two's-complement Z_t (d >= t/2 is negative)."""
    d = np.arange(t)
    return np.where(d < t // 2, d, 0).astype(np.uint32)


def quarter_square_tables(t: int):
    """q(s) = floor(s^2/4) mod t on s = x + y in [0, t), and on the signed
    lift of d = x - y in [-t/2, t/2) (q is even, so only |d| < t/2 matters)."""
    s = np.arange(t, dtype=np.int64)
    d = np.where(s < t // 2, s, s - t)
    return ((s * s // 4) % t).astype(np.uint32), ((d * d // 4) % t).astype(np.uint32)


class Arith:
    """Registers the tables once per context and evaluates batches of pairs
    (x, y given as device tensors [B][n+1] of LWE samples under s)."""

    def __init__(self, ctx):
        import torch
        self.ctx = ctx
        t = 1 << ctx.params.log2_t
        self.t = t
        self.relu = ctx.register_lut(relu_table(t))
        qs, qd = quarter_square_tables(t)
        self.qs, self.qd = ctx.register_lut(qs), ctx.register_lut(qd)
        self._torch = torch

    def _affine(self, W: np.ndarray, cts):
        torch = self._torch
        out = torch.empty((W.shape[0], cts.shape[1]), dtype=torch.int32, device=cts.device)
        affine(torch.from_numpy(W).to(cts.device), cts, out)
        return out

    def maximum(self, x, y):
        torch = self._torch
        B = int(x.shape[0])
        xy = torch.cat([x, y])
        d = self._affine(_stack_weights(B, -1), xy)  # x - y
        r = torch.empty_like(d)
        self.ctx.bootstrap_batch(d, torch.full((B,), self.relu, dtype=torch.int32, device=x.device), r)
        return self._affine(_stack_weights(B, 1), torch.cat([r, y]))  # relu(x - y) + y

    def multiply(self, x, y):
        torch = self._torch
        B = int(x.shape[0])
        xy = torch.cat([x, y])
        W = np.concatenate([_stack_weights(B, 1), _stack_weights(B, -1)])  # [x + y; x - y]
        sd = self._affine(W, xy)
        ids = torch.cat([torch.full((B,), self.qs, dtype=torch.int32, device=x.device),
                         torch.full((B,), self.qd, dtype=torch.int32, device=x.device)])
        q = torch.empty_like(sd)
        self.ctx.bootstrap_batch(sd, ids, q)
        return self._affine(_stack_weights(B, -1), q)  # q(x + y) - q(x - y)
