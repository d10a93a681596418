"""Arithmetic on encrypted Z_t values built from the bootstrap and affine
maps (Sec. "Application of Functional Bootstrapping"):

* ``maximum(x, y) = max(x - y, 0) + y``: one bootstrap per pair;
* ``multiply(x, y) = q(x + y) - q(x - y)`` with ``q(s) = floor(s^2 / 4)``
  taken on the integer lift of s: exact, since x + y and x - y have the
  same parity.  Two bootstraps per pair, issued as one batch.

Every step runs in the library's kernels (``fdfb_lincomb2``,
``fdfb_bootstrap_batch``); this module only picks the weights and builds
the tables.  Both need x, y in [0, t/2) (t = 2^log2_t): then x - y is read
correctly as a two's-complement value of Z_t and x + y < t; the product is
returned mod t.  The Chinese-remainder plaintext extension of the same
section needs pairwise coprime moduli t_i, so all but one would be odd; an
odd t_i does not divide q = 2^32, so Delta t_i is not 0 mod q and the public
mux could no longer decompose (p_B - p_A) mod t_i alone: it would need the
full-width digits of Delta (p_B - p_A), ceil(32 / log2 L_boot) sign
rotations instead of ceil(log2 t / log2 L_boot).
"""
from __future__ import annotations

import numpy as np

from . import lincomb2


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

    def _lin(self, x, y, wx: int, wy: int):
        out = self._torch.empty_like(x)
        return lincomb2(x, y, wx, wy, out)

    def maximum(self, x, y):
        torch = self._torch
        B = int(x.shape[0])
        d = self._lin(x, y, 1, -1)  # x - y
        r = torch.empty_like(d)
        self.ctx.bootstrap_batch(d, torch.full((B,), self.relu, dtype=torch.int32, device=x.device), r)
        return self._lin(r, y, 1, 1)  # relu(x - y) + y

    def multiply(self, x, y):
        torch = self._torch
        B = int(x.shape[0])
        sd = torch.cat([self._lin(x, y, 1, 1), self._lin(x, y, 1, -1)])  # [x + y; x - y]
        ids = torch.cat([torch.full((B,), self.qs, dtype=torch.int32, device=x.device),
                         torch.full((B,), self.qd, dtype=torch.int32, device=x.device)])
        q = torch.empty_like(sd)
        self.ctx.bootstrap_batch(sd, ids, q)
        return self._lin(q[:B], q[B:], 1, -1)  # q(x + y) - q(x - y)
