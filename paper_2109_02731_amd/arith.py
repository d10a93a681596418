"""Arithmetic on encrypted values built from the bootstrap and affine maps
(Sec. "Application of Functional Bootstrapping"):

* ``maximum(x, y) = max(x - y, 0) + y``: one bootstrap per pair;
* ``multiply(x, y) = q(x + y) - q(x - y)`` with ``q(s) = floor(s^2 / 4)``
  taken on the integer lift of s: exact, since x + y and x - y have the
  same parity.  Two bootstraps per pair, issued as one batch.

Both need x, y in [0, t/2) (t = 2^log2_t): then x - y is read correctly as
a two's-complement value of Z_t and x + y < t; the product is returned mod t.

* ``CRT``: the Chinese-remainder extension of the same section.  A value X
  of Z_M, M = m_1 ... m_k with pairwise coprime moduli, is held as one
  sample per residue x_i = X mod m_i.  The plaintext spaces of this
  library are Z_t with t a power of two (t | q = 2^32, so Delta t = 0 mod
  q), so an odd m_i cannot be a plaintext modulus of its own.  Each residue
  instead lives in Z_t with m_i <= t/2, and every operation ends with a
  bootstrap whose table reduces its result mod m_i.  Sums and differences
  of two residues stay inside (-m_i, 2 m_i) and are read exactly; the product
  of two residues is the quarter-square difference above, reduced by one
  more bootstrap.  Addition, subtraction and multiplication therefore take
  1, 1 and 3 bootstraps per residue, all residues of a batch in one call
  with a table per sample.

Every step runs in the library's kernels (``fdfb_lincomb2``,
``fdfb_bootstrap_batch``); this module only picks the weights and builds
the tables.
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


# ---------------------------------------------------------------------------
# Chinese-remainder representation
# ---------------------------------------------------------------------------
def mod_table(t: int, m: int, signed: bool) -> np.ndarray:
    """v mod m for v in Z_t, v read as a two's-complement value when signed."""
    v = np.arange(t, dtype=np.int64)
    if signed:
        v = np.where(v < t // 2, v, v - t)
    return (v % m).astype(np.uint32)


def crt_quarter_tables(t: int, m: int):
    """floor(s^2/4) mod m on s in [0, t), and on the signed lift of d in Z_t."""
    s = np.arange(t, dtype=np.int64)
    d = np.where(s < t // 2, s, s - t)
    return ((s * s // 4) % m).astype(np.uint32), ((d * d // 4) % m).astype(np.uint32)


def crt_split(X, moduli) -> np.ndarray:
    """Residues [B][k] of the values X (integers in [0, M))."""
    X = np.asarray(X, dtype=np.int64)
    return np.stack([X % m for m in moduli], axis=-1).astype(np.uint32)


def crt_join(res, moduli) -> np.ndarray:
    """The values in [0, M) with residues res [B][k] (Gauss's formula)."""
    M = int(np.prod(moduli))
    out = np.zeros(np.asarray(res).shape[0], dtype=object)
    for i, m in enumerate(moduli):
        Mi = M // m
        out = out + np.asarray(res)[:, i].astype(object) * Mi * pow(Mi, -1, m)
    return np.array([int(v) % M for v in out], dtype=np.int64)


class CRT:
    """Values of Z_M, M = prod(moduli), as residue samples of one context.

    A batch of B values is a device tensor [B * k][n + 1] of LWE samples,
    value b's residue i at row b k + i.  The moduli must be pairwise
    coprime and at most t/2."""

    def __init__(self, ctx, moduli):
        import math
        import torch
        t = 1 << ctx.params.log2_t
        moduli = [int(m) for m in moduli]
        if not moduli or any(m < 2 or m > t // 2 for m in moduli):
            raise ValueError(f"every modulus must lie in [2, t/2] = [2, {t // 2}]")
        if any(math.gcd(a, b) != 1 for i, a in enumerate(moduli) for b in moduli[i + 1:]):
            raise ValueError("the moduli must be pairwise coprime")
        self.ctx, self.t, self.moduli, self.k = ctx, t, moduli, len(moduli)
        self.M = int(np.prod(moduli))
        self._torch = torch
        reg = ctx.register_lut
        self.red_u = [reg(mod_table(t, m, False)) for m in moduli]
        self.red_s = [reg(mod_table(t, m, True)) for m in moduli]
        qt = [crt_quarter_tables(t, m) for m in moduli]
        self.qs = [reg(a) for a, _ in qt]
        self.qd = [reg(b) for _, b in qt]

    def encrypt_debug(self, X, seed: int = 0):
        """Host samples [B * k][n + 1] of the residues of X."""
        return self.ctx.encrypt_debug(crt_split(X, self.moduli).reshape(-1), seed=seed)

    def decrypt_debug(self, samples) -> np.ndarray:
        """The values of host samples [B * k][n + 1]."""
        m, _ = self.ctx.decrypt_debug(samples)
        return crt_join(np.asarray(m).reshape(-1, self.k), self.moduli)

    def _ids(self, tables, rows: int, device):
        ids = np.tile(np.asarray(tables, dtype=np.int32), rows // self.k)
        return self._torch.from_numpy(ids).to(device)

    def _reduce(self, v, tables):
        out = self._torch.empty_like(v)
        self.ctx.bootstrap_batch(v, self._ids(tables, int(v.shape[0]), v.device), out)
        return out

    def add(self, x, y):
        return self._reduce(lincomb2(x, y, 1, 1, self._torch.empty_like(x)), self.red_u)

    def sub(self, x, y):
        return self._reduce(lincomb2(x, y, 1, -1, self._torch.empty_like(x)), self.red_s)

    def multiply(self, x, y):
        torch = self._torch
        rows = int(x.shape[0])
        sd = torch.cat([lincomb2(x, y, 1, 1, torch.empty_like(x)), lincomb2(x, y, 1, -1, torch.empty_like(x))])
        ids = torch.cat([self._ids(self.qs, rows, x.device), self._ids(self.qd, rows, x.device)])
        q = torch.empty_like(sd)
        self.ctx.bootstrap_batch(sd, ids, q)
        return self._reduce(lincomb2(q[:rows], q[rows:], 1, -1, torch.empty_like(x)), self.red_s)
