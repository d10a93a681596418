"""Seeded synthetic workloads shared by the tests, the smoke check and the benchmark.

This module holds parameter presets and seeded generators of *plaintext-side*
inputs only (messages, lookup tables, weights, arrival times).  It contains
none of the method's arithmetic: no encryption, no decomposition, no ring
products.  Both the GPU library and the CPU oracle take what it produces as
plain inputs.

Parameter sets (q = Q = 2^32 throughout):

* ``C1`` -- tiny plain FDFB: n=64, N=256, gadget base 2^8 ell=2, key switch
  base 2^4 ell=4, noise stddev 2^-20 q (LWE) and 2^-28 q (GLWE), t=8.
* ``C2`` -- the headline batched configuration: n=630, N=1024, gadget base
  2^7 ell=3, key switch base 2^4 ell=5, t=16, same noise as ``C1``.
* ``C3B`` -- the N=2048 half of the uneven batch: n=750, N=2048, t=32,
  gadget base 2^10 ell=2, with noise chosen so that the bootstrap is correct
  at q = 2^32 (no security claim).
* ``C4`` -- parameters for the NN-shaped circuit: n=750, N=2048, t=32,
  gadget base 2^7 ell=4, boot base 2 (ell_boot=5).
* ``C1S`` -- C1's shape with four distinct noise deviations (fresh samples,
  blind-rotation key, packing key, key switching key) and one public-mux
  digit, for the per-stage noise checks.

The packing key (LWE -> RLWE) uses base 2^4 with the key-switch ell, and the
sign decomposition inside the public mux uses base 4 with
ell_boot = ceil(log_4 t) unless stated otherwise (the reading of the
accumulator builder's digit count is recorded in the design notes).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, asdict, replace

import numpy as np


@dataclass(frozen=True)
class Params:
    n: int
    N: int
    log2_t: int
    g_log2B: int
    g_ell: int
    ks_log2B: int
    ks_ell: int
    pk_log2B: int
    pk_ell: int
    boot_log2B: int
    boot_ell: int
    sigma_lwe: float
    sigma_glwe: float
    sigma_pk: float
    sigma_ks: float

    @property
    def t(self) -> int:
        return 1 << self.log2_t

    def as_dict(self) -> dict:
        return asdict(self)

    def with_(self, **kw) -> "Params":
        return replace(self, **kw)


def _boot_ell(log2_t: int, boot_log2B: int) -> int:
    return -(-log2_t // boot_log2B)


_Q = 2.0 ** 32

C1 = Params(n=64, N=256, log2_t=3, g_log2B=8, g_ell=2, ks_log2B=4, ks_ell=4,
            pk_log2B=4, pk_ell=4, boot_log2B=2, boot_ell=_boot_ell(3, 2),
            sigma_lwe=_Q * 2.0 ** -20, sigma_glwe=_Q * 2.0 ** -28,
            sigma_pk=_Q * 2.0 ** -28, sigma_ks=_Q * 2.0 ** -20)

C2 = Params(n=630, N=1024, log2_t=4, g_log2B=7, g_ell=3, ks_log2B=4, ks_ell=5,
            pk_log2B=4, pk_ell=5, boot_log2B=2, boot_ell=_boot_ell(4, 2),
            sigma_lwe=_Q * 2.0 ** -20, sigma_glwe=_Q * 2.0 ** -28,
            sigma_pk=_Q * 2.0 ** -28, sigma_ks=_Q * 2.0 ** -20)

C3B = Params(n=750, N=2048, log2_t=5, g_log2B=10, g_ell=2, ks_log2B=4, ks_ell=5,
             pk_log2B=4, pk_ell=5, boot_log2B=2, boot_ell=_boot_ell(5, 2),
             sigma_lwe=_Q * 2.0 ** -24, sigma_glwe=_Q * 2.0 ** -32,
             sigma_pk=_Q * 2.0 ** -32, sigma_ks=_Q * 2.0 ** -24)

C4 = Params(n=750, N=2048, log2_t=5, g_log2B=7, g_ell=4, ks_log2B=4, ks_ell=5,
            pk_log2B=4, pk_ell=5, boot_log2B=1, boot_ell=5,
            sigma_lwe=_Q * 2.0 ** -24, sigma_glwe=0.25,
            sigma_pk=0.25, sigma_ks=_Q * 2.0 ** -24)

# C1's shape with a different deviation for every key and for fresh samples
# (each a factor of 4 or more from the others), so that the noise of every
# stage can be told apart; one public-mux digit of base 8 (t = 8).
C1S = Params(n=64, N=256, log2_t=3, g_log2B=8, g_ell=2, ks_log2B=4, ks_ell=4,
             pk_log2B=4, pk_ell=4, boot_log2B=3, boot_ell=1,
             sigma_lwe=2.0 ** 16, sigma_glwe=64.0, sigma_pk=1024.0, sigma_ks=4096.0)

PRESETS = {"C1": C1, "C2": C2, "C3B": C3B, "C4": C4}

# Seeds fixed per configuration: key, message, LUT.
KEY_SEED = {"C1": 1001, "C2": 1002, "C3B": 1003, "C4": 1004, "C1S": 1005}
MSG_SEED = {"C1": 2001, "C2": 2002, "C3B": 2003, "C4": 2004, "C1S": 2005}
LUT_SEED = {"C1": 3001, "C2": 3002, "C3B": 3003, "C4": 3004, "C1S": 3005}
ARRIVAL_SEED = 4000


def exact(p: Params) -> Params:
    """Noise-free variant with full-width gadgets (ell * log2B = 32)."""
    return p.with_(sigma_lwe=0.0, sigma_glwe=0.0, sigma_pk=0.0, sigma_ks=0.0,
                   g_log2B=8, g_ell=4, ks_log2B=4, ks_ell=8, pk_log2B=4, pk_ell=8)


def signed_boot(p: Params) -> Params:
    """Variant with one signed public-mux digit in [-t/2, t/2) (encoded as
    boot_log2B = 0, boot_ell = 1): one sign rotation per bootstrap instead of
    ell_boot, at the price of a digit up to t/2 in magnitude."""
    return p.with_(boot_log2B=0, boot_ell=1)


def messages(seed: int, count: int, t: int) -> np.ndarray:
    """Uniform plaintexts in Z_t."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, t, size=count, dtype=np.uint32)


def random_lut(seed: int, t: int) -> np.ndarray:
    """A uniformly random table Z_t -> Z_t."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, t, size=t, dtype=np.uint32)


def named_luts(t: int) -> dict:
    """Non-negacyclic tables used by the full-domain checks."""
    m = np.arange(t, dtype=np.int64)
    return {
        "identity": m.astype(np.uint32),
        "constant": np.full(t, (3 % t), dtype=np.uint32),
        "square": ((m * m) % t).astype(np.uint32),
        # two's-complement ReLU on Z_t: values >= t/2 are negative
        "relu": np.where(m < t // 2, m, 0).astype(np.uint32),
    }


def zipf_indices(seed: int, count: int, nluts: int, s: float = 1.2) -> np.ndarray:
    """LUT index per ciphertext, P(r) proportional to r^-s for r in 1..nluts."""
    rng = np.random.default_rng(seed)
    w = np.arange(1, nluts + 1, dtype=np.float64) ** (-s)
    w /= w.sum()
    return rng.choice(nluts, size=count, p=w).astype(np.int32)


def nn_inputs(seed: int, t: int = 32):
    """Input vector and integer weights of the 784 -> 128 -> 10 circuit."""
    rng = np.random.default_rng(seed)
    x = rng.integers(0, t, size=784, dtype=np.uint32)
    w1 = rng.integers(-8, 9, size=(128, 784), dtype=np.int32)
    w2 = rng.integers(-8, 9, size=(10, 128), dtype=np.int32)
    return x, w1, w2


def poisson_arrivals(seed: int, count: int, rate: float, max_batch: int = 512):
    """Arrival times (s) and batch sizes of a Poisson request stream."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    sizes = rng.integers(1, max_batch + 1, size=count)
    which = rng.integers(0, 2, size=count)
    return np.cumsum(gaps), sizes.astype(np.int64), which.astype(np.int64)

