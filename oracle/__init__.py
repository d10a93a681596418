"""FDFB oracle -- test infrastructure only.

ctypes wrapper around ``fdfb_oracle.c``: a plain, single-threaded CPU
implementation of full-domain functional bootstrapping (arXiv 2109.02731)
at q = Q = 2^32.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package; the GPU library
never does, and this package never imports the library.

Every function here is a thin marshalling layer over the C file, whose
functions cite the passages of the paper they follow.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fdfb_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

OUT_EXTRACTED = 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, so the Gaussian
    sampler's floating-point steps are fixed)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Params(C.Structure):
    _fields_ = [("n", C.c_uint32), ("N", C.c_uint32), ("log2_t", C.c_uint32),
                ("g_log2B", C.c_uint32), ("g_ell", C.c_uint32),
                ("ks_log2B", C.c_uint32), ("ks_ell", C.c_uint32),
                ("pk_log2B", C.c_uint32), ("pk_ell", C.c_uint32),
                ("boot_log2B", C.c_uint32), ("boot_ell", C.c_uint32),
                ("sigma_lwe", C.c_double), ("sigma_glwe", C.c_double),
                ("sigma_pk", C.c_double), ("sigma_ks", C.c_double)]


class _Dumps(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in
                ("ctN", "acc_sign", "c_bits", "r_bits", "acc_f", "acc_f_br", "c_q")]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        u32, u64 = C.c_uint32, C.c_uint64
        sig = {
            "or_draw": (u64, [u64, u64, u64]),
            "or_gauss": (C.c_int64, [u64, u64, u64, C.c_double]),
            "or_negacyclic_mul": (None, [P, P, P, u32]),
            "or_monomial_mul": (None, [P, u32, P, u32]),
            "or_decomp": (None, [u32, u32, u32, P]),
            "or_gadget": (u32, [u32, u32, u32]),
            "or_modswitch": (u32, [u32, u32]),
            "or_sample_extract": (None, [P, u32, P]),
            "or_keyswitch": (None, [P, u32, P, u32, u32, u32, P]),
            "or_extprod": (None, [P, P, u32, u32, u32, P]),
            "or_cmux": (None, [P, P, P, u32, u32, u32, P]),
            "or_blind_rotate": (None, [P, P, P, P]),
            "or_setup_polynomial": (None, [P, u32, u32, P, P]),
            "or_keygen": (None, [P, u64, P, P, P, P, P]),
            "or_encrypt": (None, [P, P, u32, u64, u64, P]),
            "or_phase": (u32, [P, P, u32]),
            "or_decrypt": (u32, [P, P, u32, u32, P]),
            "or_pubmux": (None, [P, P, P, P, P]),
            "or_fdfb": (None, [P, P, P, P, P, P, P, u32, P, P]),
            "or_tfhe_bootstrap": (None, [P, P, P, P, P, u32, P]),
            "or_affine": (None, [P, u32, u32, P, u32, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.c_void_p)


def _u32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint32))


def cparams(p) -> _Params:
    d = p.as_dict() if hasattr(p, "as_dict") else dict(p)
    if d["g_ell"] * d["g_log2B"] > 32 or d["ks_ell"] * d["ks_log2B"] > 32 \
            or d["pk_ell"] * d["pk_log2B"] > 32:
        raise ValueError("ell * log2B must not exceed 32")
    return _Params(**{k: d[k] for k, _ in _Params._fields_})


# --------------------------------------------------------------------------
# scalar and polynomial primitives
# --------------------------------------------------------------------------
def draw(seed: int, stream: int, idx: int) -> int:
    return int(lib().or_draw(seed, stream, idx))


def gauss(seed: int, stream: int, idx: int, sigma: float) -> int:
    return int(lib().or_gauss(seed, stream, idx, sigma))


def negacyclic_mul(a, b) -> np.ndarray:
    a, b = _u32(a), _u32(b)
    c = np.empty_like(a)
    lib().or_negacyclic_mul(_p(a), _p(b), _p(c), a.size)
    return c


def monomial_mul(p, e: int) -> np.ndarray:
    p = _u32(p)
    out = np.empty_like(p)
    lib().or_monomial_mul(_p(p), e, _p(out), p.size)
    return out


def decomp(x: int, log2B: int, ell: int) -> np.ndarray:
    d = np.zeros(ell, dtype=np.uint32)
    lib().or_decomp(x, log2B, ell, _p(d))
    return d


def gadget(log2B: int, ell: int, j: int) -> int:
    return int(lib().or_gadget(log2B, ell, j))


def modswitch(x: int, log2_qout: int) -> int:
    return int(lib().or_modswitch(x, log2_qout))


def sample_extract(rlwe) -> np.ndarray:
    rlwe = _u32(rlwe)
    N = rlwe.size // 2
    out = np.empty(N + 1, dtype=np.uint32)
    lib().or_sample_extract(_p(rlwe), N, _p(out))
    return out


def keyswitch(ct, K, log2B: int, ell: int, out_len: int) -> np.ndarray:
    ct, K = _u32(ct), _u32(K)
    out = np.empty(out_len, dtype=np.uint32)
    lib().or_keyswitch(_p(ct), ct.size - 1, _p(K), log2B, ell, out_len, _p(out))
    return out


def extprod(Cm, d, log2B: int, ell: int) -> np.ndarray:
    Cm, d = _u32(Cm), _u32(d)
    N = d.size // 2
    out = np.empty(2 * N, dtype=np.uint32)
    lib().or_extprod(_p(Cm), _p(d), N, log2B, ell, _p(out))
    return out


def cmux(Cm, g, h, log2B: int, ell: int) -> np.ndarray:
    Cm, g, h = _u32(Cm), _u32(g), _u32(h)
    out = np.empty_like(g)
    lib().or_cmux(_p(Cm), _p(g), _p(h), g.size // 2, log2B, ell, _p(out))
    return out


def blind_rotate(params, brk, ctN, acc) -> np.ndarray:
    cp = cparams(params)
    acc = _u32(acc).copy()
    brk, ctN = _u32(brk), _u32(ctN)
    lib().or_blind_rotate(C.byref(cp), _p(brk), _p(ctN), _p(acc))
    return acc


def setup_polynomial(lut, N: int):
    lut = _u32(lut)
    p0 = np.empty(N, dtype=np.int32)
    p1 = np.empty(N, dtype=np.int32)
    lib().or_setup_polynomial(_p(lut), lut.size, N, _p(p0), _p(p1))
    return p0, p1


def pubmux(params, c, p0, p1) -> np.ndarray:
    cp = cparams(params)
    c = _u32(c)
    p0 = np.ascontiguousarray(p0, dtype=np.int64)
    p1 = np.ascontiguousarray(p1, dtype=np.int64)
    out = np.empty(2 * cp.N, dtype=np.uint32)
    lib().or_pubmux(C.byref(cp), _p(c), _p(p0), _p(p1), _p(out))
    return out


def affine(W, cts) -> np.ndarray:
    W = np.ascontiguousarray(W, dtype=np.int32)
    cts = _u32(cts)
    rows, cols = W.shape
    width = cts.shape[1]
    out = np.empty((rows, width), dtype=np.uint32)
    lib().or_affine(_p(W), rows, cols, _p(cts), width, _p(out))
    return out


# --------------------------------------------------------------------------
# keys, encryption, bootstrapping
# --------------------------------------------------------------------------
@dataclass
class Keys:
    params: object
    seed: int
    s: np.ndarray      # [n]
    sf: np.ndarray     # [N]
    brk: np.ndarray    # [n][2 g_ell][2][N]
    pk: np.ndarray     # [N][pk_ell][2][N]
    ksk: np.ndarray    # [N][ks_ell][n+1]


def keygen(params, seed: int) -> Keys:
    cp = cparams(params)
    n, N = cp.n, cp.N
    s = np.empty(n, np.uint32)
    sf = np.empty(N, np.uint32)
    brk = np.empty((n, 2 * cp.g_ell, 2, N), np.uint32)
    pk = np.empty((N, cp.pk_ell, 2, N), np.uint32)
    ksk = np.empty((N, cp.ks_ell, n + 1), np.uint32)
    lib().or_keygen(C.byref(cp), seed, _p(s), _p(sf), _p(brk), _p(pk), _p(ksk))
    return Keys(params, seed, s, sf, brk, pk, ksk)


def encrypt(params, s, msgs, seed: int, first_index: int = 0) -> np.ndarray:
    cp = cparams(params)
    s = _u32(s)
    msgs = np.asarray(msgs, dtype=np.uint32).reshape(-1)
    out = np.empty((msgs.size, cp.n + 1), np.uint32)
    for k, m in enumerate(msgs):
        row = out[k]
        lib().or_encrypt(C.byref(cp), _p(s), int(m), seed, first_index + k, _p(row))
    return out


def phase(ct, key) -> int:
    ct, key = _u32(ct), _u32(key)
    return int(lib().or_phase(_p(ct), _p(key), key.size))


def decrypt(cts, key, log2_t: int):
    """Messages and centred errors of a batch of LWE samples under `key`."""
    cts = _u32(np.atleast_2d(cts))
    key = _u32(key)
    ms = np.empty(cts.shape[0], np.uint32)
    errs = np.empty(cts.shape[0], np.int64)
    e = C.c_int64()
    for k in range(cts.shape[0]):
        row = np.ascontiguousarray(cts[k])
        ms[k] = lib().or_decrypt(_p(row), _p(key), key.size, log2_t, C.byref(e))
        errs[k] = e.value
    return ms, errs


def fdfb(keys: Keys, rotP0, rotP1, ct, flags: int = 0, dumps: bool = False):
    """One full-domain functional bootstrap of one LWE sample."""
    cp = cparams(keys.params)
    n, N, ellb = cp.n, cp.N, cp.boot_ell
    ct = _u32(ct)
    r0 = np.ascontiguousarray(rotP0, dtype=np.int32)
    r1 = np.ascontiguousarray(rotP1, dtype=np.int32)
    out = np.empty(N + 1 if flags & OUT_EXTRACTED else n + 1, np.uint32)
    d = None
    dp = None
    if dumps:
        d = {"ctN": np.empty(n + 1, np.uint32),
             "acc_sign": np.empty((ellb, 2, N), np.uint32),
             "c_bits": np.empty((ellb, N + 1), np.uint32),
             "r_bits": np.empty((ellb, 2, N), np.uint32),
             "acc_f": np.empty((2, N), np.uint32),
             "acc_f_br": np.empty((2, N), np.uint32),
             "c_q": np.empty(N + 1, np.uint32)}
        dp = _Dumps(**{k: v.ctypes.data for k, v in d.items()})
    lib().or_fdfb(C.byref(cp), _p(keys.brk), _p(keys.pk), _p(keys.ksk), _p(r0), _p(r1), _p(ct),
                  flags, _p(out), C.byref(dp) if dp is not None else None)
    return (out, d) if dumps else out


def fdfb_batch(keys: Keys, luts_rot, lut_ids, cts, flags: int = 0, threads: int | None = None):
    """Bootstrap many samples, one oracle call per sample, threads across samples."""
    cts = _u32(np.atleast_2d(cts))
    threads = threads or os.cpu_count() or 1

    def one(k):
        r0, r1 = luts_rot[int(lut_ids[k])]
        return fdfb(keys, r0, r1, cts[k], flags)

    with ThreadPoolExecutor(max_workers=threads) as ex:
        outs = list(ex.map(one, range(cts.shape[0])))
    return np.stack(outs)


def tfhe_bootstrap(keys: Keys, rotP_scaled, ct, flags: int = 0) -> np.ndarray:
    cp = cparams(keys.params)
    ct = _u32(ct)
    rp = _u32(rotP_scaled)
    out = np.empty(cp.N + 1 if flags & OUT_EXTRACTED else cp.n + 1, np.uint32)
    lib().or_tfhe_bootstrap(C.byref(cp), _p(keys.brk), _p(keys.ksk), _p(rp), _p(ct), flags, _p(out))
    return out
