"""MI355X full-domain functional bootstrapping (FDFB, arXiv 2109.02731).

Thin ctypes binding over ``libfdfb.so`` (C ABI in ``include/fdfb.h``).  The
binding only marshals arguments: every step of the bootstrap runs in the
library's HIP kernels.  PyTorch supplies device memory and streams: device
arguments are torch tensors (int32 or uint32 storage, contiguous, on the GPU)
and work is enqueued on the current torch stream unless one is given.

If the shared library is missing it is built once with hipcc; if that fails
the import fails -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import _build as _buildmod

_LIB_PATH = _buildmod.LIB

OUT_EXTRACTED = 0x1
PLAIN = 0x2
DIRECT = 0x4

FDFB_OK = 0
_ERRNAMES = {-1: "FDFB_EINVAL", -2: "FDFB_ENOMEM", -3: "FDFB_EDEVICE", -4: "FDFB_EABORTED",
             -5: "FDFB_ENOTSUP"}


class FdfbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class _Params(C.Structure):
    _fields_ = [("n", C.c_uint32), ("N", C.c_uint32), ("log2_t", C.c_uint32),
                ("g_log2B", C.c_uint32), ("g_ell", C.c_uint32),
                ("ks_log2B", C.c_uint32), ("ks_ell", C.c_uint32),
                ("pk_log2B", C.c_uint32), ("pk_ell", C.c_uint32),
                ("boot_log2B", C.c_uint32), ("boot_ell", C.c_uint32),
                ("sigma_lwe", C.c_double), ("sigma_glwe", C.c_double),
                ("sigma_pk", C.c_double), ("sigma_ks", C.c_double)]


class _ServerStats(C.Structure):
    _fields_ = [("requests_done", C.c_uint64), ("bootstraps_done", C.c_uint64), ("batches", C.c_uint64),
                ("max_in_flight_bytes", C.c_uint64), ("arena_bytes", C.c_uint64), ("seconds", C.c_double)]


class _Plan(C.Structure):
    _fields_ = [("form", C.c_uint32), ("round", C.c_uint32), ("ms", C.c_double)]

    def as_dict(self):
        return {"form": FORMS.get(self.form, self.form), "round": self.round, "ms": self.ms}


class _Job(C.Structure):
    _fields_ = [("ctx", C.c_void_p), ("d_cts", C.c_void_p), ("d_lut_ids", C.c_void_p),
                ("B", C.c_uint32), ("d_out", C.c_void_p), ("flags", C.c_uint32)]


EXPORTED = [
    "fdfb_keygen_from_seed", "fdfb_register_lut", "fdfb_bootstrap_batch", "fdfb_bootstrap_multi",
    "fdfb_bootstrap_multi_lut", "fdfb_tfhe_bootstrap_batch",
    "fdfb_keyswitch", "fdfb_modswitch", "fdfb_blind_rotate", "fdfb_sample_extract",
    "fdfb_packing_keyswitch", "fdfb_pubmux", "fdfb_encrypt_debug", "fdfb_decrypt_debug",
    "fdfb_export_keys", "fdfb_import_keys", "fdfb_get_key", "fdfb_profile", "fdfb_profile_read",
    "fdfb_br_launches", "fdfb_measure_mfma_peak", "fdfb_set_abort", "fdfb_free", "fdfb_last_error",
    "fdfb_server_create", "fdfb_server_submit", "fdfb_server_poll", "fdfb_server_wait",
    "fdfb_server_stats", "fdfb_server_destroy", "fdfb_affine", "fdfb_lincomb2", "fdfb_prepare",
    "fdfb_release_scratch", "fdfb_device_errors", "fdfb_bootstrap_batch_noalloc", "fdfb_noalloc_max_batch",
    "fdfb_bootstrap_multi_ex", "fdfb_multi_graph_create", "fdfb_graph_launch", "fdfb_graph_info",
    "fdfb_graph_free", "fdfb_br_plans", "fdfb_autotune", "fdfb_br_set_plan", "fdfb_br_get_plan",
    "fdfb_tune_save", "fdfb_tune_load", "fdfb_tune_clear", "fdfb_get_rotation_polys", "fdfb_autotune_bootstrap",
    "fdfb_bootstrap_pipeline",
]

FORMS = {0: "auto", 1: "1w", 2: "1w2", 3: "2w", 4: "queue", 5: "split"}

DEVERR_LUT_ID = 0x1

PHASES = ["modswitch_init", "sign_br", "extract_bits", "packing_ks", "pubmux", "function_br", "output"]

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            _buildmod.build()
        L = C.CDLL(_LIB_PATH)
        P, u32, u64, sz = C.c_void_p, C.c_uint32, C.c_uint64, C.c_size_t
        i = C.c_int
        sigs = {
            "fdfb_keygen_from_seed": (i, [P, u64, P]),
            "fdfb_register_lut": (i, [P, P, P]),
            "fdfb_bootstrap_batch": (i, [P, P, P, u32, P, u32, P]),
            "fdfb_bootstrap_multi_lut": (i, [P, P, P, u32, u32, P, u32, P]),
            "fdfb_tfhe_bootstrap_batch": (i, [P, P, P, u32, P, u32, P]),
            "fdfb_bootstrap_multi": (i, [P, u32, P]),
            "fdfb_bootstrap_multi_ex": (i, [P, u32, i, P]),
            "fdfb_bootstrap_pipeline": (i, [P, u32, u32, P]),
            "fdfb_multi_graph_create": (i, [P, u32, i, P]),
            "fdfb_graph_launch": (i, [P, P]),
            "fdfb_graph_info": (i, [P, P, C.POINTER(sz)]),
            "fdfb_graph_free": (None, [P]),
            "fdfb_br_plans": (i, [P, P, P]),
            "fdfb_autotune": (i, [P, u32, u32, u32, P, P, P]),
            "fdfb_br_set_plan": (i, [P, u32, P]),
            "fdfb_autotune_bootstrap": (i, [P, u32, u32, u32, P, P, P, P]),
            "fdfb_br_get_plan": (i, [P, u32, P]),
            "fdfb_tune_save": (i, [C.c_char_p]),
            "fdfb_tune_load": (i, [C.c_char_p]),
            "fdfb_tune_clear": (i, []),
            "fdfb_get_rotation_polys": (i, [P, C.c_int32, P]),
            "fdfb_keyswitch": (i, [P, P, u32, P, P]),
            "fdfb_modswitch": (i, [P, P, u32, P, P]),
            "fdfb_blind_rotate": (i, [P, P, P, u32, u32, u32, P]),
            "fdfb_sample_extract": (i, [P, P, u32, P, P]),
            "fdfb_packing_keyswitch": (i, [P, P, u32, P, P]),
            "fdfb_pubmux": (i, [P, P, P, P, u32, P, P]),
            "fdfb_encrypt_debug": (i, [P, P, u32, u64, P]),
            "fdfb_decrypt_debug": (i, [P, P, u32, u32, P, P]),
            "fdfb_export_keys": (i, [P, P, C.POINTER(sz)]),
            "fdfb_import_keys": (i, [P, sz, P]),
            "fdfb_get_key": (i, [P, u32, P, C.POINTER(sz)]),
            "fdfb_profile": (i, [P, i]),
            "fdfb_profile_read": (i, [P, P, P]),
            "fdfb_set_abort": (None, [P, i]),
            "fdfb_br_launches": (i, [P, u32, u32, u32, P]),
            "fdfb_measure_mfma_peak": (i, [P, P]),
            "fdfb_free": (None, [P]),
            "fdfb_last_error": (C.c_char_p, []),
            "fdfb_server_create": (i, [P, u32, u32, sz, u32, P]),
            "fdfb_server_submit": (i, [P, u32, P, P, u32, P, u32, P, P]),
            "fdfb_server_poll": (i, [P, C.c_uint64, P]),
            "fdfb_server_wait": (i, [P, C.c_uint64, P]),
            "fdfb_server_stats": (i, [P, P]),
            "fdfb_server_destroy": (None, [P]),
            "fdfb_affine": (i, [P, P, u32, u32, u32, P, P]),
            "fdfb_lincomb2": (i, [P, P, C.c_int32, C.c_int32, u32, u32, P, P]),
            "fdfb_prepare": (i, [P, u32]),
            "fdfb_release_scratch": (i, [P]),
            "fdfb_device_errors": (i, [P, i, P]),
            "fdfb_bootstrap_batch_noalloc": (i, [P, P, P, u32, P, u32, P]),
            "fdfb_noalloc_max_batch": (i, [P, P]),
        }
        for name, (res, args) in sigs.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != FDFB_OK:
        raise FdfbError(rc, lib().fdfb_last_error().decode())


def _np_ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.c_void_p)


def _dev_ptr(t, what: str):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a GPU torch tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if t.element_size() != 4:
        raise TypeError(f"{what} must have 32-bit elements")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream))


def params_struct(p) -> _Params:
    d = p.as_dict() if hasattr(p, "as_dict") else dict(p)
    return _Params(**{k: d[k] for k, _ in _Params._fields_})


class Context:
    """Evaluation keys (device) and secret keys (host) of one parameter set."""

    def __init__(self, handle: C.c_void_p, params):
        self._h = handle
        self.params = params

    # ---- construction --------------------------------------------------
    @classmethod
    def keygen(cls, params, seed: int) -> "Context":
        h = C.c_void_p()
        ps = params_struct(params)
        _check(lib().fdfb_keygen_from_seed(C.byref(ps), seed, C.byref(h)))
        return cls(h, params)

    @classmethod
    def import_keys(cls, blob: bytes, params=None) -> "Context":
        h = C.c_void_p()
        buf = C.create_string_buffer(blob, len(blob))
        _check(lib().fdfb_import_keys(buf, len(blob), C.byref(h)))
        return cls(h, params)

    def export_keys(self) -> bytes:
        n = C.c_size_t(0)
        _check(lib().fdfb_export_keys(self._h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(lib().fdfb_export_keys(self._h, buf, C.byref(n)))
        return buf.raw[: n.value]

    def free(self):
        if self._h:
            lib().fdfb_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    # ---- host-side helpers ----------------------------------------------
    def get_key(self, which: int) -> np.ndarray:
        n = C.c_size_t(0)
        _check(lib().fdfb_get_key(self._h, which, None, C.byref(n)))
        out = np.empty(n.value, np.uint32)
        _check(lib().fdfb_get_key(self._h, which, _np_ptr(out), C.byref(n)))
        return out

    def rotation_polys(self, lut_id: int):
        """rotP_0, rotP_1 of a registered table (int32 [N] each)."""
        out = np.empty(2 * self.params.N, np.int32)
        _check(lib().fdfb_get_rotation_polys(self._h, lut_id, _np_ptr(out)))
        return out[: self.params.N], out[self.params.N:]

    def register_lut(self, table) -> int:
        tab = np.ascontiguousarray(table, dtype=np.uint32)
        lid = C.c_int32()
        _check(lib().fdfb_register_lut(self._h, _np_ptr(tab), C.byref(lid)))
        return lid.value

    def encrypt_debug(self, msgs, seed: int) -> np.ndarray:
        m = np.ascontiguousarray(msgs, dtype=np.uint32).reshape(-1)
        out = np.empty((m.size, self.params.n + 1), np.uint32)
        _check(lib().fdfb_encrypt_debug(self._h, _np_ptr(m), m.size, seed, _np_ptr(out)))
        return out

    def decrypt_debug(self, cts) -> tuple[np.ndarray, np.ndarray]:
        cts = np.ascontiguousarray(np.atleast_2d(cts), dtype=np.uint32)
        B, width = cts.shape
        m = np.empty(B, np.uint32)
        e = np.empty(B, np.int64)
        _check(lib().fdfb_decrypt_debug(self._h, _np_ptr(cts), B, width - 1, _np_ptr(m), _np_ptr(e)))
        return m, e

    def profile(self, enable: bool = True):
        _check(lib().fdfb_profile(self._h, 1 if enable else 0))

    def profile_read(self) -> tuple[dict, int]:
        """Summed milliseconds per phase over the recorded calls, and the call count."""
        ms = (C.c_double * len(PHASES))()
        calls = C.c_uint32()
        _check(lib().fdfb_profile_read(self._h, ms, C.byref(calls)))
        return dict(zip(PHASES, list(ms))), calls.value

    def br_launches(self, accumulators: int, per_ct: int = 1, flags: int = 0) -> int:
        """Kernel launches of one batched blind rotation of this many accumulators."""
        n = C.c_uint32()
        _check(lib().fdfb_br_launches(self._h, accumulators, per_ct, flags, C.byref(n)))
        return n.value

    # ---- autotuning of the blind rotation ---------------------------------
    def br_plans(self) -> list:
        """Every issue plan (form, round) the kernels offer for this geometry."""
        n = C.c_uint32(0)
        _check(lib().fdfb_br_plans(self._h, None, C.byref(n)))
        arr = (_Plan * n.value)()
        _check(lib().fdfb_br_plans(self._h, arr, C.byref(n)))
        return [(p.form, p.round) for p in arr]

    def autotune(self, A: int, per: int = 1, reps: int = 2) -> dict:
        """Time every plan on A accumulators and record the fastest for this
        geometry and size; returns the choice and every timing."""
        best = _Plan()
        cap = 16
        tried = (_Plan * cap)()
        n = C.c_uint32(cap)
        _check(lib().fdfb_autotune(self._h, A, per, reps, C.byref(best), tried, C.byref(n)))
        return {"best": best.as_dict(), "tried": [tried[k].as_dict() for k in range(min(n.value, cap))]}

    def autotune_bootstrap(self, B: int, L: int = 1, reps: int = 2) -> dict:
        """Tune both rotation phases of a batch of B samples (L tables each) by
        timing whole batches; returns the plans chosen and every timing."""
        sb, fb = _Plan(), _Plan()
        cap = 32
        tried = (_Plan * cap)()
        n = C.c_uint32(cap)
        _check(lib().fdfb_autotune_bootstrap(self._h, B, L, reps, C.byref(sb), C.byref(fb), tried, C.byref(n)))
        return {"sign_rotations": sb.as_dict(), "function_rotation": fb.as_dict(),
                "batch_ms": [tried[k].as_dict() for k in range(min(n.value, cap))]}

    def set_plan(self, A: int, form=None, round: int = 0):
        """Force the plan for A accumulators (form None: back to the fixed rule)."""
        if form is None:
            _check(lib().fdfb_br_set_plan(self._h, A, None))
        else:
            p = _Plan(form, round, 0.0)
            _check(lib().fdfb_br_set_plan(self._h, A, C.byref(p)))

    def get_plan(self, A: int) -> dict:
        p = _Plan()
        _check(lib().fdfb_br_get_plan(self._h, A, C.byref(p)))
        return p.as_dict()

    def set_abort(self, raised: bool):
        lib().fdfb_set_abort(self._h, 1 if raised else 0)

    def prepare(self, flags: int = 0):
        """Upload keys, tables and the requested form without enqueuing work."""
        _check(lib().fdfb_prepare(self._h, flags))

    def release_scratch(self):
        """Free every scratch block (waits for the device)."""
        _check(lib().fdfb_release_scratch(self._h))

    def device_errors(self, clear: bool = True) -> int:
        """Device error bits (DEVERR_*) since the last clear; waits for the device."""
        bits = C.c_uint32()
        _check(lib().fdfb_device_errors(self._h, 1 if clear else 0, C.byref(bits)))
        return bits.value

    # ---- device entry points (torch tensors) ------------------------------
    def bootstrap_multi_lut(self, cts, lut_ids, out, flags: int = 0, stream=None):
        """L tables per sample sharing the sign rotations: lut_ids int32 [B, L],
        out [B, L, dim]."""
        B = int(cts.shape[0]) if cts.dim() > 1 else 0
        L = int(lut_ids.shape[1]) if lut_ids.dim() == 2 else 0
        _check(lib().fdfb_bootstrap_multi_lut(self._h, _dev_ptr(cts, "cts"), _dev_ptr(lut_ids, "lut_ids"), B, L,
                                              _dev_ptr(out, "out"), flags, _stream(stream)))

    def tfhe_bootstrap_batch(self, cts, lut_ids, out, flags: int = 0, stream=None):
        """Half-domain (one-rotation) bootstrap with rotP_0 of each sample's table."""
        B = int(cts.shape[0]) if cts.dim() > 1 else 0
        _check(lib().fdfb_tfhe_bootstrap_batch(self._h, _dev_ptr(cts, "cts"), _dev_ptr(lut_ids, "lut_ids"), B,
                                               _dev_ptr(out, "out"), flags, _stream(stream)))

    def bootstrap_batch(self, cts, lut_ids, out, flags: int = 0, stream=None):
        B = int(cts.shape[0]) if cts.dim() > 1 else 0
        _check(lib().fdfb_bootstrap_batch(self._h, _dev_ptr(cts, "cts"), _dev_ptr(lut_ids, "lut_ids"), B,
                                          _dev_ptr(out, "out"), flags, _stream(stream)))
        return out

    def bootstrap_batch_noalloc(self, cts, lut_ids, out, flags: int = 0, stream=None):
        """fdfb_bootstrap_batch with its scratch in the library's static buffer
        (no allocation; the context must be prepared, B <= noalloc_max_batch())."""
        B = int(cts.shape[0]) if cts.dim() > 1 else 0
        _check(lib().fdfb_bootstrap_batch_noalloc(self._h, _dev_ptr(cts, "cts"), _dev_ptr(lut_ids, "lut_ids"), B,
                                                  _dev_ptr(out, "out"), flags, _stream(stream)))
        return out

    def noalloc_max_batch(self) -> int:
        n = C.c_uint32()
        _check(lib().fdfb_noalloc_max_batch(self._h, C.byref(n)))
        return n.value

    def keyswitch(self, d_in, out, stream=None):
        _check(lib().fdfb_keyswitch(self._h, _dev_ptr(d_in, "in"), int(d_in.shape[0]),
                                    _dev_ptr(out, "out"), _stream(stream)))
        return out

    def modswitch(self, cts, out, stream=None):
        _check(lib().fdfb_modswitch(self._h, _dev_ptr(cts, "cts"), int(cts.shape[0]), _dev_ptr(out, "out"),
                                    _stream(stream)))
        return out

    def blind_rotate(self, acc, ctN, accs_per_ct: int = 1, flags: int = 0, stream=None):
        _check(lib().fdfb_blind_rotate(self._h, _dev_ptr(acc, "acc"), _dev_ptr(ctN, "ctN"), int(acc.shape[0]),
                                       accs_per_ct, flags, _stream(stream)))
        return acc

    def sample_extract(self, acc, out, stream=None):
        _check(lib().fdfb_sample_extract(self._h, _dev_ptr(acc, "acc"), int(acc.shape[0]), _dev_ptr(out, "out"),
                                         _stream(stream)))
        return out

    def packing_keyswitch(self, d_in, out, stream=None):
        _check(lib().fdfb_packing_keyswitch(self._h, _dev_ptr(d_in, "in"), int(d_in.shape[0]),
                                            _dev_ptr(out, "out"), _stream(stream)))
        return out

    def pubmux(self, rlwe, ctN, lut_ids, out, stream=None):
        _check(lib().fdfb_pubmux(self._h, _dev_ptr(rlwe, "rlwe"), _dev_ptr(ctN, "ctN"),
                                 _dev_ptr(lut_ids, "lut_ids"), int(out.shape[0]), _dev_ptr(out, "out"),
                                 _stream(stream)))
        return out


class Server:
    """Continuous-batching bootstrap server over one or more contexts."""

    def __init__(self, ctxs, max_batch: int = 1024, mem_budget: int = 1 << 30, nstreams: int = 2):
        self.ctxs = list(ctxs)  # keep the contexts alive
        arr = (C.c_void_p * len(self.ctxs))(*[c._h.value if isinstance(c._h, C.c_void_p) else c._h
                                              for c in self.ctxs])
        h = C.c_void_p()
        _check(lib().fdfb_server_create(arr, len(self.ctxs), max_batch, mem_budget, nstreams, C.byref(h)))
        self._h = h

    def submit(self, ctx_index: int, cts, lut_ids, out, flags: int = 0, stream=None) -> int:
        """Queue a request; its inputs are read after the work already queued on
        `stream` (the current torch stream by default)."""
        rid = C.c_uint64()
        _check(lib().fdfb_server_submit(self._h, ctx_index, _dev_ptr(cts, "cts"), _dev_ptr(lut_ids, "lut_ids"),
                                        int(cts.shape[0]), _dev_ptr(out, "out"), flags, _stream(stream),
                                        C.byref(rid)))
        return rid.value

    def poll(self, rid: int) -> bool:
        done = C.c_int()
        _check(lib().fdfb_server_poll(self._h, rid, C.byref(done)))
        return bool(done.value)

    def wait(self, rid: int) -> float:
        lat = C.c_double()
        _check(lib().fdfb_server_wait(self._h, rid, C.byref(lat)))
        return lat.value

    def stats(self) -> dict:
        st = _ServerStats()
        _check(lib().fdfb_server_stats(self._h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in _ServerStats._fields_}

    def close(self):
        if self._h:
            lib().fdfb_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def affine(W, cts, out, stream=None):
    """out[r] = sum_c W[r][c] * cts[c] mod 2^32 (W int32 [rows][cols] on the GPU)."""
    rows, cols = int(W.shape[0]), int(W.shape[1])
    _check(lib().fdfb_affine(_dev_ptr(W, "W"), _dev_ptr(cts, "cts"), rows, cols, int(cts.shape[1]),
                             _dev_ptr(out, "out"), _stream(stream)))
    return out


def lincomb2(x, y, wx: int, wy: int, out, stream=None):
    """out = wx * x + wy * y mod 2^32, sample by sample (x, y, out [B][width])."""
    B, width = int(x.shape[0]), int(x.shape[1])
    if tuple(y.shape) != (B, width) or tuple(out.shape) != (B, width):
        raise ValueError("x, y and out must have the same shape")
    _check(lib().fdfb_lincomb2(_dev_ptr(x, "x"), _dev_ptr(y, "y"), wx, wy, B, width, _dev_ptr(out, "out"),
                               _stream(stream)))
    return out


def _jobs(jobs):
    arr = (_Job * max(1, len(jobs)))()
    for k, (ctx, cts, ids, out, flags) in enumerate(jobs):
        arr[k] = _Job(ctx._h, _dev_ptr(cts, "cts").value, _dev_ptr(ids, "lut_ids").value, int(cts.shape[0]),
                      _dev_ptr(out, "out").value, flags)
    return arr


def bootstrap_multi(jobs, stream=None, use_queue=None):
    """jobs: list of (Context, cts, lut_ids, out, flags).  use_queue: None for
    the library's rule, True / False to force the persistent work-queue
    rotations on or off (same output bits)."""
    arr = _jobs(jobs)
    if use_queue is None:
        _check(lib().fdfb_bootstrap_multi(arr, len(jobs), _stream(stream)))
    else:
        _check(lib().fdfb_bootstrap_multi_ex(arr, len(jobs), 1 if use_queue else 0, _stream(stream)))


def bootstrap_pipeline(jobs, rounds=0, stream=None):
    """jobs: list of (Context, cts, lut_ids, out, flags), bootstrapped as a
    software pipeline (fdfb_bootstrap_pipeline): job k's function rotation
    shares persistent launches with the next jobs' sign rotations.  rounds:
    resident-capacity rounds per launch (0: the library's default)."""
    _check(lib().fdfb_bootstrap_pipeline(_jobs(jobs), len(jobs), int(rounds), _stream(stream)))


class MultiGraph:
    """A multi-job submission captured into a HIP graph (fdfb_multi_graph_create):
    replay() runs every job's bootstrap with one graph launch."""

    def __init__(self, jobs, use_queue=None):
        self._keep = list(jobs)  # contexts and tensors must outlive the graph
        h = C.c_void_p()
        q = -1 if use_queue is None else (1 if use_queue else 0)
        _check(lib().fdfb_multi_graph_create(_jobs(jobs), len(jobs), q, C.byref(h)))
        self._h = h

    def replay(self, stream=None):
        _check(lib().fdfb_graph_launch(self._h, _stream(stream)))

    def info(self) -> dict:
        q, b = C.c_uint32(), C.c_size_t()
        _check(lib().fdfb_graph_info(self._h, C.byref(q), C.byref(b)))
        return {"uses_queue": bool(q.value), "scratch_bytes": b.value}

    def close(self):
        if self._h:
            lib().fdfb_graph_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune_save(path: str):
    _check(lib().fdfb_tune_save(path.encode()))


def tune_load(path: str):
    _check(lib().fdfb_tune_load(path.encode()))


def tune_clear():
    _check(lib().fdfb_tune_clear())


def to_device(a: np.ndarray, device="cuda"):
    """uint32 numpy array -> int32 torch tensor with the same bits."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to(device)


def measure_mfma_peak() -> tuple[float, float]:
    """Sustained dense int8 MFMA rate of the current device (tera-ops/s) and the
    duration of the timed calibration launch (ms): fdfb_measure_mfma_peak."""
    tops, ms = C.c_double(), C.c_double()
    _check(lib().fdfb_measure_mfma_peak(C.byref(tops), C.byref(ms)))
    return tops.value, ms.value


def to_host(t) -> np.ndarray:
    """32-bit torch tensor -> uint32 numpy array with the same bits."""
    return t.detach().cpu().contiguous().numpy().view(np.uint32)
