"""CPU checks of the C-ABI library: symbols, host-side key generation against
the oracle's (same seed, independent implementations), debug encryption,
argument validation and serialisation.  Nothing here touches a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import paper_2109_02731_amd as fd
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "fdfb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fdfb_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 15
    L = fd.lib()
    for name in names:
        assert hasattr(L, name), name
    assert sorted(fd.EXPORTED) == names


@pytest.mark.parametrize("preset", ["C1", "C2", "C1S"])
def test_keys_equal_oracle_keys(preset, request):
    """Same seed, independent implementations: every key word agrees.  C1S
    draws every key with its own deviation, so a deviation taken for the wrong
    key in either implementation shows up here (the oracle's are pinned by the
    noise checks)."""
    p = W.C1S if preset == "C1S" else W.PRESETS[preset]
    seed = W.KEY_SEED[preset]
    ok = oracle.keygen(p, seed) if preset == "C1S" else \
        request.getfixturevalue("oracle_keys_c1" if preset == "C1" else "oracle_keys_c2")
    ctx = fd.Context.keygen(p, seed)
    for which, ref in enumerate([ok.s, ok.sf, ok.brk, ok.pk, ok.ksk]):
        got = ctx.get_key(which)
        assert np.array_equal(got, ref.reshape(-1)), which


def test_exact_keys_equal_oracle(oracle_keys_c1_exact):
    p = W.exact(W.C1)
    ctx = fd.Context.keygen(p, W.KEY_SEED["C1"])
    for which, ref in enumerate([oracle_keys_c1_exact.brk, oracle_keys_c1_exact.pk, oracle_keys_c1_exact.ksk]):
        assert np.array_equal(ctx.get_key(which + 2), ref.reshape(-1))


def test_encrypt_debug_uses_the_fresh_deviation():
    """Fresh samples of the library at C1S equal the oracle's (whose noise
    deviation is pinned to sigma_lwe)."""
    p = W.C1S
    ctx = fd.Context.keygen(p, W.KEY_SEED["C1S"])
    ok = oracle.keygen(p, W.KEY_SEED["C1S"])
    msgs = W.messages(6, 64, p.t)
    assert np.array_equal(ctx.encrypt_debug(msgs, seed=9), oracle.encrypt(p, ok.s, msgs, seed=9))


def test_encrypt_decrypt_debug_match_oracle(oracle_keys_c1):
    p = W.C1
    ctx = fd.Context.keygen(p, W.KEY_SEED["C1"])
    msgs = W.messages(5, 40, p.t)
    cts = ctx.encrypt_debug(msgs, seed=77)
    ref = oracle.encrypt(p, oracle_keys_c1.s, msgs, seed=77)
    assert np.array_equal(cts, ref)
    m, e = ctx.decrypt_debug(cts)
    mo, eo = oracle.decrypt(cts, oracle_keys_c1.s, p.log2_t)
    assert np.array_equal(m, msgs) and np.array_equal(m, mo) and np.array_equal(e, eo)


def test_rejects_bad_parameters():
    bad = [W.C1.with_(N=300), W.C1.with_(N=8192), W.C1.with_(log2_t=9),
           W.C1.with_(g_ell=5, g_log2B=8), W.C1.with_(boot_ell=1), W.C1.with_(ks_ell=9, ks_log2B=3),
           W.C1.with_(sigma_glwe=-1.0), W.C1.with_(ks_log2B=17, ks_ell=1), W.C1.with_(pk_log2B=32, pk_ell=1)]
    for p in bad:
        with pytest.raises(fd.FdfbError) as ei:
            fd.Context.keygen(p, 1)
        assert ei.value.code == -1


def test_lut_validation_and_ids():
    ctx = fd.Context.keygen(W.C1, 3)
    assert ctx.register_lut(np.arange(8)) == 0
    assert ctx.register_lut(np.zeros(8)) == 1
    with pytest.raises(fd.FdfbError):
        ctx.register_lut(np.full(8, 8))


def test_export_import_roundtrip():
    ctx = fd.Context.keygen(W.C1, 9)
    ctx.register_lut(W.random_lut(1, 8))
    blob = ctx.export_keys()
    ctx2 = fd.Context.import_keys(blob, W.C1)
    for which in range(5):
        assert np.array_equal(ctx.get_key(which), ctx2.get_key(which))
    with pytest.raises(fd.FdfbError):
        fd.Context.import_keys(blob[:100])
    with pytest.raises(fd.FdfbError):
        fd.Context.import_keys(b"x" * len(blob))


def test_abort_flag_and_empty_batch_on_host():
    """Error paths that return before any device work."""
    ctx = fd.Context.keygen(W.C1, 4)
    L = fd.lib()
    assert L.fdfb_bootstrap_batch(ctx._h, None, None, 0, None, 0, None) == 0      # B = 0 is a no-op
    assert L.fdfb_bootstrap_batch(ctx._h, None, None, 5, None, 0, None) == -1     # null buffers
    assert L.fdfb_bootstrap_batch(ctx._h, C.c_void_p(16), C.c_void_p(16), 1, C.c_void_p(16), 0x80, None) == -1
    ctx.set_abort(True)
    assert L.fdfb_bootstrap_batch(ctx._h, C.c_void_p(16), C.c_void_p(16), 1, C.c_void_p(16), 0, None) == -4
    assert b"abort" in L.fdfb_last_error()
    ctx.set_abort(False)
    with pytest.raises(fd.FdfbError):
        ctx.decrypt_debug(np.zeros((1, 5), np.uint32))  # dim is neither n nor N


def _blob_parts(blob):
    """Header layout of an exported key blob: magic, params, seed, 6 counts."""
    head = 8 + C.sizeof(fd._Params) + 8
    counts = np.frombuffer(blob[head:head + 48], np.uint64).copy()
    return head, counts


def test_import_rejects_crafted_blobs():
    """A forged or damaged blob gives FDFB_EINVAL, never an abort: huge table
    counts (whose byte sums would wrap), truncated sections, a wrong magic,
    inconsistent key sizes and non-binary secrets."""
    ctx = fd.Context.keygen(W.C1, 9)
    ctx.register_lut(W.random_lut(1, 8))
    blob = bytearray(ctx.export_keys())
    head, counts = _blob_parts(bytes(blob))

    def rejected(b, why):
        with pytest.raises(fd.FdfbError) as ei:
            fd.Context.import_keys(bytes(b))
        assert ei.value.code == -1, why

    for forged in (1 << 62, (1 << 62) + 8, (1 << 64) - 8, 8 << 40):
        b = bytearray(blob)
        c = counts.copy()
        c[5] = forged
        b[head:head + 48] = c.tobytes()
        rejected(b, f"table count {forged}")
    for cut in (len(blob) - 1, len(blob) - 4 * 8, head + 48, head + 48 + 4 * int(counts[0]) + 3):
        rejected(blob[:cut], f"truncated at {cut}")
    b = bytearray(blob)
    b[0:8] = b"FDFBKEY2"
    rejected(b, "magic")
    b = bytearray(blob)
    c = counts.copy()
    c[2] += 1  # brK section one word longer than the parameters say
    b[head:head + 48] = c.tobytes()
    rejected(b, "brK size")
    b = bytearray(blob)
    b[head + 48] = 2  # s[0] = 2: not a binary secret
    rejected(b, "secret")
    b = bytearray(blob)
    b[-4:] = np.uint32(8).tobytes()  # last table value 8 >= t
    rejected(b, "table value")
    assert fd.Context.import_keys(bytes(blob)) is not None  # the untouched blob still loads


def test_every_entry_point_survives_null_and_zero_arguments():
    """Null contexts and buffers are FDFB_EINVAL on every device entry point
    (checked before any device call)."""
    L = fd.lib()
    nul = None
    assert L.fdfb_bootstrap_multi_lut(nul, nul, nul, 1, 1, nul, 0, nul) == -1
    assert L.fdfb_tfhe_bootstrap_batch(nul, nul, nul, 1, nul, 0, nul) == -1
    assert L.fdfb_keyswitch(nul, nul, 1, nul, nul) == -1
    assert L.fdfb_blind_rotate(nul, nul, nul, 1, 1, 0, nul) == -1
    assert L.fdfb_pubmux(nul, nul, nul, nul, 1, nul, nul) == -1
    assert L.fdfb_prepare(nul, 0) == -1
    assert L.fdfb_release_scratch(nul) == -1
    assert L.fdfb_device_errors(nul, 1, nul) == -1
    assert L.fdfb_lincomb2(nul, nul, 1, 1, 2, 3, nul, nul) == -1
    assert L.fdfb_lincomb2(nul, nul, 1, 1, 0, 3, nul, nul) == 0
    ctx = fd.Context.keygen(W.C1, 4)
    assert L.fdfb_bootstrap_multi_lut(ctx._h, C.c_void_p(16), C.c_void_p(16), 1, 0, C.c_void_p(16), 0, nul) == -1
    assert L.fdfb_prepare(ctx._h, 0x80) == -1
    assert L.fdfb_prepare(ctx._h, fd.PLAIN | fd.DIRECT) == -1
    job = fd._Job(None, None, None, 1, None, 0)
    assert L.fdfb_bootstrap_multi(C.byref(job), 1, nul) == -1
    assert L.fdfb_bootstrap_pipeline(C.byref(job), 1, 0, nul) == -1
    assert L.fdfb_bootstrap_pipeline(nul, 1, 0, nul) == -1
    # the pipeline takes only rotations the work-queue kernel runs, and at most 64 rounds per launch
    plain = fd._Job(ctx._h, 16, 16, 1, 16, fd.PLAIN)
    assert L.fdfb_bootstrap_pipeline(C.byref(plain), 1, 0, nul) == -1
    assert "work-queue" in fd.lib().fdfb_last_error().decode()
    assert L.fdfb_bootstrap_pipeline(C.byref(job), 1, 65, nul) == -1
    assert L.fdfb_bootstrap_pipeline(nul, 0, 0, nul) == 0  # nothing to do


def test_context_lock_serialises_threads():
    """Host entry points on one context from several threads at once (the
    context lock orders them): tables get distinct ids and every
    encryption equals the single-threaded one."""
    import threading
    ctx = fd.Context.keygen(W.C1, 5)
    msgs = W.messages(3, 32, W.C1.t)
    ref = ctx.encrypt_debug(msgs, seed=11)
    ids, outs, errs = [], [], []

    def work(k):
        try:
            for _ in range(20):
                ids.append(ctx.register_lut(W.random_lut(k, 8)))
                outs.append(ctx.encrypt_debug(msgs, seed=11))
        except Exception as e:  # pragma: no cover - reported below
            errs.append(e)

    th = [threading.Thread(target=work, args=(k,)) for k in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errs
    assert sorted(ids) == list(range(80))
    assert all(np.array_equal(o, ref) for o in outs)


def test_tune_cache_file_roundtrip(tmp_path):
    """The autotuner's cache file: entries written by fdfb_tune_save are read
    back by fdfb_tune_load; lines that are not entries are skipped; the plans
    offered for the headline geometry are the five forms."""
    src = tmp_path / "in.json"
    src.write_text('[\n'
                   ' {"cus": 256, "N": 1024, "ell": 3, "chunks": 1, "n": 630, "A": 2048, "form": 2, "round": 0, '
                   '"ms": 31.5000},\n'
                   ' not an entry\n'
                   ' {"cus": 256, "N": 2048, "ell": 2, "chunks": 2, "n": 750, "A": 6144, "form": 4, "round": 0, '
                   '"ms": 290.2500}\n'
                   ']\n')
    fd.tune_clear()
    fd.tune_load(str(src))
    out = tmp_path / "out.json"
    fd.tune_save(str(out))
    import json
    got = json.loads(out.read_text())
    assert [(e["N"], e["A"], e["form"], e["ms"]) for e in got] == [(1024, 2048, 2, 31.5), (2048, 6144, 4, 290.25)]
    with pytest.raises(fd.FdfbError):
        fd.tune_load(str(tmp_path / "missing.json"))
    fd.tune_clear()
    fd.tune_save(str(out))
    assert json.loads(out.read_text()) == []
    ctx = fd.Context.keygen(W.C2, 1)
    forms = {f for f, _ in ctx.br_plans()}
    assert forms == {0, 1, 2, 3, 4}
    with pytest.raises(fd.FdfbError):
        ctx.set_plan(2048, form=7)


@pytest.mark.parametrize("log2_t,N", [(1, 64), (3, 256), (4, 1024), (5, 2048), (6, 64), (8, 256)])
def test_rotation_polys_equal_oracle(log2_t, N):
    """The library's rotation polynomials equal the oracle's (two independent
    derivations from the theorem's property, Sec. 3.3) for random and
    non-negacyclic tables, every t from 2 up to N/4 and the extreme t = N/8."""
    p = W.C1.with_(N=N, log2_t=log2_t, n=16, boot_log2B=2, boot_ell=(log2_t + 1) // 2)
    t = p.t
    ctx = fd.Context.keygen(p, 3)
    tables = [W.random_lut(41 + log2_t, t), np.arange(t, dtype=np.uint32), np.full(t, t - 1, np.uint32)]
    for tab in tables:
        lid = ctx.register_lut(tab)
        r0, r1 = ctx.rotation_polys(lid)
        o0, o1 = oracle.setup_polynomial(tab, N)
        assert np.array_equal(r0, o0) and np.array_equal(r1, o1), (t, N)
    with pytest.raises(fd.FdfbError):
        ctx.rotation_polys(len(tables))
