"""GPU parity: every stage of the HIP path against the CPU oracle, bit for bit,
through the C ABI, for both kernel forms (batched MFMA and plain VALU)."""
import dataclasses
import os

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
fd = pytest.importorskip("paper_2109_02731_amd")

pytestmark = pytest.mark.gpu
M32 = 1 << 32
FORMS = {"batched": 0, "plain": fd.PLAIN, "direct": fd.DIRECT}


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def c1(oracle_keys_c1):
    return fd.Context.keygen(W.C1, W.KEY_SEED["C1"]), oracle_keys_c1


@pytest.fixture(scope="module")
def c1x(oracle_keys_c1_exact):
    return fd.Context.keygen(W.exact(W.C1), W.KEY_SEED["C1"]), oracle_keys_c1_exact


@pytest.fixture(scope="module")
def c2(oracle_keys_c2):
    return fd.Context.keygen(W.C2, W.KEY_SEED["C2"]), oracle_keys_c2


def u32(g, *shape):
    return g.integers(0, M32, shape, dtype=np.uint64).astype(np.uint32)


def empty(*shape):
    return torch.empty(shape, dtype=torch.int32, device="cuda")


def run_oracle_many(fn, count, threads=16):
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(fn, range(count)))


# ----------------------------------------------------------------------------
# single procedures
# ----------------------------------------------------------------------------
def test_modswitch(c1):
    ctx, _ = c1
    p = W.C1
    cts = u32(np.random.default_rng(1), 21, p.n + 1)
    say("modswitch C1 B=21")
    out = fd.to_host(ctx.modswitch(fd.to_device(cts), empty(21, p.n + 1)))
    torch.cuda.synchronize()
    lg = int(np.log2(2 * p.N))
    ref = np.vectorize(lambda x: oracle.modswitch(int(x), lg), otypes=[np.uint32])(cts)
    assert np.array_equal(out, ref)


@pytest.mark.parametrize("form", list(FORMS))
def test_blind_rotate_c1(c1, form):
    ctx, ok = c1
    p = W.C1
    N = p.N
    g = np.random.default_rng(2)
    A, per = 9, 3
    acc = u32(g, A, 2 * N)
    ctN = g.integers(0, 2 * N, (A // per, p.n + 1)).astype(np.uint32)
    ctN[0, 1:6] = 0  # X^0 rotations: the CMux must leave the accumulator as is
    say(f"blind_rotate C1 {form} A={A}")
    d_acc = fd.to_device(acc)
    ctx.blind_rotate(d_acc, fd.to_device(ctN), accs_per_ct=per, flags=FORMS[form])
    torch.cuda.synchronize()
    got = fd.to_host(d_acc)
    for a in range(A):
        ref = oracle.blind_rotate(p, ok.brk, ctN[a // per], acc[a])
        assert np.array_equal(got[a], ref), a


@pytest.mark.parametrize("form", list(FORMS))
def test_blind_rotate_exact_params(c1x, form):
    ctx, ok = c1x
    p = W.exact(W.C1)
    N = p.N
    g = np.random.default_rng(3)
    acc = u32(g, 5, 2 * N)
    ctN = g.integers(0, 2 * N, (5, p.n + 1)).astype(np.uint32)
    say(f"blind_rotate C1-exact {form}")
    d_acc = fd.to_device(acc)
    ctx.blind_rotate(d_acc, fd.to_device(ctN), 1, FORMS[form])
    torch.cuda.synchronize()
    got = fd.to_host(d_acc)
    for a in range(5):
        assert np.array_equal(got[a], oracle.blind_rotate(p, ok.brk, ctN[a], acc[a])), a


def test_sample_extract(c1):
    ctx, _ = c1
    p = W.C1
    acc = u32(np.random.default_rng(4), 7, 2 * p.N)
    say("sample_extract C1")
    got = fd.to_host(ctx.sample_extract(fd.to_device(acc), empty(7, p.N + 1)))
    torch.cuda.synchronize()
    for a in range(7):
        assert np.array_equal(got[a], oracle.sample_extract(acc[a]))


def test_keyswitches(c1):
    ctx, ok = c1
    p = W.C1
    lwe = u32(np.random.default_rng(5), 19, p.N + 1)
    say("keyswitch / packing keyswitch C1 B=19")
    d = fd.to_device(lwe)
    ks = fd.to_host(ctx.keyswitch(d, empty(19, p.n + 1)))
    pk = fd.to_host(ctx.packing_keyswitch(d, empty(19, 2 * p.N)))
    torch.cuda.synchronize()
    for b in range(19):
        assert np.array_equal(ks[b], oracle.keyswitch(lwe[b], ok.ksk, p.ks_log2B, p.ks_ell, p.n + 1))
        assert np.array_equal(pk[b], oracle.keyswitch(lwe[b], ok.pk, p.pk_log2B, p.pk_ell, 2 * p.N))


def test_pubmux(c1):
    ctx, _ = c1
    p = W.C1
    N, eb = p.N, p.boot_ell
    g = np.random.default_rng(6)
    luts = [W.random_lut(10 + k, p.t) for k in range(3)]
    ids = np.array([0, 2, 1, 1, 0, 2, 2], dtype=np.int32)
    for lut in luts:
        ctx.register_lut(lut)
    B = len(ids)
    R = u32(g, B, eb, 2 * N)
    ctN = g.integers(0, 2 * N, (B, p.n + 1)).astype(np.uint32)
    say("pubmux C1 B=7")
    got = fd.to_host(ctx.pubmux(fd.to_device(R), fd.to_device(ctN),
                                torch.from_numpy(ids).cuda(), empty(B, 2 * N)))
    torch.cuda.synchronize()
    for b in range(B):
        r0, r1 = oracle.setup_polynomial(luts[ids[b]], N)
        e = int(ctN[b, 0])
        pa = oracle.monomial_mul(r1.view(np.uint32), e).view(np.int32).astype(np.int64)
        pb = oracle.monomial_mul(r0.view(np.uint32), e).view(np.int32).astype(np.int64)
        assert np.array_equal(got[b], oracle.pubmux(p, R[b], pa, pb)), b


# ----------------------------------------------------------------------------
# full bootstrap
# ----------------------------------------------------------------------------
def _bootstrap(ctx, cts, ids, flags, width):
    d_out = empty(len(cts), width)
    ctx.bootstrap_batch(fd.to_device(cts), torch.from_numpy(np.asarray(ids, np.int32)).cuda(), d_out,
                        flags=flags)
    torch.cuda.synchronize()
    return fd.to_host(d_out)


@pytest.mark.parametrize("form", list(FORMS))
def test_fdfb_c1_vs_oracle(c1, form):
    ctx, ok = c1
    p = W.C1
    luts = [W.random_lut(W.LUT_SEED["C1"], p.t), W.named_luts(p.t)["relu"]]
    lids = [ctx.register_lut(l) for l in luts]
    msgs = np.concatenate([np.arange(p.t), W.messages(W.MSG_SEED["C1"], 13, p.t)]).astype(np.uint32)
    B = len(msgs)  # 21: ragged against the 4-wave workgroups
    which = np.arange(B) % 2
    ids = np.array([lids[w] for w in which], np.int32)
    cts = ctx.encrypt_debug(msgs, seed=W.MSG_SEED["C1"])
    rots = [oracle.setup_polynomial(l, p.N) for l in luts]
    say(f"fdfb C1 {form} B={B}")
    out = _bootstrap(ctx, cts, ids, FORMS[form], p.n + 1)
    ref = np.stack(run_oracle_many(lambda k: oracle.fdfb(ok, *rots[which[k]], cts[k]), B))
    assert np.array_equal(out, ref)
    m, _ = ctx.decrypt_debug(out)
    want = np.array([luts[which[k]][msgs[k]] for k in range(B)])
    assert np.array_equal(m, want)
    say(f"fdfb C1 {form} extracted")
    outq = _bootstrap(ctx, cts, ids, FORMS[form] | fd.OUT_EXTRACTED, p.N + 1)
    refq = np.stack(run_oracle_many(
        lambda k: oracle.fdfb(ok, *rots[which[k]], cts[k], flags=oracle.OUT_EXTRACTED), B))
    assert np.array_equal(outq, refq)


@pytest.mark.parametrize("form", list(FORMS))
def test_fdfb_exact_noise_free(c1x, form):
    ctx, ok = c1x
    p = W.exact(W.C1)
    lut = W.named_luts(p.t)["square"]
    lid = ctx.register_lut(lut)
    msgs = np.arange(p.t, dtype=np.uint32)
    cts = ctx.encrypt_debug(msgs, seed=8)
    say(f"fdfb C1-exact {form}")
    out = _bootstrap(ctx, cts, [lid] * p.t, FORMS[form], p.n + 1)
    r0, r1 = oracle.setup_polynomial(lut, p.N)
    ref = np.stack([oracle.fdfb(ok, r0, r1, cts[k]) for k in range(p.t)])
    assert np.array_equal(out, ref)
    delta = M32 // p.t
    for k in range(p.t):
        assert oracle.phase(out[k], ok.s) == (delta * int(lut[k])) % M32


def test_batch_invariance_and_empty(c1):
    ctx, _ = c1
    p = W.C1
    lid = ctx.register_lut(W.random_lut(5, p.t))
    msgs = W.messages(17, 9, p.t)
    cts = ctx.encrypt_debug(msgs, seed=17)
    say("fdfb C1 batch invariance")
    full = _bootstrap(ctx, cts, [lid] * 9, 0, p.n + 1)
    for k in (0, 4, 8):
        alone = _bootstrap(ctx, cts[k:k + 1], [lid], 0, p.n + 1)
        assert np.array_equal(alone[0], full[k])
    ctx.bootstrap_batch(empty(0, p.n + 1), empty(0), empty(0, p.n + 1))
    assert ctx.device_errors() == 0
    bad = _bootstrap(ctx, cts[:2], [lid, 999], 0, p.n + 1)
    assert np.array_equal(bad[0], full[0])
    assert ctx.device_errors() == fd.DEVERR_LUT_ID  # the unknown id is reported ...
    assert ctx.device_errors() == 0                  # ... once (read clears)
    # the sample's accumulator is all zero before the function rotation
    acc = torch.zeros((1, 2 * p.N), dtype=torch.int32, device="cuda")
    ctx.pubmux(empty(1, p.boot_ell, 2 * p.N).zero_(), empty(1, p.n + 1).zero_(),
               torch.tensor([-1], dtype=torch.int32, device="cuda"), acc)
    torch.cuda.synchronize()
    assert not fd.to_host(acc).any() and ctx.device_errors() == fd.DEVERR_LUT_ID


def test_lincomb2(c1):
    g = np.random.default_rng(12)
    x, y = u32(g, 13, 65), u32(g, 13, 65)
    say("lincomb2 13x65")
    for wx, wy in ((1, -1), (3, 7), (-8, 0), (0x7FFFFFFF, -(1 << 31))):
        out = fd.to_host(fd.lincomb2(fd.to_device(x), fd.to_device(y), wx, wy, empty(13, 65)))
        torch.cuda.synchronize()
        ref = oracle.affine(np.array([[wx, wy]]), np.stack([x.reshape(-1), y.reshape(-1)]))[0].reshape(13, 65)
        assert np.array_equal(out, ref), (wx, wy)


def test_valu_keyswitch_base_above_2_7(oracle_keys_c1):
    """Key-switching bases above 2^7 take the VALU key switch (the MFMA one
    needs digits below 2^7): both switches and a full bootstrap against the
    oracle, bit for bit."""
    p = W.C1.with_(ks_log2B=8, ks_ell=3, pk_log2B=9, pk_ell=2)
    seed = W.KEY_SEED["C1"] + 5
    ctx, ok = fd.Context.keygen(p, seed), oracle.keygen(p, seed)
    lwe = u32(np.random.default_rng(15), 23, p.N + 1)
    say("VALU keyswitch / packing keyswitch C1 (2^8 x 3, 2^9 x 2) B=23")
    d = fd.to_device(lwe)
    ks = fd.to_host(ctx.keyswitch(d, empty(23, p.n + 1)))
    pk = fd.to_host(ctx.packing_keyswitch(d, empty(23, 2 * p.N)))
    torch.cuda.synchronize()
    for b in range(23):
        assert np.array_equal(ks[b], oracle.keyswitch(lwe[b], ok.ksk, p.ks_log2B, p.ks_ell, p.n + 1)), b
        assert np.array_equal(pk[b], oracle.keyswitch(lwe[b], ok.pk, p.pk_log2B, p.pk_ell, 2 * p.N)), b
    lut = W.random_lut(21, p.t)
    lid = ctx.register_lut(lut)
    msgs = np.arange(p.t, dtype=np.uint32)
    cts = ctx.encrypt_debug(msgs, seed=22)
    out = _bootstrap(ctx, cts, [lid] * p.t, 0, p.n + 1)
    r0, r1 = oracle.setup_polynomial(lut, p.N)
    ref = np.stack(run_oracle_many(lambda k: oracle.fdfb(ok, r0, r1, cts[k]), p.t))
    assert np.array_equal(out, ref)
    assert np.array_equal(ctx.decrypt_debug(out)[0], lut[msgs])


@pytest.mark.parametrize("form", list(FORMS))
def test_blind_rotate_c2(c2, form):
    ctx, ok = c2
    p = W.C2
    N = p.N
    g = np.random.default_rng(12)
    A = 5
    acc = u32(g, A, 2 * N)
    ctN = g.integers(0, 2 * N, (A, p.n + 1)).astype(np.uint32)
    say(f"blind_rotate C2 {form} A={A}")
    d_acc = fd.to_device(acc)
    ctx.blind_rotate(d_acc, fd.to_device(ctN), 1, FORMS[form])
    torch.cuda.synchronize()
    got = fd.to_host(d_acc)
    refs = run_oracle_many(lambda a: oracle.blind_rotate(p, ok.brk, ctN[a], acc[a]), A)
    for a in range(A):
        assert np.array_equal(got[a], refs[a]), a


def test_blind_rotate_c2_full_and_short_rounds(c2):
    """One rotation over a round that fills the device (on MI355X the
    two-wavefronts-per-SIMD kernel) and a short second round (the
    one-wavefront kernel), two accumulators per sample: every accumulator
    equals the plain VALU form bit for bit, and those at the round boundary
    and the ends match the oracle."""
    ctx, ok = c2
    p = W.C2
    N = p.N
    R = _resident_capacity(ctx)
    per = 2
    A = R + 6
    assert ctx.br_launches(A, per) == 2
    g = np.random.default_rng(41)
    acc = u32(g, A, 2 * N)
    ctN = g.integers(0, 2 * N, (A // per, p.n + 1)).astype(np.uint32)
    say(f"blind_rotate C2 rounds A={A} R={R}")
    d_acc, d_ref = fd.to_device(acc), fd.to_device(acc)
    d_ct = fd.to_device(ctN)
    ctx.blind_rotate(d_acc, d_ct, per, 0)
    ctx.blind_rotate(d_ref, d_ct, per, fd.PLAIN)
    torch.cuda.synchronize()
    got = fd.to_host(d_acc)
    assert np.array_equal(got, fd.to_host(d_ref))
    picks = [0, R - 1, R, A - 1]
    refs = run_oracle_many(lambda k: oracle.blind_rotate(p, ok.brk, ctN[picks[k] // per], acc[picks[k]]), len(picks))
    for k, a in enumerate(picks):
        assert np.array_equal(got[a], refs[k]), a


@pytest.mark.parametrize("A,zeros", [(2048, 0.5), (1500, 0.05), (512, 0.3), (96, 0.0)])
def test_blind_rotate_c2_skips_and_partial_round(c2, A, zeros):
    """Rounds of the N = 1024 kernel forms with skipped steps: a share of the
    a_i are 0, and the last 3 of every row, so the key prefetch of the final
    live step stops short of the end.  2048 and 1500 accumulators run one
    wavefront per accumulator, two per SIMD (1500 leaves some SIMDs with
    one); 512 and 96 run two wavefronts per accumulator.  Every accumulator
    equals the plain form; a few match the oracle."""
    ctx, ok = c2
    p = W.C2
    N = p.N
    per = 2
    g = np.random.default_rng(43)
    acc = u32(g, A, 2 * N)
    ctN = g.integers(0, 2 * N, (A // per, p.n + 1)).astype(np.uint32)
    ctN[:, 1:][g.random((A // per, p.n)) < zeros] = 0
    ctN[:, -3:] = 0
    say(f"blind_rotate C2 skips A={A} zeros={zeros}")
    d_acc, d_ref = fd.to_device(acc), fd.to_device(acc)
    d_ct = fd.to_device(ctN)
    ctx.blind_rotate(d_acc, d_ct, per, 0)
    ctx.blind_rotate(d_ref, d_ct, per, fd.PLAIN)
    torch.cuda.synchronize()
    got = fd.to_host(d_acc)
    assert np.array_equal(got, fd.to_host(d_ref))
    picks = [0, A // 2 + 1, A - 1]
    refs = run_oracle_many(lambda k: oracle.blind_rotate(p, ok.brk, ctN[picks[k] // per], acc[picks[k]]), len(picks))
    for k, a in enumerate(picks):
        assert np.array_equal(got[a], refs[k]), a


def test_fdfb_c2_full_batch(c2):
    """The headline configuration at its full size: 1024 samples, one random
    LUT.  Sampled outputs are recomputed one by one by the oracle; every output
    must decrypt to f(m); batched and plain forms must agree on every bit."""
    ctx, ok = c2
    p = W.C2
    B = 1024
    lut = W.random_lut(W.LUT_SEED["C2"], p.t)
    lid = ctx.register_lut(lut)
    msgs = W.messages(W.MSG_SEED["C2"], B, p.t)
    cts = ctx.encrypt_debug(msgs, seed=W.MSG_SEED["C2"])
    say("fdfb C2 batched B=1024")
    out = _bootstrap(ctx, cts, [lid] * B, 0, p.n + 1)
    m, err = ctx.decrypt_debug(out)
    assert np.array_equal(m, lut[msgs])
    r0, r1 = oracle.setup_polynomial(lut, p.N)
    # 128 samples: both ends, the middle, and a seeded spread over the batch
    sample = sorted({0, 1, 511, 512, 1022, 1023} |
                    set(np.random.default_rng(64).choice(np.setdiff1d(np.arange(2, 1022), [511, 512]), 122,
                                                         replace=False).tolist()))
    say(f"oracle on {len(sample)} samples")
    refs = run_oracle_many(lambda k: oracle.fdfb(ok, r0, r1, cts[sample[k]]), len(sample))
    for k, idx in enumerate(sample):
        assert np.array_equal(out[idx], refs[k]), idx
    say("fdfb C2 plain B=1024")
    outp = _bootstrap(ctx, cts, [lid] * B, fd.PLAIN, p.n + 1)
    assert np.array_equal(outp, out)


def test_fdfb_c2_large_batch_4096(c2):
    """A batch four times the headline size (8192 sign and 4096 function
    accumulators, several launch rounds or queue items per phase) with eight
    tables: every output decrypts to its table's value, the first 1024 rows
    equal the same samples bootstrapped alone as one batch, and sampled rows
    from every quarter match the oracle bit for bit."""
    ctx, ok = c2
    p = W.C2
    B = 4096
    tables = [W.random_lut(W.LUT_SEED["C2"] * 10 + j, p.t) for j in range(8)]
    lids = np.array([ctx.register_lut(tb) for tb in tables], dtype=np.int32)
    which = np.random.default_rng(4096).integers(0, 8, B)
    msgs = W.messages(W.MSG_SEED["C2"] + 9, B, p.t)
    cts = ctx.encrypt_debug(msgs, seed=W.MSG_SEED["C2"] + 9)
    say("fdfb C2 batched B=4096, 8 tables")
    out = _bootstrap(ctx, cts, lids[which], 0, p.n + 1)
    m, _ = ctx.decrypt_debug(out)
    assert np.array_equal(m, np.array([tables[w][x] for w, x in zip(which, msgs)]))
    assert ctx.device_errors() == 0
    part = _bootstrap(ctx, cts[:1024], lids[which[:1024]], 0, p.n + 1)
    assert np.array_equal(part, out[:1024])
    sample = [0, 1500, 2047, 2048, 3100, 4095]
    rots = {w: oracle.setup_polynomial(tables[w], p.N) for w in set(which[sample].tolist())}
    say(f"oracle on {len(sample)} samples")
    refs = run_oracle_many(lambda k: oracle.fdfb(ok, *rots[which[sample[k]]], cts[sample[k]]), len(sample))
    for k, idx in enumerate(sample):
        assert np.array_equal(out[idx], refs[k]), idx


@pytest.mark.skipif(os.environ.get("FDFB_FULL_PARITY") != "1",
                    reason="all 1024 samples through the oracle take several minutes of host time; "
                           "set FDFB_FULL_PARITY=1 to run")
def test_fdfb_c2_all_1024_vs_oracle(c2):
    """Every output of the headline batch against the oracle, bit for bit."""
    ctx, ok = c2
    p = W.C2
    B = 1024
    lut = W.random_lut(W.LUT_SEED["C2"], p.t)
    lid = ctx.register_lut(lut)
    msgs = W.messages(W.MSG_SEED["C2"], B, p.t)
    cts = ctx.encrypt_debug(msgs, seed=W.MSG_SEED["C2"])
    out = _bootstrap(ctx, cts, [lid] * B, 0, p.n + 1)
    rot = [oracle.setup_polynomial(lut, p.N)]
    for lo in range(0, B, 128):
        ref = oracle.fdfb_batch(ok, rot, np.zeros(128, int), cts[lo:lo + 128], threads=16)
        bad = np.nonzero((ref != out[lo:lo + 128]).any(axis=1))[0]
        say(f"oracle samples {lo}..{lo + 127}: {len(bad)} mismatches")
        assert len(bad) == 0, (lo + bad[:8]).tolist()


# ----------------------------------------------------------------------------
# ring degree 2048 (two wavefronts per output component, chunked key stream)
# ----------------------------------------------------------------------------
N2048 = {"C3B": W.C3B, "C4": W.C4}


@pytest.fixture(scope="module")
def keys_2048():
    cache = {}

    def get(name):
        if name not in cache:
            p = N2048[name]
            cache[name] = (fd.Context.keygen(p, W.KEY_SEED[name]), oracle.keygen(p, W.KEY_SEED[name]))
        return cache[name]
    return get


@pytest.mark.parametrize("form", ["batched", "direct", "plain"])
@pytest.mark.parametrize("name", list(N2048))
def test_blind_rotate_n2048(keys_2048, name, form):
    if form == "plain" and name == "C4":
        pytest.skip("the plain kernel's LDS cannot hold C4's key rows (N = 2048, ell = 4)")
    ctx, ok = keys_2048(name)
    p = N2048[name]
    N = p.N
    g = np.random.default_rng(31)
    A, per = 6, 2
    acc = u32(g, A, 2 * N)
    ctN = g.integers(0, 2 * N, (A // per, p.n + 1)).astype(np.uint32)
    say(f"blind_rotate {name} {form} A={A}")
    d_acc = fd.to_device(acc)
    ctx.blind_rotate(d_acc, fd.to_device(ctN), per, FORMS[form])
    torch.cuda.synchronize()
    got = fd.to_host(d_acc)
    refs = run_oracle_many(lambda a: oracle.blind_rotate(p, ok.brk, ctN[a // per], acc[a]), A)
    for a in range(A):
        assert np.array_equal(got[a], refs[a]), a


def _resident_capacity(ctx):
    """Accumulators one launch of the batched form holds (largest A taking
    one launch), found from the launch count alone."""
    lo, hi = 1, 1 << 22
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if ctx.br_launches(mid, 1) == 1:
            lo = mid
        else:
            hi = mid - 1
    return lo


def test_blind_rotate_rounds_split_samples(keys_2048):
    """Three accumulators per sample over more than one launch round: a round
    may begin inside a sample's group, so every accumulator must still read
    its own sample's row.  Every accumulator equals the rotation with the row
    repeated per accumulator (one per sample); the ones at each round
    boundary match the oracle bit for bit.  The short last round runs the
    split form (eight wavefronts per accumulator)."""
    ctx, ok = keys_2048("C3B")
    p = W.C3B
    N = p.N
    cap = _resident_capacity(ctx)
    per = 3
    A = per * (cap // per + 2)
    assert ctx.br_launches(A, per) == ctx.br_launches(A, 1) == (A + cap - 1) // cap >= 2
    g = np.random.default_rng(37)
    acc = u32(g, A, 2 * N)
    ctN = g.integers(0, 2 * N, (A // per, p.n + 1)).astype(np.uint32)
    say(f"blind_rotate C3B rounds A={A} cap={cap}")
    d_acc = fd.to_device(acc)
    ctx.blind_rotate(d_acc, fd.to_device(ctN), per, 0)
    d_rep = fd.to_device(acc)
    ctx.blind_rotate(d_rep, fd.to_device(np.repeat(ctN, per, axis=0)), 1, 0)
    torch.cuda.synchronize()
    got, rep = fd.to_host(d_acc), fd.to_host(d_rep)
    assert np.array_equal(got, rep)
    picks = sorted({0, cap - 2, cap - 1, cap, cap + 1, A - 1})
    refs = run_oracle_many(lambda k: oracle.blind_rotate(p, ok.brk, ctN[picks[k] // per], acc[picks[k]]),
                           len(picks))
    for k, a in enumerate(picks):
        assert np.array_equal(got[a], refs[k]), a


def test_split_form_rounds_inside_samples(keys_2048):
    """The split form forced in rounds of 100 accumulators at three per sample
    (every round boundary inside a sample): bit-identical to the default
    plan, and the accumulators at the boundaries match the oracle."""
    ctx, ok = keys_2048("C3B")
    p = W.C3B
    N = p.N
    per, A = 3, 210
    g = np.random.default_rng(38)
    acc = u32(g, A, 2 * N)
    ctN = g.integers(0, 2 * N, (A // per, p.n + 1)).astype(np.uint32)
    say("blind_rotate C3B split form, rounds of 100")
    ctx.set_plan(A, 5, 100)
    try:
        assert ctx.br_launches(A, per) == 3
        d_split = fd.to_device(acc)
        ctx.blind_rotate(d_split, fd.to_device(ctN), per, 0)
    finally:
        ctx.set_plan(A, None)
    d_ref = fd.to_device(acc)
    ctx.blind_rotate(d_ref, fd.to_device(ctN), per, 0)
    torch.cuda.synchronize()
    got = fd.to_host(d_split)
    assert np.array_equal(got, fd.to_host(d_ref))
    picks = [99, 100, 199, 200, 209]
    refs = run_oracle_many(lambda k: oracle.blind_rotate(p, ok.brk, ctN[picks[k] // per], acc[picks[k]]),
                           len(picks))
    for k, a in enumerate(picks):
        assert np.array_equal(got[a], refs[k]), a


@pytest.mark.parametrize("form", ["batched", "plain"])
def test_fdfb_n2048_vs_oracle(keys_2048, form):
    ctx, ok = keys_2048("C3B")
    p = W.C3B
    lut = W.random_lut(W.LUT_SEED["C3B"], p.t)
    lid = ctx.register_lut(lut)
    msgs = np.array([0, 1, p.t // 2, p.t - 1, 7, 19, 25, 30], dtype=np.uint32)
    cts = ctx.encrypt_debug(msgs, seed=W.MSG_SEED["C3B"])
    say(f"fdfb C3B {form} B=8")
    out = _bootstrap(ctx, cts, [lid] * len(msgs), FORMS[form], p.n + 1)
    m, _ = ctx.decrypt_debug(out)
    assert np.array_equal(m, lut[msgs])
    r0, r1 = oracle.setup_polynomial(lut, p.N)
    refs = run_oracle_many(lambda k: oracle.fdfb(ok, r0, r1, cts[k]), len(msgs))
    for k in range(len(msgs)):
        assert np.array_equal(out[k], refs[k]), k


def test_trace_env_prints_phase_times(capfd, monkeypatch):
    """FDFB_TRACE at context creation: the phase timings of its bootstrap
    calls are printed to stderr when the context is freed."""
    monkeypatch.setenv("FDFB_TRACE", "1")
    p = W.C1
    ctx = fd.Context.keygen(p, W.KEY_SEED["C1"])
    lid = ctx.register_lut(W.random_lut(W.LUT_SEED["C1"], p.t))
    cts = ctx.encrypt_debug(W.messages(W.MSG_SEED["C1"], 8, p.t), seed=W.MSG_SEED["C1"])
    for _ in range(2):
        _bootstrap(ctx, cts, [lid] * 8, 0, p.n + 1)
    ctx.free()
    err = capfd.readouterr().err
    assert "fdfb trace: 2 bootstrap calls" in err and "function_br" in err, err[-500:]


def test_measure_mfma_peak():
    """The calibration stream runs and reports a rate no higher than the
    device's published dense int8 peak (5.0 POPS) allows."""
    tops, ms = fd.measure_mfma_peak()
    say(f"int8 MFMA stream: {tops:.0f} TOPS in {ms:.1f} ms")
    assert ms > 0 and 0 < tops <= 1.05 * 5000


def test_br_launch_count(c2):
    """The batched form runs in rounds of the resident capacity (a round may
    split a sample's accumulators, so the count does not depend on how many
    each sample has); the plain form in one launch; nothing for no
    accumulators."""
    ctx = c2[0]
    assert ctx.br_launches(0, 2) == 0
    one = ctx.br_launches(2, 2)
    assert one == 1
    many = ctx.br_launches(1 << 16, 2)
    assert many >= 2
    for A in (1, 999, 1000, 4097, 1 << 16):
        assert len({ctx.br_launches(A, per) for per in (1, 2, 3, 5)}) == 1, A
    assert ctx.br_launches(1 << 16, 2, flags=fd.PLAIN) == 1
    assert ctx.br_launches(1 << 16, 2, flags=fd.DIRECT) == 1
    with pytest.raises(fd.FdfbError):
        ctx.br_launches(4, 0)
    with pytest.raises(fd.FdfbError):
        ctx.br_launches(4, 2, flags=fd.PLAIN | fd.DIRECT)


@pytest.mark.parametrize("flags", [0, fd.OUT_EXTRACTED])
def test_multi_lut_shares_sign_rotations(c1, flags):
    """Several tables per sample (sign accumulators reused): every output is
    bit-identical to the single-table bootstrap of that sample and table, and
    decrypts to the table's value."""
    ctx, ok = c1
    p = W.C1
    L = 3
    tables = [W.random_lut(900 + l, p.t) for l in range(L)]
    lids = [ctx.register_lut(tb) for tb in tables]
    msgs = np.arange(p.t, dtype=np.uint32).repeat(2)
    B = len(msgs)
    cts = fd.to_device(ctx.encrypt_debug(msgs, seed=77))
    rng = np.random.default_rng(5)
    pick = rng.integers(0, L, (B, L)).astype(np.int32)  # a table per (sample, slot), repeats allowed
    ids = torch.from_numpy(np.array(lids, dtype=np.int32)[pick]).cuda()
    dim = (p.N if flags else p.n) + 1
    out = torch.zeros((B, L, dim), dtype=torch.int32, device="cuda")
    ctx.bootstrap_multi_lut(cts, ids, out, flags)
    torch.cuda.synchronize()
    got = fd.to_host(out)
    for l in range(L):
        single = torch.zeros((B, dim), dtype=torch.int32, device="cuda")
        ctx.bootstrap_batch(cts, ids[:, l].contiguous(), single, flags)
        torch.cuda.synchronize()
        assert np.array_equal(fd.to_host(single), got[:, l, :]), l
        if not flags:
            m, _ = ctx.decrypt_debug(got[:, l, :])
            want = np.array([tables[pick[b, l]][msgs[b]] for b in range(B)])
            assert np.array_equal(m, want), l
    # one output against the oracle, bit for bit
    b, l = 5, 2
    r0, r1 = oracle.setup_polynomial(tables[pick[b, l]], p.N)
    ref = oracle.fdfb(ok, r0, r1, fd.to_host(cts)[b], flags=oracle.OUT_EXTRACTED if flags else 0)
    assert np.array_equal(got[b, l], ref)


def test_multi_lut_c2_and_errors(c2):
    ctx, _ = c2
    p = W.C2
    L, B = 4, 64
    tables = [W.random_lut(950 + l, p.t) for l in range(L)]
    lids = np.array([ctx.register_lut(tb) for tb in tables], dtype=np.int32)
    msgs = W.messages(123, B, p.t)
    cts = fd.to_device(ctx.encrypt_debug(msgs, seed=124))
    ids = torch.from_numpy(np.tile(lids, (B, 1))).cuda()
    out = torch.zeros((B, L, p.n + 1), dtype=torch.int32, device="cuda")
    ctx.bootstrap_multi_lut(cts, ids, out)
    torch.cuda.synchronize()
    got = fd.to_host(out)
    for l in range(L):
        single = torch.zeros((B, p.n + 1), dtype=torch.int32, device="cuda")
        ctx.bootstrap_batch(cts, ids[:, l].contiguous(), single)
        torch.cuda.synchronize()
        assert np.array_equal(fd.to_host(single), got[:, l, :]), l
        assert np.array_equal(ctx.decrypt_debug(got[:, l, :])[0], tables[l][msgs]), l
    with pytest.raises(fd.FdfbError):
        ctx.bootstrap_multi_lut(cts, ids[:, :0].contiguous(), out)  # L = 0
    ctx.bootstrap_multi_lut(cts[:0], ids[:0], out[:0])  # B = 0 is a no-op


def test_signed_boot_digit_c1_vs_oracle(oracle_keys_c1):
    """Variant with one signed public-mux digit (one sign rotation): bit for
    bit against the oracle, both forms, and full-domain decryption."""
    p = W.signed_boot(W.C1)
    ctx = fd.Context.keygen(p, W.KEY_SEED["C1"])
    ok = dataclasses.replace(oracle_keys_c1, params=p)
    lut = W.random_lut(W.LUT_SEED["C1"] + 5, p.t)
    lid = ctx.register_lut(lut)
    msgs = np.arange(p.t, dtype=np.uint32).repeat(2)
    cts = ctx.encrypt_debug(msgs, seed=31)
    r0, r1 = oracle.setup_polynomial(lut, p.N)
    refs = np.stack([oracle.fdfb(ok, r0, r1, c) for c in cts])
    for flags in (0, fd.PLAIN):
        out = torch.zeros((len(msgs), p.n + 1), dtype=torch.int32, device="cuda")
        ctx.bootstrap_batch(fd.to_device(cts), torch.full((len(msgs),), lid, dtype=torch.int32, device="cuda"),
                            out, flags)
        torch.cuda.synchronize()
        got = fd.to_host(out)
        assert np.array_equal(got, refs), flags
        assert np.array_equal(ctx.decrypt_debug(got)[0], lut[msgs])


def test_signed_boot_digit_c2_batch(c2):
    """The variant at configuration 2 on a full batch: every sample decrypts
    to f(m); sampled outputs match the oracle bit for bit; the sign phase
    runs one rotation per sample."""
    _, okc2 = c2
    p = W.signed_boot(W.C2)
    ctx = fd.Context.keygen(p, W.KEY_SEED["C2"])
    ok = dataclasses.replace(okc2, params=p)
    lut = W.random_lut(W.LUT_SEED["C2"] + 5, p.t)
    lid = ctx.register_lut(lut)
    B = 1024
    msgs = W.messages(W.MSG_SEED["C2"] + 5, B, p.t)
    cts = ctx.encrypt_debug(msgs, seed=W.MSG_SEED["C2"] + 5)
    out = torch.zeros((B, p.n + 1), dtype=torch.int32, device="cuda")
    ctx.bootstrap_batch(fd.to_device(cts), torch.full((B,), lid, dtype=torch.int32, device="cuda"), out)
    torch.cuda.synchronize()
    got = fd.to_host(out)
    assert np.array_equal(ctx.decrypt_debug(got)[0], lut[msgs])
    r0, r1 = oracle.setup_polynomial(lut, p.N)
    for k in (0, 511, 1023):
        assert np.array_equal(got[k], oracle.fdfb(ok, r0, r1, cts[k])), k
    assert ctx.br_launches(B * p.boot_ell, p.boot_ell) == ctx.br_launches(B, 1)


@pytest.mark.parametrize("form", ["batched", "plain"])
def test_tfhe_half_domain_vs_oracle(c1, form):
    """The one-rotation TFHE-style bootstrap on the same kernels: bit for bit
    against the oracle, and the half-domain behaviour it has by construction."""
    ctx, ok = c1
    p = W.C1
    t, delta = p.t, M32 // p.t
    lut = W.random_lut(61, t)
    lid = ctx.register_lut(lut)
    msgs = np.arange(t, dtype=np.uint32).repeat(2)
    cts = ctx.encrypt_debug(msgs, seed=62)
    r0, _ = oracle.setup_polynomial(lut, p.N)
    scaled = ((r0.astype(np.int64) * delta) % M32).astype(np.uint32)
    flags = fd.PLAIN if form == "plain" else 0
    for extracted in (0, fd.OUT_EXTRACTED):
        dim = (p.N if extracted else p.n) + 1
        out = torch.zeros((len(msgs), dim), dtype=torch.int32, device="cuda")
        ctx.tfhe_bootstrap_batch(fd.to_device(cts), torch.full((len(msgs),), lid, dtype=torch.int32, device="cuda"),
                                 out, flags | extracted)
        torch.cuda.synchronize()
        got = fd.to_host(out)
        for k in (0, 5, 11, len(msgs) - 1):
            ref = oracle.tfhe_bootstrap(ok, scaled, cts[k], flags=oracle.OUT_EXTRACTED if extracted else 0)
            assert np.array_equal(got[k], ref), (extracted, k)
        if not extracted:
            m, _ = ctx.decrypt_debug(got)
            for k, x in enumerate(msgs):
                if x in (0, t // 2):
                    continue  # on the wrap of the half-domain encoding
                want = lut[x] if x < t // 2 else (-int(lut[x - t // 2])) % t
                assert m[k] == want, (k, x)
