"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test checks one oracle function against an independent statement of the
paper or of plain mathematics: brute-force polynomial reduction, exact big
integer rounding, the exact identities of sample extraction and key
switching, the noise-free limit of the external product / CMux / blind
rotation / public mux / full bootstrap, the exhaustive statement of the
rotation-polynomial theorem, full-domain decryption with real noise, and the
measured noise variance against the error analysis.
"""
from fractions import Fraction

import dataclasses

import numpy as np
import pytest

import oracle
import workloads as W

M32 = 1 << 32


# ----------------------------------------------------------------------------
# independent helpers (plain Python integers)
# ----------------------------------------------------------------------------
def brute_negacyclic(a, b):
    """Full product, then reduce with X^N = -1."""
    N = len(a)
    full = [0] * (2 * N)
    for i in range(N):
        for j in range(N):
            full[i + j] += int(a[i]) * int(b[j])
    return np.array([(full[k] - full[k + N]) % M32 for k in range(N)], dtype=np.uint32)


def monomial_poly(e, N):
    """X^e as a coefficient vector mod 2^32 (X^N = -1)."""
    e %= 2 * N
    p = [0] * N
    if e < N:
        p[e] = 1
    else:
        p[e - N] = M32 - 1
    return np.array(p, dtype=np.uint32)


def rlwe_phase(ct, key):
    N = len(key)
    b, a = ct[:N], ct[N:]
    ak = brute_negacyclic(a, key)
    return ((b.astype(np.int64) - ak.astype(np.int64)) % M32).astype(np.uint32)


def lwe_phase(ct, key):
    return int((int(ct[0]) - sum(int(x) * int(k) for x, k in zip(ct[1:], key))) % M32)


def rnd(seed):
    return np.random.default_rng(seed)


# ----------------------------------------------------------------------------
# ring arithmetic
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("N", [1, 2, 4, 8, 16, 64])
def test_negacyclic_matches_bruteforce(N):
    g = rnd(N)
    for _ in range(3):
        a = g.integers(0, M32, N, dtype=np.uint64).astype(np.uint32)
        b = g.integers(0, M32, N, dtype=np.uint64).astype(np.uint32)
        assert np.array_equal(oracle.negacyclic_mul(a, b), brute_negacyclic(a, b))


@pytest.mark.parametrize("N", [4, 16, 64])
def test_monomial_group_of_order_2N(N):
    g = rnd(100 + N)
    p = g.integers(0, M32, N, dtype=np.uint64).astype(np.uint32)
    neg = ((M32 - p.astype(np.int64)) % M32).astype(np.uint32)
    assert np.array_equal(oracle.monomial_mul(p, N), neg)          # X^N = -1
    assert np.array_equal(oracle.monomial_mul(p, 0), p)
    for e in g.integers(0, 2 * N, 6):
        e = int(e)
        assert np.array_equal(oracle.monomial_mul(p, e), brute_negacyclic(p, monomial_poly(e, N)))
        f = int(g.integers(0, 2 * N))
        assert np.array_equal(oracle.monomial_mul(oracle.monomial_mul(p, e), f),
                              oracle.monomial_mul(p, (e + f) % (2 * N)))


# ----------------------------------------------------------------------------
# decomposition, modulus switching
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("log2B,ell", [(8, 2), (7, 3), (10, 2), (4, 5), (4, 8), (8, 4), (2, 2)])
def test_decomp_reconstructs_rounded_value(log2B, ell):
    g = rnd(log2B * 10 + ell)
    drop = 32 - log2B * ell
    L = 1 << log2B
    xs = [0, 1, M32 - 1, (1 << 31), (1 << drop) // 2 if drop else 7, M32 - (1 << drop) // 2 if drop else 9]
    xs += [int(v) for v in g.integers(0, M32, 200, dtype=np.uint64)]
    for x in xs:
        d = oracle.decomp(x, log2B, ell)
        assert all(0 <= int(v) < L for v in d)
        recon = sum(int(d[j]) * (1 << drop) * L ** j for j in range(ell)) % M32
        # nearest multiple of 2^drop, ties up, reduced mod 2^32
        want = (int(Fraction(x, 1 << drop) + Fraction(1, 2)) << drop) % M32 if drop else x
        assert recon == want
        err = (x - recon + M32 // 2) % M32 - M32 // 2
        assert abs(err) <= (1 << drop) // 2


@pytest.mark.parametrize("log2_q", [9, 11, 12, 16])
def test_modswitch_is_exact_rounding(log2_q):
    g = rnd(log2_q)
    sh = 32 - log2_q
    xs = [0, M32 - 1, (1 << sh) // 2, (1 << sh) // 2 - 1, 3 * (1 << sh) // 2]
    xs += [int(v) for v in g.integers(0, M32, 300, dtype=np.uint64)]
    for x in xs:
        want = int(Fraction(x * (1 << log2_q), M32) + Fraction(1, 2)) % (1 << log2_q)
        assert oracle.modswitch(x, log2_q) == want


# ----------------------------------------------------------------------------
# sample extraction and key switching (exact identities)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("N", [8, 32, 64])
def test_sample_extract_phase_identity(N):
    g = rnd(7 * N)
    key = g.integers(0, 2, N).astype(np.uint32)
    for _ in range(4):
        ct = g.integers(0, M32, 2 * N, dtype=np.uint64).astype(np.uint32)
        lwe = oracle.sample_extract(ct)
        assert lwe_phase(lwe, key) == int(rlwe_phase(ct, key)[0])


def test_keyswitch_noise_free_preserves_phase(oracle_keys_c1_exact):
    k = oracle_keys_c1_exact
    p = W.exact(W.C1)
    g = rnd(11)
    for _ in range(3):
        ct = g.integers(0, M32, p.N + 1, dtype=np.uint64).astype(np.uint32)
        out = oracle.keyswitch(ct, k.ksk, p.ks_log2B, p.ks_ell, p.n + 1)
        assert lwe_phase(out, k.s) == lwe_phase(ct, k.sf)
        r = oracle.keyswitch(ct, k.pk, p.pk_log2B, p.pk_ell, 2 * p.N)
        ph = rlwe_phase(r, k.sf)
        assert int(ph[0]) == lwe_phase(ct, k.sf)
        assert not ph[1:].any()


def test_keyswitch_error_within_bound(oracle_keys_c1):
    k = oracle_keys_c1
    p = W.C1
    g = rnd(12)
    errs = []
    for _ in range(20):
        ct = g.integers(0, M32, p.N + 1, dtype=np.uint64).astype(np.uint32)
        out = oracle.keyswitch(ct, k.ksk, p.ks_log2B, p.ks_ell, p.n + 1)
        e = (lwe_phase(out, k.s) - lwe_phase(ct, k.sf) + M32 // 2) % M32 - M32 // 2
        errs.append(e)
    # predicted variance: N*ell*E[d^2]*sigma^2 + rounding of the dropped bits
    L = 1 << p.ks_log2B
    Eu = (L - 1) * (2 * L - 1) / 6
    drop = 32 - p.ks_ell * p.ks_log2B
    var = p.N * p.ks_ell * Eu * p.sigma_ks ** 2 + (4 ** drop / 12) * int(k.sf.sum())
    assert np.max(np.abs(errs)) < 6 * np.sqrt(var)


# ----------------------------------------------------------------------------
# external product, CMux, blind rotation: noise-free limit
# ----------------------------------------------------------------------------
def test_extprod_and_cmux_noise_free(oracle_keys_c1_exact):
    k = oracle_keys_c1_exact
    p = W.exact(W.C1)
    N = p.N
    g = rnd(21)
    for i in range(4):
        Cm = k.brk[i]
        d = g.integers(0, M32, 2 * N, dtype=np.uint64).astype(np.uint32)
        h = g.integers(0, M32, 2 * N, dtype=np.uint64).astype(np.uint32)
        out = oracle.extprod(Cm, d, p.g_log2B, p.g_ell)
        want = (rlwe_phase(d, k.sf).astype(np.int64) * int(k.s[i])) % M32
        assert np.array_equal(rlwe_phase(out, k.sf), want.astype(np.uint32))
        cm = oracle.cmux(Cm, d, h, p.g_log2B, p.g_ell)
        sel = d if k.s[i] else h
        assert np.array_equal(rlwe_phase(cm, k.sf), rlwe_phase(sel, k.sf))


def test_blind_rotate_noise_free_rotates_by_minus_a_dot_s(oracle_keys_c1_exact):
    k = oracle_keys_c1_exact
    p = W.exact(W.C1)
    N = p.N
    g = rnd(22)
    for _ in range(2):
        ctN = g.integers(0, 2 * N, p.n + 1).astype(np.uint32)
        acc = g.integers(0, M32, 2 * N, dtype=np.uint64).astype(np.uint32)
        out = oracle.blind_rotate(p, k.brk, ctN, acc)
        rot = (-int(np.dot(ctN[1:].astype(np.int64), k.s.astype(np.int64)))) % (2 * N)
        want = brute_negacyclic(rlwe_phase(acc, k.sf), monomial_poly(rot, N))
        assert np.array_equal(rlwe_phase(out, k.sf), want)


# ----------------------------------------------------------------------------
# rotation polynomials (exhaustive statement of the theorem)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("N,t", [(16, 2), (16, 4), (64, 8), (256, 8), (256, 16), (1024, 16)])
def test_setup_polynomial_exhaustive(N, t):
    lut = W.random_lut(N + t, t)
    p0, p1 = oracle.setup_polynomial(lut, N)
    step = 2 * N // t
    w = -(-N // t)
    owner = {}
    holders = {}
    for m in range(t):
        for e in range(-w, w + 1):
            y = (step * m + e) % (2 * N)
            owner[y] = m
            holders.setdefault(y, set()).add(m)
    for y in range(2 * N):
        poly = p0 if y < N else p1
        # coefficient 0 of poly * X^y over the integers: X^k with k = 0 or
        # k = N (mod 2N) lands on the constant term with sign +1 / -1
        c0 = 0
        for i in range(N):
            k = (i + y) % (2 * N)
            s = 1 if (i + y) % (2 * N) < N else -1
            if k % N == 0:
                c0 += s * int(poly[i])
        if y in owner:
            assert c0 == int(lut[owner[y]]), (y, holders[y])
            if len(holders[y]) == 1:
                assert c0 == int(lut[next(iter(holders[y]))])


# ----------------------------------------------------------------------------
# public mux: noise-free limit (Lemma "Correctness of Public Mux")
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("bit", [0, 1])
def test_pubmux_selects(bit):
    p = W.C1
    N, t = p.N, p.t
    delta = M32 // t
    L = 1 << p.boot_log2B
    g = rnd(31 + bit)
    key = g.integers(0, 2, N).astype(np.uint32)
    p0 = g.integers(-(t - 1), t, N).astype(np.int64)
    p1 = g.integers(-(t - 1), t, N).astype(np.int64)
    cs = []
    for i in range(p.boot_ell):
        a = g.integers(0, M32, N, dtype=np.uint64).astype(np.uint32)
        b = brute_negacyclic(a, key).astype(np.int64)
        b[0] += bit * delta * L ** i
        cs.append(np.concatenate([(b % M32).astype(np.uint32), a]))
    out = oracle.pubmux(p, np.stack(cs), p0, p1)
    sel = p1 if bit else p0
    assert np.array_equal(rlwe_phase(out, key), ((sel * delta) % M32).astype(np.uint32))


def test_pubmux_signed_digit_is_centred():
    """The single signed digit: muxing with the trivial sample [1, 0] leaves
    out - Delta p_0 = digit, which must be the representative of
    (p_1 - p_0) mod t in [-t/2, t/2) (an unsigned digit in [0, t) would also
    select correctly in the noise-free limit, so this pins the reading)."""
    p = W.signed_boot(W.C2)
    N, t = p.N, p.t
    delta = M32 // t
    g = rnd(41)
    p0 = g.integers(-(t - 1), t, N).astype(np.int64)
    p1 = g.integers(-(t - 1), t, N).astype(np.int64)
    c = np.zeros((1, 2 * N), np.uint32)
    c[0, 0] = 1  # b = 1, a = 0: a_i(X) * 1 is the digit polynomial itself
    out = oracle.pubmux(p, c, p0, p1).astype(np.int64)
    dig = (out[:N] - (p0 * delta) % M32) % M32
    dig = np.where(dig >= M32 // 2, dig - M32, dig)
    want = (p1 - p0) % t
    want = np.where(want >= t // 2, want - t, want)
    assert np.array_equal(dig, want)
    assert dig.min() >= -(t // 2) and dig.max() < t // 2 and (dig < 0).any()
    assert not out[N:].any()


# ----------------------------------------------------------------------------
# the full bootstrap
# ----------------------------------------------------------------------------
def _luts(t, seed):
    d = dict(W.named_luts(t))
    d["random"] = W.random_lut(seed, t)
    return d


def test_fdfb_noise_free_phase_is_exact(oracle_keys_c1_exact):
    k = oracle_keys_c1_exact
    p = W.exact(W.C1)
    t, delta = p.t, M32 // p.t
    msgs = np.arange(t, dtype=np.uint32)
    cts = oracle.encrypt(p, k.s, msgs, seed=5)
    for name, lut in _luts(t, 77).items():
        r0, r1 = oracle.setup_polynomial(lut, p.N)
        for m in range(t):
            out = oracle.fdfb(k, r0, r1, cts[m])
            assert lwe_phase(out, k.s) == (delta * int(lut[m])) % M32, (name, m)
            cq = oracle.fdfb(k, r0, r1, cts[m], flags=oracle.OUT_EXTRACTED)
            assert lwe_phase(cq, k.sf) == (delta * int(lut[m])) % M32, (name, m)


def test_fdfb_full_domain_c1(oracle_keys_c1):
    k = oracle_keys_c1
    p = W.C1
    t = p.t
    msgs = np.concatenate([np.arange(t), np.arange(t)]).astype(np.uint32)
    cts = oracle.encrypt(p, k.s, msgs, seed=W.MSG_SEED["C1"])
    for name, lut in _luts(t, W.LUT_SEED["C1"]).items():
        rot = [oracle.setup_polynomial(lut, p.N)]
        outs = oracle.fdfb_batch(k, rot, np.zeros(len(msgs), int), cts)
        m, err = oracle.decrypt(outs, k.s, p.log2_t)
        assert np.array_equal(m, lut[msgs]), name
        assert np.max(np.abs(err)) < (M32 // t) // 8


def test_fdfb_full_domain_c2(oracle_keys_c2):
    k = oracle_keys_c2
    p = W.C2
    t = p.t
    msgs = np.arange(t, dtype=np.uint32)
    cts = oracle.encrypt(p, k.s, msgs, seed=W.MSG_SEED["C2"])
    lut = W.random_lut(W.LUT_SEED["C2"], t)
    rot = [oracle.setup_polynomial(lut, p.N)]
    outs = oracle.fdfb_batch(k, rot, np.zeros(t, int), cts)
    m, err = oracle.decrypt(outs, k.s, p.log2_t)
    assert np.array_equal(m, lut[msgs])
    assert np.max(np.abs(err)) < (M32 // t) // 4


def test_signed_boot_digit_noise_free_exact(oracle_keys_c1_exact):
    """Variant with one signed public-mux digit: since Delta * t = 0 mod 2^32,
    the centred digit of (p_1 - p_0) mod t selects the same plaintext, so the
    noise-free output phase is still exactly Delta * f(m) for every m."""
    k = dataclasses.replace(oracle_keys_c1_exact, params=W.signed_boot(oracle_keys_c1_exact.params))
    p = k.params
    t, delta = p.t, M32 // p.t
    msgs = np.arange(t, dtype=np.uint32)
    cts = oracle.encrypt(p, k.s, msgs, seed=6)
    for name, lut in _luts(t, 78).items():
        r0, r1 = oracle.setup_polynomial(lut, p.N)
        for m in range(t):
            out = oracle.fdfb(k, r0, r1, cts[m])
            assert lwe_phase(out, k.s) == (delta * int(lut[m])) % M32, (name, m)


def test_signed_boot_digit_full_domain_c2(oracle_keys_c2):
    """The variant at configuration-2 noise: every m decrypts to f(m), and the
    PubMux stage dump differs from the unsigned reading (the digit is used)."""
    k = dataclasses.replace(oracle_keys_c2, params=W.signed_boot(oracle_keys_c2.params))
    p = k.params
    t = p.t
    msgs = np.arange(t, dtype=np.uint32)
    cts = oracle.encrypt(p, k.s, msgs, seed=W.MSG_SEED["C2"] + 1)
    lut = W.random_lut(W.LUT_SEED["C2"] + 1, t)
    rot = [oracle.setup_polynomial(lut, p.N)]
    outs = oracle.fdfb_batch(k, rot, np.zeros(t, int), cts)
    m, err = oracle.decrypt(outs, k.s, p.log2_t)
    assert np.array_equal(m, lut[msgs])
    assert np.max(np.abs(err)) < (M32 // t) // 4


def test_tfhe_half_domain_negates_upper_half(oracle_keys_c1):
    """The problem the paper fixes (Sec. 1.2): one rotation computes F only
    for m < t/2 and returns -F(m - t/2) on the upper half."""
    k = oracle_keys_c1
    p = W.C1
    t, N, delta = p.t, p.N, M32 // p.t
    lut = W.random_lut(9, t)
    r0, _ = oracle.setup_polynomial(lut, N)
    scaled = ((r0.astype(np.int64) * delta) % M32).astype(np.uint32)
    msgs = np.arange(t, dtype=np.uint32)
    cts = oracle.encrypt(p, k.s, msgs, seed=3)
    # m = 0 and m = t/2 sit on the wrap of the half-domain encoding, where
    # the sign of the noise decides between the two halves; skip them
    for m in [m for m in range(t) if m not in (0, t // 2)]:
        out = oracle.tfhe_bootstrap(k, scaled, cts[m])
        got, _ = oracle.decrypt(out, k.s, p.log2_t)
        want = lut[m] if m < t // 2 else (-int(lut[m - t // 2])) % t
        assert int(got[0]) == want


# ----------------------------------------------------------------------------
# noise against the error analysis
# ----------------------------------------------------------------------------
def test_blind_rotate_noise_variance(oracle_keys_c1):
    """Measured variance of the blind-rotation error vs the CMux / external
    product analysis (Sec. 2 lemmas) plus the rounding of the approximate
    gadget: n*2*ell*N*E[d^2]*sigma^2 + hw(s)*(1 + hw(sf))*2^(2 drop)/12."""
    k = oracle_keys_c1
    p = W.C1
    N = p.N
    g = rnd(41)
    errs = []
    for _ in range(6):
        ctN = g.integers(0, 2 * N, p.n + 1).astype(np.uint32)
        mu = g.integers(0, M32, N, dtype=np.uint64).astype(np.uint32)
        acc = np.concatenate([mu, np.zeros(N, np.uint32)])
        out = oracle.blind_rotate(p, k.brk, ctN, acc)
        rot = (-int(np.dot(ctN[1:].astype(np.int64), k.s.astype(np.int64)))) % (2 * N)
        want = brute_negacyclic(mu, monomial_poly(rot, N)).astype(np.int64)
        e = (rlwe_phase(out, k.sf).astype(np.int64) - want + M32 // 2) % M32 - M32 // 2
        errs.append(e)
    errs = np.concatenate(errs).astype(np.float64)
    L = 1 << p.g_log2B
    Eu = (L - 1) * (2 * L - 1) / 6
    drop = 32 - p.g_ell * p.g_log2B
    pred = p.n * 2 * p.g_ell * N * Eu * p.sigma_glwe ** 2 \
        + int(k.s.sum()) * (1 + int(k.sf.sum())) * (4 ** drop) / 12
    meas = float(np.mean(errs ** 2))
    assert 0.85 * pred < meas < 1.15 * pred, (meas, pred)
    # the paper's bound (2/3) n N ell L^2 B_brK plus the rounding term
    paper = (2 / 3) * p.n * N * p.g_ell * L ** 2 * p.sigma_glwe ** 2 \
        + p.n * (1 + N) * (4 ** drop) / 12
    assert meas <= paper


def test_affine_matches_integer_arithmetic():
    g = rnd(51)
    Wm = g.integers(-8, 9, (5, 7)).astype(np.int32)
    cts = g.integers(0, M32, (7, 11), dtype=np.uint64).astype(np.uint32)
    want = (Wm.astype(object) @ cts.astype(object)) % M32
    assert np.array_equal(oracle.affine(Wm, cts), want.astype(np.uint64).astype(np.uint32))


def test_sampler_statistics():
    bits = [oracle.draw(1, 1, i) >> 63 for i in range(4000)]
    assert abs(np.mean(bits) - 0.5) < 0.04
    z = np.array([oracle.gauss(3, 4, i, 1000.0) for i in range(4000)], dtype=np.float64)
    assert abs(z.mean()) < 60 and abs(z.std() / 1000.0 - 1) < 0.05
    assert oracle.gauss(3, 4, 0, 0.0) == 0


# ----------------------------------------------------------------------------
# forced faults are caught by decryption (host only)
# ----------------------------------------------------------------------------
def test_forced_faults_are_detected(oracle_keys_c1):
    """Faults planted on the host show up as decryption mismatches against
    the plaintext function: input noise pushed past half a slot moves m to
    m + 1, and one corrupted blind-rotation key row garbles the rotation.
    Untouched inputs in the same batch still decrypt to f(m)."""
    k = oracle_keys_c1
    p = W.C1
    t, delta = p.t, M32 // p.t
    lut = W.random_lut(W.LUT_SEED["C1"] + 9, t)
    while len(set(lut.tolist())) < t // 2:  # a table that tells neighbouring slots apart
        lut = (lut * 3 + 1) % t
    msgs = np.tile(np.arange(t, dtype=np.uint32), 2)
    cts = oracle.encrypt(p, k.s, msgs, seed=W.MSG_SEED["C1"] + 9)
    rot = [oracle.setup_polynomial(lut, p.N)]
    ids = np.zeros(len(msgs), int)

    # (a) inflated noise on the first copy: +3/4 of a slot on the body
    noisy = cts.copy()
    noisy[:t, 0] = (noisy[:t, 0].astype(np.uint64) + (3 * delta) // 4).astype(np.uint32)  # body b
    m, _ = oracle.decrypt(oracle.fdfb_batch(k, rot, ids, noisy), k.s, p.log2_t)
    want = lut[msgs]
    assert np.array_equal(m[t:], want[t:])
    shifted = lut[(msgs[:t] + 1) % t]
    assert np.array_equal(m[:t], shifted)
    assert (m[:t] != want[:t]).sum() == (shifted != want[:t]).sum() > 0

    # (b) one corrupted row of the blind-rotation key
    g = np.random.default_rng(9)
    bad = dataclasses.replace(k, brk=k.brk.copy())
    bad.brk[3, 0, 1] ^= g.integers(0, M32, p.N, dtype=np.uint64).astype(np.uint32)
    m, err = oracle.decrypt(oracle.fdfb_batch(bad, rot, ids, cts), k.s, p.log2_t)
    assert (m != want).sum() >= len(msgs) // 4
    assert np.max(np.abs(err)) >= delta // 4
