"""Noise of the oracle's bootstrap, stage by stage, against the error analysis.

Every stage of the bootstrap (Sec. 3.2, Fig. 2) either adds noise or maps
the noise it is given linearly.  The correctness lemmas of Sec. 2 bound the
variance each stage adds (external product / CMux / blind rotation, key
switching, modulus switching) and Theorem "Correctness of the Bootstrapping"
composes them.  Here each stage's error is measured on the oracle with the
secret keys in hand and compared, two-sided, with the exact variance of the
same analysis: the lemmas' sums without the worst-case digit bound L^2 (the
digits are uniform, so their second moment is used), plus the rounding term
of the approximate gadget (reading R1), which the paper's bounds do not have.

The preset C1S gives every key its own deviation (fresh samples 2^16,
blind-rotation key 64, packing key 1024, key switching key 4096), so each
stage depends on one deviation only; keys generated with two deviations
swapped fail the stages that use them (the last test).

The failure probability is the one of Sec. 4, 1 - erf(q / (2 t sigma sqrt 2)).
It is pinned to Table II (one deviation per row reproduces the row; the
Theorem's bound with the Table I parameters gives that deviation within 15%)
and, where failures are frequent, to the failure rate measured on the oracle.
"""
import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import workloads as W

M32 = 1 << 32
P = W.C1S


# ----------------------------------------------------------------------------
# independent helpers (numpy integer arithmetic; nothing from the oracle)
# ----------------------------------------------------------------------------
def centred(x):
    """Values mod 2^32 as integers in [-2^31, 2^31)."""
    x = np.asarray(x, dtype=np.int64) % M32
    return np.where(x >= M32 // 2, x - M32, x)


def ring_mul_binary(a, key):
    """Negacyclic product of a (words mod 2^32) with a binary key, exact in int64."""
    N = len(key)
    full = np.convolve(np.asarray(a, np.int64), np.asarray(key, np.int64))  # length 2N - 1
    out = full[:N].copy()
    out[:N - 1] -= full[N:]  # X^N = -1
    return out % M32


def rlwe_phase(ct, key):
    N = len(key)
    return (np.asarray(ct[:N], np.int64) - ring_mul_binary(ct[N:], key)) % M32


def lwe_phase(cts, key):
    cts = np.atleast_2d(np.asarray(cts, np.int64))
    return (cts[:, 0] - cts[:, 1:] @ np.asarray(key, np.int64)) % M32


def rotate(p, e):
    """p * X^e in Z[X]/(X^N + 1) for an integer vector p."""
    p = np.asarray(p, np.int64)
    N = len(p)
    idx = (np.arange(N) - e) % (2 * N)
    return np.where(idx < N, p[idx % N], -p[idx % N])


def digits(x, log2B, ell):
    """Unsigned digits of x rounded (half up) to its top ell*log2B bits, [ell][...]."""
    drop = 32 - log2B * ell
    x = np.asarray(x, np.int64) % M32
    top = ((x + ((1 << drop) >> 1)) % M32) >> drop if drop else x
    return np.stack([(top >> (log2B * j)) & ((1 << log2B) - 1) for j in range(ell)])


# ----------------------------------------------------------------------------
# the analysis: second moments of what each stage adds
# ----------------------------------------------------------------------------
def digit_sq(log2B):
    """E[d^2] of a uniform unsigned digit in [0, 2^log2B)."""
    L = 1 << log2B
    return (L - 1) * (2 * L - 1) / 6.0


def round_sq(log2B, ell):
    """E[eps^2] of the rounding to the top ell*log2B bits: eps is uniform on
    the 2^drop integers of [-2^(drop-1), 2^(drop-1))."""
    drop = 32 - log2B * ell
    if drop == 0:
        return 0.0
    m = float(1 << drop)
    return (m * m + 2.0) / 12.0


def gauss_sq(sigma):
    """Second moment of a Gaussian of deviation sigma rounded to an integer."""
    return sigma ** 2 + (1.0 / 12.0 if sigma > 0 else 0.0)


def var_cmux(p, hw_sf, s_i):
    """Noise one CMux step adds at any coefficient (Lemma "Correctness of the
    CMux gate"): 2 ell rows of N digit-times-noise terms, plus the gadget's
    rounding error passed through the selected branch when s_i = 1."""
    return (2 * p.g_ell * p.N * digit_sq(p.g_log2B) * gauss_sq(p.sigma_glwe)
            + s_i * (1 + hw_sf) * round_sq(p.g_log2B, p.g_ell))


def var_blind_rotate(p, s, hw_sf, a_N, first_step_var=None):
    """Sum of var_cmux over the live steps (a_i != 0; a step with a_i = 0 adds
    exactly 0).  first_step_var replaces the first live step's term (used for
    the sign accumulators, whose first step still has a zero a-component)."""
    live = [i for i in range(p.n) if a_N[i] != 0]
    total = sum(var_cmux(p, hw_sf, int(s[i])) for i in live)
    if first_step_var is not None and live:
        total += first_step_var - var_cmux(p, hw_sf, int(s[live[0]]))
    return total


def var_keyswitch(N, log2B, ell, sigma, hw_sf, constant=True):
    """Noise of a key switch (Lemma "Correctness of Key Switching") at the
    constant coefficient (where the rounding of the inputs lands) or at
    another coefficient of an RLWE output (key noise only)."""
    v = N * ell * digit_sq(log2B) * gauss_sq(sigma)
    if constant:
        v += hw_sf * round_sq(log2B, ell)
    return v


def sign_first_step_var(p, b_N, a_first, scale):
    """Exact noise variance of the first live step of a sign rotation: the
    accumulator is [scale sgnP X^b, 0], so only the b-rows have digits, they
    are known exactly, and the values are multiples of the gadget's unit (no
    rounding error)."""
    sgn = np.full(p.N, -1, np.int64)
    sgn[0] = 1
    acc_b = (scale * rotate(sgn, b_N)) % M32
    d = (rotate(acc_b, -int(a_first)) - acc_b) % M32
    dg = digits(d, p.g_log2B, p.g_ell)
    return float((dg.astype(np.float64) ** 2).sum()) * gauss_sq(p.sigma_glwe)


def p_fail(sigma, q, t):
    """Sec. 4: the probability that an error of deviation sigma leaves its
    slot of width q / t, 1 - erf(q / (2 t sigma sqrt 2))."""
    return math.erfc(q / (2.0 * t * sigma * math.sqrt(2.0)))


# ----------------------------------------------------------------------------
# measurements on the oracle
# ----------------------------------------------------------------------------
@pytest.fixture(scope="module")
def keys():
    return oracle.keygen(P, W.KEY_SEED["C1S"])


def _ratio(measured_sq, predicted):
    return float(np.sum(measured_sq)) / float(np.sum(predicted))


def fresh_ratio(p_nominal, k, p_used=None, count=4000):
    """Fresh LWE samples: error variance sigma_lwe^2 (Sec. 1.2 "Regev Encryption")."""
    p_used = p_used or p_nominal
    msgs = W.messages(11, count, p_used.t)
    cts = oracle.encrypt(p_used, k.s, msgs, seed=12)
    e = centred(lwe_phase(cts, k.s) - (M32 // p_used.t) * msgs.astype(np.int64))
    return _ratio(e.astype(np.float64) ** 2, np.full(count, gauss_sq(p_nominal.sigma_lwe)))


def key_noise(p, k):
    """The noise of every key row, recovered with the secret keys: brK rows
    [n][2 ell][N] (phase minus s_i g_j in component c, Def. "Generalized-GSW
    Sample"), pK rows [N][ell][N] (phase minus s_F[i] g_j), ksK rows [N][ell]."""
    n, N = p.n, p.N
    sf = k.sf
    brk = k.brk.reshape(n, 2 * p.g_ell, 2, N)
    e_br = np.empty((n, 2 * p.g_ell, N), np.int64)
    for i in range(n):
        for r in range(2 * p.g_ell):
            c, j = divmod(r, p.g_ell)
            ph = rlwe_phase(brk[i, r].reshape(-1), sf)
            gj = (1 << (32 - p.g_ell * p.g_log2B + p.g_log2B * j)) * int(k.s[i])
            if c == 0:
                ph[0] -= gj
            else:  # the gadget sits in the a-polynomial: phase = e - g_j s_i sf
                ph = ph + gj * sf.astype(np.int64)
            e_br[i, r] = centred(ph)
    pk = k.pk.reshape(N, p.pk_ell, 2, N)
    e_pk = np.empty((N, p.pk_ell, N), np.int64)
    for i in range(N):
        for j in range(p.pk_ell):
            ph = rlwe_phase(pk[i, j].reshape(-1), sf)
            ph[0] -= (1 << (32 - p.pk_ell * p.pk_log2B + p.pk_log2B * j)) * int(sf[i])
            e_pk[i, j] = centred(ph)
    ksk = k.ksk.reshape(N, p.ks_ell, n + 1).astype(np.int64)
    gks = np.array([1 << (32 - p.ks_ell * p.ks_log2B + p.ks_log2B * j) for j in range(p.ks_ell)], np.int64)
    e_ks = centred(ksk[:, :, 0] - ksk[:, :, 1:] @ k.s.astype(np.int64) - sf[:, None].astype(np.int64) * gks)
    return {"brK": e_br, "pK": e_pk, "ksK": e_ks}


def keyswitch_ratios(p, k, count=3000):
    """ksK (LWE -> LWE) and pK (LWE -> RLWE) on uniform inputs under s_F:
    measured / predicted second moment of the added error, for the ksK output,
    the pK output's constant coefficient and its other coefficients.

    The output error is sum_i s_F[i] eps_i - sum_ij d_ij e_ij (Lemma
    "Correctness of Key Switching"): eps the inputs' rounding, d their
    unsigned digits, e the key noise.  For the given key the second moment of
    coefficient m over the inputs is Var(d) sum_ij e_ij[m]^2 + E[d]^2
    (sum_ij e_ij[m])^2, plus hw(s_F) E[eps^2] at the constant coefficient
    (its average over keys is N ell E[d^2] sigma^2, the lemma's form)."""
    g = np.random.default_rng(13)
    hw = int(k.sf.sum())
    kn = key_noise(p, k)

    def pred(e, log2B, ell, constant):  # e: key noise [N][ell] (one coefficient)
        L = 1 << log2B
        mean, var = (L - 1) / 2.0, (L * L - 1) / 12.0
        e = e.astype(np.float64)
        v = var * float((e ** 2).sum()) + mean ** 2 * float(e.sum()) ** 2
        return v + (hw * round_sq(log2B, ell) if constant else 0.0)

    p_ks = pred(kn["ksK"], p.ks_log2B, p.ks_ell, True)
    p_pk = np.array([pred(kn["pK"][:, :, m], p.pk_log2B, p.pk_ell, m == 0) for m in range(p.N)])
    ins = g.integers(0, M32, (count, p.N + 1), dtype=np.uint64).astype(np.uint32)
    ph_in = lwe_phase(ins, k.sf)
    e_ks, e_pk = [], []
    for c in range(count):
        out = oracle.keyswitch(ins[c], k.ksk, p.ks_log2B, p.ks_ell, p.n + 1)
        e_ks.append(centred(lwe_phase(out, k.s) - ph_in[c])[0])
        r = oracle.keyswitch(ins[c], k.pk, p.pk_log2B, p.pk_ell, 2 * p.N)
        ph = rlwe_phase(r, k.sf)
        ph[0] -= ph_in[c]
        e_pk.append(centred(ph))
    e_ks = np.array(e_ks, np.float64)
    e_pk = np.array(e_pk, np.float64)
    return {
        "ksK": float(np.mean(e_ks ** 2)) / p_ks,
        "pK constant": float(np.mean(e_pk[:, 0] ** 2)) / p_pk[0],
        "pK other": float(np.mean(e_pk[:, 1:] ** 2, axis=0).sum()) / float(p_pk[1:].sum()),
    }


def bootstrap_stage_ratios(p, k, count=256, threads=8):
    """Bootstraps with stage dumps: measured / predicted second moments of
    * the noise each sign rotation adds (all coefficients),
    * the noise the packing switch adds to the bit samples (non-constant
      coefficients),
    * the built accumulator's error after PubMux (a linear map of the
      switched samples' errors: sum_i sum_p delta_i[m - p]^2 Var e_Ri[p]),
    * the noise the function rotation adds (all coefficients),
    * the bootstrap's output error (normalised per sample by its predicted
      variance: PubMux error at the coefficient the rotation brings to 0,
      plus the function rotation, plus the final key switch)."""
    N, t, n = p.N, p.t, p.n
    delta = M32 // t
    hw_sf = int(k.sf.sum())
    L = 1 << p.boot_log2B
    lut = W.random_lut(W.LUT_SEED["C1S"], t)
    r0, r1 = (np.asarray(x, np.int64) for x in oracle.setup_polynomial(lut, N))
    msgs = W.messages(W.MSG_SEED["C1S"], count, t)
    cts = oracle.encrypt(p, k.s, msgs, seed=W.MSG_SEED["C1S"])

    def run(c):
        return oracle.fdfb(k, r0.astype(np.int32), r1.astype(np.int32), cts[c], dumps=True)

    with ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(run, range(count)))

    acc = {key: [0.0, 0.0] for key in ("sign", "pK", "pubmux", "function", "output")}
    v_pk0 = var_keyswitch(N, p.pk_log2B, p.pk_ell, p.sigma_pk, hw_sf)
    v_pk1 = var_keyswitch(N, p.pk_log2B, p.pk_ell, p.sigma_pk, hw_sf, constant=False)
    v_ks = var_keyswitch(N, p.ks_log2B, p.ks_ell, p.sigma_ks, hw_sf)
    sgn = np.full(N, -1, np.int64)
    sgn[0] = 1
    for c, (out, d) in enumerate(res):
        ctN = d["ctN"].astype(np.int64)
        b_N, a_N = int(ctN[0]), ctN[1:]
        r = int(a_N @ k.s.astype(np.int64)) % (2 * N)
        bit = 1 if (b_N - r) % (2 * N) < N else 0
        first = next(i for i in range(n) if a_N[i] != 0)
        v_sign = []
        for i in range(p.boot_ell):
            scale = ((delta // 2) * L ** i) % M32
            init = (scale * rotate(sgn, b_N)) % M32
            e = centred(rlwe_phase(d["acc_sign"][i].reshape(-1), k.sf) - rotate(init, -r))
            v = var_blind_rotate(p, k.s, hw_sf, a_N, sign_first_step_var(p, b_N, a_N[first], scale))
            v_sign.append(v)
            acc["sign"][0] += float((e.astype(np.float64) ** 2).sum())
            acc["sign"][1] += v * N
            # the packing switch of bit sample i (LWE under s_F -> RLWE under s_F)
            ph = rlwe_phase(d["r_bits"][i].reshape(-1), k.sf)
            ph[0] -= int(lwe_phase(d["c_bits"][i], k.sf)[0])
            e = centred(ph)[1:]
            acc["pK"][0] += float((e.astype(np.float64) ** 2).sum())
            acc["pK"][1] += v_pk1 * (N - 1)
        # PubMux: p_A = rotP_1 X^b, p_B = rotP_0 X^b, digits of (p_B - p_A) mod t
        p_A, p_B = rotate(r1, b_N), rotate(r0, b_N)
        dl = (p_B - p_A) % t
        p_sel = p_B if bit else p_A
        e_F = centred(rlwe_phase(d["acc_f"].reshape(-1), k.sf) - delta * p_sel)
        pred_F = np.zeros(N)
        for i in range(p.boot_ell):
            di = ((dl // L ** i) % L).astype(np.float64)
            pred_F += di ** 2 * (v_sign[i] + v_pk0) + (float((di ** 2).sum()) - di ** 2) * v_pk1
        acc["pubmux"][0] += float((e_F.astype(np.float64) ** 2).sum())
        acc["pubmux"][1] += float(pred_F.sum())
        # function rotation: added noise = phase(out) - phase(in) X^{-r}
        e = centred(rlwe_phase(d["acc_f_br"].reshape(-1), k.sf)
                    - rotate(rlwe_phase(d["acc_f"].reshape(-1), k.sf), -r))
        v_br = var_blind_rotate(p, k.s, hw_sf, a_N)
        acc["function"][0] += float((e.astype(np.float64) ** 2).sum())
        acc["function"][1] += v_br * N
        # output: error of Delta f(m), normalised by its own predicted variance
        e_out = float(centred(lwe_phase(out, k.s) - delta * int(lut[msgs[c]]))[0])
        acc["output"][0] += e_out ** 2 / (pred_F[r % N] + v_br + v_ks)
        acc["output"][1] += 1.0
    return {key: m / q for key, (m, q) in acc.items()}


# ----------------------------------------------------------------------------
# stage checks
# ----------------------------------------------------------------------------
def test_preset_deviations_are_distinct():
    s = sorted([P.sigma_lwe, P.sigma_glwe, P.sigma_pk, P.sigma_ks])
    assert all(b >= 4 * a for a, b in zip(s, s[1:]))


def test_fresh_sample_variance(keys):
    assert 0.9 < fresh_ratio(P, keys) < 1.1


def test_modswitch_variance(keys):
    """Input ModSwitch q -> 2N (Lemma "Correctness of Modulus Switching"):
    the phase error in Z_2N has second moment (2N/q)^2 Var(e) + (1 + hw(s))/12
    (every coordinate rounded by at most 1/2), within the lemma's bound
    (2N/q)^2 B + 2/3 + (2/3) hw(s) (Var(s) + E(s)^2) for binary s."""
    k = keys
    count = 2000
    msgs = W.messages(21, count, P.t)
    cts = oracle.encrypt(P, k.s, msgs, seed=22)
    lg = int(math.log2(2 * P.N))
    ctN = np.vectorize(lambda x: oracle.modswitch(int(x), lg), otypes=[np.int64])(cts)
    ph = (ctN[:, 0] - ctN[:, 1:] @ k.s.astype(np.int64)) % (2 * P.N)
    e = (ph - (2 * P.N // P.t) * msgs.astype(np.int64) + P.N) % (2 * P.N) - P.N
    hw = int(k.s.sum())
    scale = (2 * P.N / M32) ** 2
    pred = scale * gauss_sq(P.sigma_lwe) + (1 + hw) / 12.0
    meas = float(np.mean(e.astype(np.float64) ** 2))
    assert 0.85 * pred < meas < 1.15 * pred, (meas, pred)
    paper = scale * gauss_sq(P.sigma_lwe) + 2 / 3 + (2 / 3) * hw * (0.25 + 0.25)
    assert meas <= paper


def test_key_noise_deviations(keys):
    """Each key's noise has the deviation of its preset (and mean 0): the
    blind-rotation key sigma_glwe, the packing key sigma_pk, the key switching
    key sigma_ks (keys of Theorem "Correctness of the Bootstrapping")."""
    kn = key_noise(P, keys)
    for name, sigma in (("brK", P.sigma_glwe), ("pK", P.sigma_pk), ("ksK", P.sigma_ks)):
        e = kn[name].astype(np.float64).reshape(-1)
        assert abs(e.mean()) < 5 * sigma / math.sqrt(e.size), name
        assert 0.95 < math.sqrt(float(np.mean(e ** 2)) / gauss_sq(sigma)) < 1.05, name


def test_keyswitch_variances(keys):
    r = keyswitch_ratios(P, keys)
    for name, v in r.items():
        assert 0.85 < v < 1.15, (name, v)


@pytest.fixture(scope="module")
def stage_ratios(keys):
    return bootstrap_stage_ratios(P, keys)


@pytest.mark.parametrize("stage", ["sign", "pK", "pubmux", "function", "output"])
def test_bootstrap_stage_variance(stage_ratios, stage):
    assert 0.8 < stage_ratios[stage] < 1.2, (stage, stage_ratios[stage])


def test_blind_rotation_within_paper_bound(keys):
    """The measured blind-rotation variance is below the bound of Lemma
    "Correctness of TFHE-Style Blind-Rotation", (2/3) n N ell L^2 B_brK, plus
    the rounding term of reading R1 (which the lemma does not have)."""
    p, k = P, keys
    L = 1 << p.g_log2B
    hw_sf = int(k.sf.sum())
    a_N = np.ones(p.n, np.int64)
    exact = var_blind_rotate(p, k.s, hw_sf, a_N)
    paper = (2 / 3) * p.n * p.N * p.g_ell * L ** 2 * gauss_sq(p.sigma_glwe) \
        + p.n * (1 + p.N) * round_sq(p.g_log2B, p.g_ell)
    assert exact <= paper


# ----------------------------------------------------------------------------
# failure probability (Sec. 4)
# ----------------------------------------------------------------------------
# Table II, FDFB sets: log2 of the small modulus q and the first value of each
# column log2 t = 6..11 (0.0 where the paper prints 0.0).
TABLE_II = {
    "FDFB:80:6": (12, [2.0 ** -30, 2.0 ** -9, 0.12, 0.44, 0.70, 0.84]),
    "FDFB:100:6": (12, [2.0 ** -32, 2.0 ** -10, 0.11, 0.43, 0.69, 0.84]),
    "FDFB:80:7": (13, [0.0, 2.0 ** -31, 2.0 ** -9, 0.12, 0.44, 0.69]),
    "FDFB:100:7": (13, [0.0, 2.0 ** -31, 2.0 ** -9, 0.12, 0.44, 0.69]),
    "FDFB:80:8": (14, [0.0, 0.0, 2.0 ** -26, 2.0 ** -8, 0.16, 0.48]),
    "FDFB:100:8": (14, [0.0, 0.0, 2.0 ** -26, 2.0 ** -8, 0.16, 0.48]),
}

# Table I: ring degree, log2 Q, key switching base and deviation, Hamming
# weight of s.  Q_1 = 2^62 - 65535, Q_2 = 2^63 - 278527 (taken as 2^62, 2^63).
TABLE_I = {
    "FDFB:80:6": dict(N=2 ** 11, logQ=62, L_ks=2 ** 6, sigma_ks=2.0 ** 38, h=64),
    "FDFB:100:6": dict(N=2 ** 11, logQ=62, L_ks=2, sigma_ks=2.0 ** 41, h=64),
    "FDFB:80:7": dict(N=2 ** 12, logQ=63, L_ks=2 ** 4, sigma_ks=2.0 ** 39, h=64),
    "FDFB:100:7": dict(N=2 ** 12, logQ=63, L_ks=2, sigma_ks=2.0 ** 41, h=64),
    "FDFB:80:8": dict(N=2 ** 13, logQ=63, L_ks=2 ** 4, sigma_ks=2.0 ** 39, h=64),
    "FDFB:100:8": dict(N=2 ** 13, logQ=63, L_ks=2, sigma_ks=2.0 ** 41, h=64),
}


def _fit_sigma(logq, row):
    """The deviation that reproduces the row's entry nearest to 1/2."""
    from scipy.special import erfcinv
    k = min(range(len(row)), key=lambda j: abs(row[j] - 0.5) if row[j] > 0 else 9)
    x = float(erfcinv(row[k]))
    return 2.0 ** logq / (2.0 * 2.0 ** (6 + k) * math.sqrt(2.0) * x)


@pytest.mark.parametrize("name", list(TABLE_II))
def test_table_ii_row_is_one_deviation(name):
    """Each FDFB row of Table II is the erf formula of Sec. 4 at one deviation:
    fitted on the entry nearest 1/2, it reproduces the others (decimals to
    0.015, powers of two to one in the exponent, 0.0 entries below 2^-60)."""
    logq, row = TABLE_II[name]
    sig = _fit_sigma(logq, row)
    for j, want in enumerate(row):
        got = p_fail(sig, 2.0 ** logq, 2.0 ** (6 + j))
        if want == 0.0:
            assert got < 2.0 ** -60, (name, j, got)
        elif want < 0.01:
            assert abs(math.log2(got) - math.log2(want)) <= 1.0, (name, j, got, want)
        else:
            assert abs(got - want) <= 0.015, (name, j, got, want)


@pytest.mark.parametrize("name", list(TABLE_II))
def test_theorem_bound_reproduces_table_ii(name):
    """Approximate pin (readings of the theorem's final terms): with q = 2N for
    every FDFB set, Table II's deviation is that of the bootstrapped output,
    B_out = (q/Q)^2 (B_F + B_BR + B_KS) + 2/3 + (2/3) h (Var(s) + E(s)^2),
    where only B_KS is not negligible after the (q/Q)^2 scaling, and
    Var(s) + E(s)^2 = 1/2 for binary key entries.  It agrees with the
    variance fitted to the row within 15%."""
    logq, row = TABLE_II[name]
    t1 = TABLE_I[name]
    N, logQ = t1["N"], t1["logQ"]
    assert 2 * N == 2 ** logq  # the case "B_N = B_ct" of the theorem
    ell_ks = math.ceil(logQ / math.log2(t1["L_ks"]))
    b_ks = (1 / 3) * N * ell_ks * t1["L_ks"] ** 2 * t1["sigma_ks"] ** 2
    b_out = 2.0 ** (2 * (logq - logQ)) * b_ks + 2 / 3 + (2 / 3) * t1["h"] * 0.5
    fitted = _fit_sigma(logq, row) ** 2
    assert 0.85 * fitted < b_out < 1.15 * fitted, (name, b_out, fitted)


def test_failure_rate_matches_erf():
    """Where failures are frequent the erf formula predicts them.  Key switches
    of noise-free samples, with a key switching deviation chosen so that the
    error deviation is about Delta/2 / 1.645 (10% failures at t = 8), are
    decrypted 1000 times under each of 4 keys.  For one key the error is
    Gaussian with the mean -E[d] sum_ij e_ij and the variance Var(d) sum_ij
    e_ij^2 + hw(s_F) E[eps^2] of that key's noise (the key-switch analysis
    above), so the failure probability is the two tails of the erf formula,
    1/2 erfc((Delta/2 - mu) / (s sqrt 2)) + 1/2 erfc((Delta/2 + mu) / (s sqrt 2));
    the failures counted over all keys are within 4 binomial deviations of
    the predicted count."""
    p = W.C1.with_(sigma_ks=5.8e5, sigma_lwe=0.0)
    delta = M32 // p.t
    L = 1 << p.ks_log2B
    g = np.random.default_rng(78)
    per_key, expect, var_count, fails = 1000, 0.0, 0.0, 0
    for j in range(4):
        k = oracle.keygen(p, 77 + j)
        hw = int(k.sf.sum())
        e = key_noise(p, k)["ksK"].astype(np.float64)
        mu = -(L - 1) / 2.0 * float(e.sum())
        sd = math.sqrt((L * L - 1) / 12.0 * float((e ** 2).sum()) + hw * round_sq(p.ks_log2B, p.ks_ell))
        pk = 0.5 * (math.erfc((delta / 2 - mu) / (sd * math.sqrt(2.0)))
                    + math.erfc((delta / 2 + mu) / (sd * math.sqrt(2.0))))
        expect += per_key * pk
        var_count += per_key * pk * (1 - pk)
        msgs = g.integers(0, p.t, per_key)
        for c in range(per_key):
            a = g.integers(0, M32, p.N, dtype=np.uint64).astype(np.int64)
            b = (int(a @ k.sf.astype(np.int64)) + delta * int(msgs[c])) % M32
            ct = np.concatenate([[b], a]).astype(np.uint32)
            out = oracle.keyswitch(ct, k.ksk, p.ks_log2B, p.ks_ell, p.n + 1)
            m, _ = oracle.decrypt(out, k.s, p.log2_t)
            fails += int(m[0] != msgs[c])
    assert 0.02 * 4 * per_key < expect < 0.5 * 4 * per_key  # a regime with frequent failures
    assert abs(fails - expect) < 4 * math.sqrt(var_count), (fails, expect)


def test_predicted_failure_probability_of_presets():
    """Failure probability per output of the headline configuration from the
    variance this analysis predicts (PubMux with ell_boot digits, function
    rotation, key switch), with every PubMux digit at its maximum: far below
    any rate a test could observe."""
    p = W.C2
    hw_s, hw_sf = p.n // 2, p.N // 2
    v_br = p.n * var_cmux(p, hw_sf, 0.5)
    v_pk0 = var_keyswitch(p.N, p.pk_log2B, p.pk_ell, p.sigma_pk, hw_sf)
    v_pk1 = var_keyswitch(p.N, p.pk_log2B, p.pk_ell, p.sigma_pk, hw_sf, constant=False)
    L = 1 << p.boot_log2B
    dmax = (L - 1) ** 2
    v_f = p.boot_ell * (dmax * (v_br + v_pk0) + p.N * digit_sq(p.boot_log2B) * v_pk1)
    v_out = v_f + v_br + var_keyswitch(p.N, p.ks_log2B, p.ks_ell, p.sigma_ks, hw_sf)
    assert p_fail(math.sqrt(v_out), float(M32), float(p.t)) < 2.0 ** -100
    # the input side: the phase in Z_2N must stay within N/t of its slot
    v_in = (2 * p.N / M32) ** 2 * gauss_sq(p.sigma_lwe) + (1 + hw_s) / 12
    assert p_fail(math.sqrt(v_in), 2.0 * p.N, float(p.t)) < 2.0 ** -100


# ----------------------------------------------------------------------------
# a wrong deviation in key generation is caught
# ----------------------------------------------------------------------------
def test_swapped_deviations_fail_the_stage_checks():
    """Keys (and fresh samples) generated with two pairs of deviations swapped
    -- blind-rotation key <-> packing key, key switching key <-> fresh
    samples -- are measured against the nominal analysis: the stages that use
    them leave the 20% band by far."""
    swapped = P.with_(sigma_glwe=P.sigma_pk, sigma_pk=P.sigma_glwe,
                      sigma_ks=P.sigma_lwe, sigma_lwe=P.sigma_ks)
    k = oracle.keygen(swapped, W.KEY_SEED["C1S"])
    k_nominal_view = type(k)(P, k.seed, k.s, k.sf, k.brk, k.pk, k.ksk)
    st = bootstrap_stage_ratios(P, k_nominal_view, count=24)
    fr = fresh_ratio(P, k, p_used=swapped, count=1000)
    kn = key_noise(P, k)
    dev = {name: math.sqrt(float(np.mean(kn[name].astype(np.float64) ** 2)) / gauss_sq(s))
           for name, s in (("brK", P.sigma_glwe), ("pK", P.sigma_pk), ("ksK", P.sigma_ks))}
    assert st["sign"] > 5 and st["function"] > 5  # brK drawn with 1024 instead of 64
    assert st["pK"] < 0.2                         # pK drawn with 64 instead of 1024
    assert fr < 0.2                               # fresh samples drawn with 4096 instead of 2^16
    assert dev["brK"] > 10 and dev["pK"] < 0.1 and dev["ksK"] > 10  # and each key's own deviation
