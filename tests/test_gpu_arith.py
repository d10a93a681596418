"""Arithmetic helpers (maximum, product) built from bootstraps and affine
maps: every pair decrypts to the integer result, and sampled outputs match
the same composition on the oracle bit for bit."""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
fd = pytest.importorskip("paper_2109_02731_amd")
from paper_2109_02731_amd import arith  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _oracle_chain(ok, p, W1, cts, luts, W2):
    """affine -> bootstrap (per row table) -> affine on the oracle."""
    mid = oracle.affine(W1, cts)
    boots = np.stack([oracle.fdfb(ok, *oracle.setup_polynomial(luts[k], p.N), mid[k]) for k in range(len(mid))])
    return oracle.affine(W2, boots)


def test_maximum_and_product_c1(oracle_keys_c1):
    p = W.C1
    t = p.t
    ctx = fd.Context.keygen(p, W.KEY_SEED["C1"])
    ar = arith.Arith(ctx)
    # all pairs in [0, t/2)^2, each pair twice
    mx = [(x, y) for x in range(t // 2) for y in range(t // 2)] * 2
    pr = mx
    for pairs, op, want in ((mx, ar.maximum, lambda x, y: max(x, y)),
                            (pr, ar.multiply, lambda x, y: (x * y) % t)):
        xs = np.array([a for a, _ in pairs], np.uint32)
        ys = np.array([b for _, b in pairs], np.uint32)
        cx = ctx.encrypt_debug(xs, seed=71)
        cy = ctx.encrypt_debug(ys, seed=72)
        out = op(fd.to_device(cx), fd.to_device(cy))
        torch.cuda.synchronize()
        got = fd.to_host(out)
        m, _ = ctx.decrypt_debug(got)
        assert np.array_equal(m, [want(int(a), int(b)) for a, b in pairs]), op.__name__
        # two pairs through the same composition on the oracle
        for k in (1, len(pairs) - 1):
            stacked = np.stack([cx[k], cy[k]])
            if op == ar.maximum:
                ref = _oracle_chain(oracle_keys_c1, p, np.array([[1, -1]]), stacked, [arith.relu_table(t)],
                                    np.array([[1, 0]]))
                ref = oracle.affine(np.array([[1, 1]]), np.stack([ref[0], cy[k]]))
            else:
                qs, qd = arith.quarter_square_tables(t)
                ref = _oracle_chain(oracle_keys_c1, p, np.array([[1, 1], [1, -1]]), stacked, [qs, qd],
                                    np.array([[1, -1]]))
            assert np.array_equal(got[k], ref[0]), (op.__name__, k)


def test_crt_arithmetic_c1_all_pairs(oracle_keys_c1):
    """Z_12 as residues mod 3 and 4 in Z_8: every pair through add, sub and
    multiply decrypts to the exact result mod 12; two residues of the product
    path match the same composition on the oracle bit for bit."""
    p = W.C1
    t = p.t
    ctx = fd.Context.keygen(p, W.KEY_SEED["C1"])
    crt = arith.CRT(ctx, (3, 4))
    M = crt.M
    X = np.array([a for a in range(M) for _ in range(M)])
    Y = np.array([b for _ in range(M) for b in range(M)])
    cx, cy = crt.encrypt_debug(X, seed=81), crt.encrypt_debug(Y, seed=82)
    dx, dy = fd.to_device(cx), fd.to_device(cy)
    outs = {}
    for name, op, want in (("add", crt.add, (X + Y) % M), ("sub", crt.sub, (X - Y) % M),
                           ("mul", crt.multiply, (X * Y) % M)):
        out = op(dx, dy)
        torch.cuda.synchronize()
        outs[name] = fd.to_host(out)
        assert np.array_equal(crt.decrypt_debug(outs[name]), want), name
    assert ctx.device_errors() == 0
    # the product's residues of two values through the same steps on the oracle
    for row in (1, 2 * 77 + 1):
        i = row % crt.k
        qs, qd = arith.crt_quarter_tables(t, crt.moduli[i])
        red = arith.mod_table(t, crt.moduli[i], True)
        stacked = np.stack([cx[row], cy[row]])
        q = _oracle_chain(oracle_keys_c1, p, np.array([[1, 1], [1, -1]]), stacked, [qs, qd], np.array([[1, -1]]))
        ref = oracle.fdfb(oracle_keys_c1, *oracle.setup_polynomial(red, p.N), q[0])
        assert np.array_equal(outs["mul"][row], ref), row


def test_crt_arithmetic_c2_random():
    """Z_840 as residues mod 3, 5, 7 and 8 in Z_16 at n=630 N=1024: random
    pairs through add, sub and multiply decrypt to the exact results."""
    p = W.C2
    ctx = fd.Context.keygen(p, W.KEY_SEED["C2"])
    crt = arith.CRT(ctx, (3, 5, 7, 8))
    rng = np.random.default_rng(840)
    X, Y = rng.integers(0, crt.M, 48), rng.integers(0, crt.M, 48)
    dx, dy = fd.to_device(crt.encrypt_debug(X, seed=83)), fd.to_device(crt.encrypt_debug(Y, seed=84))
    for name, op, want in (("add", crt.add, (X + Y) % crt.M), ("sub", crt.sub, (X - Y) % crt.M),
                           ("mul", crt.multiply, (X * Y) % crt.M)):
        out = op(dx, dy)
        torch.cuda.synchronize()
        assert np.array_equal(crt.decrypt_debug(fd.to_host(out)), want), name
