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
