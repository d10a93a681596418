"""The tables and residue maps of the Chinese-remainder arithmetic
(paper_2109_02731_amd/arith.py, Sec. "Application of Functional
Bootstrapping") against plain integer arithmetic, on the CPU: the residue
split and Gauss reconstruction are inverse over all of Z_M, and for every
pair of residues of every modulus the plaintext composition the encrypted
path follows (lincomb mod t, then table lookups and a reduction) gives
x + y, x - y and x y mod m."""
import itertools

import numpy as np
import pytest

from paper_2109_02731_amd import arith


@pytest.mark.parametrize("t,moduli", [(8, (3, 4)), (16, (3, 5, 7, 8)), (32, (9, 11, 13, 16))])
def test_crt_split_join_roundtrip(t, moduli):
    M = int(np.prod(moduli))
    X = np.arange(M)
    res = arith.crt_split(X, moduli)
    assert res.shape == (M, len(moduli))
    assert np.array_equal(arith.crt_join(res, moduli), X)
    # distinct values have distinct residue vectors (pairwise coprime moduli)
    assert len({tuple(r) for r in res.tolist()}) == M


@pytest.mark.parametrize("t,moduli", [(8, (3, 4)), (16, (3, 5, 7, 8)), (32, (9, 11, 13, 16))])
def test_crt_residue_operations_through_the_tables(t, moduli):
    for m in moduli:
        red_u, red_s = arith.mod_table(t, m, False), arith.mod_table(t, m, True)
        qs, qd = arith.crt_quarter_tables(t, m)
        for x, y in itertools.product(range(m), repeat=2):
            s, d = (x + y) % t, (x - y) % t          # the linear step, mod t
            assert red_u[s] == (x + y) % m
            assert red_s[d] == (x - y) % m
            p = (int(qs[s]) - int(qd[d])) % t          # quarter-square difference, mod t
            assert red_s[p] == (x * y) % m, (m, x, y)


def test_crt_rejects_bad_moduli():
    class Ctx:  # the checks come before any table is registered
        class params:
            log2_t = 4
    with pytest.raises(ValueError):
        arith.CRT(Ctx(), (3, 9))       # not coprime
    with pytest.raises(ValueError):
        arith.CRT(Ctx(), (3, 11))      # 11 > t/2
