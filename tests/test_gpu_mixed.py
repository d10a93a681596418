"""Uneven batch over two ring degrees in one submission: 2048 samples at
n=630 N=1024 t=16 and 2048 at n=750 N=2048 t=32, 64 random tables per half
with Zipf(1.2)-distributed table ids.  Every output decrypts to its table's
value, equals the separate per-job calls, and sampled outputs match the
oracle bit for bit."""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
fd = pytest.importorskip("paper_2109_02731_amd")

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_uneven_mixed_degree_batch():
    halves = [("C2", W.C2), ("C3B", W.C3B)]
    B = 2048
    jobs, meta = [], []
    for k, (name, p) in enumerate(halves):
        ctx = fd.Context.keygen(p, W.KEY_SEED[name])
        tables = [W.random_lut(W.LUT_SEED[name] * 100 + j, p.t) for j in range(64)]
        lids = np.array([ctx.register_lut(tb) for tb in tables], dtype=np.int32)
        which = W.zipf_indices(W.LUT_SEED[name], B, 64, 1.2)
        msgs = W.messages(W.MSG_SEED[name], B, p.t)
        cts = ctx.encrypt_debug(msgs, seed=W.MSG_SEED[name])
        d_cts = fd.to_device(cts)
        d_ids = torch.from_numpy(lids[which]).cuda()
        out = torch.empty((B, p.n + 1), dtype=torch.int32, device="cuda")
        jobs.append((ctx, d_cts, d_ids, out, 0))
        meta.append((name, p, ctx, tables, which, msgs, cts))
    say("mixed N=1024 / N=2048 multi-job submission, 2 x 2048 samples")
    fd.bootstrap_multi(jobs)
    torch.cuda.synchronize()
    outs = [fd.to_host(j[3]) for j in jobs]
    for (name, p, ctx, tables, which, msgs, cts), out in zip(meta, outs):
        m, _ = ctx.decrypt_debug(out)
        want = np.array([tables[w][x] for w, x in zip(which, msgs)])
        assert np.array_equal(m, want), name
        assert len(set(which.tolist())) > 10  # skewed but many tables in use
    # same bits as separate calls
    for (ctx, d_cts, d_ids, out, fl), ref in zip(jobs, outs):
        sep = torch.empty_like(out)
        ctx.bootstrap_batch(d_cts, d_ids, sep)
        torch.cuda.synchronize()
        assert np.array_equal(fd.to_host(sep), ref)
    # sampled outputs against the oracle
    from concurrent.futures import ThreadPoolExecutor
    cases = [(0, 3), (0, 2047), (1, 1000)]
    okeys = {k: oracle.keygen(meta[k][1], W.KEY_SEED[meta[k][0]]) for k in (0, 1)}

    def ref(case):
        k, idx = case
        name, p, ctx, tables, which, msgs, cts = meta[k]
        r0, r1 = oracle.setup_polynomial(tables[which[idx]], p.N)
        return oracle.fdfb(okeys[k], r0, r1, cts[idx])

    with ThreadPoolExecutor(len(cases)) as ex:
        refs = list(ex.map(ref, cases))
    for (k, idx), r in zip(cases, refs):
        assert np.array_equal(outs[k][idx], r), (k, idx)
