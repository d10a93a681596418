"""Jobs of several contexts and ring degrees in one submission, with the
blind rotations of each phase in persistent work-queue launches.

* The uneven batch: 2048 samples at n=630 N=1024 t=16 and 2048 at n=750
  N=2048 t=32, 64 random tables per half with Zipf(1.2)-distributed ids.
  Every output decrypts to its table's value, equals the separate per-job
  calls and the submission without the queue, and sampled outputs match the
  oracle bit for bit.
* Small ragged jobs of all four queue geometries (items of four narrow
  accumulators left partly empty, several jobs on one context, a job in the
  plain form and an empty job beside them): bit-identical to separate calls,
  with oracle checks at the tiny size.
* A multi-job submission captured in a HIP graph replays to the eager
  result."""
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


@pytest.fixture(scope="module")
def ctxs():
    cache = {}

    def get(name):
        if name not in cache:
            cache[name] = fd.Context.keygen(W.PRESETS[name], W.KEY_SEED[name])
        return cache[name]
    return get


def _job(ctx, p, B, seed, tables, flags=0):
    lids = np.array([ctx.register_lut(tb) for tb in tables], dtype=np.int32)
    which = np.random.default_rng(seed).integers(0, len(tables), B)
    msgs = W.messages(seed, B, p.t)
    cts = ctx.encrypt_debug(msgs, seed=seed)
    width = (p.N if flags & fd.OUT_EXTRACTED else p.n) + 1
    out = torch.full((B, width), -1, dtype=torch.int32, device="cuda")
    return (ctx, fd.to_device(cts), torch.from_numpy(lids[which]).cuda(), out, flags), (which, msgs, cts)


def test_uneven_mixed_degree_batch(ctxs):
    halves = [("C2", W.C2), ("C3B", W.C3B)]
    B = 2048
    jobs, meta = [], []
    for k, (name, p) in enumerate(halves):
        ctx = ctxs(name)
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
    say("mixed N=1024 / N=2048 multi-job submission, 2 x 2048 samples, work-queue rotations")
    fd.bootstrap_multi(jobs)
    torch.cuda.synchronize()
    outs = [fd.to_host(j[3]) for j in jobs]
    for (name, p, ctx, tables, which, msgs, cts), out in zip(meta, outs):
        m, _ = ctx.decrypt_debug(out)
        want = np.array([tables[w][x] for w, x in zip(which, msgs)])
        assert np.array_equal(m, want), name
        assert len(set(which.tolist())) > 10  # skewed but many tables in use
        assert ctx.device_errors() == 0
    say("same submission without the queue, and each job alone")
    fd.bootstrap_multi(jobs, use_queue=False)
    torch.cuda.synchronize()
    for j, ref in zip(jobs, outs):
        assert np.array_equal(fd.to_host(j[3]), ref)
    for (ctx, d_cts, d_ids, out, fl), ref in zip(jobs, outs):
        sep = torch.empty_like(out)
        ctx.bootstrap_batch(d_cts, d_ids, sep)
        torch.cuda.synchronize()
        assert np.array_equal(fd.to_host(sep), ref)
    # sampled outputs against the oracle: first and last items of both jobs
    from concurrent.futures import ThreadPoolExecutor
    cases = [(0, 0), (0, 3), (0, 2047), (1, 0), (1, 1000), (1, 2047)]
    okeys = {k: oracle.keygen(meta[k][1], W.KEY_SEED[meta[k][0]]) for k in (0, 1)}

    def ref(case):
        k, idx = case
        name, p, ctx, tables, which, msgs, cts = meta[k]
        r0, r1 = oracle.setup_polynomial(tables[which[idx]], p.N)
        return oracle.fdfb(okeys[k], r0, r1, cts[idx])

    say(f"oracle on {len(cases)} samples")
    with ThreadPoolExecutor(len(cases)) as ex:
        refs = list(ex.map(ref, cases))
    for (k, idx), r in zip(cases, refs):
        assert np.array_equal(outs[k][idx], r), (k, idx)


def test_queue_ragged_jobs_all_geometries(ctxs, oracle_keys_c1):
    """Every queue geometry pair, ragged item counts, two jobs on one
    context, a plain-form job and an empty job in the same submission."""
    specs = [("C1", 7, 0), ("C3B", 3, 0), ("C1", 13, fd.OUT_EXTRACTED), ("C2", 5, 0), ("C4", 2, 0),
             ("C1", 6, fd.PLAIN), ("C2", 0, 0), ("C2", 1, 0)]
    jobs, meta = [], []
    for k, (name, B, flags) in enumerate(specs):
        p = W.PRESETS[name]
        tables = [W.random_lut(900 + 10 * k + j, p.t) for j in range(3)]
        job, m = _job(ctxs(name), p, B, 700 + k, tables, flags)
        jobs.append(job)
        meta.append((name, p, tables) + m)
    say(f"queue: {len(jobs)} ragged jobs over C1, C2, C3B, C4")
    fd.bootstrap_multi(jobs, use_queue=True)
    torch.cuda.synchronize()
    outs = [fd.to_host(j[3]) for j in jobs]
    for k, ((ctx, d_cts, d_ids, out, fl), (name, p, tables, which, msgs, cts)) in enumerate(zip(jobs, meta)):
        if not d_cts.shape[0]:
            continue
        sep = torch.empty_like(out)
        ctx.bootstrap_batch(d_cts, d_ids, sep, fl)
        torch.cuda.synchronize()
        assert np.array_equal(fd.to_host(sep), outs[k]), (k, name)
        if not fl & fd.OUT_EXTRACTED:
            m, _ = ctx.decrypt_debug(outs[k])
            assert np.array_equal(m, np.array([tables[w][x] for w, x in zip(which, msgs)])), (k, name)
    # the tiny jobs against the oracle, bit for bit
    for k in (0, 2):
        name, p, tables, which, msgs, cts = meta[k]
        fl = specs[k][2]
        for idx in range(len(msgs)):
            r0, r1 = oracle.setup_polynomial(tables[which[idx]], p.N)
            ref = oracle.fdfb(oracle_keys_c1, r0, r1, cts[idx],
                              flags=oracle.OUT_EXTRACTED if fl & fd.OUT_EXTRACTED else 0)
            assert np.array_equal(outs[k][idx], ref), (k, idx)


def test_multi_graph_replays(ctxs):
    """Two contexts captured in one HIP graph: every replay (with eager work
    and synchronisations between them) equals the eager submission."""
    specs = [("C1", 37), ("C2", 9), ("C1", 4)]
    jobs, meta = [], []
    for k, (name, B) in enumerate(specs):
        p = W.PRESETS[name]
        job, m = _job(ctxs(name), p, B, 800 + k, [W.random_lut(950 + 10 * k + j, p.t) for j in range(2)])
        jobs.append(job)
    fd.bootstrap_multi(jobs)
    torch.cuda.synchronize()
    want = [fd.to_host(j[3]) for j in jobs]
    say("multi-job graph: capture")
    g = fd.MultiGraph(jobs)
    assert g.info()["uses_queue"]
    for rep in range(3):
        for j in jobs:
            j[3].fill_(-1)
        other = torch.empty_like(jobs[0][3])
        jobs[0][0].bootstrap_batch(jobs[0][1], jobs[0][2], other)  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for j, w in zip(jobs, want):
            assert np.array_equal(fd.to_host(j[3]), w), rep
        assert np.array_equal(fd.to_host(other), want[0]), rep
    g.close()
