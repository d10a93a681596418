"""Sequences of batches bootstrapped as a software pipeline
(fdfb_bootstrap_pipeline): job k's function rotation shares persistent
work-queue launches with the sign rotations of the jobs after it, which are
split between launches at whole samples.

* Ragged batches at n=630 N=1024 t=16 (full 1024-sample batches, whose sign
  rotations fill a launch round exactly, and odd sizes, an empty job and a
  job with the extracted output) at one, two and the default number of
  rounds per launch: every output equals the separate fdfb_bootstrap_batch
  call bit for bit and decrypts to its table's value; sampled outputs match
  the oracle bit for bit.
* Jobs of every queue geometry in one pipeline (narrow N=256 and N=1024,
  wide N=2048 with three sign rotations per sample): bit-identical to the
  separate calls."""
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


def _jobs(ctxs, specs, seed0):
    jobs, meta = [], []
    for k, (name, B, flags) in enumerate(specs):
        p = W.PRESETS[name]
        ctx = ctxs(name)
        tables = [W.random_lut(seed0 + 10 * k + j, p.t) for j in range(3)]
        lids = np.array([ctx.register_lut(tb) for tb in tables], dtype=np.int32)
        which = np.random.default_rng(seed0 + k).integers(0, len(tables), B)
        msgs = W.messages(seed0 + k, B, p.t)
        cts = ctx.encrypt_debug(msgs, seed=seed0 + k)
        width = (p.N if flags & fd.OUT_EXTRACTED else p.n) + 1
        out = torch.full((B, width), -1, dtype=torch.int32, device="cuda")
        jobs.append((ctx, fd.to_device(cts), torch.from_numpy(lids[which]).cuda(), out, flags))
        meta.append((name, p, tables, which, msgs, cts))
    return jobs, meta


def _separate(jobs):
    refs = []
    for ctx, d_cts, d_ids, out, fl in jobs:
        sep = torch.full_like(out, -1)
        if d_cts.shape[0]:
            ctx.bootstrap_batch(d_cts, d_ids, sep, fl)
        refs.append(sep)
    torch.cuda.synchronize()
    return [fd.to_host(r) for r in refs]


def test_pipeline_ragged_batches_n1024(ctxs):
    specs = [("C2", 1024, 0), ("C2", 300, 0), ("C2", 77, fd.OUT_EXTRACTED), ("C2", 0, 0), ("C2", 1024, 0),
             ("C2", 5, 0), ("C2", 513, 0)]
    jobs, meta = _jobs(ctxs, specs, 4100)
    want = _separate(jobs)
    for rounds in (1, 2, 0):
        for j in jobs:
            j[3].fill_(-1)
        say(f"pipeline: {len(jobs)} C2 jobs ({sum(s[1] for s in specs)} samples), rounds={rounds}")
        fd.bootstrap_pipeline(jobs, rounds=rounds)
        torch.cuda.synchronize()
        for k, (j, w) in enumerate(zip(jobs, want)):
            assert np.array_equal(fd.to_host(j[3]), w), (rounds, k)
    ctx = jobs[0][0]
    assert ctx.device_errors() == 0
    for k, (name, p, tables, which, msgs, cts) in enumerate(meta):
        if len(msgs) and not specs[k][2] & fd.OUT_EXTRACTED:
            m, _ = ctx.decrypt_debug(want[k])
            assert np.array_equal(m, np.array([tables[w][x] for w, x in zip(which, msgs)])), k
    # sampled outputs against the oracle: a split job's first and last samples, the extracted job
    from concurrent.futures import ThreadPoolExecutor
    cases = [(0, 0), (0, 1023), (2, 76), (6, 256)]
    ok = oracle.keygen(W.C2, W.KEY_SEED["C2"])

    def ref(case):
        k, idx = case
        name, p, tables, which, msgs, cts = meta[k]
        r0, r1 = oracle.setup_polynomial(tables[which[idx]], p.N)
        return oracle.fdfb(ok, r0, r1, cts[idx],
                           flags=oracle.OUT_EXTRACTED if specs[k][2] & fd.OUT_EXTRACTED else 0)

    say(f"oracle on {len(cases)} samples")
    with ThreadPoolExecutor(len(cases)) as ex:
        refs = list(ex.map(ref, cases))
    for (k, idx), r in zip(cases, refs):
        assert np.array_equal(want[k][idx], r), (k, idx)


def test_pipeline_all_queue_geometries(ctxs):
    specs = [("C3B", 40, 0), ("C1", 33, 0), ("C2", 600, 0), ("C4", 9, fd.OUT_EXTRACTED), ("C3B", 7, 0),
             ("C1", 2, 0), ("C2", 130, 0)]
    jobs, meta = _jobs(ctxs, specs, 5200)
    want = _separate(jobs)
    for rounds in (1, 3):
        for j in jobs:
            j[3].fill_(-1)
        say(f"pipeline: C1, C2, C3B, C4 jobs, rounds={rounds}")
        fd.bootstrap_pipeline(jobs, rounds=rounds)
        torch.cuda.synchronize()
        for k, (j, w) in enumerate(zip(jobs, want)):
            assert np.array_equal(fd.to_host(j[3]), w), (rounds, k, specs[k][0])
    for k, (name, p, tables, which, msgs, cts) in enumerate(meta):
        if not specs[k][2] & fd.OUT_EXTRACTED:
            m, _ = ctxs(name).decrypt_debug(want[k])
            assert np.array_equal(m, np.array([tables[w][x] for w, x in zip(which, msgs)])), k
