"""The autotuner of the blind rotation: every plan it can choose (kernel
form, wavefronts per accumulator, round size, persistent queue) gives the
same bits as the fixed rule and as the oracle; the tuned plan is recorded,
used by the bootstrap, and written to the cache file."""
import json

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
fd = pytest.importorskip("paper_2109_02731_amd")

pytestmark = pytest.mark.gpu
M32 = 1 << 32


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield
    fd.tune_clear()


@pytest.mark.parametrize("name,A,per", [("C1", 37, 2), ("C2", 301, 3), ("C3B", 9, 3)])
def test_every_plan_gives_the_same_bits(name, A, per):
    p = W.PRESETS[name]
    ctx = fd.Context.keygen(p, W.KEY_SEED[name])
    g = np.random.default_rng(A)
    acc = g.integers(0, M32, (A, 2 * p.N), dtype=np.uint64).astype(np.uint32)
    ctN = g.integers(0, 2 * p.N, ((A + per - 1) // per, p.n + 1)).astype(np.uint32)
    d_ctN = fd.to_device(ctN)
    fd.tune_clear()
    ref = fd.to_device(acc)
    say(f"{name}: fixed rule, A={A}")
    ctx.blind_rotate(ref, d_ctN, per)
    torch.cuda.synchronize()
    ref = fd.to_host(ref)
    plans = ctx.br_plans()
    assert (4, 0) in plans  # the persistent queue is among them
    for form, rnd in plans:
        ctx.set_plan(A, form, rnd)
        assert ctx.get_plan(A)["form"] == fd.FORMS[form]
        d = fd.to_device(acc)
        say(f"{name}: plan {fd.FORMS[form]} round {rnd}")
        ctx.blind_rotate(d, d_ctN, per)
        torch.cuda.synchronize()
        assert np.array_equal(fd.to_host(d), ref), (form, rnd)
    ctx.set_plan(A)
    okeys = oracle.keygen(p, W.KEY_SEED[name])
    for a in (0, A - 1):
        assert np.array_equal(ref[a], oracle.blind_rotate(p, okeys.brk, ctN[a // per], acc[a])), a


def test_autotune_records_and_caches(tmp_path, monkeypatch):
    p = W.C2
    ctx = fd.Context.keygen(p, W.KEY_SEED["C2"])
    fd.tune_clear()
    path = tmp_path / "tune.json"
    monkeypatch.setenv("FDFB_TUNE_CACHE", str(path))
    say("autotune C2, 2048 sign and 1024 function accumulators")
    res_s = ctx.autotune(2048, 2)
    res_f = ctx.autotune(1024, 1)
    for res in (res_s, res_f):
        assert len(res["tried"]) >= 5 and res["best"]["ms"] > 0
        assert res["best"]["ms"] == min(t["ms"] for t in res["tried"])
    assert ctx.get_plan(2048)["form"] == res_s["best"]["form"]
    entries = json.loads(path.read_text())
    assert {e["A"] for e in entries} == {1024, 2048}
    # tuning inside whole batches (needs a table), then the cache again
    lid0 = ctx.register_lut(W.random_lut(7, p.t))
    assert lid0 == 0
    say("autotune C2 bootstrap batch of 1024")
    res_b = ctx.autotune_bootstrap(1024, 1)
    n_plans = len(ctx.br_plans())
    assert len(res_b["batch_ms"]) == 2 * n_plans
    assert res_b["sign_rotations"]["ms"] == min(t["ms"] for t in res_b["batch_ms"][:n_plans])
    assert ctx.get_plan(2048)["form"] == res_b["sign_rotations"]["form"]
    assert ctx.get_plan(1024)["form"] == res_b["function_rotation"]["form"]
    entries = json.loads(path.read_text())
    assert {e["A"] for e in entries} == {1024, 2048}
    # a bootstrap with the tuned plans: same bits as with the fixed rule
    lut = W.random_lut(W.LUT_SEED["C2"], p.t)
    lid = ctx.register_lut(lut)
    B = 1024
    res_s = {"best": ctx.get_plan(2048)}
    msgs = W.messages(W.MSG_SEED["C2"], B, p.t)
    cts = fd.to_device(ctx.encrypt_debug(msgs, seed=W.MSG_SEED["C2"]))
    ids = torch.full((B,), lid, dtype=torch.int32, device="cuda")
    tuned = torch.empty((B, p.n + 1), dtype=torch.int32, device="cuda")
    ctx.bootstrap_batch(cts, ids, tuned)
    torch.cuda.synchronize()
    fd.tune_clear()
    fixed = torch.empty_like(tuned)
    ctx.bootstrap_batch(cts, ids, fixed)
    torch.cuda.synchronize()
    assert torch.equal(tuned, fixed)
    assert np.array_equal(ctx.decrypt_debug(fd.to_host(tuned))[0], lut[msgs])
    # the file brings the choice back
    fd.tune_load(str(path))
    assert ctx.get_plan(2048)["form"] == res_s["best"]["form"]
    fd.tune_clear()
