"""The allocation-free bootstrap (scratch in the library's static device
buffer) against the allocating entry point, bit for bit, on two calls in a
row with the second one smaller, through the C ABI."""
import numpy as np
import pytest

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


@pytest.mark.parametrize("name,sizes,flags", [("C1", (61, 23), 0), ("C1", (40, 7), fd.OUT_EXTRACTED),
                                              ("C2", (1024, 300), 0)])
def test_noalloc_matches_allocating_entry_point(name, sizes, flags):
    p = W.PRESETS[name]
    ctx = fd.Context.keygen(p, W.KEY_SEED[name])
    luts = [W.random_lut(W.LUT_SEED[name] + k, p.t) for k in range(3)]
    lids = [ctx.register_lut(l) for l in luts]
    width = (p.N if flags & fd.OUT_EXTRACTED else p.n) + 1
    maxB = ctx.noalloc_max_batch()
    assert maxB >= max(sizes), maxB
    # not prepared yet: refused, nothing enqueued
    cts0 = fd.to_device(ctx.encrypt_debug(W.messages(1, 4, p.t), seed=1))
    ids0 = torch.zeros(4, dtype=torch.int32, device="cuda")
    with pytest.raises(fd.FdfbError):
        ctx.bootstrap_batch_noalloc(cts0, ids0, torch.empty((4, width), dtype=torch.int32, device="cuda"), flags)
    ctx.prepare(flags)
    for call, B in enumerate(sizes):
        msgs = W.messages(W.MSG_SEED[name] + call, B, p.t)
        which = np.random.default_rng(call).integers(0, 3, B)
        cts = fd.to_device(ctx.encrypt_debug(msgs, seed=W.MSG_SEED[name] + call))
        ids = torch.from_numpy(np.array([lids[w] for w in which], np.int32)).cuda()
        say(f"noalloc {name} call {call} B={B} flags={flags}")
        got = torch.full((B, width), -1, dtype=torch.int32, device="cuda")
        ctx.bootstrap_batch_noalloc(cts, ids, got, flags)
        ref = torch.zeros((B, width), dtype=torch.int32, device="cuda")
        ctx.bootstrap_batch(cts, ids, ref, flags)
        torch.cuda.synchronize()
        got_h, ref_h = fd.to_host(got), fd.to_host(ref)
        assert np.array_equal(got_h, ref_h), (call, B)
        if not flags & fd.OUT_EXTRACTED:
            m, _ = ctx.decrypt_debug(got_h)
            assert np.array_equal(m, np.array([luts[w][x] for w, x in zip(which, msgs)])), (call, B)
    # larger than the static buffer: refused before any device work
    big = maxB + 1
    with pytest.raises(fd.FdfbError) as ei:
        ctx.bootstrap_batch_noalloc(torch.zeros((big, p.n + 1), dtype=torch.int32, device="cuda"),
                                    torch.zeros(big, dtype=torch.int32, device="cuda"),
                                    torch.zeros((big, width), dtype=torch.int32, device="cuda"), flags)
    assert ei.value.code == -1
