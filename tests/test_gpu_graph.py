"""A bootstrap batch captured into a HIP graph (after one eager call that
uploads keys and sizes the scratch) replays to the eager result: several
replays with eager work and synchronisations between them, each checked."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
fd = pytest.importorskip("paper_2109_02731_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_bootstrap_batch_graph_replays():
    p = W.C1
    ctx = fd.Context.keygen(p, W.KEY_SEED["C1"])
    lut = W.random_lut(81, p.t)
    lid = ctx.register_lut(lut)
    B = 64
    msgs = W.messages(82, B, p.t)
    cts = fd.to_device(ctx.encrypt_debug(msgs, seed=83))
    ids = torch.full((B,), lid, dtype=torch.int32, device="cuda")
    eager = torch.zeros((B, p.n + 1), dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    # warm-up on the capture stream: keys, this stream's scratch, kernel attributes
    ctx.bootstrap_batch(cts, ids, eager, stream=s)
    torch.cuda.synchronize()
    want = fd.to_host(eager)
    assert np.array_equal(ctx.decrypt_debug(want)[0], lut[msgs])

    out = torch.zeros_like(eager)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        ctx.bootstrap_batch(cts, ids, out)
    torch.cuda.synchronize()
    for rep in range(3):
        out.zero_()
        other = torch.zeros_like(eager)
        ctx.bootstrap_batch(cts, ids, other)  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(fd.to_host(out), want), rep
        assert np.array_equal(fd.to_host(other), want), rep


def test_capture_without_scratch_is_refused():
    """A stream with no scratch block yet cannot allocate one under capture:
    the call fails with a clear error instead of breaking the capture
    silently (the capture is then invalid and is discarded)."""
    p = W.C1
    ctx = fd.Context.keygen(p, W.KEY_SEED["C1"])
    lid = ctx.register_lut(W.random_lut(81, p.t))
    ctx.prepare()
    cts = fd.to_device(ctx.encrypt_debug(W.messages(82, 8, p.t), seed=83))
    ids = torch.full((8,), lid, dtype=torch.int32, device="cuda")
    out = torch.zeros((8, p.n + 1), dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with pytest.raises(fd.FdfbError) as ei:
        with torch.cuda.graph(g, stream=s):
            ctx.bootstrap_batch(cts, ids, out)
    assert "capture" in str(ei.value)
    torch.cuda.synchronize()
