#!/usr/bin/env python3
"""FDFB benchmark on one MI355X.

One step = one full-domain functional bootstrap of a batch of 1024 LWE
samples at n=630, N=1024, q=2^32 (gadget 2^7 x 3, key switch 2^4 x 5,
t=16, one seeded random LUT): ModSwitch, 2 sign blind rotations per sample,
SampleExtract, packing key switch, public mux, the function blind rotation,
SampleExtract and the final key switch.  Inputs are resident in HBM before the
timed region.  Prints one JSON line with:

* value: bootstraps/s of the batched INT8-MFMA form (whole job, 1 GPU);
* plain: the same for the one-accumulator-per-workgroup VALU form;
* latency_ms: p50 / p99 of the per-batch latency of the batched form;
* roofline: the sign blind-rotation kernel's achieved int8 tera-ops/s (algorithmic
  schoolbook work in 8-bit limbs, divided by the kernel time measured with
  HIP events on its stream over the timed steps) against the 5.0 POPS dense
  int8 MFMA peak, plus its HBM traffic when counter data for the current
  kernel source exists;
* serving: a Poisson request stream (two parameter sets, request sizes
  1..512, a random table per request) through the continuous-batching server:
  bootstraps/s and p50 / p99 request latency, saturated and at 80% load;
* cpu_baseline: the CPU oracle on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FDFB bootstraps/s on 1 MI355X, n=630 N=1024, batched vs plain; p99 latency"
PEAK_INT8_TOPS = 5000.0   # MI355X dense int8 MFMA, tera-ops/s
PEAK_HBM_GBS = 8000.0


def br_ops_per_accumulator(p) -> float:
    """Algorithmic int8 ops of one blind rotation of one accumulator: n CMux,
    each (k+1) ell (k+1) = 4 ell negacyclic products of N^2 multiply-adds,
    every 32-bit key word split into 4 byte limbs and every digit into
    ceil(log2B / 7) 7-bit chunks; 2 ops per multiply-add."""
    chunks = (p.g_log2B + 6) // 7
    return p.n * 4 * p.g_ell * p.N * p.N * 4 * chunks * 2.0


def kernel_source_hash(src: str = None) -> str:
    """Hash of the blind-rotation kernel's source: the kernel itself and its
    launcher (other kernels in the same file do not change its traffic),
    with line comments and blank lines left out."""
    if src is None:
        with open(os.path.join(ROOT, "paper_2109_02731_amd", "csrc", "kernels.hip")) as f:
            src = f.read()
    h = hashlib.sha256()
    for start, end in (("struct BrKara {", "// launchers"),
                       ("static const void *br_kara_kernel()", "bool br_mfma_supported")):
        a = src.index(start)
        for line in src[a:src.index(end, a)].splitlines():
            code = line.split("//", 1)[0].rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def load_traffic(kernel: str):
    """HBM bytes per launch of a blind-rotation kernel from committed counter
    data, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "br_kara_traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return d.get("kernels", {}).get(kernel, {}).get("hbm_bytes_per_launch")


def host_cpu():
    """Host CPU model name and logical core count (nproc)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(p, cts, lut, threads: int, sample: int):
    """The oracle on the host: `sample` bootstraps of the bench batch, one per
    thread on `threads` threads, and one bootstrap alone on one thread."""
    import oracle
    import workloads as W
    keys = oracle.keygen(p, W.KEY_SEED["C2"])
    rot = [oracle.setup_polynomial(lut, p.N)]
    t0 = time.perf_counter()
    oracle.fdfb_batch(keys, rot, np.zeros(sample, int), cts[:sample], threads=threads)
    dt = time.perf_counter() - t0
    t1 = time.perf_counter()
    oracle.fdfb_batch(keys, rot, np.zeros(1, int), cts[sample:sample + 1], threads=1)
    one = time.perf_counter() - t1
    model, nproc = host_cpu()
    return {"value": sample / dt, "unit": "bootstraps/s", "cores": threads, "kind": "oracle",
            "sample": f"samples 0..{sample - 1} of the 1024-sample batch, one oracle bootstrap per thread on "
                      f"{threads} threads ({dt:.1f} s wall), and sample {sample} alone on one thread",
            "s_per_bootstrap_1_thread": one, "host_nproc": nproc, "host_cpu_model": model}


def oracle_timing(threads: int):
    """The oracle's time per bootstrap at the two plain-batch configurations,
    on one thread and on `threads` threads (one sample per thread), on the
    same kind of seeded inputs as the GPU runs."""
    import oracle
    import workloads as W
    res = {}
    for name, count1 in (("C1", 16), ("C2", 1)):
        p = W.PRESETS[name]
        keys = oracle.keygen(p, W.KEY_SEED[name])
        lut = W.random_lut(W.LUT_SEED[name], p.t)
        rot = [oracle.setup_polynomial(lut, p.N)]
        msgs = W.messages(W.MSG_SEED[name], max(count1, threads), p.t)
        cts = oracle.encrypt(p, keys.s, msgs, seed=W.MSG_SEED[name])
        t0 = time.perf_counter()
        oracle.fdfb_batch(keys, rot, np.zeros(count1, int), cts[:count1], threads=1)
        one = (time.perf_counter() - t0) / count1
        t0 = time.perf_counter()
        oracle.fdfb_batch(keys, rot, np.zeros(threads, int), cts[:threads], threads=threads)
        many = time.perf_counter() - t0
        res[name] = {"s_per_bootstrap_1_thread": one, "bootstraps_per_s_1_thread": 1 / one,
                     "threads": threads, "bootstraps_per_s_all_threads": threads / many,
                     "sample": f"{count1} bootstraps on 1 thread, {threads} on {threads} threads"}
    return res


def serving_run(fd, torch, W, ctxs, presets, pools, lids, count, rate, max_batch=512, nstreams=3, seed=None,
                request_max=512):
    """Poisson request stream through the continuous-batching server
    (request sizes uniform in 1..request_max; the server forms batches of up
    to max_batch samples).  Returns throughput, request latency percentiles
    and batching counters."""
    import threading
    seed = W.ARRIVAL_SEED if seed is None else seed
    times, sizes, which = W.poisson_arrivals(seed, count, rate, max_batch=request_max)
    rng = np.random.default_rng(seed + 1)
    reqs = []
    for k in range(count):
        c, B = int(which[k]), int(sizes[k])
        cts_d, _ = pools[c]
        off = int(rng.integers(0, cts_d.shape[0] - B + 1))
        j = int(rng.integers(0, len(lids[c])))
        reqs.append((c, off, B, j, cts_d[off:off + B],
                     torch.full((B,), lids[c][j], dtype=torch.int32, device="cuda"),
                     torch.empty((B, presets[c].n + 1), dtype=torch.int32, device="cuda")))
    torch.cuda.synchronize()
    srv = fd.Server(ctxs, max_batch=max_batch, mem_budget=1 << 30, nstreams=nstreams)
    ids, lat = [None] * count, [None] * count

    def waiter():
        for k in range(count):
            while ids[k] is None:
                time.sleep(1e-4)
            lat[k] = srv.wait(ids[k])

    th = threading.Thread(target=waiter)
    th.start()
    t0 = time.perf_counter()
    for k, (c, off, B, j, cts, idt, out) in enumerate(reqs):
        dt = t0 + times[k] - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        ids[k] = srv.submit(c, cts, idt, out)
    th.join()
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    # every result decrypts to its table's value
    ok = True
    for (c, off, B, j, cts, idt, out) in reqs[:: max(1, count // 40)]:
        m, _ = ctxs[c].decrypt_debug(fd.to_host(out))
        want = pools[c][1][j][off:off + B]
        ok &= bool(np.array_equal(m, want))
    lat_ms = np.array(lat) * 1e3
    return {"offered_requests_per_s": rate, "requests": count, "bootstraps": int(sizes.sum()),
            "bootstraps_per_s": float(sizes.sum() / wall), "requests_per_s": count / wall,
            "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
            "batches": st["batches"], "mean_batch": float(sizes.sum() / max(1, st["batches"])),
            "peak_admitted_mib": st["max_in_flight_bytes"] / 2 ** 20, "correct": ok}


def serving_bench(fd, torch, W, ctx2, count):
    """Config-5 shaped stream: parameter sets 50/50 (n=64 N=256 t=8 and the
    bench's n=630 N=1024 t=16), request sizes uniform in 1..512, a random
    table per request; once at 2000 requests/s (saturating) and once at 80%
    of the capacity that run measured."""
    presets = [W.C1, W.C2]
    ctx1 = fd.Context.keygen(W.C1, W.KEY_SEED["C1"])
    ctxs = [ctx1, ctx2]
    pools, lids = [], []
    for k, (c, p) in enumerate(zip(ctxs, presets)):
        tables = [W.random_lut(5000 + 100 * k + j, p.t) for j in range(16)]
        lids.append([c.register_lut(t) for t in tables])
        msgs = W.messages(6000 + k, 4096, p.t)
        cts = fd.to_device(c.encrypt_debug(msgs, seed=6100 + k))
        pools.append((cts, [t[msgs] for t in tables]))
    # the server joins requests of one parameter set into batches of up to
    # 2048 samples on two streams: a full N = 1024 batch then fills every SIMD
    # twice in both rotation phases
    kw = dict(max_batch=2048, nstreams=2)
    sat = serving_run(fd, torch, W, ctxs, presets, pools, lids, count, 2000.0, **kw)
    sus = serving_run(fd, torch, W, ctxs, presets, pools, lids, count, 0.8 * sat["requests_per_s"],
                      seed=W.ARRIVAL_SEED + 7, **kw)
    return {"saturated": sat, "sustainable": sus, "server": {"max_batch": 2048, "streams": 2, "request_max": 512}}


def mixed_bench(fd, torch, W, ctx2, steps: int):
    """Config 3, the uneven batch over two ring degrees: 2048 samples at n=630
    N=1024 and 2048 at n=750 N=2048, 64 tables per half, Zipf(1.2) ids.  One
    multi-job submission whose blind rotations run in one persistent
    work-queue launch per phase, the same captured in a HIP graph (one graph
    launch per submission), and the jobs rotated in their own launches."""
    halves = [("C2", W.C2, ctx2), ("C3B", W.C3B, None)]
    jobs, meta = [], []
    for name, p, c in halves:
        c = c or fd.Context.keygen(p, W.KEY_SEED[name])
        tables = [W.random_lut(W.LUT_SEED[name] * 100 + j, p.t) for j in range(64)]
        lids = np.array([c.register_lut(tb) for tb in tables], dtype=np.int32)
        which = W.zipf_indices(W.LUT_SEED[name], 2048, 64, 1.2)
        msgs = W.messages(W.MSG_SEED[name], 2048, p.t)
        cts = fd.to_device(c.encrypt_debug(msgs, seed=W.MSG_SEED[name]))
        ids = torch.from_numpy(lids[which]).cuda()
        out = torch.empty((2048, p.n + 1), dtype=torch.int32, device="cuda")
        jobs.append((c, cts, ids, out, 0))
        meta.append((c, np.array([tables[w][x] for w, x in zip(which, msgs)])))

    def timed(fn) -> float:
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    t_queue = timed(lambda: fd.bootstrap_multi(jobs, use_queue=True))
    ok = all(np.array_equal(c.decrypt_debug(fd.to_host(j[3]))[0], want) for j, (c, want) in zip(jobs, meta))
    t_jobs = timed(lambda: fd.bootstrap_multi(jobs, use_queue=False))
    g = fd.MultiGraph(jobs, use_queue=True)
    t_graph = timed(lambda: g.replay())
    ok = ok and all(np.array_equal(c.decrypt_debug(fd.to_host(j[3]))[0], want) for j, (c, want) in zip(jobs, meta))
    g.close()
    return {"workload": "2048 samples n=630 N=1024 t=16 + 2048 samples n=750 N=2048 t=32, "
                        "64 tables per half, Zipf(1.2) ids",
            "bootstraps_per_s": 4096 / t_graph, "ms_per_submission": t_graph * 1e3,
            "what": "one HIP graph launch per submission; blind rotations in one persistent work-queue launch "
                    "per phase for both ring degrees",
            "ms_queue_submission": t_queue * 1e3, "ms_jobs_in_own_launches": t_jobs * 1e3,
            "correct": bool(ok), "steps": steps}


def pipeline_bench(fd, torch, ctx, d_cts, d_ids, ref, batches: int, single_ms: float):
    """A stream of `batches` batches of the bench workload bootstrapped as a
    software pipeline (fdfb_bootstrap_pipeline): batch k's function rotation
    shares persistent work-queue launches with the sign rotations of the
    batches after it, at 1, 2, 4 and 8 rounds of the resident capacity per
    launch.  Every batch's output is checked bit for bit against the
    separate call's."""
    B = int(d_cts.shape[0])
    outs = [torch.empty_like(ref) for _ in range(batches)]
    jobs = [(ctx, d_cts, d_ids, o, 0) for o in outs]
    by_rounds, ok = {}, True
    for rounds in (1, 2, 4, 8):
        fd.bootstrap_pipeline(jobs, rounds=rounds)
        torch.cuda.synchronize()
        ok = ok and all(torch.equal(o, ref) for o in outs)
        t0 = time.perf_counter()
        for _ in range(2):
            fd.bootstrap_pipeline(jobs, rounds=rounds)
        torch.cuda.synchronize()
        by_rounds[rounds] = (time.perf_counter() - t0) / 2 / batches * 1e3
    best = min(by_rounds, key=by_rounds.get)
    ms = by_rounds[best]
    return {"bootstraps_per_s": B / (ms * 1e-3), "ms_per_batch": ms, "rounds_per_launch": best,
            "ms_per_batch_by_rounds": {str(k): v for k, v in by_rounds.items()}, "batches": batches,
            "vs_separate_calls": single_ms / ms, "bit_identical_to_separate_calls": bool(ok),
            "what": f"{batches} batches of {B} as one software-pipelined submission: each persistent work-queue "
                    "launch holds whole rounds of two wavefronts per SIMD, batch k's function rotation beside "
                    "the next batches' sign rotations"}


def nn_bench(fd, torch, W, steps: int):
    """Config 4, the NN-shaped circuit: x in Z_32^784 -> dense 784->128 on LWE
    samples -> FDFB ReLU on the 128 outputs (extracted) -> dense 128->10 ->
    key switch (n=750, N=2048, gadget 2^7 x 4, L_boot = 2), time per
    inference with every output checked against the plaintext evaluation."""
    p = W.C4
    ctx = fd.Context.keygen(p, W.KEY_SEED["C4"])
    relu = W.named_luts(p.t)["relu"]
    lid = ctx.register_lut(relu)
    x, w1, w2 = W.nn_inputs(W.MSG_SEED["C4"], p.t)
    cts = fd.to_device(ctx.encrypt_debug(x, seed=W.MSG_SEED["C4"]))
    d_w1, d_w2 = torch.from_numpy(w1).cuda(), torch.from_numpy(w2).cuda()
    ids = torch.full((128,), lid, dtype=torch.int32, device="cuda")
    h = torch.empty((128, p.n + 1), dtype=torch.int32, device="cuda")
    hq = torch.empty((128, p.N + 1), dtype=torch.int32, device="cuda")
    y = torch.empty((10, p.N + 1), dtype=torch.int32, device="cuda")
    yo = torch.empty((10, p.n + 1), dtype=torch.int32, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]

    def infer(mark=False):
        if mark:
            ev[0].record()
        fd.affine(d_w1, cts, h)
        if mark:
            ev[1].record()
        ctx.bootstrap_batch(h, ids, hq, flags=fd.OUT_EXTRACTED)
        if mark:
            ev[2].record()
        fd.affine(d_w2, hq, y)
        ctx.keyswitch(y, yo)
        if mark:
            ev[3].record()

    infer()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        infer()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    infer(mark=True)
    torch.cuda.synchronize()
    hp = (w1.astype(np.int64) @ x.astype(np.int64)) % p.t
    yp = (w2.astype(np.int64) @ relu[hp].astype(np.int64)) % p.t
    ok = bool(np.array_equal(ctx.decrypt_debug(fd.to_host(yo))[0], yp))
    return {"workload": "784 -> 128 -> 10 on LWE samples, FDFB ReLU on 128 outputs, n=750 N=2048 t=32",
            "ms_per_inference": dt * 1e3, "inferences_per_s": 1 / dt, "bootstraps_per_inference": 128,
            "phase_ms": {"affine_784_128": ev[0].elapsed_time(ev[1]), "bootstraps_128": ev[1].elapsed_time(ev[2]),
                         "affine_128_10_and_keyswitch": ev[2].elapsed_time(ev[3])},
            "correct": ok, "steps": steps}


def multi_lut_bench(fd, torch, W, ctx, p, d_cts, B: int, L: int, steps: int, single_ms: float):
    """L tables per sample on the bench batch: the sign rotations are shared,
    so one call does ell_boot + L blind rotations per sample."""
    lids = np.array([ctx.register_lut(W.random_lut(W.LUT_SEED["C2"] * 10 + l, p.t)) for l in range(L)],
                    dtype=np.int32)
    ids = torch.from_numpy(np.tile(lids, (B, 1))).cuda()
    out = torch.empty((B, L, p.n + 1), dtype=torch.int32, device="cuda")
    ctx.bootstrap_multi_lut(d_cts, ids, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.bootstrap_multi_lut(d_cts, ids, out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return {"tables_per_sample": L, "table_evaluations_per_s": B * L / dt, "ms_per_call": dt * 1e3,
            "speedup_vs_single_table_calls": L * single_ms / (dt * 1e3), "steps": steps}


def signed_boot_bench(fd, torch, W, B: int, steps: int):
    """Variant with one signed public-mux digit (one sign rotation per
    sample): bootstraps/s on the bench batch, outputs decrypted."""
    p = W.signed_boot(W.C2)
    ctx = fd.Context.keygen(p, W.KEY_SEED["C2"])
    lut = W.random_lut(W.LUT_SEED["C2"], p.t)
    lid = ctx.register_lut(lut)
    msgs = W.messages(W.MSG_SEED["C2"], B, p.t)
    cts = fd.to_device(ctx.encrypt_debug(msgs, seed=W.MSG_SEED["C2"]))
    ids = torch.full((B,), lid, dtype=torch.int32, device="cuda")
    out = torch.empty((B, p.n + 1), dtype=torch.int32, device="cuda")
    ctx.bootstrap_batch(cts, ids, out)
    torch.cuda.synchronize()
    correct = bool(np.array_equal(ctx.decrypt_debug(fd.to_host(out))[0], lut[msgs]))
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.bootstrap_batch(cts, ids, out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return {"bootstraps_per_s": B / dt, "ms_per_step": dt * 1e3, "blind_rotations_per_bootstrap": 2,
            "correct": correct, "steps": steps,
            "note": "variant, not the paper's digit reading: one signed public-mux digit in [-t/2, t/2)"}


def tfhe_bench(fd, torch, ctx, d_cts, d_ids, B: int, steps: int, fdfb_ms: float):
    """The one-rotation TFHE-style (half-domain) bootstrap on the same
    kernels and batch: the yardstick for FDFB's extra rotations."""
    out = torch.empty((B, ctx.params.n + 1), dtype=torch.int32, device="cuda")
    ctx.tfhe_bootstrap_batch(d_cts, d_ids, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.tfhe_bootstrap_batch(d_cts, d_ids, out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return {"bootstraps_per_s": B / dt, "ms_per_step": dt * 1e3, "blind_rotations_per_bootstrap": 1,
            "fdfb_time_ratio": fdfb_ms / (dt * 1e3), "steps": steps,
            "note": "half-domain only (m < t/2); FDFB's time over this is the price of the full domain"}


def config_sweep(fd, torch, W, B: int, steps: int):
    """bootstraps/s of every parameter preset at batch B (schoolbook int8
    work of the blind rotations over the measured time, as for the headline)."""
    res = {}
    for name, p in W.PRESETS.items():
        ctx = fd.Context.keygen(p, W.KEY_SEED[name])
        lut = W.random_lut(W.LUT_SEED[name], p.t)
        lid = ctx.register_lut(lut)
        msgs = W.messages(W.MSG_SEED[name], B, p.t)
        cts = fd.to_device(ctx.encrypt_debug(msgs, seed=W.MSG_SEED[name]))
        ids = torch.full((B,), lid, dtype=torch.int32, device="cuda")
        out = torch.empty((B, p.n + 1), dtype=torch.int32, device="cuda")
        ctx.bootstrap_batch(cts, ids, out)
        torch.cuda.synchronize()
        ok = bool(np.array_equal(ctx.decrypt_debug(fd.to_host(out))[0], lut[msgs]))
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.bootstrap_batch(cts, ids, out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        ops = br_ops_per_accumulator(p) * B * (p.boot_ell + 1)
        res[name] = {"n": p.n, "N": p.N, "t": p.t, "blind_rotations_per_bootstrap": p.boot_ell + 1,
                     "bootstraps_per_s": B / dt, "ms_per_batch": dt * 1e3, "correct": ok,
                     "schoolbook_int8_tops": ops / dt / 1e12}
        print(f"[bench] {name}: {B / dt:.0f} bootstraps/s", file=sys.stderr, flush=True)
    return {"batch": B, "steps": steps, "presets": res}


def batch_sweep(fd, torch, W, ctx, steps: int, sizes=(128, 256, 512, 1024, 2048, 4096)):
    """The bench configuration (n=630 N=1024, one table) at several batch
    sizes: bootstraps/s, time per batch and blind-rotation launches, to show
    what batching buys and what a batch costs in latency."""
    p = W.C2
    lut = W.random_lut(W.LUT_SEED["C2"], p.t)
    lid = ctx.register_lut(lut)
    res = []
    for B in sizes:
        msgs = W.messages(W.MSG_SEED["C2"] + B, B, p.t)
        cts = fd.to_device(ctx.encrypt_debug(msgs, seed=W.MSG_SEED["C2"] + B))
        ids = torch.full((B,), lid, dtype=torch.int32, device="cuda")
        out = torch.empty((B, p.n + 1), dtype=torch.int32, device="cuda")
        ctx.bootstrap_batch(cts, ids, out)
        torch.cuda.synchronize()
        ok = bool(np.array_equal(ctx.decrypt_debug(fd.to_host(out))[0], lut[msgs]))
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.bootstrap_batch(cts, ids, out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        res.append({"batch": B, "bootstraps_per_s": B / dt, "ms_per_batch": dt * 1e3, "correct": ok,
                    "br_launches": ctx.br_launches(B * p.boot_ell, p.boot_ell) + ctx.br_launches(B, 1)})
        print(f"[bench] batch {B}: {B / dt:.0f} bootstraps/s, {dt * 1e3:.1f} ms", file=sys.stderr, flush=True)
    return {"steps": steps, "sizes": res}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--serving-requests", type=int, default=4000,
                    help="requests per serving run (0 skips the serving measurement)")
    ap.add_argument("--multi-lut", type=int, default=4, metavar="L",
                    help="also time L tables per sample on the bench batch (0 skips)")
    ap.add_argument("--signed-boot-steps", type=int, default=5,
                    help="also time the one-signed-digit variant this many steps (0 skips)")
    ap.add_argument("--direct-steps", type=int, default=3,
                    help="also time the direct (non-Karatsuba) MFMA form this many steps (0 skips)")
    ap.add_argument("--tfhe-steps", type=int, default=5,
                    help="also time the one-rotation TFHE-style bootstrap this many steps (0 skips)")
    ap.add_argument("--config-sweep", type=int, default=0, metavar="STEPS",
                    help="also time every parameter preset at batch 1024 this many steps (0 skips)")
    ap.add_argument("--mixed-steps", type=int, default=2,
                    help="also time the uneven two-degree batch (one multi-job submission) this many times (0 skips)")
    ap.add_argument("--pipeline-batches", type=int, default=16,
                    help="also time a stream of this many bench batches as one software pipeline (0 skips)")
    ap.add_argument("--nn-steps", type=int, default=3,
                    help="also time the 784->128->10 circuit this many inferences (0 skips)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (the fixed plan rule issues the blind rotations)")
    ap.add_argument("--plan-sign", default=None, choices=["auto", "1w", "1w2", "2w", "queue", "split"],
                    help="issue the sign rotations with this plan instead of tuning (for profiles)")
    ap.add_argument("--plan-func", default=None, choices=["auto", "1w", "1w2", "2w", "queue", "split"],
                    help="issue the function rotation with this plan instead of tuning (for profiles)")
    ap.add_argument("--batch-sweep", type=int, default=0, metavar="STEPS",
                    help="also time the bench configuration at batch 128..4096 this many steps (0 skips)")
    ap.add_argument("--oracle-timing", action="store_true",
                    help="also time the oracle at C1 and C2 on one thread and on all host threads")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_mib": args.calibrate_copy}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(each bootstrap is independent given the keys; see the sharding notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2109_02731_amd as fd
    import workloads as W

    p = W.C2
    B = 1024
    ctx = fd.Context.keygen(p, W.KEY_SEED["C2"])
    lut = W.random_lut(W.LUT_SEED["C2"], p.t)
    lid = ctx.register_lut(lut)
    msgs = W.messages(W.MSG_SEED["C2"], B, p.t)
    cts = ctx.encrypt_debug(msgs, seed=W.MSG_SEED["C2"])
    d_cts = fd.to_device(cts)
    d_ids = torch.full((B,), lid, dtype=torch.int32, device="cuda")
    d_out = torch.empty((B, p.n + 1), dtype=torch.int32, device="cuda")

    def step(flags=0):
        ctx.bootstrap_batch(d_cts, d_ids, d_out, flags=flags)

    tuned = None
    forms = {v: k for k, v in fd.FORMS.items()}
    if args.plan_sign or args.plan_func:
        args.no_tune = True
        if args.plan_sign:
            ctx.set_plan(B * p.boot_ell, forms[args.plan_sign])
        if args.plan_func:
            ctx.set_plan(B, forms[args.plan_func])
    if not args.no_tune:
        # the autotuner times every issue plan of the two rotation phases of
        # this batch (2048 sign and 1024 function accumulators) inside whole
        # batches and records the fastest; the timed steps use them
        print("[bench] autotune", file=sys.stderr, flush=True)
        tuned = ctx.autotune_bootstrap(B, 1)
    print(f"[bench] keys ready; warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    K = args.steps
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record()
    for k in range(K):
        step()
        evs[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.profile(False)
    phases, calls = ctx.profile_read()
    step_ms = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(K)])
    out = fd.to_host(d_out)
    m, _ = ctx.decrypt_debug(out)
    correct = bool(np.array_equal(m, lut[msgs]))
    print(f"[bench] batched: {wall / K * 1e3:.2f} ms/step, correct={correct}", file=sys.stderr, flush=True)

    # plain form on the same inputs
    plain = None
    if args.plain_steps > 0:
        step(fd.PLAIN)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.plain_steps):
            step(fd.PLAIN)
        torch.cuda.synchronize()
        pw = time.perf_counter() - t1
        same = bool(np.array_equal(fd.to_host(d_out), out))
        plain = {"value": B * args.plain_steps / pw, "unit": "bootstraps/s",
                 "ms_per_step": pw / args.plain_steps * 1e3, "steps": args.plain_steps,
                 "bit_identical_to_batched": same}
        print(f"[bench] plain: {pw / args.plain_steps * 1e3:.1f} ms/step", file=sys.stderr, flush=True)

    # roofline of the dominant kernel: the sign rotations, B * ell_boot = 2048
    # accumulators, fill every SIMD of the device twice and run as one launch of
    # the two-wavefronts-per-SIMD kernel; the function rotation (B = 1024) runs
    # the one-wavefront-per-SIMD kernel.  Both rates are reported.
    ops_acc = br_ops_per_accumulator(p)
    sign_units, func_units = B * p.boot_ell, B

    def rate(units, ms, launches):
        achieved = ops_acc * units / (ms * 1e-3) / 1e12
        return {"achieved": achieved, "frac": achieved / PEAK_INT8_TOPS, "ops_per_launch_avg": ops_acc * units / launches,
                "avg_launch_ms": ms / launches, "launches_per_step": launches,
                "executed_mfma_frac": achieved * 0.75 / PEAK_INT8_TOPS}  # one Karatsuba level: 3 of 4 products

    cus = torch.cuda.get_device_properties(0).multi_processor_count

    def kernel_for(units):  # the kernel the library issues for one round of this many accumulators
        form = ctx.get_plan(units)["form"]
        if form == "queue":
            return "k_br_queue<1024, 3, 1, 2048, 2, 2>"
        if form == "1w":
            return "k_br_kara1w<1024, 3, 1>"
        if form == "1w2":
            return "k_br_kara1w2<1024, 3, 1, 1>"
        if form == "2w":
            return "k_br_kara1w2<1024, 3, 1, 2>"
        if units > 4 * cus:
            return "k_br_kara1w2<1024, 3, 1, 1>"
        return "k_br_kara1w2<1024, 3, 1, 2>" if 2 * units <= 4 * cus else "k_br_kara1w<1024, 3, 1>"

    sign_kernel, func_kernel = kernel_for(sign_units), kernel_for(func_units)
    sign = rate(sign_units, phases["sign_br"] / calls, ctx.br_launches(sign_units, p.boot_ell))
    func = rate(func_units, phases["function_br"] / calls, ctx.br_launches(func_units, 1))
    both = rate(sign_units + func_units, (phases["sign_br"] + phases["function_br"]) / calls,
                sign["launches_per_step"] + func["launches_per_step"])
    # the dense int8 rate this device sustains on a register-only MFMA stream
    mfma_tops, mfma_ms = fd.measure_mfma_peak()
    print(f"[bench] measured int8 MFMA stream: {mfma_tops:.0f} TOPS", file=sys.stderr, flush=True)
    def hbm(traffic, ms_per_launch):
        if not traffic:
            return None
        gbs = traffic / (ms_per_launch * 1e-3) / 1e9
        return {"achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS}

    sign_traffic, func_traffic = load_traffic(sign_kernel), load_traffic(func_kernel)
    roofline = {"bound": "mfma", "kernel": sign_kernel, "achieved": sign["achieved"], "peak": PEAK_INT8_TOPS,
                "unit": "TOPS", "frac": sign["frac"], "traffic": sign_traffic,
                "hbm": hbm(sign_traffic, sign["avg_launch_ms"]),
                "ops_per_launch_avg": sign["ops_per_launch_avg"], "avg_launch_ms": sign["avg_launch_ms"],
                "launches_per_step": sign["launches_per_step"], "executed_mfma_frac": sign["executed_mfma_frac"],
                "function_rotation": dict(kernel=func_kernel, traffic=func_traffic,
                                          hbm=hbm(func_traffic, func["avg_launch_ms"]), **func),
                "all_rotations": {"achieved": both["achieved"], "frac": both["frac"],
                                  "executed_mfma_frac": both["executed_mfma_frac"]},
                "measured_mfma_peak": {"tera_ops": mfma_tops, "ms": mfma_ms,
                                       "what": "independent v_mfma_i32_16x16x64_i8 from registers on every "
                                               "wave slot (fdfb_measure_mfma_peak)",
                                       "executed_frac_of_measured": sign["achieved"] * 0.75 / mfma_tops},
                "note": "unit TOPS: 10^12 int8 multiply-add halves per second.  achieved counts the schoolbook "
                        "product work of the method (63.4 G int8 ops per accumulator and rotation); the "
                        "kernels issue 3/4 of it on MFMA (one exact Karatsuba level), executed_mfma_frac is "
                        "the issued rate over the peak; kernel is the sign rotations' kernel (2048 "
                        "accumulators, the larger share of the step), function_rotation the one of the 1024 "
                        "function accumulators, all_rotations both together; hbm is the counted HBM traffic "
                        "per launch over the launch time"}

    multi_lut = None
    if args.multi_lut > 0:
        print(f"[bench] {args.multi_lut} tables per sample", file=sys.stderr, flush=True)
        multi_lut = multi_lut_bench(fd, torch, W, ctx, p, d_cts, B, args.multi_lut, 3, wall / K * 1e3)

    signed = None
    if args.signed_boot_steps > 0:
        print("[bench] signed boot digit variant", file=sys.stderr, flush=True)
        signed = signed_boot_bench(fd, torch, W, B, args.signed_boot_steps)

    direct = None
    if args.direct_steps > 0:
        print("[bench] direct (non-Karatsuba) MFMA form", file=sys.stderr, flush=True)
        out_d = torch.empty_like(d_out)
        ctx.bootstrap_batch(d_cts, d_ids, out_d, fd.DIRECT)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.direct_steps):
            ctx.bootstrap_batch(d_cts, d_ids, out_d, fd.DIRECT)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.direct_steps
        direct = {"bootstraps_per_s": B / dt, "ms_per_step": dt * 1e3, "steps": args.direct_steps,
                  "bit_identical_to_batched": bool(torch.equal(out_d, d_out))}

    tfhe = None
    if args.tfhe_steps > 0:
        print("[bench] TFHE-style yardstick", file=sys.stderr, flush=True)
        tfhe = tfhe_bench(fd, torch, ctx, d_cts, d_ids, B, args.tfhe_steps, wall / K * 1e3)

    sweep = None
    if args.config_sweep > 0:
        sweep = config_sweep(fd, torch, W, B, args.config_sweep)

    nn = None
    if args.nn_steps > 0:
        print("[bench] NN-shaped circuit", file=sys.stderr, flush=True)
        nn = nn_bench(fd, torch, W, args.nn_steps)

    pipe = None
    if args.pipeline_batches > 0:
        print(f"[bench] software pipeline of {args.pipeline_batches} batches", file=sys.stderr, flush=True)
        pipe = pipeline_bench(fd, torch, ctx, d_cts, d_ids, d_out, args.pipeline_batches, wall / K * 1e3)

    mixed = None
    if args.mixed_steps > 0:
        print("[bench] uneven two-degree batch", file=sys.stderr, flush=True)
        mixed = mixed_bench(fd, torch, W, ctx, args.mixed_steps)

    serving = None
    if args.serving_requests > 0:
        print(f"[bench] serving: {args.serving_requests} requests per run", file=sys.stderr, flush=True)
        serving = serving_bench(fd, torch, W, ctx, args.serving_requests)

    cpu = None
    if not args.no_cpu_baseline:
        # the host's CPU share on a one-GPU machine is 16 threads (os.cpu_count()
        # reports the whole machine there)
        threads = args.cpu_threads or min(os.cpu_count() or 1, 16)
        print(f"[bench] cpu baseline: oracle on {threads} threads and on one", file=sys.stderr, flush=True)
        cpu = cpu_baseline(p, cts, lut, threads, threads)

    bsweep = None
    if args.batch_sweep > 0:
        print("[bench] batch-size sweep", file=sys.stderr, flush=True)
        bsweep = batch_sweep(fd, torch, W, ctx, args.batch_sweep)

    otime = None
    if args.oracle_timing:
        threads = args.cpu_threads or min(os.cpu_count() or 1, 16)
        print(f"[bench] oracle timing on 1 and {threads} threads", file=sys.stderr, flush=True)
        otime = oracle_timing(threads)

    res = {
        "metric": METRIC,
        "value": B * K / wall,
        "unit": "bootstraps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": wall / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "FDFB batch of 1024 LWE samples, n=630 N=1024 q=2^32, gadget 2^7x3, "
                               "key switch 2^4x5, t=16, one random LUT",
                   "batch": B, "n": p.n, "N": p.N, "t": p.t, "blind_rotations_per_bootstrap": p.boot_ell + 1},
        "correct": correct,
        "plain": plain,
        "speedup_batched_vs_plain": (B * K / wall) / plain["value"] if plain else None,
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99)),
                       "what": "per-batch latency of 1024 bootstraps"},
        "phases_ms_per_step": {k: v / calls for k, v in phases.items()},
        "roofline": roofline,
        "serving": serving,
        "multi_lut": multi_lut,
        "signed_boot_digit": signed,
        "tfhe_yardstick": tfhe,
        "direct_form": direct,
        "pipeline": pipe,
        "mixed": mixed,
        "nn_circuit": nn,
        "tuned": tuned,
        "config_sweep": sweep,
        "cpu_baseline": cpu,
        "batch_sweep": bsweep,
        "oracle_timing": otime,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
