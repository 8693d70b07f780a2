"""Benchmark: full dendrogram of the n=32768 RMSD-like complete-linkage
workload on one MI355X, plus the batched workload against a per-instance
launch loop, plus the CPU oracle on a bounded sample.

Prints one JSON line.  A step is one hac_run over the whole n=32768 instance
(set-up, all 32767 merges, merge list back in device memory) with the input
already resident in HBM; HAC_PRESERVE_INPUT makes each step start from the
same input (the 4 GiB device-to-device copy is inside the timed step).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-batch] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "HBM GB/s & dendrogram s at n=32768; batched instances/s vs per-instance loop"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


PMC_PROFILE = os.path.join(ROOT, "profiles", "k_run_rmsd_like_n32768_pmc.md")
ENGINE_SOURCES = [os.path.join(ROOT, "paper_1709_06816_amd", "csrc", f) for f in ("hac_engine.hip", "hac_engine.h")]


def alg_bytes_merge_kernel(n, st):
    """Algorithmic HBM bytes of one launch of the merge kernel k_run: each
    Lance-Williams update of an entry reads D[i][k], D[j][k] and writes
    D[i][k], D[k][i] (16 bytes); each rescan reads one fp32 per live entry it
    visits; each merge writes a 16-byte record."""
    return 16.0 * st["update_elems"] + 4.0 * st["rescan_elems"] + 16.0 * (n - 1)


def alg_bytes_setup(n, preserve=True):
    """k_setup reads the strict upper triangle and writes its mirror; when the
    input is preserved it also writes the upper triangle into the library's
    working copy (no separate copy kernel)."""
    return (6.0 if preserve else 4.0) * n * (n - 1)


def measured_traffic(n):
    """HBM bytes per k_run launch from the committed counter profile, if it
    was taken on this input size with the engine sources as they are now."""
    import hashlib
    try:
        line = next(l for l in open(PMC_PROFILE) if l.startswith("pmc-json:"))
        rec = json.loads(line[len("pmc-json:"):])
    except (OSError, StopIteration, ValueError):
        return None, "no counter profile"
    h = hashlib.sha256()
    for p in ENGINE_SOURCES:
        with open(p, "rb") as fh:
            h.update(fh.read())
    if rec.get("engine_sha256") != h.hexdigest():
        return None, "engine changed since the counters were taken"
    if "n=%d" % n not in rec.get("workload", ""):
        return None, "counters were taken at another size"
    return rec["traffic_bytes"], os.path.relpath(PMC_PROFILE, ROOT)


def cpu_baseline(d, link, n, budget_s, gpu_prefix):
    """Time the oracle (unchanged) on the first K merges of the same input,
    K grown until the sample takes a few seconds of the budget, and
    extrapolate to the whole dendrogram by the number of cells its scan
    visits: merge s scans m(m-1)/2 cells with m = n - s live clusters."""
    import oracle
    threads = oracle.default_threads()
    t0 = time.perf_counter()
    oracle.run_f32(d, link, max_merges=0, threads=threads)
    t_setup = time.perf_counter() - t0
    k = 4
    t_k = None
    res = None
    while True:
        t0 = time.perf_counter()
        res = oracle.run_f32(d, link, max_merges=k, threads=threads)
        t_k = time.perf_counter() - t0
        if t_k - t_setup > budget_s / 3 or k >= n - 1:
            break
        k *= 2
    m = np.arange(2, n + 1, dtype=np.float64)
    cells_all = float(np.sum(m * (m - 1) / 2))
    ms = np.arange(n - k + 1, n + 1, dtype=np.float64)
    cells_k = float(np.sum(ms * (ms - 1) / 2))
    per_cell = max(t_k - t_setup, 1e-9) / cells_k
    t_full = t_setup + per_cell * cells_all
    prefix_ok = bool(res.tobytes() == gpu_prefix[:len(res)].tobytes())
    return {
        "value": 1.0 / t_full, "unit": "dendrograms/s", "cores": threads, "kind": "oracle",
        "sample": "first %d of %d merges of the same n=%d input (%.1f s incl. %.1f s set-up); "
                  "whole dendrogram extrapolated by scanned cells: %.0f s" % (k, n - 1, n, t_k, t_setup, t_full),
        "est_dendrogram_s": t_full,
        "parity_prefix_merges": int(len(res)),
        "parity_prefix_ok": prefix_ok,
    }


def batch_leg(torch, hac, ctx, count, n_lo, n_hi, reps):
    import synth
    spec = synth.batch_spec(count=count, n_lo=n_lo, n_hi=n_hi)
    offs, total = synth.pack_offsets(spec.ns)
    log("batch: generating %d instances (%.2f GB)" % (count, total * 4 / 1e9))
    host = np.empty(total, np.float32)
    for k, (n, s) in enumerate(zip(spec.ns, spec.seeds)):
        host[offs[k]:offs[k] + int(n) * int(n)] = synth.batch_instance(int(n), int(s)).ravel()
    src = torch.from_numpy(host).cuda()
    del host
    work = torch.empty_like(src)
    moff, mtot = synth.merge_offsets(spec.ns)
    out_b = torch.empty(mtot * 16, dtype=torch.uint8, device="cuda")
    out_l = torch.empty(mtot * 16, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    def one_batch():
        work.copy_(src)
        ctx.batch(work, offs, spec.ns, spec.linkages, out=out_b)
        ctx.sync()

    def one_loop():
        work.copy_(src)
        base = work.data_ptr()
        obase = out_l.data_ptr()
        for k in range(count):
            n = int(spec.ns[k])
            ctx.run_ptr(base + 4 * int(offs[k]), n, int(spec.linkages[k]),
                        out=obase + 16 * int(moff[k]))
        ctx.sync()

    one_batch()
    torch.cuda.synchronize()
    tb = []
    kb = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        one_batch()
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t0)
        kb.append(ctx.stats()["kernel_ms"])
    st = ctx.stats()
    # Algorithmic bytes of the batch kernel: every instance's set-up (read its
    # strict upper triangle, write the mirror) plus its merge loops, counted
    # as for the single-instance kernel.
    ns64 = spec.ns.astype(np.float64)
    alg = float(np.sum(4.0 * ns64 * (ns64 - 1.0))) + 16.0 * st["update_elems"] + 4.0 * st["rescan_elems"] \
        + 16.0 * float(mtot)
    log("batch: per-instance loop")
    one_loop()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    one_loop()
    torch.cuda.synchronize()
    tl = time.perf_counter() - t0
    same = bool(torch.equal(out_b, out_l))
    tbm = float(np.median(tb))
    return {
        "workload": "%d instances, n log-uniform in [%d, %d], linkage uniform over 4, "
                    "Gaussian mixtures in R^16, packed ragged (%.2f GB)" % (count, n_lo, n_hi, total * 4 / 1e9),
        "instances_per_s": count / tbm,
        "batch_s": tbm,
        "batch_kernel_ms": float(np.median(kb)),
        "loop_instances_per_s": count / tl,
        "loop_s": tl,
        "speedup_vs_loop": tl / tbm,
        "identical_to_loop": same,
        "merges": int(mtot),
        "alg_bytes": alg,
        "achieved_gbs": alg / (float(np.median(kb)) / 1000.0) / 1e9,
        "frac_hbm_peak": alg / (float(np.median(kb)) / 1000.0) / 1e9 / HBM_PEAK_GBS,
        "plan": {"block": st["block"], "group": st["group"], "workgroups": st["workgroups"],
                 "graph": st["graph"]},
    }


def scan_leg(torch, hac, ctx, n):
    """The paper's own step (Section 5.3 step 1): every merge rescans the live
    upper triangle instead of keeping row minima.  Same merge list as the
    cached path; reported beside it as the memory-bound reference."""
    import synth
    d = synth.mixture_8192(n=n)
    src = torch.from_numpy(d).cuda()
    out = {}
    for mode in ("cached", "scan"):
        ctx.run(src, "complete", preserve=True, scan=(mode == "scan"))
        st = ctx.stats()
        merges = ctx.run(src, "complete", preserve=True, scan=(mode == "scan"))
        st = ctx.stats()
        ab = alg_bytes_merge_kernel(n, st)
        out[mode] = {"kernel_ms": st["kernel_ms"], "alg_bytes": ab,
                     "achieved_gbs": ab / (st["kernel_ms"] / 1000.0) / 1e9,
                     "frac_hbm_peak": ab / (st["kernel_ms"] / 1000.0) / 1e9 / HBM_PEAK_GBS,
                     "scanned_elems": st["rescan_elems"], "records": merges}
    same = out["cached"].pop("records").tobytes() == out["scan"].pop("records").tobytes()
    return {"workload": "mixture n=%d (32 Gaussians in R^16), complete linkage" % n, "n": n,
            "identical_merge_lists": bool(same), **out,
            "note": "scan: every workgroup reads the live upper part of its rows before every merge"}


def serve_leg(torch, hac, ctx, requests, warmup, rate, budget_gb, big_n):
    """Continuous batching: Poisson arrivals submitted open-loop from host
    page-locked memory, latency = result on the host - scheduled arrival."""
    import synth
    n_hi = 16384
    pool_n = 2
    log("serve: generating %d pool matrices of n=%d" % (pool_n, n_hi))
    pool = [torch.empty((n_hi, n_hi), dtype=torch.float32).pin_memory() for _ in range(pool_n)]
    synth.serve_pool(pool_n, n_hi, out=[p.numpy() for p in pool])
    big = None
    if big_n:
        log("serve: generating the n=%d instance" % big_n)
        big = torch.empty((big_n, big_n), dtype=torch.float32).pin_memory()
        synth.mixture_65536(n=big_n, out=big.numpy())
    tr = synth.serve_trace(warmup + requests, rate=rate, n_hi=n_hi)
    srv = hac.Server(ctx, budget_bytes=int(budget_gb * (1 << 30)), max_jobs=1024,
                     max_n=max(n_hi, big_n or 0))
    res = {}
    try:
        big_alone = None
        if big is not None:
            log("serve: n=%d alone" % big_n)
            t0 = time.perf_counter()
            tk = srv.submit(big, "average")
            while True:
                r = srv.poll(tk)
                if r is not None:
                    break
                time.sleep(0.0005)
            big_alone = (time.perf_counter() - t0, r)
        big_at = warmup + requests // 4
        log("serve: %d requests at %.0f/s (+%d warm-up)" % (requests, rate, warmup))
        pending = {}
        done_t = {}
        results = {}
        big_mix = None
        t_start = time.perf_counter() + 0.05

        def poll_all():
            for k in list(pending):
                r = srv.poll(pending[k])
                if r is not None:
                    done_t[k] = time.perf_counter()
                    results[k] = r
                    del pending[k]

        for k in range(len(tr.ns)):
            due = t_start + float(tr.arrivals[k])
            while time.perf_counter() < due:
                poll_all()
                if due - time.perf_counter() > 0.002:
                    time.sleep(0.0005)
            n = int(tr.ns[k])
            while True:
                try:
                    pending[k] = srv.submit(pool[k % pool_n][:n, :n], int(tr.linkages[k]))
                    break
                except hac.HacError as e:
                    if e.code != hac.HAC_EBUSY:
                        raise
                    poll_all()
            if big is not None and k == big_at:
                big_mix = [time.perf_counter(), srv.submit(big, "average"), None]
            if big_mix is not None and big_mix[2] is None:
                r = srv.poll(big_mix[1])
                if r is not None:
                    big_mix[2] = (time.perf_counter() - big_mix[0], r)
        while pending or (big_mix is not None and big_mix[2] is None):
            poll_all()
            if big_mix is not None and big_mix[2] is None:
                r = srv.poll(big_mix[1])
                if r is not None:
                    big_mix[2] = (time.perf_counter() - big_mix[0], r)
            time.sleep(0.0002)
        meas = range(warmup, len(tr.ns))
        lat = np.array([done_t[k] - (t_start + float(tr.arrivals[k])) for k in meas]) * 1000.0
        span = max(done_t[k] for k in meas) - (t_start + float(tr.arrivals[warmup]))
        mbytes = float(sum(4.0 * int(tr.ns[k]) ** 2 for k in meas))
        # Alone vs in the mix: a sample of requests again, one at a time.
        rng = np.random.default_rng(7)
        sample = sorted(rng.choice(np.arange(warmup, len(tr.ns)), size=min(48, requests), replace=False))
        same = True
        for k in sample:
            n = int(tr.ns[k])
            tk = srv.submit(pool[k % pool_n][:n, :n], int(tr.linkages[k]))
            while True:
                r = srv.poll(tk)
                if r is not None:
                    break
                time.sleep(0.0002)
            same &= r.tobytes() == results[k].tobytes()
        st = srv.stats()
        res = {
            "workload": "Poisson arrivals at %.0f/s, n log-uniform on [256, %d], linkage uniform over 4, "
                        "Gaussian mixtures in R^16 (top-left blocks of %d page-locked %d-point mixtures), "
                        "HBM budget %.0f GB" % (rate, n_hi, pool_n, n_hi, budget_gb),
            "requests": requests, "warmup": warmup,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
            "jobs_per_s": requests / span, "nominal_rate_per_s": rate,
            "offered_jobs_per_s": (requests - 1) / float(tr.arrivals[len(tr.ns) - 1] - tr.arrivals[warmup]),
            "matrix_gb_per_s": mbytes / span / 1e9,
            "alone_vs_mix_identical": bool(same), "alone_vs_mix_sample": len(sample),
            "peak_gb": st["peak_bytes"] / 1e9, "kernel_launches": st["kernel_launches"],
            "workgroups": st["workgroups"], "block": st["block"],
        }
        if big is not None:
            res["big"] = {"n": big_n, "linkage": "average",
                          "alone_s": big_alone[0], "in_mix_latency_s": big_mix[2][0],
                          "identical": bool(big_alone[1].tobytes() == big_mix[2][1].tobytes())}
    finally:
        srv.close()
    return res


FP32_MFMA_PEAK_TFLOPS = 157.3


def rmsd_leg(torch, hac, ctx, n, atoms, reps):
    """The input producer (hac_rmsd): the n x n superposed-RMSD matrix of n
    conformations of ``atoms`` atoms.  Algorithmic work: the nine
    cross-covariance sums of every pair in the strict upper triangle,
    2 * 9 * atoms flops per pair on the fp32 matrix cores (the fp64
    per-pair eigenvalue epilogue is not counted).  Timed with HIP events on
    the stream the kernels run on (torch's current stream)."""
    import synth
    coords = torch.from_numpy(synth.conformations(n, atoms)).cuda()
    out = torch.empty((n, n), dtype=torch.float32, device="cuda")
    ctx.rmsd(coords, out=out)  # warm-up (workspace allocation)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        ctx.rmsd(coords, out=out)
        b.record()
    torch.cuda.synchronize()
    ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    pairs = n * (n - 1) / 2.0
    flops = pairs * 18.0 * atoms
    tflops = flops / (ms / 1000.0) / 1e12
    del out, coords
    torch.cuda.empty_cache()
    return {"workload": "%d conformations of a %d-atom chain (64 folding states, per-atom noise, random "
                        "placement)" % (n, atoms), "n": n, "atoms": atoms, "reps": reps, "ms": ms,
            "pairs_per_s": pairs / (ms / 1000.0),
            "roofline": {"bound": "mfma", "achieved": tflops, "peak": FP32_MFMA_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": tflops / FP32_MFMA_PEAK_TFLOPS,
                         "alg_flops": flops, "kernel": "k_rmsd_tiles (with k_rmsd_prep)",
                         "out_bytes": pairs * 4.0,
                         "note": "fp32 16x16x4 MFMA cross-covariances, fp64 eigenvalue epilogue per pair"}}


def rmsd_cpu_baseline(n, atoms, pairs):
    """The RMSD oracle (fp64 Kabsch, numpy) on a bounded sample of pairs of
    the same conformations, as pairs per second."""
    import synth
    from oracle import rmsd as rmsd_oracle
    coords = synth.conformations(n, atoms)
    rng = np.random.default_rng(0)
    rows = rng.integers(0, n, size=pairs)
    cols = rng.integers(0, n, size=pairs)
    t0 = time.perf_counter()
    rmsd_oracle.rmsd_pairs(coords, rows, cols)
    dt = time.perf_counter() - t0
    return {"value": pairs / dt, "unit": "pairs/s", "kind": "oracle", "cores": 1,
            "sample": "%d random pairs of the same %d conformations (%.1f s)" % (pairs, n, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-count", type=int, default=1024)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--workgroups", type=int, default=0)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-scan", action="store_true")
    ap.add_argument("--scan-n", type=int, default=8192)
    ap.add_argument("--no-rmsd", action="store_true")
    ap.add_argument("--rmsd-n", type=int, default=32768)
    ap.add_argument("--rmsd-atoms", type=int, default=128)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=100)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-budget-gb", type=float, default=200.0)
    ap.add_argument("--serve-big-n", type=int, default=65536, help="0: no big instance")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 1 GiB device-to-device (a reference kernel of known "
                         "traffic for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1709_06816_amd as hac
    import synth

    if args.calibrate_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    n = args.n
    link = "complete"
    seed = synth.BASE_SEED + 3
    log("generating rmsd_like n=%d" % n)
    d = synth.rmsd_like(seed=seed, n=n)
    src = torch.from_numpy(d).cuda()
    ctx = hac.Context(0)
    if args.workgroups:
        ctx.set_option(hac.OPT_WORKGROUPS, args.workgroups)
    out = torch.empty((n - 1) * 16, dtype=torch.uint8, device="cuda")

    def step():
        ctx.run(src, link, preserve=True, out=out)

    log("warmup %d" % args.warmup)
    for _ in range(args.warmup):
        step()
        ctx.sync()
    torch.cuda.synchronize()
    kms, ims, stats = [], [], None
    log("timing %d steps" % args.steps)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
        ctx.sync()
        stats = ctx.stats()
        kms.append(stats["kernel_ms"])
        ims.append(stats["init_ms"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = elapsed * 1000.0 / args.steps
    merges = np.frombuffer(out.cpu().numpy().tobytes(), dtype=hac.MERGE_DTYPE)
    kernel_ms = float(np.mean(kms))
    ab = alg_bytes_merge_kernel(n, stats)
    achieved = ab / (kernel_ms / 1000.0) / 1e9
    traffic, traffic_src = measured_traffic(n)
    init_ms = float(np.mean(ims))
    log("step %.1f ms, merge kernel %.1f ms, %d workgroups" % (ms_step, kernel_ms, stats["workgroups"]))

    result = {
        "metric": METRIC,
        "value": 1000.0 / ms_step,
        "unit": "dendrograms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "rmsd_like n=%d complete linkage (R^30, 64 anisotropic clusters, "
                               "distances scaled to [0,20] and rounded to 1e-3)" % n,
                   "n": n, "linkage": link, "seed": seed, "parallelism": "1 GPU"},
        "dendrogram_s": ms_step / 1000.0,
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_source": traffic_src,
            "kernel": "k_run (persistent merge kernel)", "kernel_ms": kernel_ms,
            "alg_bytes_per_launch": ab, "workgroups": stats["workgroups"],
            "rescans": stats["rescans"], "rescan_elems": stats["rescan_elems"],
            "update_elems": stats["update_elems"],
            "deferred_rescans": bool(stats["deferred"]), "forced_rounds": stats["forced_rounds"],
            "merge_rounds": stats["rounds"],
            "traffic_gbs": None if traffic is None else traffic / (kernel_ms / 1000.0) / 1e9,
            "note": "latency-bound: one grid-wide exchange per merge; rescans run during the exchange wait",
            "setup_kernel": {"kernel": "k_setup", "ms": init_ms, "alg_bytes": alg_bytes_setup(n),
                             "achieved_gbs": alg_bytes_setup(n) / (init_ms / 1000.0) / 1e9
                             if init_ms > 0 else None},
        },
    }
    if not args.no_scan:
        log("paper scan mode at n=%d" % args.scan_n)
        result["paper_scan_mode"] = scan_leg(torch, hac, ctx, args.scan_n)
    if not args.no_rmsd:
        log("input producer: rmsd n=%d atoms=%d" % (args.rmsd_n, args.rmsd_atoms))
        result["input_producer"] = rmsd_leg(torch, hac, ctx, args.rmsd_n, args.rmsd_atoms, reps=5)
        log("rmsd %.2f ms" % result["input_producer"]["ms"])
    if not args.no_batch:
        log("batch leg")
        result["batched"] = batch_leg(torch, hac, ctx, args.batch_count, 64, 4096, reps=3)
    if not args.no_serve:
        del src
        torch.cuda.empty_cache()
        log("serving leg")
        result["serving"] = serve_leg(torch, hac, ctx, args.serve_requests, args.serve_warmup,
                                      args.serve_rate, args.serve_budget_gb, args.serve_big_n)
    if not args.no_cpu and "input_producer" in result:
        log("cpu baseline of the input producer")
        result["input_producer"]["cpu_baseline"] = rmsd_cpu_baseline(args.rmsd_n, args.rmsd_atoms, 200000)
    if not args.no_cpu:
        log("cpu baseline")
        result["cpu_baseline"] = cpu_baseline(d, link, n, args.cpu_budget, merges)
    ctx.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
