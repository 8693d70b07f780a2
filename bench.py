"""Benchmark of the Lance-Williams clustering library on one MI355X.

Prints one JSON line.  The headline is the n=32768 RMSD-like complete-linkage
dendrogram through the default path of hac_run (rounds
of reciprocal-nearest-neighbour merges, the tail handed to the
one-merge-per-step kernel); a step is one hac_run over the whole instance
(set-up, all 32767 merges, records sorted into merge order in device memory)
with the input already in HBM; HAC_PRESERVE_INPUT makes each step start from
the same input (the working copy is written by the set-up kernel inside the
step).  Beside it, on the same input: the one-merge-per-step engine and the
paper's own full scan before every merge (HAC_MODE_SCAN), each compared byte
for byte with the headline list; per-workload lines for the n=512 and
n=8192 workloads (GPU and oracle times, bit-exact flags, error against an
fp64 replay); the 1024-instance batch against a per-instance loop; serving
under Poisson arrivals, at saturation and against a per-instance loop; the
RMSD input producer; and the CPU oracle on bounded samples.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-batch] [--no-cpu]
                    [--no-serve] [--no-scan] [--no-rmsd] [--no-configs]
"""
import argparse
import hashlib
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
GOLDEN = os.path.join(ROOT, "tests", "golden", "oracle_digests.json")
CSRC = os.path.join(ROOT, "paper_1709_06816_amd", "csrc")
# Counter profiles: kernel -> (file, sources whose hash the counters were taken on).
PROFILES = {
    "k_rounds": ("k_rounds_rmsd_like_n32768_pmc.md", ["hac_rounds.hip", "hac_rounds.h", "hac_dev.h",
                                                      "hac_engine.h"]),
    "k_scan": ("k_scan_rmsd_like_n32768_pmc.md", ["hac_scan.hip", "hac_scan.h", "hac_dev.h"]),
    "k_run": ("k_run_rmsd_like_n32768_pmc.md", ["hac_engine.hip", "hac_engine.h", "hac_dev.h"]),
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def alg_bytes_merge(n, st):
    """Algorithmic HBM bytes of one merge-kernel run: each Lance-Williams
    update of an entry reads D[i][k], D[j][k] and writes D[i][k], D[k][i]
    (16 bytes); each rescanned (or, in scan mode, scanned) live entry is
    read once (4 bytes); each merge writes a 16-byte record."""
    return 16.0 * st["update_elems"] + 4.0 * st["rescan_elems"] + 16.0 * (n - 1)


def alg_bytes_setup(n, preserve=True):
    """k_setup reads the strict upper triangle and writes its mirror; when the
    input is preserved it also writes the upper triangle into the library's
    working copy (no separate copy kernel)."""
    return (6.0 if preserve else 4.0) * n * (n - 1)


def measured_traffic(kernel, n):
    """HBM bytes per launch of `kernel` from its committed counter profile,
    if taken at this size on the sources as they are now."""
    fname, srcs = PROFILES[kernel]
    path = os.path.join(ROOT, "profiles", fname)
    try:
        line = next(l for l in open(path) if l.startswith("pmc-json:"))
        rec = json.loads(line[len("pmc-json:"):])
    except (OSError, StopIteration, ValueError):
        return None, "no counter profile"
    h = hashlib.sha256()
    for f in srcs:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    if rec.get("engine_sha256") != h.hexdigest():
        return None, "sources changed since the counters were taken"
    if "n=%d" % n not in rec.get("workload", ""):
        return None, "counters were taken at another size"
    return rec["traffic_bytes"], os.path.relpath(path, ROOT)


def golden(key):
    try:
        with open(GOLDEN) as f:
            return json.load(f).get(key)
    except (OSError, ValueError):
        return None


def records_sha(rec_bytes):
    return hashlib.sha256(rec_bytes).hexdigest()


def roofline(achieved_bytes, ms, traffic, traffic_src, kernel, extra=None):
    gbs = achieved_bytes / (ms / 1000.0) / 1e9
    r = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
         "traffic": traffic, "traffic_source": traffic_src, "kernel": kernel, "kernel_ms": ms,
         "alg_bytes_per_launch": achieved_bytes,
         "traffic_gbs": None if traffic is None else traffic / (ms / 1000.0) / 1e9}
    if extra:
        r.update(extra)
    return r


def cpu_baseline(d, link, n, budget_s, gpu_list, gold):
    """Time the oracle (unchanged) on the first K merges of the same input,
    K grown until the sample takes a few seconds of the budget, and
    extrapolate to the whole dendrogram by the number of cells its scan
    visits: merge s scans m(m-1)/2 cells with m = n - s live clusters.  The
    GPU list is compared with the oracle's sample and, when the stored digest
    of the oracle's full list is present, with all of it."""
    import oracle
    threads = oracle.default_threads()
    t0 = time.perf_counter()
    oracle.run_f32(d, link, max_merges=0, threads=threads)
    t_setup = time.perf_counter() - t0
    k = 4
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
    out = {
        "value": 1.0 / t_full, "unit": "dendrograms/s", "cores": threads, "kind": "oracle",
        "sample": "first %d of %d merges of the same n=%d input (%.1f s incl. %.1f s set-up); "
                  "whole dendrogram extrapolated by scanned cells: %.0f s" % (k, n - 1, n, t_k, t_setup, t_full),
        "est_dendrogram_s": t_full,
        "sample_merges_identical": bool(res.tobytes() == gpu_list[:len(res)].tobytes()),
    }
    if gold is not None:
        out["full_list_identical_to_oracle"] = records_sha(gpu_list.tobytes()) == gold["records_sha256"]
        out["oracle_full_run_s"] = gold["oracle_seconds"]
        out["oracle_full_run_threads"] = gold["oracle_threads"]
        out["oracle_full_run_note"] = "measured when the stored digest was written (tests/golden/make_digests.py)"
    return out


def run_timed(ctx, src, link, steps, out, **kw):
    """`steps` hac_run calls; returns (median kernel_ms, median init_ms, wall ms per step, stats)."""
    kms, ims = [], []
    st = None
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.run(src, link, preserve=True, out=out, **kw)
        ctx.sync()
        st = ctx.stats()
        kms.append(st["kernel_ms"])
        ims.append(st["init_ms"])
    wall = (time.perf_counter() - t0) * 1000.0 / steps
    return float(np.median(kms)), float(np.median(ims)), wall, st


def engines_leg(torch, hac, ctx, src, n, link, headline_rec, scan):
    """The other engines on the headline input: one merge per step (64
    workgroups, deferred rescans) and the paper's full scan before every
    merge, each with its bytes and time; lists compared with the headline's."""
    res = {}
    out = torch.empty((n - 1) * 16, dtype=torch.uint8, device="cuda")
    ctx.set_option(hac.OPT_ROUNDS, 0)
    try:
        log("one-merge-per-step engine")
        run_timed(ctx, src, link, 1, out)
        kms, ims, wall, st = run_timed(ctx, src, link, 3, out)
    finally:
        ctx.set_option(hac.OPT_ROUNDS, 1)
    ab = alg_bytes_merge(n, st)
    traffic, tsrc = measured_traffic("k_run", n)
    res["one_merge_per_step"] = {
        "kernel": "k_run (%d workgroups, deferred rescans)" % st["workgroups"], "dendrogram_ms": wall,
        "kernel_ms": kms, "alg_bytes": ab,
        "roofline": roofline(ab, kms, traffic, tsrc, "k_run"),
        "forced_rounds": st["forced_rounds"],
        "identical_to_headline": out.cpu().numpy().tobytes() == headline_rec}
    if scan:
        log("paper scan mode (Section 5.3 step 1) at n=%d" % n)
        kms, ims, wall, st = run_timed(ctx, src, link, 1, out, scan=True)
        ab = alg_bytes_merge(n, st)
        traffic, tsrc = measured_traffic("k_scan", n)
        res["paper_scan_mode"] = {
            "kernel": "k_scan (%d workgroups)" % st["workgroups"], "dendrogram_ms": wall, "kernel_ms": kms,
            "compactions": st["compactions"], "scanned_live_entries": st["rescan_elems"],
            "roofline": roofline(ab, kms, traffic, tsrc, "k_scan",
                                 {"note": "the whole live upper triangle read before every merge; 4 B per "
                                          "live entry scanned + 16 B per updated entry + 16 B per record"}),
            "identical_to_headline": out.cpu().numpy().tobytes() == headline_rec}
    del out
    return res


def config_lines(torch, hac, ctx, cpu):
    """Workloads 1 and 2: GPU time (default path), the oracle's time on this
    host, bit-exactness, and the largest relative height error against an
    fp64 replay of the same merge list."""
    import oracle
    import synth
    lines = []
    jobs = [("mixture n=512 (8 isotropic Gaussians in R^8)", synth.mixture_512(), ["complete"], synth.BASE_SEED + 1),
            ("mixture n=8192 (32 Gaussians in R^16)", synth.mixture_8192(), ["single", "complete", "average", "ward"],
             synth.BASE_SEED + 2)]
    threads = oracle.default_threads()
    for name, d, links, seed in jobs:
        n = d.shape[0]
        src = torch.from_numpy(d).cuda()
        out = torch.empty((n - 1) * 16, dtype=torch.uint8, device="cuda")
        for link in links:
            log("workload %s %s" % (name, link))
            run_timed(ctx, src, link, 1, out)
            kms, ims, wall, st = run_timed(ctx, src, link, 5, out)
            got = np.frombuffer(out.cpu().numpy().tobytes(), dtype=hac.MERGE_DTYPE)
            line = {"workload": name, "n": n, "linkage": link, "seed": seed, "gpu_ms": wall, "kernel_ms": kms,
                    "setup_ms": ims, "engine": "rounds" if st["rounds"] else "one merge per step",
                    "rounds": st["rounds"], "handed_over": bool(st["handed_over"])}
            if cpu:
                t0 = time.perf_counter()
                exp = oracle.run_f32(d, link, threads=threads)
                t_or = time.perf_counter() - t0
                h64, _ = oracle.replay_f64(d, link, got, threads=threads)
                err = np.abs(got["h"].astype(np.float64) - h64) / np.maximum(np.abs(h64), 1e-300)
                line.update({"oracle_s": t_or, "oracle_cores": threads, "speedup": t_or * 1000.0 / wall,
                             "bit_exact": got.tobytes() == exp.tobytes(),
                             "max_rel_err_vs_fp64": float(err.max()) if len(err) else 0.0})
            lines.append(line)
        del src, out
    return lines


def batch_leg(torch, hac, ctx, count, n_lo, n_hi, reps, cpu):
    import synth
    spec = synth.batch_spec(count=count, n_lo=n_lo, n_hi=n_hi)
    offs, total = synth.pack_offsets(spec.ns)
    log("batch: generating %d instances (%.2f GB)" % (count, total * 4 / 1e9))
    host = np.empty(total, np.float32)
    for k, (n, s) in enumerate(zip(spec.ns, spec.seeds)):
        host[offs[k]:offs[k] + int(n) * int(n)] = synth.batch_instance(int(n), int(s)).ravel()
    src = torch.from_numpy(host).cuda()
    work = torch.empty_like(src)
    moff, mtot = synth.merge_offsets(spec.ns)
    out_b = torch.empty(mtot * 16, dtype=torch.uint8, device="cuda")
    out_l = torch.empty(mtot * 16, dtype=torch.uint8, device="cuda")

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
            ctx.run_ptr(base + 4 * int(offs[k]), n, int(spec.linkages[k]), out=obase + 16 * int(moff[k]))
        ctx.sync()

    one_batch()
    torch.cuda.synchronize()
    tb, kb = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        one_batch()
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t0)
        kb.append(ctx.stats()["kernel_ms"])
    st = ctx.stats()
    ns64 = spec.ns.astype(np.float64)
    # Set-up (read the upper triangle, write its mirror), then 12 B per updated
    # entry (the batch kernel's lazy mirror reads D_ik, D_jk and writes D_ik
    # only), 4 B per rescanned live entry and 16 B per record.
    alg = float(np.sum(4.0 * ns64 * (ns64 - 1.0))) + 12.0 * st["update_elems"] + 4.0 * st["rescan_elems"] \
        + 16.0 * float(mtot)
    log("batch: per-instance loop")
    one_loop()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    one_loop()
    torch.cuda.synchronize()
    tl = time.perf_counter() - t0
    rec = out_b.cpu().numpy().tobytes()
    same = rec == out_l.cpu().numpy().tobytes()
    tbm = float(np.median(tb))
    kbm = float(np.median(kb))
    res = {
        "workload": "%d instances, n log-uniform in [%d, %d], linkage uniform over 4, "
                    "Gaussian mixtures in R^16, packed ragged (%.2f GB)" % (count, n_lo, n_hi, total * 4 / 1e9),
        "instances_per_s": count / tbm, "batch_s": tbm, "batch_kernel_ms": kbm,
        "loop_instances_per_s": count / tl, "loop_s": tl, "speedup_vs_loop": tl / tbm,
        "identical_to_loop": same, "merges": int(mtot), "alg_bytes": alg,
        "achieved_gbs": alg / (kbm / 1000.0) / 1e9, "frac_hbm_peak": alg / (kbm / 1000.0) / 1e9 / HBM_PEAK_GBS,
        "plan": {"block": st["block"], "group": st["group"], "workgroups": st["workgroups"], "graph": st["graph"],
                 "share_quarters": st["plan_share"], "update_chunks": st["plan_update"], "source": st["plan_source"]},
    }
    gold = golden("batch_1024")
    if gold is not None and count == gold["count"]:
        bad = [k for k, n in enumerate(spec.ns)
               if records_sha(rec[16 * int(moff[k]):16 * (int(moff[k]) + int(n) - 1)]) != gold["records_sha256"][k]]
        res["instances_identical_to_oracle"] = count - len(bad)
        res["oracle_full_batch_s"] = gold["oracle_seconds"]
        res["oracle_full_batch_threads"] = gold["oracle_threads"]
    if cpu:
        # The oracle, one instance per thread, on a bounded sample of the
        # instances; extrapolated to the batch by its scanned cells.
        import concurrent.futures as cf
        import oracle
        rng = np.random.default_rng(3)
        pick = rng.choice(count, size=min(48, count), replace=False)
        threads = oracle.default_threads()

        def one(k):
            n = int(spec.ns[k])
            return oracle.run_f32(host[offs[k]:offs[k] + n * n].reshape(n, n), int(spec.linkages[k]), threads=1)

        t0 = time.perf_counter()
        with cf.ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(one, pick))
        t_s = time.perf_counter() - t0
        cells = ns64 ** 3 / 6.0
        res["cpu_baseline"] = {"value": len(pick) / t_s * float(cells[pick].sum() / len(pick)) / float(cells.mean()),
                               "unit": "instances/s", "cores": threads, "kind": "oracle",
                               "sample": "%d random instances of the batch, one per thread (%.1f s), scaled to the "
                                         "batch's mix by n^3/6 scanned cells" % (len(pick), t_s)}
    del src, work, out_b, out_l, host
    torch.cuda.empty_cache()
    return res


def serve_leg(torch, hac, ctx, requests, warmup, rate, budget_gb, big_n, loop_jobs):
    """Continuous batching: Poisson arrivals submitted open-loop from host
    page-locked memory, latency = result on the host - scheduled arrival;
    then every request at once (saturation); then the same jobs through a
    per-instance hac_run loop (copy in, run, records back) with the same
    arrival times.  Requests cut the top-left n x n block of one of 16
    independent Gaussian mixtures of 16384 points each (block = the distance
    matrix of the mixture's first n points)."""
    import synth
    n_hi, pool_n = 16384, 16
    log("serve: generating %d mixtures of n=%d" % (pool_n, n_hi))
    pool = [torch.empty((n_hi, n_hi), dtype=torch.float32).pin_memory() for _ in range(pool_n)]
    synth.serve_pool(pool_n, n_hi, out=[p.numpy() for p in pool])
    tr = synth.serve_trace(warmup + requests, rate=rate, n_hi=n_hi)
    srv = hac.Server(ctx, budget_bytes=int(budget_gb * 1e9), max_jobs=1024, max_n=max(n_hi, big_n or 0))
    res = {}

    def job(k):
        n = int(tr.ns[k])
        return pool[k % pool_n][:n, :n], int(tr.linkages[k])

    def wait(tk):
        while True:
            r = srv.poll(tk)
            if r is not None:
                return r
            time.sleep(0.0002)

    try:
        big = None
        if big_n:
            log("serve: generating the n=%d instance" % big_n)
            big = torch.empty((big_n, big_n), dtype=torch.float32).pin_memory()
            synth.mixture_65536(n=big_n, out=big.numpy())
            log("serve: n=%d alone" % big_n)
            t0 = time.perf_counter()
            big_alone = (None, wait(srv.submit(big, "average")))
            big_alone = (time.perf_counter() - t0, big_alone[1])
        big_at = warmup + requests // 4
        log("serve: %d requests at %.0f/s (+%d warm-up)" % (requests, rate, warmup))
        pending, done_t, results = {}, {}, {}
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
            m, link = job(k)
            while True:
                try:
                    pending[k] = srv.submit(m, link)
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

        log("serve: saturation (all %d requests at once)" % requests)
        sat_pending, sat_res = {}, {}
        t0 = time.perf_counter()
        for k in meas:
            m, link = job(k)
            while True:
                try:
                    sat_pending[k] = srv.submit(m, link)
                    break
                except hac.HacError as e:
                    if e.code != hac.HAC_EBUSY:
                        raise
                    for q in list(sat_pending):
                        r = srv.poll(sat_pending[q])
                        if r is not None:
                            sat_res[q] = r
                            del sat_pending[q]
        while sat_pending:
            for q in list(sat_pending):
                r = srv.poll(sat_pending[q])
                if r is not None:
                    sat_res[q] = r
                    del sat_pending[q]
            time.sleep(0.0002)
        t_sat = time.perf_counter() - t0
        same = all(sat_res[k].tobytes() == results[k].tobytes() for k in meas)
        st = srv.stats()
    finally:
        srv.close()

    # The same jobs, one hac_run after another on one stream, arriving at the
    # same (relative) times: a job starts when it has arrived and the
    # previous one is done.
    log("serve: per-instance hac_run loop over %d of the requests" % loop_jobs)
    lk = list(range(warmup, warmup + loop_jobs))
    dev = torch.empty((n_hi, n_hi), dtype=torch.float32, device="cuda")
    loop_lat, same_loop = [], True
    t0 = time.perf_counter() + 0.05
    base = float(tr.arrivals[lk[0]])
    for k in lk:
        due = t0 + float(tr.arrivals[k]) - base
        while time.perf_counter() < due:
            time.sleep(0.0002)
        m, link = job(k)
        n = m.shape[0]
        d = dev.view(-1)[:n * n].view(n, n)
        d.copy_(m, non_blocking=True)
        r = ctx.run(d, link)
        loop_lat.append((time.perf_counter() - due) * 1000.0)
        same_loop &= r.tobytes() == results[k].tobytes()
    t_loop = time.perf_counter() - t0 - 0.05
    del dev
    torch.cuda.empty_cache()
    res = {
        "workload": "Poisson arrivals at %.0f/s, n log-uniform on [256, %d], linkage uniform over 4, "
                    "top-left blocks of %d independent Gaussian mixtures in R^16 (K ~ U{2..32}, sigma ~ "
                    "U[0.5, 2]) in page-locked memory, HBM budget %.0f GB" % (rate, n_hi, pool_n, budget_gb),
        "requests": requests, "warmup": warmup,
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
        "jobs_per_s": requests / span, "nominal_rate_per_s": rate,
        "offered_jobs_per_s": (requests - 1) / float(tr.arrivals[len(tr.ns) - 1] - tr.arrivals[warmup]),
        "matrix_gb_per_s": mbytes / span / 1e9,
        "saturation_jobs_per_s": requests / t_sat, "saturation_s": t_sat,
        "saturation_identical_to_poisson_run": bool(same),
        "peak_gb": st["peak_bytes"] / 1e9, "kernel_launches": st["kernel_launches"],
        "workgroups": st["workgroups"], "block": st["block"],
        "per_instance_loop": {"jobs": loop_jobs, "p50_ms": float(np.percentile(loop_lat, 50)),
                              "p99_ms": float(np.percentile(loop_lat, 99)), "jobs_per_s": loop_jobs / t_loop,
                              "identical_to_served": bool(same_loop),
                              "note": "hac_run per job (host-to-device copy, run, records back) with the same "
                                      "relative arrival times"},
    }
    if big is not None:
        res["big"] = {"n": big_n, "linkage": "average", "alone_s": big_alone[0], "in_mix_latency_s": big_mix[2][0],
                      "identical": bool(big_alone[1].tobytes() == big_mix[2][1].tobytes())}
        del big
    del pool
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
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-scan", action="store_true")
    ap.add_argument("--no-engines", action="store_true", help="skip the other engines on the headline input")
    ap.add_argument("--no-configs", action="store_true", help="skip the n=512 and n=8192 workload lines")
    ap.add_argument("--no-rmsd", action="store_true")
    ap.add_argument("--rmsd-n", type=int, default=32768)
    ap.add_argument("--rmsd-atoms", type=int, default=128)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=100)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-budget-gb", type=float, default=200.0)
    ap.add_argument("--serve-big-n", type=int, default=65536, help="0: no big instance")
    ap.add_argument("--serve-loop-jobs", type=int, default=400)
    ap.add_argument("--only-scan", action="store_true", help="headline input through scan mode only (profiling)")
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
    out = torch.empty((n - 1) * 16, dtype=torch.uint8, device="cuda")
    if args.only_scan:
        kms, ims, wall, st = run_timed(ctx, src, link, 1, out, scan=True)
        print(json.dumps({"only_scan": True, "n": n, "kernel_ms": kms, "dendrogram_ms": wall,
                          "alg_bytes": alg_bytes_merge(n, st), "compactions": st["compactions"],
                          "scanned_live_entries": st["rescan_elems"], "update_elems": st["update_elems"]}),
              flush=True)
        ctx.close()
        return

    log("warmup %d" % args.warmup)
    for _ in range(args.warmup):
        ctx.run(src, link, preserve=True, out=out)
        ctx.sync()
    torch.cuda.synchronize()
    log("timing %d steps" % args.steps)
    kms, ims, rms, stats = [], [], [], None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.run(src, link, preserve=True, out=out)
        ctx.sync()
        stats = ctx.stats()
        kms.append(stats["kernel_ms"])
        ims.append(stats["init_ms"])
        rms.append(stats["rounds_ms"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = elapsed * 1000.0 / args.steps
    rec = out.cpu().numpy().tobytes()
    merges = np.frombuffer(rec, dtype=hac.MERGE_DTYPE)
    kernel_ms = float(np.mean(kms))
    init_ms = float(np.mean(ims))
    rounds_ms = float(np.mean(rms))
    # The round engine's kernel alone (HIP events around its launch): its own
    # updated and rescanned entries, and the records of its merges.
    ab = alg_bytes_merge(n, {"update_elems": stats["rounds_update_elems"],
                             "rescan_elems": stats["rounds_rescan_elems"]})
    traffic, traffic_src = measured_traffic("k_rounds", n)
    gold = golden("rmsd_like_n32768_complete") if n == 32768 else None
    log("step %.1f ms, merge kernels %.1f ms, %d rounds" % (ms_step, kernel_ms, stats["rounds"]))

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
        "config": {"workload": "rmsd_like n=%d complete linkage (R^30, 64 anisotropic clusters, distances scaled "
                               "to [0,20] and rounded to 1e-3)" % n,
                   "n": n, "linkage": link, "seed": seed, "parallelism": "1 GPU"},
        "dendrogram_s": ms_step / 1000.0,
        "full_list_identical_to_oracle": None if gold is None else records_sha(rec) == gold["records_sha256"],
        "roofline": roofline(ab, rounds_ms, traffic, traffic_src,
                             "k_rounds (rounds of reciprocal-nearest-neighbour merges)",
                             {"merge_phase_ms": kernel_ms,
                              "merge_phase_note": "k_rounds, the one-merge-per-step kernel that takes over for "
                                                  "the last merges, and the record sort",
                              "workgroups": stats["workgroups"], "rounds": stats["rounds"],
                              "handed_over": bool(stats["handed_over"]), "rescans": stats["rescans"],
                              "rescan_elems": stats["rescan_elems"], "update_elems": stats["update_elems"],
                              "setup_kernel": {"kernel": "k_setup", "ms": init_ms, "alg_bytes": alg_bytes_setup(n),
                                               "achieved_gbs": alg_bytes_setup(n) / (init_ms / 1000.0) / 1e9
                                               if init_ms > 0 else None}}),
    }
    if not args.no_engines:
        result["engines"] = engines_leg(torch, hac, ctx, src, n, link, rec, not args.no_scan)
    del src
    torch.cuda.empty_cache()
    if not args.no_configs:
        result["workloads"] = config_lines(torch, hac, ctx, not args.no_cpu)
    if not args.no_rmsd:
        log("input producer: rmsd n=%d atoms=%d" % (args.rmsd_n, args.rmsd_atoms))
        result["input_producer"] = rmsd_leg(torch, hac, ctx, args.rmsd_n, args.rmsd_atoms, reps=5)
    if not args.no_batch:
        log("batch leg")
        result["batched"] = batch_leg(torch, hac, ctx, args.batch_count, 64, 4096, 3, not args.no_cpu)
    if not args.no_serve:
        log("serving leg")
        result["serving"] = serve_leg(torch, hac, ctx, args.serve_requests, args.serve_warmup, args.serve_rate,
                                      args.serve_budget_gb, args.serve_big_n, args.serve_loop_jobs)
    if not args.no_cpu and "input_producer" in result:
        log("cpu baseline of the input producer")
        result["input_producer"]["cpu_baseline"] = rmsd_cpu_baseline(args.rmsd_n, args.rmsd_atoms, 200000)
    if not args.no_cpu:
        log("cpu baseline")
        result["cpu_baseline"] = cpu_baseline(d, link, n, args.cpu_budget, merges, gold)
    ctx.close()
    torch.cuda.synchronize()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
