"""Write the oracle's full merge lists for the large workloads as SHA-256
digests into tests/golden/oracle_digests.json.

Calls only ``oracle`` (the fp32 Lance-Williams loop of Section 4, steps 1-4,
with the Table 1 coefficients) and ``synth`` (the seeded inputs); nothing here
touches the GPU library.  The GPU tests compare the device's merge lists with
these digests byte for byte.

Each entry records the workload, the SHA-256 of the input's strict upper
triangle (so a test can tell a different input from a different result), the
number of merges and the SHA-256 of the merge records (16 bytes each:
int32 i, int32 j, float32 height, int32 size, little-endian), plus the first
and last records in clear.

    python tests/golden/make_digests.py [--only KEY ...] [--threads T]

Keys:
  rmsd_like_n32768_complete   n=32768 RMSD-like matrix, complete linkage
                              (R^30, 64 anisotropic clusters, scaled to
                              [0, 20], rounded to 1e-3), seed 170906819
  batch_1024                  the 1024 ragged instances (n log-uniform in
                              [64, 4096], linkage uniform over 4), one digest
                              per instance, seed 170906820
  mixture_n65536_average      n=65536 mixture (R^16, 64 clusters), average
                              linkage, seed 170906822: the full list (hours
                              of CPU time)
  mixture_n65536_average_p512 the same, first 512 merges only
"""
import argparse
import concurrent.futures as cf
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "oracle_digests.json")


def upper_sha(d):
    h = hashlib.sha256()
    n = d.shape[0]
    for a in range(n - 1):
        h.update(d[a, a + 1:].tobytes())
    return h.hexdigest()


def rec_list(m):
    return [[int(r["i"]), int(r["j"]), float(r["h"]), int(r["size"])] for r in m]


def entry(d, link, merges, what, seed, t, threads):
    return {"workload": what, "seed": seed, "n": int(d.shape[0]), "linkage": link,
            "input_upper_sha256": upper_sha(d), "merges": int(len(merges)),
            "records_sha256": hashlib.sha256(merges.tobytes()).hexdigest(),
            "first": rec_list(merges[:4]), "last": rec_list(merges[-4:]),
            "oracle_seconds": round(t, 1), "oracle_threads": threads}


def load():
    if os.path.exists(OUT):
        with open(OUT) as f:
            return json.load(f)
    return {}


def save(doc):
    doc["_about"] = ("SHA-256 digests of the CPU oracle's merge lists (records: int32 i, int32 j, "
                     "float32 height, int32 size, little-endian); written by make_digests.py from "
                     "oracle/ and synth/ only")
    tmp = OUT + ".tmp"
    with open(tmp, "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
    os.replace(tmp, OUT)


def do_rmsd_like(threads):
    seed = synth.BASE_SEED + 3
    d = synth.rmsd_like(seed=seed, n=32768)
    t0 = time.time()
    m = oracle.run_f32(d, "complete", threads=threads)
    t = time.time() - t0
    return entry(d, "complete", m, "rmsd_like n=32768 (R^30, 64 anisotropic clusters, [0, 20], 1e-3)",
                 seed, t, threads)


def do_big(threads, max_merges):
    seed = synth.BASE_SEED + 6
    d = synth.mixture_65536(seed=seed)
    t0 = time.time()
    m = oracle.run_f32(d, "average", max_merges=max_merges, threads=threads)
    t = time.time() - t0
    return entry(d, "average", m, "mixture n=65536 (R^16, 64 clusters, sigma ~ U[0.5, 2])", seed, t, threads)


def do_batch(threads):
    spec = synth.batch_spec(count=1024, n_lo=64, n_hi=4096)
    names = ("single", "complete", "average", "ward")

    def one(k):
        n, s = int(spec.ns[k]), int(spec.seeds[k])
        d = synth.batch_instance(n, s)
        m = oracle.run_f32(d, int(spec.linkages[k]), threads=1)
        return k, hashlib.sha256(m.tobytes()).hexdigest(), upper_sha(d)

    t0 = time.time()
    rec = [None] * len(spec.ns)
    inp = [None] * len(spec.ns)
    order = sorted(range(len(spec.ns)), key=lambda k: -int(spec.ns[k]))
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        for k, h, hi in ex.map(one, order):
            rec[k] = h
            inp[k] = hi
    return {"workload": "1024 instances, n log-uniform in [64, 4096], linkage uniform over "
                        "single/complete/average/Ward, Gaussian mixtures in R^16",
            "seed": synth.BASE_SEED + 4, "count": len(spec.ns), "ns": [int(x) for x in spec.ns],
            "linkages": [names[int(x)] for x in spec.linkages],
            "input_upper_sha256": inp, "records_sha256": rec,
            "oracle_seconds": round(time.time() - t0, 1), "oracle_threads": threads}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", nargs="*", default=["rmsd_like_n32768_complete", "batch_1024",
                                                   "mixture_n65536_average_p512"])
    ap.add_argument("--threads", type=int, default=oracle.default_threads())
    a = ap.parse_args()
    for key in a.only:
        print("computing", key, flush=True)
        t0 = time.time()
        if key == "rmsd_like_n32768_complete":
            e = do_rmsd_like(a.threads)
        elif key == "batch_1024":
            e = do_batch(a.threads)
        elif key == "mixture_n65536_average":
            e = do_big(a.threads, -1)
        elif key == "mixture_n65536_average_p512":
            e = do_big(a.threads, 512)
        else:
            raise SystemExit("unknown key " + key)
        doc = load()
        doc[key] = e
        save(doc)
        print("done", key, "%.0f s" % (time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
