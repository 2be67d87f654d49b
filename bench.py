#!/usr/bin/env python3
"""HT-RISE ingest throughput on one MI355X.

Workload: the 96x96x96x3 drifting separable-field stream, N = 32 samples per
batch, 20 batches, eps = 1e-4, rank capacity 48 (84,934,656 elements per
batch).  One step compresses the whole stream from scratch: BHT-l2r on batch 0
and HT-RISE on batches 1..19, every batch already resident in HBM as float32.
`value` is elements ingested per second over the timed steps.

Also reported: the roofline position of the dominant kernel class, measured
live with the library's HIP-event instrumentation over the timed steps, and the
FP64 NumPy oracle timed on this host on a bounded sample of the same stream.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "HT-RISE ingest elements/s at rel. err ≤1e-4, mixed-prec batched vs FP64 plain"
EPS = 1e-4
RANK_CAP = 48
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_digest() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2412_16544_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(kind: str):
    """HBM bytes per launch of `kind` from a committed counter summary, if it still matches the source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except ValueError:
        return None
    if data.get("source_digest") != source_digest():
        return None
    ent = data.get("kernels", {}).get(kind)
    return None if ent is None else ent.get("hbm_bytes_per_launch")


def cpu_baseline(spec, n_sample: int):
    """The oracle as it stands, on the first n_sample batches of the same stream (host cores)."""
    import numpy as np
    import datagen
    from oracle import ht_oracle as ho
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [os.cpu_count() or 1])
    except Exception:  # pragma: no cover
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    ys = list(datagen.separable_field_stream(spec, batches=range(n_sample)))
    st = ho.BHT(ys[0].shape[1:], EPS)
    t0 = time.perf_counter()
    st.init_batch(ys[0])
    for y in ys[1:]:
        st.update(y)
    dt = time.perf_counter() - t0
    elems = n_sample * spec.elements_per_batch
    return {"value": elems / dt, "unit": "elements/s", "cores": int(threads), "kind": "oracle",
            "sample": "first %d of %d batches (BHT-l2r + %d HT-RISE updates), FP64 NumPy, %.1f s"
                      % (n_sample, spec.n_batches, n_sample - 1, dt),
            "ranks_after_sample": st.ranks}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=4, help="batches of the oracle baseline (0 = skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs a stream on a single device and this build "
              "has no multi-GPU path (requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import datagen
    from paper_2412_16544_amd import htrise as H

    spec = datagen.field_96_spec()
    E = spec.elements_per_batch
    nb = spec.n_batches
    t0 = time.perf_counter()
    ys = [torch.from_numpy(y).to("cuda:0") for y in datagen.separable_field_stream(spec)]
    torch.cuda.synchronize()
    log("staged %d batches of %d elements in HBM (%.1f s)" % (nb, E, time.perf_counter() - t0))

    st = H.HTStream(spec.n, EPS, RANK_CAP, spec.N, spec.N * nb, "float32")

    def one_pass():
        st.reset()
        return [st.push(y) for y in ys]

    for w in range(args.warmup):
        one_pass()
        log("warmup %d done" % w)
    torch.cuda.synchronize()
    H.ht_profile_enable(True)
    t0 = time.perf_counter()
    for k in range(args.steps):
        infos = one_pass()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = H.ht_profile_read_all()
    H.ht_profile_enable(False)
    log("timed %d steps in %.3f s" % (args.steps, elapsed))

    # correctness of the last timed pass, outside the timed region
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "field96_trace.json")))
    ranks, nacc = st.ranks()
    parity = ranks == golden["batches"][-1]["ranks"] and nacc == spec.N * nb
    parity = parity and all(i.skipped == g["skipped"] for i, g in zip(infos[1:], golden["batches"][1:]))
    worst = 0.0
    for k in (0, nb // 2, nb - 1):
        rec = st.reconstruct(spec.N * k, spec.N)
        yk = ys[k].double()
        worst = max(worst, (torch.linalg.vector_norm(rec - yk) / torch.linalg.vector_norm(yk)).item())
    parity = parity and worst <= EPS
    log("parity vs oracle trace: %s, worst sampled relative error %.3e" % (parity, worst))

    # roofline of the dominant kernel class
    kinds = {k: v for k, v in prof.items() if v["launches"] > 0}
    dom = max(("gram", "ttm_contract", "ttm_expand", "sumsq"), key=lambda k: kinds.get(k, {"ms": 0})["ms"])
    d = kinds[dom]
    if dom == "gram":
        achieved = d["flops"] / (d["ms"] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_TFLOPS}
    else:
        achieved = d["bytes"] / (d["ms"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS}
    roof["kernel"] = dom
    roof["launches"] = d["launches"]
    roof["avg_launch_ms"] = d["ms"] / d["launches"]
    roof["traffic"] = traffic_for(dom)

    upd = [i for i in infos[1:]]
    upd_ms = sum(i.device_ms for i in upd)
    line = {
        "metric": METRIC,
        "value": nb * E * args.steps / elapsed,
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "96x96x96x3 drifting separable field, N=32 per batch, 20 batches, eps=1e-4, "
                               "rank_cap 48; step = BHT-l2r on batch 0 + HT-RISE on batches 1-19",
                   "form": "fp64 plain", "elements_per_batch": E, "batches": nb},
        "roofline": roof,
        "rise_update_elements_per_s": (nb - 1) * E / (upd_ms * 1e-3) if upd_ms > 0 else None,
        "init_batch_ms": infos[0].device_ms,
        "update_batch_ms": sum(i.device_ms for i in upd if not i.skipped) / max(1, sum(not i.skipped for i in upd)),
        "skip_batch_ms": sum(i.device_ms for i in upd if i.skipped) / max(1, sum(i.skipped for i in upd)),
        "kernel_ms_per_step": {k: v["ms"] / args.steps for k, v in kinds.items()},
        "parity_vs_oracle_trace": bool(parity),
    }
    if args.cpu_sample > 0:
        log("timing the oracle on %d batches of the same stream..." % args.cpu_sample)
        line["cpu_baseline"] = cpu_baseline(spec, args.cpu_sample)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
