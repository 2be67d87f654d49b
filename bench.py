#!/usr/bin/env python3
"""HT-RISE ingest throughput on one MI355X: mixed precision form vs plain FP64.

Headline workload: the 48x48x48x48x4 drifting separable-field stream (d = 5), N = 16
samples per batch, 100 batches, eps = 1e-4, rank capacity 64 (339,738,624 elements
per batch, 136 GB of float32 staged in HBM before timing by datagen's device
generator).  One step compresses the whole stream from scratch: BHT-l2r on batch 0
and HT-RISE on batches 1..99.  Both forms run on the same staged data:

  fp64   every contraction and Gram product on FP64 matrix cores;
  mixed  HT-RISE contractions and residual Grams on FP32 matrix cores with FP64
         sums and certified decisions (an uncertified one is taken again in FP64);
         BHT-l2r, eigen solves, decisions and expansion in FP64.

`value` is the mixed form's elements ingested per second over the timed steps; the
plain form's rate and the ratio are reported beside it, together with the
HT-RISE-only rates (update calls only, as the paper times updates) and per-call
device times of the uninstrumented steps.  After timing, an untimed pass is checked
batch by batch against the oracle's stored rank / skip trace, and sampled batches
against the per-batch error bound.  Also reported: the roofline position of the mixed
form's dominant kernel class (HIP-event timing inside the library on the launch
stream, on one more pass after the timed ones), the 96x96x96x3 stream (N = 32, 20 batches) the same way,
the many-streams form, and the FP64 NumPy oracle timed on this host on a bounded
sample of the headline stream.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--form both|mixed|fp64]
                    [--workload field48|field96] [--only] [--no-many] [--cpu-sample B]
    python bench.py --copy-probe      # a plain 2 GiB device copy (counter calibration)
    python bench.py --bw-probe        # achievable HBM rates: a read-only sum and a copy
    python bench.py --ingest-counters FETCH_DB WRITE_DB COPY_FETCH_DB COPY_WRITE_DB
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "HT-RISE ingest elements/s at rel. err ≤1e-4, mixed-prec batched vs FP64 plain"
EPS = 1e-4
BOUND_SLACK = 1e-3
# MI355X datasheet peaks (dense)
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}
PEAK_HBM_GBS = 8000.0
# profile kind -> arithmetic type of its products
KIND_TYPE = {"gram": "f64", "ttm_contract": "f64", "ttm_expand": "f64", "sumsq": "f64", "gram_f32": "f32",
             "ttm_contract_f32": "f32", "gram_f32_reg": "f32", "ttm_contract_f32_reg": "f32", "gram_reg64": "f64",
             "ttm_contract_reg64": "f64"}


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


def roofline(kind: str, d: dict) -> dict:
    """Achieved rate of a kernel class against the roofline that bounds it."""
    ty = KIND_TYPE.get(kind, "f64")
    peak_f = PEAK_TFLOPS[ty]
    ai = d["flops"] / d["bytes"] if d["bytes"] > 0 else float("inf")
    sec = d["ms"] * 1e-3
    if ai > peak_f * 1e12 / (PEAK_HBM_GBS * 1e9):
        ach = d["flops"] / sec / 1e12
        r = {"bound": "mfma", "achieved": ach, "peak": peak_f, "unit": "TFLOP/s", "frac": ach / peak_f}
    else:
        ach = d["bytes"] / sec / 1e9
        r = {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": ach / PEAK_HBM_GBS}
    r.update({"kernel": kind, "dtype": ty, "launches": d["launches"], "avg_launch_ms": d["ms"] / d["launches"],
              "flops_per_launch": d["flops"] / d["launches"], "bytes_per_launch": d["bytes"] / d["launches"],
              "traffic": traffic_for(kind)})
    return r


def cpu_info() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        return int(max([p.get("num_threads", 1) for p in threadpool_info()] or [os.cpu_count() or 1]))
    except Exception:  # pragma: no cover
        return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def cpu_baseline(spec, n_batches: int, n_samples: int):
    """The oracle as it stands on a bounded sample of the same stream: the first n_batches
    batches (BHT-l2r + updates), each cut to its first n_samples samples (the generator
    draws them first, so they are the full batches' first samples), on the host cores;
    then the same on one thread."""
    import dataclasses
    import datagen
    from oracle import ht_oracle as ho
    sub = dataclasses.replace(spec, N=n_samples, n_batches=n_batches)
    ys = [datagen.exact_field_batch(sub, k) for k in range(n_batches)]

    def timed():
        st = ho.BHT(ys[0].shape[1:], EPS)
        t0 = time.perf_counter()
        st.init_batch(ys[0])
        for y in ys[1:]:
            st.update(y)
        return time.perf_counter() - t0, st

    dt, st = timed()
    elems = n_batches * sub.elements_per_batch
    out = {"value": elems / dt, "unit": "elements/s", "cores": _oracle_threads(), "kind": "oracle",
           "sample": "first %d batches (BHT-l2r + %d HT-RISE updates) of the stream, first %d of %d samples each, "
                     "FP64 NumPy, %.1f s" % (n_batches, n_batches - 1, n_samples, spec.N, dt),
           "cpu_model": cpu_info(), "ranks_after_sample": st.ranks}
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(1):
            dt1, _ = timed()
        out["value_1_thread"] = elems / dt1
    except Exception as e:  # pragma: no cover
        out["value_1_thread"] = None
        out["one_thread_error"] = str(e)
    return out


def copy_probe():
    """A plain device copy of 2 GiB (well above the 256 MB last-level cache): the reference
    for the HBM byte counters."""
    import torch
    n = 1 << 28  # doubles
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8, "launches": 3}), flush=True)


def bw_probe():
    """Achievable HBM rates on this device with library-free kernels: a read-only
    reduction (torch.sum) and a copy (half reads, half writes), each over 1.36 GB of
    FP32 (the size of one 48^4 x 4 x 16 batch), the median of 10 launches."""
    import torch
    n = 16 * 48 ** 4 * 4
    x = torch.ones(n, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    res = {}
    for name, fn, nbytes in (("read_sum", lambda: x.sum(), 4 * n), ("copy", lambda: y.copy_(x), 8 * n)):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(10):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        ms = sorted(ts)[len(ts) // 2]
        res[name] = {"bytes": nbytes, "ms": round(ms, 4), "GB_per_s": round(nbytes / ms / 1e6, 1)}
    print(json.dumps({"bw_probe": res}), flush=True)


def run_form(form, spec, ys, golden, steps, warmup, rank_cap):
    """Times `steps` passes over the staged stream (BHT-l2r on batch 0, HT-RISE on the
    rest) in one precision form, then checks an untimed pass batch by batch against
    the oracle's stored trace and the per-batch error bound."""
    import torch
    from paper_2412_16544_amd import htrise as H
    nb = len(ys)
    prec = H.HT_FP32 if form == "mixed" else H.HT_FP64
    st = H.HTStream(spec.n, EPS, rank_cap, spec.N, spec.N * nb, "float32", prec=prec)

    def one_pass():
        st.reset()
        return [st.push(y) for y in ys]

    for w in range(warmup):
        one_pass()
        log("%s: warmup %d done" % (form, w))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    passes = []
    for s in range(steps):
        passes.append(one_pass())
        log("%s: timed step %d done" % (form, s))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log("%s: timed %d steps in %.3f s" % (form, steps, elapsed))
    # per-kernel HIP events (two records around every launch) on one more pass, after
    # the timing, so the timed passes run uninstrumented
    H.ht_profile_enable(True)
    one_pass()
    torch.cuda.synchronize()
    prof = H.ht_profile_read_all()
    H.ht_profile_enable(False)

    # ---- untimed checks: ranks and skips after every batch against the oracle's trace,
    #      the skips of every timed pass, and the error bound on sampled batches
    from datagen import gpu as G
    st.reset()
    rows = golden["batches"]
    mismatch = [] if len(rows) == nb else ["trace has %d batches" % len(rows)]
    mismatch += ["data %d" % k for k in range(min(nb, len(rows)))
                 if G.checksum(ys[k]) != rows[k].get("data_checksum")]
    for k, y in enumerate(ys):
        info = st.push(y)
        if k >= len(rows):
            continue
        if st.ranks()[0] != rows[k]["ranks"] or (k > 0 and bool(info.skipped) != rows[k]["skipped"]):
            mismatch.append(k)
    for p in passes:
        for k, info in enumerate(p[1:len(rows)], 1):
            if bool(info.skipped) != rows[k]["skipped"]:
                mismatch.append(k)
    worst = 0.0
    for k in sorted({0, 1, nb // 2, nb - 1}):
        rec = st.reconstruct(spec.N * k, spec.N)
        yk = ys[k].double()
        worst = max(worst, (torch.linalg.vector_norm(rec - yk) / torch.linalg.vector_norm(yk)).item())
        del rec, yk
    # held-out batches after the stream: relative test error (Sec. 4.1), against the
    # oracle's stored values when the trace has them
    rte = None
    ref = golden.get("rte_heldout")
    if ref is not None:
        import dataclasses
        ext = dataclasses.replace(spec, n_batches=spec.n_batches + len(ref["batches"]))
        yk = torch.empty_like(ys[0])
        vals, diff = [], 0.0
        for k, cs, errs in zip(ref["batches"], ref["data_checksum"], ref["rel_err"]):
            G.field_batch_into(ext, k, yk)
            if G.checksum(yk) != cs:
                mismatch.append("held-out data %d" % k)
            e = st.rte(yk)
            vals += e
            diff = max(diff, max(abs(a - b) for a, b in zip(e, errs)))
        rte = {"batches": ref["batches"], "mean": sum(vals) / len(vals), "max": max(vals),
               "oracle_mean": sum(sum(x) for x in ref["rel_err"]) / sum(len(x) for x in ref["rel_err"]),
               "max_abs_diff_vs_oracle": diff}
        del yk
    ok = not mismatch and worst <= EPS * (1 + BOUND_SLACK)
    log("%s: ranks/skips at every batch vs oracle trace and error bound: %s (mismatches %s, worst sampled "
        "relative error %.3e)" % (form, ok, sorted(set(map(str, mismatch)))[:10], worst))
    E = spec.elements_per_batch
    # per-call device times from the (uninstrumented) timed passes
    plain = passes
    upd = [i for p in plain for i in p[1:] if not i.skipped]
    skp = [i for p in plain for i in p[1:] if i.skipped]
    upd_ms = sum(i.device_ms for p in plain for i in p[1:]) / len(plain)
    kinds = {k: v for k, v in prof.items() if v["launches"] > 0}
    cand = [k for k in KIND_TYPE if k in kinds]
    dom = max(cand, key=lambda k: kinds[k]["ms"])
    last = plain[-1]
    st.close()
    del st
    torch.cuda.empty_cache()
    return {
        "value": nb * E * steps / elapsed,
        "ms_per_step": elapsed * 1e3 / steps,
        "rise_update_elements_per_s": (nb - 1) * E / (upd_ms * 1e-3) if upd_ms > 0 else None,
        "init_batch_ms": sum(p[0].device_ms for p in plain) / len(plain),
        "update_batch_ms": sum(i.device_ms for i in upd) / max(1, len(upd)),
        "skip_batch_ms": sum(i.device_ms for i in skp) / max(1, len(skp)),
        "updates_per_pass": sum(not i.skipped for i in last[1:]),
        "skips_per_pass": sum(bool(i.skipped) for i in last[1:]),
        "fp64_recomputed_decisions_per_pass": sum(i.recomputed for i in last[1:]),
        "updates_run_in_fp64_per_pass": sum(i.prec_used == H.HT_FP64 for i in last[1:] if not i.skipped)
        if form == "mixed" else None,
        "kernel_ms_profiled_pass": {k: round(v["ms"], 3) for k, v in kinds.items()},
        "roofline": roofline(dom, kinds[dom]),
        # every contraction / Gram class of the profiled pass against its own roofline
        "rooflines": {k: {x: v for x, v in roofline(k, kinds[k]).items() if x in ("bound", "achieved", "unit", "frac",
                                                                                  "launches", "avg_launch_ms")}
                      for k in cand},
        "parity_vs_oracle_trace": bool(ok),
        "worst_sampled_rel_error": worst,
        "rte_heldout": rte,
    }


def stage(spec):
    """Every batch of the stream generated straight into HBM (datagen's device generator,
    bit for bit its host generator, which the oracle's trace was computed from)."""
    import torch
    from datagen import gpu as G
    t0 = time.perf_counter()
    ys = []
    for k in range(spec.n_batches):
        y = torch.empty((spec.N,) + spec.n, dtype=torch.float32, device="cuda:0")
        G.field_batch_into(spec, k, y)
        ys.append(y)
        if k % 25 == 24:
            log("staged %d of %d batches" % (k + 1, spec.n_batches))
    torch.cuda.synchronize()
    log("staged %d batches of %d elements in HBM (%.1f s)" % (spec.n_batches, spec.elements_per_batch,
                                                              time.perf_counter() - t0))
    return ys


def run_variants(steps, warmup):
    """The method's variants beside the headline: the adaptive error budget (App. C) and
    ST-HOSVD within a layer on the 96^3 x 3 stream (both forms, timed like the
    headline, ranks and skips checked at every batch against the oracle's variant
    traces), and the plain leaves-to-root HT (Sec. 2.3.1) against BHT-l2r on the first
    batch of both field streams (the format comparison of App. D.1): device time of the
    one-shot decomposition, ranks against the oracle's, compression ratios."""
    import torch
    import datagen
    from paper_2412_16544_amd import htrise as H
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "variants_trace.json")))
    spec = datagen.field_96_spec()
    ys = stage(spec)
    E = spec.elements_per_batch
    out = {"workload": WORKLOADS["field96"][0]}
    for name, flags in (("adaptive_budget", H.HT_ADAPTIVE_BUDGET), ("st_hosvd", H.HT_ST_HOSVD)):
        rows = gold["field96_" + ("adaptive" if name == "adaptive_budget" else name)]
        out[name] = {}
        for form, prec in (("mixed", H.HT_FP32), ("fp64", H.HT_FP64)):
            st = H.HTStream(spec.n, EPS, 48, spec.N, spec.N * len(ys), prec=prec, flags=flags)
            for _ in range(warmup):
                st.reset()
                for y in ys:
                    st.push(y)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                st.reset()
                for y in ys:
                    st.push(y)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            st.reset()
            ok = True
            for k, y in enumerate(ys):
                info = st.push(y)
                ok = ok and st.ranks()[0] == rows[k]["ranks"] and (k == 0 or bool(info.skipped) == rows[k]["skipped"])
            cr = len(ys) * E / len(st.export())
            out[name][form] = {"value": len(ys) * E / dt, "ms_per_step": dt * 1e3, "final_ranks": st.ranks()[0],
                               "compression_ratio": cr, "parity_vs_oracle_trace": bool(ok)}
            log("variant %s %s: %.3e elements/s, ranks %s, parity %s" % (name, form, len(ys) * E / dt,
                                                                         st.ranks()[0], ok))
            st.close()
            del st
    del ys
    torch.cuda.empty_cache()
    # plain HT (batch as a mode, one tensor) against BHT-l2r on the first batch
    out["bht_vs_plain_ht"] = {}
    for wname, sp, rc in (("field96", spec, 48), ("field48", datagen.field_48_spec(), 64)):
        from datagen import gpu as G
        y = G.field_batch(sp, 0)
        ref = gold[wname + "_batch0_plain_ht"]
        res = {}
        for fmt in ("bht_l2r", "plain_ht"):
            times = []
            for _ in range(3):
                if fmt == "bht_l2r":
                    st = H.HTStream(sp.n, EPS, rc, sp.N, sp.N)
                    info = st.push(y)
                else:
                    st = H.HTStream((sp.N,) + sp.n, EPS, 64, 1, 1, flags=H.HT_PLAIN_HT_BUDGET)
                    info = st.push(y.view((1, sp.N) + sp.n))
                times.append(info.device_ms)
                ranks = st.ranks()[0]
                size = len(st.export())
                st.close()
                del st
            res[fmt] = {"device_ms": sorted(times)[1], "ranks": ranks, "compression_ratio": sp.elements_per_batch / size}
        res["plain_ht_ranks_match_oracle"] = res["plain_ht"]["ranks"] == ref["ranks"]
        res["plain_ht_over_bht_time"] = res["plain_ht"]["device_ms"] / res["bht_l2r"]["device_ms"]
        out["bht_vs_plain_ht"][wname] = res
        log("%s batch 0: BHT-l2r %.2f ms (CR %.1f), plain HT %.2f ms (CR %.1f), HT ranks match oracle %s"
            % (wname, res["bht_l2r"]["device_ms"], res["bht_l2r"]["compression_ratio"], res["plain_ht"]["device_ms"],
               res["plain_ht"]["compression_ratio"], res["plain_ht_ranks_match_oracle"]))
        del y
        torch.cuda.empty_cache()
    return out


def run_workload(name, spec, rank_cap, forms, steps, warmup):
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", name + "_trace.json")))
    ys = stage(spec)
    res = {f: run_form(f, spec, ys, golden, steps, warmup, rank_cap) for f in forms}
    del ys
    import torch
    torch.cuda.empty_cache()
    return res


def run_many(count=64, cap=1 << 20, d_choices=(3, 4), rank_hi=12, on_device=False):
    """The many-streams workload: updates timed one by one and in lock step, both forms.

    With on_device the streams' batches are built on the device round by round
    (datagen.gpu.model_batches), outside the timed calls; else they are generated on
    the host once and kept resident."""
    import torch
    import datagen
    from datagen import gpu as G
    from paper_2412_16544_amd import htrise as H
    specs = datagen.multi_stream_specs(count=count, max_elements=cap, d_choices=d_choices, rank_hi=rank_hi)
    nb = specs[0].n_batches
    upd_elems = sum(sp.elements_per_batch for sp in specs) * (nb - 1)
    data = None
    if not on_device:
        t0 = time.perf_counter()
        data = [[torch.from_numpy(y).to("cuda:0") for y in datagen.ht_model_stream(sp)] for sp in specs]
        torch.cuda.synchronize()
        log("many streams: %d streams staged (%.1f s), %d update elements" % (count, time.perf_counter() - t0,
                                                                             upd_elems))

    def rounds():
        """round k -> the k-th batch of every stream (device tensors)"""
        if data is not None:
            for k in range(nb):
                yield [ys[k] for ys in data]
            return
        gens = [G.model_batches(sp) for sp in specs]
        for _ in range(nb):
            yield [next(g) for g in gens]

    def one(prec, batched):
        sts = [H.HTStream(sp.n, EPS, 32, sp.N, sp.N * nb, prec=prec) for sp in specs]
        dt = 0.0
        for k, ys in enumerate(rounds()):
            if k == 0:
                for st, y in zip(sts, ys):
                    st.push(y)
                continue
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            if batched:
                code, _ = H.HTStream.update_many(sts, ys)
                assert code == H.HT_OK
            else:
                for st, y in zip(sts, ys):
                    st.update(y)
            torch.cuda.synchronize()
            dt += time.perf_counter() - t1
        ranks = [st.ranks() for st in sts]
        # untimed: every batch of every stream within its error bound (HT-RISE theorem)
        worst = 0.0
        for k, ys in enumerate(rounds()):
            for st, y, sp in zip(sts, ys, specs):
                rec = st.reconstruct(k * sp.N, sp.N)
                yk = y.double()
                worst = max(worst, (torch.linalg.vector_norm(rec - yk) / torch.linalg.vector_norm(yk)).item())
                del rec, yk
        for st in sts:
            st.close()
        torch.cuda.empty_cache()
        return upd_elems / dt, dt, ranks, worst

    one(H.HT_FP64, False)  # warm-up: first launches of every kernel shape
    res = {}
    for name, prec, batched in (("fp64_one_by_one", H.HT_FP64, False), ("fp64_batched", H.HT_FP64, True),
                                ("mixed_one_by_one", H.HT_FP32, False), ("mixed_batched", H.HT_FP32, True)):
        v, dt, ranks, worst = one(prec, batched)
        res[name] = {"elements_per_s": v, "seconds": dt, "ranks": ranks, "worst": worst}
        log("many streams (<= %d): %s: %.3e elements/s (%.3f s), worst batch error %.3e" % (cap, name, v, dt, worst))
    same = all(res[k]["ranks"] == res["fp64_one_by_one"]["ranks"] for k in res)
    worst = max(r["worst"] for r in res.values())
    out = {"workload": "%d exact-rank streams (d %s, n_i 16-128, N 4-32, rank 2-%d + 2 directions at batches 4 "
                       "and 8, <= %d elements per batch), 10 HT-RISE updates each, eps=1e-4, rank_cap 32%s"
                       % (count, "-".join(map(str, (min(d_choices), max(d_choices)))), rank_hi, cap,
                          "; batches built on the device per round, outside the timing" if on_device else ""),
           "update_elements": upd_elems, "ranks_agree_across_runs": bool(same),
           "worst_batch_rel_error": worst, "error_bound_holds": bool(worst <= EPS * (1 + BOUND_SLACK))}
    for k, v in res.items():
        out[k] = v["elements_per_s"]
    out["mixed_batched_over_fp64_one_by_one"] = res["mixed_batched"]["elements_per_s"] / res["fp64_one_by_one"][
        "elements_per_s"]
    out["mixed_batched_over_fp64_batched"] = res["mixed_batched"]["elements_per_s"] / res["fp64_batched"][
        "elements_per_s"]
    return out


# kernel-name patterns of each profile kind (the template's second argument is the
# compute type of the panel kernels)
KIND_KERNELS = {
    "ttm_contract_f32_reg": ("ttm_reg_kernel<",),
    "gram_f32_reg": ("gram_reg_kernel<",),
    "ttm_contract_reg64": ("ttm_reg64_kernel<",),
    "gram_reg64": ("gram_reg64_kernel<",),
    "ttm_contract_f32": ("ttm_panel_kernel<float, float", "ttm_panel_kernel<double, float"),
    "ttm_contract": ("ttm_panel_kernel<float, double", "ttm_panel_kernel<double, double", "ttm_direct_kernel<"),
    "gram_f32": ("gram_panel_kernel<float, float", "gram_panel_kernel<double, float"),
    "gram": ("gram_panel_kernel<float, double", "gram_panel_kernel<double, double", "gram_partial_kernel<",
             "gram_small_kernel<"),
    "ttm_expand": ("ttm_expand_kernel<",),
    "sumsq": ("sumsq_partial_kernel<",),
}


def ingest_counters(fetch_db, write_db, copy_fetch_db, copy_write_db, out_path):
    """HBM bytes per launch of each kernel kind from two rocprofv3 --pmc runs (FETCH_SIZE,
    WRITE_SIZE, KiB per dispatch), scaled by what the same counters read for a plain
    copy of known size."""
    import sqlite3

    def rows(db, counter):
        con = sqlite3.connect(db)
        q = "select kernel_name, value from counters_collection where counter_name = ?"
        return list(con.execute(q, (counter,)))

    copy_bytes = (1 << 28) * 8
    cf = [v for n, v in rows(copy_fetch_db, "FETCH_SIZE") if "copyBuffer" in n and v * 1024 > copy_bytes / 4]
    cw = [v for n, v in rows(copy_write_db, "WRITE_SIZE") if "copyBuffer" in n and v * 1024 > copy_bytes / 4]
    f_fetch = copy_bytes / (sum(cf) / len(cf) * 1024)
    f_write = copy_bytes / (sum(cw) / len(cw) * 1024)
    fr, wr = rows(fetch_db, "FETCH_SIZE"), rows(write_db, "WRITE_SIZE")
    kernels = {}
    for kind, pats in KIND_KERNELS.items():
        fv = [v for n, v in fr if any(p in n for p in pats)]
        wv = [v for n, v in wr if any(p in n for p in pats)]
        if not fv or not wv:
            continue
        fb = sum(fv) / len(fv) * 1024 * f_fetch
        wb = sum(wv) / len(wv) * 1024 * f_write
        kernels[kind] = {"dispatches": len(fv), "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
                         "hbm_bytes_per_launch": fb + wb}
    out = {"source_digest": source_digest(), "copy_probe_bytes": copy_bytes,
           "counter_scale": {"FETCH_SIZE": f_fetch, "WRITE_SIZE": f_write}, "kernels": kernels}
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


WORKLOADS = {
    "field48": ("48x48x48x48x4 drifting separable field (d=5, 16 terms switching on, oscillating drift), N=16 per "
                "batch, 100 batches, eps=1e-4, rank_cap 64; step = BHT-l2r on batch 0 + HT-RISE on batches 1-99", 64),
    "field96": ("96x96x96x3 drifting separable field, N=32 per batch, 20 batches, eps=1e-4, rank_cap 48; "
                "step = BHT-l2r on batch 0 + HT-RISE on batches 1-19", 48),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--form", choices=("both", "mixed", "fp64"), default="both")
    ap.add_argument("--workload", choices=("field48", "field96"), default="field48",
                    help="the headline stream (the other one is measured beside it unless --only)")
    ap.add_argument("--only", action="store_true", help="measure the headline stream only")
    ap.add_argument("--cpu-sample", type=int, default=2, help="batches of the oracle baseline (0 = skip)")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--bw-probe", action="store_true")
    ap.add_argument("--no-many", action="store_true", help="skip the many-streams measurement")
    ap.add_argument("--ingest-counters", nargs=4, metavar=("FETCH_DB", "WRITE_DB", "COPY_FETCH_DB", "COPY_WRITE_DB"),
                    help="write profiles/traffic.json from rocprofv3 --pmc databases (host only)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs a stream on a single device and this build "
              "has no multi-GPU path (requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.bw_probe:
        bw_probe()
        return
    if args.copy_probe:
        copy_probe()
        return
    if args.ingest_counters:
        ingest_counters(*args.ingest_counters, os.path.join(ROOT, "profiles", "traffic.json"))
        return

    import datagen

    specs = {"field48": datagen.field_48_spec(), "field96": datagen.field_96_spec()}
    forms = ["mixed", "fp64"] if args.form == "both" else [args.form]
    head_name = args.workload
    spec = specs[head_name]
    desc, rank_cap = WORKLOADS[head_name]
    res = run_workload(head_name, spec, rank_cap, forms, args.steps, args.warmup)
    head = res[forms[0]]
    line = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if forms[0] == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": desc, "form": forms[0], "elements_per_batch": spec.elements_per_batch,
                   "batches": spec.n_batches},
        "roofline": head["roofline"],
        "forms": res,
    }
    if len(forms) == 2:
        line["mixed_over_fp64"] = res["mixed"]["value"] / res["fp64"]["value"]
        r1, r2 = res["mixed"]["rise_update_elements_per_s"], res["fp64"]["rise_update_elements_per_s"]
        line["mixed_over_fp64_rise_updates"] = r1 / r2 if r1 and r2 else None
    line["parity_vs_oracle_trace"] = all(r["parity_vs_oracle_trace"] for r in res.values())
    if not args.only:
        other = "field96" if head_name == "field48" else "field48"
        ores = run_workload(other, specs[other], WORKLOADS[other][1], forms, args.steps, args.warmup)
        line["also"] = {other: {"workload": WORKLOADS[other][0], "forms": ores}}
        if len(forms) == 2:
            line["also"][other]["mixed_over_fp64"] = ores["mixed"]["value"] / ores["fp64"]["value"]
        line["parity_vs_oracle_trace"] = line["parity_vs_oracle_trace"] and all(
            r["parity_vs_oracle_trace"] for r in ores.values())
    if not args.no_many and args.form == "both":
        # small streams (launch-bound), then the configured sizes (up to 2^25 elements
        # per batch, 3-5 modes, generating ranks 2-16)
        line["many_streams"] = run_many()
        line["many_streams_configured"] = run_many(cap=1 << 25, d_choices=(3, 4, 5), rank_hi=16, on_device=True)
    if not args.only and args.form == "both":
        line["variants"] = run_variants(max(1, args.steps // 4), min(args.warmup, 1))
    if args.cpu_sample > 0:
        log("timing the oracle on a sample of the same stream...")
        line["cpu_baseline"] = cpu_baseline(spec, args.cpu_sample, 1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
