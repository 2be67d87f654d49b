"""Writes the stored expected values under tests/golden/ by calling only the oracle.

    python tests/golden/make_golden.py [field96|field48|all]

field96_trace.json: per batch of the 96x96x96x3, N=32, 20-batch drifting-field
stream at eps = 1e-4 - an exact checksum of the batch's float32 values (the sum of
their bit patterns, so a GPU run can prove it saw the same data), the oracle's skip
flags, HT rank vectors, relative
projection errors, the smallest relative distance of any rank decision from its
threshold (on either side: the kept tail and the tail one rank lower) and whether
any decision sat within 1e-6 eps_nw^2 of its threshold.  GPU tests compare the
HIP library's full-size run with it.

Both also hold the oracle's per-sample relative test errors (Sec. 4.1) of the two
batches that follow the stream, encoded and decoded with the final cores
("rte_heldout"; for field48 written from the trace's final checkpoint).

variants_trace.json: the adaptive-budget (App. C) and ST-HOSVD variants on the
96^3 x 3 stream, and the plain leaves-to-root HT (Sec. 2.3.1) of the first batch of
both field streams as one tensor with the batch as a mode.

field48_trace.json: the same for all 100 batches of the 48^4 x 4, N=16 stream
(d = 5, a three-level tree), the large-stream workload, plus the oracle's
reconstruction of the first batches at fixed sampled element positions (the
reconstruction of a past batch never changes, so the values hold at any later
point of the stream).
"""

import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import datagen  # noqa: E402
from oracle import ht_oracle as ho  # noqa: E402

SAMPLE_POSITIONS = 4096
SAMPLED_BATCHES = (0, 1, 2)


def decision_margin(info):
    """Smallest |tail - thr| / thr over the batch's decisions, both sides of each."""
    best = None
    for t in info.decisions.values():
        thr = t.eps_nw ** 2
        cands = [abs(t.tail2 - thr) / thr]
        if math.isfinite(t.tail2_prev):
            cands.append(abs(t.tail2_prev - thr) / thr)
        m = min(cands)
        best = m if best is None else min(best, m)
    return best


def sample_positions(shape, seed=7):
    g = datagen.rng(seed)
    per = int(np.prod(shape[1:]))
    return np.sort(g.choice(per * shape[0], size=SAMPLE_POSITIONS, replace=False))


def _gen(args):
    spec, k = args
    return datagen.exact_field_batch(spec, k)


def prefetch(spec, first=0):
    """Generates the batches from `first` on in a separate process, one ahead of the
    oracle (a process, not a thread: the oracle's BLAS calls must not run concurrently
    with the generator's in one process)."""
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(1) as pool:
        for y in pool.imap(_gen, [(spec, k) for k in range(first, spec.n_batches)]):
            yield y


def save_state(path, st, rows, samples):
    """Checkpoint of a long trace: the oracle's cores and root and the rows so far."""
    arrays = {"root": st.root}
    for idx, u in st.core.items():
        arrays["core_%d" % idx] = u
    tmp = path + ".tmp.npz"
    np.savez(tmp, meta=np.frombuffer(json.dumps({"rows": rows, "samples": samples}).encode(), dtype=np.uint8),
             **arrays)
    os.replace(tmp, path)


def load_state(path, st):
    with np.load(path) as z:
        meta = json.loads(bytes(z["meta"]).decode())
        st.root = z["root"]
        st.core = {int(k[5:]): z[k] for k in z.files if k.startswith("core_")}
    return meta["rows"], meta["samples"]


def trace(spec, eps, label, sampled=(), checkpoint=None, state=None):
    st = state if state is not None else ho.BHT(spec.n, eps)
    rows = []
    samples = {}
    if checkpoint and os.path.exists(checkpoint):
        rows, samples = load_state(checkpoint, st)
        print("resuming after batch %d" % (len(rows) - 1), flush=True)
    first = len(rows)
    for k, y in enumerate(prefetch(spec, first), first):
        if k == 0:
            info = st.init_batch(y)
        else:
            info = st.update(y)
        rows.append({"batch": k, "data_checksum": datagen.checksum(y), "skipped": bool(info.skipped),
                     "ranks": info.ranks,
                     "eps_proj_rel": info.eps_proj / info.norm_y,
                     "near_tie_1e-6": bool(info.any_near_tie(1e-6)),
                     "min_decision_margin_rel": decision_margin(info)})
        if k in sampled:
            pos = sample_positions(y.shape)
            rec = st.reconstruct(k * spec.N, spec.N).reshape(-1)
            err = float(np.linalg.norm(rec - y.reshape(-1).astype(np.float64)))
            samples[str(k)] = {"positions": pos.tolist(), "values": rec[pos].tolist(),
                               "error_rel": err / info.norm_y}
            del rec
        print(rows[-1], flush=True)
        if checkpoint and (k % 5 == 4 or k == spec.n_batches - 1):
            save_state(checkpoint, st, rows, samples)
    out = {"stream": label, "eps": eps, "source": "oracle/ht_oracle.py via tests/golden/make_golden.py",
           "batches": rows}
    if sampled:
        out["sampled_reconstruction"] = samples
    return out


HELDOUT = 2  # held-out batches after the stream (the next batches of the same generator)


def heldout_rte(st, spec):
    """The oracle's per-sample relative test errors on the HELDOUT batches that follow
    the stream (Sec. 4.1, Eq. generalization_performance)."""
    import dataclasses
    ext = dataclasses.replace(spec, n_batches=spec.n_batches + HELDOUT)
    out = {"batches": [], "data_checksum": [], "rel_err": []}
    for k in range(spec.n_batches, spec.n_batches + HELDOUT):
        y = datagen.exact_field_batch(ext, k)
        out["batches"].append(k)
        out["data_checksum"].append(datagen.checksum(y))
        out["rel_err"].append([float(e) for e in st.relative_test_errors(y)])
    return out


def field96_trace(eps=1e-4):
    spec = datagen.field_96_spec()
    st = ho.BHT(spec.n, eps)
    data = trace(spec, eps, "field_96 (96x96x96x3, N=32, 20 batches, drift 3e-4, widths [0.2,0.5], exact generator)",
                 state=st)
    data["rte_heldout"] = heldout_rte(st, spec)
    return data


def field48_rte(checkpoint, eps=1e-4):
    """Adds the held-out relative test errors to field48_trace.json from the final
    checkpoint of the field48 trace."""
    spec = datagen.field_48_spec()
    st = ho.BHT(spec.n, eps)
    rows, _ = load_state(checkpoint, st)
    assert len(rows) == spec.n_batches, "the checkpoint is not the end of the stream"
    path = os.path.join(HERE, "field48_trace.json")
    data = json.load(open(path))
    data["rte_heldout"] = heldout_rte(st, spec)
    with open(path, "w") as f:
        json.dump(data, f, indent=1)


def field48_trace(eps=1e-4, checkpoint=None):
    return trace(datagen.field_48_spec(), eps,
                 "field_48 (48x48x48x48x4, N=16, 100 batches, 16 terms switching on from 6 every 9 batches, "
                 "oscillating drift 1e-3 period 25, widths [0.2,0.5], noise 1e-6, exact generator)",
                 sampled=SAMPLED_BATCHES, checkpoint=checkpoint)


def variants():
    """The method's variants on the 96^3 x 3 stream (adaptive budget, ST-HOSVD: per batch
    ranks, skips and projection errors) and the plain leaves-to-root HT of the first
    batch of both field streams, taken as one tensor with the batch as its first mode
    (ranks and core element counts)."""
    out = {"source": "oracle/ht_oracle.py via tests/golden/make_golden.py"}
    spec = datagen.field_96_spec()
    ys = [datagen.exact_field_batch(spec, k) for k in range(spec.n_batches)]
    for name, kw in (("field96_adaptive", dict(adaptive=True)), ("field96_st_hosvd", dict(st_hosvd=True))):
        st = ho.BHT(spec.n, 1e-4, **kw)
        rows = []
        for k, y in enumerate(ys):
            info = st.init_batch(y) if k == 0 else st.update(y)
            rows.append({"batch": k, "skipped": bool(info.skipped), "ranks": info.ranks,
                         "eps_proj_rel": info.eps_proj / info.norm_y,
                         "min_decision_margin_rel": decision_margin(info)})
            print(name, rows[-1], flush=True)
        out[name] = rows
    del ys
    for name, sp in (("field96_batch0_plain_ht", spec), ("field48_batch0_plain_ht", datagen.field_48_spec())):
        y = datagen.exact_field_batch(sp, 0)
        ht = ho.PlainHT(y, 1e-4)
        out[name] = {"shape": list(y.shape), "ranks": ht.ranks, "core_elements": ht.num_elements(),
                     "error_rel": math.sqrt(ho.fro2(ht.reconstruct() - y) / ho.fro2(y))}
        print(name, out[name], flush=True)
        del y, ht
    with open(os.path.join(HERE, "variants_trace.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    # optional second argument: a checkpoint file for the long field48 trace (written
    # every five batches; a rerun with the same file resumes from it)
    which = sys.argv[1] if len(sys.argv) > 1 else "all"
    ckpt = sys.argv[2] if len(sys.argv) > 2 else None
    if which in ("field96", "all"):
        data = field96_trace()
        with open(os.path.join(HERE, "field96_trace.json"), "w") as f:
            json.dump(data, f, indent=1)
    if which in ("field48", "all"):
        data = field48_trace(checkpoint=ckpt)
        with open(os.path.join(HERE, "field48_trace.json"), "w") as f:
            json.dump(data, f, indent=1)
    if which in ("field48rte", "all") and ckpt:
        field48_rte(ckpt)
    if which in ("variants", "all"):
        variants()
