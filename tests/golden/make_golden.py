"""Writes the stored expected values under tests/golden/ by calling only the oracle.

    python tests/golden/make_golden.py [field96|field48|all]

field96_trace.json: per batch of the 96x96x96x3, N=32, 20-batch drifting-field
stream at eps = 1e-4 - the oracle's skip flags, HT rank vectors, relative
projection errors, the smallest relative distance of any rank decision from its
threshold (on either side: the kept tail and the tail one rank lower) and whether
any decision sat within 1e-6 eps_nw^2 of its threshold.  GPU tests compare the
HIP library's full-size run with it.

field48_trace.json: the same for all 100 batches of the 48^4 x 4, N=16 stream
(d = 5, a three-level tree), the large-stream workload, plus the oracle's
reconstruction of the first batches at fixed sampled element positions (the
reconstruction of a past batch never changes, so the values hold at any later
point of the stream).
"""

import json
import math
import os
import queue
import sys
import threading

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


def prefetch(spec):
    """Generates the batches in a background thread, one ahead of the oracle."""
    q = queue.Queue(maxsize=1)

    def work():
        for k in range(spec.n_batches):
            q.put(datagen.exact_field_batch(spec, k))
        q.put(None)

    threading.Thread(target=work, daemon=True).start()
    while True:
        y = q.get()
        if y is None:
            return
        yield y


def trace(spec, eps, label, sampled=()):
    st = None
    rows = []
    samples = {}
    for k, y in enumerate(prefetch(spec)):
        if k == 0:
            st = ho.BHT(y.shape[1:], eps)
            info = st.init_batch(y)
        else:
            info = st.update(y)
        rows.append({"batch": k, "skipped": bool(info.skipped), "ranks": info.ranks,
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
    out = {"stream": label, "eps": eps, "source": "oracle/ht_oracle.py via tests/golden/make_golden.py",
           "batches": rows}
    if sampled:
        out["sampled_reconstruction"] = samples
    return out


def field96_trace(eps=1e-4):
    return trace(datagen.field_96_spec(), eps,
                 "field_96 (96x96x96x3, N=32, 20 batches, drift 3e-4, widths [0.2,0.5], exact generator)")


def field48_trace(eps=1e-4):
    return trace(datagen.field_48_spec(), eps,
                 "field_48 (48x48x48x48x4, N=16, 100 batches, 16 terms switching on from 6 every 9 batches, "
                 "oscillating drift 1e-3 period 25, widths [0.2,0.5], noise 1e-6, exact generator)",
                 sampled=SAMPLED_BATCHES)


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "all"
    if which in ("field96", "all"):
        data = field96_trace()
        with open(os.path.join(HERE, "field96_trace.json"), "w") as f:
            json.dump(data, f, indent=1)
    if which in ("field48", "all"):
        data = field48_trace()
        with open(os.path.join(HERE, "field48_trace.json"), "w") as f:
            json.dump(data, f, indent=1)
