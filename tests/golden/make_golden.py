"""Writes the stored expected values under tests/golden/ by calling only the oracle.

    python tests/golden/make_golden.py [field96|field48|all]

field96_trace.json: per batch of the 96x96x96x3, N=32, 20-batch drifting-field
stream at eps = 1e-4 - the oracle's skip flags, HT rank vectors, relative
projection errors and whether any rank decision sat within 1e-6 eps_nw^2 of
its threshold.  GPU tests compare the HIP library's full-size run with it.

field48_trace.json: the same for the first 4 batches of the 48^4 x 4, N=16
drifting-field stream (d = 5, a three-level tree), the large-stream workload.
"""

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import datagen  # noqa: E402
from oracle import ht_oracle as ho  # noqa: E402


def field96_trace(eps=1e-4):
    spec = datagen.field_96_spec()
    st = None
    rows = []
    for k, y in enumerate(datagen.separable_field_stream(spec)):
        if k == 0:
            st = ho.BHT(y.shape[1:], eps)
            info = st.init_batch(y)
        else:
            info = st.update(y)
        margin = min((abs(t.tail2 - t.eps_nw ** 2) / t.eps_nw ** 2 for t in info.decisions.values()), default=None)
        rows.append({"batch": k, "skipped": bool(info.skipped), "ranks": info.ranks,
                     "eps_proj_rel": info.eps_proj / info.norm_y,
                     "near_tie_1e-6": bool(info.any_near_tie(1e-6)),
                     "min_decision_margin_rel": margin})
        print(rows[-1], flush=True)
    return {"stream": "field_96 (96x96x96x3, N=32, 20 batches, drift 3e-4, widths [0.2,0.5])",
            "eps": eps, "source": "oracle/ht_oracle.py via tests/golden/make_golden.py", "batches": rows}


def trace(spec, eps, label):
    st = None
    rows = []
    for k, y in enumerate(datagen.separable_field_stream(spec)):
        if k == 0:
            st = ho.BHT(y.shape[1:], eps)
            info = st.init_batch(y)
        else:
            info = st.update(y)
        margin = min((abs(t.tail2 - t.eps_nw ** 2) / t.eps_nw ** 2 for t in info.decisions.values()), default=None)
        rows.append({"batch": k, "skipped": bool(info.skipped), "ranks": info.ranks,
                     "eps_proj_rel": info.eps_proj / info.norm_y,
                     "near_tie_1e-6": bool(info.any_near_tie(1e-6)),
                     "min_decision_margin_rel": margin})
        print(rows[-1], flush=True)
    return {"stream": label, "eps": eps, "source": "oracle/ht_oracle.py via tests/golden/make_golden.py",
            "batches": rows}


def field48_trace(eps=1e-4, n_batches=4):
    spec = datagen.field_48_spec(n_batches=n_batches)
    return trace(spec, eps, "field_48 (48x48x48x48x4, N=16, first %d batches, drift 1e-4, widths [0.2,0.5], "
                            "noise 1e-6)" % n_batches)


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "all"
    if which in ("field96", "all"):
        with open(os.path.join(HERE, "field96_trace.json"), "w") as f:
            json.dump(field96_trace(), f, indent=1)
    if which in ("field48", "all"):
        with open(os.path.join(HERE, "field48_trace.json"), "w") as f:
            json.dump(field48_trace(), f, indent=1)
