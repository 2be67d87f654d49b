"""FP64 CPU oracle for BHT-l2r / HT-RISE (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library.
"""

from .ht_oracle import (  # noqa: F401
    BHT,
    BatchInfo,
    DimTree,
    Node,
    Truncation,
    compress_stream,
    contract_mode,
    contract_mode_t,
    fro2,
    sign_normalise,
    truncated_svd,
    unfold,
)
