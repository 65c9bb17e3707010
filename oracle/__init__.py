"""CPU oracle for the LCS dynamic program (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never imports, links or
calls it.
"""
from .oracle import (  # noqa: F401
    build_oracle,
    use_native_build,
    lcs_length,
    lcs_traceback,
    lcs_traceback_ckpt,
    lcs_tables,
    brute_force_length,
    brute_force_all_lcs,
    recursive_length,
    is_subsequence,
    similarity_percent,
    threshold_pass,
    DIAG,
    UP,
    LEFT,
)
