"""CPU oracle for batched Lottery BP (+OSD): test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg
may import this package.  The product path (``paper_2605_00038_amd``) never
imports it and shares no code with it.
"""
from .oracle import (  # noqa: F401
    OracleParams, build, decode, osd, lottery_pick, philox4x64_10, store, prior_int8, prior_fixed, policy_code,
    CN_RANDOM, CN_WORST, VN_PROPOSED, VN_Q_FIRST, VN_UNRELIABLE, VN_RANDOM,
    FP32, FP16, INT8, FP64, FLIP_MSG, FLIP_LLR, OSD_NONE, OSD_0, OSD_CS,
    FLAG_CONVERGED, FLAG_OSD, FLAG_OSD_INCONSISTENT,
)
