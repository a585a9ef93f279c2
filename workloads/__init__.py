"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

Holds code construction, error/syndrome sampling, bit packing and the
logical-failure check; none of the decoding method's arithmetic lives here.
"""
from . import codes, sample, logical  # noqa: F401

# Named configurations: workload name -> (p, max_iter, message formats, lottery, osd, shots, seeds)
CONFIGS = {
    "surface5_cc": dict(p=0.05, max_iter=50, scale_mode="const", scale=0.625, lottery=False,
                        osd="osd0", shots=10_000, seed=1001, lottery_seed=2001),
    "surface11_phen": dict(p=0.01, max_iter=100, scale_mode="paper", lottery=True,
                           osd="osd0", shots=1_000_000, seed=1002, lottery_seed=2002),
    "bb144_cc": dict(p=0.01, max_iter=100, scale_mode="paper", lottery=True,
                     osd="osd0", shots=1_000_000, seed=1030, lottery_seed=2030),
    "bb144_phen": dict(p=0.003, max_iter=200, scale_mode="paper", lottery=True,
                       osd="osd_cs", osd_order=10, shots=1_000_000, seed=1004, lottery_seed=2004),
}
