"""Float BP's accuracy criterion: the logical error rate of the GPU's FP32 and
FP16 decoders falls inside the 95% Wilson interval of the pure-FP64 oracle's
rate on the same seeded shots (with at least 100 oracle failures, so that the
interval is narrow enough to mean something).  Bit-level identity is tested
against the storage-matched oracle in test_gpu_parity; this is the comparison
with exact arithmetic.

Workloads: rotated surface d=9 over 9 rounds with the noiseless final read-out
(BP without OSD at p=0.004: the failures are shots BP leaves with a residual
syndrome) and BB[[144,12,12]] code capacity at p=0.05 with OSD-0 (every failure
is a logical error)."""
import sys

import numpy as np
import pytest

import oracle
from tests.gpu_util import batch, gpu_decode, oracle_params
from workloads import codes, sample
from workloads.logical import LogicalChecker, failures_packed, wilson

pytestmark = pytest.mark.gpu

CASES = [
    ("surface9_phenpf", 0.004, 10000, 1301, dict(max_iter=100, lottery=True, osd=0, seed=31)),
    ("bb144_cc", 0.05, 10000, 1302, dict(max_iter=100, lottery=True, osd=1, seed=32)),
]


def _failures(name, e, corr, n):
    h, hc, r = codes.workload_matrices(name)
    single = h[: h.shape[0] // r, : hc.shape[1]]
    sf, lf = failures_packed(LogicalChecker(single, hc, r), sample.pack_sparse(e), corr, n)
    return int((sf | lf).sum()), int(lf.sum())


@pytest.mark.parametrize("msg", [0, 1], ids=["fp32", "fp16"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_float_ler_inside_fp64_oracle_interval(case, msg):
    from paper_2605_00038_amd import DecoderParams
    name, p, shots, seed, kw = case
    h, e, syn = batch(name, p, shots, seed)
    prm = DecoderParams(msg=msg, **kw)
    g = gpu_decode(h, p, prm, syn)
    o = oracle.decode(h, p, oracle_params(prm, msg=oracle.FP64), syn, n_threads=8)
    kg, lg = _failures(name, e, g["corr"], h.shape[1])
    ko, lo_ = _failures(name, e, o["corr"], h.shape[1])
    lo, hi = wilson(ko, shots)
    same = (g["corr"] == o["corr"]).all(axis=1).mean()
    print(f"{name} msg={msg}: GPU {kg} ({lg} logical), FP64 oracle {ko} ({lo_} logical) of {shots}; "
          f"oracle 95% [{lo:.4f}, {hi:.4f}], GPU {kg / shots:.4f}; identical corrections {same:.4f}",
          file=sys.stderr, flush=True)
    assert ko >= 100
    assert lo <= kg / shots <= hi
