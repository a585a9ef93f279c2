"""Helpers shared by the GPU tests: run the HIP decoder and the oracle on the same inputs."""
from __future__ import annotations

import numpy as np

import oracle
from workloads import codes, sample

MSG_TO_ORACLE = {0: oracle.FP32, 1: oracle.FP16, 2: oracle.INT8}


def gpu_decode(h, prior, prm, syn, first_shot_id=0, want_llr=False, max_batch=None, osd_cap=None):
    import torch
    from paper_2605_00038_amd import Code, Decoder
    code = Code.from_scipy(h, prior)
    dec = Decoder(code, prm, max_batch or max(1, syn.shape[0]))
    if osd_cap is not None:
        dec.set_osd_capacity(osd_cap)
    s = torch.from_numpy(np.ascontiguousarray(syn).view(np.int32)).cuda()
    corr, flags, iters, llr = dec.decode(s, first_shot_id=first_shot_id, want_llr=want_llr)
    torch.cuda.synchronize()
    out = dict(corr=corr.cpu().numpy().view(np.uint32), flags=flags.cpu().numpy(), iters=iters.cpu().numpy(),
               llr=llr.cpu().numpy() if llr is not None else None)
    return out


def oracle_params(prm, **kw):
    fixed = prm.msg & 0x100
    o = oracle.OracleParams(max_iter=prm.max_iter, scale_mode=prm.scale_mode, scale=prm.scale,
                            msg=oracle.INT8 if fixed else MSG_TO_ORACLE[prm.msg], lottery=prm.lottery,
                            lottery_skip=prm.lottery_skip, flip=prm.flip, osd=prm.osd, osd_order=prm.osd_order,
                            policy=prm.lottery_rule, fx_int=(prm.msg >> 4) & 15 if fixed else 3,
                            fx_frac=prm.msg & 15 if fixed else 4, seed=prm.seed)
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def batch(name, p, shots, seed, first_shot=0):
    h, hc, r = codes.workload_matrices(name)
    e, syn = sample.make_batch(h, p, shots, seed, first_shot)
    return h, e, syn
