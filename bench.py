#!/usr/bin/env python
"""Decoded syndromes/s and p99 latency on one MI355X: BB[[144,12,12]] phenomenological.

Workload: the space-time matrix of BB[[144,12,12]] over 12 rounds (864 checks x
2592 columns, 6840 edges), i.i.d. flips at p = 0.003, Lottery BP with at most
200 iterations, then OSD-CS order 10 on the shots BP does not converge.  One
step decodes the whole batch (10^6 syndromes by default) through the C ABI;
inputs are resident in HBM before the timed region starts.

Prints one JSON line (see the field list at the end of main()).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from workloads import codes, sample  # noqa: E402
from workloads.logical import LogicalChecker, failures_packed, wilson  # noqa: E402

WORKLOAD = "bb144_phen"
P_ERR = 0.003
MAX_ITER = 200
OSD_ORDER = 10
DATA_SEED = 1004
LOTTERY_SEED = 2004
MSG_CODES = {"fp32": 0, "fp16": 1, "int8": 2}
# VALU issue peak: 256 CUs x 4 SIMD16 x 16 lanes x 2.4 GHz (32-bit ops, no packing)
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# LDS peak: 256 CUs x 128 bytes per clock x 2.4 GHz
LDS_PEAK_TBS = 256 * 128 * 2.4e9 / 1e12
# Algorithmic 32-bit ALU operations per edge-update of NMS BP:
# VN: add into lambda, subtract for alpha, saturate/round; CN: |alpha|, two
# compares for min1/min2, sign xor, select min1/min2, sign apply; hard decision
# and syndrome xor amortized to one more op.
ALG_OPS_PER_EDGE = 10


def _chunk_job(args):
    k, n_total = args
    h, _, _ = codes.workload_matrices(WORKLOAD)
    lo = k * sample.CHUNK
    hi = min(n_total, lo + sample.CHUNK)
    e, syn = sample.make_batch(h, P_ERR, hi - lo, DATA_SEED, first_shot=lo)
    return k, sample.pack_sparse(e), syn


def make_inputs(shots: int, workers: int):
    nchunks = (shots + sample.CHUNK - 1) // sample.CHUNK
    errs = [None] * nchunks
    syns = [None] * nchunks
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        for k, e, s in ex.map(_chunk_job, [(k, shots) for k in range(nchunks)]):
            errs[k] = e
            syns[k] = s
    return np.concatenate(errs), np.concatenate(syns)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_format(torch, h, syn_dev, msg: str, steps: int, warmup: int, shots: int):
    from paper_2605_00038_amd import Code, Decoder, DecoderParams
    prm = DecoderParams(max_iter=MAX_ITER, msg=MSG_CODES[msg], lottery=True, lottery_skip=6, osd=2,
                        osd_order=OSD_ORDER, seed=LOTTERY_SEED)
    dec = Decoder(Code.from_scipy(h, P_ERR), prm, shots)
    corr = torch.empty((shots, dec.nw), dtype=torch.int32, device="cuda")
    flags = torch.empty(shots, dtype=torch.uint8, device="cuda")
    iters = torch.empty(shots, dtype=torch.int32, device="cuda")
    out = (corr, flags, iters, None)
    for _ in range(warmup):
        dec.decode(syn_dev, out=out)
    torch.cuda.synchronize()
    dec.kernel_times()
    dec.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        dec.decode(syn_dev, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dec.set_timing(False)
    bp_ms, bp_n, osd_ms, osd_n = dec.kernel_times()
    # after the timed region: five steps each bracketed by its own synchronisation (their median)
    runs = []
    for _ in range(5):
        torch.cuda.synchronize()
        t = time.perf_counter()
        dec.decode(syn_dev, out=out)
        torch.cuda.synchronize()
        runs.append((time.perf_counter() - t) * 1e3)
    res = dict(seconds=t1 - t0, bp_ms=bp_ms, bp_launches=bp_n, osd_ms=osd_ms, osd_launches=osd_n, step_ms_runs=runs,
               corr=corr.cpu().numpy().view(np.uint32), flags=flags.cpu().numpy(), iters=iters.cpu().numpy())
    return dec, res


def latency(torch, dec, syn_dev, requests: int):
    """Single-syndrome requests, each from the host call to stream completion."""
    corr = torch.empty((1, dec.nw), dtype=torch.int32, device="cuda")
    flags = torch.empty(1, dtype=torch.uint8, device="cuda")
    out = (corr, flags, None, None)
    for k in range(20):
        dec.decode(syn_dev[k:k + 1], first_shot_id=k, out=out)
    torch.cuda.synchronize()
    lat = np.empty(requests)
    for k in range(requests):
        t0 = time.perf_counter()
        dec.decode(syn_dev[k:k + 1], first_shot_id=k, out=out)
        torch.cuda.synchronize()
        lat[k] = time.perf_counter() - t0
    return lat * 1e6


def baseline_row(torch, h, syn_dev, shots: int, warmup: int):
    """The plain global-memory FP32 path (lbp_decode_baseline) on the first `shots` syndromes."""
    from paper_2605_00038_amd import Code, Decoder, DecoderParams
    prm = DecoderParams(max_iter=MAX_ITER, msg=0, lottery=True, lottery_skip=6, osd=2, osd_order=OSD_ORDER,
                        seed=LOTTERY_SEED)
    dec = Decoder(Code.from_scipy(h, P_ERR), prm, shots)
    s = syn_dev[:shots]
    for _ in range(max(1, warmup)):
        dec.decode_baseline(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    corr, flags, iters = dec.decode_baseline(s)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = dict(corr=corr.cpu().numpy().view(np.uint32), flags=flags.cpu().numpy(), iters=iters.cpu().numpy())
    del dec
    torch.cuda.empty_cache()
    return dt, out


def host_buffer_rate(h, syn, shots: int):
    """lbp_decode_host: host arrays in and out (PCIe copies and device staging
    allocation included); reported beside the HBM-resident value, never as it."""
    from paper_2605_00038_amd import Code, Decoder, DecoderParams
    prm = DecoderParams(max_iter=MAX_ITER, msg=2, lottery=True, lottery_skip=6, osd=2, osd_order=OSD_ORDER,
                        seed=LOTTERY_SEED)
    dec = Decoder(Code.from_scipy(h, P_ERR), prm, shots)
    part = np.ascontiguousarray(syn[:shots])
    dec.decode_host(part[:1024])  # warm-up
    t0 = time.perf_counter()
    dec.decode_host(part)
    dt = time.perf_counter() - t0
    return dict(kind="lbp_decode_host: host syndromes in, host corrections/flags/iters out", shots=shots,
                seconds=dt, syndromes_per_s=shots / dt)


def serving(h, syn, n_requests: int, shots_per_request: int = 1, msg: str = "int8", p50_runs: int = 3):
    """Serving loop under Poisson requests of `shots_per_request` syndromes
    (latency from the scheduled arrival to the poll-visible result).  The rates
    tried are fractions of the back-to-back (flood) rate, up to 1.2x flood; the
    sustained saturation is the highest offered rate with achieved >= 97% of
    offered and a median latency under 2 ms (no backlog).  p50/p99 are then
    reported at 50% (p50_runs independent runs) and 90% of that rate."""
    from paper_2605_00038_amd import Code, DecoderParams, Server
    prm = DecoderParams(max_iter=MAX_ITER, msg=MSG_CODES[msg], lottery=True, lottery_skip=6, osd=2,
                        osd_order=OSD_ORDER)
    srv = Server(max_slots=1)
    slot = srv.add_code(Code.from_scipy(h, P_ERR), prm)
    pool = syn[: min(len(syn), 1 << 18)]

    def run(rate, n, seed):
        lat, _, el = srv.run_load([slot], [pool], n, shots_per_request, rate, seed)
        return dict(offered_requests_per_s=rate, achieved_requests_per_s=n / el, requests=n,
                    p50_us=float(np.percentile(lat, 50)), p99_us=float(np.percentile(lat, 99)),
                    p999_us=float(np.percentile(lat, 99.9)))

    run(0.0, min(n_requests, 20000), LOTTERY_SEED)  # warm-up
    flood = run(0.0, n_requests, LOTTERY_SEED)
    sweep, sat, limit = [], None, None

    def sustained(r, rate):
        return r["achieved_requests_per_s"] >= 0.97 * rate and r["p50_us"] < 2000.0

    fracs = (0.05, 0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9, 0.95, 1.0, 1.05, 1.1, 1.2)
    lo_frac, hi_frac = 0.0, None
    for k, frac in enumerate(fracs):
        rate = frac * flood["achieved_requests_per_s"]
        r = run(rate, int(max(20000, min(n_requests, rate * 0.5))), LOTTERY_SEED + 1 + k)
        r["fraction_of_flood"] = frac
        sweep.append(r)
        if sustained(r, rate):
            sat, lo_frac = rate, frac
        else:
            limit = "achieved < 97% of offered" if r["achieved_requests_per_s"] < 0.97 * rate else "p50 >= 2 ms"
            hi_frac = frac
            break
    # between the last sustained rate and the first that was not: three bisection steps
    for k in range(3 if hi_frac is not None else 0):
        frac = 0.5 * (lo_frac + hi_frac)
        rate = frac * flood["achieved_requests_per_s"]
        r = run(rate, int(max(20000, min(n_requests, rate * 0.5))), LOTTERY_SEED + 40 + k)
        r["fraction_of_flood"] = frac
        sweep.append(r)
        if sustained(r, rate):
            sat, lo_frac = rate, frac
        else:
            hi_frac = frac
    out = dict(msg=msg, shots_per_request=shots_per_request, flood=flood, sweep=sweep,
               saturation_requests_per_s=sat, saturation_syndromes_per_s=(sat or 0.0) * shots_per_request,
               sweep_stopped_by=limit or "every rate tried was sustained")
    if sat:
        runs = [run(0.5 * sat, int(max(20000, min(n_requests, 0.5 * sat))), LOTTERY_SEED + 20 + i)
                for i in range(p50_runs)]
        out["load50_runs"] = runs
        out["load50"] = sorted(runs, key=lambda r: r["p99_us"])[len(runs) // 2]  # the run with the median p99
        out["load90"] = run(0.9 * sat, int(max(20000, min(n_requests, 0.9 * sat))), LOTTERY_SEED + 29)
    out["slot"] = srv.slot_info(slot)
    srv.close()
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(h, syn, seconds: float, gpu=None):
    """The oracle on the host cores over a bounded prefix of the benchmark batch;
    with the GPU's outputs for the same shots, also the number of shots whose
    correction, flags or iteration count differ (the oracle runs the same Int3.4
    arithmetic, lottery and OSD-CS(10), so the expected count is 0)."""
    import oracle
    threads = os.cpu_count() or 1
    prm = oracle.OracleParams(max_iter=MAX_ITER, msg=oracle.INT8, lottery=True, lottery_skip=6,
                              osd=oracle.OSD_CS, osd_order=OSD_ORDER, seed=LOTTERY_SEED)
    cal = min(len(syn), 2000 * threads)
    t0 = time.perf_counter()
    oracle.decode(h, P_ERR, prm, syn[:cal], n_threads=threads)
    rate = cal / (time.perf_counter() - t0)
    n = int(min(len(syn), max(cal, rate * seconds)))
    t0 = time.perf_counter()
    o = oracle.decode(h, P_ERR, prm, syn[:n], n_threads=threads)
    dt = time.perf_counter() - t0
    n1 = int(min(n, max(1000, rate / threads * seconds / 4)))  # one thread, about a quarter of the time
    t1 = time.perf_counter()
    oracle.decode(h, P_ERR, prm, syn[:n1], n_threads=1)
    dt1 = time.perf_counter() - t1
    out = dict(value=n / dt, unit="syndromes/s", cores=threads, kind="oracle", cpu_model=cpu_model(),
               sample=f"first {n} shots of the benchmark batch, Int3.4 oracle with the same lottery "
                      f"and OSD-CS(10), {threads} threads, {dt:.1f} s",
               single_thread_value=n1 / dt1, single_thread_sample=f"first {n1} shots, 1 thread, {dt1:.1f} s")
    if gpu is not None:
        bad = ((o["corr"] != gpu["corr"][:n]).any(axis=1) | (o["flags"] != gpu["flags"][:n]) |
               (o["iters"] != gpu["iters"][:n]))
        out.update(compared_shots=n, mismatched_shots=int(bad.sum()),
                   osd_shots_compared=int(((o["flags"] & 2) != 0).sum()))
    return out


def bp_kernel_name(msg: str) -> str:
    # Int3.4 codes with at most 1024 checks run the check-centric kernel
    return "bp_int8_kernel" if msg == "int8" else f"bp_kernel_{msg}"


def bp_kernel_source(msg: str) -> str:
    return "bp_int8_kernel.hip" if msg == "int8" else "bp_kernel.hip"


def profile_figures(msg: str) -> dict:
    """Per-launch figures of the committed rocprofv3 PMC summary for the Int3.4
    headline: {"bp_hbm_bytes", "bp_lds_bytes", "osd_hbm_bytes"}, each present
    only while the summary's sha256 of that kernel's source matches the tree."""
    out = {}
    path = os.path.join(ROOT, "profiles", f"{bp_kernel_name(msg)}_{WORKLOAD}_pmc.md")
    if not os.path.exists(path):
        return out
    text = open(path).read()
    csrc = os.path.join(ROOT, "paper_2605_00038_amd", "csrc")
    for kern, src in (("bp", bp_kernel_source(msg)), ("osd", "osd_kernel.hip")):
        m = re.search(rf"{kern}_source_sha256:\s*([0-9a-f]{{64}})", text)
        if not m or hashlib.sha256(open(os.path.join(csrc, src), "rb").read()).hexdigest() != m.group(1):
            continue
        for field in ("hbm", "lds"):
            b = re.search(rf"{kern}_{field}_bytes_per_launch:\s*([0-9.eE+]+)", text)
            if b:
                out[f"{kern}_{field}_bytes"] = float(b.group(1))
    return out


# ---------------------------------------------------------------- experiments
# The paper's ablations and accuracy studies on synthetic phenomenological
# inputs: lottery rules (Sec. III-B, Table I), the skip-K sweep, iteration
# histograms, LER and OSD invoke rate vs p (Sec. VII-A), LLR vs message flip.
# Each prints one JSON object with every point; progress goes to stderr.

def _sample_job(args):
    name, p, seed, lo, hi = args
    h, _, _ = codes.workload_matrices(name)
    e, syn = sample.make_batch(h, p, hi - lo, seed, first_shot=lo)
    return lo, sample.pack_sparse(e), syn


def sample_workload(name: str, p: float, shots: int, seed: int, workers: int):
    """Errors (packed) and syndromes for `shots` shots, chunked by sample.CHUNK."""
    jobs = [(name, p, seed, lo, min(shots, lo + sample.CHUNK)) for lo in range(0, shots, sample.CHUNK)]
    parts = {}
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        for lo, e, s in ex.map(_sample_job, jobs):
            parts[lo] = (e, s)
    keys = sorted(parts)
    return np.concatenate([parts[k][0] for k in keys]), np.concatenate([parts[k][1] for k in keys])


def checker_for(name: str):
    h, hc, r = codes.workload_matrices(name)
    single = h[: h.shape[0] // r, : hc.shape[1]]
    return h, LogicalChecker(single, hc, r)


def decode_point(torch, h, checker, p, err, syn, prm, batch: int = 1 << 18, plain_path: bool = False):
    """Decode every shot (in device batches) and summarize accuracy and iterations;
    plain_path decodes with lbp_decode_baseline (the global-memory FP32 path)."""
    from paper_2605_00038_amd import Code, Decoder
    shots = syn.shape[0]
    dec = Decoder(Code.from_scipy(h, p), prm, min(batch, shots))
    corr = np.empty((shots, dec.nw), np.uint32)
    flags = np.empty(shots, np.uint8)
    iters = np.empty(shots, np.int32)
    dec.kernel_times()
    dec.set_timing(True)
    t0 = t_say = time.perf_counter()
    for lo in range(0, shots, batch):
        hi = min(shots, lo + batch)
        s = torch.from_numpy(np.ascontiguousarray(syn[lo:hi]).view(np.int32)).cuda()
        if plain_path:
            c, f, it = dec.decode_baseline(s, first_shot_id=lo)
        else:
            c, f, it, _ = dec.decode(s, first_shot_id=lo)
        corr[lo:hi] = c.cpu().numpy().view(np.uint32)
        flags[lo:hi] = f.cpu().numpy()
        iters[lo:hi] = it.cpu().numpy()
        if time.perf_counter() - t_say > 20.0:   # long OSD-heavy points: show progress
            t_say = time.perf_counter()
            log(f"    {hi}/{shots} shots decoded, {t_say - t0:.0f} s")
    gpu_s = time.perf_counter() - t0
    bp_ms, bp_n, osd_ms, osd_n = dec.kernel_times()
    dec.set_timing(False)
    del dec
    sf, lf = failures_packed(checker, err, corr, h.shape[1])
    k = int((sf | lf).sum())
    conv = (flags & 1) != 0
    hist = np.bincount(iters, minlength=prm.max_iter + 1)
    return dict(shots=shots, failures=k, ler=k / shots, ler_ci95=list(wilson(k, shots)),
                synd_fail=int(sf.sum()), logical_fail=int(lf.sum()),
                not_converged=float((~conv).mean()), osd_invoke_rate=float(((flags & 2) != 0).mean()),
                mean_iters=float(iters.mean()), max_iter_hits=int((~conv).sum()),
                iter_hist={int(i): int(c) for i, c in enumerate(hist) if c}, decode_s=gpu_s,
                bp_kernel_ms=bp_ms, osd_kernel_ms=osd_ms,
                kernel_syndromes_per_s=shots / max(1e-9, (bp_ms + osd_ms) / 1e3),
                osd_us_per_osd_shot=1e3 * osd_ms / max(1, int(((flags & 2) != 0).sum())))


# The serving mix: single-syndrome requests drawn uniformly over seven codes
# (surface d = 5..21 over d rounds, BB144 over 12 and BB288 over 18 rounds),
# p = 0.003, Int3.4 lottery BP + OSD-0, Poisson arrivals at fractions of the
# mix's flood rate; latency from the scheduled arrival to the poll-visible result.
SERVE_MIX = [("surface5_phen", 100), ("surface9_phen", 100), ("surface13_phen", 100), ("surface17_phen", 100),
             ("surface21_phen", 100), ("bb144_phen", 200), ("bb288_phen", 200)]


def serving_mix(n: int, fracs=(0.1, 0.3, 0.5, 0.7)) -> dict:
    """Single-syndrome Poisson requests drawn uniformly over the seven codes of
    SERVE_MIX, n requests per point, at fractions of the mix's back-to-back
    rate; p50/p99/p99.9 overall and per code."""
    from paper_2605_00038_amd import Code, DecoderParams, Server
    t_start = time.perf_counter()
    srv = Server(device_mem_budget=64 << 30, max_slots=len(SERVE_MIX))  # seven rings, 64 GiB of 288
    slots, pools, names = [], [], []
    for j, (name, iters) in enumerate(SERVE_MIX):
        h, _, _ = codes.workload_matrices(name)
        _, syn = sample.make_batch(h, P_ERR, 4096, 5000 + j)
        prm = DecoderParams(max_iter=iters, msg=2, lottery=True, lottery_skip=6, osd=1, seed=5000 + j)
        slots.append(srv.add_code(Code.from_scipy(h, P_ERR), prm))
        pools.append(syn)
        names.append(name)
        log(f"[servemix] {name} {h.shape[0]}x{h.shape[1]}: slot {slots[-1]} {srv.slot_info(slots[-1])}")

    def stats(lat):
        return dict(requests=int(lat.size), p50_us=float(np.percentile(lat, 50)), p99_us=float(np.percentile(lat, 99)),
                    p999_us=float(np.percentile(lat, 99.9)))

    def run(rate, n, seed):
        lat, code, el = srv.run_load(slots, pools, n, 1, rate, seed)
        r = dict(offered_requests_per_s=rate, achieved_requests_per_s=n / el, overall=stats(lat),
                 per_code={names[k]: stats(lat[code == k]) for k in range(len(names)) if (code == k).any()})
        log(f"[servemix] offered {rate:.0f}/s achieved {n / el:.0f}/s overall p50 {r['overall']['p50_us']:.0f} "
            f"p99 {r['overall']['p99_us']:.0f} p99.9 {r['overall']['p999_us']:.0f} us")
        return r

    run(0.0, min(n, 5000), LOTTERY_SEED)  # warm-up
    flood = run(0.0, n, LOTTERY_SEED)
    points = [run(frac * flood["achieved_requests_per_s"], n, LOTTERY_SEED + 1 + k) for k, frac in enumerate(fracs)]
    srv.close()
    return dict(codes=[dict(workload=nm, max_iter=it) for nm, it in SERVE_MIX], p=P_ERR,
                data="synthetic: i.i.d. Bernoulli(p) flips on every column of H_st, 4096-shot pool per code",
                flood=flood, points=points, seconds=time.perf_counter() - t_start)


def run_servemix(args):
    import torch
    assert torch.cuda.is_available(), "experiments need a GPU"
    out = dict(experiment="servemix", **serving_mix(args.exp_shots))
    text = json.dumps(out)
    if args.exp_out:
        with open(args.exp_out, "w") as f:
            f.write(text + "\n")
    print(text, flush=True)


# The batching configuration: BB[[144,12,12]] code capacity (72 x 144) at four
# error rates, 10^6 shots each (I=100, lottery, OSD-0), packed into one
# persistent launch with the rotated surface d=5 code-capacity shots (12 x 25,
# FP32, constant scale 0.625, plain BP, I=50, OSD-0, 10^4 shots) through an
# autotuned multi-group plan replayed from a HIP graph; the same groups decoded
# by one lbp_decode call each are timed beside it.
BATCH_P = [0.01, 0.02, 0.04, 0.06]


def run_batching(args):
    import torch
    assert torch.cuda.is_available(), "experiments need a GPU"
    from paper_2605_00038_amd import Code, Decoder, DecoderParams, Plan
    t_start = time.perf_counter()
    shots = args.exp_shots
    h_bb, _, _ = codes.workload_matrices("bb144_cc")
    h_s5, _, _ = codes.workload_matrices("surface5_cc")
    out = dict(experiment="batching", data="synthetic: i.i.d. Bernoulli(p) flips on every column, seeded (PCG64, "
               "chunked)", shots_per_p=shots, formats={})
    inputs = []
    for j, p in enumerate(BATCH_P):
        err, syn = sample_workload("bb144_cc", p, shots, 1030 + j, args.workers)
        inputs.append(("bb144_cc", h_bb, p, err, syn, 2030 + j))
    err, syn = sample_workload("surface5_cc", 0.05, 10000, 1001, args.workers)
    inputs.append(("surface5_cc", h_s5, 0.05, err, syn, 2001))
    log(f"[batching] sampled {len(BATCH_P)} x {shots} BB144 code-capacity shots + 10^4 surface d=5 shots")
    for fmt in ("int8", "fp16"):
        groups, decs, meta = [], [], []
        for j, (name, h, p, err, syn, seed) in enumerate(inputs):
            if name == "surface5_cc":
                prm = DecoderParams(max_iter=50, msg=0, scale_mode=1, scale=0.625, lottery=False, osd=1, seed=seed)
            else:
                prm = DecoderParams(max_iter=100, msg=MSG_CODES[fmt], lottery=True, lottery_skip=6, osd=1, seed=seed)
            dec = Decoder(Code.from_scipy(h, p), prm, syn.shape[0])
            s = torch.from_numpy(np.ascontiguousarray(syn).view(np.int32)).cuda()
            groups.append((dec, s, 0))
            decs.append(dec)
            meta.append((name, h, p, err, syn, prm))
        total = sum(g[1].shape[0] for g in groups)
        t0 = time.perf_counter()
        plan = Plan(groups, autotune=True)
        create_s = time.perf_counter() - t0
        wpb, blocks, cand_ms = plan.info()
        runs = []
        for _ in range(args.exp_reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.launch()
            torch.cuda.synchronize()
            runs.append(time.perf_counter() - t0)
        plan_s = float(np.median(runs))
        # the same groups, one lbp_decode each, back to back on one stream
        sep = []
        outs = [(torch.empty((g[1].shape[0], d.nw), dtype=torch.int32, device="cuda"),
                 torch.empty(g[1].shape[0], dtype=torch.uint8, device="cuda"),
                 torch.empty(g[1].shape[0], dtype=torch.int32, device="cuda"), None) for g, d in zip(groups, decs)]
        for rep in range(args.exp_reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for (dec, s, first), o in zip(groups, outs):
                dec.decode(s, first_shot_id=first, out=o)
            torch.cuda.synchronize()
            if rep:
                sep.append(time.perf_counter() - t0)
        sep_s = float(np.median(sep))
        per_group = []
        for g, (name, h, p, err, syn, prm) in enumerate(meta):
            corr, flags, iters = (t.cpu().numpy() for t in plan.outputs[g])
            same_sep = bool(np.array_equal(corr, outs[g][0].cpu().numpy()))
            h_, hc, r = codes.workload_matrices(name)
            sf, lf = failures_packed(LogicalChecker(h_, hc, r), err, corr.view(np.uint32), h.shape[1])
            k = int((sf | lf).sum())
            per_group.append(dict(workload=name, p=p, shots=int(syn.shape[0]), msg=int(prm.msg),
                                  max_iter=prm.max_iter, lottery=bool(prm.lottery), ler=k / syn.shape[0],
                                  ler_ci95=list(wilson(k, syn.shape[0])),
                                  osd_invoke_rate=float(((flags & 2) != 0).mean()), mean_iters=float(iters.mean()),
                                  equal_to_lone_decode=same_sep))
            log(f"[batching] {fmt} {name} p={p}: LER {k / syn.shape[0]:.3e} invoke "
                f"{per_group[-1]['osd_invoke_rate']:.3e} equal to the lone decode: {same_sep}")
        out["formats"][fmt] = dict(
            total_shots=total, plan_create_s=create_s, waves_per_block=wpb, blocks=blocks,
            autotune_candidates_ms=cand_ms, plan_replay_s=plan_s, plan_syndromes_per_s=total / plan_s,
            separate_decodes_s=sep_s, separate_syndromes_per_s=total / sep_s, groups=per_group)
        log(f"[batching] {fmt}: plan {total / plan_s:.3e} syndromes/s ({plan_s * 1e3:.1f} ms, {wpb} waves x "
            f"{blocks} blocks, candidates {[round(x, 2) for x in cand_ms]}), separate decodes "
            f"{total / sep_s:.3e} syndromes/s ({sep_s * 1e3:.1f} ms)")
        del plan, decs, groups, outs
        torch.cuda.empty_cache()
    out["seconds"] = time.perf_counter() - t_start
    text = json.dumps(out)
    if args.exp_out:
        with open(args.exp_out, "w") as f:
            f.write(text + "\n")
    print(text, flush=True)


def run_experiment(args):
    import torch
    assert torch.cuda.is_available(), "experiments need a GPU"
    from paper_2605_00038_amd import DecoderParams, lottery_rule, CN_RANDOM, CN_WORST, VN_PROPOSED, \
        VN_Q_FIRST, VN_UNRELIABLE, VN_RANDOM
    rules = {"proposed": lottery_rule(CN_RANDOM, VN_PROPOSED),
             "proposed_q_first": lottery_rule(CN_RANDOM, VN_Q_FIRST),
             "worst_cn+unreliable_vn": lottery_rule(CN_WORST, VN_UNRELIABLE),
             "worst_cn+random_vn": lottery_rule(CN_WORST, VN_RANDOM),
             "random_cn+unreliable_vn": lottery_rule(CN_RANDOM, VN_UNRELIABLE),
             "random_cn+random_vn": lottery_rule(CN_RANDOM, VN_RANDOM)}
    osd_modes = {"none": 0, "osd_cs10": 2}
    shots = args.exp_shots
    grid = []  # (workload, p, label, params)

    def prm(**kw):
        base = dict(max_iter=args.exp_max_iter, msg=MSG_CODES[args.msg], lottery=True, lottery_skip=6, osd=0,
                    osd_order=OSD_ORDER, seed=LOTTERY_SEED)
        base.update(kw)
        return DecoderParams(**base)

    ps = [float(x) for x in args.exp_p.split(",")] if args.exp_p else None
    sd9 = args.exp_surface
    if args.experiment == "policies":      # Table I / Fig. 5a: surface d = 9
        for p in ps or [0.5e-3, 1e-3, 2e-3]:
            for o, om in osd_modes.items():
                grid.append((sd9, p, f"plain_bp/{o}", prm(lottery=False, osd=om)))
                for r, code in rules.items():
                    grid.append((sd9, p, f"{r}/{o}", prm(lottery_rule=code, osd=om)))
    elif args.experiment == "skip":        # Fig. 5b: when to start the lottery
        for p in ps or [0.5e-3, 1e-3, 2e-3]:
            for k in (0, 1, 2, 4, 6, 8, 12, 16):
                grid.append((sd9, p, f"skip{k}", prm(lottery_skip=k)))
    elif args.experiment == "iters":       # Fig. 6: iteration distribution at p = 1e-4
        for name in (sd9, args.exp_bb):
            for p in ps or [1e-4]:
                grid.append((name, p, "plain_bp", prm(lottery=False)))
                grid.append((name, p, "lottery_bp", prm()))
    elif args.experiment == "ler":         # Fig. 13 / Fig. 14: LER and OSD invoke rate on H_st
        for name in args.exp_workloads.split(","):
            for p in ps or [1e-3, 2e-3, 3e-3, 5e-3]:
                for o, om in osd_modes.items():
                    grid.append((name, p, f"plain_bp/{o}", prm(lottery=False, osd=om)))
                    grid.append((name, p, f"lottery_bp/{o}", prm(osd=om)))
    elif args.experiment == "quant":       # Fig. 15: message formats, surface d = 9
        from paper_2605_00038_amd import msg_fixed
        fmts = [("int2.4", msg_fixed(2, 4)), ("int3.3", msg_fixed(3, 3)), ("int4.2", msg_fixed(4, 2)),
                ("int2.5", msg_fixed(2, 5)), ("int3.4", msg_fixed(3, 4)), ("int4.3", msg_fixed(4, 3)),
                ("fp16", MSG_CODES["fp16"]), ("fp32", MSG_CODES["fp32"])]
        for p in ps or [1e-3, 2e-3, 4e-3]:
            for o, om in osd_modes.items():
                for label, code in fmts:
                    grid.append((sd9, p, f"{label}/{o}", prm(msg=code, osd=om)))
    elif args.experiment == "osdheavy":    # where OSD dominates: high invoke rate, large m
        for name, p in [("bb144_cc", 0.06), ("bb144_cc", 0.08), ("bb288_phen", 0.003), ("surface17_phen", 0.003)]:
            for lot in (False, True):
                grid.append((name, p, ("lottery_bp" if lot else "plain_bp") + "/osd_cs10",
                             prm(lottery=lot, osd=2, max_iter=args.exp_max_iter)))
    elif args.experiment == "scale":       # the paper's code sizes: surface d up to 27 with the final read-out
        for d in [int(x) for x in args.exp_distances.split(",")]:
            for p in ps or [1e-3]:
                for lot in (False, True):
                    grid.append((f"surface{d}_phenpf", p, ("lottery_bp" if lot else "plain_bp") + "/osd0",
                                 prm(lottery=lot, osd=1)))
    elif args.experiment == "formats":     # equal LER across the headline's formats, where logical errors occur
        for p in ps or [7e-3, 1e-2]:
            for o, om in osd_modes.items():
                for label, code in (("int3.4", MSG_CODES["int8"]), ("fp16", MSG_CODES["fp16"]),
                                    ("fp32", MSG_CODES["fp32"])):
                    grid.append((args.exp_bb, p, f"{label}/{o}", prm(msg=code, osd=om)))
                grid.append((args.exp_bb, p, f"plain_fp32_path/{o}", prm(msg=MSG_CODES["fp32"], osd=om)))
    elif args.experiment == "flip":        # what the lottery negates: next messages or lambda itself
        for name in (sd9, args.exp_bb):
            for p in ps or [1e-3, 3e-3]:
                for o, om in osd_modes.items():
                    grid.append((name, p, f"msg_flip/{o}", prm(flip=0, osd=om)))
                    grid.append((name, p, f"llr_flip/{o}", prm(flip=1, osd=om)))
    else:
        raise SystemExit(f"unknown experiment {args.experiment}")

    inputs = {}
    points = []
    t_start = time.perf_counter()
    for name, p, label, pr in grid:
        key = (name, p)
        if key not in inputs:
            inputs.clear()
            t0 = time.perf_counter()
            err, syn = sample_workload(name, p, shots, DATA_SEED, args.workers)
            h, checker = checker_for(name)
            inputs[key] = (h, checker, err, syn)
            log(f"[{args.experiment}] sampled {name} p={p} shots={shots} in {time.perf_counter() - t0:.1f} s")
        h, checker, err, syn = inputs[key]
        # above 16K columns (surface d >= 25), batches of ~2^28 columns keep OSD staging bounded and progress visible
        nb = 1 << 18 if h.shape[1] <= 16384 else max(4096, (1 << 28) // h.shape[1])
        r = decode_point(torch, h, checker, p, err, syn, pr, batch=nb, plain_path=label.startswith("plain_fp32_path"))
        r.update(workload=name, p=p, label=label, max_iter=pr.max_iter, lottery=bool(pr.lottery),
                 lottery_skip=pr.lottery_skip, lottery_rule=pr.lottery_rule, flip=pr.flip, osd=pr.osd,
                 msg=pr.msg)
        points.append(r)
        log(f"[{args.experiment}] {name} p={p} {label}: LER {r['ler']:.3e} "
            f"[{r['ler_ci95'][0]:.2e},{r['ler_ci95'][1]:.2e}] not-conv {r['not_converged']:.3e} "
            f"mean-iter {r['mean_iters']:.2f} BP {r['bp_kernel_ms']:.1f} ms OSD {r['osd_kernel_ms']:.1f} ms "
            f"({r['decode_s']:.1f} s)")
        torch.cuda.empty_cache()
    out = dict(experiment=args.experiment, shots_per_point=shots, data_seed=DATA_SEED, lottery_seed=LOTTERY_SEED,
               data="synthetic: i.i.d. Bernoulli(p) flips on every column of H_st, seeded (PCG64, chunked)",
               seconds=time.perf_counter() - t_start, points=points)
    text = json.dumps(out)
    if args.exp_out:
        with open(args.exp_out, "w") as f:
            f.write(text + "\n")
    print(text, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--shots", type=int, default=1_000_000)
    ap.add_argument("--msg", default="int8", choices=list(MSG_CODES))
    ap.add_argument("--formats", default="int8,fp16,fp32", help="formats timed besides --msg (LER comparison)")
    ap.add_argument("--latency-requests", type=int, default=3000)
    ap.add_argument("--baseline-shots", type=int, default=262_144,
                    help="shots for the plain global-memory FP32 comparison row (0 = skip)")
    ap.add_argument("--no-host-rate", dest="host_rate", action="store_false",
                    help="skip the PCIe-inclusive lbp_decode_host rate")
    ap.add_argument("--serve-requests", type=int, default=200_000,
                    help="single-syndrome requests per serving-loop run (0 = skip)")
    ap.add_argument("--mix-requests", type=int, default=20_000,
                    help="requests per load point of the seven-code serving mix (0 = skip)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-ler", action="store_true")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--experiment", choices=["policies", "skip", "iters", "ler", "flip", "quant", "osdheavy", "scale",
                                             "servemix", "batching", "formats"],
                    help="run one of the paper's ablations instead of the benchmark (prints a JSON table)")
    ap.add_argument("--exp-shots", type=int, default=1 << 20, help="shots per experiment point")
    ap.add_argument("--exp-p", default="", help="comma-separated physical error rates (default: per experiment)")
    ap.add_argument("--exp-max-iter", type=int, default=300, help="BP iteration limit in experiments")
    ap.add_argument("--exp-workloads", default="surface5_phenpf,surface9_phenpf,surface13_phenpf,bb144_phenpf",
                    help="workloads of the ler experiment")
    ap.add_argument("--exp-surface", default="surface9_phenpf", help="surface-code workload of the ablations")
    ap.add_argument("--exp-bb", default="bb144_phenpf", help="BB-code workload of the ablations")
    ap.add_argument("--exp-distances", default="13,17,21,25,27",
                    help="surface-code distances of the scale experiment (d rounds, final read-out)")
    ap.add_argument("--exp-out", default="", help="also write the experiment's JSON to this file")
    ap.add_argument("--exp-reps", type=int, default=5, help="timed repetitions (batching experiment)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (HBM counter calibration)")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch
        src = torch.empty(args.copy_calibration, dtype=torch.uint8, device="cuda")
        src.fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_calibration, "copies": 3}))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: shots are independent, so N GPUs would each decode a disjoint "
              "range of shots with no exchange; only --gpus 1 is supported here.", file=sys.stderr)
        sys.exit(2)
    if args.experiment:
        if args.experiment == "servemix":
            run_servemix(args)
        elif args.experiment == "batching":
            run_batching(args)
        else:
            run_experiment(args)
        return

    h, hc, rounds = codes.workload_matrices(WORKLOAD)
    m, n, E = h.shape[0], h.shape[1], h.nnz
    # inputs are sampled by forked workers before this process touches the GPU
    t0 = time.perf_counter()
    err_p, syn = make_inputs(args.shots, args.workers)
    log(f"sampled {args.shots} shots in {time.perf_counter() - t0:.1f} s")

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    import paper_2605_00038_amd  # noqa: F401  (fails loudly without liblbp.so)
    syn_dev = torch.from_numpy(syn.view(np.int32)).cuda()
    hx, hz = codes.bb144()
    checker = LogicalChecker(hx, hz, rounds)

    formats = [args.msg] + [f for f in args.formats.split(",") if f and f != args.msg]
    per_fmt = {}
    head_dec = None
    for fmt in formats:
        steps = args.steps if fmt == args.msg else max(1, min(args.steps, 2))
        dec, r = time_format(torch, h, syn_dev, fmt, steps, args.warmup, args.shots)
        rate = args.shots * steps / r["seconds"]
        edges = float(r["iters"].astype(np.int64).sum()) * E
        entry = dict(syndromes_per_s=rate, ms_per_step=1e3 * r["seconds"] / steps,
                     bp_ms_per_launch=r["bp_ms"] / max(1, r["bp_launches"]),
                     osd_ms_per_launch=r["osd_ms"] / max(1, r["osd_launches"]),
                     mean_iters=float(r["iters"].mean()), osd_invoke_rate=float(((r["flags"] & 2) != 0).mean()),
                     edge_updates_per_step=edges, steps=steps,
                     step_ms_median_of_5=float(np.median(r["step_ms_runs"])), osd_blocks=dec.shape()["osd_blocks"],
                     bp_waves_per_block=dec.shape()["bp_waves_per_block"], bp_blocks=dec.shape()["bp_blocks"])
        if not args.no_ler:
            sf, lf = failures_packed(checker, err_p, r["corr"], n)
            k = int((sf | lf).sum())
            lo, hi = wilson(k, args.shots)
            entry.update(ler=k / args.shots, ler_ci95=[lo, hi], ler_synd_part=int(sf.sum()), ler_logical_part=int(lf.sum()))
        per_fmt[fmt] = entry
        log(fmt, json.dumps({k: v for k, v in entry.items()}))
        if fmt == args.msg:
            head_dec, head = dec, entry
            head_out = dict(corr=r["corr"], flags=r["flags"], iters=r["iters"])
            if fmt == "int8":
                # OSD alone (its grid otherwise runs alongside BP): the OSD roofline's launch time
                prev = os.environ.get("LBP_EARLY_OSD")
                os.environ["LBP_EARLY_OSD"] = "0"
                try:
                    d2, r2 = time_format(torch, h, syn_dev, fmt, 2, 1, args.shots)
                finally:
                    if prev is None:
                        del os.environ["LBP_EARLY_OSD"]
                    else:
                        os.environ["LBP_EARLY_OSD"] = prev
                entry["osd_alone_ms_per_launch"] = r2["osd_ms"] / max(1, r2["osd_launches"])
                entry["ms_per_step_osd_after_bp"] = 1e3 * r2["seconds"] / 2
                del d2
        else:
            del dec
        torch.cuda.empty_cache()

    base = None
    if args.baseline_shots > 0:
        B = min(args.baseline_shots, args.shots)
        dt, r = baseline_row(torch, h, syn_dev, B, args.warmup)
        base = dict(kind="plain FP32 path: messages in global memory, one thread per check/column, "
                         "a launch per half-iteration (lbp_decode_baseline)",
                    shots=B, seconds=dt, syndromes_per_s=B / dt, mean_iters=float(r["iters"].mean()),
                    osd_invoke_rate=float(((r["flags"] & 2) != 0).mean()))
        if not args.no_ler:
            sf, lf = failures_packed(checker, err_p[:B], r["corr"], n)
            k = int((sf | lf).sum())
            base.update(ler=k / B, ler_ci95=list(wilson(k, B)))
        base["speedup_of_headline"] = head["syndromes_per_s"] / base["syndromes_per_s"]
        log("baseline", json.dumps(base))
    lat = latency(torch, head_dec, syn_dev, args.latency_requests) if args.latency_requests > 0 else None
    del head_dec
    pcie = host_buffer_rate(h, syn, min(args.shots, 262_144)) if args.host_rate else None
    if pcie:
        log("pcie", json.dumps(pcie))
    torch.cuda.empty_cache()
    serve = None
    if args.serve_requests > 0:
        serve = serving(h, syn, args.serve_requests)
        log("serving", json.dumps(serve))
        # what bounds saturation: the same loop with 64-shot requests (the per-request
        # host cost is then spread over 64 syndromes), and the FP32 decoder's tail
        serve["requests_of_64_shots"] = serving(h, syn, max(2000, args.serve_requests // 32), 64, p50_runs=1)
        log("serving 64-shot", json.dumps(serve["requests_of_64_shots"]))
        serve["fp32_decoder"] = serving(h, syn, args.serve_requests, 1, msg="fp32", p50_runs=1)
        log("serving fp32", json.dumps(serve["fp32_decoder"]))
    mix = None
    if args.mix_requests > 0:
        mix = serving_mix(args.mix_requests)
        log("serving mix", json.dumps(mix))
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(h, syn, args.cpu_seconds, head_out)
        log("cpu", json.dumps(cpu))

    bp_s = head["bp_ms_per_launch"] / 1e3
    ops = head["edge_updates_per_step"] * ALG_OPS_PER_EDGE
    achieved = ops / bp_s / 1e12
    prof = profile_figures(args.msg)
    traffic = prof.get("bp_hbm_bytes")
    lds = None
    if "bp_lds_bytes" in prof:
        lds_tbs = prof["bp_lds_bytes"] / bp_s / 1e12
        lds = {"achieved": lds_tbs, "peak": LDS_PEAK_TBS, "unit": "TB/s", "frac": lds_tbs / LDS_PEAK_TBS,
               "bytes_per_launch": prof["bp_lds_bytes"],
               "kind": "lane bytes of LDS loads, stores and atomics (rocprofv3 SQ_INSTS_LDS_*_BANDWIDTH) "
                       "over this run's BP launch time"}
    # OSD: the dense Gauss-Jordan equivalent of Algorithm 2 per OSD shot, m pivots each
    # XORing an m-bit row into m rows (ceil(m/32) words), over the OSD launch time
    osd_s = head.get("osd_alone_ms_per_launch", head["osd_ms_per_launch"]) / 1e3
    n_osd = head["osd_invoke_rate"] * args.shots
    osd_ops = n_osd * m * m * ((m + 31) // 32)
    osd_tops = osd_ops / osd_s / 1e12 if osd_s > 0 else 0.0
    osd_roof = {"bound": "latency", "achieved": osd_tops, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                "frac": osd_tops / VALU_PEAK_TOPS, "kind": "dense Gauss-Jordan word-XOR equivalent",
                "kernel": "osd_reg_kernel", "launch_ms": 1e3 * osd_s, "osd_shots": int(round(n_osd)),
                "traffic": prof.get("osd_hbm_bytes"),
                "us_per_shot_per_block": (1e6 * osd_s * head["osd_blocks"] / max(1.0, n_osd))}
    line = {
        "metric": "decoded syndromes/sec and p99 latency on 1 MI355X, BB-144 phenomenological",
        "value": head["syndromes_per_s"],
        "unit": "syndromes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.msg,
        "data": "synthetic: i.i.d. Bernoulli(p) flips on every column of H_st, seeded (PCG64, chunked)",
        "config": {"workload": "BB[[144,12,12]] phenomenological, 12 rounds, H_st 864x2592 (6840 edges), "
                               "p=0.003, Lottery BP I=200 K=6, OSD-CS(10)",
                   "shots_per_step": args.shots, "data_seed": DATA_SEED, "lottery_seed": LOTTERY_SEED},
        "p99_latency_us": (serve["load50"]["p99_us"] if serve is not None and "load50" in serve
                           else float(np.percentile(lat, 99)) if lat is not None else None),
        "p99_latency_kind": ("serving loop, single-syndrome Poisson requests at 50% of saturation, "
                             "arrival to poll-visible result (median p99 of three runs)" if serve is not None
                             else "single-syndrome decode, host call to stream completion"),
        "serving": serve,
        "serving_mix": mix,
        "latency_us": ({"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                        "p99.9": float(np.percentile(lat, 99.9)), "requests": int(len(lat)),
                        "kind": "single-syndrome lbp_decode, host call to stream completion"}
                       if lat is not None else None),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                     "frac": achieved / VALU_PEAK_TOPS, "traffic": traffic,
                     "kernel": bp_kernel_name(args.msg), "launch_ms": head["bp_ms_per_launch"],
                     "edge_updates_per_s": head["edge_updates_per_step"] / bp_s,
                     "ops_per_edge_update": ALG_OPS_PER_EDGE, "lds": lds},
        "osd_roofline": osd_roof,
        "cpu_baseline": cpu,
        "gpu_plain_fp32_baseline": base,
        "pcie_inclusive": pcie,
        "formats": per_fmt,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
