#!/usr/bin/env python3
"""Benchmark: decoded information throughput of the MI355X turbo decoder.

Workload (one step = one launch decoding the whole batch):
  4096 code blocks of K = 6144 (6120 payload bits + CRC24B), 16QAM over AWGN
  at Es/N0 = 8 dB, int16 LLRs (scale 8, clamp +-2047), windowed max-log-MAP
  with 32 windows of 192 steps and previous-iteration boundary init,
  exactly 6 iterations (early stop off).
Metric: decoded payload Gbit/s at 6 iterations = 4096 * 6120 * steps / wall.
The LLRs are resident in device memory before the timed region starts.

Also reported (stderr + extra JSON fields): the same batch as configured
(at most 8 iterations with CRC24B early stop), the kernel's VALU roofline
fraction, the CPU oracle's throughput on a bounded sample, and short
re-checks of the other workloads' headline figures (--no-checks skips them):
the serving loop at rho = 1 (launch lanes, then ring mode) and the cells
count at its calibrated Es/N0, 1000 TTIs each, every served TB checked
against the oracle.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-checks]
       python bench.py --workload {tb,mixed,serving,cells} [options]

The default workload is the uniform batch above; the others measure the
remaining configurations and print one JSON line each:
  tb      : one 75376-bit transport block (13 x K5824), QPSK Es/N0 2 dB,
            exactly 6 iterations: latency alone (device and host-to-host) at
            full length and at the library's window choice, and throughput
            over a stream of such blocks;
  mixed   : TTIs of 64 transport blocks (log-uniform sizes, QPSK/16QAM/64QAM,
            Es/N0 uniform in [0, 18] dB, <= 8 iterations with CRC stop), each
            TTI one captured-graph launch with autotuned windows;
  serving : the serving loop under Poisson arrivals of 338*rho TBs per 1 ms
            TTI (64QAM, Es/N0 uniform in [12, 22] dB, 3 ms deadline, 8 GB
            slot budget): p50/p99 latency, misses, rejections, Gbit/s;
  cells   : cells of 2 layers x one 75376-bit TB per TTI at 256QAM near 30 %
            TB error rate (Es/N0 calibrated on 2048 TBs per point), 8
            iterations forced: the most cells whose p99 latency stays within
            3 ms (binary search).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_CB = 4096
K = 6144
N_WIN = 32
PAYLOAD = K - 24
ITERS = 6
MOD, ESN0 = "16qam", 8.0
# max-log-MAP work per trellis step and half-iteration: branch metrics 2,
# forward ACS 24, backward ACS 24, extrinsic 39 -> 89; two half-iterations.
OPS_PER_KBIT_ITER = 178
# packed int16 VALU peak: 256 CUs x 4 SIMDs x 16 lanes x 2 halves x 2.4 GHz
PEAK_INT16_TOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "turbo_decode_k6144x4096_traffic.json")
KERNEL_SRC = [os.path.join(ROOT, "paper_1905_01141_amd", "csrc", f)
              for f in ("dec_kernels.hip", "tdec_internal.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    """Hash of the decode kernel's sources (the traffic figures hold for it only)."""
    h = hashlib.sha256()
    for p in KERNEL_SRC:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_src_sha256_16") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def build_inputs(T, D, torch):
    import numpy as np
    import workload as wl
    descs, n_llr, n_bytes = T.make_descs([(K, 0, T.CRC24B)] * N_CB)
    pay_bits = wl.random_bits(wl.rng(2, 0), N_CB * PAYLOAD)
    pay = torch.from_numpy(np.packbits(pay_bits)).cuda()
    coded = torch.zeros(n_llr, dtype=torch.uint8, device="cuda")
    D.cb_encode_batch(descs, pay, coded)  # GPU turbo encoder (CRC24B + 2 RSC + QPP)
    torch.cuda.synchronize()
    llr = wl.channel_blocks(coded.cpu().numpy(), [(K, 0)] * N_CB, MOD, ESN0, wl.rng(2, 1))
    return descs, llr, pay_bits, n_bytes


def host_cpu():
    """What /proc/cpuinfo says about the host: the model name line as given
    (virtual machines often shorten it), family / model / stepping, the
    logical CPUs it lists and the CPUs this process may run on."""
    info = {"model_name": "", "family": None, "model": None, "stepping": None,
            "logical_cpus": 0, "affinity": None}
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                k, _, v = ln.partition(":")
                k, v = k.strip(), v.strip()
                if k == "processor":
                    info["logical_cpus"] += 1
                elif k == "model name" and not info["model_name"]:
                    info["model_name"] = v
                elif k == "cpu family" and info["family"] is None:
                    info["family"] = int(v)
                elif k == "model" and info["model"] is None:
                    info["model"] = int(v)
                elif k == "stepping" and info["stepping"] is None:
                    info["stepping"] = int(v)
    except (OSError, ValueError):
        pass
    try:
        info["affinity"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    return info


def cpu_baseline(llr, sample_cbs: int, threads: int):
    """The plain C oracle (never tuned) on `sample_cbs` blocks of the same
    workload, one block per task on a thread pool (the paper's code block
    parallelism); returns the timing record and, per block, the oracle's
    packed payload bytes, CRC flag and iteration count."""
    from concurrent.futures import ThreadPoolExecutor
    import numpy as np
    import oracle as O
    blk = 3 * (K + 4)
    p = O.params(ITERS, 0, N_WIN, 1)

    def one(i):
        r = O.cb_decode(llr[i * blk:(i + 1) * blk], K, 0, O.CRC24B, p)
        return np.packbits(r["bits"][:PAYLOAD]), r["ok"], r["iters"]

    def timed(n, t):
        t0 = time.perf_counter()
        with ThreadPoolExecutor(max_workers=t) as ex:
            out = list(ex.map(one, range(n)))
        return time.perf_counter() - t0, out

    O.lib()
    dt, out = timed(sample_cbs, threads)
    # also one thread and the paper's six dedicated cores, on 256 blocks each
    sweep = []
    for t in (1, 6):
        n = min(256, sample_cbs)
        d, _ = timed(n, t)
        sweep.append({"threads": t, "value": round(n * PAYLOAD / d / 1e9, 6), "blocks": n})
    cpu = host_cpu()
    rec = {"value": round(sample_cbs * PAYLOAD / dt / 1e9, 6), "unit": "Gbit/s",
           "cores": threads, "kind": "oracle",
           "sample": f"{sample_cbs} of the {N_CB} code blocks, {ITERS} iterations, "
                     f"{N_WIN} windows, one block per task; {dt:.2f} s wall, "
                     f"{sum(o[1] for o in out)} CRC pass",
           "by_threads": sweep, "cpu": cpu["model_name"], "cpu_info": cpu,
           "threads_note": "the host grants 16 CPUs per GPU; the pool uses "
                           "min(16, CPUs this process may run on)"}
    return rec, out


def oracle_tb_reference(llr, lo, tbs, iters, early_stop, nws, threads):
    """The cpu_baseline leg of the transport block workloads: the plain C
    oracle decodes every transport block of a workload's pool once (one TB
    per task on a thread pool) with the decoder's window counts per block.
    Returns the timing record and, per TB, (payload bytes, tb_ok,
    max_iters_used): the reference every served result is checked against."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle as O
    O.lib()
    p = O.params(iters, early_stop, 0, 1)

    def one(i):
        t = int(tbs[i])
        b, r = O.tb_decode_windows(llr[int(lo[i]):int(lo[i]) + O.tb_llr_count(t)], t, p, nws[i])
        return b, int(r["tb_ok"]), int(r["max_iters_used"])

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        out = list(ex.map(one, range(len(tbs))))
    dt = time.perf_counter() - t0
    rec = {"value": round(float(sum(int(t) for t in tbs)) / dt / 1e9, 6), "unit": "Gbit/s",
           "cores": threads, "kind": "oracle",
           "sample": f"the {len(tbs)} transport blocks of the pool once, {iters} iterations"
                     f"{' with CRC stop' if early_stop else ' forced'}, the decoder's window "
                     f"counts; {dt:.2f} s wall"}
    return rec, out


def oracle_threads():
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = os.cpu_count() or 1
    return max(1, min(16, avail))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-checks", action="store_true",
                    help="uniform workload: skip the short serving (rho = 1, both forms) and cells "
                         "re-checks")
    ap.add_argument("--cpu-sample", type=int, default=N_CB)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    ap.add_argument("--workload", default="uniform",
                    choices=["uniform", "tb", "mixed", "serving", "cells", "ratematch", "encode",
                             "stop", "peaks"])
    ap.add_argument("--rho", type=str, default="0.25,0.5,1,2,4",
                    help="serving: load points (fractions of 40 cells' capacity)")
    ap.add_argument("--ttis", type=int, default=3000, help="serving/cells: measured TTIs")
    ap.add_argument("--mode", default="continuous", choices=["continuous", "per-tb", "ring"],
                    help="serving/cells: batching form (ring: one persistent kernel fed from a "
                         "work ring)")
    ap.add_argument("--min-w", type=int, default=0,
                    help="mixed/serving/cells: shortest window the autotuner may choose, in steps "
                         "(0: 32 for the mixed TTIs, 64 for serving and cells)")
    ap.add_argument("--inflight", type=int, default=0,
                    help="serving/cells: launches in flight at once (0: the server's default, 3)")
    ap.add_argument("--windows", default="tuned", choices=["tuned", "rule"],
                    help="serving/cells: autotuned window counts (latency objective) or the "
                         "library's built-in rule")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (code blocks, "
              "transport blocks and cells are independent, so GPUs would shard by cell)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1905_01141_amd as T

    torch.cuda.set_device(0)
    if args.workload != "uniform":
        import bench_workloads as BW
        args.oracle_ref = oracle_tb_reference
        args.oracle_threads = oracle_threads()
        line = getattr(BW, "run_" + args.workload)(args)
        print(json.dumps(line), flush=True)
        return
    D = T.Decoder(0)
    log("[bench] building inputs: GPU encoder + 16QAM AWGN channel")
    descs, llr_h, pay_bits, n_bytes = build_inputs(T, D, torch)
    x = torch.from_numpy(llr_h).cuda()
    bits = torch.zeros(n_bytes, dtype=torch.uint8, device="cuda")
    ok = torch.zeros(N_CB, dtype=torch.uint8, device="cuda")
    it = torch.zeros(N_CB, dtype=torch.uint8, device="cuda")
    p6 = T.params(ITERS, 0, N_WIN, 1)
    stream = torch.cuda.current_stream()

    log(f"[bench] warmup {args.warmup}")
    for _ in range(args.warmup):
        D.cb_decode_batch(descs, x, p6, bits, ok, it, stream=stream)
    torch.cuda.synchronize()

    log(f"[bench] timing {args.steps} steps")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        D.cb_decode_batch(descs, x, p6, bits, ok, it, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dev_ms = e0.elapsed_time(e1)
    ms_step = wall * 1e3 / args.steps
    value = N_CB * PAYLOAD * args.steps / wall / 1e9
    launch_s = dev_ms / 1e3 / args.steps
    ops = OPS_PER_KBIT_ITER * N_CB * K * ITERS
    achieved = ops / launch_s / 1e12

    # the timed run's outputs, kept for the comparison with the oracle
    bits6 = bits.cpu().numpy().copy()
    ok6 = ok.cpu().numpy().copy()
    it6 = it.cpu().numpy().copy()
    # correctness of the timed output against the transmitted payload
    got = np.unpackbits(bits6)
    okh = ok6
    errs = int(np.count_nonzero(got.reshape(N_CB, -1)[:, :PAYLOAD] !=
                                pay_bits.reshape(N_CB, PAYLOAD)))
    log(f"[bench] 6-iteration run: {value:.3f} Gbit/s, {ms_step:.3f} ms/step, "
        f"kernel {launch_s * 1e3:.3f} ms, CRC pass {int(okh.sum())}/{N_CB}, bit errors {errs}")

    # as configured: <= 8 iterations, CRC24B early stop
    p8 = T.params(8, 1, N_WIN, 1)
    D.cb_decode_batch(descs, x, p8, bits, ok, it, stream=stream)
    torch.cuda.synchronize()
    n_cfg = max(1, args.steps // 2)
    t1 = time.perf_counter()
    for _ in range(n_cfg):
        D.cb_decode_batch(descs, x, p8, bits, ok, it, stream=stream)
    torch.cuda.synchronize()
    wall8 = time.perf_counter() - t1
    iters8 = it.cpu().numpy()
    as_cfg = {"value": round(N_CB * PAYLOAD * n_cfg / wall8 / 1e9, 4), "unit": "Gbit/s",
              "max_iters": 8, "early_stop": 1, "mean_iters": round(float(iters8.mean()), 4),
              "max_iters_seen": int(iters8.max()),
              "crc_pass": int(ok.cpu().numpy().sum())}
    log(f"[bench] as configured: {as_cfg}")

    if args.copy_probe_mib:
        n = args.copy_probe_mib << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {n} bytes read + {n} bytes written")

    cpu = None
    parity = None
    # the packed int16 VALU rate this device delivers with the decoder's ACS
    # instructions (independent chains, every CU), beside the published peak
    valu_meas = max(T.probe_valu_int16(0) for _ in range(3))  # the first run is the lowest
    log(f"[bench] measured packed int16 VALU rate {valu_meas:.2f} TOP/s")
    if not args.no_cpu_baseline:
        threads = oracle_threads()
        log(f"[bench] CPU oracle baseline on {threads} threads, {args.cpu_sample} blocks")
        cpu, ref = cpu_baseline(llr_h, args.cpu_sample, threads)
        # every sampled block of the timed 6-iteration run against the oracle:
        # payload bits, CRC flag and iteration count
        per = PAYLOAD // 8
        bad = [i for i, (ob, ook, oit) in enumerate(ref)
               if not (np.array_equal(bits6[i * per:(i + 1) * per], ob) and ok6[i] == ook
                       and it6[i] == oit)]
        parity = {"blocks": len(ref), "mismatches": len(bad), "compared": "payload bits, CRC "
                  "flag and iteration count of the timed 6-iteration run, block by block",
                  "first_mismatches": bad[:8]}
        log(f"[bench] parity against the oracle: {parity}")

    checks = None
    if not args.no_checks:
        import bench_workloads as BW
        args.oracle_ref = None if args.no_cpu_baseline else oracle_tb_reference
        args.oracle_threads = oracle_threads()
        log("[bench] re-checks: serving at rho = 1 (launch lanes and ring mode) and the cells "
            "count, 1000 TTIs each")
        checks = BW.default_checks(args)
        log(f"[bench] re-checks: {checks}")

    line = {
        "metric": "decoded info Gbit/s @6 iters",
        "value": round(value, 4),
        "unit": "Gbit/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int16",
        "data": "synthetic (random payload, GPU turbo encoder, 16QAM AWGN, quantised LLRs)",
        "config": {"workload": "uniform batch: 4096 code blocks K=6144 with CRC24B, 16QAM AWGN "
                               "Es/N0 8 dB, int16 LLRs, 32 windows x 192 steps with "
                               "previous-iteration boundary init, exactly 6 iterations",
                   "n_cb": N_CB, "K": K, "n_windows": N_WIN, "win_init": 1,
                   "max_iters": ITERS, "early_stop": 0, "modulation": MOD, "esn0_db": ESN0},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3),
                     "peak": round(PEAK_INT16_TOPS, 2), "unit": "TOP/s",
                     "frac": round(achieved / PEAK_INT16_TOPS, 4),
                     "traffic": measured_traffic(),
                     "peak_measured": round(valu_meas, 2),
                     "frac_of_measured": round(achieved / valu_meas, 4)},
        "cpu_baseline": cpu,
        "parity": parity,
        "as_configured": as_cfg,
        "kernel_ms": round(launch_s * 1e3, 4),
        "checks": checks,
    }
    print(json.dumps(line), flush=True)
    if parity and parity["mismatches"]:
        sys.exit(3)


if __name__ == "__main__":
    main()
