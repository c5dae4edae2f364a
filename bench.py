"""Benchmark: MHD cell-updates/s on one MI355X.

Headline workload (one "step"): configuration 3 at full size, the batched
configuration -- 4096 equal-size patches in a periodic unit box whose
interior sizes are drawn uniformly from {16^3, 24^3, 32^3} (6.9e7 cells),
lognormal density (sigma_ln rho = 2), p = 0.01 rho, B along z at beta = 1 --
advanced with local time steps (dt = dt_base 2^-k, k = 0..7) over its whole
run, t = 0 -> 8 dt_base, in FP32.  A step re-initialises the set from a
device-resident copy of the initial state and runs the whole hot path every
round: readiness scan, guard fill (time interpolation, resampling across
resolution jumps), Courant levels, MUSCL-Hancock + HLLD + CT, publish.

Printed: one JSON line with the batched FP32 rate of that workload as
`value` and its roofline record (HBM bound: the algorithmic bytes of every
patch update -- own slice read and written, the two guard layers the stencil
reads from one or two time slices -- over the HIP-event time of the rounds'
update launches, against 8 TB/s).  Beside it: configuration 2 (512 patches of
16^3, Mach-5 turbulence) in FP32 with its own roofline record, FP64 batched,
the plain one-patch-per-launch FP64 path, the adjoint leg, the local-dt
saving, the copy bandwidth, and the CPU oracle on the host cores.
"""
import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK = 157.3  # TFLOP/s, MI355X dense FP32 vector
HBM_PEAK = 8000.0         # GB/s
SOURCES = ("dsp_fused.hip", "dsp_guard.h", "mhd_dev.h")


def source_digest():
    h = hashlib.sha256()
    for name in SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1705_10774_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(profile):
    """HBM bytes per update launch sequence from a committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy), or None when the
    kernel sources have changed since the counters were taken."""
    try:
        text = open(os.path.join(ROOT, "profiles", profile)).read()
    except OSError:
        return None
    fields = dict(line.split(":", 1) for line in text.splitlines()
                  if line.startswith(("source_sha256_16:", "hbm_bytes_per_launch:")))
    if fields.get("source_sha256_16", "").strip() != source_digest():
        return None
    return float(fields["hbm_bytes_per_launch"])


def roofline(res, kernel, profile, flops):
    """HBM roofline record of the update launches of a run (res from
    run_batched): algorithmic bytes per launch sequence over its average
    HIP-event duration."""
    kern_s = res["kern_ms"] / 1e3
    launches = max(res["kern_launches"], 1)
    achieved = res["algo_bytes"] / kern_s / 1e9 if kern_s > 0 else 0.0
    rec = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK, "unit": "GB/s",
           "frac": achieved / HBM_PEAK, "traffic": measured_traffic(profile), "kernel": kernel,
           "launches": res["kern_launches"], "avg_launch_ms": res["kern_ms"] / launches,
           "algorithmic_bytes_per_launch": res["algo_bytes"] / launches,
           "algorithmic_bytes_per_update": res["algo_bytes"] / max(res["updates"], 1)}
    # context: the vector-ALU side of the same launches (the oracle's tally of
    # operations per update; FP32 vector peak)
    if flops:
        per_update = flops["flops_per_update"] if res["fused"] == 2 else flops["step_flops_per_update"]
        tflops = per_update * res["updates"] / kern_s / 1e12 if kern_s > 0 else 0.0
        rec["alu"] = {"achieved": tflops, "peak": FP32_VECTOR_PEAK, "unit": "TFLOP/s",
                      "frac": tflops / FP32_VECTOR_PEAK, "flops_per_update": per_update}
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-baselines", action="store_true", help="only the headline workload")
    ap.add_argument("--cpu-rounds", type=int, default=3, help="rounds of the CPU oracle sample")
    ap.add_argument("--only", choices=["cfg3", "cfg2", "cfg2-fp64", "adjoint"],
                    help="run one leg alone (for profiling)")
    ap.add_argument("--dispatch", choices=["auto", "rounds", "queue"], default="auto",
                    help="dispatch of the local steps: the autotuner's choice, the rounds, or the persistent queue "
                         "(where available)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run 3 plain device copies of 256 MiB (scale for the FETCH_SIZE / "
                         "WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU sharding "
                                   "is not part of this build"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1705_10774_amd import dsp
    from paper_1705_10774_amd import inputs as I

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        a = torch.ones(256 * 1024 * 1024 // 4, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"copies": 3, "bytes_each": a.numel() * 4}}), flush=True)
        return
    flops = json.load(open(os.path.join(ROOT, "tests", "golden", "flops_per_update.json")))

    def run_batched(pr, t_end, steps, warmup, prec, dispatch=None):
        """steps timed runs t 0 -> t_end from a device-resident initial state."""
        s = dsp.PatchSet(dataclasses.replace(pr.cfg, prec=prec), pr.patches)
        tdt = torch.float32 if prec == I.F32 else torch.float64
        U0 = torch.from_numpy(pr.U0).to(dev).to(tdt).contiguous()
        dispatch = dispatch or args.dispatch
        avail = s.dispatch()[1]
        if dispatch == "rounds" or (dispatch == "queue" and not avail):
            s.set_dispatch(dsp.DSP_DISPATCH_ROUNDS)
        elif dispatch == "queue":
            s.set_dispatch(dsp.DSP_DISPATCH_QUEUE)
        elif avail and pr.cfg.dt_mode == I.DT_LOCAL:
            # the autotuner picks rounds or the persistent queue on the first
            # dt_base of this workload (timed from the initial state, which
            # it restores)
            s.init_device(U0.data_ptr())
            s.autotune(pr.cfg.dt_base)
        for _ in range(warmup):
            s.init_device(U0.data_ptr())
            s.advance_to(t_end)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s.init_device(U0.data_ptr())
            s.advance_to(t_end)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = s.stats()
        ks = s.kernel_stats()  # update launches of the last step: ms, launches, algorithmic bytes
        mode = s.dispatch()[0]
        s.close()
        del U0
        return dict(sec=(t1 - t0) / max(steps, 1), updates=st[0], rounds=st[13], kern_ms=ks[0],
                    kern_launches=ks[1], algo_bytes=ks[2], fused=ks[3], floor_hits=st[10],
                    cells=pr.cells, patches=len(pr.patches),
                    dispatch="queue" if mode == dsp.DSP_DISPATCH_QUEUE else "rounds")

    def run_adjoint():
        # adjoint: 64 patches of 16^3, 32 fixed FP64 steps, checkpoints every 8
        pr5 = I.cfg5_adjoint(prec=I.F64)
        s = dsp.PatchSet(pr5.cfg, pr5.patches)
        U5 = torch.from_numpy(pr5.U0).to(dev)
        # warm-up of both passes: the reverse allocates its work buffers on
        # first use, which the timed run must not include
        UTw, ckw = s.fixed_steps_fwd(U5, pr5.nsteps)
        s.fixed_steps_adj(ckw, torch.ones_like(UTw), pr5.nsteps)
        del UTw, ckw
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        UT5, ck5 = s.fixed_steps_fwd(U5, pr5.nsteps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s.fixed_steps_adj(ck5, torch.ones_like(UT5), pr5.nsteps)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        s.close()
        return {"workload": "64 patches of 16^3, 32 fixed FP64 steps, checkpoints every 8",
                "forward_ms": (t1 - t0) * 1e3, "adjoint_ms": (t2 - t1) * 1e3,
                "adjoint_over_forward": (t2 - t1) / (t1 - t0)}

    if args.only == "adjoint":
        print(json.dumps({"adjoint": run_adjoint()}), flush=True)
        return
    if args.only in ("cfg2", "cfg2-fp64"):
        pr = I.cfg2_turb()
        prec = I.F32 if args.only == "cfg2" else I.F64
        r = run_batched(pr, pr.t_end, args.steps, args.warmup, prec)
        print(json.dumps({args.only: {"value": r["updates"] / r["sec"], "ms_per_step": r["sec"] * 1e3,
                                      "dispatch": r["dispatch"],
                                      "roofline": roofline(r, "k_step2<float, 16>" if prec == I.F32 else
                                                           "k_step<double, 16>", "", flops)}}), flush=True)
        return

    # ---- headline: configuration 3 at full size over its whole run, FP32
    pr3 = I.cfg3_uneven(prec=I.F32)
    T3 = pr3.t_end  # 8 dt_base
    r3 = run_batched(pr3, T3, args.steps, args.warmup, I.F32)
    value = r3["updates"] / r3["sec"]
    out = {
        "metric": "MHD cell-updates/s on 1 GPU, batched FP32 vs plain FP64; % of HBM peak",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r3["sec"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded lognormal density, E(k)~k^-2, uneven patch sizes)",
        "config": {"workload": "cfg3: 4096 patches of 16^3/24^3/32^3 (6.9e7 cells, periodic), local dt, "
                               "t 0 -> 8 dt_base",
                   "patches": r3["patches"], "cells": r3["cells"],
                   "updates_per_step": r3["updates"], "rounds_per_step": r3["rounds"]},
        "roofline": roofline(r3, "round update sequence: k_gfill<float> + k_courant<float> + k_step2<float, 0>",
                             "update_cfg3_fp32_traffic.md", flops),
    }
    if args.only == "cfg3" or args.no_baselines:
        print(json.dumps(out), flush=True)
        return
    # local-dt saving of the headline workload: updates with one global
    # quantised step (the finest level of the set) over local steps
    s = dsp.PatchSet(dataclasses.replace(pr3.cfg, dt_mode=I.DT_GLOBAL_QUANT), pr3.patches)
    s.init(pr3.U0)
    s.advance_to(pr3.cfg.dt_base)
    upd_g = s.stats()[0]
    s.close()
    s = dsp.PatchSet(pr3.cfg, pr3.patches)
    s.init(pr3.U0)
    s.advance_to(pr3.cfg.dt_base)
    upd_l = s.stats()[0]
    s.close()
    out["local_dt_saving"] = {"cfg3_first_dt_base": upd_g / upd_l}

    # ---- configuration 2 (512 patches of 16^3, Mach 5), FP32 and FP64
    pr2 = I.cfg2_turb()
    r2 = run_batched(pr2, pr2.t_end, args.steps, args.warmup, I.F32)
    out["cfg2_fp32"] = {"workload": "cfg2: 512 patches of 16^3 (128^3 periodic), local dt, t 0 -> 0.02",
                        "value": r2["updates"] / r2["sec"], "ms_per_step": r2["sec"] * 1e3,
                        "updates_per_step": r2["updates"], "rounds_per_step": r2["rounds"],
                        "roofline": roofline(r2, "k_step2<float, 16>", "k_step2_cfg2_fp32_traffic.md", flops)}
    r64 = run_batched(pr2, pr2.t_end, 1, 1, I.F64)
    out["fp64_batched"] = {"workload": "cfg2, t 0 -> 0.02", "value": r64["updates"] / r64["sec"],
                           "ms_per_step": r64["sec"] * 1e3,
                           "roofline": roofline(r64, "k_step<double, 16>", "k_step_cfg2_fp64_traffic.md", None)}
    # plain path: one patch per launch sequence, host round trip per update;
    # a bounded leg (the first 4 dt_base of configuration 2)
    s = dsp.PatchSet.from_problem(pr2)
    T = 4 * pr2.cfg.dt_base
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.advance_to_plain(T)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pst = s.stats()
    s.close()
    plain_rate = pst[0] / (t1 - t0)
    out["fp64_plain"] = {"value": plain_rate, "sample": "cfg2, t 0 -> 4 dt_base", "updates": pst[0],
                         "note": "the plain method: the host picks one ready patch at a time and launches its "
                                 "fill, Courant, step and publish kernels, synchronising for every dt; bound by "
                                 "launch and round-trip latency, not by the kernels (slower than the CPU oracle "
                                 "on 16 cores), so the speedup over it measures the batching, not kernel quality"}
    out["speedup_batched_fp32_vs_plain_fp64"] = {"cfg2": out["cfg2_fp32"]["value"] / plain_rate,
                                                 "cfg2_fp64_batched": out["fp64_batched"]["value"] / plain_rate}
    s = dsp.PatchSet.from_problem(pr2, dt_mode=I.DT_GLOBAL_QUANT, prec=I.F32)
    s.advance_to(pr2.t_end)
    out["local_dt_saving"]["cfg2"] = s.stats()[0] / r2["updates"]
    s.close()
    out["adjoint"] = run_adjoint()
    # plain device copy bandwidth on this GPU (256 MiB, read + write)
    a = torch.ones(64 * 1024 * 1024, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        b.copy_(a)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    out["copy_GBs"] = 10 * 2 * a.numel() * 4 / (t1 - t0) / 1e9
    del a, b

    # ---- CPU baseline: the oracle on the host cores, on a bounded sample of
    # the headline workload (its first rounds; every patch is ready in the
    # first round, the finer ones in the next)
    from oracle import oracle
    cores = len(os.sched_getaffinity(0))
    o = oracle.OracleSet.from_problem(pr3)
    o.set_order(2, 1, cores)
    t0 = time.perf_counter()
    o.advance_limited(T3, args.cpu_rounds)
    t1 = time.perf_counter()
    ost = o.stats()
    o.close()
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    rate = ost[0] / (t1 - t0)
    out["cpu_baseline"] = {"value": rate, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
                           "sample": f"cfg3 full size, first {args.cpu_rounds} rounds ({int(ost[0])} updates, "
                                     f"{t1 - t0:.1f} s), FP64",
                           "per_core": rate / cores, "cpu_model": model}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
