"""Benchmark: MHD cell-updates/s on one MI355X.

Workload (one "step"): configuration 2 at full size -- 512 patches of 16^3
(128^3 cells, periodic), rho = 1, beta = 0.1 field along x, seeded Gaussian
velocity with E(k) ~ k^-2 over 1 <= |k| <= 4 at rms Mach 5 -- advanced with
local time steps (dt = dt_base 2^-k) from t = 0 to t = 0.02 (0.1 crossing
time).  A step re-initialises the set from a device-resident copy of the
initial state and runs the whole hot path: readiness scan, guard fill,
Courant levels, MUSCL-Hancock + HLLD + CT, publish.

Printed: one JSON line (rank 0) with the batched FP32 rate as `value`, plus
the batched FP64 and plain one-patch-per-launch FP64 rates, the roofline
record of the dominant kernel (vector-ALU bound: the oracle's operation
tally per update over the measured kernel time, against the FP32 vector
peak) and the CPU-oracle baseline.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK = 157.3  # TFLOP/s, MI355X dense FP32 vector
HBM_PEAK = 8000.0         # GB/s


def measured_traffic(algo_bytes_per_launch):
    """HBM bytes per launch of the step kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy), or None when
    the kernel source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_step2_cfg2_fp32_traffic.md")
    src = os.path.join(ROOT, "paper_1705_10774_amd", "csrc", "dsp_fused.hip")
    try:
        text = open(path).read()
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    fields = dict(line.split(":", 1) for line in text.splitlines() if line.startswith(("source_sha256_16:", "hbm_bytes_per_launch:")))
    if fields.get("source_sha256_16", "").strip() != digest:
        return None
    return float(fields["hbm_bytes_per_launch"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-baselines", action="store_true", help="skip FP64, plain and CPU legs")
    ap.add_argument("--cpu-sample", type=int, default=64, help="dt_base units of the CPU sample")
    ap.add_argument("--adjoint", action="store_true",
                    help="only the adjoint leg (64 patches of 16^3, 32 fixed FP64 steps)")
    ap.add_argument("--cfg3", action="store_true",
                    help="only the full-size uneven configuration (FP32, t 0 -> dt_base per step)")
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

    def run_cfg3(steps, warmup):
        # uneven patches at full size (4096 patches of 16^3, 24^3 or 32^3,
        # levels 0..7; two-by-two tiles and a separate Courant pass for the
        # larger patches): FP32, each step t 0 -> dt_base from the
        # device-resident initial state
        pr3 = I.cfg3_uneven(prec=I.F32)
        U3 = torch.from_numpy(pr3.U0).to(dev).float()
        s = dsp.PatchSet(pr3.cfg, pr3.patches)
        del pr3.U0
        for _ in range(warmup):
            s.init_device(U3.data_ptr())
            s.advance_to(pr3.cfg.dt_base)
        ms, upd3 = 0.0, 0.0
        for _ in range(steps):
            s.init_device(U3.data_ptr())
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.advance_to(pr3.cfg.dt_base)
            torch.cuda.synchronize()
            ms += (time.perf_counter() - t0) * 1e3
            upd3 += s.stats()[0]
        s.close()
        return {"workload": "cfg3: 4096 patches of 16^3/24^3/32^3, t 0 -> dt_base",
                "value": upd3 / (ms * 1e-3), "unit": "cell-updates/s", "updates_per_step": upd3 / steps,
                "ms_per_step": ms / steps}

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

    if args.adjoint:
        print(json.dumps({"adjoint": run_adjoint()}), flush=True)
        return

    if args.cfg3:
        print(json.dumps({"cfg3_fp32": run_cfg3(args.steps, args.warmup)}), flush=True)
        return

    def run_batched(prec, steps, warmup):
        pr = I.cfg2_turb(prec=prec)
        s = dsp.PatchSet.from_problem(pr)
        tdt = torch.float32 if prec == I.F32 else torch.float64
        U0 = torch.from_numpy(pr.U0).to(dev).to(tdt).contiguous()
        for _ in range(warmup):
            s.init_device(U0.data_ptr())
            s.advance_to(pr.t_end)
        torch.cuda.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s.init_device(U0.data_ptr())
            s.advance_to(pr.t_end)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = s.stats()
        ks = s.kernel_stats()  # dominant kernel of the last step: ms, launches, algorithmic bytes
        s.close()
        return dict(sec=(t1 - t0) / steps, updates=st[0], rounds=st[13], kern_ms=ks[0],
                    kern_launches=ks[1], algo_bytes=ks[2], fused=ks[3], floor_hits=st[10],
                    cells=pr.cells, patches=len(pr.patches))

    res32 = run_batched(I.F32, args.steps, args.warmup)
    value = res32["updates"] / res32["sec"]
    out = {
        "metric": "MHD cell-updates/s on 1 GPU, batched FP32 vs plain FP64; % of HBM peak",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res32["sec"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Gaussian turbulence, E(k)~k^-2, rms Mach 5)",
        "config": {"workload": "cfg2: 512 patches of 16^3 (128^3 periodic), local dt, t 0 -> 0.02",
                   "patches": res32["patches"], "cells": res32["cells"],
                   "updates_per_step": res32["updates"], "rounds_per_step": res32["rounds"]},
    }
    # dominant kernel: the fused patch step, timed with HIP events on its
    # stream.  Its arithmetic per cell update is the CPU oracle's tally on this
    # workload; it is bound by vector ALU work, not by HBM (about 80
    # algorithmic bytes per update).
    flops = json.load(open(os.path.join(ROOT, "tests", "golden", "flops_per_update.json")))
    kern_s = res32["kern_ms"] / 1e3
    launches = max(res32["kern_launches"], 1)
    # the step kernel also takes the Courant rate when it runs the local
    # step of single-tile patches (kernel_stats()[3] == 2)
    per_update = flops["flops_per_update"] if res32["fused"] == 2 else flops["step_flops_per_update"]
    step_flops = per_update * res32["updates"]
    ach = step_flops / kern_s / 1e12 if kern_s > 0 else 0.0
    hbm = res32["algo_bytes"] / kern_s / 1e9 if kern_s > 0 else 0.0
    out["roofline"] = {"bound": "alu", "achieved": ach, "peak": FP32_VECTOR_PEAK, "unit": "TFLOP/s",
                       "frac": ach / FP32_VECTOR_PEAK,
                       "traffic": measured_traffic(res32["algo_bytes"] / launches),
                       "kernel": "k_step2<float, 16>", "launches": res32["kern_launches"],
                       "avg_launch_ms": res32["kern_ms"] / launches,
                       "flops_per_update": per_update,
                       "algorithmic_bytes_per_update": res32["algo_bytes"] / max(res32["updates"], 1),
                       "algorithmic_hbm_GBs": hbm, "algorithmic_hbm_frac": hbm / HBM_PEAK}
    if not args.no_baselines:
        res64 = run_batched(I.F64, 1, 0)
        out["fp64_batched"] = {"value": res64["updates"] / res64["sec"], "ms_per_step": res64["sec"] * 1e3}
        # plain path: one patch per launch sequence, host round trip per update;
        # a bounded leg (the first 4 dt_base of the same workload)
        pr = I.cfg2_turb(prec=I.F64)
        s = dsp.PatchSet.from_problem(pr)
        T = 4 * pr.cfg.dt_base
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.advance_to_plain(T)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pst = s.stats()
        s.close()
        plain_rate = pst[0] / (t1 - t0)
        out["fp64_plain"] = {"value": plain_rate, "sample": "cfg2, t 0 -> 4 dt_base",
                             "updates": pst[0]}
        out["speedup_batched_fp32_vs_plain_fp64"] = value / plain_rate
        # local-dt saving: cell updates of the same run with one global
        # quantised step (the smallest level of the set) over local steps
        pr_g = I.cfg2_turb(prec=I.F32)
        s = dsp.PatchSet.from_problem(pr_g, dt_mode=I.DT_GLOBAL_QUANT)
        s.advance_to(pr_g.t_end)
        upd_global = s.stats()[0]
        s.close()
        out["local_dt_saving"] = upd_global / res32["updates"]
        out["adjoint"] = run_adjoint()
        out["cfg3_fp32"] = run_cfg3(1, 1)
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
        # CPU baseline: the oracle on the host cores, bounded sample
        from oracle import oracle
        cores = len(os.sched_getaffinity(0))
        o = oracle.OracleSet.from_problem(pr)
        o.set_order(2, 1, cores)
        Tc = args.cpu_sample * pr.cfg.dt_base
        t0 = time.perf_counter()
        o.advance_to(Tc)
        t1 = time.perf_counter()
        ost = o.stats()
        o.close()
        # the same oracle on one thread, over the first 4 dt_base
        o1 = oracle.OracleSet.from_problem(pr)
        o1.set_order(2, 1, 1)
        t2 = time.perf_counter()
        o1.advance_to(4 * pr.cfg.dt_base)
        t3 = time.perf_counter()
        one = o1.stats()[0] / (t3 - t2)
        o1.close()
        model = ""
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
        rate = ost[0] / (t1 - t0)
        out["cpu_baseline"] = {"value": rate, "unit": "cell-updates/s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"cfg2 t 0 -> {args.cpu_sample} dt_base ({int(ost[0])} updates, "
                                         f"{t1 - t0:.1f} s)",
                               "per_core": rate / cores, "one_thread": one, "cpu_model": model}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
