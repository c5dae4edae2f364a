"""Configuration 3 at full size (4096 patches of 16^3, 24^3 or 32^3, lognormal
density, levels 0..7) over the first dt_base and over its whole run, checked
by properties that hold
at any size (the oracle runs its reduced version, 4^3 patches, in
test_gpu_parity.py):
* every patch ends exactly at dt_base (and at the end of the run), through
  steps dt_base 2^-k that keep its time a multiple of the step (the level
  log, summed in ticks);
* the levels span the range of the signal speeds;
* div B stays at rounding (constrained transport);
* the FP32 run follows the FP64 run: the same schedule, and states within
  the FP32 bar (relative L1 1e-4)."""
import numpy as np
import pytest

from paper_1705_10774_amd import inputs as I
from tests.test_gpu_parity import rel_l1

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cfg3_runs():
    from paper_1705_10774_amd import dsp
    dsp.load()
    pr = I.cfg3_uneven(prec=I.F64)
    print("cfg3: patches", len(pr.patches), "cells", pr.cells, flush=True)
    T = pr.cfg.dt_base
    out = {}
    for prec in (I.F64, I.F32):
        s = dsp.PatchSet.from_problem(pr, prec=prec)
        s.advance_to(T)
        U = s.read_state()
        steps, kh, kl = s.read_schedule(klog_cap=256)
        st = s.stats()
        s.close()
        out[prec] = (U, steps, kh, kl, st)
        print("cfg3", "f64" if prec == I.F64 else "f32", "updates", st[0], "rounds", st[13], "div B", st[9],
              flush=True)
    return pr, T, out


def test_cfg3_full_size_schedule(cfg3_runs):
    pr, T, out = cfg3_runs
    U, steps, kh, kl, st = out[I.F64]
    kmax = pr.cfg.kmax
    Tt = int(round(T / pr.cfg.dt_base)) << kmax
    assert st[14] == st[15] == T
    levels = set()
    for p in range(len(pr.patches)):
        t = 0
        for k in kl[p, :steps[p]]:
            dt = 1 << (kmax - int(k))
            assert t % dt == 0
            t += dt
            levels.add(int(k))
        assert t == Tt
    print("levels", sorted(levels))
    assert min(levels) <= 1 and max(levels) >= 5


@pytest.mark.parametrize("prec", [I.F64, I.F32], ids=["f64", "f32"])
def test_cfg3_full_size_divergence_free(cfg3_runs, prec):
    pr, T, out = cfg3_runs
    st = out[prec][4]
    # |B| = 0.14 on cells down to dx = 1/512: rounding of the face differences
    assert st[9] <= (1e-9 if prec == I.F64 else 1e-2)


def test_cfg3_full_size_fp32_follows_fp64(cfg3_runs):
    pr, T, out = cfg3_runs
    U64, s64, k64, _, _ = out[I.F64]
    U32, s32, k32, _, _ = out[I.F32]
    assert np.array_equal(s64, s32) and np.array_equal(k64, k32)
    assert rel_l1(U32, U64, pr.patches) <= 1e-4


def test_cfg3_whole_run_properties():
    """The whole run (8 dt_base, the benchmark's workload): every patch lands
    on t_end through aligned steps in both precisions, div B stays at
    rounding, and the FP32 schedule is reported against the FP64 one (a
    level can flip at a near-tie of the Courant rate; the count is printed
    and bounded)."""
    from paper_1705_10774_amd import dsp
    dsp.load()
    pr = I.cfg3_uneven(prec=I.F64)
    T = pr.t_end
    kmax = pr.cfg.kmax
    Tt = int(round(T / pr.cfg.dt_base)) << kmax
    res = {}
    for prec in (I.F64, I.F32):
        s = dsp.PatchSet.from_problem(pr, prec=prec)
        s.advance_to(T)
        steps, kh, kl = s.read_schedule(klog_cap=256)  # the set logs the first 256 levels of each patch
        st = s.stats()
        U = s.read_state()
        s.close()
        assert st[14] == st[15] == T  # every patch at t_end
        for p in range(len(pr.patches)):
            m = min(int(steps[p]), 256)
            dts = np.left_shift(np.int64(1), kmax - kl[p, :m].astype(np.int64))
            ends = np.cumsum(dts)
            assert ((ends - dts) % dts == 0).all()  # aligned steps over the logged part
            if steps[p] <= 256:
                assert ends[-1] == Tt
        assert st[9] <= (1e-9 if prec == I.F64 else 1e-2)
        res[prec] = (steps, kh, st, U)
        print("cfg3 whole run", "f64" if prec == I.F64 else "f32", "updates", st[0], "rounds", st[13],
              "div B", st[9], flush=True)
    flips = int((res[I.F64][1] != res[I.F32][1]).sum())
    print("cfg3 whole run: patches whose FP32 level sequence differs from FP64:", flips)
    assert flips <= len(pr.patches) // 100
    # the FP32 state against the FP64 one (the oracle cannot hold this set);
    # measured 6.1e-5
    err = rel_l1(res[I.F32][3], res[I.F64][3], pr.patches)
    print("cfg3 whole run: FP32 against FP64, relative L1", err)
    assert err <= 1e-4
