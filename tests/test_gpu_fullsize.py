"""Configuration 3 at full size (4096 patches of 16^3, 24^3 or 32^3, lognormal
density, levels 0..6) over the first dt_base, checked by properties that hold
at any size (the oracle runs its reduced version, 4^3 patches, in
test_gpu_parity.py):
* every patch ends exactly at dt_base, through steps dt_base 2^-k that keep
  its time a multiple of the step (the level log, summed in ticks);
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
