"""Wrong-slot guard reads: with DSP_POISON=1 every ring slot but the initial
one holds NaN from the start, so a guard value read from a slot that was
never written makes the state non-finite (DSP_ENONFINITE) at once.  Runs
that exercise the slot rules (local steps with a level spread, resolution
jumps, three nested levels, quadratic time interpolation with more slots,
a grace) must finish and equal the unpoisoned run bit for bit."""
import os

import numpy as np
import pytest

from paper_1705_10774_amd import inputs as I

pytestmark = pytest.mark.gpu


def _dsp():
    from paper_1705_10774_amd import dsp
    dsp.load()
    return dsp


def _run(pr, T, poison, **over):
    dsp = _dsp()
    old = os.environ.get("DSP_POISON")
    os.environ["DSP_POISON"] = "1" if poison else "0"
    try:
        s = dsp.PatchSet.from_problem(pr, **over)
    finally:
        if old is None:
            del os.environ["DSP_POISON"]
        else:
            os.environ["DSP_POISON"] = old
    s.advance_to(T)
    U = s.read_state()
    st, kh = s.read_schedule()
    s.close()
    return U, st, kh


CASES = {
    "spread": (lambda: I.turbulence(npd=3, n=8, mach=5.0, seed=5, dt_base=0.02 / 32), 6, {}),
    "jumps": (lambda: I.uneven(npd=4, seed_sizes=1013, seed_rho=2013, prec=I.F64, box=0.25, name="m",
                               dt_base=2.0 ** -11), 2, {}),
    "smr": (lambda: I.cfg4_smr(n=8), 1, {}),
    "torder2": (lambda: I.turbulence(npd=3, n=8, mach=5.0, seed=5, dt_base=0.02 / 32), 4,
                {"torder": 2, "nslots": 4}),
    "grace": (lambda: I.level_row(), 2, {"grace": 0.5}),
}


@pytest.mark.parametrize("prec", [I.F64, I.F32], ids=["f64", "f32"])
@pytest.mark.parametrize("case", list(CASES))
def test_no_read_of_unwritten_slots(case, prec):
    make, nbase, over = CASES[case]
    pr = make()
    T = nbase * pr.cfg.dt_base
    a = _run(pr, T, True, prec=prec, **over)
    b = _run(pr, T, False, prec=prec, **over)
    assert np.isfinite(a[0]).all()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def _snapshot_slots(path, patches):
    """Ring slot values per patch, [nslots][V], from a snapshot file (the
    record layout dsp_save_snapshot documents)."""
    b = open(path, "rb").read()
    assert b[:8] == b"DSPSNAP1"
    npatch, ns, prec, kmax, klog_cap = np.frombuffer(b, np.int32, 5, 8)
    dt = np.float32 if prec == 1 else np.float64
    off = 8 + 20 + 8
    out = []
    for q in patches:
        off += 8 + 8 + 8 + 4 + 8 + 8 + ns * 17 + klog_cap
        V = 5 * q.n ** 3 + 3 * q.n * q.n * (q.n + 1)
        out.append(np.frombuffer(b, dt, V * ns, off).reshape(ns, V))
        off += V * ns * np.dtype(dt).itemsize
    assert off == len(b)
    return out


@pytest.mark.parametrize("prec", [I.F64, I.F32], ids=["f64", "f32"])
def test_poison_is_applied(prec, tmp_path):
    """The switch works: right after init every slot but slot 0 is NaN, and
    slot 0 holds the initial state (without the switch the other slots hold
    whatever the allocation held)."""
    dsp = _dsp()
    pr = I.turbulence(npd=2, n=8, mach=5.0, seed=5, dt_base=0.02 / 32)
    os.environ["DSP_POISON"] = "1"
    try:
        s = dsp.PatchSet.from_problem(pr, prec=prec)
    finally:
        del os.environ["DSP_POISON"]
    path = str(tmp_path / "poisoned.snap")
    s.save(path)
    s.close()
    for sl in _snapshot_slots(path, pr.patches):
        assert np.isfinite(sl[0]).all()
        assert np.isnan(sl[1:]).all()
