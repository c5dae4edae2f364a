"""The persistent dispatcher (DSP_DISPATCH_QUEUE: one persistent kernel fed
by a device ready queue, launched as a captured hipGraph) against the
rounds (DSP_DISPATCH_ROUNDS) and against the oracle.  With g = 0 the result
does not depend on the order of the updates, so the two modes must agree
bit for bit; the autotuner must leave the set's state as it found it."""
import dataclasses
import os

import numpy as np
import pytest

from paper_1705_10774_amd import inputs as I
from tests.test_gpu_parity import elem_rel, orc_run, rel_l1

pytestmark = pytest.mark.gpu


def _dsp():
    from paper_1705_10774_amd import dsp
    dsp.load()
    return dsp


def _run(pr, mode, t_end=None, workers=0):
    dsp = _dsp()
    s = dsp.PatchSet.from_problem(pr)
    s.set_dispatch(mode, workers)
    s.advance_to(pr.t_end if t_end is None else t_end)
    U = s.read_state()
    st, kh, kl = s.read_schedule(klog_cap=64)
    stats = s.stats()
    ks = s.kernel_stats()
    s.close()
    return U, st, kh, kl, stats, ks


def _spread(n=16):
    return I.turbulence(npd=3, n=n, mach=5.0, seed=5, dt_base=0.02 / 32, prec=I.F32)


def test_queue_available_and_default():
    dsp = _dsp()
    s = dsp.PatchSet.from_problem(_spread())
    mode, avail, workers = s.dispatch()
    s.close()
    assert avail and workers >= 1
    assert mode == (dsp.DSP_DISPATCH_ROUNDS if os.environ.get("DSP_DISPATCH") == "rounds" else dsp.DSP_DISPATCH_QUEUE)
    # not available: double precision
    s = dsp.PatchSet.from_problem(_spread(), prec=I.F64)
    assert not s.dispatch()[1]
    with pytest.raises(dsp.DspError):
        s.set_dispatch(dsp.DSP_DISPATCH_QUEUE)
    s.close()
    # patches of more than one tile: available, but new sets start in the rounds
    s = dsp.PatchSet.from_problem(_mini(I.F32))
    mode, avail, workers = s.dispatch()
    s.close()
    assert avail and mode == dsp.DSP_DISPATCH_ROUNDS


@pytest.mark.parametrize("n", [8, 16])
def test_queue_equals_rounds_bitwise(orc, n):
    dsp = _dsp()
    pr = _spread(n)
    T = 8 * pr.cfg.dt_base
    a = _run(pr, dsp.DSP_DISPATCH_ROUNDS, T)
    b = _run(pr, dsp.DSP_DISPATCH_QUEUE, T)
    assert len(set(a[1].tolist())) > 1  # genuinely local steps
    for x, y in zip(a[:4], b[:4]):
        assert np.array_equal(x, y)
    assert a[4][0] == b[4][0] and a[4][10] == b[4][10] and a[4][11] == b[4][11]
    assert b[5][1] == 1 and b[5][0] > 0 and b[5][2] > 0  # one persistent launch, timed, bytes counted
    Uo, so, ko, _ = orc_run(orc, pr, t_end=T, prec=I.F64)
    assert np.array_equal(b[1], so) and np.array_equal(b[2], ko)
    assert rel_l1(b[0], Uo, pr.patches) <= 1e-4


@pytest.mark.parametrize("workers", [1, 7, 64])
def test_queue_any_worker_count(workers):
    dsp = _dsp()
    pr = _spread(8)
    T = 4 * pr.cfg.dt_base
    a = _run(pr, dsp.DSP_DISPATCH_ROUNDS, T)
    b = _run(pr, dsp.DSP_DISPATCH_QUEUE, T, workers=workers)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_queue_resolution_jumps_bitwise(orc):
    """Patches of 8^3 and 16^3 (the worker resamples its guard regions)."""
    dsp = _dsp()
    pr = I.uneven(npd=4, seed_sizes=1013, seed_rho=2013, prec=I.F32, box=0.25, name="mini816",
                  dt_base=2.0 ** -11, sizes=(8, 16))
    T = 2 * pr.cfg.dt_base
    a = _run(pr, dsp.DSP_DISPATCH_ROUNDS, T)
    b = _run(pr, dsp.DSP_DISPATCH_QUEUE, T)
    assert len(set(a[1].tolist())) >= 3
    for x, y in zip(a[:4], b[:4]):
        assert np.array_equal(x, y)
    Uo, so, ko, _ = orc_run(orc, pr, t_end=T, prec=I.F64)
    assert np.array_equal(b[1], so) and np.array_equal(b[2], ko)
    assert rel_l1(b[0], Uo, pr.patches) <= 1e-4


def _mini(prec):
    # configuration 3 in small: 4^3 patches of n in {16, 24, 32}
    return I.uneven(npd=4, seed_sizes=1013, seed_rho=2013, prec=prec, box=0.25, name="cfg3_mini",
                    dt_base=2.0 ** -11)


@pytest.mark.parametrize("workers", [0, 7])
def test_queue_multi_tile_bitwise(orc, workers):
    """Patches of 24^3 and 32^3 (four tiles each, run one after another by
    the worker, the first with the Courant level of the whole patch) beside
    16^3 ones, with resampled guard regions: the queue gives the rounds'
    bits, and the oracle's schedule (one worker per CU, and 7 workers)."""
    dsp = _dsp()
    pr = _mini(I.F32)
    T = 2 * pr.cfg.dt_base
    a = _run(pr, dsp.DSP_DISPATCH_ROUNDS, T)
    b = _run(pr, dsp.DSP_DISPATCH_QUEUE, T, workers=workers)
    assert len(set(a[1].tolist())) >= 3
    for x, y in zip(a[:4], b[:4]):
        assert np.array_equal(x, y)
    assert a[4][0] == b[4][0] and a[4][10] == b[4][10] and a[4][11] == b[4][11]
    assert b[5][1] == 1  # one persistent launch
    Uo, so, ko, _ = orc_run(orc, pr, t_end=T, prec=I.F64)
    assert np.array_equal(b[1], so) and np.array_equal(b[2], ko)
    assert rel_l1(b[0], Uo, pr.patches) <= 1e-4


def test_queue_cfg2_full_run_bitwise():
    """Configuration 2 (512 patches of 16^3) over its whole run: the queue
    and the rounds agree bit for bit."""
    dsp = _dsp()
    pr = I.cfg2_turb(prec=I.F32)
    a = _run(pr, dsp.DSP_DISPATCH_ROUNDS)
    b = _run(pr, dsp.DSP_DISPATCH_QUEUE)
    for x, y in zip(a[:4], b[:4]):
        assert np.array_equal(x, y)
    print("rounds ms", a[4][12], "queue ms", b[4][12])


def test_queue_advance_in_pieces_and_to_current_time():
    dsp = _dsp()
    pr = _spread(8)
    dtb = pr.cfg.dt_base
    s = dsp.PatchSet.from_problem(pr)
    s.set_dispatch(dsp.DSP_DISPATCH_QUEUE)
    for m in (1, 1, 3, 5):  # the second call advances to the current time: nothing to do
        s.advance_to(m * dtb)
    U = s.read_state()
    st = s.read_schedule()
    s.close()
    a = _run(pr, dsp.DSP_DISPATCH_ROUNDS, 5 * dtb)
    assert np.array_equal(U, a[0]) and np.array_equal(st[0], a[1]) and np.array_equal(st[1], a[2])


def test_autotune_restores_state_and_selects(tmp_path):
    dsp = _dsp()
    pr = _spread(16)
    dtb = pr.cfg.dt_base
    s = dsp.PatchSet.from_problem(pr)
    s.advance_to(dtb)
    cache = tmp_path / "tune.jsonl"
    ms = s.autotune(2 * dtb, cache)
    assert ms[0] > 0 and ms[1] > 0  # rounds and the queue were timed
    mode, _, workers = s.dispatch()
    s.advance_to(3 * dtb)
    U = s.read_state()
    st, kh = s.read_schedule()
    s.close()
    ref = _run(pr, dsp.DSP_DISPATCH_ROUNDS, 3 * dtb)
    assert np.array_equal(U, ref[0]) and np.array_equal(st, ref[1]) and np.array_equal(kh, ref[2])
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and '"dispatch": %d' % mode in lines[0]
    # the cached choice is taken without timing
    s = dsp.PatchSet.from_problem(pr)
    ms2 = s.autotune(2 * dtb, cache)
    assert np.all(ms2 == -1) and s.dispatch()[0] == mode
    s.close()
    print("autotune ms", ms, "chosen", mode, workers)


@pytest.mark.parametrize("cap", [1, 5])
def test_capped_rounds_equal_whole_rounds(cap, monkeypatch):
    """Rounds that take at most `cap` ready patches (the rest wait for the
    next round; large sets are capped this way) give the same bits as whole
    rounds, in FP64 and with a resolution jump."""
    dsp = _dsp()
    outs = []
    for env in (None, str(cap)):
        if env is None:
            monkeypatch.delenv("DSP_ROUND_CAP", raising=False)
        else:
            monkeypatch.setenv("DSP_ROUND_CAP", env)
        for pr in (_spread(), I.uneven(npd=4, seed_sizes=1013, seed_rho=2013, prec=I.F64, box=0.25, name="m",
                                       dt_base=2.0 ** -11)):
            s = dsp.PatchSet.from_problem(pr, prec=I.F64)
            s.advance_to(4 * pr.cfg.dt_base)
            outs.append((s.read_state(), *s.read_schedule(), s.stats()[13]))
            s.close()
    for a, b in zip(outs[:2], outs[2:]):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    assert outs[2][3] > outs[0][3]  # the capped run took more rounds
