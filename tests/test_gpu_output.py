"""Output cadence (Sec. 3E): every patch writes its new slice into the frame
of an output time when it reaches that time, on its own.  The frames are
checked against the oracle's state at the same times (element by element,
FP64 within 1e-10; FP32 within 1e-4 relative L1), against runs of the GPU
path stopped at those times (bit for bit, both dispatch modes: with g = 0 the
result does not depend on where a run stops), and for the frame ring and the
argument checks."""
import numpy as np
import pytest

from paper_1705_10774_amd import inputs as I
from tests.test_gpu_parity import elem_rel, rel_l1, spread

pytestmark = pytest.mark.gpu


def _dsp():
    from paper_1705_10774_amd import dsp
    dsp.load()
    return dsp


def _frames_run(pr, out_dt, nframes, T, dispatch=None, **over):
    dsp = _dsp()
    s = dsp.PatchSet.from_problem(pr, **over)
    if dispatch is not None:
        s.set_dispatch(dispatch)
    frames = s.set_output(out_dt, nframes)
    s.advance_to(T)
    F = frames.double().cpu().numpy()
    U = s.read_state()
    s.close()
    return F, U


def _with_prec(pr, prec):
    import dataclasses
    pr.cfg = dataclasses.replace(pr.cfg, prec=prec)
    return pr


CASES = {"spread": lambda prec: _with_prec(spread(8), prec),
         "smr": lambda prec: I.cfg4_smr(n=8, prec=prec)}


@pytest.mark.parametrize("case", ["spread", "smr"])
def test_frames_match_oracle_fp64(orc, case):
    pr = CASES[case](I.F64)
    db = pr.cfg.dt_base
    nout = 4 if case == "spread" else 2
    out_dt = 2 * db if case == "spread" else db
    T = nout * out_dt
    F, U = _frames_run(pr, out_dt, nout, T)
    o = orc.OracleSet.from_problem(pr)
    for f in range(nout):
        o.advance_to((f + 1) * out_dt)
        Uo = o.read_state()
        e = elem_rel(F[f], Uo, pr.patches)
        print(case, "frame", f, "element-wise", e)
        assert e <= 1e-10
    o.close()
    assert np.array_equal(F[nout - 1], U)  # the last frame is the final state


def test_frames_match_oracle_fp32(orc):
    pr = CASES["spread"](I.F32)
    db = pr.cfg.dt_base
    F, U = _frames_run(pr, 2 * db, 2, 4 * db)
    o = orc.OracleSet.from_problem(pr, prec=I.F64)
    for f in range(2):
        o.advance_to((f + 1) * 2 * db)
        assert rel_l1(F[f], o.read_state(), pr.patches) <= 1e-4
    o.close()


@pytest.mark.parametrize("mode", ["rounds", "queue"])
def test_frames_equal_stopped_runs(mode):
    """FP32 (the queue is available): each frame equals, bit for bit, the
    state of a run stopped at its time."""
    dsp = _dsp()
    pr = CASES["spread"](I.F32)
    db = pr.cfg.dt_base
    m = dsp.DSP_DISPATCH_ROUNDS if mode == "rounds" else dsp.DSP_DISPATCH_QUEUE
    F, _ = _frames_run(pr, 2 * db, 3, 6 * db, dispatch=m)
    for f in range(3):
        s = dsp.PatchSet.from_problem(pr)
        s.set_dispatch(dsp.DSP_DISPATCH_ROUNDS)
        s.advance_to((f + 1) * 2 * db)
        Us = s.read_state()
        s.close()
        assert np.array_equal(F[f], Us), f


def test_frame_ring_wraps_and_off():
    dsp = _dsp()
    pr = spread(8)
    db = pr.cfg.dt_base
    F, _ = _frames_run(pr, db, 2, 4 * db)  # outputs at 1..4 dt_base into frames 0, 1, 0, 1
    G, _ = _frames_run(pr, db, 4, 4 * db)
    assert np.array_equal(F[0], G[2]) and np.array_equal(F[1], G[3])
    # turned off: the frames keep what they held
    s = dsp.PatchSet.from_problem(pr)
    frames = s.set_output(db, 1)
    s.set_output(db, 0)
    s.advance_to(2 * db)
    assert np.isnan(frames.cpu().numpy()).all()
    s.close()


def test_output_rejects_bad_arguments():
    import torch
    dsp = _dsp()
    pr = spread(8)
    s = dsp.PatchSet.from_problem(pr)
    buf = torch.zeros((1, s.nvals), dtype=torch.float64, device="cuda")
    for dt in (0.0, -pr.cfg.dt_base, 1.5 * pr.cfg.dt_base):
        with pytest.raises(dsp.DspError) as e:
            dsp.dsp_set_output(s.h, dt, buf.data_ptr(), 1)
        assert e.value.code == dsp.DSP_EINVAL
    s.close()
    g = dsp.PatchSet.from_problem(I.uniform(npd=2, n=8, mode=I.DT_GLOBAL_EXACT, dt_base=1.0 / 64))
    with pytest.raises(dsp.DspError):
        dsp.dsp_set_output(g.h, 1.0 / 64, buf.data_ptr(), 1)
    g.close()
