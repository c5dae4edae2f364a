"""Edge sizes of the GPU path against the oracle (schedule bit-exact, FP64
state within 1e-10, FP32 within 1e-4): a single periodic patch (its own
neighbour on every side), the smallest patches (n = 4), tiles that do not
divide the patch (n = 20: 2 x 2 tiles of 10; n = 40: 3 x 3 tiles of 13 or 14),
the largest patch (n = 64: 4 x 4 tiles), and an advance to the current time
(nothing to do)."""
import numpy as np
import pytest

from paper_1705_10774_amd import inputs as I
from tests.test_gpu_parity import gpu_run, orc_run, rel_l1

pytestmark = pytest.mark.gpu


def turb(npd, n, prec=I.F64, mach=2.0):
    return I.turbulence(npd=npd, n=n, mach=mach, seed=11, dt_base=0.02 / 32, prec=prec)


@pytest.mark.parametrize("npd,n,prec", [(1, 16, I.F64), (2, 4, I.F64), (1, 20, I.F64), (1, 40, I.F64),
                                        (1, 40, I.F32), (1, 64, I.F32)],
                         ids=["single-16", "smallest-4", "ragged-20", "ragged-40", "ragged-40-f32", "largest-64-f32"])
def test_edge_sizes(orc, npd, n, prec):
    pr = turb(npd, n, prec)
    T = 2 * pr.cfg.dt_base
    Ug, sg, kg, stg = gpu_run(pr, t_end=T)
    Uo, so, ko, sto = orc_run(orc, pr, t_end=T)
    print("steps", sg.tolist(), "rounds", stg[13])
    assert np.array_equal(sg, so) and np.array_equal(kg, ko)
    assert rel_l1(Ug, Uo, pr.patches) <= (1e-10 if prec == I.F64 else 1e-4)


def test_advance_to_current_time_is_a_no_op():
    from paper_1705_10774_amd import dsp
    dsp.load()
    pr = turb(2, 8)
    s = dsp.PatchSet.from_problem(pr)
    s.advance_to(pr.cfg.dt_base)
    U1 = s.read_state()
    st1, kh1 = s.read_schedule()
    s.advance_to(pr.cfg.dt_base)
    s.advance_to(0.0)  # already past: nothing is ready, nothing runs
    assert np.array_equal(s.read_state(), U1)
    st2, kh2 = s.read_schedule()
    assert np.array_equal(st1, st2) and np.array_equal(kh1, kh2)
    s.close()


@pytest.mark.parametrize("npd", [1, 2], ids=["single-patch", "equal-patches"])
def test_create_leaves_no_hip_error(npd):
    """Creating a set with no resampling plan and (one patch) no neighbour
    list leaves no pending HIP error for the caller's next call."""
    import torch
    from paper_1705_10774_amd import dsp
    dsp.load()
    s = dsp.PatchSet.from_problem(turb(npd, 8))
    x = torch.ones(4, device="cuda") * 2.0
    torch.cuda.synchronize()
    assert float(x.sum()) == 8.0
    s.close()


def test_torch_caching_allocator():
    """A set whose device memory comes from torch's caching allocator (the
    allocator hook of dsp_create): its memory shows in torch's statistics
    while it lives and goes back when it is closed, and it runs bit for bit
    as a set on hipMalloc memory."""
    import torch
    from paper_1705_10774_amd import dsp
    dsp.load()
    pr = turb(2, 8)
    T = 2 * pr.cfg.dt_base
    torch.cuda.synchronize()
    m0 = torch.cuda.memory_allocated()
    s = dsp.PatchSet.from_problem(pr, allocator="torch")
    assert torch.cuda.memory_allocated() - m0 >= 3 * s.nvals * 8  # the three FP64 ring slots at least
    s.advance_to(T)
    Ua = s.read_state()
    s.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == m0
    s = dsp.PatchSet.from_problem(pr)
    s.advance_to(T)
    Ub = s.read_state()
    s.close()
    assert np.array_equal(Ua, Ub)
