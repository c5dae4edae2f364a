"""GPU parity with a grace g > 0 in Eq. (1).  A patch may then run ahead of a
coarser neighbour and extrapolate it in time, and the result depends on the
order of execution.  Each GPU path is compared with the oracle run in the
same order: the batched rounds (the whole ready set at once) with the
oracle's rounds, the plain path (oldest ready patch first, ties by id) with
its oldest-first order.  Bars as for g = 0: schedule bit-exact, FP64 state
within 1e-10 and FP32 within 1e-4 (relative L1).

When every ready patch updates at once, a patch gets ahead of a coarser
neighbour only where that neighbour waits for a still finer one: the row of
levels (0, 0, 1, 0, 2) has such places; the 3-D local-step spread and the
resolution jumps run the same schedule as with g = 0."""
import os

import numpy as np
import pytest

from paper_1705_10774_amd import inputs as I
from tests.test_gpu_parity import gpu_run, mini_uneven, rel_l1, rel_l1_grouped, spread

pytestmark = pytest.mark.gpu
NT = max(1, min(16, len(os.sched_getaffinity(0))))


def orc_run(orc, prob, t_end, order=2, **over):
    s = orc.OracleSet.from_problem(prob, **over)
    s.set_order(order, 1, NT if order == 2 else 1)
    s.advance_to(t_end)
    U = s.read_state()
    steps, kh = s.read_schedule()
    st = s.stats()
    ne = s.extrapolated()
    s.close()
    return U, steps, kh, st, ne


@pytest.mark.parametrize("prec", [I.F64, I.F32], ids=["f64", "f32"])
def test_grace_level_row_extrapolates(orc, prec):
    # FP32 resolves a wave of amplitude A to about 1e-7 / A relative: A = 0.05
    pr = I.level_row(prec=prec, grace=0.75, amp=1e-3 if prec == I.F64 else 0.05)
    T = 4 * pr.cfg.dt_base
    Ug, sg, kg, stg = gpu_run(pr, t_end=T)
    Uo, so, ko, sto, ne = orc_run(orc, pr, T)
    U0, s0, k0, st0, _ = orc_run(orc, pr, T, grace=0.0)
    print("rounds: gpu", stg[13], "oracle", sto[13], "extrapolated updates", ne,
          "change from g = 0", np.abs(Uo - U0).max())
    assert ne > 0
    assert np.abs(Uo - U0).max() > 0  # the grace changed the result
    assert np.array_equal(sg, so) and np.array_equal(kg, ko)
    assert stg[13] == sto[13]
    assert rel_l1(Ug, Uo, pr.patches) <= (1e-10 if prec == I.F64 else 1e-4)


@pytest.mark.parametrize("prec", [I.F64, I.F32], ids=["f64", "f32"])
def test_grace_spread_rounds(orc, prec):
    pr = spread(8)
    over = dict(grace=0.75, nslots=4, prec=prec)
    T = 4 * pr.cfg.dt_base
    Ug, sg, kg, stg = gpu_run(pr, t_end=T, **over)
    Uo, so, ko, sto, ne = orc_run(orc, pr, T, **over)
    print("rounds: gpu", stg[13], "oracle", sto[13], "extrapolated", ne)
    assert np.array_equal(sg, so) and np.array_equal(kg, ko)
    assert stg[13] == sto[13]
    assert rel_l1(Ug, Uo, pr.patches) <= (1e-10 if prec == I.F64 else 1e-4)


def test_grace_plain_oldest_first(orc):
    pr = spread(8)
    over = dict(grace=0.75, nslots=4)
    T = 4 * pr.cfg.dt_base
    Ug, sg, kg, stg = gpu_run(pr, t_end=T, plain=True, **over)
    Uo, so, ko, sto, ne = orc_run(orc, pr, T, order=0, **over)
    assert np.array_equal(sg, so) and np.array_equal(kg, ko)
    assert rel_l1(Ug, Uo, pr.patches) <= 1e-10


def test_grace_cross_resolution(orc):
    pr = mini_uneven(I.F64)
    over = dict(grace=0.5, nslots=5)
    T = 2 * pr.cfg.dt_base
    Ug, sg, kg, stg = gpu_run(pr, t_end=T, **over)
    Uo, so, ko, sto, ne = orc_run(orc, pr, T, **over)
    assert np.array_equal(sg, so) and np.array_equal(kg, ko)
    assert rel_l1(Ug, Uo, pr.patches) <= 1e-10


def test_grace_smr_blast(orc):
    pr = I.cfg4_smr()
    over = dict(grace=0.5, nslots=5)
    T = pr.cfg.dt_base
    Ug, sg, kg, stg = gpu_run(pr, t_end=T, **over)
    Uo, so, ko, sto, ne = orc_run(orc, pr, T, **over)
    assert np.array_equal(sg, so) and np.array_equal(kg, ko)
    assert rel_l1_grouped(Ug, Uo, pr.patches) <= 1e-10


def test_grace_with_three_slots(orc):
    """nslots = 3 with a grace: the free-slot rule keeps every needed slice."""
    pr = I.level_row(grace=0.75, nslots=3)
    T = 4 * pr.cfg.dt_base
    Ug, sg, kg, stg = gpu_run(pr, t_end=T)
    Uo, so, ko, sto, ne = orc_run(orc, pr, T)
    assert np.array_equal(sg, so) and np.array_equal(kg, ko)
    assert rel_l1(Ug, Uo, pr.patches) <= 1e-10
