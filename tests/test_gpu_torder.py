"""GPU parity of the quadratic guard time interpolation (time order 2: three
slices, Lagrange weights; Sec. 3B) against the oracle, in the batched rounds
and in the plain oldest-first path, on the local-step spread, resolution
jumps and the mixed-level row with a grace (quadratic extrapolation).  Bars as
for linear interpolation: schedule bit-exact, FP64 state within 1e-10 and
FP32 within 1e-4 (relative L1)."""
import numpy as np
import pytest

from paper_1705_10774_amd import inputs as I
from tests.test_gpu_grace import orc_run
from tests.test_gpu_parity import gpu_run, mini_uneven, rel_l1, spread

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [I.F64, I.F32], ids=["f64", "f32"])
def test_order2_spread_rounds(orc, prec):
    pr = spread(8)
    over = dict(torder=2, nslots=4, prec=prec)
    T = 4 * pr.cfg.dt_base
    Ug, sg, kg, stg = gpu_run(pr, t_end=T, **over)
    Uo, so, ko, sto, _ = orc_run(orc, pr, T, **over)
    U1, _, _, _, _ = orc_run(orc, pr, T, nslots=4)
    print("change from linear interpolation", np.abs(Uo - U1).max())
    assert np.abs(Uo - U1).max() > 0
    assert np.array_equal(sg, so) and np.array_equal(kg, ko)
    assert rel_l1(Ug, Uo, pr.patches) <= (1e-10 if prec == I.F64 else 1e-4)


def test_order2_plain_oldest_first(orc):
    pr = spread(8)
    over = dict(torder=2, nslots=4)
    T = 4 * pr.cfg.dt_base
    Ug, sg, kg, stg = gpu_run(pr, t_end=T, plain=True, **over)
    Uo, so, ko, sto, _ = orc_run(orc, pr, T, order=0, **over)
    assert np.array_equal(sg, so) and np.array_equal(kg, ko)
    assert rel_l1(Ug, Uo, pr.patches) <= 1e-10


def test_order2_cross_resolution(orc):
    pr = mini_uneven(I.F64)
    over = dict(torder=2, nslots=4)
    T = 2 * pr.cfg.dt_base
    Ug, sg, kg, stg = gpu_run(pr, t_end=T, **over)
    Uo, so, ko, sto, _ = orc_run(orc, pr, T, **over)
    assert np.array_equal(sg, so) and np.array_equal(kg, ko)
    assert rel_l1(Ug, Uo, pr.patches) <= 1e-10


def test_order2_grace_extrapolation(orc):
    pr = I.level_row(grace=0.75, nslots=5)
    T = 4 * pr.cfg.dt_base
    Ug, sg, kg, stg = gpu_run(pr, t_end=T, torder=2)
    Uo, so, ko, sto, ne = orc_run(orc, pr, T, torder=2)
    assert ne > 0
    assert np.array_equal(sg, so) and np.array_equal(kg, ko)
    assert rel_l1(Ug, Uo, pr.patches) <= 1e-10
