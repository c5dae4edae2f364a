"""The C-shock of Sec. 5.4 on the GPU: a row of five patches between two
boundary patches (fixed upstream and downstream states), ambipolar or Ohmic
diffusion, local steps.  Parity with the oracle over 16 dt_base (schedule
bit-exact, FP64 state within 1e-10); boundary patches never change."""
import numpy as np
import pytest

from paper_1705_10774_amd import inputs as I
from tests.test_cshock import problem
from tests.test_gpu_parity import gpu_run, orc_run, rel_l1

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", ["ad_noniso", "ad_iso", "ohm"])
def test_cshock_parity(orc, case):
    pr = problem(case)
    T = 16 * pr.cfg.dt_base
    Ug, sg, kg, stg = gpu_run(pr, t_end=T)
    Uo, so, ko, sto = orc_run(orc, pr, t_end=T)
    assert np.array_equal(sg, so) and np.array_equal(kg, ko)
    assert sg[0] == sg[-1] == 0
    Vg, V0 = I.patch_views(Ug, pr.patches), I.patch_views(pr.U0, pr.patches)
    for m in (0, len(pr.patches) - 1):  # the boundary patches keep their state bitwise
        assert all(np.array_equal(a, b) for a, b in zip(Vg[m], V0[m]))
    err = rel_l1(Ug, Uo, pr.patches)
    print(case, "rel L1", err, "steps", sg.tolist())
    assert err <= 1e-10


def test_cshock_isothermal_steady_profile():
    """The isothermal ambipolar C-shock settles, within t = 1.5, into the
    steady structure: B_y along the row follows the semi-analytic profile
    (aligned at its mid-height) to 0.5% of the jump, spread over more than
    15 cells; the mass and momentum fluxes are uniform through it; the row
    ends in the table's upstream and downstream states."""
    from paper_1705_10774_amd import dsp
    from tests.test_cshock import TABLE, fluxes, steady_isothermal_cshock
    dsp.load()
    c = TABLE["ad_iso"]
    pr = problem("ad_iso")
    s = dsp.PatchSet.from_problem(pr)

    def profile():
        xs, W = [], []
        for q, v in zip(pr.patches[1:-1], I.patch_views(s.read_state(), pr.patches)[1:-1]):
            rho = v[0].mean(axis=(0, 1))
            mx, my, E = (v[m].mean(axis=(0, 1)) for m in (1, 2, 4))
            bx = 0.5 * (v[5][..., :-1] + v[5][..., 1:]).mean(axis=(0, 1))
            by = 0.5 * (v[6][:, :-1, :] + v[6][:, 1:, :]).mean(axis=(0, 1))
            vx, vy = mx / rho, my / rho
            p = (c["gamma"] - 1.0) * (E - 0.5 * rho * (vx ** 2 + vy ** 2) - 0.5 * (bx ** 2 + by ** 2))
            xs.append(I.cell_coords(q)[0])
            W.append(np.stack([rho, vx, vy, bx, by, p]))
        return np.concatenate(xs), np.concatenate(W, axis=1)

    s.advance_to(round(1.0 / pr.cfg.dt_base) * pr.cfg.dt_base)
    _, W1 = profile()
    s.advance_to(round(1.5 / pr.cfg.dt_base) * pr.cfg.dt_base)
    x, W = profile()
    s.close()
    print("change from t = 1 to 1.5", np.abs(W - W1).max())
    assert np.abs(W - W1).max() <= 2e-3
    # mass, x- and y-momentum fluxes (no non-ideal term) uniform through the shock
    f0 = fluxes(c["pre"], c["gamma"], True)[:3]
    f = np.stack([fluxes(W[:, m], c["gamma"], True)[:3] for m in range(W.shape[1])], axis=1)
    dev = np.abs(f - f0[:, None]).max(axis=1) / np.abs(f0)
    print("flux deviations", dev)
    assert np.all(dev <= 2e-3)
    # end states
    for w, ref in ((W[:, 0], c["pre"]), (W[:, -1], c["post"])):
        assert np.all(np.abs(w - np.array(ref)) <= 1e-3 * np.maximum(1.0, np.abs(ref)))
    # the structure against the semi-analytic steady profile
    xo, byo, _ = steady_isothermal_cshock()
    by0, by1 = c["pre"][4], c["post"][4]
    mid = 0.5 * (by0 + by1)
    by = W[4]

    def cross(xx, yy):
        i = int(np.argmax(yy > mid))
        return xx[i - 1] + (mid - yy[i - 1]) * (xx[i] - xx[i - 1]) / (yy[i] - yy[i - 1])

    pred = np.interp(x - (cross(x, by) - cross(xo, byo)), xo, byo, left=by0, right=byo[-1])
    err = np.abs(pred - by).max() / (by1 - by0)
    width = int((np.abs(np.diff(by)) > 0.01 * (by1 - by0)).sum())
    print("C-shock profile error", err, "cells across", width)
    assert err <= 5e-3
    assert width > 15
