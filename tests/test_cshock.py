"""The non-ideal C-shock of Sec. 5.4: the table of upstream and downstream
states (tests/golden/cshock_table.json, transcribed from the paper) and runs
of the oracle on a row of five patches between two boundary patches."""
import json
import math
import os

import numpy as np
import pytest

from paper_1705_10774_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = json.load(open(os.path.join(HERE, "golden", "cshock_table.json")))
CASES = ["ad_iso", "ad_noniso", "ohm"]


def fluxes(w, gamma, isothermal):
    """Shock-frame fluxes along x of a uniform state (rho, vx, vy, Bx, By, P)
    with B_z = v_z = 0: mass, x- and y-momentum, E_z = vx By - vy Bx, and
    (adiabatic) energy."""
    rho, vx, vy, bx, by, p = w
    out = [rho * vx, rho * vx * vx + p + 0.5 * (bx * bx + by * by) - bx * bx, rho * vx * vy - bx * by,
           vx * by - vy * bx]
    if not isothermal:
        e = p / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy) + 0.5 * (bx * bx + by * by)
        out.append((e + p + 0.5 * (bx * bx + by * by)) * vx - bx * (vx * bx + vy * by))
    return np.array(out)


@pytest.mark.parametrize("case", CASES)
def test_table_states_satisfy_jump_conditions(case):
    """The two states of each row of the table carry the same fluxes (the
    non-ideal terms vanish in uniform states).  The table prints 4-5 digits,
    and its adiabatic ambipolar row matches to 5e-4 of the flux (the
    y-momentum flux), so the bar is 1e-3; a transcription slip in a leading
    digit breaks it.  The isothermal row keeps P / rho, the sound speed
    squared."""
    c = TABLE[case]
    iso = case == "ad_iso"
    fa = fluxes(c["pre"], c["gamma"], iso)
    fb = fluxes(c["post"], c["gamma"], iso)
    scale = np.maximum(np.abs(fa), 1.0)
    print(case, "relative flux jumps", (fb - fa) / scale)
    assert np.all(np.abs(fb - fa) <= 1e-3 * scale)
    if iso:
        assert abs(c["post"][5] / c["post"][0] - c["pre"][5] / c["pre"][0]) <= 1e-3


def problem(case, **kw):
    c = TABLE[case]
    return I.cshock(c["pre"], c["post"], c["gamma"], eta=c["eta"], gamma_ad=c["gamma_ad"], rho_ion=c["rho_ion"],
                    **kw)


@pytest.mark.parametrize("case", ["ad_noniso", "ohm"])
def test_cshock_levels_and_boundary_patches(orc, case):
    """Over 16 dt_base: the boundary patches keep their state bitwise and are
    never updated, the five row patches end at the same time, and the local
    steps follow the non-ideal limits: with ambipolar diffusion the downstream
    patches (larger B^2 / rho) step twice as often as the upstream ones; with
    Ohmic diffusion (a fixed eta and dx) every patch takes the same step."""
    pr = problem(case)
    s = orc.OracleSet.from_problem(pr)
    s.set_order(2, 1, 8)
    T = 16 * pr.cfg.dt_base
    s.advance_to(T)
    U = s.read_state()
    st, kh, kl = s.read_schedule(klog_cap=64)
    stats = s.stats()
    s.close()
    V, V0 = I.patch_views(U, pr.patches), I.patch_views(pr.U0, pr.patches)
    for m in (0, len(pr.patches) - 1):
        assert st[m] == 0
        assert all(np.array_equal(a, b) for a, b in zip(V[m], V0[m]))
    assert stats[14] == stats[15] == T
    lev = [sorted(set(kl[m, :st[m]].tolist())) for m in range(1, len(pr.patches) - 1)]
    print(case, "levels per row patch", lev)
    assert all(len(x) == 1 for x in lev)
    k = [x[0] for x in lev]
    if case == "ohm":
        assert len(set(k)) == 1
    else:
        assert k[0] == k[1] and k[2] == k[3] == k[4] == k[0] + 1


def steady_isothermal_cshock(case="ad_iso", x_end=1.0):
    """Steady isothermal C-shock with ambipolar diffusion, from the upstream
    state of the table: with j = rho u, the x- and y-momentum fluxes and the
    z electric field uniform (B_x fixed, B_z = v_z = 0, sound speed
    c^2 = P / rho), u, v and rho follow from B_y algebraically, and
    dB_y/dx = (u B_y - v B_x - E_0) / eta_AD with eta_AD = B^2 / (gamma_AD rho
    rho_i) (Eq. AD for a current along z).  Returns x and B_y along the
    solution, started a hair above the upstream state."""
    from scipy.integrate import solve_ivp
    c = TABLE[case]
    rho0, u0, v0, bx, by0, p0 = c["pre"]
    c2 = p0 / rho0
    j = rho0 * u0
    px = rho0 * u0 * u0 + p0 + 0.5 * by0 * by0
    py = rho0 * u0 * v0 - bx * by0
    e0 = u0 * by0 - v0 * bx

    def state(by):
        v = (py + bx * by) / j
        a = px - 0.5 * by * by
        u = (a + math.sqrt(max(a * a - 4.0 * j * j * c2, 0.0))) / (2.0 * j)  # the supersonic branch
        return u, v, j / u

    def rhs(x, y):
        u, v, rho = state(y[0])
        eta = (bx * bx + y[0] * y[0]) / (c["gamma_ad"] * rho * c["rho_ion"])
        return [(u * y[0] - v * bx - e0) / eta]

    sol = solve_ivp(rhs, [0.0, x_end], [by0 + 1e-6], max_step=1e-3, rtol=1e-10, atol=1e-12)
    return sol.t, sol.y[0], state


def test_steady_cshock_ends_in_the_table_state():
    """The steady isothermal C-shock, integrated from the table's upstream
    state, ends in the table's downstream state (to its printed digits)."""
    x, by, state = steady_isothermal_cshock()
    u, v, rho = state(by[-1])
    post = TABLE["ad_iso"]["post"]
    got = [rho, u, v, by[-1]]
    want = [post[0], post[1], post[2], post[4]]
    print("downstream of the steady C-shock", got, "table", want)
    assert all(abs(a - b) <= 1e-4 * max(1.0, abs(b)) for a, b in zip(got, want))
