"""Plane-parallel test problems and the cyclic axis permutation of a problem.

A problem that varies along x only, run along x, y and z, must give the same
result with the axes permuted: the method treats the three directions alike
(the solver rotates each face to (normal, t1, t2) = (x, y, z), (y, z, x) or
(z, x, y); the edge EMFs of constrained transport are cyclic in (a, b, c)).
Permuting cyclically keeps the rotated frames of the faces in step, so every
face flux of the permuted run is computed from the same numbers in the same
order.  Sums over the lab axes (kinetic and magnetic energy, the Courant rate)
add the same terms in another order; with at most two non-zero vector
components, as in every problem here, such a sum is exact in any order, and dt
is fixed or quantised, so the results must agree bit for bit.  This pins the y- and z-direction arithmetic of the oracle (the predictor
terms, the face states and fluxes, the E_x and E_y edge EMFs and their
upwinding, the non-ideal E_x) against its x-direction arithmetic, which the
one-dimensional closed-form pins check.

Input construction only: nothing here computes any step of the method."""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from paper_1705_10774_amd import inputs as I


def _fields_1d(patches, prof):
    """Per-patch primitive arrays from prof(x_cell, x_face) -> dict with
    rho, vx, vy, vz, p (functions of the cell x) and bx (face x), by, bz
    (cell x).  Uniform along y and z."""
    rho, vel, pres, bf = [], [], [], []
    for q in patches:
        x = I.cell_coords(q)[0]
        xf = I.face_coords(q, 0)[0]
        f = prof(x, xf)
        n = q.n
        # a profile entry is a scalar or one value per cell (face) along x
        col = lambda a, shape: np.broadcast_to((np.asarray(a, dtype=float) * np.ones(shape[-1]))[None, None, :],
                                               shape).copy()
        rho.append(col(f["rho"], (n, n, n)))
        vel.append([col(f["vx"], (n, n, n)), col(f["vy"], (n, n, n)), col(f["vz"], (n, n, n))])
        pres.append(col(f["p"], (n, n, n)))
        bf.append((col(f["bx"], (n, n, n + 1)), col(f["by"], (n, n + 1, n)), col(f["bz"], (n + 1, n, n))))
    return rho, vel, pres, bf


def plane_problem(kind: str, npx: int = 4, n: int = 8, prec=I.F64) -> I.Problem:
    """A problem along x on a periodic row of npx patches of n^3 cells.

    sod          hydrodynamic shock tube (Sod's states, gamma 1.4, B = 0), fixed dt
    briowu       MHD shock tube (Brio & Wu's states, gamma 2, B_n = 0.75,
                 B_t = +-1 along y), fixed dt: fast and slow shocks, a compound
                 wave and a contact, every HLLD branch
    alfven_y     Alfven wave of amplitude 1e-3 polarised along y, local steps
    alfven_z     the same wave polarised along z (the t2 component of x-faces)
    beltrami_ni  force-free field B = (0, sin, cos)(2 pi x) with Ohmic and
                 ambipolar diffusion, fixed dt
    Two discontinuities (at 0.5 and at the periodic boundary) in the tubes."""
    patches, box = I.row(npx, n)
    gamma = 5.0 / 3.0
    cfg_kw = {}
    if kind == "sod":
        gamma = 1.4

        def prof(x, xf):
            L = x < 0.5
            return dict(rho=np.where(L, 1.0, 0.125), vx=0.0, vy=0.0, vz=0.0, p=np.where(L, 1.0, 0.1),
                        bx=0.0, by=0.0, bz=0.0)
        cfg_kw = dict(dt_mode=I.DT_FIXED, dt_fixed=2e-3)
        t_end = 0.06
    elif kind == "briowu":
        gamma = 2.0

        def prof(x, xf):
            L = x < 0.5
            return dict(rho=np.where(L, 1.0, 0.125), vx=0.0, vy=0.0, vz=0.0, p=np.where(L, 1.0, 0.1),
                        bx=0.75, by=np.where(L, 1.0, -1.0), bz=0.0)
        cfg_kw = dict(dt_mode=I.DT_FIXED, dt_fixed=1.5e-3)
        t_end = 0.045
    elif kind in ("alfven_y", "alfven_z"):
        amp = 1e-3
        pol = kind[-1]

        def prof(x, xf):
            s = amp * np.sin(2 * np.pi * x)
            return dict(rho=1.0, vx=0.0, vy=-s if pol == "y" else 0.0, vz=-s if pol == "z" else 0.0, p=0.6,
                        bx=1.0, by=s if pol == "y" else 0.0, bz=s if pol == "z" else 0.0)
        # fast speed 1 along x and sqrt 2 across: dt_base puts the patches at r ~ 0.75
        rate = (1.0 + 2.0 * math.sqrt(2.0)) / (1.0 / (npx * n))
        cfg_kw = dict(dt_mode=I.DT_LOCAL, dt_base=0.75 * 0.4 / rate)
        t_end = 6 * cfg_kw["dt_base"]
    elif kind == "beltrami_ni":
        def prof(x, xf):
            return dict(rho=1.0, vx=0.0, vy=0.0, vz=0.0, p=1.0, bx=0.0, by=np.sin(2 * np.pi * x),
                        bz=np.cos(2 * np.pi * x))
        cfg_kw = dict(dt_mode=I.DT_FIXED, dt_fixed=2e-4, eta=0.02, gamma_ad=20.0, rho_ion=1.0)
        t_end = 0.004
    else:
        raise ValueError(kind)
    rho, vel, pres, bf = _fields_1d(patches, prof)
    U = I.assemble(patches, rho, vel, pres, bf, gamma)
    cfg = I.Config(gamma=gamma, prec=prec, box_hi=box, kmax=30, **cfg_kw)
    return I.Problem(f"{kind}_x", cfg, patches, U, t_end)


# ---------------------------------------------------------------------------
# cyclic permutation of the axes: lab axis d of the old problem becomes axis
# (d + 1) mod 3 of the new one (x -> y -> z -> x)


def _cyc(t):
    return (t[2], t[0], t[1])


def permute_state(U: np.ndarray, patches) -> np.ndarray:
    """State of the permuted problem (patches in the same id order)."""
    out = np.empty_like(U)
    Vi = I.patch_views(U, patches)
    Vo = I.patch_views(out, patches)
    for vi, vo in zip(Vi, Vo):
        tr = lambda a: np.transpose(a, (1, 2, 0))
        vo[0][...] = tr(vi[0])
        vo[1][...] = tr(vi[3])  # new m_x = old m_z
        vo[2][...] = tr(vi[1])
        vo[3][...] = tr(vi[2])
        vo[4][...] = tr(vi[4])
        vo[5][...] = tr(vi[7])  # new B_x = old B_z
        vo[6][...] = tr(vi[5])
        vo[7][...] = tr(vi[6])
    return out


def permute_problem(pr: I.Problem, times: int = 1) -> I.Problem:
    patches, U, cfg = pr.patches, pr.U0, pr.cfg
    for _ in range(times):
        U = permute_state(U, patches)
        patches = [dataclasses.replace(q, origin=_cyc(q.origin)) for q in patches]
        cfg = dataclasses.replace(cfg, box_lo=_cyc(cfg.box_lo), box_hi=_cyc(cfg.box_hi))
    axis = "xyz"[times % 3]
    return dataclasses.replace(pr, name=pr.name[:-1] + axis, cfg=cfg, patches=patches, U0=U)


def permute_result(U: np.ndarray, patches, times: int) -> np.ndarray:
    """A state of the original problem's geometry mapped to the permuted one."""
    for _ in range(times):
        U = permute_state(U, patches)
    return U
