"""Seeded synthetic inputs: patch layouts, configurations and initial states.

This module is the only code shared by the GPU library's tests/benchmark and
the CPU oracle.  It holds no part of the patch-update method itself: it lays
out patches (the paper's *cartesian* component, Sec. 2.3, and the nested
"Rubik's Revenge" component for static refinement), draws seeded random
fields as finite Fourier sums over integer wavevectors, and writes initial
states in the host layout of the library:

* per patch, in id order: rho, mx, my, mz, E, each [n][n][n] (z, y, x order,
  x fastest), then Bx [n][n][n+1], By [n][n+1][n], Bz [n+1][n][n];
* every patch stores both of its boundary faces.

All arrays are float64.  Random fields are evaluated at cell and face
centres and do not depend on the resolution, so patches of different n
sample the same field.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

# dt modes and precisions, numbered as in include/dsp.h
DT_LOCAL, DT_GLOBAL_QUANT, DT_GLOBAL_EXACT, DT_FIXED = 0, 1, 2, 3
F32, F64 = 1, 2


@dataclasses.dataclass
class Config:
    gamma: float = 5.0 / 3.0
    courant: float = 0.4
    dt_base: float = 0.0
    dt_fixed: float = 0.0
    grace: float = 0.0
    p_floor: float = 0.0
    kmax: int = 30
    nslots: int = 3
    nguard: int = 3
    limiter: int = 0
    prec: int = F64
    dt_mode: int = DT_LOCAL
    periodic: Tuple[int, int, int] = (1, 1, 1)
    box_lo: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    box_hi: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    eta: float = 0.0       # Ohmic resistivity (Sec. 4.3.1); 0 = none
    gamma_ad: float = 0.0  # ambipolar drift coefficient (Sec. 4.3.2); 0 = none
    rho_ion: float = 1.0   # ion density of the ambipolar term
    torder: int = 1        # guard time interpolation: 1 linear, 2 quadratic (three slices)


@dataclasses.dataclass
class Patch:
    origin: Tuple[float, float, float]
    size: float
    n: int
    level: int = 0
    frozen: bool = False  # boundary patch: never updated, its state holds at every time


@dataclasses.dataclass
class Problem:
    name: str
    cfg: Config
    patches: List[Patch]
    U0: np.ndarray
    t_end: float
    nsteps: Optional[int] = None
    extra: dict = dataclasses.field(default_factory=dict)

    @property
    def cells(self) -> int:
        return sum(p.n ** 3 for p in self.patches)


# ---------------------------------------------------------------------------
# host layout

def slice_size(n: int) -> int:
    return 5 * n ** 3 + 3 * n * n * (n + 1)


def offsets(patches) -> np.ndarray:
    off = np.zeros(len(patches) + 1, dtype=np.int64)
    for i, p in enumerate(patches):
        off[i + 1] = off[i] + slice_size(p.n)
    return off


def split_slice(u: np.ndarray, n: int):
    """Views (rho, mx, my, mz, E, Bx, By, Bz) of one patch slice."""
    n3, nf = n ** 3, n * n * (n + 1)
    cells = [u[v * n3:(v + 1) * n3].reshape(n, n, n) for v in range(5)]
    bx = u[5 * n3:5 * n3 + nf].reshape(n, n, n + 1)
    by = u[5 * n3 + nf:5 * n3 + 2 * nf].reshape(n, n + 1, n)
    bz = u[5 * n3 + 2 * nf:5 * n3 + 3 * nf].reshape(n + 1, n, n)
    return cells + [bx, by, bz]


def patch_views(U: np.ndarray, patches):
    off = offsets(patches)
    return [split_slice(U[off[i]:off[i + 1]], p.n) for i, p in enumerate(patches)]


# ---------------------------------------------------------------------------
# components (patch layouts)

def cartesian(npd: int, n, box: float = 1.0, origin=(0.0, 0.0, 0.0), level: int = 0):
    """npd^3 equal non-overlapping patches tiling a cube, id = (z*npd + y)*npd + x.
    n is an int or a per-patch sequence of interior sizes."""
    size = box / npd
    out = []
    for pz in range(npd):
        for py in range(npd):
            for px in range(npd):
                i = (pz * npd + py) * npd + px
                nn = n if isinstance(n, (int, np.integer)) else int(n[i])
                out.append(Patch((origin[0] + px * size, origin[1] + py * size,
                                  origin[2] + pz * size), size, int(nn), level))
    return out


def rubiks_revenge(levels: int = 3, n: int = 16):
    """Nested 4x4x4 sets (Sec. 2.3): level l covers the centred cube of side
    2^-l of the unit box with 4^3 patches; the central 2x2x2 patches of each
    level but the finest are covered by the next level and left out."""
    out = []
    for lev in range(levels):
        side = 0.5 ** lev
        lo = 0.5 - side / 2
        size = side / 4
        for pz in range(4):
            for py in range(4):
                for px in range(4):
                    covered = lev < levels - 1 and all(1 <= q <= 2 for q in (px, py, pz))
                    if covered:
                        continue
                    out.append(Patch((lo + px * size, lo + py * size, lo + pz * size),
                                     size, n, lev))
    return out


# ---------------------------------------------------------------------------
# coordinates of the sample points of one patch

def cell_coords(p: Patch):
    dx = p.size / p.n
    return [p.origin[d] + (np.arange(p.n) + 0.5) * dx for d in range(3)]


def face_coords(p: Patch, d: int):
    """Coordinates of the d-faces of patch p: face positions along d, centres
    along the other axes."""
    dx = p.size / p.n
    c = cell_coords(p)
    c[d] = p.origin[d] + np.arange(p.n + 1) * dx
    return c


# ---------------------------------------------------------------------------
# seeded random fields as finite Fourier sums


class FourierField:
    """Real field f(x) = Re sum_k c_k exp(2 pi i k.x / L) over integer
    wavevectors with kmin <= |k| <= kmax, complex Gaussian coefficients with
    |c_k| proportional to |k|^-slope (slope 2 gives a shell spectrum
    E(k) ~ k^-2)."""

    def __init__(self, rng: np.random.Generator, kmin: float, kmax: float, slope: float,
                 box: float = 1.0):
        K = int(math.floor(kmax))
        ks = np.arange(-K, K + 1)
        kx, ky, kz = np.meshgrid(ks, ks, ks, indexing="ij")
        kk = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
        mask = (kk >= kmin) & (kk <= kmax)
        amp = np.zeros_like(kk)
        amp[mask] = kk[mask] ** (-slope)
        c = (rng.standard_normal(kk.shape) + 1j * rng.standard_normal(kk.shape)) * amp
        self.c = c  # indexed [kx + K, ky + K, kz + K]
        self.K = K
        self.box = box

    def sample(self, x, y, z) -> np.ndarray:
        """Values on the tensor grid x (nx), y (ny), z (nz) -> array [nz, ny, nx]."""
        K, L = self.K, self.box
        ks = np.arange(-K, K + 1)
        ex = np.exp(2j * np.pi * np.outer(np.asarray(x), ks) / L)  # [nx, kx]
        ey = np.exp(2j * np.pi * np.outer(np.asarray(y), ks) / L)
        ez = np.exp(2j * np.pi * np.outer(np.asarray(z), ks) / L)
        t1 = np.einsum("zc,abc->zab", ez, self.c)          # [nz, kx, ky]
        t2 = np.einsum("yb,zab->zya", ey, t1)              # [nz, ny, kx]
        f = np.einsum("xa,zya->zyx", ex, t2)               # [nz, ny, nx]
        return f.real.copy()


# ---------------------------------------------------------------------------
# initial state assembly

def assemble(patches, rho, vel, pres, bfaces, gamma) -> np.ndarray:
    """Host-layout state from per-patch primitive samples.
    rho, pres: list of [n,n,n]; vel: list of 3-lists; bfaces: list of
    (Bx [n,n,n+1], By [n,n+1,n], Bz [n+1,n,n]).  The total energy uses the
    cell-centred field taken as the mean of the two faces of each cell."""
    U = np.zeros(int(offsets(patches)[-1]), dtype=np.float64)
    views = patch_views(U, patches)
    for i, p in enumerate(patches):
        r, v, pr = rho[i], vel[i], pres[i]
        bx, by, bz = bfaces[i]
        v_ = views[i]
        v_[0][...] = r
        for d in range(3):
            v_[1 + d][...] = r * v[d]
        bcx = 0.5 * (bx[:, :, :-1] + bx[:, :, 1:])
        bcy = 0.5 * (by[:, :-1, :] + by[:, 1:, :])
        bcz = 0.5 * (bz[:-1, :, :] + bz[1:, :, :])
        ke = 0.5 * r * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2)
        me = 0.5 * (bcx ** 2 + bcy ** 2 + bcz ** 2)
        v_[4][...] = pr / (gamma - 1.0) + ke + me
        v_[5][...] = bx
        v_[6][...] = by
        v_[7][...] = bz
    return U


def _uniform_b(patches, B):
    out = []
    for p in patches:
        n = p.n
        out.append((np.full((n, n, n + 1), B[0]), np.full((n, n + 1, n), B[1]),
                    np.full((n + 1, n, n), B[2])))
    return out


# ---------------------------------------------------------------------------
# problems


def uniform(npd=2, n=16, rho=1.0, v=(0.0, 0.0, 0.0), p=0.6, B=(1.0, 0.0, 0.0),
            gamma=5.0 / 3.0, mode=DT_GLOBAL_EXACT, t_end=0.1, dt_base=0.0, prec=F64):
    patches = cartesian(npd, n)
    sh = [(q.n,) * 3 for q in patches]
    U = assemble(patches, [np.full(s, rho) for s in sh],
                 [[np.full(s, v[d]) for d in range(3)] for s in sh],
                 [np.full(s, p) for s in sh], _uniform_b(patches, B), gamma)
    cfg = Config(gamma=gamma, dt_mode=mode, dt_base=dt_base, prec=prec, kmax=30)
    return Problem("uniform", cfg, patches, U, t_end)


def row(npx: int, n: int, length: float = 1.0):
    """npx cubic patches in a row along x: a periodic box of length x
    (length/npx) x (length/npx), for problems that vary along x only."""
    size = length / npx
    return [Patch((i * size, 0.0, 0.0), size, n) for i in range(npx)], (length, size, size)


def linear_wave(kind="alfven", npd=2, n=16, amp=1e-6, gamma=5.0 / 3.0, t_end=1.0,
                mode=DT_GLOBAL_EXACT, prec=F64, courant=0.4, npx_row=0, p0=0.6, row_levels=()):
    """Plane waves along x on rho = 1, p = 0.6, B = (1, 0, 0) (c_s = v_A = 1),
    point-sampled at cell and face centres.
    alfven: right-going, y-polarised, dBy = A sin 2 pi x, dvy = -A sin 2 pi x.
    sound:  right-going sound wave, drho = A sin, dvx = c_s A sin, dp = c_s^2 A sin
            with c_s^2 = gamma p0 (p0 sets the background pressure).
    npx_row > 0 lays the patches out in a row along x instead of a cube;
    row_levels = (k_0, k_1, ...) lays out a row whose patch i has n 2^k_i
    cells per edge."""
    box = (1.0, 1.0, 1.0)
    if row_levels:
        patches, box = row(len(row_levels), n)
        patches = [Patch(q.origin, q.size, n << k) for q, k in zip(patches, row_levels)]
    elif npx_row > 0:
        patches, box = row(npx_row, n)
    else:
        patches = cartesian(npd, n)
    rho, vel, pres, bf = [], [], [], []
    for q in patches:
        x, y, z = cell_coords(q)
        s = np.broadcast_to(np.sin(2 * np.pi * x)[None, None, :], (q.n,) * 3)
        r = np.ones((q.n,) * 3)
        v = [np.zeros((q.n,) * 3) for _ in range(3)]
        pr = np.full((q.n,) * 3, p0)
        bx = np.ones((q.n, q.n, q.n + 1))
        by = np.zeros((q.n, q.n + 1, q.n))
        bz = np.zeros((q.n + 1, q.n, q.n))
        if kind == "alfven":
            v[1] = -amp * s
            by[...] = amp * np.sin(2 * np.pi * x)[None, None, :]
        elif kind == "sound":
            cs = math.sqrt(gamma * p0)
            r = r + amp * s
            v[0] = cs * amp * s
            pr = pr + gamma * p0 * amp * s
        else:
            raise ValueError(kind)
        rho.append(r); vel.append(v); pres.append(pr); bf.append((bx, by, bz))
    U = assemble(patches, rho, vel, pres, bf, gamma)
    cfg = Config(gamma=gamma, courant=courant, dt_mode=mode, prec=prec, box_hi=box)
    return Problem(f"{kind}_wave", cfg, patches, U, t_end, extra={"amp": amp})


def level_row(levels=(0, 0, 1, 0, 2), n=8, amp=1e-3, prec=F64, dt_base=None, nslots=4, grace=0.0):
    """A sound wave (A = 1e-3) along a periodic row of equal-size patches with
    n 2^k cells per edge: LOCAL steps in which patch i keeps level k_i (the
    Courant rate doubles with the resolution; dt_base puts the coarsest at
    r ~ 0.75).  A row of mixed levels is where a grace lets patches run ahead
    of a coarser neighbour even when every ready patch updates at once."""
    pr = linear_wave("sound", n=n, amp=amp, prec=prec, mode=DT_LOCAL, row_levels=tuple(levels))
    if dt_base is None:
        # c_s = v_A = 1 with B along x: fast speed 1 along x, sqrt 2 across
        rate = (1.0 + 2.0 * math.sqrt(2.0)) / (pr.patches[0].size / n)
        dt_base = 0.75 * pr.cfg.courant / rate
    pr.cfg = dataclasses.replace(pr.cfg, dt_base=dt_base, nslots=nslots, grace=grace)
    pr.name = "level_row"
    return pr


def field_1d(kind="beltrami", npd=2, n=16, B0=1.0, b=0.1, p0=1.0, eta=0.0, gamma_ad=0.0, rho_ion=1.0,
             mode=DT_FIXED, dt_fixed=1e-3, dt_base=0.0, prec=F64, t_end=0.1):
    """Fields along x on rho = 1, p = p0, v = 0, sampled at face centres, for
    the non-ideal terms (Sec. 4.3); k = 2 pi.
    beltrami:   B = B0 (0, sin kx, cos kx), force free (J = k B), |B| = B0;
    transverse: B = (0, B0 + b sin kx, 0), J = b k cos kx z (J x B != 0);
    alfven:     B = (B0, b sin kx, 0), J perpendicular to B, |B|^2 = B0^2 + O(b^2)."""
    patches = cartesian(npd, n)
    rho, vel, pres, bf = [], [], [], []
    for q in patches:
        x = cell_coords(q)[0]
        sx = np.sin(2 * np.pi * x)[None, None, :]
        cx = np.cos(2 * np.pi * x)[None, None, :]
        bx = np.zeros((q.n, q.n, q.n + 1))
        by = np.zeros((q.n, q.n + 1, q.n))
        bz = np.zeros((q.n + 1, q.n, q.n))
        if kind == "beltrami":
            by[...] = B0 * sx
            bz[...] = B0 * cx
        elif kind == "transverse":
            by[...] = B0 + b * sx
        elif kind == "alfven":
            bx[...] = B0
            by[...] = b * sx
        else:
            raise ValueError(kind)
        rho.append(np.ones((q.n,) * 3))
        vel.append([np.zeros((q.n,) * 3) for _ in range(3)])
        pres.append(np.full((q.n,) * 3, p0))
        bf.append((bx, by, bz))
    U = assemble(patches, rho, vel, pres, bf, 5.0 / 3.0)
    cfg = Config(dt_mode=mode, dt_fixed=dt_fixed, dt_base=dt_base, prec=prec, eta=eta, gamma_ad=gamma_ad,
                 rho_ion=rho_ion)
    return Problem(f"{kind}_1d", cfg, patches, U, t_end, extra={"B0": B0, "b": b, "p0": p0})


def cshock(pre, post, gamma, eta=0.0, gamma_ad=0.0, rho_ion=1.0, n=16, npatch=5, size=0.2, dt_base=2.5e-4,
           t_end=1.0, prec=F64):
    """A stationary shock along x between two states (rho, vx, vy, Bx, By, P)
    of the shock frame: a row of npatch patches of size `size` (n^3 cells,
    uniform in y and z) with the upstream state left of the middle of the
    row and the downstream state right of it, between two boundary patches
    that hold the upstream (left) and downstream (right) state."""
    patches, box = row(npatch + 2, n, length=size * (npatch + 2))
    patches = [Patch(q.origin, q.size, q.n, frozen=(m == 0 or m == npatch + 1)) for m, q in enumerate(patches)]
    xm = size * (1 + npatch / 2.0)
    rho, vel, pres, bf = [], [], [], []
    for q in patches:
        x = cell_coords(q)[0]
        xf = face_coords(q, 0)[0]
        up = (x < xm)[None, None, :]
        sel = lambda a, b: np.broadcast_to(np.where(up, a, b), (q.n,) * 3).copy()
        rho.append(sel(pre[0], post[0]))
        vel.append([sel(pre[1], post[1]), sel(pre[2], post[2]), np.zeros((q.n,) * 3)])
        pres.append(sel(pre[5], post[5]))
        bx = np.broadcast_to(np.where(xf < xm, pre[3], post[3])[None, None, :], (q.n, q.n, q.n + 1)).copy()
        by = np.broadcast_to(np.where(up, pre[4], post[4]), (q.n, q.n + 1, q.n)).copy()
        bz = np.zeros((q.n + 1, q.n, q.n))
        bf.append((bx, by, bz))
    U = assemble(patches, rho, vel, pres, bf, gamma)
    cfg = Config(gamma=gamma, dt_mode=DT_LOCAL, dt_base=dt_base, prec=prec, eta=eta, gamma_ad=gamma_ad,
                 rho_ion=rho_ion, box_hi=box)
    return Problem("cshock", cfg, patches, U, t_end, extra={"pre": pre, "post": post, "xm": xm})


def cfg1_alfven(prec=F64):
    """2x2x2 patches of 16^3, global exact dt, Alfven wave A = 1e-6, t = 1."""
    pr = linear_wave("alfven", npd=2, n=16, amp=1e-6, prec=prec)
    pr.name = "cfg1_alfven"
    return pr


def turbulence(npd=8, n=16, mach=5.0, seed=1002, dt_base=None, t_end=0.02, prec=F64,
               mode=DT_LOCAL, name="cfg2_turb", p_floor=0.0):
    """rho = 1, p = 0.6 (c_s = 1), B = (sqrt 12, 0, 0) (beta = 0.1); Gaussian
    random velocity with shell spectrum E(k) ~ k^-2 over 1 <= |k| <= 4, mean
    removed, scaled to rms |v| = mach."""
    patches = cartesian(npd, n)
    rng = np.random.Generator(np.random.PCG64(seed))
    fields = [FourierField(rng, 1.0, 4.0, 2.0) for _ in range(3)]
    vel = []
    for q in patches:
        x, y, z = cell_coords(q)
        vel.append([f.sample(x, y, z) for f in fields])
    allv = [np.concatenate([v[d].ravel() for v in vel]) for d in range(3)]
    means = [a.mean() for a in allv]
    rms = math.sqrt(sum(((a - m) ** 2).mean() for a, m in zip(allv, means)))
    scale = mach / rms
    vel = [[(v[d] - means[d]) * scale for d in range(3)] for v in vel]
    sh = [(q.n,) * 3 for q in patches]
    U = assemble(patches, [np.ones(s) for s in sh], vel, [np.full(s, 0.6) for s in sh],
                 _uniform_b(patches, (math.sqrt(12.0), 0.0, 0.0)), 5.0 / 3.0)
    if dt_base is None:
        dt_base = t_end / 128.0
    # Mach-5 turbulence drives the pressure to zero in a few cells near the end
    # of the run (the FP64 oracle too), so a counted floor is part of the setup
    cfg = Config(dt_mode=mode, dt_base=dt_base, prec=prec, kmax=30, p_floor=p_floor)
    return Problem(name, cfg, patches, U, t_end)


def cfg2_turb(prec=F64, npd=8):
    return turbulence(npd=npd, prec=prec, p_floor=1e-10)


def cfg2_smooth(prec=F64, npd=8):
    return turbulence(npd=npd, mach=0.5, seed=1012, prec=prec, name="cfg2_smooth")


def uneven(npd=16, seed_sizes=1003, seed_rho=2003, prec=F32, box=1.0, name="cfg3_uneven",
           dt_base=None, nsteps_base=8, sizes=(16, 24, 32)):
    """npd^3 equal-size patches with n drawn uniformly from `sizes`;
    lognormal density ln rho = 2 G - 2 (G: unit-variance field, E(k) ~ k^-2,
    1 <= |k| <= 4), renormalised to <rho> = 1; p = 0.01 rho; B = (0, 0,
    sqrt 0.02) (beta = 1 at <p>); v = 0.  Runs to nsteps_base * dt_base."""
    rs = np.random.Generator(np.random.PCG64(seed_sizes))
    ns = rs.choice(np.array(sizes), size=npd ** 3)
    patches = cartesian(npd, ns, box=box)
    rng = np.random.Generator(np.random.PCG64(seed_rho))
    G = FourierField(rng, 1.0, 4.0, 2.0, box=box)
    g = []
    for q in patches:
        x, y, z = cell_coords(q)
        g.append(G.sample(x, y, z))
    # unit variance and zero mean over the volume (cells weighted by volume)
    w = [np.full(a.shape, (q.size / q.n) ** 3) for a, q in zip(g, patches)]
    W = sum(a.sum() for a in w)
    mean = sum((a * b).sum() for a, b in zip(g, w)) / W
    var = sum((((a - mean) ** 2) * b).sum() for a, b in zip(g, w)) / W
    rho = [np.exp(2.0 * (a - mean) / math.sqrt(var) - 2.0) for a in g]
    rmean = sum((a * b).sum() for a, b in zip(rho, w)) / W
    rho = [a / rmean for a in rho]
    vel = [[np.zeros_like(a) for _ in range(3)] for a in rho]
    pres = [0.01 * a for a in rho]
    U = assemble(patches, rho, vel, pres, _uniform_b(patches, (0.0, 0.0, math.sqrt(0.02))),
                 5.0 / 3.0)
    if dt_base is None:
        dt_base = 2.0 ** -9
    cfg = Config(dt_mode=DT_LOCAL, dt_base=dt_base, prec=prec, kmax=30, p_floor=1e-10,
                 box_hi=(box, box, box))
    return Problem(name, cfg, patches, U, nsteps_base * dt_base,
                   extra={"sizes": ns.tolist()})


def uneven_smooth(npd=3, sizes=(4, 16), seed_sizes=1021, prec=F64, box=0.1875, dt_base=2.0 ** -11,
                  nsteps_base=4, name="uneven_smooth"):
    """npd^3 equal-size patches with n drawn uniformly from `sizes` (wide
    resolution jumps between neighbours) carrying a smooth periodic state:
    rho = 1 + 0.2 sin(kx) sin(ky) sin(kz), v = 0.1 (cos ky, cos kz, cos kx),
    p = 0.6, B = (0.5, 0.3, 0.2), k = 2 pi / box.  Runs to nsteps_base * dt_base."""
    rs = np.random.Generator(np.random.PCG64(seed_sizes))
    ns = rs.choice(np.array(sizes), size=npd ** 3)
    patches = cartesian(npd, ns, box=box)
    kw = 2.0 * math.pi / box
    rho, vel, pres = [], [], []
    for q in patches:
        x, y, z = cell_coords(q)
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        rho.append(1.0 + 0.2 * np.sin(kw * X) * np.sin(kw * Y) * np.sin(kw * Z))
        vel.append([0.1 * np.cos(kw * Y), 0.1 * np.cos(kw * Z), 0.1 * np.cos(kw * X)])
        pres.append(np.full(X.shape, 0.6))
    U = assemble(patches, rho, vel, pres, _uniform_b(patches, (0.5, 0.3, 0.2)), 5.0 / 3.0)
    cfg = Config(dt_mode=DT_LOCAL, dt_base=dt_base, prec=prec, kmax=30, box_hi=(box, box, box))
    return Problem(name, cfg, patches, U, nsteps_base * dt_base, extra={"sizes": ns.tolist()})


def cfg3_uneven(prec=F32):
    return uneven(prec=prec)


def cfg3_mini(prec=F32):
    return uneven(npd=4, seed_sizes=1013, seed_rho=2013, prec=prec, box=0.25, name="cfg3_mini")


# blast centre: the centre of the box (the nested levels are centred on it)
SMR_CENTRE = (0.5, 0.5, 0.5)


def cfg4_smr(prec=F64, t_end=0.01, dt_base=None, levels=3, n=16):
    """Three nested levels (factor 2) of 4^3 patches of 16^3; blast wave of
    radius 0.1 at p = 100 in p = 1, rho = 1, B = (1, 1, 0)/sqrt 2, centred at
    SMR_CENTRE."""
    patches = rubiks_revenge(levels, n)
    cx, cy, cz = SMR_CENTRE
    rho, vel, pres = [], [], []
    for q in patches:
        x, y, z = cell_coords(q)
        r2 = ((x[None, None, :] - cx) ** 2 + (y[None, :, None] - cy) ** 2 +
              (z[:, None, None] - cz) ** 2)
        pres.append(np.where(r2 < 0.01, 100.0, 1.0))
        rho.append(np.ones((q.n,) * 3))
        vel.append([np.zeros((q.n,) * 3) for _ in range(3)])
    b = 1.0 / math.sqrt(2.0)
    U = assemble(patches, rho, vel, pres, _uniform_b(patches, (b, b, 0.0)), 5.0 / 3.0)
    if dt_base is None:
        dt_base = t_end / 8.0
    cfg = Config(dt_mode=DT_LOCAL, dt_base=dt_base, prec=prec, kmax=30, p_floor=1e-10)
    return Problem("cfg4_smr", cfg, patches, U, t_end)


def cfg5_adjoint(prec=F64, npd=4, n=16, nsteps=32, dt=1.6e-3, seed_init=1005,
                 seed_target=2005, B=(0.6, 0.4, 0.2), V=(0.3, 0.2, 0.1), dp=True):
    """4^3 patches of 16^3; rho = 1, p = 0.6, uniform oblique B and uniform
    flow V; smooth perturbations of rho and v (1 <= |k| <= 3, max |.| = 1e-3);
    target density rho* = 1 + the same recipe with another seed; fixed dt.
    The oblique field keeps the HLLD star states away from their degenerate
    limit, the mean flow keeps every face mass flux away from zero, and the
    (fixed) pressure carries its own smooth perturbation so that no limited
    slope starts at exactly zero: the fixed-dt map is then smooth at the
    initial state.  B = (1, 0, 0), V = 0, dp = False give the background
    as specified (uniform p = 0.6, fluid at rest)."""
    patches = cartesian(npd, n)

    def smooth(seed, ncomp):
        rng = np.random.Generator(np.random.PCG64(seed))
        fs = [FourierField(rng, 1.0, 3.0, 0.0) for _ in range(ncomp)]
        out = []
        for f in fs:
            vals = []
            for q in patches:
                x, y, z = cell_coords(q)
                vals.append(f.sample(x, y, z))
            mx = max(np.abs(a).max() for a in vals)
            out.append([1e-3 * a / mx for a in vals])
        return out

    if seed_init is None:  # the unperturbed background
        pert = [[np.zeros((q.n,) * 3) for q in patches] for _ in range(4)]
    else:
        pert = smooth(seed_init, 4)
    target = smooth(seed_target, 1)[0]
    rho = [1.0 + pert[0][i] for i in range(len(patches))]
    vel = [[V[d] + pert[1 + d][i] for d in range(3)] for i in range(len(patches))]
    pres = [0.6 * (1.0 + a) for a in smooth(3005, 1)[0]] if dp else [np.full((q.n,) * 3, 0.6) for q in patches]
    U = assemble(patches, rho, vel, pres, _uniform_b(patches, B), 5.0 / 3.0)
    cfg = Config(dt_mode=DT_FIXED, dt_fixed=dt, prec=prec, kmax=30)
    return Problem("cfg5_adjoint", cfg, patches, U, nsteps * dt, nsteps=nsteps,
                   extra={"rho0": rho, "v0": vel, "p0": pres,
                          "rho_target": [1.0 + a for a in target]})
