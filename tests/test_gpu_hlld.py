"""The HLLD face flux on the GPU (dsp_hlld_faces: the step kernels' own
flux arithmetic) against the oracle's orc_hlld_flux, face by face, on random
states and on the degenerate and special cases of the solver: vanishing
normal field, vanishing transverse field (degenerate star states), equal
states, a stationary contact, supersonic flow either way, strong jumps and
near-vacuum densities."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

G = 5.0 / 3.0


def _dsp():
    from paper_1705_10774_amd import dsp
    dsp.load()
    return dsp


def _faces(seed=21):
    rng = np.random.default_rng(seed)
    L, R, B, tags = [], [], [], []

    def st(rho=None, u=None, p=None, bt=1.0, vt=1.0):
        return np.array([rng.uniform(0.1, 3.0) if rho is None else rho,
                         rng.normal(0, 1.5) if u is None else u,
                         vt * rng.normal(0, 1), vt * rng.normal(0, 1),
                         rng.uniform(0.05, 3.0) if p is None else p,
                         bt * rng.normal(0, 1), bt * rng.normal(0, 1)])

    def add(tag, l, r, bn):
        L.append(l); R.append(r); B.append(bn); tags.append(tag)

    for _ in range(4000):
        add("random", st(), st(), rng.normal(0, 1.2))
    for _ in range(500):
        add("bn=0", st(), st(), 0.0)
    for _ in range(500):
        add("bt=0", st(bt=0.0), st(bt=0.0), rng.normal(0, 1.2))
    for _ in range(500):
        add("bt=0,vt=0", st(bt=0.0, vt=0.0), st(bt=0.0, vt=0.0), rng.normal(0, 1.2))
    for _ in range(300):
        w = st()
        add("equal", w, w.copy(), rng.normal(0, 1.2))
    for _ in range(300):
        p = rng.uniform(0.1, 2.0)
        v1, v2, b1, b2 = rng.normal(0, 1, 4)
        add("contact", np.array([rng.uniform(0.1, 3), 0.0, v1, v2, p, b1, b2]),
            np.array([rng.uniform(0.1, 3), 0.0, v1, v2, p, b1, b2]), rng.normal(0, 1))
    for _ in range(300):
        add("supersonic+", st(u=rng.uniform(6, 10)), st(u=rng.uniform(6, 10)), rng.normal(0, 0.5))
        add("supersonic-", st(u=-rng.uniform(6, 10)), st(u=-rng.uniform(6, 10)), rng.normal(0, 0.5))
    for _ in range(300):
        add("strong jump", st(rho=1.0, p=1000.0), st(rho=0.125, p=0.1), rng.normal(0, 1.2))
        add("near vacuum", st(rho=1e-4, p=1e-5), st(rho=2.0, p=1.0), rng.normal(0, 0.3))
    return np.array(L), np.array(R), np.array(B), np.array(tags)


def _oracle(orc, L, R, B):
    return np.array([orc.hlld_flux(l, r, b, G, 1e-12) for l, r, b in zip(L, R, B)])


def _scale(L, R, B):
    """Natural size of each face's fluxes: (rho + p + B^2)(1 + |u| + c) of
    the larger side, so that a relative bound is met by every component."""
    def side(W):
        bb = B ** 2 + W[:, 5] ** 2 + W[:, 6] ** 2
        v = np.sqrt(W[:, 1] ** 2 + W[:, 2] ** 2 + W[:, 3] ** 2)
        c = np.sqrt((G * W[:, 4] + bb) / W[:, 0])
        return (W[:, 0] * (1 + v * v) + W[:, 4] + bb) * (1 + v + c)
    return np.maximum(side(L), side(R))


def test_hlld_faces_fp64_match_oracle(orc):
    dsp = _dsp()
    L, R, B, tags = _faces()
    got = dsp.dsp_hlld_faces(dsp.DSP_F64, L, R, B, G)
    want = _oracle(orc, L, R, B)
    sc = _scale(L, R, B)[:, None]
    rel = np.abs(got[:, :7] - want[:, :7]) / sc
    for t in sorted(set(tags)):
        print(f"{t:14s} worst {rel[tags == t].max():.2e}")
    assert rel.max() <= 1e-14
    # the upwind speed: same value to rounding, and exactly zero where the
    # oracle's is (the stationary contact)
    us = np.abs(got[:, 7] - want[:, 7]) / (1 + np.abs(want[:, 7]))
    assert us.max() <= 1e-14
    assert np.all(got[want[:, 7] == 0.0, 7] == 0.0)
    assert np.all(got[tags == "contact", 0] == want[tags == "contact", 0]) or \
        np.abs(got[tags == "contact", 0]).max() <= 1e-14 * sc[tags == "contact"].max()


def test_hlld_faces_fp32_match_oracle(orc):
    dsp = _dsp()
    L, R, B, tags = _faces(22)
    ok = tags != "near vacuum"  # 1e-4 densities: FP32 rounding of the inputs dominates
    L, R, B, tags = L[ok], R[ok], B[ok], tags[ok]
    got = dsp.dsp_hlld_faces(dsp.DSP_F32, L, R, B, G)
    # the oracle on the same FP32-rounded inputs
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    want = _oracle(orc, f32(L), f32(R), f32(B))
    sc = _scale(L, R, B)[:, None]
    rel = np.abs(got[:, :7] - want[:, :7]) / sc
    for t in sorted(set(tags)):
        print(f"{t:14s} worst {rel[tags == t].max():.2e}")
    assert rel.max() <= 2e-5


def test_hlld_faces_argument_errors():
    dsp = _dsp()
    with pytest.raises(dsp.DspError):
        dsp.dsp_hlld_faces(3, np.zeros((1, 7)), np.zeros((1, 7)), np.zeros(1))
    with pytest.raises(ValueError):
        dsp.dsp_hlld_faces(dsp.DSP_F64, np.zeros((2, 7)), np.zeros((1, 7)), np.zeros(1))
    assert dsp.dsp_hlld_faces(dsp.DSP_F64, np.zeros((0, 7)), np.zeros((0, 7)), np.zeros(0)).shape == (0, 8)
