"""GPU adjoint of the fixed-dt step (through the C ABI), against the oracle.

* Dot-product test: <lam_T, J delta> with J delta from the oracle's forward
  mode (dual numbers, exact along the branches taken) equals <J^T lam_T, delta>
  from the GPU adjoint.
* Gradient of J = 1/2 sum (rho_T - rho*)^2 dV against a central difference of
  the GPU forward run, in the cancellation-free form
  Delta J = 1/2 sum (rho+ - rho-)(rho+ + rho- - 2 rho*) dV.
* The autograd function returns the adjoint's gradient."""
import numpy as np
import pytest

from paper_1705_10774_amd import inputs as I

pytestmark = pytest.mark.gpu


def _setup(prec=I.F64):
    import torch
    from paper_1705_10774_amd import dsp
    dsp.load()
    pr = I.cfg5_adjoint(prec=prec)
    s = dsp.PatchSet(pr.cfg, pr.patches)
    dt = torch.float64 if prec == I.F64 else torch.float32
    return torch, dsp, pr, s, dt


def _rho_mask(pr):
    """The cell volume on the density entries of the host layout, 0 elsewhere."""
    m = np.zeros(pr.U0.size)
    for v, q in zip(I.patch_views(m, pr.patches), pr.patches):
        v[0][...] = (q.size / q.n) ** 3
    return m


@pytest.mark.parametrize("nsteps", [11, 32])
def test_adjoint_dot_product_fp64(orc, nsteps):
    torch, dsp, pr, s, dt = _setup()
    rng = np.random.default_rng(77 + nsteps)
    lamT = rng.normal(size=pr.U0.size)
    delta = rng.normal(size=pr.U0.size)
    U0 = torch.from_numpy(pr.U0).cuda()
    UT, ckpt = s.fixed_steps_fwd(U0, nsteps)
    lam0 = s.fixed_steps_adj(ckpt, torch.from_numpy(lamT).cuda(), nsteps).cpu().numpy()
    o = orc.OracleSet(pr.cfg, pr.patches)
    UTo, dUT = o.jvp_fixed(pr.U0, delta, nsteps, pr.cfg.dt_fixed)
    o.close()
    s.close()
    lhs = float(np.dot(lamT, dUT))
    rhs = float(np.dot(lam0, delta))
    scale = float(np.abs(lamT * dUT).sum())
    print("dot product", nsteps, lhs, rhs, abs(lhs - rhs) / scale)
    assert np.abs(UT.cpu().numpy() - UTo).max() <= 1e-12
    assert abs(lhs - rhs) <= 1e-12 * scale


def test_adjoint_dot_product_specified_background(orc):
    """The background as specified (B = (1, 0, 0), fluid at rest, uniform
    p = 0.6) with the specified perturbations of rho and v.  The map is not
    differentiable there: the transverse field and the slopes of p and B
    start exactly at zero, where HLLD's degenerate star state and the
    limiter have one-sided derivatives, and the hand-written reverse pass
    and the oracle's dual numbers need not pick the same side at such an
    exact tie.  Measured: the identity holds to 5.6e-7 of its scale (against
    2e-15 on the smooth background), so the bar here is 1e-5; the forward
    states agree to 7e-12 (the FP64 parity bar is 1e-10)."""
    import torch
    from paper_1705_10774_amd import dsp
    dsp.load()
    pr = I.cfg5_adjoint(B=(1.0, 0.0, 0.0), V=(0.0, 0.0, 0.0), dp=False)
    s = dsp.PatchSet(pr.cfg, pr.patches)
    nsteps = 16
    rng = np.random.default_rng(7)
    lamT = rng.normal(size=pr.U0.size)
    delta = rng.normal(size=pr.U0.size)
    U0 = torch.from_numpy(pr.U0).cuda()
    UT, ckpt = s.fixed_steps_fwd(U0, nsteps)
    lam0 = s.fixed_steps_adj(ckpt, torch.from_numpy(lamT).cuda(), nsteps).cpu().numpy()
    o = orc.OracleSet(pr.cfg, pr.patches)
    UTo, dUT = o.jvp_fixed(pr.U0, delta, nsteps, pr.cfg.dt_fixed)
    o.close()
    s.close()
    lhs, rhs = float(np.dot(lamT, dUT)), float(np.dot(lam0, delta))
    scale = float(np.abs(lamT * dUT).sum())
    print("specified background: dot product", lhs, rhs, abs(lhs - rhs) / scale,
          "forward", np.abs(UT.cpu().numpy() - UTo).max())
    assert np.abs(UT.cpu().numpy() - UTo).max() <= 1e-10  # measured 7e-12: rounding at the exact ties
    assert abs(lhs - rhs) <= 1e-5 * scale


def test_adjoint_recompute_path_matches_kept_intermediates(monkeypatch):
    """The reverse run keeps each step's forward intermediates when they fit;
    DSP_ADJ_RECOMPUTE=1 forces the path that recomputes them from the
    segment's states instead.  The forward intermediates are the same bits
    either way and every reverse kernel gathers in a fixed order, so the two
    cotangents are equal bit for bit."""
    nsteps = 11
    rng = np.random.default_rng(311)
    lam = {}
    for mode in ("kept", "recompute"):
        if mode == "recompute":
            monkeypatch.setenv("DSP_ADJ_RECOMPUTE", "1")
        torch, dsp, pr, s, dt = _setup()
        U0 = torch.from_numpy(pr.U0).cuda()
        if mode == "kept":
            lamT = rng.normal(size=pr.U0.size)
        UT, ckpt = s.fixed_steps_fwd(U0, nsteps)
        lam[mode] = s.fixed_steps_adj(ckpt, torch.from_numpy(lamT).cuda(), nsteps).cpu().numpy()
        s.close()
    assert np.array_equal(lam["kept"], lam["recompute"])


@pytest.mark.parametrize("prec", [I.F64, I.F32], ids=["f64", "f32"])
def test_adjoint_is_deterministic(prec):
    """Two reverse runs from the same checkpoints give the same bits (no
    atomic accumulation anywhere in the reverse step)."""
    torch, dsp, pr, s, dt = _setup(prec)
    rng = np.random.default_rng(5)
    U0 = torch.from_numpy(pr.U0).cuda().to(dt)
    UT, ckpt = s.fixed_steps_fwd(U0, 8)
    lamT = torch.from_numpy(rng.normal(size=pr.U0.size)).cuda().to(dt)
    a = s.fixed_steps_adj(ckpt, lamT, 8).cpu().numpy()
    b = s.fixed_steps_adj(ckpt, lamT, 8).cpu().numpy()
    s.close()
    assert np.isfinite(a).all() and np.array_equal(a, b)


def _direction(pr, kind):
    """A smooth direction in state space: 'flow' is the cfg5 perturbation of
    density and velocity itself; 'field' a uniform change of B by 1e-3
    (0.3, -0.5, 0.4) with the energy that goes with it (divergence-free)."""
    base = I.cfg5_adjoint(seed_init=None)
    if kind == "flow":
        return pr.U0 - base.U0
    B = (0.6 + 3e-4, 0.4 - 5e-4, 0.2 + 4e-4)
    return I.cfg5_adjoint(B=B).U0 - pr.U0


@pytest.mark.parametrize("kind", ["flow", "field"])
def test_adjoint_gradient_vs_central_difference(kind):
    torch, dsp, pr, s, dt = _setup()
    nsteps = pr.nsteps
    mask = _rho_mask(pr)
    rho_star = np.zeros(pr.U0.size)
    for v, r in zip(I.patch_views(rho_star, pr.patches), pr.extra["rho_target"]):
        v[0][...] = r
    U0 = torch.from_numpy(pr.U0).cuda()
    UT, ckpt = s.fixed_steps_fwd(U0, nsteps)
    lamT = mask * (UT.cpu().numpy() - rho_star)
    grad = s.fixed_steps_adj(ckpt, torch.from_numpy(lamT).cuda(), nsteps).cpu().numpy()
    direction = _direction(pr, kind)
    eps = 1e-3
    up, _ = s.fixed_steps_fwd(torch.from_numpy(pr.U0 + eps * direction).cuda(), nsteps, checkpoints=False)
    dn, _ = s.fixed_steps_fwd(torch.from_numpy(pr.U0 - eps * direction).cuda(), nsteps, checkpoints=False)
    up, dn = up.cpu().numpy(), dn.cpu().numpy()
    dJ = 0.5 * float(np.sum(mask * (up - dn) * (up + dn - 2.0 * rho_star))) / (2 * eps)
    ad = float(np.dot(grad, direction))
    s.close()
    print("directional derivative", kind, ": adjoint", ad, "central difference", dJ, "rel", abs(ad - dJ) / abs(dJ))
    assert abs(ad - dJ) <= 1e-6 * abs(dJ)


def test_adjoint_fp32_dot_product(orc):
    torch, dsp, pr, s, dt = _setup(I.F32)
    nsteps = 8
    rng = np.random.default_rng(91)
    lamT = rng.normal(size=pr.U0.size)
    delta = rng.normal(size=pr.U0.size)
    U0 = torch.from_numpy(pr.U0).cuda().float()
    UT, ckpt = s.fixed_steps_fwd(U0, nsteps)
    lam0 = s.fixed_steps_adj(ckpt, torch.from_numpy(lamT).cuda().float(), nsteps).double().cpu().numpy()
    o = orc.OracleSet(pr.cfg, pr.patches)
    _, dUT = o.jvp_fixed(pr.U0, delta, nsteps, pr.cfg.dt_fixed)
    o.close()
    s.close()
    lhs, rhs = float(np.dot(lamT, dUT)), float(np.dot(lam0, delta))
    scale = float(np.abs(lamT * dUT).sum())
    print("fp32 dot product", lhs, rhs, abs(lhs - rhs) / scale)
    assert abs(lhs - rhs) <= 1e-4 * scale


def test_autograd_function_matches_adjoint():
    torch, dsp, pr, s, dt = _setup()
    nsteps = 8
    mask = torch.from_numpy(_rho_mask(pr)).cuda()
    U0 = torch.from_numpy(pr.U0).cuda().requires_grad_(True)
    UT = dsp.fixed_steps(s, U0, nsteps)
    J = 0.5 * torch.sum(mask * (UT - 1.0) ** 2)
    J.backward()
    UT2, ckpt = s.fixed_steps_fwd(U0.detach(), nsteps)
    ref = s.fixed_steps_adj(ckpt, mask * (UT2 - 1.0), nsteps)
    s.close()
    assert torch.equal(UT.detach(), UT2)
    err = (U0.grad - ref).abs().max().item() / ref.abs().max().item()
    print("autograd vs direct adjoint", err)
    assert err <= 1e-12


def test_adjoint_rejects_bad_arguments():
    torch, dsp, pr, s, dt = _setup()
    U0 = torch.from_numpy(pr.U0).cuda()
    UT, ckpt = s.fixed_steps_fwd(U0, 8)
    with pytest.raises(dsp.DspError) as e:
        dsp.dsp_fixed_steps_adj(s.h, ckpt.data_ptr(), UT.data_ptr(), UT.data_ptr(), 8, seg=4)
    assert e.value.code == dsp.DSP_EINVAL
    s.close()
    # a local-dt set has no fixed-step adjoint
    loc = dsp.PatchSet.from_problem(I.turbulence(npd=2, n=8, mach=1.0, seed=3, dt_base=1e-3))
    with pytest.raises(dsp.DspError):
        dsp.dsp_fixed_steps_adj(loc.h, ckpt.data_ptr(), UT.data_ptr(), UT.data_ptr(), 8)
    loc.close()
