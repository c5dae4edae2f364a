"""Snapshot files (restart): a run saved part-way and restored into a new set
continues bit for bit as the uninterrupted run (state, step counts and level
hashes); mismatching sets and damaged files are refused."""
import numpy as np
import pytest

from paper_1705_10774_amd import inputs as I

pytestmark = pytest.mark.gpu


def _dsp():
    from paper_1705_10774_amd import dsp
    dsp.load()
    return dsp


def spread(prec):
    # 27 patches of 8^3 whose local steps differ (levels 0 and 1)
    return I.turbulence(npd=3, n=8, mach=5.0, seed=5, dt_base=0.02 / 32, prec=prec)


def smr(prec):
    # three refinement levels: guard zones filled across resolutions
    return I.cfg4_smr(prec=prec, n=8)


@pytest.mark.parametrize("make", [spread, smr], ids=["spread", "smr"])
@pytest.mark.parametrize("prec", [I.F64, I.F32], ids=["f64", "f32"])
def test_restart_continues_bitwise(tmp_path, make, prec):
    dsp = _dsp()
    pr = make(prec)
    dtb = pr.cfg.dt_base
    a = dsp.PatchSet.from_problem(pr)
    a.advance_to(2 * dtb)
    f = tmp_path / "snap.bin"
    a.save(f)
    a.advance_to(5 * dtb)
    Ua = a.read_state()
    sa, ka, la = a.read_schedule(klog_cap=64)
    a.close()

    b = dsp.PatchSet.from_problem(pr)  # initial state, then overwritten by the file
    b.load(f)
    b.advance_to(5 * dtb)
    Ub = b.read_state()
    sb, kb, lb = b.read_schedule(klog_cap=64)
    b.close()
    print("steps per patch", sorted(set(sa.tolist())))
    assert sa.min() >= 5
    assert np.array_equal(sa, sb)
    assert np.array_equal(ka, kb)
    assert np.array_equal(la, lb)
    assert np.array_equal(Ua, Ub)


def test_snapshot_refuses_mismatch_and_damage(tmp_path):
    dsp = _dsp()
    pr = spread(I.F64)
    a = dsp.PatchSet.from_problem(pr)
    a.advance_to(pr.cfg.dt_base)
    f = tmp_path / "snap.bin"
    a.save(f)
    U = a.read_state()
    a.close()
    # another precision
    b = dsp.PatchSet.from_problem(spread(I.F32))
    with pytest.raises(dsp.DspError) as e:
        b.load(f)
    assert e.value.code == dsp.DSP_EINVAL
    b.close()
    # other patches
    c = dsp.PatchSet.from_problem(I.turbulence(npd=2, n=8, mach=5.0, seed=5, dt_base=0.02 / 32))
    with pytest.raises(dsp.DspError):
        c.load(f)
    c.close()
    # truncated file, wrong magic, missing file: the set keeps working
    raw = f.read_bytes()
    (tmp_path / "short.bin").write_bytes(raw[: len(raw) // 2])
    (tmp_path / "magic.bin").write_bytes(b"XXXXXXXX" + raw[8:])
    d = dsp.PatchSet.from_problem(pr)
    for name in ("short.bin", "magic.bin", "absent.bin"):
        with pytest.raises(dsp.DspError) as e:
            d.load(tmp_path / name)
        assert e.value.code == dsp.DSP_EINVAL
    d.load(f)
    assert np.array_equal(d.read_state(), U)
    d.close()


@pytest.mark.parametrize("make", [spread, smr], ids=["spread", "smr"])
@pytest.mark.parametrize("prec", [I.F64, I.F32], ids=["f64", "f32"])
def test_restart_matches_oracle(orc, tmp_path, make, prec):
    """A run saved at 2 dt_base, restored into a new set and continued to
    5 dt_base equals the oracle's uninterrupted run: the schedule bit for bit,
    the state within the precision's tolerance (relative L1 and element-wise)."""
    from tests.test_gpu_parity import elem_rel, orc_run, rel_l1, rel_l1_grouped
    dsp = _dsp()
    pr = make(prec)
    dtb = pr.cfg.dt_base
    a = dsp.PatchSet.from_problem(pr)
    a.advance_to(2 * dtb)
    f = tmp_path / "snap.bin"
    a.save(f)
    a.close()
    b = dsp.PatchSet.from_problem(pr)
    b.load(f)
    b.advance_to(5 * dtb)
    Ub = b.read_state()
    sb, kb = b.read_schedule()
    b.close()
    Uo, so, ko, _ = orc_run(orc, pr, t_end=5 * dtb, prec=I.F64)
    assert np.array_equal(sb, so) and np.array_equal(kb, ko)
    err = rel_l1_grouped(Ub, Uo, pr.patches) if make is smr else rel_l1(Ub, Uo, pr.patches)
    el = elem_rel(Ub, Uo, pr.patches)
    print(make.__name__, prec, "restart vs oracle: rel L1", err, "element-wise", el)
    if prec == I.F64:
        assert err <= 1e-10 and el <= 1e-10
    else:
        assert err <= 1e-4
