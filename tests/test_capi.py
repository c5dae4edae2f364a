"""CPU checks of the C ABI: libdsp.so builds for gfx950, loads, exports every
entry point that include/dsp.h declares, and rejects invalid configurations
in host code (before any device work)."""
import ctypes as C
import dataclasses
import os
import re

import pytest

from paper_1705_10774_amd import dsp
from paper_1705_10774_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "dsp.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dsp_[a-z_]+)\s*\(", txt)))


def test_header_matches_binding():
    assert _declared() == sorted(dsp.EXPORTS)


def test_library_exports_every_symbol():
    L = dsp.load()
    for name in _declared():
        assert hasattr(L, name), name


def test_struct_layout_matches_header():
    # 6 doubles, 6 int32, 3 int32, 6 doubles -> 48 + 24 + 12 (+4 pad) + 48
    assert C.sizeof(dsp.dsp_config) == 136
    assert C.sizeof(dsp.dsp_patch_desc) == 56


@pytest.mark.parametrize("bad", [dict(grace=1.0), dict(grace=-0.1), dict(grace=0.5, nslots=2),
                                 dict(grace=0.5, dt_mode=2), dict(periodic=(1, 0, 1)), dict(nguard=1),
                                 dict(limiter=1), dict(kmax=41), dict(nslots=1), dict(prec=3),
                                 dict(dt_base=0.0), dict(gamma=1.0)])
def test_invalid_config_rejected_on_host(bad):
    pr = I.cfg2_turb(npd=2)
    cfg = dataclasses.replace(pr.cfg, **bad)
    with pytest.raises(dsp.DspError) as e:
        dsp.dsp_create(cfg, pr.patches)
    assert e.value.code == dsp.DSP_EINVAL
    assert dsp.load().dsp_last_error()


def test_invalid_geometry_rejected_on_host():
    pr = I.cfg2_turb(npd=2)
    p = list(pr.patches)
    p[1] = I.Patch(p[0].origin, p[0].size, p[0].n)  # overlapping patches
    with pytest.raises(dsp.DspError) as e:
        dsp.dsp_create(pr.cfg, p)
    assert e.value.code == dsp.DSP_EINVAL
    q = list(pr.patches)
    q[0] = I.Patch((0.1, 0.0, 0.0), q[0].size, q[0].n)  # off the lattice / gap
    with pytest.raises(dsp.DspError):
        dsp.dsp_create(pr.cfg, q)
