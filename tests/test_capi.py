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


STRUCTS = (("dsp_config", dsp.dsp_config), ("dsp_patch_desc", dsp.dsp_patch_desc),
           ("dsp_allocator", dsp.dsp_allocator))


def test_struct_layout_matches_header(tmp_path):
    """Size and every field offset of the binding's structures against the C
    compiler's layout of include/dsp.h."""
    import subprocess
    lines = []
    for cname, ct in STRUCTS:
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in ct._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "dsp.h"\nint main(void) {\n' +
                   "\n".join(lines) + "\nreturn 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    want = []
    for cname, ct in STRUCTS:
        want.append(f"{cname} size {C.sizeof(ct)}")
        for f, _ in ct._fields_:
            want.append(f"{cname} {f} {getattr(ct, f).offset}")
    assert [g for g in got if g] == want


@pytest.mark.parametrize("bad", [dict(grace=1.0), dict(grace=-0.1), dict(grace=0.5, nslots=2),
                                 dict(grace=0.5, dt_mode=2), dict(periodic=(1, 0, 1)), dict(nguard=1),
                                 dict(limiter=1), dict(kmax=41), dict(nslots=1), dict(prec=3),
                                 dict(dt_base=0.0), dict(gamma=1.0), dict(eta=-1.0), dict(gamma_ad=-1.0),
                                 dict(gamma_ad=1.0, rho_ion=0.0), dict(torder=3), dict(torder=2, nslots=2)])
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


def test_boundary_patches_rejected_on_host():
    """Boundary patches need LOCAL steps, and at least one patch must update."""
    pr = I.cfg2_turb(npd=2)
    p = [I.Patch(q.origin, q.size, q.n, frozen=(m == 0)) for m, q in enumerate(pr.patches)]
    with pytest.raises(dsp.DspError) as e:
        dsp.dsp_create(dataclasses.replace(pr.cfg, dt_mode=I.DT_GLOBAL_EXACT), p)
    assert e.value.code == dsp.DSP_EINVAL
    allf = [I.Patch(q.origin, q.size, q.n, frozen=True) for q in pr.patches]
    with pytest.raises(dsp.DspError) as e:
        dsp.dsp_create(pr.cfg, allf)
    assert e.value.code == dsp.DSP_EINVAL


def test_snapshot_rejects_bad_path_on_host(tmp_path):
    """A missing file is refused before any device work (null set handles too)."""
    L = dsp.load()
    assert L.dsp_load_snapshot(None, str(tmp_path / "absent.bin").encode()) == dsp.DSP_EINVAL
    assert L.dsp_save_snapshot(None, str(tmp_path / "x.bin").encode()) == dsp.DSP_EINVAL
