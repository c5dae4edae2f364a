"""Build libdsp.so (HIP, gfx950) in place: paper_1705_10774_amd/libdsp.so.

Each kernel source is compiled once per precision.  The double-precision
objects are built without floating-point contraction (-ffp-contract=off):
every product and sum rounds on its own, as in the FP64 oracle, so that
expressions that cancel exactly by symmetry (the contact speed of a face on
a mirror plane, for one) cancel on both sides.  The single-precision objects
keep hipcc's default contraction into fused multiply-adds."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
OUT = os.path.join(PKG, "libdsp.so")
F64 = ["-DDSP_TU_F64", "-ffp-contract=off"]
F32 = ["-DDSP_TU_F32"]
# (source, object tag, extra flags)
OBJECTS = [
    ("dsp_kernels.hip", "common", ["-DDSP_TU_COMMON", "-ffp-contract=off"]),
    ("dsp_kernels.hip", "f32", F32),
    ("dsp_kernels.hip", "f64", F64),
    ("dsp_fused.hip", "f32", F32),
    ("dsp_fused.hip", "f64", F64),
    ("dsp_adjoint.hip", "f32", F32),
    ("dsp_adjoint.hip", "f64", F64),
    ("dsp_runtime.hip", "host", ["-ffp-contract=off"]),
]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions (v_pk_*_f32) anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def build(verbose=False, jobs=None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)

    def one(item):
        src, tag, extra = item
        obj = os.path.join(HERE, "_build", f"{src}.{tag}.o")
        cmd = [hipcc] + FLAGS + extra + ["-c", os.path.join(HERE, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        return obj

    jobs = jobs or max(1, min(len(OBJECTS), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(one, OBJECTS))
    tmp = OUT + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.check_call(cmd)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
