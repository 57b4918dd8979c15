"""Build step of the HIP library: hipcc for gfx950, in-tree libhhg.so."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhhg.so")
SOURCES = ["hhg_kernels.hip", "hhg_learned.hip", "hhg_ctx.hip", "hhg2d.hip"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         # no packed-FP32 instructions (some of their forms have given silently
         # wrong results on this hardware)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # matrix-core results in ordinary VGPRs (no accumulation-register
         # copies after each product in the learned-correction kernels)
         "-mllvm", "-amdgpu-mfma-vgpr-form",
         "-I", os.path.join(ROOT, "include")]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def build(verbose=False):
    """Compile every HIP source into paper_1709_06793_amd/libhhg.so (always rebuilds)."""
    tmp = LIB + ".tmp"
    cmd = ["hipcc"] + FLAGS + ["-o", tmp] + sources()
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stderr[-6000:])
    if verbose and res.stderr:
        print(res.stderr[-2000:])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
