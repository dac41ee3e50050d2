"""Build the HIP library liblbm_sc.so for gfx950 in-tree with hipcc: every translation unit is
compiled in parallel (the fused step kernels are split into one unit per precision), then linked."""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm_sc.so")
OBJ = os.path.join(HERE, "_build")
SOURCES = [os.path.join(CSRC, n) for n in ("step_f32.hip", "step_m64.hip", "step_f64.hip",
                                            "kernels.hip", "lbm_sc.hip")]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # packed FP32 instructions are kept out of the generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def compile_command(src, obj):
    return [hipcc(), *FLAGS, "-I", os.path.join(os.path.dirname(HERE), "include"), "-c", src,
            "-o", obj]


def link_command(objs, out):
    return [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", out]


def build(verbose=False):
    """Compile every source (always, also when a library is already there) and link."""
    os.makedirs(OBJ, exist_ok=True)
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(OBJ, os.path.basename(src) + ".o")
        cmd = compile_command(src, obj)
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd)))
        objs.append(obj)
    failed = [src for src, p in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, "hipcc -c " + " ".join(failed))
    tmp = LIB + ".tmp"
    cmd = link_command(objs, tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
