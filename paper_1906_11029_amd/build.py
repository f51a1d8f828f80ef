"""Build the MTP C-ABI shared library (libmtp.so) for gfx950 with hipcc.

Usage: python -m paper_1906_11029_amd.build   (or call build())
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libmtp.so")
SOURCES = ["mesh.cpp", "pitch.cpp", "refelem.cpp", "dag.cpp", "capi.cpp", "tune.cpp", "curved.cpp",
           "tent_kernel.hip", "tent_mfma.hip",
           "tent_mfma_2d_p12.hip", "tent_mfma_2d_p3.hip", "tent_mfma_2d_p4.hip", "tent_mfma_2d_p5.hip",
           "tent_mfma_3d_p1.hip", "tent_mfma_3d_p2.hip", "tent_mfma_3d_p3.hip", "tent_mfma_3d_p4_f64.hip",
           "tent_mfma_3d_p4_f32.hip", "tent_mfma_3d_p5.hip", "noalloc.hip", "tent_curved.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         # packed FP32 instructions off for all device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-ffp-contract=fast", "-Wall", "-Wno-unused-function", "-I" + INCLUDE]


def build(verbose=False, jobs=8):
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [HIPCC] + FLAGS + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            failed.append((src, out.decode()))
        elif verbose and out:
            print(out.decode())
    if failed:
        msg = "\n".join(f"--- {s}\n{o}" for s, o in failed)
        raise RuntimeError("hipcc failed:\n" + msg)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
