"""Build libqfs.so (HIP for gfx950) in-tree with hipcc.

The library is written for gfx950 only.  All device code is compiled with
packed-FP32 instructions disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libqfs.so")
SOURCES = ["qfs_api.cpp", "qfs_batched.hip", "qfs_theta.hip", "qfs_plain.hip", "qfs_reduced.hip", "qfs_diag.hip"]
ARCH = os.environ.get("QFS_OFFLOAD_ARCH", "gfx950")

COMMON = [
    "-O3", "-std=c++20", "-fPIC", "-Wall", "-Wno-unused-function",
    "-fconstexpr-steps=400000000",
    "-I", os.path.join(ROOT, "include"),
]
DEVICE = [
    "--offload-arch=" + ARCH,
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        sys.stderr.write(out + "\n")
        raise RuntimeError("command failed: " + " ".join(cmd))
    return out


def build(jobs=None):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        lang = ["-x", "hip"]
        cmd = ["hipcc", *lang, *COMMON, *DEVICE, "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    failed = False
    for cmd, pr in procs:
        out, _ = pr.communicate()
        out = "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l)
        if pr.returncode != 0:
            sys.stderr.write(out + "\n")
            failed = True
    if failed:
        raise RuntimeError("libqfs compile failed")
    tmp = LIB + ".tmp%d" % os.getpid()
    _run(["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
