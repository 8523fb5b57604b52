"""Builds liblbm.so (the gfx950 HIP library) in-tree with hipcc."""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "liblbm.so")
EXAMPLE_SRC = os.path.join(PKG, "examples", "lbm_channel.c")
EXAMPLE_BIN = os.path.join(PKG, "examples", "lbm_channel")
SOURCES = [os.path.join(PKG, "csrc", name) for name in
           ("lbm.hip", "lattice_d2q9.hip", "lattice_d3q19.hip", "lattice_d3q27.hip")]
BUILD_DIR = os.path.join(PKG, "_build")

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # Contract a*b+c into FMA only within one expression (C semantics), so the
    # same source expression rounds the same way in every kernel.
    "-ffp-contract=on",
    # No packed-FP32 instructions anywhere in the device code.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def _filtered(text):
    # hipcc's host pass warns that it does not know the packed-fp32 feature.
    return "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)


def build(verbose: bool = False) -> str:
    """Compiles each translation unit to an object in parallel, then links."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
        cmd = [hipcc, *HIPCC_FLAGS, "-c", "-I", os.path.join(ROOT, "include"), "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        jobs.append((cmd, subprocess.Popen(cmd, cwd=PKG, stdout=subprocess.PIPE,
                                           stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    failed = []
    for cmd, proc in jobs:
        out, _ = proc.communicate()
        msg = _filtered(out or "")
        if proc.returncode != 0:
            failed.append(f"{' '.join(cmd)}\n{msg}")
        elif verbose and msg.strip():
            print(msg)
    if failed:
        raise RuntimeError("hipcc failed:\n" + "\n".join(failed))
    link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp", *objs]
    if verbose:
        print(" ".join(link), flush=True)
    res = subprocess.run(link, cwd=PKG, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed ({res.returncode}):\n{_filtered(res.stdout + res.stderr)}")
    os.replace(LIB + ".tmp", LIB)
    build_example(verbose)
    return LIB


def build_example(verbose: bool = False) -> str:
    """Compiles the C99 driver examples/lbm_channel.c against include/lbm.h
    and liblbm.so (plain C compiler; the HIP runtime API header selects the
    AMD platform by the macro hipcc would define)."""
    cc = os.environ.get("CC", "gcc")
    cmd = [cc, "-std=c99", "-O2", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include",
           "-o", EXAMPLE_BIN + ".tmp", EXAMPLE_SRC, "-L", PKG, "-llbm",
           "-L", "/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,$ORIGIN/.."]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"example build failed:\n{res.stdout}{res.stderr}")
    os.replace(EXAMPLE_BIN + ".tmp", EXAMPLE_BIN)
    return EXAMPLE_BIN


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
