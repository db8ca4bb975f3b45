"""Build libsldg.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libsldg.so")
SOURCES = [os.path.join(CSRC, f) for f in ("sldg_host.hip", "sldg_batch.hip", "sldg_kernels.hip",
                                          "sldg_ref.hip", "sldg_field.hip", "sldg_colloc.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("sldg_internal.h", "ab_poly.h", "sldg_ref.h",
                                          "sldg_field.h", "sldg_colloc.h")] + \
    [os.path.join(ROOT, "include", "sldg.h")]
ARCH = os.environ.get("SLDG_OFFLOAD_ARCH", "gfx950")


def hipcc():
    for cand in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in cand or os.path.exists(cand):
            return cand
    return "hipcc"


def command(out):
    return [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            # packed FP32 instructions stay off (the compiler would form them from
            # float code; this library never needs them)
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC,
            "-o", out] + SOURCES


def up_to_date():
    if not os.path.exists(LIB):
        return False
    t = os.path.getmtime(LIB)
    return all(os.path.getmtime(f) <= t for f in SOURCES + HEADERS)


def build(force=True, verbose=False):
    if not force and up_to_date():
        return LIB
    tmp = LIB + ".tmp"
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose=True))
    sys.exit(0)
