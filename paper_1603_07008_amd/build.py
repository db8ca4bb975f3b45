"""Build libsldg.so (HIP, gfx950) in-tree with hipcc.

Every translation unit is compiled to its own object, in parallel, then the
objects are linked.  The sweep kernels' instantiation unit is compiled once
per (degree, storage tier) pair, so the template-heavy part of the library
compiles on several cores.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libsldg.so")
PLAIN = ["sldg_host.hip", "sldg_batch.hip", "sldg_kernels.hip", "sldg_ref.hip", "sldg_field.hip",
         "sldg_colloc.hip"]
INST = "sldg_sweep_inst.hip"
DEGREES = (1, 2, 3)
TIERS = (0, 1, 2, 3)
SOURCES = [os.path.join(CSRC, f) for f in PLAIN + [INST]]
HEADERS = [os.path.join(CSRC, f) for f in ("sldg_internal.h", "sldg_sweep.h", "ab_poly.h",
                                          "sldg_ref.h", "sldg_field.h", "sldg_colloc.h",
                                          "sldg_fused.h", "sldg_staged.h")] + \
    [os.path.join(ROOT, "include", "sldg.h")]
ARCH = os.environ.get("SLDG_OFFLOAD_ARCH", "gfx950")


def hipcc():
    for cand in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in cand or os.path.exists(cand):
            return cand
    return "hipcc"


def _flags():
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            # packed FP32 instructions stay off (the compiler would form them from
            # float code; this library never needs them)
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def units():
    """(source, object, extra defines) of every translation unit."""
    out = []
    for f in PLAIN:
        out.append((os.path.join(CSRC, f), os.path.join(OBJ, f[:-4] + ".o"), []))
    for k in DEGREES:
        for t in TIERS:
            out.append((os.path.join(CSRC, INST), os.path.join(OBJ, f"sldg_sweep_k{k}_t{t}.o"),
                        [f"-DSLDG_K={k}", f"-DSLDG_TIER={t}"]))
    return out


def command(out):
    """The compile commands of every unit and the link command."""
    cmds = [[hipcc()] + _flags() + d + ["-c", "-o", o, s] for s, o, d in units()]
    link = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out] + \
        [o for _, o, _ in units()]
    return cmds, link


def up_to_date():
    if not os.path.exists(LIB):
        return False
    t = os.path.getmtime(LIB)
    return all(os.path.getmtime(f) <= t for f in SOURCES + HEADERS)


def _jobs():
    for var in ("MAX_JOBS", "CMAKE_BUILD_PARALLEL_LEVEL"):
        v = os.environ.get(var)
        if v and v.isdigit() and int(v) > 0:
            return min(int(v), 16)
    return max(1, min(len(os.sched_getaffinity(0)), 16))


def build(force=True, verbose=False):
    """Compile every unit (force) or only those older than a source or header,
    then link libsldg.so."""
    if not force and up_to_date():
        return LIB
    os.makedirs(OBJ, exist_ok=True)
    tmp = LIB + ".tmp"
    cmds, link = command(tmp)
    newest_hdr = max(os.path.getmtime(h) for h in HEADERS)

    def stale(cmd):
        obj, src = cmd[-2], cmd[-1]
        if force or not os.path.exists(obj):
            return True
        return os.path.getmtime(obj) < max(os.path.getmtime(src), newest_hdr)

    todo = [c for c in cmds if stale(c)]
    if verbose:
        print(f"compiling {len(todo)} of {len(cmds)} units on {_jobs()} jobs", flush=True)

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        return cmd, r.returncode, r.stdout

    failed = []
    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        for cmd, rc, log in ex.map(run, todo):
            # the host pass does not know the packed-FP32 feature flag: harmless
            lines = [ln for ln in log.splitlines() if "packed-fp32-ops" not in ln]
            if lines and (verbose or rc):
                print("\n".join(lines), flush=True)
            if rc:
                failed.append(cmd[-1])
    if failed:
        raise subprocess.CalledProcessError(1, f"hipcc failed on {failed}")
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--incremental" not in sys.argv, verbose=True))
    sys.exit(0)
