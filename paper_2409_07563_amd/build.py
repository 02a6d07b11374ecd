"""Build libmppi.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmppi.so")
# measured ceilings for the benchmark (not part of the MPPI path)
CEIL_LIB = os.path.join(HERE, "libmppi_ceilings.so")
CEIL_SOURCES = ["ceilings.hip"]
SOURCES = ["mppi.hip", "noise.hip", "rollout.hip", "rollout_scan.hip", "rollout_tiles.hip",
           "softmin.hip", "batch.hip", "adjoint.hip", "split.hip", "controls.hip"]
ARCH = os.environ.get("MPPI_OFFLOAD_ARCH", "gfx950")

# -packed-fp32-ops: keep the compiler from emitting packed FP32 VALU
# instructions (v_pk_fma_f32 and friends).
HIPCC_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               f"-I{os.path.join(ROOT, 'include')}"]


def build(verbose: bool = False, jobs: int = 4, incremental: bool = False) -> str:
    """Compile and link both libraries.  incremental=True recompiles only the
    sources whose object is older than the source or any header (a developer
    shortcut; the default always recompiles everything)."""
    _build_lib(SOURCES, LIB, verbose, jobs, incremental)
    _build_lib(CEIL_SOURCES, CEIL_LIB, verbose, jobs, incremental)
    return LIB


def _headers_mtime():
    paths = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    inc = os.path.join(ROOT, "include")
    paths += [os.path.join(inc, f) for f in os.listdir(inc) if f.endswith(".h")]
    return max(os.path.getmtime(p) for p in paths)


def _build_lib(sources, lib, verbose, jobs, incremental=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    hdr = _headers_mtime() if incremental else None
    for src in sources:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        if incremental and os.path.exists(obj) and os.path.getmtime(obj) > max(
                hdr, os.path.getmtime(os.path.join(CSRC, src))):
            continue
        cmd = [hipcc, *HIPCC_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        if len(procs) >= jobs:
            if procs.pop(0).wait() != 0:
                raise RuntimeError("hipcc failed")
    for p in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed")
    tmp = lib + ".tmp"
    cmd = [hipcc, "-shared", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, jobs=8, incremental="--incremental" in sys.argv))
