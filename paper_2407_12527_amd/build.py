"""Build librom.so (gfx950) in-tree with hipcc.

    python -m paper_2407_12527_amd.build

Device code is compiled for gfx950 only, with packed-FP32 instruction selection switched off;
host code is compiled without floating-point contraction so that generated ordinate sets are
reproducible bit for bit.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librom.so")
BUILD = os.path.join(HERE, "_build")
ARCH = os.environ.get("ROM_OFFLOAD_ARCH", "gfx950")

DEVICE_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-builtin-sin", "-fno-builtin-cos", "-D__HIP_PLATFORM_AMD__",
              "-I/opt/rocm/include", "-x", "c++"]


def _hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops' is not a recognized" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"build step failed: {' '.join(cmd)}\n{out}")
    return out


def _stale(src: str, obj: str) -> bool:
    """An object is stale when it is missing or older than its source or any header of csrc/."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [src] + [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")]
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose: bool = False, out: str = LIB, defines=(), incremental: bool = False) -> str:
    """Compile every source under csrc/ and link `out` (default: the in-tree librom.so).
    `defines` are extra -D flags for the device sources (build variants for A/B timing);
    `incremental` recompiles only sources whose objects are stale."""
    build_dir = BUILD if not defines else BUILD + "_" + "_".join(d.replace("=", "") for d in defines)
    os.makedirs(build_dir, exist_ok=True)
    hipcc = _hipcc()
    jobs = []
    objs = []
    for src in sorted(os.listdir(CSRC)):
        path = os.path.join(CSRC, src)
        obj = os.path.join(build_dir, src + ".o")
        if src.endswith(".hip"):
            cmd = [hipcc, *DEVICE_FLAGS, *[f"-D{d}" for d in defines], "-c", path, "-o", obj]
        elif src.endswith(".cpp"):
            cmd = [hipcc, *HOST_FLAGS, "-c", path, "-o", obj]
        else:
            continue
        objs.append(obj)
        if not incremental or _stale(path, obj):
            jobs.append(cmd)
    with cf.ThreadPoolExecutor(max_workers=max(1, min(8, len(jobs)))) as ex:
        for log in ex.map(_run, jobs):
            if verbose and log.strip():
                print(log)
    tmp = out + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv))
