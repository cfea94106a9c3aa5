"""Build libraspen.so (HIP for gfx950) in-tree with hipcc.

``python -m paper_2411_00546_amd.build`` compiles every source under csrc/ and
links ``paper_2411_00546_amd/libraspen.so``.  It always recompiles.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libraspen.so")
BUILD = os.path.join(HERE, "_build")
ARCH = os.environ.get("RSP_OFFLOAD_ARCH", "gfx950")

SOURCES = ["kernels_local.hip", "kernels_global.hip", "kernels_factor.hip", "kernels_solve.hip",
           "kernels_gmres.hip", "kernels_coarse.hip", "noalloc.hip", "raspen.cpp", "server.cpp", "tune.cpp"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-x", "hip", "--offload-arch=" + ARCH,
    # packed FP32 instructions are not used (compiler generated forms only, and off)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-function", "-Wno-unknown-warning-option",
]


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found")
    return exe


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj, r.stderr


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(4, len(SOURCES))) as ex:
        results = list(ex.map(_compile, SOURCES))
    objs = [o for o, _ in results]
    if verbose:
        for _, err in results:
            if err.strip():
                sys.stderr.write(err)
    tmp = OUT + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, OUT)
    return OUT


HOST_SOURCES = ["raspen.cpp", "server.cpp", "tune.cpp"]
# host code only: the sanitizers instrument the host pass of each file, never the GPU code
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def build_host_check():
    """Build ``_build/sanitize/host_check``: the host sources (engine, server, tuner)
    with AddressSanitizer and UndefinedBehaviorSanitizer, linked with the kernel objects
    of :func:`build` (compiled if missing) and the CPU driver tests/host/host_check.cpp.
    Returns the executable's path."""
    out_dir = os.path.join(BUILD, "sanitize")
    os.makedirs(out_dir, exist_ok=True)
    jobs = []
    for src in SOURCES:
        if src in HOST_SOURCES:
            jobs.append((os.path.join(CSRC, src), os.path.join(out_dir, os.path.splitext(src)[0] + ".o"), True))
        else:
            obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
            if not os.path.exists(obj) or os.path.getmtime(obj) < os.path.getmtime(os.path.join(CSRC, src)):
                jobs.append((os.path.join(CSRC, src), obj, False))
    jobs.append((os.path.join(ROOT, "tests", "host", "host_check.cpp"), os.path.join(out_dir, "host_check.o"), True))

    def comp(job):
        src, obj, san = job
        cmd = [hipcc()] + FLAGS + (SANITIZE if san else []) + ["-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
        return obj

    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=4) as ex:
        list(ex.map(comp, jobs))
    objs = [os.path.join(out_dir, "host_check.o")]
    for src in SOURCES:
        base = os.path.splitext(src)[0] + ".o"
        objs.append(os.path.join(out_dir if src in HOST_SOURCES else BUILD, base))
    exe = os.path.join(out_dir, "host_check")
    cmd = [hipcc(), "--offload-arch=" + ARCH] + SANITIZE + ["-o", exe] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return exe


if __name__ == "__main__":
    print(build(verbose=True))
