"""Build libsdme.so in-tree for gfx950 (hipcc) -- the package's only native
artefact.  ``python -m paper_2104_13466_amd.build`` or ``build()``."""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libsdme.so")
BUILD = os.path.join(ROOT, "_build")

HIP_SOURCES = ["elem_dispatch.hip", "vec_kernels.hip", "load_kernels.hip", "condense_kernels.hip",
               "assemble_kernels.hip", "api.hip"]
# element kernels: one translation unit per polynomial order
ORDERS = range(1, 9)
HOST_SOURCES = ["basis.cpp"]

ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.environ.get("HIPCC", os.path.join(ROCM, "bin", "hipcc"))
HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
    # packed FP32 VALU ops stay off (hipcc device-side feature flag)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed: %s\n%s" % (" ".join(cmd), r.stdout))
    return r.stdout


def build(verbose=False, jobs=None):
    os.makedirs(BUILD, exist_ok=True)
    cmds = []
    objs = []
    for s in HIP_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        objs.append(o)
        cmds.append([HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, s), "-o", o])
    for p in ORDERS:
        o = os.path.join(BUILD, "elem_kernels_p%d.o" % p)
        objs.append(o)
        cmds.append([HIPCC] + HIP_FLAGS + ["-DSDME_P=%d" % p, "-c",
                                           os.path.join(CSRC, "elem_kernels.hip"), "-o", o])
    for s in HOST_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        objs.append(o)
        cmds.append(["g++"] + HOST_FLAGS + ["-c", os.path.join(CSRC, s), "-o", o])
    jobs = jobs or min(len(cmds), os.cpu_count() or 1, 16)
    with cf.ThreadPoolExecutor(jobs) as ex:
        for out in ex.map(_run, cmds):
            if verbose and out.strip():
                print(out)
    tmp = OUT + ".tmp%d" % os.getpid()
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs +
         ["-L" + os.path.join(ROCM, "lib"), "-lrocprofiler-sdk-roctx",
          "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
