"""Build the wgrid HIP library (libwgrid.so, gfx950) in-tree with hipcc.

The gridder/degridder kernels of each kernel support are a translation unit
of their own (csrc/vis_launch.hip with -DWG_ALPHA=N), compiled in parallel
with the rest; the objects are then linked into one shared library.
"""
import concurrent.futures
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libwgrid.so")
SUPPORTS = list(range(4, 17))
HEADERS = ["device_common.hpp", "fft_lds.hpp", "kernels_apply.hpp", "kernels_index.hpp", "host_math.hpp",
           "plan_internal.hpp", "vis_launch.hpp", "kernel_table_search.inc"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off: some of their forms have returned
    # wrong results on this hardware, without any error
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _units():
    units = [("wgrid.o", os.path.join(CSRC, "wgrid.hip"), []),
             ("host_math.o", os.path.join(CSRC, "host_math.cpp"), [])]
    for a in SUPPORTS:
        units.append((f"vis_a{a}.o", os.path.join(CSRC, "vis_launch.hip"), [f"-DWG_ALPHA={a}"]))
    return units


def _compile(unit, verbose):
    name, src, extra = unit
    out = os.path.join(OBJ, name)
    cmd = ["hipcc"] + FLAGS + extra + ["-c", src, "-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {name}:\n" + res.stdout + res.stderr)
    os.replace(out + ".tmp", out)
    return out


def build(verbose=False, jobs=None):
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or max(1, min(16, len(os.sched_getaffinity(0))))
    units = _units()
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda u: _compile(u, verbose), units))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
