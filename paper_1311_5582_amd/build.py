"""Build the HIP library paper_1311_5582_amd/libea_mi355x.so for gfx950.

hipcc cross-compiles for gfx950 without a GPU.  Every build compiles from
source (no caching), so a stale library is never picked up after an edit.
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libea_mi355x.so")
# issue-rate probe behind the roofline pricing (bench.py --valu-rate); not part of the ABI
PROBE_LIB = os.path.join(PKG, "libea_valu_probe.so")
PROBE_SRC = os.path.join(PKG, "csrc", "valu_probe.hip")
SOURCES = [os.path.join(PKG, "csrc", f) for f in ("ea_kernels.hip", "ea_workspace.hip", "ea_api.cpp", "ea_runtime.cpp", "ea_server.cpp")]
ARCH = os.environ.get("EA_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    "-ffp-contract=off",
    # packed FP32 instructions stay off for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"),
]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def build(verbose: bool = False) -> str:
    import concurrent.futures as cf
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(PKG, "csrc", os.path.basename(src) + ".o")
        cmds.append([hipcc()] + HIPCC_FLAGS + ["-x", "hip", "-c", src, "-o", obj])
        objs.append(obj)
    probe_tmp = PROBE_LIB + ".tmp"
    cmds.append([hipcc()] + HIPCC_FLAGS + ["-x", "hip", "-shared", PROBE_SRC, "-o", probe_tmp])
    # the translation units are independent: compile them side by side
    with cf.ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as ex:
        for cmd in cmds:
            if verbose:
                print(" ".join(cmd), flush=True)
        for f in [ex.submit(subprocess.run, cmd, check=True) for cmd in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    os.replace(probe_tmp, PROBE_LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
