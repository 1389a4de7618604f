"""Builds libpsc.so (the C-ABI library: IR, schedulers, HIP and AQL dispatchers and gfx950 kernels)
in place.

Usage: python paper_2009_07482_amd/build.py  (run as a script: importing the package would load
the previous libpsc.so), or __graft_entry__.build().  Every source is compiled
with hipcc for gfx950 into _build/, then linked into paper_2009_07482_amd/libpsc.so.

The AQL dispatcher loads the kernels' gfx950 code object itself: it is taken out of the fat binary
that hipcc embedded in kernels.hip.o (the object the HIP path runs) into libpsc_kernels.hsaco, and
its kernel metadata (the size of each kernel's explicit argument record and the offsets and kinds
of the implicit arguments) is written to libpsc_kernels.kargs, one kernel per line.
"""
import os
import subprocess
import sys

import yaml
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libpsc.so")
BUILD = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are disabled for all device code.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]

SOURCES = ["dag.cpp", "spec.cpp", "sched.cpp", "dispatch.cpp", "capi.cpp", "runtime.cpp", "aql.cpp", "persist.cpp", "kernels.hip",
           "mlp.hip", "persistent.hip"]
LLVM = "/opt/rocm/llvm/bin"
HSACO = os.path.join(PKG, "libpsc_kernels.hsaco")
KARGS = os.path.join(PKG, "libpsc_kernels.kargs")
# implicit argument kinds the AQL dispatcher fills (codes shared with csrc/aql.cpp)
HIDDEN = {"hidden_block_count_x": 1, "hidden_block_count_y": 2, "hidden_block_count_z": 3,
          "hidden_group_size_x": 4, "hidden_group_size_y": 5, "hidden_group_size_z": 6,
          "hidden_remainder_x": 7, "hidden_remainder_y": 8, "hidden_remainder_z": 9,
          "hidden_global_offset_x": 10, "hidden_global_offset_y": 11, "hidden_global_offset_z": 12,
          "hidden_grid_dims": 13}


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd)} failed:\n{r.stderr}")
    return r.stdout


def code_object(kernels_obj):
    """libpsc_kernels.hsaco (the gfx950 code object inside kernels.hip.o) and its argument table."""
    fat = os.path.join(BUILD, "kernels.fatbin")
    _run([os.path.join(LLVM, "llvm-objcopy"), f"--dump-section=.hip_fatbin={fat}", kernels_obj,
          os.path.join(BUILD, "kernels.strip.o")])
    tmp = HSACO + ".tmp"
    _run([os.path.join(LLVM, "clang-offload-bundler"), "--type=o", "--targets=hipv4-amdgcn-amd-amdhsa--gfx950",
          f"--input={fat}", f"--output={tmp}", "--unbundle"])
    notes = _run([os.path.join(LLVM, "llvm-readelf"), "--notes", tmp])
    i = notes.index("---")
    meta = yaml.safe_load(notes[i:notes.index("\n...", i) + 4])
    lines = []
    for k in meta["amdhsa.kernels"]:
        explicit, hidden = 0, []
        for a in k.get(".args", []):
            kind = a[".value_kind"]
            if kind.startswith("hidden_"):
                hidden.append(f"{a['.offset']}:{HIDDEN.get(kind, 0)}")
            else:
                explicit = max(explicit, a[".offset"] + a[".size"])
        lines.append(f"{k['.name']} {explicit} {len(hidden)} {' '.join(hidden)}".rstrip())
    with open(KARGS + ".tmp", "w") as fh:
        fh.write("\n".join(lines) + "\n")
    os.replace(tmp, HSACO)
    os.replace(KARGS + ".tmp", KARGS)
    return len(lines)


def _compile(src):
    obj = os.path.join(BUILD, src + ".o")
    cmd = [HIPCC] + FLAGS + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in (r.stderr or "").splitlines()
                    if "is not a recognized feature for this target" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{err}")
    return obj, err


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        results = list(ex.map(_compile, SOURCES))
    for (obj, err) in results:
        if err.strip() and verbose:
            print(err, file=sys.stderr)
    n_kernels = code_object(os.path.join(BUILD, "kernels.hip.o"))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [o for o, _ in results] + \
          ["-L/opt/rocm/lib", "-lhsa-runtime64", "-ldl"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT} and {os.path.basename(HSACO)} ({n_kernels} kernels)")
    return OUT


if __name__ == "__main__":
    build()
