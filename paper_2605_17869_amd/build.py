"""Build the HIP library of the SIFT path for gfx950 (in-tree shared object).

``python -m paper_2605_17869_amd.build`` compiles ``csrc/*.hip`` and
``csrc/*.cpp`` with hipcc into ``libsift_mi355x.so`` next to this file.
"""
from __future__ import annotations

import os
import re
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
CSRC = PKG / "csrc"
LIB = PKG / "libsift_mi355x.so"
# the same sources with bounds checks in the kernels (-DSIFT_DEBUG_BOUNDS)
LIB_BOUNDS = PKG / "libsift_mi355x_bounds.so"
ARCH = "gfx950"

HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # no reassociation or contraction: every fused multiply-add is explicit,
    # so results do not depend on what the optimiser chose per instantiation
    "-ffp-contract=off", "-fno-fast-math",
    # keep the compiler from emitting packed fp32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def hipcc() -> str:
    root = os.environ.get("ROCM_PATH", "/opt/rocm")
    cand = Path(root) / "bin" / "hipcc"
    return str(cand) if cand.exists() else "hipcc"


SMEM_RE = re.compile(r"^\s+(s_(?:load|store|buffer_load|buffer_store|atomic)\w*)\s+(.*)$")


def smem_misaligned(asm_text: str) -> list:
    """Scalar-memory instructions whose immediate byte offset is not a multiple
    of 4.  The scalar memory unit ignores the low two bits of the base
    register, so such an instruction (a misaligned base compensated by an odd
    immediate) reads or writes the wrong dword.  Returns [(kernel, line)]."""
    bad, fn = [], None
    for line in asm_text.splitlines():
        m = re.match(r"^(_Z\w+):", line)
        if m:
            fn = m.group(1)
        m = SMEM_RE.match(line)
        if not m:
            continue
        imm = m.group(2).split(",")[-1].strip()
        try:
            v = int(imm, 16) if imm.startswith("0x") else int(imm)
        except ValueError:
            continue
        if v % 4:
            bad.append((fn, line.strip()))
    return bad


MIX_RE = re.compile(r"^\s+(v_(?:fma|mad)_mix\w*)\s")


def mixed_f16_fma(asm_text: str) -> list:
    """Mixed-precision fused multiply-adds (v_fma_mix*, v_mad_mix*).  The
    compiler may fold an fp16 conversion into the fma that produced its input,
    rounding the exact product-sum to fp16 once instead of the fp32 result; at
    fp16 ties that gives the other neighbour, so levels stored in fp16 would
    depend on how a kernel was compiled.  Returns [(kernel, line)]."""
    bad, fn = [], None
    for line in asm_text.splitlines():
        m = re.match(r"^(_Z\w+):", line)
        if m:
            fn = m.group(1)
        if MIX_RE.match(line):
            bad.append((fn, line.strip()))
    return bad


def device_asm_cmd(src: Path, out: Path, extra=()) -> list:
    return [hipcc(), "-x", "hip", *HIP_FLAGS, *extra, "--offload-device-only", "-S", str(src),
            "-o", str(out)]


def check_smem(asm_files):
    """Fail the build if any kernel has a misaligned scalar-memory immediate
    or a mixed-precision fma."""
    problems, mixed = [], []
    for path in asm_files:
        text = Path(path).read_text()
        problems += smem_misaligned(text)
        mixed += mixed_f16_fma(text)
    if problems:
        lines = "\n".join(f"  {fn}: {ins}" for fn, ins in problems[:20])
        raise RuntimeError(f"scalar memory access with a misaligned immediate offset:\n{lines}")
    if mixed:
        lines = "\n".join(f"  {fn}: {ins}" for fn, ins in mixed[:20])
        raise RuntimeError(f"mixed-precision fma (an fp16 rounding folded into an fma):\n{lines}")


def kernel_source_hash(names=("sift_blur.hip", "sift_device.h", "sift_internal.h")) -> str:
    """Short digest of kernel sources (default: those the blur kernel is built
    from); measured figures recorded for a kernel name the digest they hold for."""
    import hashlib
    h = hashlib.sha256()
    for name in names:
        h.update((CSRC / name).read_bytes())
    return h.hexdigest()[:16]


def _start(verbose: bool, bounds: bool) -> dict:
    """Start the compiles of one library (objects and device assembly)."""
    extra = ["-DSIFT_DEBUG_BOUNDS"] if bounds else []
    out_dir = PKG / ("_build_bounds" if bounds else "_build")
    out_dir.mkdir(exist_ok=True)
    job = {"lib": LIB_BOUNDS if bounds else LIB, "objs": [], "asm": [], "procs": []}
    for src in sorted(CSRC.glob("*.hip")) + sorted(CSRC.glob("*.cpp")):
        obj = out_dir / (src.name + ".o")
        cmd = [hipcc(), "-x", "hip", *HIP_FLAGS, *extra, "-c", str(src), "-o", str(obj)]
        if verbose:
            print(" ".join(cmd), flush=True)
        job["procs"].append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                   stderr=subprocess.STDOUT)))
        job["objs"].append(obj)
        if src.suffix == ".hip":
            asm = out_dir / (src.name + ".s")
            job["procs"].append((src, subprocess.Popen(device_asm_cmd(src, asm, extra),
                                                       stdout=subprocess.PIPE,
                                                       stderr=subprocess.STDOUT)))
            job["asm"].append(asm)
    return job


def _finish(job: dict, verbose: bool) -> Path:
    """Wait for the compiles, lint the device assembly, link the library."""
    failed = []
    for src, pr in job["procs"]:
        out, _ = pr.communicate()
        if pr.returncode != 0:
            failed.append((src, out.decode(errors="replace")))
        elif verbose and out:
            print(out.decode(errors="replace"))
    if failed:
        msg = "\n".join(f"--- {s}\n{o}" for s, o in failed)
        raise RuntimeError(f"hipcc failed:\n{msg}")
    check_smem(job["asm"])
    lib = job["lib"]
    tmp = lib.with_suffix(".so.tmp")
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", str(tmp),
           *map(str, job["objs"])]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


def build_library(verbose: bool = False, bounds: bool = False) -> Path:
    """Compile every source into the shared library (with bounds checks in the
    kernels: the second library); returns its path."""
    return _finish(_start(verbose, bounds), verbose)


def build_all(verbose: bool = False) -> list:
    """Both libraries, their compiles run side by side; returns their paths."""
    jobs = [_start(verbose, False), _start(verbose, True)]
    return [_finish(j, verbose) for j in jobs]


if __name__ == "__main__":
    for path in build_all(verbose="-v" in sys.argv):
        print(path)
