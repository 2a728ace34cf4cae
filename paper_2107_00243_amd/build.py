"""Build libgpmll.so (HIP, gfx950) in the package directory.

    python -m paper_2107_00243_amd.build

Compiles every .hip source under csrc/ with hipcc for gfx950 only and links one
shared library next to this file.  Runs on a machine without a GPU.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgpmll.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 ALU instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libgpmll.so)")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


# host-side AddressSanitizer and UndefinedBehaviorSanitizer (device code is built as
# usual); the library then needs the sanitizer runtime preloaded into the process
SANITIZE_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-omit-frame-pointer"]


def build(verbose: bool = False, jobs: int | None = None, sanitize: bool = False) -> str:
    cc = hipcc()
    srcs = sources()
    extra = SANITIZE_FLAGS if sanitize else []
    lib = LIB.replace(".so", "_san.so") if sanitize else LIB
    jobs = jobs or min(9, int(os.environ.get("MAX_JOBS", "8")))
    tmp = tempfile.mkdtemp(prefix="gpmll_build_")
    try:
        objs, procs = [], []
        units = []
        for src in srcs:
            if os.path.basename(src) == "k_khat.hip":
                # one translation unit per tile precision (part 0: staging and
                # reduction; 1 BF16x3, 2 FP32, 3 FP64, 4 FP16x3), compiled in parallel
                units += [(src, [f"-DGPMLL_KHAT_PART={p}"], f".part{p}") for p in range(5)]
            else:
                units.append((src, [], ""))
        for src, defs, tag in units:
            obj = os.path.join(tmp, os.path.basename(src) + tag + ".o")
            objs.append(obj)
            cmd = [cc, *HIPCC_FLAGS, *extra, *defs, "-c", src, "-o", obj]
            procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
            if len(procs) >= jobs:
                _drain(procs, verbose)
        _drain(procs, verbose)
        out_tmp = lib + ".tmp"
        cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *extra, "-o", out_tmp, *objs]
        _run(cmd, verbose)
        os.replace(out_tmp, lib)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return lib


def _run(cmd, verbose):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("command failed:\n" + " ".join(cmd) + "\n" + r.stdout)
    if verbose and r.stdout.strip():
        print(r.stdout)


def _drain(procs, verbose):
    errors = []
    for cmd, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            errors.append(" ".join(cmd) + "\n" + out)
        elif verbose and out.strip():
            print(out)
    procs.clear()
    if errors:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errors))


if __name__ == "__main__":
    path = build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv)
    print(path)
