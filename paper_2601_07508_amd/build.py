"""Builds libmmp.so (HIP, gfx950) in the package directory.

Every source under csrc/ is compiled by hipcc for gfx950 only, in parallel,
then linked into one shared library.  Device code is built without fast-math
and with floating-point contraction off: the modular reductions rely on
explicit fma and on each operation being rounded on its own.
"""
import concurrent.futures
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmmp.so")
OBJDIR = os.path.join(ROOT, "_build", "mmp")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(HERE, "csrc"),
    "-Wno-unused-command-line-argument",
    # MFMA accumulators in ordinary VGPRs: the in-loop reductions are VALU
    # work on those accumulators, and AGPR copies would double it.
    "-mllvm", "-amdgpu-mfma-vgpr-form",
]


# (u, v) word pairs the FP64-word kernel is instantiated for (u, v <= 4, uv <= 8).
WORD_PAIRS = [(1, 1), (1, 2), (2, 1), (1, 3), (3, 1), (2, 2), (1, 4), (4, 1), (2, 3), (3, 2),
              (2, 4), (4, 2)]
PER_PAIR = {"mmp_fp64_words.hip"}  # compiled once per word pair
PER_DIGITS = {"mmp_int8_digits.hip"}  # compiled once per digit count 1..8


def sources():
    """(source, extra flags, object name) for every compile job."""
    out = []
    for src in sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")) +
                      glob.glob(os.path.join(HERE, "csrc", "*.cpp"))):
        base = os.path.basename(src)
        if base in PER_PAIR:
            for u, v in WORD_PAIRS:
                out.append((src, [f"-DMMP_U={u}", f"-DMMP_V={v}"], f"{base}.{u}{v}.o"))
        elif base in PER_DIGITS:
            for d in range(1, 9):
                out.append((src, [f"-DMMP_D={d}"], f"{base}.{d}.o"))
        else:
            out.append((src, [], base + ".o"))
    return out


def _compile(job):
    src, extra, name = job
    obj = os.path.join(OBJDIR, name)
    cmd = [HIPCC] + FLAGS + extra + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{err}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = sources()
    jobs = min(len(srcs), max(1, min(16, os.cpu_count() or 1)))
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
