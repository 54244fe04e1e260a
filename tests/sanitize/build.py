"""Sanitizer builds of the library's host code plus tests/sanitize/host_driver.cpp.

The host-side sources (the planner, the C-ABI checks, batches, the server,
the tuner, the timers, the fixed-workspace entry point) are compiled with
AddressSanitizer + UndefinedBehaviorSanitizer ("asan") or ThreadSanitizer
("tsan"); the kernel sources are linked from the product build
(_build/mmp, written by paper_2601_07508_amd/build.py) as they are, since
nothing here launches a kernel.  The driver and the final link use ROCm's
clang++, whose sanitizer runtimes match the compiler.  Objects go to
_build/sanitize/<kind>/ and are rebuilt when a source or a flag changes.
"""
import concurrent.futures
import hashlib
import importlib.util
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
PKG = os.path.join(ROOT, "paper_2601_07508_amd")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANGXX = "/opt/rocm/llvm/bin/clang++"  # the sanitizer runtimes must match the compiler

SAN = {
    "asan": ["address", "undefined"],
    "tsan": ["thread"],
}


def _lib_sources():
    spec = importlib.util.spec_from_file_location("mmp_build", os.path.join(PKG, "build.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    return b.sources()  # (source, extra defines, object name)


def _host_flags(kind):
    flags = []
    for s in SAN[kind]:
        flags += ["-Xarch_host", "-fsanitize=" + s]
    return flags + ["-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def build(kind, jobs=8):
    out = os.path.join(ROOT, "_build", "sanitize", kind)
    os.makedirs(out, exist_ok=True)
    common = ["-x", "hip", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(PKG, "csrc"),
              "-Wno-unused-command-line-argument"] + _host_flags(kind)

    def one(job):
        src, extra, name = job
        obj = os.path.join(out, name)
        cmd = [HIPCC] + common + extra + ["-c", src, "-o", obj]
        key = hashlib.sha256((" ".join(cmd) + open(src, "rb").read().hex()).encode()).hexdigest()
        for hdr in sorted(os.listdir(os.path.join(PKG, "csrc"))):
            if hdr.endswith(".h"):
                key += hashlib.sha256(open(os.path.join(PKG, "csrc", hdr), "rb").read()).hexdigest()[:8]
        stamp = obj + ".key"
        if os.path.exists(obj) and os.path.exists(stamp) and open(stamp).read() == key:
            return obj
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"{src}: {r.stderr}")
        open(stamp, "w").write(key)
        return obj

    host_side = [j for j in _lib_sources() if j[0].endswith(".cpp") or os.path.basename(j[0]) == "mmp_static.hip"]
    kernels = [os.path.join(ROOT, "_build", "mmp", j[2]) for j in _lib_sources() if j not in host_side]
    missing = [o for o in kernels if not os.path.exists(o)]
    if missing:
        raise RuntimeError("product objects missing (run paper_2601_07508_amd/build.py first): " + missing[0])
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(one, host_side)) + kernels
    exe = os.path.join(out, "host_driver")
    san = ["-fsanitize=" + s for s in SAN[kind]]
    cmd = ([CLANGXX, "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer", "-I" + os.path.join(ROOT, "include")] +
           san + [os.path.join(HERE, "host_driver.cpp")] + objs +
           ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64", "-lpthread", "-o", exe])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link: " + r.stderr)
    return exe


if __name__ == "__main__":
    import sys
    for k in sys.argv[1:] or ["asan", "tsan"]:
        print(build(k))
