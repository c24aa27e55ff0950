"""Build libpfx.so (gfx950) in-tree with hipcc.

    python -m paper_1904_10585_amd.build        # or build() from Python

Objects go to paper_1904_10585_amd/_build/, the library next to this file.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpfx.so")
SOURCES = ["k_contract.hip", "k_filter.hip", "k_small.hip", "k_block.hip", "k_nce.hip", "pipeline.cpp", "capi.cpp",
           "server.cpp", "lanczos.cpp", "nce.cpp", "noalloc.cpp"]
ARCH = "gfx950"


def hipcc():
    for cand in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


# host-side address and undefined-behaviour sanitizers (device code is
# built as usual): the library of the host checks under tests/host
SANITIZE_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def common_flags():
    return [
        "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
        "-Wall", "-Wno-unused-result", "-Wno-unknown-pragmas",
        # no packed FP32 instructions in device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(HERE, "..", "include"),
    ]


def _compile(src, build_dir=BUILD, extra=()):
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + common_flags() + list(extra) + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{errs}")
    return obj, errs


def build(verbose=False, sanitize=False):
    """Build libpfx.so; with sanitize=True instead _build_san/libpfx_san.so,
    whose host code carries the sanitizers (for the host checks only)."""
    build_dir = os.path.join(HERE, "_build_san") if sanitize else BUILD
    lib = os.path.join(build_dir, "libpfx_san.so") if sanitize else LIB
    extra = SANITIZE_FLAGS if sanitize else []
    os.makedirs(build_dir, exist_ok=True)
    jobs = min(len(SOURCES), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda src: _compile(src, build_dir, extra), SOURCES))
    if verbose:
        for _, e in results:
            if e.strip():
                print(e)
    objs = [o for o, _ in results]
    tmp = lib + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
