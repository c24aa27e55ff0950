"""Build the host checks: admission_check (the serving loop's admission
bookkeeping) and capi_check (host paths of the C ABI through a library
whose host code carries address and undefined-behaviour sanitizers).

    python tests/host/build_checks.py      # binaries in tests/host/_build/
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "_build")
CLANG = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang++")
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-g", "-O1", "-std=c++17"]


def build():
    sys.path.insert(0, ROOT)
    from paper_1904_10585_amd.build import build as build_lib
    os.makedirs(OUT, exist_ok=True)
    subprocess.run([CLANG] + SAN + [os.path.join(HERE, "admission_check.cpp"), "-o",
                                    os.path.join(OUT, "admission_check")], check=True)
    lib = build_lib(sanitize=True)
    libdir = os.path.dirname(lib)
    subprocess.run([CLANG] + SAN + [os.path.join(HERE, "capi_check.cpp"), "-o", os.path.join(OUT, "capi_check"),
                                    "-L", libdir, "-lpfx_san", f"-Wl,-rpath,{libdir}",
                                    "-L", "/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"], check=True)
    return OUT


if __name__ == "__main__":
    print(build())
