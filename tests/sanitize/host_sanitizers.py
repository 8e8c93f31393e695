"""Host AddressSanitizer + UndefinedBehaviorSanitizer run (CPU only).

Builds the library's sources with the sanitizers on the host pass only (the
gfx950 device code is compiled as usual and never runs here) and the oracle
with the same clang, then runs the CPU test suite against those builds with
the clang ASan runtime preloaded into Python.  Any report ends the run with
a non-zero status.

    python tests/sanitize/host_sanitizers.py [pytest args...]

Leak checking is off: the Python interpreter itself keeps allocations alive
at exit.  The builds go to tests/sanitize/_build/.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from paper_2311_09275_amd import build as B  # noqa: E402

OUT = os.path.join(HERE, "_build")
CLANG = "/opt/rocm/llvm/bin/clang"
SAN = ["address", "undefined"]
# every sanitizer flag applies to the host pass only
HOST_SAN = [x for s in SAN for x in ("-Xarch_host", f"-fsanitize={s}")] + [
    "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
    "-Xarch_host", "-g"]


def _compile(src: str) -> str:
    out = os.path.join(OUT, os.path.splitext(src)[0] + ".o")
    flags = [f for f in B.FLAGS if f != "-O3"] + ["-O1"]
    r = subprocess.run(["hipcc", *flags, *HOST_SAN, "-c", os.path.join(B.CSRC, src), "-o", out],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    return out


def build_library() -> str:
    with cf.ThreadPoolExecutor(max_workers=min(len(B.SOURCES), 8)) as ex:
        objs = list(ex.map(_compile, B.SOURCES))
    lib = os.path.join(OUT, "libising.so")
    cmd = ["hipcc", f"--offload-arch={B.ARCH}", "-shared", "-fPIC", "-o", lib, *objs, "-lpthread",
           "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib",
           *HOST_SAN]
    subprocess.run(cmd, check=True)
    return lib


def build_oracle() -> str:
    lib = os.path.join(OUT, "liboracle.so")
    src = os.path.join(ROOT, "oracle", "ising_oracle.c")
    subprocess.run([CLANG, "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-pthread",
                    "-ffp-contract=off", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all",
                    *[f"-fsanitize={s}" for s in SAN], "-o", lib, src, "-lm"], check=True)
    return lib


def main() -> int:
    os.makedirs(OUT, exist_ok=True)
    lib, olib = build_library(), build_oracle()
    rt = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"],
                        capture_output=True, text=True, check=True).stdout.strip()
    env = dict(os.environ)
    env.update({
        "ISING_LIB": lib, "ISING_ORACLE_LIB": olib, "LD_PRELOAD": rt,
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
    })
    args = sys.argv[1:] or [os.path.join(ROOT, "tests"), "-m", "not gpu", "-q", "-p", "no:cacheprovider"]
    print(f"sanitized library {lib}\nsanitized oracle  {olib}\nruntime           {rt}", flush=True)
    return subprocess.run([sys.executable, "-m", "pytest", *args], env=env, cwd=ROOT).returncode


if __name__ == "__main__":
    sys.exit(main())
