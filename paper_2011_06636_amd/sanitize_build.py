"""Host-sanitizer builds of the library's host code and of the CPU oracle.

Usage (CPU only, no GPU needed):
    python -m paper_2011_06636_amd.sanitize_build
then run the CPU tests against the instrumented libraries, one runtime per
process (clang's AddressSanitizer runtime for the HIP library, gcc's for the
oracle), as the printed commands show.

The HIP library is compiled with AddressSanitizer and UndefinedBehavior-
Sanitizer on the host side only (device code is built as usual) into
_build/san/libsrj.so; the oracle with gcc's sanitizers into
_build/san_oracle/liboracle.so.  paper_2011_06636_amd.abi and oracle load
these when SRJ_LIB_PATH / SRJ_ORACLE_LIB name them.
"""
from __future__ import annotations

import concurrent.futures
import glob
import os
import subprocess
import sys

from . import build as libbuild

ROOT = libbuild.ROOT
SAN_DIR = os.path.join(ROOT, "_build", "san")
ORACLE_DIR = os.path.join(ROOT, "_build", "san_oracle")
# host-only instrumentation: each sanitizer flag is preceded by -Xarch_host
HOST_SAN = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined " \
           "-Xarch_host -fno-omit-frame-pointer -Xarch_host -fno-sanitize-recover=undefined".split()


def _compile(src: str) -> str:
    obj = os.path.join(SAN_DIR, os.path.basename(src) + ".o")
    cmd = [libbuild.hipcc(), "-x", "hip", "-c", src, "-o", obj] + libbuild.FLAGS + HOST_SAN
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build_library() -> str:
    os.makedirs(SAN_DIR, exist_ok=True)
    srcs = libbuild.sources()
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    lib = os.path.join(SAN_DIR, "libsrj.so")
    cmd = [libbuild.hipcc(), "-shared", "-o", lib] + objs + \
          [f"--offload-arch={libbuild.ARCH}", "-fPIC", "-shared-libsan"] + HOST_SAN
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    return lib


def build_oracle() -> str:
    os.makedirs(ORACLE_DIR, exist_ok=True)
    srcs = [os.path.join(ROOT, "oracle", "srj_oracle.c"), os.path.join(ROOT, "oracle", "srj_mg.c")]
    lib = os.path.join(ORACLE_DIR, "liboracle.so")
    cmd = ["gcc", "-O1", "-g", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-o", lib] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    return lib


def clang_asan_runtime() -> str:
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise RuntimeError("clang AddressSanitizer runtime not found under /opt/rocm/llvm")
    return hits[-1]


def gcc_asan_runtime() -> str:
    return subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True, check=True).stdout.strip()


def main() -> int:
    lib = build_library()
    orc = build_oracle()
    env = "ASAN_OPTIONS=detect_leaks=0 UBSAN_OPTIONS=halt_on_error=1"
    print(f"built {lib}\nbuilt {orc}\nrun:")
    print(f"  {env} LD_PRELOAD={clang_asan_runtime()} SRJ_LIB_PATH={lib} "
          "python -m pytest tests/test_abi_cpu.py tests/test_solver_checks_cpu.py -q")
    print(f"  {env} LD_PRELOAD={gcc_asan_runtime()} SRJ_ORACLE_LIB={orc} "
          "python -m pytest tests -m 'not gpu' -q -k 'oracle and not abi'")
    return 0


if __name__ == "__main__":
    sys.exit(main())
