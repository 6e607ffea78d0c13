"""Builds tests/c_abi/solve_c, a plain C program that calls the library
through include/srj.h (gcc, host code only; links libsrj.so and the HIP
runtime)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
BINARY = os.path.join(HERE, "solve_c")


def build() -> str:
    libdir = os.path.join(ROOT, "paper_2011_06636_amd")
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROCM, "include"),
           os.path.join(HERE, "solve_c.c"), "-L" + libdir, "-lsrj",
           "-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
           # the library is found relative to the binary wherever the tree lives
           "-Wl,-rpath,$ORIGIN/../../paper_2011_06636_amd",
           "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", BINARY]
    subprocess.run(cmd, check=True)
    return BINARY


if __name__ == "__main__":
    print(build())
