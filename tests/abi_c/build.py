"""Builds solve_example (a C program that uses libdpm through its C ABI only) next to this file."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
PKG = os.path.join(ROOT, "paper_1811_03557_amd")
EXE = os.path.join(HERE, "solve_example")


def build() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    # plain C: gcc against the HIP runtime's C API; libdpm found next to the package ($ORIGIN)
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(rocm, "include"),
           os.path.join(HERE, "solve_example.c"), "-L" + PKG, "-ldpm",
           "-Wl,-rpath,$ORIGIN/../../paper_1811_03557_amd", "-L" + os.path.join(rocm, "lib"),
           "-lamdhip64", "-Wl,-rpath," + os.path.join(rocm, "lib"), "-lm", "-o", EXE]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("building solve_example failed:\n" + r.stderr)
    return EXE


if __name__ == "__main__":
    print(build())
