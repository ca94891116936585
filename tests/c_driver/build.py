"""Build the C driver of the library (tests/c_driver/gbr_c_driver) with the
host C compiler: include/gbr.h and the HIP runtime API headers, linked
against the in-tree libgbr.so and the system HIP runtime."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
PKG = os.path.join(ROOT, "paper_2305_00762_amd")
EXE = os.path.join(HERE, "gbr_c_driver")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"),
           os.path.join(HERE, "gbr_c_driver.c"), "-o", EXE + ".tmp",
           # the library is found next to the tree wherever the tree is copied
           "-L", PKG, "-lgbr", "-Wl,-rpath,$ORIGIN/../../paper_2305_00762_amd",
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(EXE + ".tmp", EXE)
    return EXE


if __name__ == "__main__":
    build(verbose=True)
