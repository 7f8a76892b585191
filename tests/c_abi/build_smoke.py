"""Build the C caller of the library (``abi_smoke``) with gcc as C99: the
header, the library and the HIP runtime's C API are all it uses.  Run by
``__graft_entry__.build()`` after the library itself."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "abi_smoke.c")
EXE = os.path.join(HERE, "abi_smoke")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def c_flags():
    return ["-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
            "-D__HIP_PLATFORM_AMD__", "-isystem", os.path.join(ROCM, "include"),
            "-I", os.path.join(ROOT, "include")]


def build() -> str:
    pkg = os.path.join(ROOT, "paper_2306_09537_amd")
    tmp = EXE + ".tmp"
    subprocess.check_call(["gcc", *c_flags(), SRC, "-o", tmp,
                           "-L", pkg, "-lquadswarm", "-Wl,-rpath,$ORIGIN/../../paper_2306_09537_amd",
                           "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
                           "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-lm"])
    os.replace(tmp, EXE)
    return EXE


if __name__ == "__main__":
    print(build())
