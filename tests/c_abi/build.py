"""Build the plain-C driver of the C ABI (walk_from_c) next to this file."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "walk_from_c.c")
OUT = os.path.join(HERE, "walk_from_c")


def build(out: str = OUT) -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-O2", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(rocm, "include"), "-o", out, SRC,
           "-L", os.path.join(ROOT, "paper_2107_11983_amd"), "-ltrw", "-L", os.path.join(rocm, "lib"), "-lamdhip64",
           "-Wl,-rpath," + os.path.join("$ORIGIN", "..", "..", "paper_2107_11983_amd")]
    subprocess.check_call(cmd)
    return out


if __name__ == "__main__":
    print(build())
