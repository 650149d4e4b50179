"""Build the plain C caller of libcem.so (tests/c_abi/cube_force) with gcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "cube_force.c")
BIN = os.path.join(HERE, "cube_force")


def command(out=BIN):
    return ["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-O2",
            "-I", os.path.join(ROOT, "include"), SRC, "-o", out,
            "-L", os.path.join(ROOT, "paper_2508_04076_amd"), "-lcem", "-lm",
            # libcem.so found next to the package wherever the tree is copied
            "-Wl,-rpath,$ORIGIN/../../paper_2508_04076_amd", "-Wl,-rpath-link,/opt/rocm/lib"]


def build(out=BIN):
    subprocess.run(command(out), check=True)
    return out


if __name__ == "__main__":
    print(build())
