"""Build the oracle's shared library (liboracle.so) with gcc.

Test infrastructure only: the oracle is loaded by tests/, by
__graft_entry__.smoke() and by the cpu_baseline leg of bench.py.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(force: bool = True, out: str = LIB, plant: int = 0) -> str:
    """Compile oracle.c into `out`.  plant != 0 builds the variant with one
    deliberate mistake (ORC_PLANT, see oracle.c) for the planted-mistake test;
    the library the tests normally load is always built with plant = 0."""
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(SRC):
        return out
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-Wno-unused-parameter", f"-DORC_PLANT={int(plant)}", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
