"""Build the CPU oracle (test infrastructure only) with gcc.

Produces oracle/libppc_oracle.so from oracle/ppc_oracle.c.  ``build(plant=id,
out=path)`` builds a variant with one planted mistake, for the test that shows
the oracle's pins catch such mistakes.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ppc_oracle.c")
LIB = os.path.join(HERE, "libppc_oracle.so")
CFLAGS = ["-O2", "-std=gnu11", "-Wall", "-Wextra", "-pthread", "-shared", "-fPIC"]


def build(plant: int = 0, out: str = LIB) -> str:
    cmd = ["gcc", *CFLAGS]
    if plant:
        cmd.append(f"-DPPC_ORACLE_PLANT={int(plant)}")
    tmp = out + ".tmp"
    cmd += ["-o", tmp, SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(int(sys.argv[1]) if len(sys.argv) > 1 else 0))
