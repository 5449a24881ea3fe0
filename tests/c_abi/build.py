"""Builds abi_check, the C caller of include/pospopcnt.h, with gcc against the in-tree
libpospopcnt.so.  The header alone is first compiled as strict C99 (-pedantic
-Werror); the caller, which also includes HIP's runtime header (not strict C99), is
built as gnu11."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
PKG = os.path.join(ROOT, "paper_1911_02696_amd")
INCLUDE = os.path.join(ROOT, "include")
EXE = os.path.join(HERE, "abi_check")


def check_header_c99() -> None:
    subprocess.run(["gcc", "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror",
                    "-fsyntax-only", "-x", "c", "-"], check=True, text=True,
                   input='#include "pospopcnt.h"\nint main(void) { return 0; }\n',
                   cwd=INCLUDE)


def build() -> str:
    check_header_c99()
    tmp = EXE + ".tmp"
    subprocess.run(["gcc", "-std=gnu11", "-Wall", "-Wextra", "-Werror",
                    "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", f"-I{INCLUDE}", "-o", tmp,
                    os.path.join(HERE, "abi_check.c"), f"-L{PKG}", "-lpospopcnt",
                    f"-Wl,-rpath,{PKG}", "-L/opt/rocm/lib", "-lamdhip64",
                    "-Wl,-rpath,/opt/rocm/lib"], check=True)
    os.replace(tmp, EXE)
    return EXE


if __name__ == "__main__":
    print(build())
