"""Host-code sanitizer run (CPU only): builds AddressSanitizer + UndefinedBehavior-
Sanitizer variants of the oracle, the input generator and the library's host code
into _build/asan/, then runs the CPU test files against them in a fresh Python with
the ASan runtime preloaded.

    python tests/sanitize/run.py [extra pytest args]

All three libraries are built with ROCm's clang so that one ASan runtime serves the
process.  In the library only host code is instrumented (hipcc's -Xarch_host); its
kernels are built as usual but never run here.  Leak detection is off: the Python
interpreter itself keeps allocations until exit.  Exit status: pytest's.
"""
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(ROOT, "_build", "asan")
LLVM = "/opt/rocm/lib/llvm"
CLANG = os.path.join(LLVM, "bin", "clang")
SAN_C = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
         "-fno-omit-frame-pointer", "-shared-libsan", "-g", "-O1"]
TESTS = ["tests/test_oracle_pins.py", "tests/test_abi.py", "tests/test_serve_scheduler.py",
         "tests/test_bench_cli.py"]


def asan_runtime() -> str:
    hits = glob.glob(os.path.join(LLVM, "lib", "clang", "*", "lib", "linux",
                                  "libclang_rt.asan-x86_64.so"))
    if not hits:
        raise FileNotFoundError("clang's ASan runtime (libclang_rt.asan-x86_64.so) not found")
    return hits[0]


def build() -> dict:
    sys.path.insert(0, ROOT)
    from paper_1911_02696_amd import build as pbuild
    os.makedirs(OUT, exist_ok=True)
    libs = {"PPC_ORACLE_LIB": os.path.join(OUT, "libppc_oracle.so"),
            "PPC_GEN_LIB": os.path.join(OUT, "libppc_gen.so"),
            "PPC_LIB": os.path.join(OUT, "libpospopcnt.so")}
    for key, src in (("PPC_ORACLE_LIB", os.path.join(ROOT, "oracle", "ppc_oracle.c")),
                     ("PPC_GEN_LIB", pbuild.GEN_SRC)):
        subprocess.run([CLANG, "-std=gnu11", "-Wall", "-pthread", "-shared", "-fPIC", *SAN_C,
                        "-o", libs[key], src], check=True)
    srcs = [os.path.join(pbuild.CSRC, s) for s in pbuild.HIP_SOURCES]
    host_san = []
    for flag in SAN_C:
        host_san += ["-Xarch_host", flag]
    cmd = [pbuild.hipcc(), *pbuild.HIPCC_FLAGS, *host_san, f"-I{pbuild.INCLUDE}",
           f"-I{pbuild.CSRC}", "-o", libs["PPC_LIB"], *srcs, "-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(res.stderr)
    return libs


def main() -> int:
    libs = build()
    env = dict(os.environ, **libs)
    env["LD_PRELOAD"] = asan_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:strict_string_checks=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    cmd = [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", *TESTS, *sys.argv[1:]]
    return subprocess.run(cmd, cwd=ROOT, env=env).returncode


if __name__ == "__main__":
    sys.exit(main())
