"""C-ABI contract checks that need no GPU: the library loads, exports every
function include/*.h declares, and rejects bad arguments before any HIP call."""
import ctypes
import importlib.util
import os
import re
import subprocess

import pytest

from paper_1911_02696_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")


def declared_functions():
    names = set()
    for fn in sorted(os.listdir(INCLUDE)):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(INCLUDE, fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        text = re.sub(r"typedef[^;]*;", "", text)  # function-pointer typedefs
        # declarations "name(args);" -- not function-pointer members "(*name)(args);"
        for m in re.finditer(r"\b([A-Za-z_]\w*)\s*\((?!\s*\*)[^;{}]*\)\s*;", text):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.fail(f"{L.LIB_PATH} not built: run python -m paper_1911_02696_amd.build")
    return L.lib()


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("pospopcnt_u8", "pospopcnt_u16", "pospopcnt_u32", "pospopcnt",
                 "ppc_status_string"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = sorted(declared_functions() - exported)
    assert not missing, f"declared but not exported: {missing}"


def test_binding_covers_every_declared_symbol(lib):
    import paper_1911_02696_amd.api  # noqa: F401
    import paper_1911_02696_amd.serve  # noqa: F401  (registers its signatures)
    known = set(L.SIGNATURES)
    for table in L._extensions:
        known |= set(table)
    missing = sorted(declared_functions() - known)
    assert not missing, f"no Python signature for: {missing}"


def test_status_strings(lib):
    for code, name in L.STATUS_NAMES.items():
        assert lib.ppc_status_string(code).decode().startswith(name)
    assert b"unknown" in lib.ppc_status_string(12345)


@pytest.mark.parametrize("k", [0, 1, 7, 12, 24, 48, 128, -8])
def test_bad_width(lib, k):
    assert lib.pospopcnt(0x1000, 4, k, 0x8000, None) == 3  # PPC_ERR_WIDTH


def test_k64_arguments(lib):
    assert lib.pospopcnt_u64(None, 0, None, None) == 0
    assert lib.pospopcnt(None, 0, 64, None, None) == 0
    assert lib.pospopcnt_u64(None, 5, 0x8000, None) == 1
    assert lib.pospopcnt_u64(0x1000, 5, 0x8004, None) == 2
    assert lib.pospopcnt_u64(0x1000, 2**61, 0x8, None) == 4
    # counts (64 x 8 bytes) ending inside the input
    assert lib.pospopcnt_u64(0x1000, 8, 0x1000 - 64 * 8 + 8, None) == 8
    # the ballot variants have no 64-bit form; other configuration errors as for k <= 32
    for cfg in (L.LaunchConfig(variant=1), L.LaunchConfig(variant=2), L.LaunchConfig(depth=12),
                L.LaunchConfig(block_threads=512), L.LaunchConfig(grid=-1)):
        assert lib.pospopcnt_ex(0x1000, 64, 64, 0x80000, None, ctypes.byref(cfg)) == 7


def test_planes_arguments(lib):
    P = ctypes.c_void_p * 40
    planes = P(*[0x100000 * (j + 1) for j in range(40)])
    assert lib.pospopcnt_planes16(planes, 0, 10, 0x8000, None) == 7
    assert lib.pospopcnt_planes16(planes, L.MAX_PLANES + 1, 10, 0x8000, None) == 7
    assert lib.pospopcnt_planes16(planes, 4, 0, None, None) == 0  # nothing to count
    assert lib.pospopcnt_planes16(None, 4, 10, 0x8000, None) == 1
    assert lib.pospopcnt_planes16(planes, 4, 10, None, None) == 1
    with_null = P(*([0x100000, 0] + [0x300000] * 38))
    assert lib.pospopcnt_planes16(with_null, 2, 10, 0x8000, None) == 1
    assert lib.pospopcnt_planes16(planes, 4, 10, 0x8003, None) == 2
    assert lib.pospopcnt_planes16(planes, 4, 2**63, 0x8, None) == 4
    # counts (4 x 16 x 8 bytes) overlapping the third plane
    assert lib.pospopcnt_planes16(planes, 4, 10, 0x300000 + 8, None) == 8
    cfg = L.LaunchConfig(variant=1)
    assert lib.pospopcnt_planes16_ex(planes, 4, 10, 0x8000, None, ctypes.byref(cfg)) == 7


def test_batched_forms_reject_k64(lib):
    import numpy as np
    descs = np.zeros(1, dtype=[("ptr", "<u8"), ("n", "<u8"), ("k", "<u4"), ("reserved", "<u4"),
                               ("counts", "<u8")])
    descs[0] = (0x1000, 4, 64, 0, 0x80000)
    assert lib.pospopcnt_each(descs.ctypes.data, 1, None) == 3


def test_zero_length_is_a_no_op(lib):
    # n = 0: OK without touching pointers or launching (NULL pointers allowed)
    for fn in (lib.pospopcnt_u8, lib.pospopcnt_u16, lib.pospopcnt_u32):
        assert fn(None, 0, None, None) == 0
    assert lib.pospopcnt(None, 0, 16, None, None) == 0


def test_null_pointers(lib):
    assert lib.pospopcnt(None, 5, 16, 0x8000, None) == 1
    assert lib.pospopcnt(0x1000, 5, 16, None, None) == 1


def test_misaligned_counts(lib):
    for off in range(1, 8):
        assert lib.pospopcnt(0x1000, 5, 16, 0x8000 + off, None) == 2


def test_counts_overlapping_input(lib):
    # input [0x1000, 0x1000 + 100) ; counts of 16 x 8 bytes
    assert lib.pospopcnt(0x1000, 50, 16, 0x1000 + 96, None) == 8
    assert lib.pospopcnt(0x1000, 50, 16, 0x1000 - 8 * 16 + 8, None) == 8
    # adjacent ranges do not overlap; the call then needs a device and fails with
    # a HIP error here (no GPU in this check), never with an overlap status
    assert lib.pospopcnt(0x1000, 50, 16, 0x1000 + 104, None) in (0, 5)


def test_length_overflow(lib):
    assert lib.pospopcnt(0x1000, 2**63, 16, 0x8, None) == 4
    assert lib.pospopcnt(0x1000, 2**62, 32, 0x8, None) == 4
    assert lib.pospopcnt(2**64 - 64, 100, 8, 0x8, None) == 4  # address wraps


def test_bad_launch_config(lib):
    bad = [L.LaunchConfig(variant=7), L.LaunchConfig(depth=12), L.LaunchConfig(depth=64),
           L.LaunchConfig(depth=2), L.LaunchConfig(depth=-4),
           L.LaunchConfig(block_threads=96), L.LaunchConfig(block_threads=512),
           L.LaunchConfig(block_threads=32), L.LaunchConfig(blocks_per_cu=-1),
           L.LaunchConfig(grid=-5)]
    for cfg in bad:
        st = lib.pospopcnt_ex(0x1000, 64, 16, 0x80000, None, ctypes.byref(cfg))
        # configuration checks run before the device is queried
        assert st == 7, (cfg.variant, cfg.depth, cfg.block_threads, st)


def test_ceiling_arguments(lib):
    assert lib.ppc_read_ceiling(None, 0, None, None, None) == 0
    assert lib.ppc_read_ceiling(None, 10, 0x8000, None, None) == 1
    assert lib.ppc_read_ceiling(0x1000, 10, 0x8003, None, None) == 2


def test_no_device_reports_hip_error(lib):
    """With no GPU the first call that needs the device fails as PPC_ERR_HIP."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    info = L.DeviceInfo()
    assert lib.ppc_get_device_info(ctypes.byref(info)) == 5
    assert lib.ppc_last_hip_error() != 0


def test_batch_arguments(lib):
    import numpy as np
    assert lib.pospopcnt_batch(None, None, 0, None) == 1       # NULL plan
    assert lib.ppc_plan_destroy(None) == 0
    assert lib.ppc_plan_create(None, None) == 1
    h = ctypes.c_void_p()
    assert lib.ppc_plan_create(ctypes.byref(L.WorkloadHint(0, 0)), ctypes.byref(h)) == 7
    assert lib.ppc_plan_create(ctypes.byref(L.WorkloadHint(1 << 27, 0)), ctypes.byref(h)) == 7
    assert lib.ppc_plan_get_config(None, None) == 1
    assert lib.ppc_plan_set_config(None, None) == 1
    assert lib.ppc_plan_save(None, b"x") == 1
    assert lib.ppc_plan_load(None, b"x") == 1
    assert lib.ppc_plan_autotune(None, None, 0, None, None) == 1
    u = ctypes.c_uint32()
    assert lib.ppc_plan_rejected(None, None, ctypes.byref(u)) == 1
    # one launch per descriptor: validated on the host before anything is launched
    from paper_1911_02696_amd.batch import descriptors
    assert lib.pospopcnt_each(None, 0, None) == 0
    assert lib.pospopcnt_each(None, 3, None) == 1
    good = descriptors([0x1000, 0x2000], [10, 10], [8, 16], [0x9000, 0xA000])
    for field, value, status in ((2, 12, 3), (2, 16 | (1 << 32), 7), (3, 0x9004, 2),
                                 (0, 0, 1), (3, 0x2000, 8)):
        d = good.copy()
        d[1, field] = value
        assert lib.pospopcnt_each(d.ctypes.data, 2, None) == status, (field, value)


def test_static_batch_arguments(lib):
    """pospopcnt_batch_static validates before any device call: no descriptors, a
    misaligned table, more streams than its fixed scratch holds, a bad config."""
    assert lib.pospopcnt_batch_static(None, 0, None, None) == 0
    assert lib.pospopcnt_batch_static(None, 5, None, None) == 1
    assert lib.pospopcnt_batch_static(0x1004, 5, None, None) == 2
    assert lib.pospopcnt_batch_static(0x1000, L.STATIC_MAX_STREAMS + 1, None, None) == 10
    bad = L.BatchConfig(12, 64, 4, 4096)  # no kernel for 12-dword circuits
    assert lib.pospopcnt_batch_static(0x1000, 5, ctypes.byref(bad), None) == 7
    bad = L.BatchConfig(16, 64, 0, 4096)
    assert lib.pospopcnt_batch_static(0x1000, 5, ctypes.byref(bad), None) == 7


def test_plan_needs_a_device(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert lib.ppc_plan_create(ctypes.byref(L.WorkloadHint(16, 0)), ctypes.byref(h)) == 5
    assert not h.value


def test_histogram_arguments(lib):
    assert lib.ppc_histogram_u8(None, 0, 8, None, None) == 0           # n = 0: no-op
    for bins in (0, 33, 64):
        assert lib.ppc_histogram_u8(0x1000, 5, bins, 0x8000, None) == 3
    assert lib.ppc_histogram_u8(None, 5, 8, 0x8000, None) == 1
    assert lib.ppc_histogram_u8(0x1000, 5, 8, None, None) == 1
    assert lib.ppc_histogram_u8(0x1000, 5, 8, 0x8004, None) == 2
    assert lib.ppc_histogram_u16(0x1001, 5, 8, 0x8000, None) == 2      # u16 ids 2-aligned
    assert lib.ppc_histogram_u8(0x1000, 100, 8, 0x1000 + 64, None) == 8  # counts inside ids
    assert lib.ppc_histogram_u16(0x1000, 2**63, 8, 0x8, None) == 4
    assert lib.ppc_histogram_ex(0x1000, 5, 3, 8, 0x8000, None, None) == 7
    bad = L.LaunchConfig(depth=16)
    assert lib.ppc_histogram_ex(0x1000, 5, 1, 8, 0x8000, None, ctypes.byref(bad)) == 7


def _c_caller():
    exe = os.path.join(ROOT, "tests", "c_abi", "abi_check")
    if not os.path.exists(exe):
        spec = importlib.util.spec_from_file_location(
            "ppc_c_abi_build", os.path.join(ROOT, "tests", "c_abi", "build.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.build()
    return exe


def test_header_is_strict_c99_and_callable_from_c():
    """include/pospopcnt.h compiles as strict C99, and a C program linked against the
    library gets the documented statuses for calls that launch nothing."""
    spec = importlib.util.spec_from_file_location(
        "ppc_c_abi_build", os.path.join(ROOT, "tests", "c_abi", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod.check_header_c99()
    res = subprocess.run([_c_caller(), "cpu"], capture_output=True, text=True, timeout=60)
    assert res.returncode == 0, res.stdout + res.stderr


def test_missing_library_fails_loudly(tmp_path):
    """Without the built library every entry point raises ImportError naming the
    build command: the binding has no CPU fallback.  Run in a fresh interpreter, with
    the loader pointed at a path that does not exist."""
    import sys
    code = "\n".join([
        "import sys",
        f"sys.path.insert(0, {ROOT!r})",
        "from paper_1911_02696_amd import _lib as L",
        f"L.LIB_PATH = {str(tmp_path / 'libpospopcnt.so')!r}",
        "from paper_1911_02696_amd import api, batch, serve",
        "calls = [lambda: api.pospopcnt_ptr(0, 0, 16, 0), lambda: api.device_info(),",
        "         lambda: batch.Plan(4), lambda: serve.Server(1 << 20), L.lib]",
        "for call in calls:",
        "    try:",
        "        call()",
        "    except ImportError as e:",
        "        assert 'is missing' in str(e) and 'build' in str(e), e",
        "    else:",
        "        sys.exit('no error raised')",
        "print('all raised')",
    ])
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all raised" in r.stdout


def _in_fresh_process(env_extra: dict, code: str) -> str:
    """Runs `code` in a new Python (the overrides are read once per process)."""
    env = dict(os.environ, **env_extra)
    res = subprocess.run(["python", "-c", "import sys; sys.path.insert(0, %r)\n" % ROOT + code],
                         env=env, capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr
    return res.stdout.strip()


CALL = """
import ctypes
from paper_1911_02696_amd import _lib as L
lib = L.lib()
cfg = L.LaunchConfig(0, 16, 0, 0, 0)
print(lib.pospopcnt(0x1000, 64, 16, 0x80000, None), lib.pospopcnt_u8(0x1000, 64, 0x80000, None),
      lib.pospopcnt_ex(0x1000, 64, 16, 0x80000, None, ctypes.byref(cfg)),
      lib.pospopcnt(0x1000, 0, 16, 0x80000, None))
"""


@pytest.mark.parametrize("env,expect", [
    # a variable that does not parse: every launching call fails with PPC_ERR_ARG
    ({"PPC_LAUNCH": "depth16"}, "7 7 7 0"),
    ({"PPC_LAUNCH": "depth=16,colour=red"}, "7 7 7 0"),
    # parses, but out of range: the fields it fills fail validation; an explicit
    # depth replaces the bad one and the call gets as far as the device (no GPU here)
    ({"PPC_LAUNCH": "depth=12"}, "7 7 5 0"),
    # a per-width variable wins over the general one
    ({"PPC_LAUNCH": "depth=12", "PPC_LAUNCH_U16": "depth=8"}, "5 7 5 0"),
    ({"PPC_LAUNCH_U8": "variant=hybrid,block_threads=96"}, "5 7 5 0"),
    ({"PPC_LAUNCH": "variant=ballot,depth=32,block_threads=256,blocks_per_cu=2,grid=0"},
     "5 5 5 0"),
])
def test_launch_overrides_from_the_environment(env, expect):
    assert _in_fresh_process(env, CALL) == expect


PLAN = """
import ctypes
from paper_1911_02696_amd import _lib as L
h = ctypes.c_void_p()
hint = L.WorkloadHint(16, 0)
print(L.lib().ppc_plan_create(ctypes.byref(hint), ctypes.byref(h)))
"""


@pytest.mark.parametrize("value,expect", [
    ("depth=12", "7"), ("blocks_per_cu=17", "7"), ("stream_weight", "7"), ("threads=64", "7"),
    # valid: plan creation then needs the device, which this machine lacks
    ("depth=4,block_threads=256,blocks_per_cu=2,stream_weight=100", "5"),
])
def test_batch_config_override_is_checked_before_the_device(value, expect):
    assert _in_fresh_process({"PPC_BATCH_CONFIG": value}, PLAN) == expect
