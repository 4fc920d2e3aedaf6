"""Host validation under AddressSanitizer (no GPU).

The library's host code (scene validation, work lists, tuning checks, argument
checks of every entry point) is rebuilt with AddressSanitizer instrumentation
for the host pass only, linked with the kernels of the regular build, and the
host-side ABI tests run against it in a child process with the ASan runtime
preloaded.  Any out-of-bounds read or write, use after free or double free in
that code aborts the child with an ASan report.
"""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2408_06506_amd")
BUILD = os.path.join(PKG, "_build")
KERNEL_OBJS = [os.path.join(BUILD, f + ".o") for f in ("tacsl_kernels.hip", "tacsl_impulse.hip", "tacsl_depth.hip")]

CHILD = r"""
import sys
sys.path.insert(0, {root!r})
from paper_2408_06506_amd import _abi
_abi.LIB_PATH = {lib!r}
import tests.test_abi_host as t
t.test_library_exports_every_declared_symbol()
t.test_status_strings()
t.test_valid_scenes_pass()
t.test_null_pointers_rejected()
t.test_invalid_descriptions_return_codes()
t.test_empty_scene_is_valid()
for tile in (0, 64, 192, 1024):
    for order in range(6):
        t.test_worklist_covers_every_taxel_once(tile, order)
t.test_xcd_order_groups_objects()
t.test_bad_tunings_rejected()
t.test_contact_impulse_host_validation()
t.test_pose_step_host_validation()
print("host checks passed under ASan", flush=True)
"""


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_host_code_under_asan():
    from paper_2408_06506_amd import build as b
    try:
        cc = b.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")
    rt = _asan_runtime()
    if rt is None or not all(os.path.exists(o) for o in KERNEL_OBJS):
        pytest.skip("ASan runtime or the regular build's kernel objects missing (run __graft_entry__.build())")
    out = os.path.join(BUILD, "asan")
    os.makedirs(out, exist_ok=True)
    obj = os.path.join(out, "tacsl_plan.cpp.o")
    lib = os.path.join(out, "libtacsl_asan.so")
    # host pass instrumented; the device code is not built from this source
    subprocess.check_call([cc] + b.flags() + ["-O1", "-Xarch_host", "-fsanitize=address",
                                              "-Xarch_host", "-fno-omit-frame-pointer",
                                              "-c", os.path.join(PKG, "csrc", "tacsl_plan.cpp"), "-o", obj])
    # the ASan runtime is not linked in: it is preloaded into the child
    subprocess.check_call([cc, f"--offload-arch={b.ARCH}", "-shared", "-fPIC", "-o", lib, obj] + KERNEL_OBJS +
                          ["-Wl,-rpath,/opt/rocm/lib", "-L/opt/rocm/lib", "-lamdhip64", "-lrocprofiler-sdk-roctx"])
    nm = shutil.which("nm")
    if nm:
        undef = subprocess.run([nm, "-D", "--undefined-only", lib], capture_output=True, text=True).stdout
        assert "__asan_report_load" in undef  # the instrumentation is really there
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, lib=lib)], env=env, cwd=ROOT,
                       capture_output=True, text=True, timeout=600)
    assert "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, r.stderr[-4000:]
    assert "host checks passed under ASan" in r.stdout
