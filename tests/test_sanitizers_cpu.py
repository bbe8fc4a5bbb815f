"""Host-side race and memory checks (CPU only): the FP64 oracle built with
AddressSanitizer and UndefinedBehaviorSanitizer runs a selection of its pins,
and the C ABI's host code (argument checks, workspace sizing, the
allocation-free entry point's refusals) runs its validation tests with the
same sanitizers.  Device code is not instrumented; the GPU-side race check
is the deterministic-scatter test."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _gcc_runtime(name):
    try:
        p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True,
                           check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _child(cmd, env):
    return subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    import oracle
    asan = _gcc_runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = oracle.build(out=str(tmp_path / "liboracle_asan.so"),
                       extra=["-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                              "-fno-sanitize-recover=all", "-g"])
    env = dict(os.environ, PXM_ORACLE_LIB=lib, LD_PRELOAD=asan, OMP_NUM_THREADS="4",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    sel = ("sh_degree or grid_backward or pose_backward or tv_ or upsample or prune or trace or "
           "early_termination or jacobian or slab or opaque or shifted_relu or binding_sample_cap")
    res = _child([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                  "tests/test_oracle_pins.py", "tests/test_oracle_pins_workload_settings.py",
                  "tests/test_oracle_pins_sh_degree.py", "-k", sel], env)
    out = res.stdout[-3000:] + res.stderr[-3000:]
    assert res.returncode == 0, out
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out
    assert " passed" in res.stdout


def _clang_asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_abi_host_checks_under_asan_and_ubsan(tmp_path):
    from paper_2307_03404_amd import build as hb
    rt = _clang_asan_runtime()
    if rt is None or not os.path.exists(os.path.join(ROOT, "_build", "render.o")):
        pytest.skip("clang's AddressSanitizer runtime or the built objects are missing")
    hipcc = hb.hipcc()
    abi = str(tmp_path / "abi_asan.o")
    # sanitizers on the host side of the C ABI only (device code is not instrumented)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    subprocess.run([hipcc, *hb.HIPCC_FLAGS, *san, "-c", os.path.join(hb.CSRC, "abi.hip"), "-o", abi],
                   check=True, capture_output=True)
    objs = [os.path.join(ROOT, "_build", s.replace(".hip", ".o")) for s in hb.SOURCES if s != "abi.hip"]
    lib = str(tmp_path / "libpxm_asan.so")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *san, "-o", lib, abi, *objs],
                   check=True, capture_output=True)
    env = dict(os.environ, PXM_LIBRARY=lib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    probe = _child([sys.executable, "-c", "import os; from paper_2307_03404_amd import pxm; "
                    "assert pxm.lib()._name == os.environ['PXM_LIBRARY'], pxm.lib()._name"], env)
    assert probe.returncode == 0, probe.stderr[-2000:]
    res = _child([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                  "tests/test_abi_cpu.py"], env)
    out = res.stdout[-3000:] + res.stderr[-3000:]
    assert res.returncode == 0, out
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out
