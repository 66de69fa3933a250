"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* libepm's host side: api.cpp is rebuilt with the sanitizers on its host
  pass (device code unchanged, the other translation units as the normal
  build made them) and linked into tests/sanitize/abi_host_checks.cpp, which
  drives validation, the FP64 pair setup of hundreds of geometries, the
  workspace layout, the pose and feature tables and every error path's
  clean-up, up to the first device call (no GPU here: that call fails, and
  the driver checks that it does).
* The C oracle: oracle.c built with gcc's sanitizers, loaded into a child
  interpreter that preloads gcc's runtimes, running the oracle's pins.

Any report aborts the child (-fno-sanitize-recover=all), so a clean exit is
the pass condition; leak checking is on for the C++ driver."""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2603_18401_amd")
SAN_DIR = os.path.join(ROOT, "_build", "sanitize")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


@pytest.mark.timeout(600)
def test_library_host_code_under_asan_ubsan():
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    from paper_2603_18401_amd import build as B
    os.makedirs(SAN_DIR, exist_ok=True)
    objs = []
    for src in B.sources():
        name = os.path.basename(src)
        if name == "api.cpp":
            obj = os.path.join(SAN_DIR, "api_san.o")
            flags = [f for f in B.CFLAGS if f != "-O3"] + ["-O1", "-g"] + HOST_SAN
            _run(["hipcc", "-c", "-x", "hip", src, "-o", obj] + flags)
        else:
            obj = os.path.join(B.BUILD, name + ".o")
            if not os.path.exists(obj) or os.path.getmtime(obj) < os.path.getmtime(src):
                obj = B._compile(src)
        objs.append(obj)
    lib = os.path.join(SAN_DIR, "libepm_san.so")
    _run(["hipcc", "-shared", "-fPIC", f"--offload-arch={B.ARCH}", "-o", lib] + objs)
    exe = os.path.join(SAN_DIR, "abi_host_checks")
    _run(["/opt/rocm/llvm/bin/clang++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__",
          "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include",
          os.path.join(ROOT, "tests", "sanitize", "abi_host_checks.cpp"), "-o", exe,
          lib, f"-Wl,-rpath,{SAN_DIR}", "-L/opt/rocm/lib", "-lamdhip64",
          "-Wl,-rpath,/opt/rocm/lib"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", HIP_VISIBLE_DEVICES="")
    r = _run([exe], env=env, timeout=300)
    assert "libepm host checks passed" in r.stdout


PIN_SCRIPT = r"""
import sys
sys.path.insert(0, {root!r})
import oracle
from tests import test_oracle_mutants as M
lib = oracle.OracleLib({so!r})
pins = M.CANDIDATE_PINS + M.MATCH_PINS + M.TERM_PINS
for pin in pins:
    pin(lib)
print("oracle pins passed under the sanitizers:", len(pins))
"""


@pytest.mark.timeout(600)
def test_oracle_under_asan_ubsan():
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    import oracle
    os.makedirs(SAN_DIR, exist_ok=True)
    so = os.path.join(SAN_DIR, "liboracle_san.so")
    flags = ["-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             "-pthread", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             "-fno-omit-frame-pointer"]
    _run(["gcc"] + flags + [os.path.join(os.path.dirname(oracle.__file__), "oracle.c"), "-o", so,
                            "-lm"])
    rt = [_run(["gcc", f"-print-file-name={n}"]).stdout.strip() for n in ("libasan.so",
                                                                          "libubsan.so")]
    if not all(os.path.isabs(p) and os.path.exists(p) for p in rt):
        pytest.skip("gcc sanitizer runtimes not installed")
    env = dict(os.environ, LD_PRELOAD=":".join(rt),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = _run([sys.executable, "-c", PIN_SCRIPT.format(root=ROOT, so=so)], env=env, timeout=500,
             cwd=ROOT)
    assert "oracle pins passed" in r.stdout
