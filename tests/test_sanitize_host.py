"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two drivers in tests/sanitize/ are built with -fsanitize=address,undefined and
run, so an out-of-bounds access, a leak or undefined behaviour aborts them:

* the oracle (oracle/chp.c, with gcc) on random circuits of many sizes,
  every gate kind, all three measurement bases, resets and whole shots;
* the library's host code (the C ABI's gate encoders, argument checks and
  error paths; api.hip built with the sanitizers on its host side only,
  linked with the library's other objects) on random layers and gate lists,
  malformed ones included.  Nothing there launches a kernel.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout[-3000:], r.stderr[-3000:])
    return r


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-std=c11", "-Wall", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", os.path.join(SAN, "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "chp.c"), "-o", exe])
    r = _run([exe], env=ENV, timeout=300)
    assert "oracle sanitizer run ok" in r.stdout


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm toolchain not present")
def test_abi_host_code_under_sanitizers(tmp_path):
    build_dir = os.path.join(ROOT, "paper_2408_00384_amd", "_build")
    csrc = os.path.join(ROOT, "paper_2408_00384_amd", "csrc")
    others = sorted(os.path.join(build_dir, f[:-4] + ".o") for f in os.listdir(csrc)
                    if f.endswith(".hip") and f != "api.hip")
    if not all(os.path.exists(o) for o in others):
        import importlib.util
        spec = importlib.util.spec_from_file_location("_cliff_build", os.path.join(ROOT, "paper_2408_00384_amd",
                                                                                   "build.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.build()
    api = str(tmp_path / "api_san.o")
    # sanitizers on the host side of api.hip only (-Xarch_host before each)
    _run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          "-Xarch_host", "-fno-sanitize-recover=all", "-c", os.path.join(csrc, "api.hip"), "-o", api])
    drv = str(tmp_path / "drv.o")
    _run([CLANG, "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-I", os.path.join(ROOT, "include"), "-c", os.path.join(SAN, "abi_driver.c"), "-o", drv])
    exe = str(tmp_path / "abi_driver")
    _run([CLANG + "++", "-fsanitize=address,undefined", drv, api, *others, "-L/opt/rocm/lib", "-lamdhip64",
          "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    r = _run([exe], env=ENV, timeout=300)
    assert "abi sanitizer run ok" in r.stdout
