"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU
needed): the oracle's C (oracle/orc.c) driven through every entry point on
small 2-D and 3-D grids, and the library's C ABI argument checks
(tests/sanitize/abi_checks.cpp) against the library's host logic built with
the sanitizers on host code only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, **kw):
    p = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert p.returncode == 0, (f"{' '.join(cmd)}\n{p.stdout[-4000:]}"
                               f"\n{p.stderr[-4000:]}")
    return p


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "orc_checks")
    _run(["gcc", "-O1", "-g", "-std=c11", "-D_DEFAULT_SOURCE",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", "-o", exe,
          os.path.join(HERE, "orc_checks.c"),
          os.path.join(ROOT, "oracle", "orc.c"), "-lm"])
    p = _run([exe], env=SAN_ENV)
    assert "oracle checks passed" in p.stdout
    assert "runtime error" not in p.stderr


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="no hipcc")
def test_abi_checks_under_asan_ubsan(tmp_path):
    """The host logic of the C ABI (engine.hip: argument checks, the
    window's slots, the solver's host side) instrumented, linked with the
    library's other objects as built for the product (the kernels and their
    launchers, uninstrumented)."""
    from paper_1801_00819_amd import build as hipbuild
    objdir = os.path.join(ROOT, "paper_1801_00819_amd", "_build")
    others = [os.path.join(objdir, os.path.splitext(s)[0] + ".o")
              for s in hipbuild.SOURCES if s != "engine.hip"]
    if not all(os.path.exists(o) for o in others):
        hipbuild.build()
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host",
           "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=all"]
    flags = [f for f in hipbuild.FLAGS if f != "-O3"] + ["-O1", "-g"] + san
    inc = ["-I", os.path.join(ROOT, "include"), "-I",
           os.path.join(ROOT, "paper_1801_00819_amd", "csrc")]
    eng = str(tmp_path / "engine.o")
    _run([HIPCC] + flags + ["-c"] + inc +
         ["-o", eng, os.path.join(ROOT, "paper_1801_00819_amd", "csrc",
                                  "engine.hip")])
    drv = str(tmp_path / "abi_checks.o")
    _run([HIPCC] + flags + ["-c"] + inc + ["-x", "c++", "-o", drv,
                                             os.path.join(HERE,
                                                          "abi_checks.cpp")])
    exe = str(tmp_path / "abi_checks")
    _run([HIPCC] + flags + ["-o", exe, drv, eng] + others + hipbuild.LIBS)
    # the HIP runtime's own allocations outlive main: leaks are not checked
    env = dict(SAN_ENV, ASAN_OPTIONS="detect_leaks=0")
    p = _run([exe], env=env)
    assert "ABI checks passed" in p.stdout
    assert "runtime error" not in p.stderr
