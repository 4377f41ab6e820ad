"""CPU-only sanitizer builds of the host registry builder and of the C oracle.

`registry.cpp` (host-only registries: no GPU is touched) and
`oracle/gnm_oracle.c` are compiled with AddressSanitizer and
UndefinedBehaviorSanitizer, every finding fatal, and driven over edge
registries and records (tests/sanitize/).  A planted copy of the oracle whose
prefix mask shifts by 32 at length 0 must be caught, which shows the builds
detect the mistake they are here for.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="halt_on_error=1:detect_leaks=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _need(tool):
    if shutil.which(tool) is None:
        pytest.skip("%s not installed" % tool)


def _run(exe):
    return subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)


def test_registry_builder_under_sanitizers(tmp_path):
    _need("g++")
    if not os.path.exists("/opt/rocm/include/hip/hip_runtime.h"):
        pytest.skip("HIP headers not installed")
    exe = str(tmp_path / "registry_san")
    subprocess.check_call(
        ["g++", "-std=c++17"] + SAN + ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                                       "-I", os.path.join(ROOT, "include"),
                                       "-I", os.path.join(ROOT, "paper_1108_1785_amd", "csrc"),
                                       os.path.join(ROOT, "tests", "sanitize", "registry_san.cpp"),
                                       os.path.join(ROOT, "paper_1108_1785_amd", "csrc", "registry.cpp"),
                                       "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    r = _run(exe)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "registry_san: ok" in r.stdout


def _build_oracle_driver(tmp_path, oracle_src):
    d = tmp_path / "t" / "sanitize"
    d.mkdir(parents=True)
    (tmp_path / "oracle").mkdir()
    shutil.copy(os.path.join(ROOT, "tests", "sanitize", "oracle_san.c"), d / "oracle_san.c")
    (tmp_path / "oracle" / "gnm_oracle.c").write_text(oracle_src)
    exe = str(tmp_path / "oracle_san")
    subprocess.check_call(["gcc", "-std=c11"] + SAN + ["-fopenmp", str(d / "oracle_san.c"), "-o", exe])
    return exe


def test_oracle_under_sanitizers(tmp_path):
    _need("gcc")
    src = open(os.path.join(ROOT, "oracle", "gnm_oracle.c")).read()
    r = _run(_build_oracle_driver(tmp_path, src))
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "oracle_san: ok" in r.stdout


def test_sanitizer_catches_a_shift_by_32(tmp_path):
    """Planted in a copy of the oracle: the mask without its length-0 guard."""
    _need("gcc")
    src = open(os.path.join(ROOT, "oracle", "gnm_oracle.c")).read()
    guarded = "return len == 0 ? 0u : (uint32_t)(0xFFFFFFFFu << (32u - len));"
    assert guarded in src
    planted = src.replace(guarded, "return (uint32_t)(0xFFFFFFFFu << (32u - len));")
    r = _run(_build_oracle_driver(tmp_path, planted))
    assert r.returncode != 0
    assert "shift exponent 32" in r.stderr
