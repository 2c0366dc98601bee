"""Host AddressSanitizer and UndefinedBehaviorSanitizer runs (no GPU):
the CPU oracle, and the library's host side (queries, argument validation,
cell segments, pass splits, timing records) built with the sanitizers on the
host pass only.  Each driver exits non-zero on a failed check, and any
sanitizer report aborts it (-fno-sanitize-recover)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1811_06378_amd", "csrc")
BUILD = os.path.join(ROOT, "_build")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
KERNEL_UNITS = ["fht_misc", "fht_fwd_u8", "fht_fwd_i32", "fht_fwd_f32", "fht_fwd_u8_max", "fht_fwd_i32_max",
                "fht_fwd_f32_max", "fht_adj_i32", "fht_adj_f32"]
HOST_UNITS = ["fht_api", "fht_batch", "fht_lines", "fht_timing", "fht_noalloc"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, **kw)
    assert r.returncode == 0, "%s\n%s" % (" ".join(cmd), r.stdout[-4000:])
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-O1", "-g", "-std=c99"] + SAN + ["-o", exe, os.path.join(HERE, "oracle_driver.c"),
                                                   os.path.join(ROOT, "oracle", "fht_oracle.c"), "-lm"])
    assert "clean" in _run([exe])


@pytest.mark.slow
@pytest.mark.skipif(not all(os.path.exists(os.path.join(BUILD, u + ".hip.o")) for u in KERNEL_UNITS),
                    reason="kernel objects not built (run the library build first)")
def test_library_host_side_under_asan_ubsan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    host_san = []
    for f in SAN:
        host_san += ["-Xarch_host", f]
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-I" + os.path.join(ROOT, "include"),
             "-I" + CSRC, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument", "-Wno-unused-value"] + host_san
    objs = []
    for u in HOST_UNITS:
        o = str(tmp_path / (u + ".o"))
        _run([hipcc] + flags + ["-c", os.path.join(CSRC, u + ".hip"), "-o", o])
        objs.append(o)
    drv = str(tmp_path / "driver.o")
    _run([hipcc] + flags + ["-c", os.path.join(HERE, "abi_driver.cpp"), "-o", drv])
    exe = str(tmp_path / "abi_san")
    _run([hipcc, "--offload-arch=gfx950"] + host_san + ["-o", exe, drv] + objs +
         [os.path.join(BUILD, u + ".hip.o") for u in KERNEL_UNITS])
    assert "clean" in _run([exe])
