"""Host code under AddressSanitizer, UndefinedBehaviorSanitizer and
LeakSanitizer (no GPU).

Plan creation, plan info and workspace layout: the library's host
translation unit is rebuilt with the sanitizers on its host pass only and
linked with the kernel objects of the in-tree build;
`tests/host/plan_sanitize.cpp` drives it over seeded random shapes,
acquisitions and decompositions and the benchmark grids.  The FP64 oracle:
`tests/host/oracle_sanitize.c` calls every entry point on small grids."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer"]


def _objects():
    from paper_1804_01184_amd import build as B
    obj_dir = os.path.join(ROOT, "_build", "fwi2d")
    objs = [os.path.join(obj_dir, s.replace(".hip", ".o")) for s in B.SOURCES
            if s != "fwi2d_api.hip"]
    if not all(os.path.exists(o) for o in objs):
        B.build()
    return B, objs


def test_plan_tables_under_sanitizers(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm compilers not found")
    B, objs = _objects()
    api_o = str(tmp_path / "fwi2d_api_san.o")
    flags = [f for f in B.FLAGS if f != "-O3"] + ["-O1", "-g"]
    subprocess.run([HIPCC, *flags, *SAN, "-c", os.path.join(B.CSRC, "fwi2d_api.hip"),
                    "-o", api_o], check=True, capture_output=True)
    lib = str(tmp_path / "libfwi2d_san.so")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", api_o, *objs, "-o", lib],
                   check=True, capture_output=True)
    exe = str(tmp_path / "plan_sanitize")
    rocm_lib = os.path.join(os.path.dirname(os.path.dirname(shutil.which(HIPCC) or HIPCC)), "lib")
    subprocess.run([CLANG, "-g", "-O1", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "host", "plan_sanitize.cpp"), "-o", exe, lib,
                    f"-Wl,-rpath,{tmp_path}", f"-L{rocm_lib}", "-lamdhip64",
                    f"-Wl,-rpath,{rocm_lib}"], check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe, "300"], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    ok = int(r.stdout.split("plans ok ")[1].split()[0])
    assert ok >= 200, r.stdout


def test_oracle_under_sanitizers(tmp_path):
    """Every oracle entry point on small grids (with and without an
    absorbing layer, per-shot wavelets, checkpoints every 1, 7 and nt
    steps, one and two threads) under AddressSanitizer, UBSan and
    LeakSanitizer; checkpointed gradients equal the whole-history one."""
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_sanitize")
    subprocess.run([gcc, "-g", "-O1", "-std=c99", "-fopenmp", "-fsanitize=address,undefined",
                    "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "oracle"),
                    os.path.join(ROOT, "tests", "host", "oracle_sanitize.c"),
                    os.path.join(ROOT, "oracle", "fwi2d_oracle.c"), "-o", exe, "-lm"],
                   check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "oracle ok" in r.stdout
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
