"""The library's host code (api.hip: planning, tables, tiling, schedules,
the tuning file, argument checks) built with AddressSanitizer and
UndefinedBehaviorSanitizer on the host side only (its device code as
usual), and driven through the C ABI on a host-only context by
tests/host_asan/driver.cpp, with a tuning file that holds malformed
entries; any sanitizer report fails the test."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"
HIP_FLAGS = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# sanitizers for the host pass only (each option after -Xarch_host)
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
CPU_SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _run(cmd, **kw):
    res = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert res.returncode == 0, "%s\n%s%s" % (" ".join(cmd), res.stdout[-3000:], res.stderr[-3000:])
    return res


def test_host_code_under_sanitizers(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("no ROCm toolchain")
    src = os.path.join(ROOT, "paper_0812_0244_amd", "csrc")
    here = os.path.join(ROOT, "tests", "host_asan")
    api_o, stubs_o, drv_o, exe = (str(tmp_path / x) for x in ("api.o", "stubs.o", "driver.o", "driver"))
    procs = [subprocess.Popen([HIPCC] + HIP_FLAGS + HOST_SAN + ["-c", "-o", api_o, os.path.join(src, "api.hip")],
                              stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True),
             subprocess.Popen([HIPCC] + HIP_FLAGS + ["-c", "-o", stubs_o, os.path.join(here, "launch_stubs.hip")],
                              stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True),
             subprocess.Popen([CLANG] + CPU_SAN + ["-O1", "-g", "-std=c++17", "-c", "-o", drv_o,
                                                   os.path.join(here, "driver.cpp")],
                              stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)]
    for p in procs:
        out, err = p.communicate()
        assert p.returncode == 0, out + err
    _run([CLANG] + CPU_SAN + ["-o", exe, api_o, stubs_o, drv_o, "-L/opt/rocm/lib", "-lamdhip64",
                              "-Wl,-rpath,/opt/rocm/lib"])
    # a tuning file with entries the parser must skip without harm
    tune = tmp_path / "tuning.json"
    tune.write_text("{\n"
                    ' "gfx950/p32/g0/l65536/n7/0123456789abcdef": [65536, 65536, 65536, 65536, 65536, 1, 0, 0, 0, 0, 0],\n'
                    ' "/p32/g0/l65536/n1/ffffffffffffffff": [1e400, -5, "x"],\n'
                    ' "truncated": [1, 2,\n'
                    '"no closing quote: [4096]\n'
                    ' "": []\n'
                    + " " * 5000 + "\n"
                    + ' "long": [' + ", ".join(["1"] * 500) + "]\n}\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1",
               VDWNL_TUNE_CACHE=str(tune))
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    report = res.stdout[-3000:] + res.stderr[-6000:]
    assert res.returncode == 0, report
    assert "host driver ok" in res.stdout, report
    assert "AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr, report
