"""The host runtime built with the address and undefined-behaviour
sanitizers (g++, no GPU): graph validation and staging for every node kind,
the host assembly of results, the minimiser, and the ABI's error paths when
no device can be reached (tests/host_sanitize/driver.cpp; kernel launches
are replaced by stand-ins that report an error)."""
import concurrent.futures
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1311_1753_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "host_sanitize")
FLAGS = ["-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
         "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
         "-Wno-unused-result"]
SOURCES = [os.path.join(CSRC, f) for f in ("graph.cpp", "api.cpp", "minimiser.cpp", "fit.cpp", "batch.cpp")] + \
          [os.path.join(HERE, f) for f in ("stubs.cpp", "driver.cpp")]


@pytest.mark.timeout(600)
def test_host_runtime_under_sanitizers(tmp_path):
    if shutil.which("g++") is None or not os.path.exists("/opt/rocm/lib/libamdhip64.so"):
        pytest.skip("needs g++ and the HIP runtime library")

    def cc(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        r = subprocess.run(["g++"] + FLAGS + ["-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    with concurrent.futures.ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(cc, SOURCES))
    exe = str(tmp_path / "host_sanitize")
    r = subprocess.run(["g++"] + FLAGS + objs + ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib",
                                                 "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert "host sanitizer checks: ok" in r.stdout
