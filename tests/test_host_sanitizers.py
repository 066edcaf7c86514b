"""Host code under the sanitizers: the library's host files (exponents,
hierarchy enumeration and pruning, neighbour tables, dictionary, the
one-time table and plan upload, argument checks, error plumbing) built with
g++ under AddressSanitizer + UndefinedBehaviorSanitizer (leak checks on), and
under ThreadSanitizer, and driven through the C ABI by
tests/sanitize/host_driver.c.  The driver queries one handle from four
threads at once, and has four threads make the first heom_prepare on one
fresh handle at the same moment (the upload must run once).  Kernel launches
are replaced by stubs that fail and device memory by host memory
(tests/sanitize/host_stubs.cpp); no GPU is used."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2306_07522_amd", "csrc")
SAN = os.path.join(ROOT, "tests", "sanitize")
HOST_FILES = [os.path.join(CSRC, "host_hierarchy.cpp"), os.path.join(CSRC, "device_tables.cpp"),
              os.path.join(CSRC, "dense.cpp"), os.path.join(CSRC, "abi.cpp"), os.path.join(SAN, "host_stubs.cpp")]


def _build(tmp_path, flags):
    if not shutil.which("g++") or not shutil.which("gcc"):
        pytest.skip("no host compiler")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", "/opt/rocm/include", "-D__HIP_PLATFORM_AMD__"]
    objs = []
    for src in HOST_FILES:
        o = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *flags, *inc, "-c", src, "-o", o],
                       check=True, capture_output=True, text=True)
        objs.append(o)
    o = str(tmp_path / "driver.o")
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", *flags, "-I",
                    os.path.join(ROOT, "include"), "-c", os.path.join(SAN, "host_driver.c"), "-o", o],
                   check=True, capture_output=True, text=True)
    exe = str(tmp_path / "host_driver")
    subprocess.run(["g++", *flags, "-o", exe, o, *objs, "-lpthread"], check=True, capture_output=True, text=True)
    return exe


@pytest.mark.parametrize("kind", ["address,undefined", "thread"])
def test_host_code_under_sanitizers(tmp_path, kind):
    flags = [f"-fsanitize={kind}"]
    if "undefined" in kind:
        flags.append("-fno-sanitize-recover=undefined")
    try:
        exe = _build(tmp_path, flags)
    except subprocess.CalledProcessError as e:
        pytest.fail(f"sanitizer build failed:\n{e.stdout}\n{e.stderr}")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "all checks passed" in out
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out and "WARNING: ThreadSanitizer" not in out
