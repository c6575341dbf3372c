"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code, on
the CPU: the oracle (gcc) under its own pin tests, and the library's host
runtime (plan, Holstein tables, C ABI argument checks, built by hipcc with
the sanitizers on the host side only) under a host driver and the ABI tests.
Each sanitizer run is a subprocess with the sanitizer runtime preloaded; any
report ends it with a nonzero status."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0907_3022_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_0907_3022_amd", "_build")
HIPCC = "/opt/rocm/bin/hipcc"
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
GCC_SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _run(cmd, env=None, timeout=900):
    r = subprocess.run(cmd, cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       timeout=timeout)
    return r.returncode, r.stdout


def _gcc_asan():
    return subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()


def _clang_asan():
    libs = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    assert libs, "clang's AddressSanitizer runtime is missing"
    return libs[0]


def test_gcc_sanitizers_report_a_planted_overflow(tmp_path):
    # the harness has teeth: an out-of-bounds read built with the same flags
    # ends with a report
    src = tmp_path / "oob.c"
    src.write_text("#include <stdlib.h>\nint main(int c, char **v) {\n"
                   "  int *a = malloc(4 * sizeof(int));\n  int s = a[c + 3];\n  free(a);\n  return s & 1;\n}\n")
    exe = str(tmp_path / "oob")
    subprocess.check_call(["gcc", "-O0", "-g", *GCC_SAN, "-o", exe, str(src)])
    rc, out = _run([exe])
    assert rc != 0 and "heap-buffer-overflow" in out


def test_oracle_pins_under_sanitizers(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", *GCC_SAN, "-std=c11", "-fPIC", "-shared", "-o", lib,
                           os.path.join(ROOT, "oracle", "chebtd_oracle.c"), "-lm"])
    env = dict(os.environ, LD_PRELOAD=_gcc_asan(), ASAN_OPTIONS="detect_leaks=0", ORACLE_LIB=lib)
    # the subprocess must load this build, not the plain one
    rc, out = _run([sys.executable, "-c", "import oracle as O; O._load(); print(O._LIB_PATH)"], env)
    assert rc == 0 and out.strip().endswith("liboracle_san.so"), out
    rc, out = _run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                    "tests/test_oracle_pins.py", "tests/test_windows.py", "tests/test_reverse_recursion.py"], env)
    assert rc == 0, out[-3000:]


@pytest.fixture(scope="module")
def host_san(tmp_path_factory):
    """The library with its host code (*.cpp) rebuilt under the sanitizers and
    linked with the device objects build() made; and the host driver."""
    dev_objs = sorted(glob.glob(os.path.join(BUILD, "*.hip.o")))
    if not dev_objs:
        pytest.fail("the library's objects are missing: run build() first")
    d = tmp_path_factory.mktemp("hostsan")
    common = ["--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17", "-I", os.path.join(ROOT, "include"),
              "-I", CSRC, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *SAN_HOST]
    procs, objs = [], []
    for src in sorted(glob.glob(os.path.join(CSRC, "*.cpp"))) + [os.path.join(ROOT, "tests", "sanitize",
                                                                             "host_check.cpp")]:
        obj = str(d / (os.path.basename(src) + ".o"))
        procs.append(subprocess.Popen([HIPCC, *common, "-x", "hip", "-c", src, "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
        objs.append(obj)
    for p in procs:
        out, _ = p.communicate(timeout=900)
        assert p.returncode == 0, out
    lib_objs = [o for o in objs if not o.endswith("host_check.cpp.o")]
    lib = str(d / "libchebtd_san.so")
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *SAN_HOST[:4], "-o", lib,
                           *lib_objs, *dev_objs])
    exe = str(d / "host_check")
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", *SAN_HOST[:4], "-o", exe, *objs, *dev_objs])
    return lib, exe


def test_host_runtime_driver_under_sanitizers(host_san):
    _, exe = host_san
    rc, out = _run([exe], dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert rc == 0 and "0 failures" in out, out[-3000:]


def test_abi_host_tests_under_sanitizers(host_san):
    lib, _ = host_san
    env = dict(os.environ, LD_PRELOAD=_clang_asan(), ASAN_OPTIONS="detect_leaks=0", CHEBTD_LIB=lib)
    rc, out = _run([sys.executable, "-c", "from paper_0907_3022_amd import _lib as L; L.lib(); print(L.LIB_PATH)"],
                   env)
    assert rc == 0 and out.strip().endswith("libchebtd_san.so"), out
    rc, out = _run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "tests/test_abi_host.py"],
                   env)
    assert rc == 0, out[-3000:]
