"""Failure paths of the C ABI, on the CPU (no GPU is touched).

* Allocation failures: SFFT_FAIL_ALLOC=n makes the n-th allocation of an
  sfft_plan call fail; every such call must return SFFT_ERR_ALLOC, leave the
  handle NULL and release what it took.
* A host build of the plan and ABI code with AddressSanitizer and
  UndefinedBehaviorSanitizer runs tests/abi_host_check.cpp: host-only plans
  over a spread of shapes, introspection, parameter validation and the
  allocation-failure sweep.  Any out-of-bounds access, use after free,
  undefined behaviour or leak in that code fails the test.
"""

import ctypes
import hashlib
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2011_05698_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build", "sanitized")

sfft = pytest.importorskip("paper_2011_05698_amd.sfft", reason="libsfft.so not built")


@pytest.fixture
def fail_alloc(monkeypatch):
    def set_n(n):
        if n is None:
            monkeypatch.delenv("SFFT_FAIL_ALLOC", raising=False)
        else:
            monkeypatch.setenv("SFFT_FAIL_ALLOC", str(n))
    yield set_n
    monkeypatch.delenv("SFFT_FAIL_ALLOC", raising=False)


def _host_plan(loops=6):
    return sfft.Plan(2 ** 14, 50, 512, 7169, loops, 16, 1, delta=1e-8, seed=102, host_only=True)


def test_injected_allocation_failures(fail_alloc):
    loops = 6
    # the plan object, then each iteration's host tables
    for n in range(1, loops + 2):
        fail_alloc(n)
        with pytest.raises(sfft.SfftError) as exc:
            _host_plan(loops)
        assert exc.value.status == 3, exc.value  # SFFT_ERR_ALLOC
    # past the last host allocation a host-only plan builds normally
    fail_alloc(loops + 2)
    p = _host_plan(loops)
    assert p.loops == loops
    p.close()
    # the device allocation of a full plan fails by injection, before any HIP call
    with pytest.raises(sfft.SfftError) as exc:
        sfft.Plan(2 ** 14, 50, 512, 7169, loops, 16, 1, delta=1e-8, seed=102)
    assert exc.value.status == 3 and "hipMalloc(plan)" in str(exc.value)
    fail_alloc(None)
    p = _host_plan(loops)
    assert p.samples > 0


def test_injection_ignores_malformed_values(fail_alloc):
    for v in ("0", "-3", "abc", ""):
        fail_alloc(v)
        _host_plan(3).close()


def _hipcc():
    for c in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    pytest.skip("hipcc not found")


def _sanitized_checker():
    """Builds the checker once per source state: plan.cpp and api.hip with
    host AddressSanitizer and UndefinedBehaviorSanitizer (device code of the
    kernel sources compiled as usual: only their host launchers are linked)."""
    from paper_2011_05698_amd.build import SOURCES

    srcs = list(SOURCES)
    h = hashlib.sha256()
    for f in srcs + sorted(f for f in os.listdir(CSRC) if f.endswith(".h")):
        h.update(open(os.path.join(CSRC, f), "rb").read())
    h.update(open(os.path.join(INCLUDE, "sfft.h"), "rb").read())
    h.update(open(os.path.join(ROOT, "tests", "abi_host_check.cpp"), "rb").read())
    exe = os.path.join(BUILD, "abi_host_check_" + h.hexdigest()[:16])
    if os.path.exists(exe):
        return exe
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    common = ["--offload-arch=gfx950", "-std=c++17", "-fPIC", "-g", "-I", INCLUDE, "-I", CSRC,
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument"]
    objs = []
    for f in srcs:
        obj = os.path.join(BUILD, f + ".o")
        cmd = [hipcc, *common]
        if f.endswith(".cpp"):
            cmd += ["-x", "hip"]
        if f in ("plan.cpp", "api.hip"):
            cmd += ["-O1", *san]
        else:
            cmd += ["-O3"]
        subprocess.run(cmd + ["-c", os.path.join(CSRC, f), "-o", obj], check=True, capture_output=True)
        objs.append(obj)
    drv = os.path.join(BUILD, "abi_host_check.o")
    subprocess.run([hipcc, *common, "-O1", *san, "-x", "hip", "-c", os.path.join(ROOT, "tests", "abi_host_check.cpp"),
                    "-o", drv], check=True, capture_output=True)
    clangxx = os.path.join(os.path.dirname(os.path.realpath(hipcc)), "..", "llvm", "bin", "clang++")
    if not os.path.exists(clangxx):
        clangxx = "/opt/rocm/llvm/bin/clang++"
    # host link with the sanitizer runtimes; the objects carry their device code
    tmp = exe + ".tmp"
    subprocess.run([clangxx, "-fsanitize=address,undefined", drv, *objs, "-o", tmp, "-L/opt/rocm/lib",
                    "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-lpthread"], check=True, capture_output=True)
    os.replace(tmp, exe)
    return exe


def test_sanitized_host_abi(tmp_path):
    exe = _sanitized_checker()
    supp = tmp_path / "lsan.supp"
    # allocations the HIP runtime makes for itself when it is loaded
    supp.write_text("leak:libamdhip64\nleak:libhsa-runtime64\nleak:libamd_comgr\n")
    env = dict(os.environ)
    env.pop("SFFT_FAIL_ALLOC", None)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:exitcode=97"
    env["LSAN_OPTIONS"] = f"suppressions={supp}:print_suppressions=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "0 failed expectations" in r.stdout
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out and "LeakSanitizer" not in out
