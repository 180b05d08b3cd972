"""AddressSanitizer + UndefinedBehaviorSanitizer build of the host code: the
planner (csrc/plan.cpp: validation, lowering, tables, describe, the live-plan
registry, the workspace check of the allocation-free call) and the FP64
oracle (oracle/oracle.c), linked with host-only stand-ins for the HIP calls
(tests/host_sanitize/hip_stubs.cpp) and driven through their host paths by
tests/host_sanitize/driver.cpp.  Built with g++/gcc (no GPU code), run on the
CPU; any sanitizer report or failed expectation fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "host_sanitize")
CSRC = os.path.join(ROOT, "paper_0803_2386_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, **kw):
    res = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert res.returncode == 0, f"{' '.join(cmd)}\n{res.stdout}\n{res.stderr}"
    return res


@pytest.mark.timeout(900)
def test_planner_and_oracle_under_asan_ubsan(tmp_path):
    if not shutil.which("g++") or not shutil.which("gcc"):
        pytest.skip("gcc toolchain missing")
    inc = ["-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-D__HIP_PLATFORM_AMD__"]
    objs = []
    for src, lang in ((os.path.join(CSRC, "plan.cpp"), "c++"), (os.path.join(HERE, "hip_stubs.cpp"), "c++"),
                      (os.path.join(HERE, "driver.cpp"), "c++"), (os.path.join(ROOT, "oracle", "oracle.c"), "c")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        if lang == "c++":
            cmd = ["g++", "-std=c++17"] + SAN + inc + ["-c", src, "-o", obj]
        else:
            cmd = ["gcc", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-ffp-contract=off"] + SAN + ["-c", src, "-o", obj]
        _run(cmd)
        objs.append(obj)
    exe = str(tmp_path / "driver")
    _run(["g++"] + SAN + ["-fopenmp"] + objs + ["-o", exe, "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="4")
    res = _run([exe], env=env, timeout=600)
    assert "all paths clean" in res.stdout
    assert "runtime error" not in res.stderr and "Sanitizer" not in res.stderr, res.stderr


@pytest.mark.timeout(900)
def test_hypercube_kernel_addressing_on_the_cpu(tmp_path):
    """The hyper-cube kernels' index arithmetic, run for every workgroup and
    thread on the CPU from the arguments the host planner fills
    (tests/host_sanitize/hypercube_emul.cpp): every global offset inside the
    array, every LDS slot inside the allocation and written once before it
    is read, and the result equal to the definition (the bit permutation of
    the transpose; G rho G^H of the gate), under ASan/UBSan."""
    if not shutil.which("g++"):
        pytest.skip("gcc toolchain missing")
    exe = str(tmp_path / "hc_emul")
    _run(["g++", "-std=c++17"] + SAN + ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
                                        os.path.join(HERE, "hypercube_emul.cpp"), "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    res = _run([exe], env=env, timeout=600)
    assert "all cases clean" in res.stdout
