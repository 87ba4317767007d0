"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the C ABI
(argument validation, plan and arena layout), the LRS fit and the autotuner
of liblbm_hip.so, and the oracle, rebuilt with clang's sanitizers on the host
side and exercised by every CPU test of this directory in a child process
that preloads the sanitizer runtime.  A sanitizer report aborts the child."""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(os.environ.get("LBM_HIP_LIB") is not None, reason="already inside the sanitizer run")
@pytest.mark.skipif(shutil.which("hipcc") is None or not os.path.exists("/opt/rocm/llvm/bin/clang"),
                    reason="needs hipcc and ROCm's clang")
def test_cpu_suite_clean_under_asan_and_ubsan(tmp_path):
    sys.path.insert(0, ROOT)
    import oracle
    from paper_2609_32892_amd import build

    hip_lib = build.build_sanitized(str(tmp_path))
    orc_lib = oracle.build_sanitized(str(tmp_path))
    env = dict(os.environ)
    env.update(LD_PRELOAD=build.asan_runtime(), ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", LBM_HIP_LIB=hip_lib, LBM_ORACLE_LIB=orc_lib)
    cmd = [sys.executable, "-m", "pytest", HERE, "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
           "--deselect", f"{os.path.relpath(__file__, ROOT)}::test_cpu_suite_clean_under_asan_and_ubsan"]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out and "failed" not in out, out[-2000:]
