"""Host-only self-tests of the library (no GPU): the block pool and its
fingerprint index under random operation sequences against a plain model,
and the same self-tests plus the planner, readiness segments and setup
orchestrator built with AddressSanitizer and UndefinedBehaviorSanitizer."""
import os
import subprocess

import pytest


@pytest.mark.parametrize("budget", [1, 2, 5, 33, 257])
def test_pool_stress_against_model(budget):
    from paper_2404_14691_amd import sage as S
    for seed in range(8):
        assert S.sage_selftest_pool(seed, 3000, budget) == 3000


def test_pool_stress_rejects_bad_arguments():
    from paper_2404_14691_amd import sage as S
    with pytest.raises(S.SageError) as e:
        S.sage_selftest_pool(0, 100, 0)
    assert e.value.status == S.SAGE_EINVAL


def test_host_selftests_under_asan_and_ubsan():
    from paper_2404_14691_amd import build as B
    exe = B.build_sanitized()
    env = dict(os.environ)
    # the HIP runtime's own allocations at exit are not this library's
    supp = os.path.join(os.path.dirname(exe), "lsan.supp")
    with open(supp, "w") as fh:
        fh.write("leak:libamdhip64\nleak:libhsa-runtime64\nleak:librocprofiler\n")
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=1"
    env["LSAN_OPTIONS"] = f"suppressions={supp}"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "host self-tests passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
