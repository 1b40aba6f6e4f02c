"""The C oracle and the input generators under the host sanitizers:
AddressSanitizer + UndefinedBehaviorSanitizer over every entry point of
oracle/oracle.c and gen/gen.c, ThreadSanitizer over the oracle's pthread pool
(tests/sanitizer_driver.c drives them and cross-checks the results).  Host
code only; nothing here touches a GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = [os.path.join(ROOT, "tests", "sanitizer_driver.c"), os.path.join(ROOT, "oracle", "oracle.c"),
           os.path.join(ROOT, "gen", "gen.c")]

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")


def _build_and_run(tmp_path, flags, args=(), env=None):
    exe = tmp_path / "driver"
    subprocess.run(["gcc", "-std=gnu11", "-O1", "-g", "-fno-omit-frame-pointer", *flags, *SOURCES,
                    "-o", str(exe), "-pthread", "-lm"], check=True, capture_output=True, text=True)
    run_env = dict(os.environ, **(env or {}))
    run_env.pop("LD_PRELOAD", None)
    return subprocess.run([str(exe), *args], capture_output=True, text=True, env=run_env, timeout=300)


def test_oracle_and_generators_under_asan_ubsan(tmp_path):
    r = _build_and_run(tmp_path, ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
                       env={"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0", "UBSAN_OPTIONS": "print_stacktrace=1"})
    assert r.returncode == 0, r.stderr[-4000:]
    assert "all checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


def test_oracle_thread_pool_under_tsan(tmp_path):
    r = _build_and_run(tmp_path, ["-fsanitize=thread"], args=("threads",),
                       env={"TSAN_OPTIONS": "halt_on_error=1"})
    if r.returncode != 0 and "unexpected memory mapping" in r.stderr:
        pytest.skip("ThreadSanitizer cannot map its shadow memory in this environment")
    assert r.returncode == 0, r.stderr[-4000:]
    assert "all checks passed" in r.stdout
    assert "WARNING: ThreadSanitizer" not in r.stderr
