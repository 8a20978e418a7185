"""The host logic (validation, analysis, temporaries, memoisation, window
sizing, plan cache) under AddressSanitizer and UndefinedBehaviorSanitizer:
the host sources are rebuilt with both, loaded into a child Python in place
of libdfx.so, and the analysis-only test modules run there.  Any report
aborts the child (no recovery), which fails this test."""
import os
import shutil
import subprocess
import sys

import pytest

from paper_2406_18109_amd import build as B

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_logic_under_asan_ubsan():
    B.build_sanitized()
    env = B.sanitizer_env()
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
           os.path.join(HERE, "test_analysis_abi.py"), os.path.join(HERE, "test_plan_cache.py"),
           os.path.join(HERE, "test_oracle_analysis.py")]
    r = subprocess.run(cmd, env=env, cwd=os.path.dirname(HERE), capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out
    # the child really ran on the sanitizer build
    probe = subprocess.run([sys.executable, "-c", "import paper_2406_18109_amd as d; d.Context(device=-1);"
                            "print(any('libdfx_san' in l for l in open('/proc/self/maps')))"],
                           env=env, capture_output=True, text=True, timeout=120)
    assert probe.stdout.strip().endswith("True"), probe.stdout + probe.stderr
