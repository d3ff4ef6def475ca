"""The serving loop under concurrent use, with AddressSanitizer (host code).

``tests/native/server_stress`` (built by ``tests/native/build_stress.py``,
which ``__graft_entry__.build()`` runs) serves three databases while six
threads submit and wait and a seventh pauses, resumes and reads the
counters; it then drains and compares every answer with the oracle's
single-query Answer (Definition 1).  A memory error in the host code
(overflow, use after free) ends it with exit code 67.  Skipped when the
binary has not been built or is older than its sources.
"""
import glob
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
EXE = os.path.join(HERE, "native", "server_stress")


def _sources():
    pats = ["paper_2510_03631_amd/csrc/*.hip", "paper_2510_03631_amd/csrc/*.h", "include/*.h",
            "tests/native/server_stress.cpp", "oracle/pir_oracle.c"]
    return [f for p in pats for f in glob.glob(os.path.join(ROOT, p))]


@pytest.mark.parametrize("graphs", [0, 1])
def test_server_stress_sanitized_and_exact(gpu, graphs):
    if not os.path.exists(EXE):
        pytest.skip("tests/native/server_stress is not built (python tests/native/build_stress.py)")
    newest = max(os.path.getmtime(f) for f in _sources())
    if os.path.getmtime(EXE) < newest:
        pytest.skip("tests/native/server_stress is older than its sources "
                    "(python tests/native/build_stress.py)")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:exitcode=67")
    print(f"server_stress graphs={graphs}", flush=True)
    res = subprocess.run([EXE, str(graphs)], capture_output=True, text=True, timeout=240, env=env)
    assert res.returncode == 0, (res.stdout + res.stderr)[-6000:]
    assert res.stdout.startswith("ok:"), res.stdout
