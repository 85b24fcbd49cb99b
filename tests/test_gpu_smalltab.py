"""The round kernel's rarely taken paths, made common by a test build with
tiny on-chip tables, checked against the oracle in a child process."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu


def test_small_tables_match_oracle():
    from paper_2212_00977_amd import native

    assert os.path.exists(native.SMALL_TABLES_PATH), "test build missing: run __graft_entry__.build()"
    r = subprocess.run([sys.executable, "-u", "-m", "tests.smalltab_check"], cwd=ROOT,
                       capture_output=True, text=True, timeout=600)
    print(r.stdout[-4000:])
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
