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
    # the child's lines go straight to this process's output (shown live
    # when pytest runs with -s)
    r = subprocess.run([sys.executable, "-u", "-m", "tests.smalltab_check"], cwd=ROOT, timeout=600)
    assert r.returncode == 0, "small-table check failed (its output above)"
