"""The round-trip check __graft_entry__.smoke() performs, run as a GPU test so a
change of plan or kernel that breaks it shows up with the other GPU tests."""
import os
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_smoke():
    sys.path.insert(0, ROOT)
    import __graft_entry__ as entry
    entry.smoke()
