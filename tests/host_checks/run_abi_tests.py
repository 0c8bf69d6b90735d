"""Runs tests/test_abi.py against another build of libpdiv (the path given
as the first argument), e.g. the host-sanitized one; exits with pytest's
status."""

import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import paper_2510_01190_amd as P  # noqa: E402

P.LIB_PATH = sys.argv[1]
P._lib = None

import pytest  # noqa: E402

sys.exit(pytest.main(["-q", "-p", "no:cacheprovider", os.path.join(ROOT, "tests", "test_abi.py")]))
