"""The stored expected value of the benchmark's timed solve (the SHA-256 of
the 512x512x256 layered model's arrival times, written by
tests/golden/make_golden.py from the oracle) still matches a fresh oracle
solve.  The benchmark checks its timed output against this hash."""
import json
import os

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.slow
def test_headline_hash_is_the_oracles(oracle_lib):
    import sys
    sys.path.insert(0, os.path.join(HERE, "golden"))
    import make_golden
    with open(make_golden.OUT) as f:
        stored = json.load(f)
    fresh = make_golden.layered_golden()
    assert fresh["input_sha256_16"] == stored["input_sha256_16"]
    assert fresh["times_sha256"] == stored["times_sha256"]
