"""The stored single-heap fixture (written by tests/golden/make_golden.py from
the oracle) still matches the generator and the oracle."""
import json
import os

from golden.make_golden import digest, single_heap_fixture
from paper_2405_07079_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def test_single_heap_fixture_is_current():
    stored = json.load(open(os.path.join(HERE, "golden", "single_heap_64KiB.json")))
    assert stored == single_heap_fixture()


def test_generator_is_stable():
    stored = json.load(open(os.path.join(HERE, "golden", "single_heap_64KiB.json")))
    assert digest(W.single_heap().req) == stored["trace_sha256"]
