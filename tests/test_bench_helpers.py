"""CPU checks of the benchmark's reporting helpers."""
import importlib.util
import math
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_tts_scan_eq5():
    # Eq. 5: TTS = T ln(0.01) / ln(1 - P_s), minimised over the candidate T
    from paper_2606_25203_amd.tts import scan

    def best(times, n):
        r = scan(times, n)[1]
        return None if r is None else r[2]
    assert best([], 4) is None
    assert best([0.3, 0.3, 0.4, 0.5], 4) == 0.5          # every run hit by 0.5 s
    half = 0.5 * math.log(0.01) / math.log(0.5)
    quarter = 0.4 * math.log(0.01) / math.log(0.75)
    assert best([0.4, 0.5], 4) == pytest.approx(min(half, quarter))
    # a later T with a higher success fraction can win
    assert best([1.0, 1.1, 1.2], 4) == pytest.approx(1.2 * math.log(0.01) / math.log(0.25))


def test_incremental_field_bytes(bench):
    # 5 + p (1 + 8 deg) + 8 deg / 64 at the torus's degree 4
    assert bench.incremental_field_bytes_per_attempt(0.0, 4.0) == pytest.approx(5.5)
    assert bench.incremental_field_bytes_per_attempt(0.1, 4.0) == pytest.approx(5.5 + 3.3)


def test_percentile(bench):
    assert bench.percentile([3, 1, 2], 0.5) == 2
    assert bench.percentile([], 0.5) is None
    assert bench.percentile([0.0, 10.0], 0.99) == pytest.approx(9.9)
