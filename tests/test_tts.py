"""Eq. 5 and the P_s scan of the time-to-solution protocol (benchmark
section), on hit-time sets whose answers follow by hand."""
import math

import pytest

from paper_2606_25203_amd import tts


def test_eq5_values():
    # one success in two runs: ln(0.01) / ln(0.5) = 6.6439 runs' worth of time
    assert tts.tts(2.0, 0.5) == pytest.approx(2.0 * math.log(0.01) / math.log(0.5))
    assert tts.tts(2.0, 0.5) == pytest.approx(13.2877, abs=1e-4)
    # P_s = 0.9: two runs are 99 % sure
    assert tts.tts(1.0, 0.9) == pytest.approx(2.0)
    assert tts.tts(3.0, 0.0) == math.inf
    # Eq. 5 has no finite value at P_s = 1; one run suffices there
    assert tts.tts(3.0, 1.0) == 3.0 and tts.tts(3.0, 0.995) == 3.0


def test_scan_picks_the_cheapest_candidate():
    # 10 runs: 9 succeed at 1 s, one at 10 s.  Candidate 1 s: P_s = 0.9,
    # TTS = 2 s; candidate 10 s: P_s = 1, TTS = 10 s.
    rows, best = tts.scan([1.0] * 9 + [10.0], 10)
    assert [(T, ps) for T, ps, _ in rows] == [(1.0, 0.9), (10.0, 1.0)]
    assert best[0] == 1.0 and best[2] == pytest.approx(2.0)
    # failures count in the denominator: 1 of 4 at 1 s
    rows, best = tts.scan([1.0], 4)
    assert best[1] == 0.25 and best[2] == pytest.approx(math.log(0.01) / math.log(0.75))
    assert tts.scan([], 5) == ([], None)


def test_scan_is_monotone_in_ps_and_rejects_bad_input():
    times = [0.5, 0.7, 0.7, 1.1, 2.0]
    rows, _ = tts.scan(times, 8)
    ps = [r[1] for r in rows]
    assert ps == sorted(ps) and ps[-1] == 5 / 8 and rows[1][1] == 3 / 8
    with pytest.raises(ValueError):
        tts.scan([1.0, 2.0], 1)
    with pytest.raises(ValueError):
        tts.scan([], 0)
