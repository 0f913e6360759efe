"""Host logic of the phase-stamp tool: spans, gaps and per-block phase
medians from synthetic stamp arrays (no GPU)."""
import numpy as np
import pytest

from paper_1308_3290_amd import phase_stamps as ps


def _launch(starts, durations, nslots):
    """Stamps [n, 8]: slot 0 at each start, later slots after the given
    per-phase durations (ticks)."""
    a = np.zeros((len(starts), 8), dtype=np.int64)
    for b, (t0, d) in enumerate(zip(starts, durations)):
        a[b, 0] = t0
        for k in range(1, nslots):
            a[b, k] = a[b, k - 1] + d[k - 1]
    return a


def test_launch_summary_spans_gap_and_phase_medians():
    us = 0.01  # 100 MHz clock: 10 ns per tick
    b = _launch([1000, 1002, 1001], [[10, 20, 30], [12, 20, 28], [11, 22, 30]], 4)
    f = _launch([1200, 1210], [[5, 6, 7, 8, 9, 10], [5, 6, 7, 8, 9, 12]], 7)
    s = ps.launch_summary(b, f, us)
    assert s["b_blocks"] == 3 and s["f_blocks"] == 2
    # pass B: first start 1000, last end max(1060, 1062, 1064) = 1064
    assert s["b_span"] == pytest.approx(64 * us)
    assert s["b_start_spread"] == pytest.approx(2 * us)
    assert s["b_phases"] == pytest.approx([11 * us, 20 * us, 30 * us])
    # gap: fused first start 1200 - pass B last end 1064
    assert s["gap_b_to_f"] == pytest.approx(136 * us)
    # fused: first start 1200, last end max(1245, 1257) = 1257
    assert s["f_span"] == pytest.approx(57 * us)
    assert s["f_start_spread"] == pytest.approx(10 * us)
    assert s["f_phases"] == pytest.approx([5 * us, 6 * us, 7 * us, 8 * us, 9 * us, 11 * us])


def test_phase_names_match_the_slots():
    # pass B: slots 0-3 (three phases); fused pass: slots 0-6 (six phases)
    assert len(ps.B_PHASES) == 3
    assert len(ps.F_PHASES) == 6
