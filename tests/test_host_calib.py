"""Host-side checks of the calibration loop configuration (no device needed)."""
import pytest

from paper_2403_11577_amd import calib as cb


def test_stages_need_the_field_model():
    with pytest.raises(ValueError, match="field model"):
        cb.Calibrator(None, cb.CalibConfig(stages=((0.1, 10),), model="independent"))


def test_paper_schedules_sum_to_the_paper_step_counts():
    # Sec. IV-B: 4000 + 1000 + 1000 steps at 10, 5, 2 cm; camera-LiDAR only: 2000 + 500 + 500
    assert sum(n for _, n in cb.PAPER_STAGES) == 6000
    assert sum(n for _, n in cb.PAPER_STAGES_LIDAR_CAMERA) == 3000
    assert [v for v, _ in cb.PAPER_STAGES] == [0.10, 0.05, 0.02]
