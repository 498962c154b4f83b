"""The mission harness with the HIP controller in the loop (Sec. VI set-up,
synthetic layouts): five seeded experiments per mission.  The controller's
arithmetic is deterministic, so the outcomes repeat; the assertions leave a
margin of one run for the quadrotor, whose slow mission can time out."""
import pytest

from paper_2504_06437_amd import mission as M

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mission,min_success", [(1, 80.0), (2, 100.0), (3, 100.0)])
def test_missions_with_the_hip_controller(mission, min_success):
    r = M.run_mission(mission, runs=5)
    v = M.MISSIONS[mission]["v_set"]
    assert r["runs"] == 5 and r["collisions"] == 0
    assert r["success_pct"] >= min_success, r
    assert 0.7 * v < r["avg_speed"] <= 1.05 * v
    assert 0.0 <= r["error_m"] < 2.0
