"""Host logic of bench.py (no GPU): the one-GPU guard and the group counts its dependent-step
figures rest on, checked against the oracle's partition of an axis (Sec. 3 and the notes at
the end of Sec. 4.2)."""
import os
import subprocess
import sys

import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


@pytest.mark.parametrize("n,b,d", [(127, 5, 5), (127, 5, 3), (127, 5, 1), (63, 6, 1), (255, 4, 1),
                                   (16, 3, 2), (17, 3, 2), (15, 4, 1)])
def test_group_count_matches_the_oracle_partition(n, b, d):
    assert bench.group_count(n, b, d, 1) == len(O.groups(n, b, d))
    assert bench.group_count(n, b, d, 2) == len(O.groups_two_fronts(n, b, d))


def test_dependent_steps_of_the_127_cubed_workload():
    # 26 groups per axis, middle group 13: 13 front groups below it, 12 above (the chain runs
    # through the 13); every line solve is two-sided, 127 dependent steps.  Per slab 13 lines
    # forward, the middle line, 13 backward; per sweep 13 slabs forward, the middle slab, 13
    # backward.
    S2 = 127
    sweep, kernel = bench.dependent_steps(127, 5, 5, 2, 2)
    assert sweep == 27 * 27 * S2 == 92583
    assert kernel == 13 * S2
    # a line that took more steps lengthens the chain by what it adds
    longer = lambda g, l: 253 if (g, l) == (13, 13) else S2
    assert bench.dependent_steps(127, 5, 5, 2, 2, longer)[0] == 92583 + 126
    # one front per axis: 2G - 1 slabs of 2G - 1 lines
    G = bench.group_count(127, 5, 5, 1)
    assert bench.dependent_steps(127, 5, 5, 1, 1)[0] == (2 * G - 1) ** 2 * S2
