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
    # through the 13); a two-sided line solve takes 127 steps, a one-chain one 253.  As
    # factored at this width only the middle-middle line (81 unknowns per block) takes one
    # chain: per front slab 2 x 13 inner-front lines and the middle line, all two-sided; the
    # middle slab the same but its middle line one chain.
    S2, S1 = 127, 253
    two_sided_but_middle = lambda g, l: S1 if (g, l) == (13, 13) else S2
    sweep, kernel = bench.dependent_steps(127, 5, 5, 2, 2, two_sided_but_middle)
    front_slab = 2 * 13 * S2 + S2
    middle_slab = 2 * 13 * S2 + S1
    assert sweep == 2 * 13 * front_slab + middle_slab == 92709
    assert kernel == 13 * S2
    # the default: every line on a middle group one chain
    sweep_all_middle, _ = bench.dependent_steps(127, 5, 5, 2, 2)
    assert sweep_all_middle == 2 * 13 * (2 * 13 * S2 + S1) + (2 * 13 * S1 + S1)
    # one front per axis: 2G - 1 slabs of 2G - 1 lines, all two-sided
    G = bench.group_count(127, 5, 5, 1)
    assert bench.dependent_steps(127, 5, 5, 1, 1)[0] == (2 * G - 1) ** 2 * S2
