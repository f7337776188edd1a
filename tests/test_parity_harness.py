"""Host checks of the parity harness itself (tests/parity.py): the rules that
explain a particle alive on one side only, and the waiting-time comparison
of capped GPU words against uncapped oracle waits.  Synthetic states only."""
import numpy as np
import pytest

from parity import WAIT_CAPPED, WAIT_MAX, check_children, compare_particles

N = 64


def state(ids, xi, vx=None, wait=None, capped=None):
    n = len(ids)
    vx = np.full(n, 1.0e5) if vx is None else np.asarray(vx, float)
    d = dict(id=np.asarray(ids, np.uint64), xi=np.asarray(xi, float), vx=vx,
             vy=np.zeros(n), vz=np.zeros(n), vel_unit=1.0e6,
             wait=np.zeros(n, np.int64) if wait is None else np.asarray(wait, np.int64))
    if capped is not None:
        d["wait_capped"] = np.asarray(capped, bool)
    return d


def test_identical_states_compare_clean():
    g = state([1, 2, 3], [0.5, 10.25, 63.5])
    err, mism = compare_particles(g, dict(g), N, False, 1.0e5)
    assert mism == 0 and err["n"] == 3 and err["pos"] == 0.0


def test_one_sided_particle_at_an_electrode_is_an_absorption_decision():
    g = state([1, 2, 3], [0.5, 10.25, 63.99999999])
    o = state([1, 2], [0.5, 10.25])
    err, mism = compare_particles(g, o, N, False, 1.0e5, prev_ids=[1, 2, 3])
    assert mism == 1 and err["children"] == 0
    g = state([1, 2, 3], [1e-9, 10.25, 40.0])
    o = state([2, 3], [10.25, 40.0])
    err, mism = compare_particles(g, o, N, False, 1.0e5, prev_ids=[1, 2, 3])
    assert mism == 1


def test_one_sided_particle_mid_gap_fails():
    g = state([1, 2, 3], [0.5, 10.25, 33.0])
    o = state([1, 2], [0.5, 10.25])
    with pytest.raises(AssertionError, match="alive only on the GPU side"):
        compare_particles(g, o, N, False, 1.0e5, prev_ids=[1, 2, 3])
    with pytest.raises(AssertionError, match="alive only on the oracle side"):
        compare_particles(o, g, N, False, 1.0e5, prev_ids=[1, 2, 3])
    # periodic boxes absorb nothing
    g = state([1, 2], [0.5, 1e-9])
    o = state([1], [0.5])
    with pytest.raises(AssertionError):
        compare_particles(g, o, N, True, 1.0e5, prev_ids=[1, 2])


def test_implicit_kept_side_may_sit_a_predicted_move_inside():
    # the implicit state holds x~ = x + v~: 0.4 cells from the electrode at
    # 0.5 cells per step is within reach, 0.6 is not
    g = state([1, 2], [5.0, 0.4], vx=[1e5, -5e5])
    o = state([1], [5.0])
    err, mism = compare_particles(g, o, N, False, 1.0e5, prev_ids=[1, 2], implicit=True)
    assert mism == 1
    g = state([1, 2], [5.0, 0.6], vx=[1e5, -5e5])
    with pytest.raises(AssertionError):
        compare_particles(g, o, N, False, 1.0e5, prev_ids=[1, 2], implicit=True)


def test_one_sided_children_need_a_parent_decision():
    kid = (1 << 63) | 12345
    g = state([1, 2, kid], [0.5, 10.25, 20.0])
    o = state([1, 2], [0.5, 10.25])
    err, _ = compare_particles(g, o, N, False, 1.0e5, prev_ids=[1, 2])
    assert err["children"] == 1
    with pytest.raises(AssertionError, match="children"):
        check_children([dict(decisions=0, children=0), err])
    check_children([dict(decisions=1, children=0), err])
    # an old child (present before the step) is no excuse
    with pytest.raises(AssertionError):
        compare_particles(g, o, N, False, 1.0e5, prev_ids=[1, 2, kid])


def test_capped_wait_bounds_the_oracle_wait():
    g = state([1, 2, 3], [0.5, 1.5, 2.5], wait=[7, WAIT_MAX, WAIT_MAX - 5],
              capped=[False, True, True])
    ok = state([1, 2, 3], [0.5, 1.5, 2.5], wait=[7, 300000, WAIT_MAX - 4])
    err, mism = compare_particles(g, ok, N, False, 1.0e5)
    assert mism == 0
    bad = state([1, 2, 3], [0.5, 1.5, 2.5], wait=[8, WAIT_MAX, WAIT_MAX - 4])
    err, mism = compare_particles(g, bad, N, False, 1.0e5)
    assert mism == 2
    assert WAIT_CAPPED == WAIT_MAX + 1


def test_open_trials_are_left_out():
    g = state([1, 2], [0.5, 1.5], wait=[3, 0])
    o = state([1], [0.5], wait=[3])
    err, mism = compare_particles(g, o, N, False, 1.0e5, prev_ids=[1, 2], exclude=[2])
    assert mism == 0 and err["open"] == 1
