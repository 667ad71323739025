"""Per-kernel timing (dba_set_kernel_timing / dba_kernel_times): timed
iterations with use_graph (event-record nodes in captured graphs where the HIP
runtime accepts them, eager launches where it does not) and without it both
count every launch, report positive times that agree, and leave the iterates
bitwise unchanged; the sampled mode times the first local launch of each
batch of iterations, the rest of the batch replayed from a graph."""
import numpy as np
import pytest

from paper_1708_07954_amd import binding
from scenes import make_sphere_scene

pytestmark = pytest.mark.gpu

KW = dict(precision="fp32", loss="student_t", loss_param=4.0, rho=1e3, block_waves=1, persistent=0,
          segment_schedule=1)


def run(sc, n, timed, use_graph):
    s = binding.Solver(use_graph=use_graph, **KW).set_scene(sc)
    s.iterate(2)  # the schedule's warm-up and single candidate, untimed
    if timed:
        binding.dba_set_kernel_timing(s.h, True)
    s.iterate(n)
    kt = binding.dba_kernel_times(s.h) if timed else None
    cams, pts = s.params()
    s.close()
    return cams, pts, kt


@pytest.mark.parametrize("n", [1, 16, 37])
def test_timed_iterations_count_every_launch_and_change_nothing(n):
    sc = make_sphere_scene(seed=21, n_cams=30, n_points=3000)
    ref_c, ref_p, _ = run(sc, n, False, True)
    avg = {}
    for use_graph in (True, False):
        c, p, kt = run(sc, n, True, use_graph)
        assert np.array_equal(c, ref_c) and np.array_equal(p, ref_p), use_graph
        for k in ("local", "consensus", "norms"):
            total, launches = kt[k]
            assert launches == n and total > 0, (use_graph, k, kt[k])
        avg[use_graph] = kt["local"][0] / n
    print(n, "local kernel ms, graph / eager:", avg[True], avg[False])
    assert 0.5 < avg[True] / avg[False] < 2.0


def test_timing_off_again_uses_the_untimed_graphs():
    sc = make_sphere_scene(seed=22, n_cams=20, n_points=1500)
    s = binding.Solver(**KW).set_scene(sc)
    s.iterate(2)
    binding.dba_set_kernel_timing(s.h, True)
    s.iterate(20)
    binding.dba_set_kernel_timing(s.h, False)
    s.iterate(20)
    kt = binding.dba_kernel_times(s.h)
    assert kt["local"][1] == 0
    c, p = s.params()
    s.close()
    ref_c, ref_p, _ = run(sc, 40, False, True)
    assert np.array_equal(c, ref_c) and np.array_equal(p, ref_p)


def test_local_only_timing_times_the_local_solve_alone():
    sc = make_sphere_scene(seed=23, n_cams=20, n_points=1500)
    s = binding.Solver(**KW).set_scene(sc)
    s.iterate(2)
    binding.dba_set_kernel_timing(s.h, True, local_only=True)
    s.iterate(21)
    kt = binding.dba_kernel_times(s.h)
    assert kt["local"][1] == 21 and kt["local"][0] > 0
    assert kt["consensus"][1] == 0 and kt["norms"][1] == 0
    # switching back to every kernel recaptures the timed graphs
    binding.dba_set_kernel_timing(s.h, True)
    s.iterate(17)
    kt = binding.dba_kernel_times(s.h)
    assert all(kt[k][1] == 17 for k in ("local", "consensus", "norms"))
    assert binding.STATUS[binding.load().dba_set_kernel_timing(s.h, 4)] == "DBA_E_INVALID_ARG"
    s.close()


def test_sampled_timing_times_the_first_iteration_of_each_replay():
    """Mode 3 times the local solve in the first iteration of each graph
    replay: one launch per 16-iteration replay and one per single-iteration
    replay, at the same average as every launch timed, and the iterates
    bitwise unchanged."""
    sc = make_sphere_scene(seed=24, n_cams=30, n_points=3000)
    s = binding.Solver(**KW).set_scene(sc)
    s.iterate(2)
    binding.dba_set_kernel_timing(s.h, True, sampled=True)
    s.iterate(17)  # captures the timed graphs
    binding.dba_set_kernel_timing(s.h, True, sampled=True)
    s.iterate(16 * 5 + 3)
    kt = binding.dba_kernel_times(s.h)
    assert kt["local"][1] == 5 + 3 and kt["local"][0] > 0, kt["local"]
    assert kt["consensus"][1] == 0 and kt["norms"][1] == 0
    sampled = kt["local"][0] / kt["local"][1]
    binding.dba_set_kernel_timing(s.h, True, local_only=True)
    s.iterate(17)
    binding.dba_set_kernel_timing(s.h, True, local_only=True)
    s.iterate(64)
    kt = binding.dba_kernel_times(s.h)
    every = kt["local"][0] / kt["local"][1]
    binding.dba_set_kernel_timing(s.h, False)
    c, p = s.params()
    s.close()
    print("local kernel ms, sampled / every launch:", sampled, every)
    assert 0.5 < sampled / every < 2.0
    ref_c, ref_p, _ = run(sc, 17 + 16 * 5 + 3 + 17 + 64, False, True)
    assert np.array_equal(c, ref_c) and np.array_equal(p, ref_p)
