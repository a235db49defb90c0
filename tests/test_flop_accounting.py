"""Flop accounting of the benchmark (CPU): the transposed task that the
backward's d psi evaluates costs exactly what the task costs (the two
evaluation orders of L A R^T and of L^T G R form the same pair of costs), and
the phase split of the forward adds up to the task table's total apart from
the identity-only tasks, which run no GEMM."""
import numpy as np

from synth import synthetic_problem
from oracle import heff as oheff


def _dims(P, t):
    s2, s = t[0], t[1]
    q, r = int(P.dimL[P.psi_sec[s2, 0]]), int(P.dimR[P.psi_sec[s2, 3]])
    m, n = int(P.dimL[P.psi_sec[s, 0]]), int(P.dimR[P.psi_sec[s, 3]])
    return q, m, n, r


def test_adjoint_task_costs_what_the_task_costs():
    P = synthetic_problem(22, 22, 0, 700, 23, 187, 120, seed=12)
    tasks = oheff.enumerate_tasks(P)
    assert tasks
    for t in tasks:
        q, m, n, r = _dims(P, t)
        hasL, hasR = t[3] >= 0, t[4] >= 0
        cost, order = oheff.task_cost(q, m, n, r, hasL, hasR)
        # transposed task: output and input sectors swapped
        cost_t, order_t = oheff.task_cost(m, q, r, n, hasL, hasR)
        assert cost_t == cost == t[7]
        if hasL and hasR and order == 1:
            assert order_t == 0   # the cheaper order flips with the transpose


def test_bench_flop_splits():
    import bench
    P = synthetic_problem(16, 16, 0, 96, 8, 24, 60, seed=5, gapped=True)
    tab, _ = oheff.task_table(P)
    a, b = bench.phase_flops(P, tab)
    # tasks with the identity on both sides cost 2 m n (a scaled copy) and run
    # no GEMM in either phase
    both = (tab["lblk"] < 0) & (tab["rblk"] < 0)
    assert both.any()
    assert a + b + int(tab["cost"][both].sum()) == int(tab["cost"].sum())
    dpsi, dops = bench.backward_flops(P, tab)
    assert dpsi == int(tab["cost"].sum())
    assert dops > 0
