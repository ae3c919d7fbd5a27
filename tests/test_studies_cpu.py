"""The effectiveness-study helpers (Sec. V-A / V-C N_correct criterion and
the end-point clustering proposed in Sec. VI) on constructed end points whose
counts and groups follow from the definitions by hand."""
import numpy as np

from paper_2603_28770_amd import studies as S


def test_n_correct_radius_is_strict_and_euclidean():
    # distances to 0 in 2-D: 0.3, 0.5 (not < 0.5), 0.4999, sqrt(0.18) ~ 0.424
    x = np.array([[0.3, 0.0], [0.0, -0.5], [0.4999, 0.0], [0.3, 0.3]])
    assert S.n_correct(x, "rastrigin") == 3
    assert S.n_correct(x, "rastrigin", mask=[True, True, False, True]) == 2
    assert S.n_correct(np.zeros((0, 2)), "rastrigin") == 0


def test_n_correct_uses_each_objectives_minimiser():
    x = np.array([[1.0, 1.0, 1.0], [0.0, 0.0, 0.0]])
    assert S.n_correct(x, "rosenbrock") == 1
    assert S.n_correct(x, "rastrigin") == 1
    st = np.full((1, 4), S.XSTAR["styblinski_tang"] + 0.2)  # distance 0.4
    assert S.n_correct(st, "styblinski_tang") == 1


def test_cluster_minima_groups_by_leader_in_f_order():
    x = np.array([[0.0, 0.0], [5.0, 5.0], [0.1, 0.0], [5.05, 5.0], [0.0, 0.1], [9.0, 9.0]])
    f = np.array([1.0, 0.5, 1.2, 0.6, 1.1, np.nan])
    g = S.cluster_minima(x, f, 0.5)
    # lowest first: the (5, 5) group led by row 1 (f 0.5), then (0, 0) led by row 0
    assert [(c["leader"], c["count"]) for c in g] == [(1, 2), (0, 3)]
    assert g[0]["f"] == 0.5


def test_cluster_minima_ties_and_empty():
    x = np.array([[0.0], [3.0], [3.1]])
    f = np.array([2.0, 2.0, 2.0])
    g = S.cluster_minima(x, f, 0.5)  # equal f: the lower index leads
    assert [(c["leader"], c["count"]) for c in g] == [(0, 1), (1, 2)]
    assert S.cluster_minima(np.zeros((0, 2)), np.zeros(0), 0.5) == []


def test_run_summary_counts():
    # row 0 did not converge (it is left out of the groups); the lowest
    # converged group is the one at the origin, led by row 2
    out = {"x": np.array([[3.0, 3.0], [0.1, 0.0], [0.0, 0.2], [2.0, 2.0], [0.0, 0.0]]),
           "f": np.array([-1.0, 0.2, 0.1, 8.0, 0.0]),
           "status": np.array([0, 1, 1, 1, 0], dtype=np.int8), "summary": {"best_f": -1.0}}
    s = S.run_summary(out, "rastrigin")
    assert s["n_correct"] == 3 and s["n_correct_converged"] == 2 and s["n_converged"] == 3
    assert s["groups"] == 2 and s["lowest_group_count"] == 2 and s["lowest_group_correct"]
    # the lowest converged group far from the minimiser is not correct, even
    # though the (unconverged) first row sits on the minimiser
    out["x"][0] = [0.0, 0.0]
    out["x"][1] = [4.1, 4.0]
    out["x"][2] = [4.0, 4.0]
    out["f"][1] = 0.05
    s = S.run_summary(out, "rastrigin")
    assert s["lowest_group_count"] == 2 and not s["lowest_group_correct"]
