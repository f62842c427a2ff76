"""The whole-evaluation work model: closed forms on constant rank tables."""
import numpy as np
import pytest

from paper_2402_09356_amd import roofline as R


def test_zero_ranks_leave_dense_diagonal_work_only():
    nt, nb = 10, 100
    r = np.zeros((nt, nt))
    w = R.phase_work(nt * nb, nb, r, r)
    assert w["tlr_potrf"][0] == pytest.approx(nt * nb ** 3 / 3)
    ntiles = nt * (nt - 1) // 2
    assert w["compress"][0] == pytest.approx(4.0 * nb * nb * 8 * ntiles)
    assert w["gen_tiles"][1] == pytest.approx(8.0 * (nt + 2 * ntiles) * nb * nb)


def test_constant_rank_counts():
    nt, nb, rk = 6, 64, 5
    r = np.full((nt, nt), rk, dtype=float)
    w = R.phase_work(nt * nb, nb, r, r)
    ntiles = nt * (nt - 1) // 2
    triples = nt * (nt - 1) * (nt - 2) // 6
    s = 2 * rk
    upd = 4 * nb * rk * rk + 2 * (4 * nb * s * s - 4 * s ** 3 / 3) + 22 * s ** 3 + 4 * nb * s * rk
    expect = nt * nb ** 3 / 3 + 3 * nb * nb * rk * ntiles + triples * upd
    assert w["tlr_potrf"][0] == pytest.approx(expect)
    assert w["tlr_potrf"][1] == pytest.approx(16.0 * nt * nb * nb + triples * 8 * nb * 8 * rk)
    # negative entries (dense markers) and the upper triangle are ignored
    r2 = r.copy()
    r2[np.triu_indices(nt)] = 99
    assert R.phase_work(nt * nb, nb, r2, r2) == w


def test_roofline_sum_of_phase_maxima():
    work = {"a": (1e12, 1e9), "b": (1e9, 8e10)}
    rec = R.roofline_eval(work, t_measured_ms=100.0, peak_flops_tf=50.0, peak_gbs=4000.0)
    assert rec["phases"]["a"]["bound"] == "fp64" and rec["phases"]["b"]["bound"] == "hbm"
    assert rec["t_roof_ms"] == pytest.approx(20.0 + 20.0)
    assert rec["frac"] == pytest.approx(0.4)
