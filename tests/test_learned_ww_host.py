"""Host-side logic of the learned weight-window generator (CPU): adjoint
problem construction, network features, source cells, window centres."""
import math

import numpy as np
import pytest

import workloads as w
from paper_2305_07636_amd import learned_ww as lw


def test_adjoint_problem_transposes_and_moves_source():
    p = w.cfg5_dogleg()
    a = lw.adjoint_problem(p)
    np.testing.assert_array_equal(a["sigma_s"][0], p["sigma_s"][0].T)
    np.testing.assert_array_equal(a["sigma_t"], p["sigma_t"])
    np.testing.assert_array_equal(a["source"]["lo"], p["qoi"]["lo"])
    np.testing.assert_array_equal(a["source"]["hi"], p["qoi"]["hi"])
    assert math.isclose(a["source"]["group_pmf"].sum(), 1.0)
    assert a["qoi"] is None
    for k in range(3):
        np.testing.assert_array_equal(a["tally"]["mesh"][k], p["ww_mesh"][k])
    # the adjoint of the adjoint scatters like the original
    p2 = dict(a)
    p2["qoi"] = p["qoi"]
    np.testing.assert_array_equal(lw.adjoint_problem(p2)["sigma_s"], p["sigma_s"])


def test_adjoint_rejects_time_dependent_and_weighted():
    p = w.cfg2_slab_pulse()
    p["ww_mesh"] = [p["tally"]["mesh"][0], np.zeros(0), np.zeros(0)]
    p["qoi"] = {"lo": np.array([0.0, 0, 0]), "hi": np.array([1.0, 0, 0]), "group_mask": np.array([1])}
    with pytest.raises(ValueError):
        lw.adjoint_problem(p)
    q = w.cfg5_dogleg()
    q["sigma_s"] = q["sigma_s"].copy()
    q["sigma_s"][0, 0, 1] = 0.0
    q["sigma_s"][0, 1, 0] = 1.2      # transposed row 0 would exceed sigma_t
    with pytest.raises(ValueError):
        lw.adjoint_problem(q)


def test_features_layout():
    p = w.cfg5_dogleg()
    X = lw.cell_features(p)
    assert X.shape == (2 * 10 * 10 * 40, 8) and X.dtype == np.float32
    X5 = X.reshape(1, 2, 10, 10, 40, 8)
    assert np.allclose(X5[0, 0, 0, 0, :, 0], (np.arange(40) + 0.5) / 40)
    assert np.allclose(X5[0, 1, 3, :, 0, 1], (np.arange(10) + 0.5) / 10)
    assert (X5[0, 0, ..., 3] == 1).all() and (X5[0, 0, ..., 4] == 0).all()
    assert (X5[0, 1, ..., 4] == 1).all()
    assert (X5[..., 5:] == 0).all()


def test_source_cells():
    p = w.cfg5_dogleg()
    sc = lw.source_cells(p)
    assert sc.shape == (10, 10, 40)
    # source box x in [0,1] (cells 0,1 of 0.75), y in [1,3] (cells 1,2), z in [4,6] (cells 4,5)
    assert sc.sum() == 2 * 2 * 2 and sc[4:6, 1:3, 0:2].all()


def test_centres_from_log_importance():
    logI = np.array([-3.0, -2.0, -1.0, 0.0, -np.inf])
    c = lw.centres_from_log_importance(logI, -2.0, (5,))
    assert c[0] == 0.0 and c[4] == 0.0            # below the reference: analog
    assert np.isclose(c[1], 1.0) and np.isclose(c[2], 0.1) and np.isclose(c[3], 0.01)
