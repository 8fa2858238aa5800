"""Brute force on tiny inputs: the oracle's event-by-event traces equal those
of a separately written pure-Python tracer bit for bit (positions, times,
groups, optical depths), so a slip of index, sign or order in either shows."""
import math

import numpy as np
import pytest

import oracle
import workloads as w
from refs import PyTracer


def tiny_lattice():
    # 3x2 lattice with a mesh that does not coincide with the geometry,
    # three groups with up-scatter, two materials, one void-free, mixed BCs,
    # finite time grid so census, surface, collision and cut-off all occur
    st = [[1.0, 1.5, 2.0], [0.4, 0.8, 0.3]]
    ss = [[[0.3, 0.4, 0.1], [0.0, 0.6, 0.5], [0.0, 0.2, 1.2]],
          [[0.1, 0.1, 0.0], [0.0, 0.3, 0.2], [0.0, 0.0, 0.25]]]
    planes = [np.array([0.0, 1.0, 2.5, 3.0]), np.array([0.0, 0.7, 2.0]), np.array([0.0, 1.5])]
    mat = np.array([[[0, 1, 0], [1, 1, 0]]])
    mesh = [np.array([0.5, 1.0, 2.0, 3.0]), np.array([0.0, 1.0, 2.0]), np.array([0.0, 0.75, 1.5])]
    src = {"kind": "isotropic", "lo": [0.2, 0.1, 0.3], "hi": [2.9, 1.9, 1.2],
           "group_pmf": [0.5, 0.3, 0.2], "t_lo": 0.0, "t_hi": 0.5}
    tally = {"mesh": mesh, "time_edges": [0.0, 0.4, 1.0, 2.5, 6.0], "n_batches": 4}
    return w.make_problem(st, ss, [3.0, 2.0, 1.0], planes, mat, [1, 0, 0, 1, 1, 0], src, tally)


CASES = {
    "lattice": (tiny_lattice, 40),
    "slab_cosine": (lambda: w.cfg1_slab_steady(c=0.5, mu_law="cosine"), 40),
    "slab_beam": (lambda: w.cfg1_slab_steady(c=0.7, mu_law="beam"), 30),
    "slab_uniform": (lambda: w.cfg1_slab_steady(c=0.7, mu_law="uniform"), 30),
    "pulse": (lambda: w.cfg2_slab_pulse(c=0.9), 20),
    "void_box": (lambda: w.void_box(), 30),
    "reflective_mg": (lambda: w.reflective_box([1.0, 1.5], [[0.5, 0.3], [0.1, 1.2]], [2.0, 1.0],
                                               time_edges=[0.0, 1.0, 3.0]), 30),
    # speeds that are not powers of two and many census edges: the census
    # time snap differs from t + d / v in the last bit here
    "census_heavy": (lambda: w.reflective_box([0.3, 0.5], [[0.1, 0.15], [0.0, 0.4]], [0.7, 1.3],
                                              time_edges=np.linspace(0.0, 9.1, 71)), 200),
}


@pytest.mark.parametrize("name", list(CASES))
def test_trace_matches_python_tracer(name):
    make, n = CASES[name]
    p = make()
    N, seed = 1000, 77
    tr = PyTracer(p, N, seed)
    for i in [0, 1, 2, 3, 999] + list(range(10, 10 + n)):
        a = oracle.trace(p, N, seed, i)
        b = np.array(tr.history(i), dtype=float)
        assert a.shape == b.shape, (name, i, a.shape, b.shape)
        assert np.array_equal(a, b), (name, i, np.argwhere(a != b)[:5])


def test_trace_consistent_with_run_records():
    p = tiny_lattice()
    N, seed = 200, 9
    res = oracle.run(p, N, seed, records=True)
    for i in range(N):
        rows = oracle.trace(p, N, seed, i)
        ev = rows[:-1, 0]
        rec = res["rec"][i]
        assert rec[0] == (ev == 0).sum() and rec[1] == (ev == 1).sum() and rec[2] == (ev == 2).sum()
        assert rec[4] == 1 << int(rows[-1, 0] - 10)


def test_trace_exercises_every_event_and_termination():
    p = tiny_lattice()
    seen_ev, seen_term = set(), set()
    for i in range(300):
        rows = oracle.trace(p, 1000, 3, i)
        seen_ev |= set(rows[:-1, 0].astype(int))
        seen_term.add(int(rows[-1, 0]) - 10)
    assert seen_ev == {0, 1, 2}
    assert {oracle.T_ABSORB, oracle.T_LEAK, oracle.T_TIME} <= seen_term


def test_union_grid_dedups_coincident_planes():
    p = w.cfg3_lattice()
    ux = oracle.union_planes(p, 0)
    assert ux.size == 18                        # mesh planes coincide with the lattice
    uz = oracle.union_planes(p, 2)
    np.testing.assert_array_equal(uz, np.linspace(0.0, 50.0, 11))
    p5 = w.cfg5_dogleg()
    ux5 = oracle.union_planes(p5, 0)
    # 41 mesh planes (0.75 apart, 12 = 16 * 0.75 coincides) plus the
    # geometry plane at 10 and the detector face at 29
    assert ux5.size == 43 and 10.0 in ux5 and 29.0 in ux5 and ux5[-1] == 30.0
