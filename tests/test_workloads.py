"""Seeded input generators (the only module the oracle and the GPU path share)."""
import math

import numpy as np

from paper_1709_08803_amd import workloads as W


def test_sweep_is_reproducible_and_follows_the_mesh_rule():
    a = W.sweep_instances(16, seed=3)
    b = W.sweep_instances(16, seed=3)
    for p, q in zip(a, b):
        assert p.name == q.name and p.froude == q.froude
        assert np.array_equal(p.beta, q.beta)
        assert 61 <= p.N <= 181 and p.N % 3 == 1 and p.M == (p.N - 1) // 3 + 1
        assert math.isclose(p.dx, p.dy) and p.half_domain and p.y1 == 0.0
        assert 0.5 <= p.froude <= 2.0


def test_sweep_ranges_and_kinds_can_be_narrowed():
    ps = W.sweep_instances(40, seed=5, fixed_n=31, domain=(-15.0, 15.0, 10.0), froude=(0.8, 1.8),
                           height=(0.1, 0.3), width=(0.7, 1.5), kinds=(0, 2))
    for p in ps:
        assert (p.N, p.M) == (31, 11) and math.isclose(p.x1, -15.0)
        assert 0.8 <= p.froude <= 1.8
        assert "-k1-" not in p.name  # no transverse ridges
        assert 0.1 <= p.beta.max() + 1.0 <= 0.3 + 1e-12


def test_default_ranges_keep_the_original_random_stream():
    # narrowing nothing must reproduce the default sweep draw for draw
    a = W.sweep_instances(8, seed=9)
    b = W.sweep_instances(8, seed=9, froude=(0.5, 2.0), width=(0.5, 2.0), kinds=(0, 1, 2))
    assert [p.name for p in a] == [p.name for p in b]
    assert all(np.array_equal(p.beta, q.beta) for p, q in zip(a, b))


def test_half_domain_topography_is_even_in_y():
    p = W.make_problem(41, 15, -10, 10, 0, 7, 1.0, [W.Bump(0.2, 1.0, 1.0, cx=1.0, cy=2.0)])
    full = W.make_problem(41, 29, -10, 10, -7, 7, 1.0, [W.Bump(0.2, 1.0, 1.0, cx=1.0, cy=2.0),
                                                       W.Bump(0.2, 1.0, 1.0, cx=1.0, cy=-2.0)],
                          half_domain=False)
    assert np.allclose(full.beta[14:], p.beta)        # rows y >= 0
    assert np.allclose(full.beta[14::-1], p.beta)     # mirrored rows
    assert np.allclose(full.beta_y[14:], p.beta_y)
