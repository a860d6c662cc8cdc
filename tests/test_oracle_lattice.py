"""Pins of the oracle's block reuse on regular arrays (Section 4, the
identical-scatterer paragraph; Table 7): the reuse ratio against the printed
Reuse column, the count of distinct displacements against the closed form,
and the block-table apply against the brute-force-pinned pair sum."""
import os

import numpy as np
import pytest

from oracle import geometry as geo
from oracle import lattice, pairsum
from paper_2606_31380_amd import scenarios as sc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table7_block_reuse.txt")


def test_reuse_ratio_matches_table7():
    rows = np.loadtxt(GOLDEN)
    assert rows.shape == (5, 3)
    for P, ngeo, pct in rows:
        P = int(P)
        assert P ** 3 == int(ngeo)
        # printed to one decimal
        assert abs(100.0 * lattice.reuse_ratio(P, P, P) - pct) <= 0.05 + 1e-9


@pytest.mark.parametrize("dims", [(2, 3, 4), (1, 3, 2), (3, 1, 1), (2, 2, 2)])
def test_distinct_displacement_count(dims):
    P, Q, R = dims
    d = lattice.distinct_displacements(P, Q, R)
    assert len(d) == (2 * P - 1) * (2 * Q - 1) * (2 * R - 1) - 1
    assert (0, 0, 0) not in d


def test_lattice_sites_recovers_shuffled_array():
    s = sc.identical_array((2, 3, 2), (3.0, 2.5, 3.5), seed=3)
    sites, dims, h = lattice.lattice_sites(np.stack([s.bodies["cx"], s.bodies["cy"], s.bodies["cz"]], 1))
    assert dims == (2, 3, 2)
    assert np.allclose(h, [3.0, 2.5, 3.5])
    assert np.allclose(sites * h, np.stack([s.bodies["cx"], s.bodies["cy"], s.bodies["cz"]], 1))
    with pytest.raises(ValueError):
        lattice.lattice_sites(np.array([[0.0, 0, 0], [1.0, 0, 0], [2.5, 0, 0]]))
    with pytest.raises(ValueError):
        lattice.lattice_sites(np.array([[0.0, 0, 0], [1.0, 0, 0], [0.0, 1.0, 0]]))


@pytest.mark.parametrize("eta,single", [(None, False), (1.4, False), (None, True)])
def test_block_table_apply_equals_pair_sum(eta, single):
    s = sc.identical_array((2, 2, 3), (3.0, 2.5, 3.5), seed=1)
    d = geo.discretize(s)
    n = d.pos.shape[0]
    rng = np.random.default_rng(2)
    mu = rng.standard_normal((n, 2)) + 1j * rng.standard_normal((n, 2))
    got = lattice.lattice_apply(d, 2.0, mu, eta=eta, single=single)
    want = pairsum.pair_sum(d, s.k, mu, eta=eta, single=single)
    assert np.abs(got - want).max() < 1e-13 * np.abs(want).max()
