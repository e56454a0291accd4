"""Oracle pins on the paper's 3D lattices (open simple cubic boxes): brute
force on boxes of up to 24 spins, planted instances at full size, and the
diagonal-plane elimination order the GPU parity tests hand to the oracle."""
import itertools

import numpy as np
import pytest

from oracle import spinglass as O
from paper_2008_06888_amd import instances as I


def diagonal_order(Lx, Ly, Lz):
    """Spins sorted by x + y + z (then z, y, x): an elimination order of the
    oracle's own whose induced width grows like the largest diagonal plane."""
    pts = sorted(itertools.product(range(Lx), range(Ly), range(Lz)), key=lambda p: (sum(p), p[2], p[1], p[0]))
    return [(z * Ly + y) * Lx + x for x, y, z in pts]


def test_edge_count_and_indexing():
    for dims in ((2, 2, 2), (3, 4, 5), (6, 6, 6)):
        Lx, Ly, Lz = dims
        e = I.cubic_lattice(*dims)
        assert len(e) == (Lx - 1) * Ly * Lz + Lx * (Ly - 1) * Lz + Lx * Ly * (Lz - 1)
        deg = np.bincount(e.reshape(-1), minlength=Lx * Ly * Lz)
        assert deg.max() <= 6 and deg.min() == 3       # corners have three neighbours


@pytest.mark.parametrize("dims", [(2, 2, 2), (2, 3, 3), (2, 3, 4)])
def test_cubic_elimination_equals_brute_force(dims):
    x = I.cubic_instances(*dims)[0]
    bf = O.brute_force(x.n, x.edges, x.J, None)
    for order in (None, diagonal_order(*dims)):
        r = O.eliminate(x.n, x.edges, x.J, None, order=order, counts="exact")
        assert r["energy"] == bf["energy"] and r["count"] == bf["count"]
        assert O.energy(x.n, x.edges, x.J, None, r["sigma"]) == bf["energy"]


def test_cubic_gauss_with_fields_unique_ground_state():
    x = I.cubic_instances(2, 3, 3, coupling="gauss", field_std=0.1)[0]
    bf = O.brute_force(x.n, x.edges, x.J, x.h)
    r = O.eliminate(x.n, x.edges, x.J, x.h, order=diagonal_order(2, 3, 3))
    assert abs(r["energy"] - bf["energy"]) < 1e-9 and np.array_equal(r["sigma"], bf["sigma"])


def test_diagonal_order_width():
    # buckets hold about one diagonal plane plus the spin eliminated: widths 15 and 22 here,
    # against 18 and 30 for the oracle's min-fill order
    for L, w_max in ((4, 15), (5, 22)):
        e = I.cubic_lattice(L)
        assert O.induced_width(L ** 3, e, diagonal_order(L, L, L)) <= w_max


def test_planted_cubic_closed_form():
    e = I.cubic_lattice(4)
    x, tau = I.planted(e, 64, np.random.default_rng([6, 99]))
    r = O.eliminate(64, e, x.J, None, order=diagonal_order(4, 4, 4), counts="exact")
    assert r["energy"] == -len(e) and r["count"] == 2
    assert np.array_equal(r["sigma"], tau) or np.array_equal(r["sigma"], -tau)
