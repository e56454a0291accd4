"""CPU checks of the 3-state (Potts) plans: the encoded passes the library
would upload, executed by a host emulation of the kernels' algorithm, give the
oracle's ground-state energy and degeneracy."""
import numpy as np
import pytest

import potts_emulator as PE
from oracle import potts as OP
from paper_2008_06888_amd import binding as B
from paper_2008_06888_amd import instances as I


def _cases():
    out = []
    for L, Lc in ((2, 2), (3, 3), (4, 5), (6, 6)):
        for x in I.potts_lattice(L, batch=2, Lc=Lc):
            out.append((f"lat{L}x{Lc}", x, list(range(L * Lc))))
    rng = np.random.default_rng([21, 0])
    for n in (8, 12, 16):
        e = I.random_regular(n, 3, rng)
        x = I.make(e, n, rng, "pm1")
        out.append((f"reg3_{n}", x, None))
    e = I.path(7)
    out.append(("path7", I.make(e, 7, rng, "pm1"), None))
    out.append(("isolated", I.Instance(n=3, edges=np.zeros((0, 2), np.int32), J=np.zeros(0, np.int32), h=None), None))
    return out


@pytest.mark.parametrize("case", range(13))
@pytest.mark.parametrize("tiles", [(4, 3), (2, 2), (3, 2)])
def test_encoded_potts_program_matches_oracle(case, tiles):
    name, x, order = _cases()[case]
    plan = B.Plan(x.n, x.edges, order=order, q=3, tile_bits=tiles[0], count_tile_bits=tiles[1])
    info = plan.info()
    w = info["width"]
    ref = OP.eliminate(x.n, x.edges, x.J, counts="exact")
    ep = PE.parse_passes(plan.program(7))
    cp = PE.parse_passes(plan.program(8))
    red = PE.parse_reduce(plan.program(9))
    assert len(ep) == info["n_passes"] and len(cp) == info["n_count_passes"]
    best, _ = PE.run(ep, red, x.J, w)
    assert -best == ref["energy2"], name
    best_c, g = PE.run(cp, red, x.J, w, count=True)
    assert -best_c == ref["energy2"] and g == ref["count"], name


def test_potts_plan_options_validated():
    e = I.square_lattice(3)
    with pytest.raises(B.TTError):
        B.Plan(9, e, q=3, has_field=True)
    with pytest.raises(B.TTError):
        B.Plan(9, e, q=3, tile_bits=5)
    with pytest.raises(B.TTError):
        B.Plan(9, e, q=3, count_tile_bits=1)
    with pytest.raises(B.TTError):
        B.Plan(9, e, q=4)
    p = B.Plan(9, e, q=3, order=list(range(9)))
    # an Ising call on a 3-state plan is refused before any device work
    with pytest.raises(B.TTError):
        B.lib().tt_contract(p.handle, 1, 0, None, None, None, None) and B._check(-1)
    code = B.lib().tt_contract(p.handle, 1, 0, None, None, None, None)
    assert code == B.TT_E_INVAL and "3-state" in B.last_error()


def test_potts_width_limit():
    # a 21 x 21 lattice in raster order needs 3^21 entries per instance: refused at planning
    e = I.square_lattice(21)
    with pytest.raises(B.TTError) as ei:
        B.Plan(441, e, order=list(range(441)), q=3)
    assert ei.value.code == B.TT_E_TOOBIG
