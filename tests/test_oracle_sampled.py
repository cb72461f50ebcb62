"""The oracle's sampled evaluation (used where the O(N^2) sweep cannot run)
against its full evaluation: every sampled sphere and clump must get exactly
the force, torque and contact list the full sweep gives it, also with
tangential history carried over from earlier steps and with boundary contacts."""
import numpy as np

import oracle
from paper_2307_03445_amd import inputs as I


def _setup(steps):
    d = I.walled_box(dense=True, n_clumps=400)
    o = oracle.Oracle(d)
    o.step(steps)
    n = o.eval()
    assert n > 0
    return d, o


def test_sampled_spheres_equal_full_evaluation():
    d, o = _setup(30)
    c = o.contacts()
    sF, sT = o.sphere_forces()
    g = np.random.default_rng(0)
    # spheres with sphere and boundary contacts, and some without any
    with_wall = np.unique(c["a"][c["b"] >= o.n_spheres])[:5]
    ids = np.unique(np.r_[g.choice(o.n_spheres, 40, replace=False), with_wall, c["a"][:5], c["b"][:5]])
    ids = ids[ids < o.n_spheres]
    F, T, sc = o.sample_spheres(ids)
    assert np.array_equal(F, sF[ids]) and np.array_equal(T, sT[ids])
    for k, s in enumerate(ids):
        full = (c["a"] == s) | (c["b"] == s)
        mine = slice(sc["beg"][k], sc["beg"][k + 1])
        assert np.all((sc["a"][mine] == s) | (sc["b"][mine] == s))
        # the full list is ascending by (a, b); the sample's ascending by partner
        ka = np.lexsort((c["b"][full], c["a"][full]))
        partner = np.where(sc["a"][mine] == s, sc["b"][mine], sc["a"][mine])
        assert np.all(np.diff(partner.astype(np.int64)) > 0)
        kb = np.lexsort((sc["b"][mine], sc["a"][mine]))
        assert np.array_equal(c["a"][full][ka], sc["a"][mine][kb])
        assert np.array_equal(c["b"][full][ka], sc["b"][mine][kb])
        assert np.array_equal(c["delta"][full][ka], sc["delta"][mine][kb])
        assert np.array_equal(c["F"][full][ka], sc["F"][mine][kb])
    assert np.any(sc["b"] >= o.n_spheres)


def test_sampled_clumps_equal_full_evaluation():
    d, o = _setup(25)
    Fc, Tc = o.clump_forces()
    ids = np.arange(0, d.n_clumps, 7)
    F, T = o.sample_clumps(ids)
    assert np.array_equal(F, Fc[ids]) and np.array_equal(T, Tc[ids])


def test_sampled_rejects_bad_ids():
    _, o = _setup(0)
    for bad in ([-1], [o.n_spheres]):
        try:
            o.sample_spheres(bad)
        except ValueError:
            pass
        else:
            raise AssertionError("out-of-range sphere id accepted")
