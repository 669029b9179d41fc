"""Pins of the oracle's cube/subcube grid (locate, neighbours) by brute force."""
import numpy as np

import oracle
import synth


def _grid_session():
    w = synth.small_disk(nb=8, n_sizes=1, nl=8)
    return w, oracle.Session(w)


def test_leaf_volumes_fill_the_box():
    w = synth.c2_disk(n_packets=10)
    lo, side = w.grid.leaf_boxes_cm()
    assert abs((side ** 3).sum() / (w.grid.nb * w.grid.base_size) ** 3 - 1) < 1e-12
    assert w.grid.n_cells == 262480


def test_locate_equals_brute_force():
    w, s = _grid_session()
    g = w.grid
    nf = 1 << g.max_level
    lo = g.leaf_lo.astype(np.int64)
    span = (nf >> g.leaf_level.astype(np.int64))
    rng = np.random.default_rng(5)
    pts = rng.integers(0, g.nb * nf, size=(3000, 3))
    # make sure the refined region is hit
    pts[:500] = rng.integers(g.nb * nf // 2 - 6, g.nb * nf // 2 + 6, size=(500, 3))
    for F in pts:
        inside = np.all((lo <= F) & (F < lo + span[:, None]), axis=1)
        assert inside.sum() == 1
        c, lev, clo = s.locate(F)
        assert c == int(np.nonzero(inside)[0][0])
        assert lev == g.leaf_level[c] and tuple(clo) == tuple(lo[c])
    assert s.locate([-1, 0, 0])[0] == -1
    assert s.locate([0, g.nb * nf, 0])[0] == -1


def test_face_neighbours_are_symmetric():
    w, s = _grid_session()
    g = w.grid
    nf = 1 << g.max_level
    rng = np.random.default_rng(9)
    for c in rng.choice(g.n_cells, 400, replace=False).tolist() + list(range(min(g.n_cells, 64))):
        lo = g.leaf_lo[c].astype(np.int64)
        span = nf >> int(g.leaf_level[c])
        for ax in range(3):
            for sgn in (+1, -1):
                F = lo + rng.integers(0, span, size=3)
                F[ax] = lo[ax] + span if sgn > 0 else lo[ax] - 1
                c2, lev2, lo2 = s.locate(F)
                if c2 < 0:
                    continue
                lo2 = np.array(lo2)
                span2 = nf >> lev2
                # touching across the face, footprint containing F
                assert (lo2[ax] == lo[ax] + span) if sgn > 0 else (lo2[ax] + span2 == lo[ax])
                back = F.copy()
                back[ax] = lo2[ax] - 1 if sgn > 0 else lo2[ax] + span2
                # stepping back from c2 at a point of c2's face inside c's footprint returns c
                assert s.locate(back)[0] == c
