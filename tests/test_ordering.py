"""The locality renumbering of a grid (host-side helper): a permutation of
buses, lines and generators that keeps the network, and narrows the band
of a randomly numbered grid."""
import dataclasses

import numpy as np

from synth.grids import grid_2000, power_flow_start
from oracle import acopf
from paper_2310_13143_amd.ordering import locality_order, reorder


def _shuffle(g, seed):
    rng = np.random.default_rng(seed)
    return reorder(g, rng.permutation(g.n_bus), rng.permutation(g.n_line), rng.permutation(g.n_gen))


def test_reorder_keeps_the_network_and_narrows_the_band():
    g = grid_2000()
    h = _shuffle(g, 7)
    band = lambda x: int(np.abs(x.f - x.t).max())
    bp, lp, gp = locality_order(h.n_bus, h.f, h.t, h.gbus)
    for p, n in ((bp, h.n_bus), (lp, h.n_line), (gp, h.n_gen)):
        assert np.array_equal(np.sort(p), np.arange(n))
    o = reorder(h, bp, lp, gp)
    assert band(o) < band(h) / 5
    # lines sorted by their (lower, higher) end bus, generators by bus
    key = np.minimum(o.f, o.t) * o.n_bus + np.maximum(o.f, o.t)
    assert np.all(np.diff(key) >= 0) and np.all(np.diff(o.gbus) >= 0)
    # the same network: the balance at a renumbered point equals the
    # renumbered balance
    s = power_flow_start(h)
    x = acopf.Iterate(s["pg"], s["qg"], s["w"], s["th"], s["wR"], s["wI"])
    xo = acopf.Iterate(x.pg[gp], x.qg[gp], x.w[bp], x.th[bp], x.wR[lp], x.wI[lp])
    rp, rq = acopf.balance(h, x)
    rpo, rqo = acopf.balance(o, xo)
    np.testing.assert_allclose(rpo, rp[bp], atol=1e-12)
    np.testing.assert_allclose(rqo, rq[bp], atol=1e-12)
    assert o.ref == int(np.nonzero(bp == h.ref)[0][0])
    assert dataclasses.fields(o) == dataclasses.fields(h)


def test_segment_schedules_are_permutations():
    """Scenario orders of a packed batch (the autotuner's segment
    schedules): each is a permutation; 'largest_first' sorts by line count
    keeping the given order among equal sizes; 'interleaved' takes one
    scenario of each size in turn, largest first, each size in given order."""
    from types import SimpleNamespace
    from paper_2310_13143_amd.solver import SCHEDULES, schedule_order
    sizes = [405, 2700, 13500, 405, 2700, 13500, 405, 2700, 13500, 405]
    grids = [SimpleNamespace(n_line=n) for n in sizes]
    for kind in SCHEDULES:
        assert sorted(schedule_order(grids, kind)) == list(range(len(grids)))
    assert schedule_order(grids, "given") == list(range(len(grids)))
    lf = schedule_order(grids, "largest_first")
    assert [sizes[k] for k in lf] == sorted(sizes, reverse=True)
    assert lf[:3] == [2, 5, 8] and lf[-4:] == [0, 3, 6, 9]
    il = schedule_order(grids, "interleaved")
    assert il == [2, 1, 0, 5, 4, 3, 8, 7, 6, 9]
