"""The autotuner's candidate lists (host logic, no GPU): every compiled launch shape appears,
each candidate once, with valid chunking and worker settings."""
import pytest

import paper_2105_08772_amd.tune as tune


def shape_key(c):
    return (c["waves"], c["rows"], c["prefetch"], c["tile_x"])


def test_shapes_are_the_compiled_ones():
    want = set()
    for tx in (64, 32):
        for r in ((1, 2, 4) if tx == 64 else (1, 2)):
            for pf in (0, 1):
                want.add((4, r, pf, tx))
        for r in (1, 2):
            want.add((8, r, 0, tx))
    want |= {(8, 2, 0, 0), (8, 4, 0, 0), (8, 8, 0, 0), (4, 4, 0, 0)}
    got = [shape_key(s) for s in tune.SHAPES]
    assert len(got) == len(set(got))
    assert set(got) == want


def test_group_candidates_are_unique_and_valid():
    cands = tune.group_candidates()
    keys = [tuple(sorted(c.items())) for c in cands]
    assert len(keys) == len(set(keys))
    for c in cands:
        assert c["z_chunk"] >= 0 and c["xcd_remap"] == 1
        if c["z_chunk"] == 0:
            assert c["items_per_cu"] in (4, 8, 16)
        else:
            assert c["items_per_cu"] == 0
        if c["persistent"]:
            assert c["workers"] in (256, 512) and c["workers"] % 8 == 0
        else:
            assert c["workers"] == 0
    # every shape with every chunking, one-workgroup-per-item and both persistent grids; every
    # two-step shape with its chunkings, one workgroup per item
    one = [c for c in cands if c["steps_per_pass"] == 1]
    two = [c for c in cands if c["steps_per_pass"] == 2]
    assert len(one) == len(tune.SHAPES) * (5 + 3) * 3
    assert len(two) == len(tune.SHAPES2) * (5 + 3) and not any(c["persistent"] for c in two)
    assert all(c["z_chunk"] == 0 or c["z_chunk"] >= 16 for c in two)
    assert len(tune.group_candidates(two_step=False)) == len(one)


def test_box_candidates_respect_the_box_height():
    for nz in (4, 20, 300):
        cands = tune.box_candidates(nz)
        assert cands
        assert all(c["z_chunk"] <= max(nz, 8) for c in cands)
        keys = [tuple(sorted(c.items())) for c in cands]
        assert len(keys) == len(set(keys))


def test_tune_group_keeps_the_graph_chunk_and_refuses_when_nothing_fits(monkeypatch):
    """On a stand-in group: the fastest candidate is set with the group's own graph chunk length
    restored (candidates are timed with chunks of `steps`), and a group that no candidate fits
    raises instead of failing on an empty result."""
    from paper_2105_08772_amd import LbmScError

    class FakeGroup:
        def __init__(self, cost, fits=lambda c: True):
            self.shape = dict(graph_steps=64, rows=1)
            self.cost, self.fits = cost, fits

        def set_launch(self, **kw):
            if not self.fits(kw):
                raise LbmScError(-1, "does not fit")
            self.shape.update(kw)

        def launch(self):
            return dict(self.shape)

        def step(self, n):
            clock[0] += n * self.cost[self.shape["rows"]]

    clock = [0.0]
    monkeypatch.setattr(tune, "_sync", lambda: None)
    monkeypatch.setattr(tune.time, "perf_counter", lambda: clock[0])
    cands = [dict(rows=r) for r in (1, 2, 4)]
    g = FakeGroup({1: 3.0, 2: 1.0, 4: 2.0}, fits=lambda c: c.get("rows") != 4)
    best = tune.tune_group(g, steps=8, candidates=cands)
    assert best["rows"] == 2 and best["seconds_per_step"] == 1.0
    assert g.launch() == dict(graph_steps=64, rows=2)
    with pytest.raises(ValueError):
        tune.tune_group(FakeGroup({}, fits=lambda c: False), candidates=cands)
