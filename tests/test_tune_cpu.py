"""The autotuner's candidate lists (host logic, no GPU): every compiled launch shape appears,
each candidate once, with valid chunking and worker settings."""
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
    # every shape with every chunking, one-workgroup-per-item and both persistent grids
    assert len(cands) == len(tune.SHAPES) * (5 + 3) * 3


def test_box_candidates_respect_the_box_height():
    for nz in (4, 20, 300):
        cands = tune.box_candidates(nz)
        assert cands
        assert all(c["z_chunk"] <= max(nz, 8) for c in cands)
        keys = [tuple(sorted(c.items())) for c in cands]
        assert len(keys) == len(set(keys))
