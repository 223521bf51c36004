"""The tile cache of cq_crowd_autotune_tiles (host code only, CPU): entries round-trip, the
last matching entry wins, keys must all match, the file stays a valid JSON array, lines that
do not parse are skipped, and bad arguments are refused."""
import json
import os

import pytest

import paper_2209_14487_amd as cq

DEV = "gfx950:sramecc+:xnack-/256cu"


def test_store_and_find_round_trip(tmp_path):
    p = str(tmp_path / "tiles.json")
    assert cq.tile_cache_find(p, DEV, 1024, 128, "mixed", 32) is None  # no file yet
    cq.tile_cache_store(p, DEV, 1024, 128, "mixed", 32, 64, 2, 31.5)
    cq.tile_cache_store(p, DEV, 256, 512, "mixed", 32, 48, 1, 6.25)
    cq.tile_cache_store(p, DEV, 1024, 128, "fp64", 32, 88, 3, 60.0, update_kernel=2)
    T = lambda q, g, u=0: dict(candidates=q, gather_blocks_per_cu=g, update_kernel=u)
    assert cq.tile_cache_find(p, DEV, 1024, 128, "mixed", 32) == T(64, 2)
    assert cq.tile_cache_find(p, DEV, 256, 512, "mixed", 32) == T(48, 1)
    assert cq.tile_cache_find(p, DEV, 1024, 128, "fp64", 32) == T(88, 3, 2)
    # every key must match
    assert cq.tile_cache_find(p, DEV, 1024, 128, "mixed", 16) is None
    assert cq.tile_cache_find(p, DEV, 1024, 64, "mixed", 32) is None
    assert cq.tile_cache_find(p, DEV, 512, 128, "mixed", 32) is None
    assert cq.tile_cache_find(p, "gfx942/304cu", 1024, 128, "mixed", 32) is None
    # a later entry for the same key wins
    cq.tile_cache_store(p, DEV, 1024, 128, "mixed", 32, 48, 1, 30.0)
    assert cq.tile_cache_find(p, DEV, 1024, 128, "mixed", 32) == T(48, 1)
    # the file is a JSON array of the stored objects, in order
    rec = json.load(open(p))
    assert [r["candidates"] for r in rec] == [64, 48, 88, 48]
    assert rec[0] == dict(device=DEV, n=1024, walkers=128, precision="mixed", delay_rank=32, candidates=64,
                          gather_blocks_per_cu=2, update_kernel=0, ms_per_sweep=31.5)
    assert rec[2]["update_kernel"] == 2


def test_lines_that_do_not_parse_are_skipped(tmp_path):
    p = str(tmp_path / "tiles.json")
    good = ('{"device": "%s", "n": 64, "walkers": 16, "precision": "fp64", "delay_rank": 8, '
            '"candidates": 16, "gather_blocks_per_cu": 2, "ms_per_sweep": 1.5}' % DEV)
    with open(p, "w") as f:
        f.write("[\n")
        f.write('{"device": "%s", "n": 64, "walkers": 16, "precision": "fp64", "delay_rank": 8, '
                '"candidates": "many", "gather_blocks_per_cu": 2},\n' % DEV)  # not a number
        f.write('{"device": "%s", "n": 64, "walkers": 16, "precision": "fp64", "delay_rank": 8\n' % DEV)  # cut
        f.write("garbage\n")
        f.write('{"device": "%s", "n": 64, "walkers": 16, "precision": "fp64", "delay_rank": 8, '
                '"gather_blocks_per_cu": 2},\n' % DEV)  # no candidates
        f.write(good + "\n]\n")
    # (an entry written without update_kernel reads it as 0)
    assert cq.tile_cache_find(p, DEV, 64, 16, "fp64", 8) == dict(candidates=16, gather_blocks_per_cu=2, update_kernel=0)
    # storing rewrites the file as valid JSON: the objects that parse (with or without the
    # fields a lookup needs) and the new one; the cut line and the garbage are dropped
    cq.tile_cache_store(p, DEV, 64, 16, "mixed", 8, 12, 1, 1.0)
    rec = json.load(open(p))
    assert len(rec) == 4 and rec[0]["candidates"] == "many" and rec[-1]["precision"] == "mixed"
    assert not os.path.exists(p + ".tmp")


@pytest.mark.parametrize("dev,n,w,k,q,g,ms,u", [
    ('bad"name', 64, 16, 8, 16, 1, 1.0, 0), ("", 64, 16, 8, 16, 1, 1.0, 0), ("x" * 128, 64, 16, 8, 16, 1, 1.0, 0),
    (DEV, 0, 16, 8, 16, 1, 1.0, 0), (DEV, 64, 0, 8, 16, 1, 1.0, 0), (DEV, 64, 16, 0, 16, 1, 1.0, 0),
    (DEV, 64, 16, 8, -1, 1, 1.0, 0), (DEV, 64, 16, 8, 16, 65, 1.0, 0), (DEV, 64, 16, 8, 16, 1, float("nan"), 0),
    (DEV, 64, 16, 8, 16, 1, 1.0, 3), (DEV, 64, 16, 8, 16, 1, 1.0, -1)])
def test_bad_entries_are_refused(tmp_path, dev, n, w, k, q, g, ms, u):
    p = str(tmp_path / "tiles.json")
    with pytest.raises(cq.CqError) as ei:
        cq.tile_cache_store(p, dev, n, w, "mixed", k, q, g, ms, update_kernel=u)
    assert ei.value.status == cq.CQ_EINVAL
    assert not os.path.exists(p)


def test_unwritable_cache_is_an_io_error(tmp_path):
    p = str(tmp_path / "no_such_dir" / "tiles.json")
    with pytest.raises(cq.CqError) as ei:
        cq.tile_cache_store(p, DEV, 64, 16, "mixed", 8, 16, 1, 1.0)
    assert ei.value.status == cq.CQ_EIO
    assert cq.tile_cache_find(p, DEV, 64, 16, "mixed", 8) is None  # missing file: no entry, no error
