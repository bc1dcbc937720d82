"""Host logic of the apply_H autotuner: candidate shapes, cache keys, the
cache file round trip and the choice of the fastest candidate (no GPU)."""
import json

import pytest
import torch

from paper_2002_05725_amd import autotune


def test_candidates_cover_valid_tiles():
    assert autotune.candidates(52) == [(tb, x, 1) for tb in (8, 9, 10, 11) for x in (1, 0)]
    assert autotune.candidates(18) == [(8, 1, 1), (8, 0, 1), (9, 1, 1), (9, 0, 1)]
    assert autotune.candidates(8) == [(4, 1, 1), (4, 0, 1)]
    # two columns per workgroup: even blocks, tiles of 2^10 and 2^11 rows only
    assert autotune.candidates(52, 64) == autotune.candidates(52) + [(10, 1, 2), (10, 0, 2), (11, 1, 2), (11, 0, 2)]
    assert autotune.candidates(52, 3) == autotune.candidates(52)
    assert autotune.candidates(18, 64) == autotune.candidates(18)
    assert autotune.candidates(20, 2) == autotune.candidates(20) + [(10, 1, 2), (10, 0, 2)]
    for N in (8, 12, 18, 24, 52, 60):
        for nvec in (1, 2, 5, 64):
            for tb, x, nc in autotune.candidates(N, nvec):
                assert tb <= N // 2 and tb <= 11 and x in (0, 1) and nc in (1, 2)
                assert nc == 1 or (tb >= 10 and nvec % 2 == 0)


def test_cache_key_separates_every_field():
    keys = {autotune.cache_key(a, N, d, b) for a in ("gfx950", "gfx942") for N in (36, 40)
            for d in (torch.complex64, torch.complex128) for b in (1, 64)}
    assert len(keys) == 16
    with pytest.raises(KeyError):
        autotune.cache_key("gfx950", 36, torch.float32, 1)


def test_cache_round_trip(tmp_path):
    p = str(tmp_path / "sub" / "tune.json")
    assert autotune.read_cache(p) == {}
    autotune.write_cache(p, "k1", {"tile_bits": 11, "xcd_remap": 1, "ms": 2.0})
    autotune.write_cache(p, "k2", {"tile_bits": 9, "xcd_remap": 0, "ms": 1.0})
    autotune.write_cache(p, "k1", {"tile_bits": 10, "xcd_remap": 0, "ms": 1.5})
    d = json.load(open(p))
    assert d == {"k1": {"tile_bits": 10, "xcd_remap": 0, "ms": 1.5}, "k2": {"tile_bits": 9, "xcd_remap": 0, "ms": 1.0}}


def test_pick_fastest_first_on_ties():
    t = [{"tile_bits": 8, "xcd_remap": 1, "ms": 3.0}, {"tile_bits": 9, "xcd_remap": 1, "ms": 2.0},
         {"tile_bits": 10, "xcd_remap": 0, "ms": 2.0}]
    assert autotune.pick(t)["tile_bits"] == 9
    with pytest.raises(ValueError):
        autotune.pick([])
