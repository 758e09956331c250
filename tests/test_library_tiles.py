"""Tile cache of the batched ensemble step (host only, no device): entries
written by the library read back unchanged; a cache in the same format
written by hand (extra keys, candidates, other key order) parses; malformed
files and inadmissible tiles (a z-tile other than 4, 8, 16, gm = 4 for
mp = 2, tz = 8 with the radix-16 length 192) are rejected."""
import json

import pytest

import paper_1705_03838_amd as opf

ENTRIES = [dict(N=32, M=16, K=24, mp=1, precision=opf.OPF_MIXED, gm=2, tz=8, ztile=4),
           dict(N=48, M=24, K=32, mp=1, precision=opf.OPF_MIXED, gm=4, tz=4, ztile=8),
           dict(N=21, M=6, K=4, mp=2, precision=opf.OPF_FP64, gm=1, tz=2, ztile=16)]
KEYS = ("N", "M", "K", "mp", "precision", "gm", "tz", "ztile")


def test_round_trip(tmp_path):
    path = str(tmp_path / "tiles.json")
    opf.tile_cache_write(ENTRIES, path)
    back = opf.tile_cache_read(path)
    assert [{k: e[k] for k in KEYS} for e in back] == ENTRIES
    text = json.load(open(path))
    assert text["version"] == 1 and len(text["classes"]) == 3


def test_hand_written_cache_parses(tmp_path):
    path = tmp_path / "hand.json"
    path.write_text(json.dumps({"version": 1, "note": "tuned elsewhere", "classes": [
        {"ztile": 8, "tz": 4, "gm": 4, "precision": 1, "mp": 1, "K": 48, "M": 32, "N": 64, "members": 32,
         "us_per_step": 1.5, "candidates": [{"gm": 1, "tz": 4, "ztile": 8, "us_per_step": 3.0}]}]}, indent=2))
    back = opf.tile_cache_read(str(path))
    assert [{k: e[k] for k in KEYS} for e in back] == [dict(N=64, M=32, K=48, mp=1, precision=1, gm=4, tz=4,
                                                             ztile=8)]


@pytest.mark.parametrize("bad", [
    dict(ENTRIES[0], ztile=32, K=64),   # z tiles are 4, 8 or 16 radial lines
    dict(ENTRIES[0], tz=8, M=64),       # length 192 in theta: 8 x 16 > 64
    dict(ENTRIES[2], gm=4),             # mp = 2 shares at most 2 m
    dict(ENTRIES[0], tz=3),
])
def test_inadmissible_tiles_rejected(tmp_path, bad):
    with pytest.raises(opf.OpfError):
        opf.tile_cache_write([bad], str(tmp_path / "x.json"))
    path = tmp_path / "y.json"
    path.write_text(json.dumps({"version": 1, "classes": [bad]}))
    with pytest.raises(opf.OpfError):
        opf.tile_cache_read(str(path))


@pytest.mark.parametrize("text", ["", "{", "[]", '{"classes": {}}', '{"classes": [{"N": 1}]}',
                                  '{"classes": [{"N": 32, "M": 16, "K": 24, "mp": 1, "precision": 1, "gm": 2.5, '
                                  '"tz": 4, "ztile": 8}]}', '{"classes": []} trailing'])
def test_malformed_cache_rejected(tmp_path, text):
    path = tmp_path / "m.json"
    path.write_text(text)
    with pytest.raises(opf.OpfError):
        opf.tile_cache_read(str(path))
    with pytest.raises(opf.OpfError):
        opf.tile_cache_read(str(tmp_path / "missing.json"))
