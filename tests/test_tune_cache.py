"""Autotuning table (no GPU): the JSON cache round trip and the keying of lookups.

A lookup matches the device architecture, dim, n, entries per row and
precision exactly and takes, among the tuned counts, the largest one not above
the requested count; anything else is "no entry"."""
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture()
def pfc():
    if not os.path.exists(os.path.join(ROOT, "paper_1501_06852_amd", "libpfc.so")):
        pytest.skip("library not built")
    from paper_1501_06852_amd import pfc as lib
    lib.pfc_tune_clear()
    yield lib
    lib.pfc_tune_clear()


def _entry(count, rpt, **kw):
    e = dict(arch="gfx950", dim=2, n=16384, z=7, precision=1, count=count, rows_per_thread=rpt, ticks_per_graph=64,
             pcg_steps_per_launch=1, grid_columns=1, shared_ops=1, ms_per_step=10.0 * count, ms_default=11.0 * count,
             candidates=9)
    e.update(kw)
    return e


def test_lookup_takes_largest_tuned_count_not_above(pfc, tmp_path):
    p = tmp_path / "tune.json"
    entries = [_entry(1, 1), _entry(16, 2), _entry(256, 4, ticks_per_graph=128),
               _entry(16, 8, precision=0), _entry(16, 8, arch="gfx942"), _entry(16, 8, z=15, dim=3)]
    p.write_text(json.dumps({"format": "pfc-tune-1", "entries": entries}))
    pfc.pfc_tune_load(str(p))
    look = lambda count, **kw: pfc.pfc_tune_lookup(kw.get("dim", 2), kw.get("n", 16384), kw.get("z", 7),
                                                   kw.get("precision", 1), count, arch=kw.get("arch", "gfx950"))
    assert look(1)["rows_per_thread"] == 1
    assert look(15)["rows_per_thread"] == 1
    assert look(16)["rows_per_thread"] == 2
    assert look(255)["rows_per_thread"] == 2
    e = look(300)
    assert (e["rows_per_thread"], e["ticks_per_graph"], e["count"], e["from_cache"]) == (4, 128, 256, 1)
    assert look(16, precision=0)["rows_per_thread"] == 8
    assert look(16, arch="gfx942")["rows_per_thread"] == 8
    assert look(16, dim=3, z=15)["rows_per_thread"] == 8
    # no entry: other n, other z, other precision with a smaller count, unknown architecture
    assert look(16, n=4096) is None
    assert look(16, z=15) is None
    assert look(8, precision=0) is None
    assert look(16, arch="gfx90a") is None


def test_save_load_round_trip_and_replacement(pfc, tmp_path):
    p = tmp_path / "a.json"
    p.write_text(json.dumps({"format": "pfc-tune-1", "entries": [_entry(16, 2), _entry(1, 1)]}))
    pfc.pfc_tune_load(str(p))
    q = tmp_path / "b.json"
    pfc.pfc_tune_save(str(q))
    d = json.loads(q.read_text())
    assert d["format"] == "pfc-tune-1" and len(d["entries"]) == 2
    got = {e["count"]: e for e in d["entries"]}
    for k, v in _entry(16, 2).items():
        assert got[16][k] == v, k
    # an entry with the same key and count replaces the table's
    p.write_text(json.dumps({"format": "pfc-tune-1", "entries": [_entry(16, 4)]}))
    pfc.pfc_tune_load(str(p))
    assert pfc.pfc_tune_lookup(2, 16384, 7, 1, 16, arch="gfx950")["rows_per_thread"] == 4
    pfc.pfc_tune_clear()
    assert pfc.pfc_tune_lookup(2, 16384, 7, 1, 16, arch="gfx950") is None
    pfc.pfc_tune_load(str(q))
    assert pfc.pfc_tune_lookup(2, 16384, 7, 1, 16, arch="gfx950")["rows_per_thread"] == 2


def test_malformed_cache_is_refused(pfc, tmp_path):
    for text in ["", "{}", '{"entries": [{"arch": "gfx950", "dim": 2}]}', '{"entries": [{"dim": 2, "n": }]}',
                 '{"entries": [{"arch": "gfx950", "dim": 2, "n": 1, "z": 7, "precision": 1, "count": 1}']:
        p = tmp_path / "bad.json"
        p.write_text(text)
        with pytest.raises(pfc.PFCError):
            pfc.pfc_tune_load(str(p))
    with pytest.raises(pfc.PFCError):
        pfc.pfc_tune_load(str(tmp_path / "missing.json"))
