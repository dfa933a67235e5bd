"""The batched autotuner's cache on disk (lfft_batch_tune_save / _load /
_clear), host side: the file format, the architecture filter, and that a
malformed file changes nothing.  (The GPU test of the batched path checks
that a loaded choice is applied without timing.)"""
import json

import pytest

from paper_1107_5415_amd import lfft


def entry(arch="gfx950", d=2, flags=0, mats=(4, 1, 0, 8), tile_lg=13, order=3, ms=0.5):
    return {"arch": arch, "d": d, "flags": flags, "matrices": list(mats), "tile_lg": tile_lg,
            "order": order, "ms": ms}


def write(path, entries, **top):
    doc = {"format": "lfft-batch-tune", "version": 1, "entries": entries}
    doc.update(top)
    path.write_text(json.dumps(doc))
    return str(path)


@pytest.fixture(autouse=True)
def clean_cache():
    lfft.tune_clear()
    yield
    lfft.tune_clear()


def test_round_trip_and_arch_filter(tmp_path):
    src = write(tmp_path / "a.json", [
        entry(),
        entry(mats=(1, 0, 0, 1024, 32, 0, 0, 32), order=1, ms=1.25),
        entry(arch="gfx942", tile_lg=12),
        entry(d=3, mats=(2, 0, 0, 0, 4, 0, 0, 0, 8), flags=2, tile_lg=11, order=7, ms=-1),
    ])
    assert lfft.tune_load(src, arch="gfx950") == 3
    assert lfft.tune_clear() == 3
    assert lfft.tune_load(src, arch="gfx942") == 1
    assert lfft.tune_load(src, arch="gfx950") == 3
    out = tmp_path / "b.json"
    lfft.tune_save(str(out))
    doc = json.loads(out.read_text())
    assert doc["format"] == "lfft-batch-tune" and doc["version"] == 1
    got = sorted((e["arch"], e["d"], e["flags"], tuple(e["matrices"]), e["tile_lg"], e["order"])
                 for e in doc["entries"])
    want = sorted([("gfx950", 2, 0, (4, 1, 0, 8), 13, 3),
                   ("gfx950", 2, 0, (1, 0, 0, 1024, 32, 0, 0, 32), 13, 1),
                   ("gfx942", 2, 0, (4, 1, 0, 8), 12, 3),
                   ("gfx950", 3, 2, (2, 0, 0, 0, 4, 0, 0, 0, 8), 11, 7)])
    assert got == want
    ms = {tuple(e["matrices"]): e["ms"] for e in doc["entries"] if e["arch"] == "gfx950"}
    assert ms[(1, 0, 0, 1024, 32, 0, 0, 32)] == pytest.approx(1.25)
    # the saved file loads back into the same set
    assert lfft.tune_clear() == 4
    assert lfft.tune_load(str(out), arch="gfx950") == 3
    assert lfft.tune_load(str(out), arch="gfx942") == 1
    # same key: replaced, not duplicated
    assert lfft.tune_load(str(out), arch="gfx950") == 3
    assert lfft.tune_clear() == 4


def test_empty_cache_saves_an_empty_list(tmp_path):
    out = tmp_path / "e.json"
    lfft.tune_save(str(out))
    doc = json.loads(out.read_text())
    assert doc["entries"] == []
    assert lfft.tune_load(str(out), arch="gfx950") == 0


BAD = [
    "",
    "[]",
    "{\"format\": \"something else\", \"version\": 1, \"entries\": []}",
    "{\"format\": \"lfft-batch-tune\", \"version\": 2, \"entries\": []}",
    "{\"format\": \"lfft-batch-tune\", \"version\": 1}",
    "{\"format\": \"lfft-batch-tune\", \"version\": 1, \"entries\": [}",
    "{\"format\": \"lfft-batch-tune\", \"version\": 1, \"entries\": []} trailing",
]


@pytest.mark.parametrize("text", BAD)
def test_malformed_files_are_refused(tmp_path, text):
    good = write(tmp_path / "g.json", [entry()])
    assert lfft.tune_load(good, arch="gfx950") == 1
    bad = tmp_path / "bad.json"
    bad.write_text(text)
    with pytest.raises(lfft.LfftError) as e:
        lfft.tune_load(str(bad), arch="gfx950")
    assert e.value.code == -9
    assert lfft.tune_clear() == 1


@pytest.mark.parametrize("field,value", [
    ("d", 5), ("d", 0), ("tile_lg", 14), ("tile_lg", 10), ("order", 8), ("order", -1),
    ("matrices", [1, 2, 3]), ("matrices", []), ("matrices", [1.5, 0, 0, 1]), ("arch", 7),
    ("ms", "fast"), ("flags", -1),
])
def test_bad_entries_change_nothing(tmp_path, field, value):
    e = entry()
    e[field] = value
    path = write(tmp_path / "x.json", [entry(mats=(8, 0, 0, 8)), e])
    with pytest.raises(lfft.LfftError) as err:
        lfft.tune_load(path, arch="gfx950")
    assert err.value.code == -9
    assert lfft.tune_clear() == 0


def test_missing_file_and_bad_path(tmp_path):
    with pytest.raises(lfft.LfftError) as e:
        lfft.tune_load(str(tmp_path / "does_not_exist.json"), arch="gfx950")
    assert e.value.code == -9
    assert lfft.lib().lfft_batch_tune_save(b"") == -1
    assert lfft.lib().lfft_batch_tune_load(None, b"gfx950", None) == -1
    with pytest.raises(lfft.LfftError) as e:
        lfft.tune_save(str(tmp_path / "no_such_dir" / "x.json"))
    assert e.value.code == -9
