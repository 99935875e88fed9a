"""Host logic of the autotuner: size classes, the margin rule, and the cache
being applied only on the GPU architecture it was written on."""
import json

from paper_2101_03240_amd import autotune


def test_size_classes():
    assert autotune.size_class((32, 32, 32)) == "small"
    assert autotune.size_class((1, 96, 96)) == "small"
    assert autotune.size_class((97, 8, 8)) == "medium"
    assert autotune.size_class((256, 256, 256)) == "medium"
    assert autotune.size_class((512, 300, 1)) == "large"
    assert autotune.size_class((513, 4, 4)) == "xlarge"


def test_margin_keeps_the_default_inside_the_spread():
    t = {"-1": 100.0, "32768": 97.0, "131072": 96.0}
    assert autotune.pick(t, "-1", 0.05) == "-1"        # 4 % better: noise
    assert autotune.pick(t, "-1", 0.0) == "131072"     # no margin: the fastest
    t["524288"] = 90.0
    assert autotune.pick(t, "-1", 0.05) == "524288"    # 10 % better: taken
    assert autotune.pick({"a": 1.0, "b": 2.0}, "a", 0.05) == "a"


def test_cache_is_for_one_architecture(tmp_path, monkeypatch):
    doc = {"arch": "gfx950:sramecc+:xnack-", "edt": {}, "batch": {"batch_wide": -1}}
    p = tmp_path / "cache.json"
    p.write_text(json.dumps(doc))
    monkeypatch.setattr(autotune, "CACHE", str(p))
    assert autotune.load("gfx950")["batch"]["batch_wide"] == -1
    assert autotune.load("gfx942:sramecc+:xnack-") is None
    p.write_text("not json")
    assert autotune.load("gfx950") is None


def test_committed_cache_is_well_formed():
    with open(autotune.CACHE) as f:
        doc = json.load(f)
    assert doc["arch"].split(":")[0] == "gfx950"
    for cls in ("small", "medium", "large"):
        e = doc["edt"][cls]
        assert (e["edt_tile_y"], e["edt_tile_x"]) in autotune.EDT_TILES
        # the choice is the default unless it beat the default by the margin
        best = "%dx%d" % (e["edt_tile_y"], e["edt_tile_x"])
        assert best == autotune.pick(e["ms"], "%dx%d" % autotune.EDT_TILES[0], doc.get("margin_edt", 0.0))
    assert doc["batch"]["batch_wide"] in autotune.BATCH_WIDE
    assert doc["serve"]["serve_wide"] in autotune.SERVE_WIDE
