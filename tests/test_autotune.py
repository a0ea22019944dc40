"""CPU checks of the autotuner's bookkeeping: size buckets, the candidate
filter, and the lookup of the committed cache (defaults where it has no
entry)."""
import json

from paper_2405_10923_amd import autotune, schedules


def test_buckets():
    assert autotune.bucket(1 << 22, 256) == "n2^22|m256"
    assert autotune.bucket((1 << 22) - 5, 200) == "n2^22|m256"
    assert autotune.bucket((1 << 21) + 1, 257) == "n2^22|m512"
    assert autotune.key("float16", 1 << 20, 128) == "float16|n2^20|m128"


def test_candidate_filter():
    assert autotune.valid((8, 32, 0), 256, 8)
    assert not autotune.valid((8, 12, 0), 256, 8)       # outer not a multiple of the panel
    assert not autotune.valid((16, 64, 0), 256, 8)      # outer wider than 32
    assert not autotune.valid((16, 0, 1), 256, 2)       # 2-byte storage needs 2 tiles
    assert not autotune.valid((32, 0, 0), 16, 8)        # panel wider than m


def test_lookup_cache_and_default(tmp_path, monkeypatch):
    path = tmp_path / "c.json"
    path.write_text(json.dumps({"float64|n2^22|m256": {"panel": 4, "outer": 16, "tpw": 2,
                                                        "ms": 1.0}}))
    monkeypatch.setattr(autotune, "CACHE", str(path))
    assert schedules.lookup("float64", 1 << 22, 256) == (4, 16, 2, "autotuned")
    assert schedules.lookup("float64", 1 << 22, 250) == (4, 16, 2, "autotuned")
    assert schedules.lookup("float32", 1 << 22, 256) == (8, 32, 0, "default")
    assert schedules.lookup("float16", 1 << 10, 8) == (16, 0, 0, "default")


def test_committed_cache_is_well_formed():
    for k, v in autotune.load().items():
        name, nb, mb = k.split("|")
        assert name in schedules.DEFAULT
        assert autotune.valid((v["panel"], v["outer"], v.get("tpw", 0)), 1 << 30,
                              2 if name in ("float16", "bfloat16") else 8)
        assert v["ms"] > 0
