"""The launch-configuration tuning cache of the C-ABI library (host memory
only: no GPU is touched): entries go in and come out by key, invalid ones are
refused, and the JSON file form round-trips."""
import json
import os

import pytest

from paper_2604_07248_amd import binding as B


@pytest.fixture
def cache():
    if not os.path.exists(B.LIB_PATH):
        pytest.fail("libturpy.so is not built (run __graft_entry__.build())")
    from paper_2604_07248_amd import api
    api.tune_cache_clear()
    yield api
    api.tune_cache_clear()


def entry(kernel="col_fresnel", n=1024, batch_class=7, width=8, arch="gfx950", us=240.0, radix=0, waves=0,
          us_default=300.0, configs=9):
    return {"arch": arch, "kernel": kernel, "n": n, "batch_class": batch_class, "width": width, "radix": radix,
            "waves": waves, "configs": configs, "us": us, "us_default": us_default}


def test_put_get_in_key_order_and_replace(cache):
    assert cache.tune_cache() == []
    es = [entry("synth", 1024, 6, 4, us=87.0), entry(), entry("col_angular", 256, 3, 16),
          entry("row_fwd", 1024, 6, 0, waves=4, radix=0)]
    B.tune_cache_put(es)
    got = cache.tune_cache()
    assert len(got) == 4
    # key order: arch, kernel, n, batch class
    assert [(g["kernel"], g["n"]) for g in got] == [("col_fresnel", 1024), ("col_angular", 256), ("synth", 1024),
                                                   ("row_fwd", 1024)]
    for g in got:
        ref = next(e for e in es if e["kernel"] == g["kernel"])
        for f in ("width", "batch_class", "radix", "waves", "configs"):
            assert g[f] == ref[f]
        assert g["arch"] == "gfx950"
        assert g["us"] == pytest.approx(ref["us"]) and g["us_default"] == pytest.approx(ref["us_default"])
    # same key: replaced, not added
    B.tune_cache_put([entry(width=4, radix=8, us=1.0)])
    got = cache.tune_cache()
    assert len(got) == 4 and (got[0]["width"], got[0]["radix"]) == (4, 8)
    # another architecture or batch class is another key
    B.tune_cache_put([entry(arch="gfx942"), entry(batch_class=5)])
    assert len(cache.tune_cache()) == 6


@pytest.mark.parametrize("bad,needle", [
    (dict(n=2048, width=16), "not built"),   # 16 columns of 2048 rows exceed one block
    (dict(width=5), "not built"),
    (dict(n=100), "not built"),
    (dict(n=4096, width=4), "not built"),
    (dict(kernel=9), "unknown kernel"),
    (dict(batch_class=0), "batch class"),
    (dict(radix=2), "not built"),             # second-pass radices 8 and 4 only
    (dict(n=256, radix=8), "not built"),      # alternative plans from N = 512
    (dict(waves=3), "not built"),             # column kernels take no occupancy hint
    (dict(kernel="row_fwd", width=0, waves=5), "not built"),
    (dict(kernel="row_bwd", n=128, width=0, waves=2), "not built"),
    (dict(kernel="row_fwd", width=8, waves=3), "not built"),
])
def test_invalid_entries_refused(cache, bad, needle):
    B.tune_cache_put([entry(batch_class=3)])
    with pytest.raises(B.TurpyError) as e:
        B.tune_cache_put([entry(**bad)])
    assert e.value.status == B.E_INVALID and needle in str(e.value)
    assert len(cache.tune_cache()) == 1
    with pytest.raises(ValueError):
        B.tune_cache_put([entry(arch="x" * 40)])


def test_widths_built_per_grid_size(cache):
    """Every width is accepted where it fits and refused where it does not:
    K N / 16 threads <= 1024 and (K N + 2 N) complex words <= 160 KiB."""
    for n in (16, 32, 64, 128, 256, 512, 1024, 2048):
        for k in (4, 8, 16):
            fits = k <= n and k * n // 16 <= 1024 and (k * n + 2 * n) * 8 <= 160 * 1024
            if fits:
                B.tune_cache_put([entry(n=n, width=k)])
            else:
                with pytest.raises(B.TurpyError):
                    B.tune_cache_put([entry(n=n, width=k)])
    assert len(cache.tune_cache()) == 8  # one key per n


def test_json_round_trip(cache, tmp_path):
    es = [entry(), entry("synth", 2048, 2, 4, us=98.0, radix=8), entry("col_as_table", 64, 2, 16),
          entry("row_bwd", 512, 3, 0, waves=2)]
    B.tune_cache_put(es)
    path = tmp_path / "tune.json"
    cache.tune_cache_save(str(path))
    doc = json.loads(path.read_text())
    assert doc["format"] == "turpy-tune-cache" and doc["version"] == 2 and len(doc["entries"]) == 4
    before = cache.tune_cache()
    cache.tune_cache_clear()
    assert cache.tune_cache() == []
    assert cache.tune_cache_load(str(path)) == 4
    assert cache.tune_cache() == before
    bad = tmp_path / "bad.json"
    for doc in ({"format": "other", "version": 2, "entries": []},
                {"format": "turpy-tune-cache", "version": 1, "entries": []}):  # the strip-width-only form
        bad.write_text(json.dumps(doc))
        with pytest.raises(ValueError):
            cache.tune_cache_load(str(bad))


def test_cache_file_from_environment(cache, tmp_path, monkeypatch):
    """$TURPY_TUNE_CACHE names a cache file that plans read before they are
    created (once per process and path) and that tuning writes back."""
    path = tmp_path / "env_tune.json"
    B.tune_cache_put([entry(n=512, width=16, batch_class=4)])
    cache.tune_cache_save(str(path))
    cache.tune_cache_clear()
    monkeypatch.setenv(cache.TUNE_CACHE_ENV, str(path))
    monkeypatch.setattr(cache, "_env_cache_read", [])
    assert cache.tune_cache_from_env() == 1
    assert [(e["n"], e["width"]) for e in cache.tune_cache()] == [(512, 16)]
    assert cache.tune_cache_from_env() == 0  # read once
    monkeypatch.setenv(cache.TUNE_CACHE_ENV, str(tmp_path / "missing.json"))
    assert cache.tune_cache_from_env() == 0
