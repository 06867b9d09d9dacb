"""The autotuner's cache (CPU): shape buckets, exact and nearest lookup, and
that a cache entry selects its kernel variants on a problem (a stand-in
object with the binding's set_tuning interface, so no GPU is needed; the
GPU tests check what each variant computes)."""
import json

import pytest

from paper_2008_01996_amd import autotune


def test_shape_key_buckets():
    assert autotune.shape_key("fp32", 48641, 256, 1024) == "fp32/bp256/mx65536/nt1024"
    assert autotune.shape_key("fp64", 16129, 128, 256) == "fp64/bp128/mx16384/nt256"
    assert autotune.shape_key("fp32", 225, 16, 16) == "fp32/bp16/mx256/nt16"
    assert autotune.padded_band(5) == 16 and autotune.padded_band(250) == 256


class _Stub:
    def __init__(self, precision, Mx, half_band, Nt):
        self.precision, self.Mx, self.Nt = precision, Mx, Nt
        self.setup_report = {"half_band": half_band}
        self.applied = None

    def set_tuning(self, **kw):
        self.applied = kw


ENTRIES = {
    "fp32/bp256/mx65536/nt1024": {"tuning": {"sweep_tile_min_rhs": 4, "gemm_tile_m_fp32": 128,
                                             "gemm_tile_m_fp64": 64, "gemm_n_fast": 1}},
    "fp32/bp128/mx16384/nt256": {"tuning": {"sweep_tile_min_rhs": 8, "gemm_tile_m_fp32": 64,
                                            "gemm_tile_m_fp64": 64, "gemm_n_fast": 0}},
}


def test_entry_selects_its_variant(tmp_path, monkeypatch):
    path = tmp_path / "cache.json"
    path.write_text(json.dumps({"entries": ENTRIES}))
    monkeypatch.setenv(autotune.CACHE_ENV, str(path))
    p = _Stub("fp32", 48641, 256, 1024)
    got = autotune.apply(p)
    # an entry without the FP64 tile width keeps the 64-column tile it was tuned with
    want = dict(ENTRIES["fp32/bp256/mx65536/nt1024"]["tuning"], gemm_tile_n_fp64=64)
    assert p.applied == want == got


def test_nearest_bucket_and_no_match():
    # same precision and band, other sizes: the nearest bucket
    t = autotune.lookup(ENTRIES, "fp32", 40000, 250, 700)
    assert t == ENTRIES["fp32/bp256/mx65536/nt1024"]["tuning"]
    # no entry for this precision or band: nothing is applied
    assert autotune.lookup(ENTRIES, "fp64", 48641, 256, 1024) is None
    p = _Stub("fp64", 48641, 256, 1024)
    assert autotune.apply(p, ENTRIES) is None and p.applied is None


def test_store_round_trip(tmp_path):
    path = str(tmp_path / "c.json")
    autotune.store("fp64/bp16/mx256/nt16", {"tuning": {"sweep_tile_min_rhs": 0}}, path)
    autotune.store("fp32/bp16/mx256/nt16", {"tuning": {"sweep_tile_min_rhs": 2}}, path)
    e = autotune.load_cache(path)
    assert e["fp64/bp16/mx256/nt16"]["tuning"]["sweep_tile_min_rhs"] == 0
    assert e["fp32/bp16/mx256/nt16"]["tuning"]["sweep_tile_min_rhs"] == 2


def test_committed_cache_is_well_formed():
    for key, e in autotune.load_cache(autotune.DEFAULT_CACHE).items():
        prec, bp, mx, nt = key.split("/")
        assert prec in ("fp32", "fp64") and bp.startswith("bp") and mx.startswith("mx") and nt.startswith("nt")
        assert set(e["tuning"]) <= set(autotune.FIELDS)
        assert e["tuning"]["gemm_tile_m_fp32"] in (64, 128)
        assert (e["tuning"]["gemm_tile_m_fp64"], e["tuning"].get("gemm_tile_n_fp64", 64)) in autotune.FP64_TILES
