"""Host-side parts of the autotuner: the cache key and the cache file."""
import synth
from paper_2505_10144_amd import tune as T


def _cfg():
    scene, cams, fovs, params = synth.config_batch(0, n=100, sizes=[(64, 64), (32, 48)])
    return cams, fovs


def test_signature_is_stable_and_sensitive():
    cams, fovs = _cfg()
    sp, ref = dict(T.DEFAULT_SPACE), {"tile": 16, "window": 16}
    a = T.signature(1_000_000, cams, fovs, 3, sp, ref, 1e-3)
    assert a == T.signature(1_000_000, cams, fovs, 3, sp, ref, 1e-3)
    assert a == T.signature(1_004_000, cams, fovs, 3, sp, ref, 1e-3)   # same 2 significant digits
    assert a != T.signature(2_000_000, cams, fovs, 3, sp, ref, 1e-3)
    assert a != T.signature(1_000_000, cams[:-1], fovs[:-1], 3, sp, ref, 1e-3)
    assert a != T.signature(1_000_000, cams, fovs, 3, dict(sp, window=(16,)), ref, 1e-3)
    assert a != T.signature(1_000_000, cams, fovs, 3, sp, ref, 1e-2)


def test_cache_roundtrip(tmp_path):
    p = str(tmp_path / "c" / "tune.json")
    assert T._load_cache(p) == {}
    T._store_cache(p, {"k": {"choice": {"tile": 32}}})
    assert T._load_cache(p) == {"k": {"choice": {"tile": 32}}}
    open(p, "w").write("{not json")
    assert T._load_cache(p) == {}
