"""Host-side tests of the autotuner's cache: keys, exact and nearest
lookup by plan statistics.  No GPU."""
import json

import pytest

from workloads import get_config, patterns as P

autotune = pytest.importorskip("paper_1203_2742_amd.autotune")


def _entry(pat, k, device, relax, wide):
    return {"pattern": autotune.pattern_hash(pat), "k": k, "device": device, "stats": autotune.plan_stats(pat),
            "forward": {"relax": relax, "wide_j": wide, "ms": 1.0},
            "fundamental": {"wide_j": wide, "big_a": 256, "ms": 2.0}}


def test_pattern_hash_and_stats():
    a, b = get_config("grid3d_8"), get_config("grid3d_12")
    assert autotune.pattern_hash(a) == autotune.pattern_hash(get_config("grid3d_8"))
    assert autotune.pattern_hash(a) != autotune.pattern_hash(b)
    st = autotune.plan_stats(b)
    assert st["n"] == 1728 and st["nnz"] == int(b[1][-1]) and st["nsuper"] > 0


def test_lookup_exact_nearest_and_missing(tmp_path):
    small, mid, big = get_config("grid3d_8"), get_config("grid3d_12"), get_config("grid2d_48")
    db = {}
    for pat, relax, wide in ((small, 0.01, 128), (big, 0.1, 256)):
        e = _entry(pat, 4, "devA", relax, wide)
        db[f"{e['pattern']}:k4:devA"] = e
    path = tmp_path / "tuned.json"
    path.write_text(json.dumps(db))
    got = autotune.lookup(small, 4, "devA", cache=str(path))
    assert got["match"] == "exact" and got["forward"]["relax"] == 0.01
    # an unseen pattern takes the entry with the nearest statistics
    near = autotune.lookup(mid, 4, "devA", cache=str(path))
    assert near["match"] == "nearest"
    st = autotune.plan_stats(mid)
    d = {}
    for e in db.values():
        d[e["pattern"]] = sum((__import__("math").log(st[f]) - __import__("math").log(e["stats"][f])) ** 2
                              for f in ("nnz", "nsuper", "max_front"))
    assert near["pattern"] == min(d, key=d.get)
    # another k or device: nothing
    assert autotune.lookup(small, 8, "devA", cache=str(path)) is None
    assert autotune.lookup(small, 4, "devB", cache=str(path)) is None
    assert autotune.lookup(P.band(30, 2), 4, "devA", cache=str(tmp_path / "none.json")) is None
