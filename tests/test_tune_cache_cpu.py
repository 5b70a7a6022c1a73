"""The autotune cache of the multi-UE launch on the host: batch classes and the cache file."""
import json

from paper_2510_07843_amd import tune
from synth import SlotShape


def _ues(prbs, nr=16, nl=4, qm=6):
    return [SlotShape(p, 14, nr, nl, qm, 2, 2, (2,), 1) for p in prbs]


def test_batch_class_groups_alike_batches():
    a = tune.batch_class(_ues([100, 200, 50]), "MI355X", 256)
    # same kinds, UE order and a total within the same two-significant-bit bucket
    b = tune.batch_class(_ues([50, 205, 100]), "MI355X", 256)
    assert a == b
    assert tune.batch_class(_ues([100, 200, 50]), "MI355X", 128) != a   # another GPU
    assert tune.batch_class(_ues([100, 200, 50], qm=8), "MI355X", 256) != a  # other kinds
    assert tune.batch_class(_ues([400, 800, 200]), "MI355X", 256) != a   # 4x the REs
    k = json.loads(a)
    assert k["kinds"] == [[16, 4, 1, 4, 6, 3]] and k["cus"] == 256


def test_cache_file_round_trip(tmp_path):
    f = str(tmp_path / "sub" / "tune.json")
    assert tune.load_cache(f) == {}
    e1 = dict(tile_re=512, blocks_per_cu=2, ms=1.5, table=[])
    tune.store_cache(f, "k1", e1)
    tune.store_cache(f, "k2", dict(e1, tile_re=256))
    c = tune.load_cache(f)
    assert c["k1"] == e1 and c["k2"]["tile_re"] == 256
    # another version of the file is ignored, not misread
    json.dump(dict(version=tune.CACHE_VERSION + 1, entries=c), open(f, "w"))
    assert tune.load_cache(f) == {}
