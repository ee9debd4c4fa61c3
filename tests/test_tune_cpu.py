"""Host side of the tuner: cache keys, column buckets and the JSON store."""
import json

from paper_2506_04710_amd import tune


def test_buckets():
    assert [tune._bucket(n) for n in (1, 2, 7, 8, 15, 16, 31, 32, 81, 200)] == [1, 2, 2, 8, 8, 16, 16, 32, 64, 128]


def test_store_and_load_roundtrip(tmp_path):
    p = str(tmp_path / "sub" / "t.json")
    assert tune._load(p) == {}
    tune._store(p, {"dev": {"k": {"spectrum_pass": 2}}})
    assert tune._load(p) == {"dev": {"k": {"spectrum_pass": 2}}}
    with open(p, "w") as fh:
        fh.write("{broken")
    assert tune._load(p) == {}
    json.dumps(tune._load(p))


def test_plan_key_separates_shapes():
    class FakePlan:
        def __init__(self, **d):
            self.d = d
            self.pbuf = None

        def info(self):
            return self.d
    base = dict(Nx=32, Ny=32, b=64, Nr=256, nrc=8, Px=63, Py=63, half_spectrum=1, prec=2)
    a = tune.plan_key(FakePlan(**base), "mixed", 1)
    assert a != tune.plan_key(FakePlan(**dict(base, nrc=0)), "mixed", 1)
    assert a != tune.plan_key(FakePlan(**base), "fp64", 1)
    assert a != tune.plan_key(FakePlan(**base), "mixed", 16)
    assert tune.plan_key(FakePlan(**base), "mixed", 20) == tune.plan_key(FakePlan(**base), "mixed", 31)
