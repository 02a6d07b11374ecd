"""Host logic of the autotuner's cache: keys, report parsing, storage."""
import json
import types

import workloads as W
from paper_2409_07563_amd import autotune as A


def test_k_bucket():
    assert [A.k_bucket(k) for k in (1, 2, 3, 1000, 1024, 1025, 8192)] == \
        [1, 2, 4, 1024, 1024, 2048, 8192]


def test_key_separates_what_decides_the_choice():
    def ctl(probs, grad=False):
        return types.SimpleNamespace(problems=probs, n_inst=len(probs), device="cuda:0",
                                     requires_grad=grad)
    a = A.key(ctl([W.c2("circles", K=8192)]), "gfx950")
    b = A.key(ctl([W.c2("circles", K=8000)]), "gfx950")   # same K bucket
    c = A.key(ctl([W.c2("circles", K=9000)]), "gfx950")
    d = A.key(ctl([W.c2("circles", K=8192, T=50)]), "gfx950")
    e = A.key(ctl([W.c2("circles", K=8192)]), "gfx942")
    f = A.key(ctl(W.c4(n_instances=3)), "gfx950")
    g = A.key(ctl([W.c2("circles", K=8192)], grad=True), "gfx950")
    assert a == b and len({a, c, d, e, f, g}) == 6
    assert "H64" in A.key(ctl([W.c5()]), "gfx950")


def test_report_parsing():
    rep = ("sample lanes=4 block=64 tile=256 calls=1 7.50\n"
           "rollout lanes=1 block=128 tile=256 calls=2 40.25\n"
           "chosen lanes=4 block=64 tile=256 calls=1 0.00\n")
    r = A.parse_report(rep)
    assert [x["phase"] for x in r] == ["sample", "rollout", "chosen"]
    assert r[1] == {"phase": "rollout", "lanes": 1, "block": 128, "tile": 256, "calls": 2,
                    "us": 40.25}


def test_store_and_load_roundtrip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert A.load(path) == {}
    t1 = {"lanes_per_sample": 4, "rollout_block": 64, "batch_tile": 256, "noise_calls": 2}
    A.store(path, "k1", {"tuning": t1, "timings": [{"phase": "sample", "us": 1.0}]})
    A.store(path, "k2", {"tuning": dict(t1, noise_calls=1)})
    data = A.load(path)
    assert data["k1"]["tuning"] == t1 and data["k2"]["tuning"]["noise_calls"] == 1
    json.dumps(data)
