"""The autotuner's search logic on synthetic cost functions (no GPU)."""
import itertools

from paper_2108_09337_amd import tune


def test_exhaustive_when_small():
    spaces = {"x": {"a": [1, 2, 3], "b": [10, 20]}}
    seen = []

    def cost(p):
        seen.append(p)
        return (p["a"] - 2) ** 2 + (p["b"] - 20) ** 2

    res = tune._search("x", cost, spaces)
    assert len(seen) == 6 and len(res) == 6
    assert min(res, key=lambda r: r[0])[1] == {"a": 2, "b": 20}


def test_coordinate_descent_on_separable_cost():
    spaces = {"x": {n: list(range(5)) for n in "abc"}}  # 125 points: coordinate descent
    target = {"a": 3, "b": 0, "c": 4}
    calls = []

    def cost(p):
        calls.append(tuple(sorted(p.items())))
        return sum((p[k] - target[k]) ** 2 for k in target)

    res = tune._search("x", cost, spaces)
    assert min(res, key=lambda r: r[0])[1] == target
    assert len(calls) == len(set(calls)) <= 2 * 15  # every point timed once, two sweeps at most
    assert len(calls) < 125


def test_failing_points_are_not_chosen():
    spaces = {"x": {"a": [0, 1], "b": [0, 1]}}
    res = tune._search("x", lambda p: float("inf") if p["a"] == 1 else 1.0 + p["b"], spaces)
    assert min(res, key=lambda r: r[0])[1] == {"a": 0, "b": 0}


def test_cache_keys_and_apply_nearest_bucket():
    class H:
        def __init__(self):
            self.p = {}

        def set_param(self, k, v):
            self.p[k] = v

    cache = {tune.key("getrf", "f64", 8192): {"params": {"lu_nb": 256}},
             tune.key("getrf", "f64", 65536): {"params": {"lu_nb": 512}}}
    assert tune.key("getrf", "f64", 9000) == "getrf/f64/8192"
    h = H()
    assert tune.apply(h, "getrf", 50000, cache=cache) == {"lu_nb": 512} and h.p == {"lu_nb": 512}
    assert tune.apply(H(), "potrf", 50000, cache=cache) == {}
    assert list(itertools.islice(tune.SPACES, 4)) == ["getrf", "potrf", "mixed_getrf", "vbatch"]
