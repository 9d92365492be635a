"""Host logic of the launch-option autotuner: workload signature, coordinate
descent, JSON cache (no device needed)."""
import itertools

from paper_2503_22767_amd import autotune as A
from paper_2503_22767_amd import workloads as W


def test_cache_key_separates_what_matters():
    a = W.make_tiny(seed=0, dim=2, n_grid=16)
    b = W.make_tiny(seed=1, dim=2, n_grid=16)          # same shapes, other values
    c = W.make_tiny(seed=0, dim=2, n_grid=32)          # other grid
    d = W.make_tiny(seed=0, dim=3, n_grid=16)          # other dimension
    assert A.cache_key([a], 4) == A.cache_key([b], 4)
    assert A.cache_key([a], 4) != A.cache_key([a], 8)
    assert A.cache_key([a], 4) != A.cache_key([c], 4)
    assert A.cache_key([a], 4) != A.cache_key([d], 4)
    assert A.cache_key([a], 4) != A.cache_key([a, b], 4)


def test_particles_per_cell():
    inst = W.make_quadruped3d(n_steps=1).instances[0]
    assert A.particles_per_cell(inst.params) == 27
    assert A.particles_per_cell(W.make_cantilever2d().instances[0].params) == 4


def test_coordinate_descent_finds_separable_optimum():
    space = dict(a=[0, 1, 2], b=[10, 20, 30], c=[5, 6])
    best_true = dict(a=2, b=10, c=6)

    def cost(o):   # separable: one pass of coordinate descent is exact
        return abs(o["a"] - 2) + abs(o["b"] - 10) / 10 + (0 if o["c"] == 6 else 0.5) + 1.0

    best, t, table = A.coordinate_descent(cost, space, dict(a=0, b=30, c=5))
    assert best == best_true and t == 1.0
    # every evaluated option set is recorded once
    keys = [tuple(sorted(o.items())) for o, _ in table]
    assert len(keys) == len(set(keys))
    # and never more evaluations than the start plus one per alternative value
    assert len(table) <= 1 + sum(len(v) - 1 for v in space.values())


def test_coordinate_descent_never_returns_worse_than_start():
    space = dict(a=[0, 1, 2, 3], b=[0, 1, 2])
    for start in itertools.product(space["a"], space["b"]):
        s = dict(a=start[0], b=start[1])
        cost = lambda o: (o["a"] * 7 + o["b"] * 3) % 5 + 0.1 * o["a"]
        best, t, _ = A.coordinate_descent(cost, space, s, rounds=3)
        assert t <= cost(s)
        assert t == cost(best)


def test_cache_round_trip(tmp_path):
    p = str(tmp_path / "sub" / "tune.json")
    assert A.load_cache(p) == {}
    A.save_cache(p, {"k": {"options": {"graph": 1}}})
    assert A.load_cache(p)["k"]["options"]["graph"] == 1
    (tmp_path / "bad.json").write_text("{not json")
    assert A.load_cache(str(tmp_path / "bad.json")) == {}


def test_search_space_starts_at_the_library_defaults():
    for k, v in A.DEFAULTS.items():
        assert v in A.SPACE[k]
