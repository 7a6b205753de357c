"""The binding's tuned-parameter cache (host logic, no device)."""
import os

from paper_1804_06231_amd.pvl import PARAMS, TuneCache, tune_key


def test_key_groups_sizes_by_power_of_two():
    a = tune_key("gfx950", "density", 1 << 20, 17 ** 3, 1)
    assert a == tune_key("gfx950", "density", int(1.2 * (1 << 20)), 17 ** 3, 1)
    assert a != tune_key("gfx950", "density", 1 << 22, 17 ** 3, 1)        # another N class
    assert a != tune_key("gfx950", "density", 1 << 20, 8 ** 3, 1)         # denser cells
    assert a != tune_key("gfx950", "adjoint", 1 << 20, 17 ** 3, 1)
    assert a != tune_key("gfx942", "density", 1 << 20, 17 ** 3, 1)
    assert a != tune_key("gfx950", "density", 1 << 20, 17 ** 3, 3)        # batched boxes


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "tune.json")
    c = TuneCache(path)
    k = tune_key("gfx950", "density", 1 << 20, 4913, 1)
    assert c.get(k) is None
    params = {name: i for i, name in enumerate(PARAMS)}
    c.put(k, dict(params, unrelated=7))
    assert os.path.exists(path)
    again = TuneCache(path)                     # a later process
    assert again.get(k) == params
    assert again.get(tune_key("gfx950", "plain", 1 << 20, 4913, 1)) is None


def test_cache_ignores_unknown_parameters(tmp_path):
    path = str(tmp_path / "tune.json")
    with open(path, "w") as f:
        f.write('{"k": {"no_such_param": 1}}')
    assert TuneCache(path).get("k") is None
