"""The batched form's autotuner: cache key, JSON cache and choice logic (CPU).

The timing itself runs in the library on the GPU (qbsm_batch_autotune,
exercised by the GPU tests); here a stand-in library returns fixed timings
so that the search over leaf options and the cache round trip can be checked
without a device.
"""
import json

import pytest

from paper_2011_11762_amd import autotune as T


class FakeLib:
    """qbsm stand-in: batch_autotune answers from a table keyed by the leaf
    sizes of the pairs it is given; counts its calls."""

    class QbsmError(RuntimeError):
        pass

    def __init__(self, table):
        self.table = table
        self.calls = []

    def batch_autotune(self, pairs, mode, reps=1):
        sizes = tuple(sorted({a for a, _ in pairs}))
        self.calls.append((mode, sizes, len(pairs)))
        r = self.table.get(sizes)
        if r is None:
            raise self.QbsmError("no unit side")
        unit, occ, ms = r
        return {"unit": unit, "wg_per_cu": occ, "ms": ms, "table": {unit: {occ: ms}}}


def members(n=16):
    # even members: fixed leaf size 32; odd members: flexible, given at 64
    out = []
    for m in range(n):
        flexible = m % 2 == 1
        given = 64 if flexible else 32
        out.append({"bs": given, "flexible": flexible,
                    "build": (lambda bs, g=given, f=flexible: (bs, bs) if (f or bs == g) else (_ for _ in ()).throw(
                        AssertionError("fixed member re-stored")))})
    return out


INFOS = [{"nprod": 4 ** (m % 5), "nblk_out": 1} for m in range(16)]


def test_key_depends_on_mode_leaf_sizes_and_segments():
    k = T.batch_key("f32", [32, 64, 64], INFOS[:3])
    assert k == T.batch_key("f32", [64, 32, 64], INFOS[:3])          # order does not matter
    assert k != T.batch_key("bf16x3", [32, 64, 64], INFOS[:3])
    assert k != T.batch_key("f32", [64, 64, 64], INFOS[:3])
    assert k != T.batch_key("f32", [32, 64, 64], INFOS[1:4])
    h = T.segment_histogram([{"nprod": 5, "nblk_out": 1}, {"nprod": 8, "nblk_out": 2}, {"nprod": 0, "nblk_out": 0}])
    assert h == {0: 1, 2: 2}  # 5 -> 2^2, 4 -> 2^2, empty -> bin 0


def test_tuning_picks_the_fastest_leaf_option_and_caches_it(tmp_path):
    path = str(tmp_path / "cache.json")
    # given (32 and 64): unit 128, 2 WG/CU, 10 ms; flexible at 32: 12 ms; at 64: same sizes as given
    lib = FakeLib({(32, 64): (128, 2, 10.0), (32,): (64, 1, 12.0)})
    choice, key, cached = T.tune_batch(lib, "f32", members(), sample_every=3, infos=INFOS, cache_path=path)
    assert not cached and choice["leaf"] == "given" and (choice["unit"], choice["wg_per_cu"]) == (128, 2)
    assert {c[1] for c in lib.calls} == {(32, 64), (32,)}
    assert all(c[2] == 6 for c in lib.calls)  # members 0, 3, .., 15 of 16: fixed and flexible ones
    stored = json.load(open(path))
    assert stored[key]["unit"] == 128 and set(stored[key]["trials_ms"]) == {"given", "32", "64"}
    # the second call is served from the cache without timing anything
    lib2 = FakeLib({})
    choice2, key2, cached2 = T.tune_batch(lib2, "f32", members(), sample_every=3, infos=INFOS, cache_path=path)
    assert cached2 and key2 == key and choice2["unit"] == 128 and not lib2.calls
    # force re-tunes; a faster leaf option wins
    lib3 = FakeLib({(32, 64): (128, 2, 10.0), (32,): (128, 1, 7.5)})
    choice3, _, cached3 = T.tune_batch(lib3, "f32", members(), sample_every=3, infos=INFOS, cache_path=path,
                                       force=True)
    assert not cached3 and choice3["leaf"] == 32 and choice3["ms"] == 7.5
    assert T.load_cache(path)[key]["leaf"] == 32


def test_invalid_or_foreign_entries_are_not_used(tmp_path):
    path = str(tmp_path / "cache.json")
    key = T.batch_key("f32", [m["bs"] for m in members()], INFOS)
    T.save_cache({key: {"unit": 96, "wg_per_cu": 1, "leaf": "given"}}, path)  # not a unit side
    lib = FakeLib({(32, 64): (64, 3, 4.0), (32,): (64, 1, 9.0)})
    choice, _, cached = T.tune_batch(lib, "f32", members(), sample_every=3, infos=INFOS, cache_path=path)
    assert not cached and choice["unit"] == 64 and lib.calls
    with open(path, "w") as fh:
        fh.write("[1, 2]")
    with pytest.raises(ValueError):
        T.load_cache(path)


def test_no_valid_setting_is_an_error(tmp_path):
    with pytest.raises(RuntimeError):
        T.tune_batch(FakeLib({}), "f32", members(), infos=INFOS, cache_path=str(tmp_path / "c.json"))
