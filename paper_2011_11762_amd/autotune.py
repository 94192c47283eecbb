"""Autotuner of the batched form, with a JSON cache of its choices.

The batched numeric phase runs many multiplies of uneven sizes in one
persistent launch.  Three settings decide its speed:

* the work-unit side: how many leaves one workgroup's dense tile covers,
  which fixes the MFMA wave tile, the LDS stage and the occupancy of the
  leaf-product kernel (one side for the whole batch);
* the persistent occupancy: workgroups per compute unit of the launch;
* the leaf size of the members whose leaf size is a storage choice (a matrix
  given by its elements, stored as 32 x 32 or 64 x 64 leaves); a member whose
  block pattern is defined at its leaf size keeps it.

The first two are timed by the library (``qbsm_batch_autotune``) on a sample
of the batch's members; the leaf size is tried here, batch-wide, over the
members that allow it.  A choice is cached under a key made of the mode, the
members' leaf sizes as given and a histogram of their segment lengths (leaf
products per output block, in powers of two), so a batch of the same shape
is not tuned again.  The cache is plain JSON (``load_cache``/``save_cache``).
"""
from __future__ import annotations

import json
import math
import os
from collections import Counter

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tuning", "batch_tuning.json")
LEAF_OPTIONS = ("given", 32, 64)


def segment_histogram(infos) -> dict:
    """Members per power-of-two bin of their mean segment length (leaf
    products per output block), from plan infos."""
    bins = Counter()
    for i in infos:
        seg = i["nprod"] / max(i["nblk_out"], 1)
        bins[int(math.floor(math.log2(seg))) if seg >= 1 else 0] += 1
    return dict(sorted(bins.items()))


def batch_key(mode: str, leaf_sizes, infos) -> str:
    """Cache key: mode, leaf sizes as given (counts) and the segment histogram."""
    bs = dict(sorted(Counter(int(b) for b in leaf_sizes).items()))
    seg = segment_histogram(infos)
    return (f"{mode}|bs:" + ",".join(f"{k}x{v}" for k, v in bs.items())
            + "|seg:" + ",".join(f"2^{k}x{v}" for k, v in seg.items()))


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        data = json.load(fh)
    if not isinstance(data, dict):
        raise ValueError(f"{path}: not a tuning cache")
    return data


def save_cache(cache: dict, path: str = DEFAULT_CACHE) -> None:
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
        fh.write("\n")
    os.replace(tmp, path)


def valid_entry(e) -> bool:
    return (isinstance(e, dict) and e.get("unit") in (64, 128, 256) and isinstance(e.get("wg_per_cu"), int)
            and 1 <= e["wg_per_cu"] <= 4 and e.get("leaf") in LEAF_OPTIONS)


def tune_batch(qbsm, mode, members, sample_every: int = 7, reps: int = 1, cache_path: str = DEFAULT_CACHE,
               infos=None, force: bool = False, log=None):
    """Chooses (leaf option, unit side, occupancy) for a batch.

    members: list of dicts with "bs" (leaf size as given) and "build"
    (callable taking a leaf size and returning the member's (A, B) handles;
    a member whose leaf size is fixed accepts only its own).  "flexible"
    marks members that may be stored at 32 or 64.  infos: plan infos of the
    batch as given (for the key).  Returns (choice dict, key, cached flag).
    """
    key = batch_key(mode, [m["bs"] for m in members], infos or [])
    cache = load_cache(cache_path)
    if not force and valid_entry(cache.get(key)):
        return cache[key], key, True
    sample = members[::max(sample_every, 1)]
    best, trials = None, {}
    for leaf in LEAF_OPTIONS:
        if leaf != "given" and not any(m.get("flexible") for m in sample):
            continue
        pairs = []
        for m in sample:
            bs = m["bs"] if (leaf == "given" or not m.get("flexible")) else leaf
            pairs.append(m["build"](bs))
        try:
            r = qbsm.batch_autotune(pairs, mode, reps=reps)
        except qbsm.QbsmError:  # no unit side serves every member at this leaf choice
            continue
        finally:
            del pairs
        trials[str(leaf)] = {str(u): {str(o): round(t, 4) for o, t in row.items()} for u, row in r["table"].items()}
        if log:
            log(f"autotune leaf={leaf}: unit {r['unit']}, {r['wg_per_cu']} WG/CU, {r['ms']:.3f} ms per sample run")
        if best is None or r["ms"] < best["ms"]:
            best = {"leaf": leaf, "unit": r["unit"], "wg_per_cu": r["wg_per_cu"], "ms": round(r["ms"], 4)}
    if best is None:
        raise RuntimeError("no setting of the batch could be timed")
    best["sample"] = f"every {sample_every}th member ({len(sample)} of {len(members)})"
    best["trials_ms"] = trials
    cache[key] = best
    save_cache(cache, cache_path)
    return best, key, False
