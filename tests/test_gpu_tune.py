"""The autotuner of the factorisation's schedule: a choice timed once is
kept (per architecture, runtime, precision and order rounded to a power of
two), reused from memory and, after the in-memory table is dropped, from the
JSON file named by SPD_TUNE_CACHE; factorisations under the tuned schedule
still match the oracle (the schedule orders the work, it changes no
result's bar)."""
import json
import os
import sys

import numpy as np
import pytest

import spdgen

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_tuned_schedule_cached_and_reused(spd, orc, tmp_path):
    import torch
    path = str(tmp_path / "spd_tune.json")
    old = os.environ.get("SPD_TUNE_CACHE")
    os.environ["SPD_TUNE_CACHE"] = path
    spd.autotune_clear()
    try:
        r1 = spd.autotune(2000, "fp32")
        _say("tuned", r1)
        assert r1["from_cache"] == 0 and r1["n"] == 2048 and r1["group"] in (2, 4, 6, 8)
        with open(path) as f:
            tab = json.load(f)
        key = next(k for k in tab if k.endswith("|fp32|2048"))
        assert tab[key]["a"] == r1["group"] and tab[key]["b"] == r1["upd_slots"]
        assert tab[key]["c"] == r1["small_tiles"] and r1["small_tiles"] in (0, 1)
        # the same bucket again: held in memory
        r2 = spd.autotune(2100, "fp32")
        assert r2["from_cache"] == 1 and (r2["group"], r2["upd_slots"]) == (r1["group"], r1["upd_slots"])
        # a fresh table reads the file
        spd.autotune_clear()
        r3 = spd.autotune(2048, "fp32")
        assert r3["from_cache"] == 2 and (r3["group"], r3["upd_slots"]) == (r1["group"], r1["upd_slots"])
        # a half format has its own entry
        r4 = spd.autotune(3000, "fp16")
        _say("tuned fp16", r4)
        assert r4["from_cache"] == 0 and r4["n"] == 4096 and r4["group"] in (2, 4, 8)
        # a solve under the tuned schedule meets the bars
        cond = 1e4
        s = spdgen.system(2000, cond, 2, config=0, index=41)
        X, rep, F = spd.posv(torch.from_numpy(s.A).cuda(), torch.from_numpy(np.ascontiguousarray(s.Bt)).cuda(),
                             prec="fp32")
        F.close()
        Xh = X.cpu().numpy()
        assert rep.status == 0 and spd.PREC_NAME[rep.prec_used] == "fp32"
        assert np.all(orc.backward_error(s.A, Xh, s.Bt) <= 1e-14)
        assert np.abs(Xh - s.Xt).max() / np.abs(s.Xt).max() <= 10 * cond * U64
    finally:
        if old is None:
            os.environ.pop("SPD_TUNE_CACHE", None)
        else:
            os.environ["SPD_TUNE_CACHE"] = old
        spd.autotune_clear()
