"""The factorisation's schedule decides only which workgroup computes which
trailing-update tile -- the cap on the group update's workgroups, whole
rounds over them, a short last round split into 64-tiles, 64-tile launches
for a group's thin updates -- and never the order of any element's sums, so
factors computed under different schedules with the same group width G must
agree bit for bit (the group width does change the order: it is held
fixed).  Each handle reads its schedule from the environment when it is
created.  The caps below make launches run as one round, as several whole
rounds with a split last round, as rounds whose last one is too full to
split, and (uncapped, n = 8192) as one workgroup per tile."""
import sys

import pytest

import spdgen

pytestmark = pytest.mark.gpu

# (SPD_UPD_SLOTS, SPD_SMALL_MAIN)
SCHEDULES = [(0, 0), (448, 0), (120, 0), (64, 0), (8, 0), (0, 1)]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("prec,n", [("fp32", 3000), ("fp32", 8192), ("fp64", 3000), ("fp16", 3000)])
def test_factor_bitwise_equal_across_schedules(spd, monkeypatch, prec, n):
    import torch
    _say(f"schedules {prec} n={n}")
    A = spdgen.logspaced(n, 10.0, 9000 + n, backend="torch", device="cuda")
    ref = None
    for slots, small in SCHEDULES:
        monkeypatch.setenv("SPD_GROUP", "4")
        monkeypatch.setenv("SPD_GROUP_HALF", "8")
        monkeypatch.setenv("SPD_UPD_SLOTS", str(slots))
        monkeypatch.setenv("SPD_SMALL_MAIN", str(small))
        F, info, st = spd.factor(A, prec=prec)
        assert st == 0 and info == 0, (slots, small, st, info)
        L = spd.export(F)[0]
        F.close()
        if ref is None:
            ref = L
        else:
            assert torch.equal(L, ref), (prec, n, slots, small)
