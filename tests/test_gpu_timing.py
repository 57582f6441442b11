"""Per-kernel timing switched per stretch of steps (mc_set_timing): launches
are counted only while the events are on, the times gathered so far are
kept across a switch, and the results of the steps do not depend on it."""
import sys

import numpy as np
import pytest

from paper_2609_31258_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _sim(timing):
    from paper_2609_31258_amd import mucite
    f, ions, srcs, op, _ = synth.config_c2(n_packs=4000, packs_per_step=400)
    op.sc_every = 4
    g = mucite.Sim(seed=5, pack_capacity=4000, precision=1, timing=timing)
    g.setup(f, ions, srcs, op)
    return g


def test_timing_switch_counts_only_timed_launches():
    _say("timing switch, C2 at 4000 packs")
    g = _sim(False)
    g.step(3)
    t = g.read_timing()
    assert t["launches"]["step"] == 0 and t["ms"]["step"] == 0.0
    g.set_timing(True)
    g.reset_timing()
    g.step(8)
    t = g.read_timing()
    assert t["launches"]["step"] == 8 and t["ms"]["step"] > 0.0
    assert t["launches"]["poisson"] == 2  # updates at steps 4 and 8 of the run (3..10)
    g.set_timing(False)
    g.step(5)
    t2 = g.read_timing()
    assert t2["launches"] == t["launches"] and t2["ms"] == t["ms"]
    a = g.read_packs()
    g.close()
    # the same 16 steps with the events on throughout
    h = _sim(True)
    h.step(16)
    b = h.read_packs()
    h.close()
    for k in ("id", "x", "vx", "e_int", "status"):
        assert np.array_equal(a[k], b[k]), k
