"""Slot sorting (sort_every): runs whose slots are reordered by (species, CIC
cell) every few steps, with terminal slots dropped, against the same runs
without it, through the C ABI.

Slot order enters no pack's arithmetic (the random streams are keyed by pack
id and step) and no integer tally, so the sorted run must reproduce bit for
bit: every active pack's state (compared by id), the int64 tallies and
histograms, the exit records, the charge grid of the last deposit (which a
sorting context adds straight into a zeroed grid, with wavefront sums where
a wavefront's packs share a cell) and the space-charge potential and field.
Only the FP64 sums over the active population, reduced in slot order, may
differ in their last bits.  Also: the deposit of a sorting context against
the oracle, bit for bit, on packs grouped by cell; compaction of terminal
slots; several species; the adaptive step; checkpoint and resume.
"""
import sys

import numpy as np
import pytest

from paper_2609_31258_amd import synth
from tests.parity_util import by_id

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _active(p):
    keep = p["status"] == 0
    return by_id({k: v[keep] for k, v in p.items()})


def _compare(a, b, *, sums_rtol=1e-12):
    """Bit-for-bit equality of two runs that differ only in slot order."""
    pa, pb = _active(a.read_packs()), _active(b.read_packs())
    assert len(pa["id"]) == len(pb["id"]) > 0
    for k in pa:
        assert np.array_equal(pa[k], pb[k]), k
    ta, tb = a.read_tallies(), b.read_tallies()
    for k, v in ta.items():
        if k.startswith("sum_w_"):
            assert v == pytest.approx(tb[k], rel=sums_rtol, abs=1e-300), k
        else:
            assert np.array_equal(np.asarray(v), np.asarray(tb[k])), k
    ea, eb = a.read_exits(), b.read_exits()
    assert np.array_equal(ea, eb)
    assert np.array_equal(a.read_charge(), b.read_charge())
    for x, y in zip(a.read_sc(), b.read_sc()):
        assert np.array_equal(x, y)
    return ta, len(ea)


def _run_pair(f, ions, srcs, op, cap, steps, sort_every, precision, snapshot=None, **kw):
    from paper_2609_31258_amd import mucite
    out = []
    for s in (0, sort_every):
        op.sort_every = s
        g = mucite.Sim(seed=synth.SEED, pack_capacity=cap, precision=precision, **kw)
        g.setup(f, ions, srcs, op)
        if snapshot is not None:
            g.write_packs(snapshot)
        g.step(steps)
        out.append(g)
    return out


@pytest.mark.parametrize("precision", [0, 1])
def test_sorted_run_equals_unsorted_run(precision):
    """Space-charge configuration at 100 packs per step: 160 steps, 16
    deposits, 23 sorts (every 7 steps)."""
    _say("sorted vs unsorted, precision", precision)
    f, ions, srcs, op, _ = synth.config_c2(n_packs=20_000, packs_per_step=100)
    a, b = _run_pair(f, ions, srcs, op, 20_000, 160, 7, precision, timing=True)
    t, n_exits = _compare(a, b)
    ia, ib = a.info(), b.info()
    _say(f"  active {t['class_n'][0]}, slots {ia['n_slots']} / {ib['n_slots']}, exits {n_exits}, "
         f"sorts {b.read_timing()['launches']['sort']}")
    assert b.read_timing()["launches"]["sort"] > 0
    assert t["class_n"][0] > 10_000
    assert int(a.read_charge().sum()) > 0
    a.close()
    b.close()


def test_compaction_drops_terminal_slots():
    """Terminal-event configuration: after a sort the slots hold the active
    packs only; packs and exits equal the unsorted run's."""
    _say("compaction")
    f, ions, srcs, op, meta = synth.config_c1x(4000, 2000)
    from paper_2609_31258_amd import mucite
    runs = []
    for s in (0, 100):
        op.sort_every = s
        g = mucite.Sim(seed=synth.SEED, pack_capacity=6000, precision=0)
        g.setup(f, ions, srcs, op)
        g.inject(0, 4000)
        g.inject(1, 2000)
        g.step(600)  # last sort at the start of step 500
        runs.append(g)
    a, b = runs
    t, n_exits = _compare(a, b)
    ia, ib = a.info(), b.info()
    pb = b.read_packs()
    _say(f"  active {t['class_n'][0]}, exits {n_exits}, slots {ia['n_slots']} unsorted, {ib['n_slots']} sorted")
    assert n_exits > 500 and t["class_n"][0] > 0
    assert ia["n_slots"] == 6000
    # terminal slots of the first 500 steps are gone; those of the last 100 remain
    assert t["class_n"][0] <= ib["n_slots"] < ia["n_slots"]
    assert int((pb["status"] != 0).sum()) == ib["n_slots"] - t["class_n"][0]
    a.close()
    b.close()


def test_sorted_species_mix_equals_unsorted():
    """Three species assigned round robin (every wavefront mixes them until
    the first sort), FP32 form with BF16 tables, space charge every 5 steps."""
    _say("species mix")
    f, ions, srcs, op, _ = synth.config_c5(n_packs=30_000, emit_steps=100, nr=128, nz=512)
    ions = ions[::4]  # three species: 200 Da, about 4 kDa and 5e4 Da
    n = 30_000
    snap = synth.pack_snapshot(n, f, seed=3, z_hi=2e-3, r_hi=3e-4, v_sigma=50.0, v_drift=300.0)
    snap["tag"] = (np.arange(n) % len(ions)).astype(np.int32)
    dof = np.array([3 * i.n_atoms - 6 for i in ions], float)[snap["tag"]]
    snap["e_int"] = dof * 1.380649e-23 * 600.0
    a, b = _run_pair(f, ions, [], op, n, 23, 5, 1, snapshot=snap)
    t, _ = _compare(a, b)
    _say(f"  active {t['class_n'][0]}, candidates {t['n_cand']}")
    pb = b.read_packs()
    # after the sort at step 20 the species occupy contiguous slot ranges
    tags = pb["tag"][pb["status"] == 0]
    assert np.count_nonzero(np.diff(tags)) <= len(ions) - 1 + int((pb["status"] != 0).sum())
    a.close()
    b.close()


def test_sorted_adaptive_run_equals_unsorted():
    """Adaptive step (Eq. 1) on the hybrid branch: stretches end at the
    sorted steps."""
    _say("adaptive with sorting")
    f, ions, srcs, op, _ = synth.config_c2(n_packs=8_000, packs_per_step=100)
    op.langevin_on, op.lv_z_lo, op.lv_z_hi, op.lv_switch = 1, 0.0, 1e-3, 0.05
    op.adaptive, op.dt, op.lv_dt_max = 1, 2e-9, 2e-9
    a, b = _run_pair(f, ions, srcs, op, 8_000, 150, 6, 0)
    t, _ = _compare(a, b)
    assert a.info()["time"] == b.info()["time"]
    _say(f"  active {t['class_n'][0]}, time {b.info()['time']:.3e}")
    a.close()
    b.close()


def test_sorted_deposit_matches_oracle_bit_exact():
    """The deposit of a sorting context (one kernel adding straight into the
    grid, wavefront sums where 64 packs share a cell) against the oracle on
    2e5 packs written in cell order: most wavefronts lie in one cell, some
    straddle two."""
    from oracle.binding import OracleSim
    from paper_2609_31258_amd import mucite
    _say("sorted deposit vs oracle")
    f, ions, srcs, op, _ = synth.config_c2(n_packs=200_000)
    n = 200_000
    snap = synth.pack_snapshot(n, f, seed=11, z_hi=4e-4, r_hi=2e-4, v_sigma=20.0)
    g = f.grid
    cell = (np.floor(snap["z"] / g.dz).astype(np.int64) * g.nr + np.floor(np.hypot(snap["x"], snap["y"]) / g.dr))
    order = np.argsort(cell, kind="stable")
    snap = {k: v[order] for k, v in snap.items()}
    op.sort_every = 50
    gpu = mucite.Sim(seed=synth.SEED, pack_capacity=n, precision=0)
    gpu.setup(f, ions, [], op)
    gpu.write_packs(snap)
    orc = OracleSim(synth.SEED)
    orc.setup(f, ions, [], op)
    orc.write_packs(snap)
    for rep in range(2):
        gpu.pic_update()
        orc.pic_update()
        qg, qo = gpu.read_charge(), orc.read_charge()
        _say(f"  update {rep}: cells {int((qo != 0).sum())}, total {int(qo.sum())}")
        assert np.array_equal(qg, qo)
    phi_g, _, _ = gpu.read_sc()
    phi_o, _, _ = orc.read_sc()
    assert np.allclose(phi_g, phi_o, rtol=1e-10, atol=1e-10 * np.abs(phi_o).max())
    gpu.close()
    orc.close()


def test_checkpoint_resume_with_sorting(tmp_path):
    """A sorting run saved between sorts and resumed continues bit for bit."""
    from paper_2609_31258_amd import mucite
    _say("checkpoint with sorting")
    path = str(tmp_path / "sorted.ckpt")
    f, ions, srcs, op, _ = synth.config_c2(n_packs=10_000, packs_per_step=200)
    op.sort_every = 9

    def make():
        g = mucite.Sim(seed=synth.SEED, pack_capacity=10_000, precision=1)
        g.setup(f, ions, srcs, op)
        return g

    a = make()
    a.step(31)
    a.save_state(path)
    a.step(40)
    b = make()
    b.load_state(path)
    b.step(40)
    pa, pb = a.read_packs(), b.read_packs()
    for k in pa:
        assert np.array_equal(pa[k], pb[k]), k
    ta, tb = a.read_tallies(), b.read_tallies()
    for k in ta:
        assert np.array_equal(np.asarray(ta[k]), np.asarray(tb[k])), k
    assert np.array_equal(a.read_charge(), b.read_charge())
    a.close()
    b.close()
