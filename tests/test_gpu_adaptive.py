"""Adaptive global step (Eq. 1) on the GPU against the oracle.

Bars: the FP64 step sequence equals the oracle's within 1e-12 relative (both
take the same minimum over the same packs; rounding differs only inside the
per-pack terms), the states then agree pathwise within 1e-6 for 99 % of the
packs; space-charge updates land on their times; the FP32 form's first step
is within 1e-5 of the oracle's and every step within 5 % (its trajectories,
and so the extreme pack that sets the step, drift apart statistically); the
server runs adaptive queries (their parity with single runs is in test_gpu_serving.py)."""
import sys

import numpy as np
import pytest

from paper_2609_31258_amd import synth
from tests.parity_util import by_id, make_pair, thermal_speed

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("precision", [0, 1])
def test_adaptive_steps_match_oracle(precision):
    f, ions, srcs, op, _ = synth.config_c1t(3000)
    op.adaptive = 1
    op.sc_on, op.sc_every = 1, 4
    ions[0].ccs_m2 = 2e-18
    _say("adaptive steps, precision", precision)
    g, o = make_pair(f, ions, srcs, op, cap=3000, precision=precision)
    g.inject(0, 3000)
    o.inject(0, 3000)
    dg, do, tg, to = [], [], [], []
    for _ in range(40):
        g.step(1)
        o.step(1)
        i = g.info()
        dg.append(i["last_dt"])
        tg.append(i["time"])
        do.append(o.last_dt)
        to.append(o.time)
    dg, do = np.array(dg), np.array(do)
    rel = np.abs(dg - do) / do
    _say(f"  dt range {do.min():.3e}..{do.max():.3e} s, max rel diff {rel.max():.2e}, t {to[-1]:.3e} s")
    assert do.min() < 0.5 * op.dt  # the step really adapts
    if precision == 0:
        assert rel.max() <= 1e-12
        assert np.allclose(tg, to, rtol=1e-12, atol=0)
        a, b = by_id(g.read_packs()), by_id(o.read_packs())
        dv = np.linalg.norm(np.stack([a[k] - b[k] for k in ("vx", "vy", "vz")], 1), axis=1)
        vn = np.linalg.norm(np.stack([b[k] for k in ("vx", "vy", "vz")], 1), axis=1)
        good = np.mean(dv <= 1e-6 * (vn + thermal_speed()))
        _say(f"  pathwise-identical fraction {good:.5f}")
        assert good >= 0.99
    else:
        assert rel[0] <= 1e-5 and rel.max() <= 0.05
    g.close()


def test_space_charge_times_and_langevin_cap_on_gpu():
    from paper_2609_31258_amd import mucite
    h = 5e-5
    f = synth.uniform_fields(16, 256, h, p=1e5, t_gas=300.0)
    ion = synth.Ion(500.0, 1, 2e-18, 150)
    op = synth.Operating(dt=1e-9, z_det=f.grid.L, r_det=f.grid.R, collisions_on=1, adaptive=1, sc_on=1, sc_every=3,
                         langevin_on=1, lv_switch=0.05, lv_dt_max=0.7e-9)
    n = 100
    snap = dict(x=np.zeros(n), y=np.zeros(n), z=np.linspace(1e-3, 2e-3, n), vx=np.zeros(n), vy=np.zeros(n),
                vz=np.zeros(n), e_int=np.full(n, 1e-19), h=np.zeros(n), w=np.ones(n),
                id=np.arange(n, dtype=np.int64), tag=np.zeros(n, np.int32))
    g, o = make_pair(f, [ion], [], op, cap=n)
    g.write_packs(snap)
    o.write_packs(snap)
    tg, to = [g.info()["time"]], [o.time]
    for _ in range(12):
        g.step(1)
        o.step(1)
        tg.append(g.info()["time"])
        to.append(o.time)
    assert np.allclose(tg, to, rtol=1e-13, atol=0)
    d = np.diff(tg)
    assert d.max() <= 0.7e-9 * (1 + 1e-12)  # the Langevin cap
    for k in (1, 2):
        assert np.min(np.abs(np.array(tg) - k * 3e-9)) <= 1e-6 * 1e-9
    assert g.read_tallies()["n_langevin"] > 0
    g.close()


def test_server_runs_adaptive_queries_and_refuses_a_negative_langevin_cap():
    from paper_2609_31258_amd import mucite
    f = synth.ring_fields(64, 256)
    ion = synth.Ion(500.0, 1, 2e-18, 150)
    src = synth.Source(kind=1, current_a=1e-9, packs_per_step=10, n_total=100, sigma_r=1e-4, r_trunc=3e-4)
    op = synth.Operating(dt=1e-9, z_det=f.grid.L, r_det=f.grid.R, adaptive=1)
    with mucite.Server(f, hbm_budget=1 << 28, precision=0, max_resident=2) as s:
        r = s.wait(s.submit(ion, src, op, n_steps=10, seed=1))
        assert r["state"] == mucite.Q_DONE and r["tallies"]["pack_steps"] > 0
        with pytest.raises(mucite.MucateError) as e:
            s.submit(ion, src, synth.Operating(**{**op.__dict__, "lv_dt_max": -1.0}), n_steps=10, seed=1)
        assert e.value.code == mucite.MC_EINVAL


def test_collapsed_step_halts_the_run_like_the_oracle():
    """A largest step of 1 s against a collision limit near 1e-12 s: the first
    Eq. 1 step collapses below 1e-9 of the largest step.  Both sides stop
    there with the step counter at 0, after the samples of step 0; the GPU's
    later steps of the same call take no samples and advance no pack."""
    from oracle.binding import OracleSim
    from paper_2609_31258_amd import mucite
    f = synth.uniform_fields(16, 128, 5e-5, p=1e5, t_gas=300.0)
    ion = synth.Ion(500.0, 1, 2e-18, 150)
    op = synth.Operating(dt=1.0, z_det=f.grid.L, r_det=f.grid.R, collisions_on=1, adaptive=1, sample_every=1,
                         sample_stride=1)
    n = 100
    snap = dict(x=np.zeros(n), y=np.zeros(n), z=np.linspace(1e-3, 2e-3, n), vx=np.zeros(n), vy=np.zeros(n),
                vz=np.full(n, 50.0), e_int=np.full(n, 1e-19), h=np.zeros(n), w=np.ones(n),
                id=np.arange(n, dtype=np.int64), tag=np.zeros(n, np.int32))
    _say("collapsed adaptive step")
    g = mucite.Sim(seed=7, pack_capacity=n, precision=0, sample_capacity=10 * n)
    g.setup(f, [ion], [], op)
    g.write_packs(snap)
    o = OracleSim(7)
    o.setup(f, [ion], [], op)
    o.write_packs(snap)
    with pytest.raises(mucite.MucateError) as e:
        g.step(5)
    assert e.value.code == mucite.MC_ENUMERIC
    with pytest.raises(Exception):
        o.step(5)
    assert g.info()["step"] == o.current_step == 0
    assert len(g.read_samples()) == len(o.read_samples()) == n
    assert g.read_tallies()["pack_steps"] == 0
    p = g.read_packs()
    assert np.array_equal(p["z"], snap["z"]) and np.array_equal(p["vz"], snap["vz"])
    g.close()
