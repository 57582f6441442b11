"""Oracle pins for the adaptive global step of Eq. 1: each term alone against
its closed form (CFL, acceleration, collision, RF, Langevin cap), the
space-charge updates landing on their times, emission following the varying
step (Eq. 5 over simulated time), and the fixed-step mode unchanged."""
import math

import numpy as np
import pytest

from oracle import binding as O
from paper_2609_31258_amd import synth

KB, QE, DA = 1.380649e-23, 1.602176634e-19, 1.66053906892e-27
MG = 28.0134 * DA


def _snap(z, vz, e_int=1e-19):
    n = len(z)
    return dict(x=np.zeros(n), y=np.zeros(n), z=np.asarray(z, float), vx=np.zeros(n), vy=np.zeros(n),
                vz=np.asarray(vz, float), e_int=np.full(n, e_int), h=np.zeros(n), w=np.ones(n),
                id=np.arange(n, dtype=np.int64), tag=np.zeros(n, np.int32))


def _sim(f, op, ion=None, srcs=()):
    s = O.OracleSim(7)
    s.setup(f, [ion or synth.Ion(500.0, 1, 2e-18, 150)], list(srcs), op)
    return s


def _first_dt(f, op, snap, ion=None):
    s = _sim(f, op, ion)
    s.write_packs(snap)
    s.step(1)
    return s.last_dt


def test_cfl_term():
    h = 5e-5
    f = synth.uniform_fields(16, 256, h)
    op = synth.Operating(dt=1e-6, z_det=f.grid.L, r_det=f.grid.R, collisions_on=0, adaptive=1)
    dt = _first_dt(f, op, _snap([2e-3, 3e-3], [40.0, -130.0]))
    assert dt == pytest.approx(0.5 * h / 130.0, rel=1e-14)


def test_acceleration_term():
    h, ez, m = 5e-5, 3e3, 500.0
    f = synth.uniform_fields(16, 256, h, ez=ez, t_gas=0.0)  # no gas at all
    op = synth.Operating(dt=1e-6, z_det=f.grid.L, r_det=f.grid.R, collisions_on=0, adaptive=1)
    a = QE * ez / (m * DA)
    # a pack at rest with no gas: the time to move half a spacing from rest
    assert _first_dt(f, op, _snap([2e-3], [0.0])) == pytest.approx(math.sqrt(h / a), rel=1e-12)
    # a moving pack: a tenth of its speed per step (CFL looser here)
    v = 2.0
    assert _first_dt(f, op, _snap([2e-3], [v])) == pytest.approx(0.1 * v / a, rel=1e-12)
    # in a still gas at 300 K (collisions off) the speed scale adds the ion's
    # thermal speed sqrt(kB T / m): a pack at rest takes a tenth of it
    tg = 300.0
    g = synth.uniform_fields(16, 256, h, ez=ez, p=1e3, t_gas=tg)
    vth = math.sqrt(KB * tg / (m * DA))
    assert _first_dt(g, op, _snap([2e-3], [0.0])) == pytest.approx(0.1 * vth / a, rel=1e-12)
    assert _first_dt(g, op, _snap([2e-3], [v])) == pytest.approx(0.1 * (v + vth) / a, rel=1e-12)


def test_collision_term_limits_the_collision_probability():
    tg, p = 300.0, 2e4
    f = synth.uniform_fields(16, 256, 5e-5, p=p, t_gas=tg)
    ion = synth.Ion(500.0, 1, 2e-18, 150)
    op = synth.Operating(dt=1e-6, z_det=f.grid.L, r_det=f.grid.R, collisions_on=1, adaptive=1)
    dt = _first_dt(f, op, _snap([2e-3], [0.0]), ion)
    abar = math.sqrt(8 * KB * tg / (math.pi * MG))
    lam = p / (KB * tg) * 2e-18 * abar
    assert dt == pytest.approx(0.1 / lam, rel=1e-12)
    # over many steps the collision probability per step stays near 1 - exp(-0.1)
    s = _sim(f, op, ion)
    n = 4000
    s.write_packs(_snap(np.full(n, 2e-3), np.zeros(n)))
    s.step(30)
    t = s.read_tallies()
    assert t["n_cand"] / (30 * n) < 0.1 * 1.01


def test_rf_term_and_largest_step():
    f = synth.uniform_fields(16, 256, 5e-5)
    op = synth.Operating(dt=1e-6, v_rf=10.0, f_rf=2e6, z_det=f.grid.L, r_det=f.grid.R, collisions_on=0, adaptive=1)
    assert _first_dt(f, op, _snap([2e-3], [0.0])) == pytest.approx(0.05 / 2e6, rel=1e-14)
    op2 = synth.Operating(dt=3e-9, z_det=f.grid.L, r_det=f.grid.R, collisions_on=0, adaptive=1)
    assert _first_dt(f, op2, _snap([2e-3], [0.0])) == 3e-9


def test_langevin_cap():
    f = synth.uniform_fields(16, 256, 5e-5, p=1e5, t_gas=300.0)
    op = synth.Operating(dt=5e-9, z_det=f.grid.L, r_det=f.grid.R, collisions_on=1, adaptive=1, langevin_on=1,
                         lv_switch=0.05, lv_dt_max=2e-9)
    # every pack on the Langevin branch: no collision term, the cap instead
    assert _first_dt(f, op, _snap([2e-3, 3e-3], [0.0, 0.0])) == 2e-9


def test_space_charge_updates_land_on_their_times():
    h = 5e-5
    f = synth.uniform_fields(16, 256, h)
    dt_max, every = 1e-9, 3
    op = synth.Operating(dt=dt_max, z_det=f.grid.L, r_det=f.grid.R, collisions_on=0, adaptive=1, sc_on=1,
                         sc_every=every)
    v = 0.5 * h / 0.7e-9  # CFL step 0.7 ns, not a divisor of the 3 ns period
    s = _sim(f, op)
    s.write_packs(_snap([1e-3], [v]))
    times, dts = [], []
    for _ in range(14):
        times.append(s.time)
        s.step(1)
        dts.append(s.last_dt)
    times.append(s.time)
    assert np.allclose(np.diff(times), dts, rtol=1e-14, atol=0)
    period = every * dt_max
    for k in range(1, 3):  # the step before each update is shortened to land on it
        hit = np.min(np.abs(np.array(times) - k * period))
        assert hit <= 1e-6 * dt_max
    assert max(dts) <= 0.7e-9 * (1 + 1e-12)


def test_emission_follows_simulated_time():
    tg = 300.0
    f = synth.uniform_fields(16, 256, 5e-5)
    ion = synth.Ion(500.0, 1, 2e-18, 150)
    cur = 2e-9
    src = synth.Source(kind=2, current_a=cur, weight=200.0, n_total=10 ** 6, sigma_r=1e-5, r_trunc=3e-5,
                       z_inj=1e-3)
    op = synth.Operating(dt=1e-9, z_det=f.grid.L, r_det=f.grid.R, collisions_on=0, adaptive=1)
    s = _sim(f, op, ion, [src])
    s.write_packs(_snap([2e-3], [6e4]))  # its CFL step (0.42 ns) sets the pace
    total = 0.0
    for _ in range(200):
        s.step(1)
        total += s.last_dt
    t = s.read_tallies()
    real = cur * total / QE
    assert total < 150e-9  # the CFL step, not the 1 ns largest step
    assert abs(t["emitted_w"] * 2.0 ** -32 - real) <= 200.0
    assert total == pytest.approx(s.time, rel=1e-14)


def test_fixed_step_mode_unchanged():
    f = synth.uniform_fields(16, 256, 5e-5, ez=1e3)
    op = synth.Operating(dt=1e-9, z_det=f.grid.L, r_det=f.grid.R, collisions_on=0)
    s = _sim(f, op)
    s.write_packs(_snap([2e-3], [10.0]))
    s.step(7)
    assert s.last_dt == 1e-9 and s.time == 7 * 1e-9
