"""Oracle pins for the hybrid Langevin branch (collision section; Ermak and
Buckholz).  The friction rate against the heavy-sphere (Epstein, specular)
drag law, the relaxation against the Ornstein-Uhlenbeck semigroup and
equipartition, the drawn normals against the normal law, the drift in a
uniform field against the splitting factor that the explicit branch obeys,
and the branch selection (window, switch, frozen T_eff and hazard)."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import binding as O
from paper_2609_31258_amd import synth

KB, QE, DA = 1.380649e-23, 1.602176634e-19, 1.66053906892e-27
MG = 28.0134 * DA


def _snap(n, z, e_int=1e-19, v=(0.0, 0.0, 0.0)):
    full = lambda x: np.full(n, float(x))
    return dict(x=full(0.0), y=full(0.0), z=full(z), vx=full(v[0]), vy=full(v[1]), vz=full(v[2]),
                e_int=full(e_int), h=np.zeros(n), w=full(1.0), id=np.arange(n, dtype=np.int64),
                tag=np.zeros(n, np.int32))


def _sim(f, ion, op, seed=7):
    s = O.OracleSim(seed)
    s.setup(f, [ion], [], op)
    return s


def test_friction_rate_heavy_sphere_limit():
    """A sphere much heavier than the gas molecules, reflecting them
    specularly, feels the drag F = (4/3) n sigma mg cbar v (Epstein), so
    gamma -> (4/3) n sigma mg cbar / m; at finite mass the reduced mass
    enters as sqrt(mu / mg)."""
    tg, ns = 300.0, 3.7e7
    cbar = math.sqrt(8 * KB * tg / (math.pi * MG))
    for m_da in (1e7, 5e3, 500.0):
        m = m_da * DA
        mu = m * MG / (m + MG)
        epstein = (4.0 / 3.0) * ns * MG * cbar / m
        g = O.langevin_gamma(m, MG, ns, tg)
        assert g == pytest.approx(epstein * math.sqrt(mu / MG), rel=1e-12)
        if m_da >= 1e7:
            assert g == pytest.approx(epstein, rel=2e-6)


def test_relaxation_is_an_ornstein_uhlenbeck_semigroup():
    """Two half steps equal one full step: the mean part composes as
    exp(-g dt/2)^2 and the variances of the random parts add to the one-step
    variance (checked through the response to unit normals)."""
    m, g, tg, dt = 500 * DA, 1.3e9, 410.0, 0.9e-9
    u = np.array([3.0, -2.0, 250.0])
    v = np.array([40.0, 15.0, -70.0])
    z3 = np.zeros(3)
    one = O.langevin_relax(m, g, tg, u, dt, z3, v)
    half = O.langevin_relax(m, g, tg, u, dt / 2, z3, O.langevin_relax(m, g, tg, u, dt / 2, z3, v))
    assert np.allclose(one, half, rtol=1e-13, atol=1e-12)
    assert np.allclose(one - u, (v - u) * math.exp(-g * dt), rtol=1e-13)
    e = np.array([1.0, 0.0, 0.0])
    s1 = (O.langevin_relax(m, g, tg, u, dt, e, v) - one)[0]
    a = (O.langevin_relax(m, g, tg, u, dt / 2, e, v) - O.langevin_relax(m, g, tg, u, dt / 2, z3, v))[0]
    # response of the two-step map to a unit normal in the first half step
    b = (O.langevin_relax(m, g, tg, u, dt / 2, z3, v + np.array([a, 0, 0])) -
         O.langevin_relax(m, g, tg, u, dt / 2, z3, v))[0]
    assert s1 ** 2 == pytest.approx(b ** 2 + a ** 2, rel=1e-12)
    # long step: the random part alone is the Maxwellian width sqrt(kB T / m)
    big = O.langevin_relax(m, g, tg, u, 60.0 / g, e, v) - O.langevin_relax(m, g, tg, u, 60.0 / g, z3, v)
    assert big[0] == pytest.approx(math.sqrt(KB * tg / m), rel=1e-12)


def _box(p, tg, ez=0.0, nz=256):
    return synth.uniform_fields(16, nz, 5e-5, ez=ez, p=p, t_gas=tg)


def test_drawn_normals_follow_the_normal_law_and_freeze_internal_state():
    """With gamma dt >> 1 one step leaves v = sqrt(kB T/m) xi: the 3 n
    components must be standard normal (KS test), independent across axes
    (uncorrelated, and their squares' products of mean 1); internal energy
    and hazard stay exactly as they were."""
    tg = 350.0
    f = _box(1e5, tg)
    ion = synth.Ion(500.0, 1, 2e-18, 150, act_kind=1, act_p1=100e3, act_p2=-80.0)
    op = synth.Operating(dt=5e-8, z_det=f.grid.L, r_det=f.grid.R, collisions_on=1, langevin_on=1, lv_switch=0.05)
    s = _sim(f, ion, op)
    n = 20000
    s.write_packs(_snap(n, 3e-3, e_int=3.3e-19, v=(500.0, -200.0, 100.0)))
    s.step(1)
    p = s.read_packs()
    t = s.read_tallies()
    assert t["n_langevin"] == n and t["n_cand"] == 0
    assert np.all(p["e_int"] == 3.3e-19) and np.all(p["h"] == 0.0)
    xi = np.stack([p["vx"], p["vy"], p["vz"]]) / math.sqrt(KB * tg / (500 * DA))
    for row in xi:
        assert stats.kstest(row, "norm").pvalue > 1e-3
    c = np.corrcoef(xi)
    assert np.abs(c[np.triu_indices(3, 1)]).max() < 0.03
    # independence beyond correlation: for independent standard normals
    # E[xi_a^2 xi_b^2] = 1 (variance 8); normals that share a Box-Muller
    # radius or angle across axes are uncorrelated but fail this
    for a, b in ((0, 1), (0, 2), (1, 2)):
        m22 = float(np.mean(xi[a] ** 2 * xi[b] ** 2))
        assert abs(m22 - 1.0) < 6.0 * math.sqrt(8.0 / n), (a, b, m22)


def test_equipartition_and_rest_mean():
    tg = 500.0
    f = _box(2e4, tg)
    ion = synth.Ion(500.0, 1, 2e-18, 150)
    op = synth.Operating(dt=1e-9, z_det=f.grid.L, r_det=f.grid.R, collisions_on=1, langevin_on=1, lv_switch=0.05)
    s = _sim(f, ion, op)
    n = 4000
    s.write_packs(_snap(n, 3e-3))
    s.step(50)
    ke, mv = [], []
    m = 500 * DA
    for _ in range(40):
        s.step(5)
        p = s.read_packs()
        ke.append(0.5 * m * (p["vx"] ** 2 + p["vy"] ** 2 + p["vz"] ** 2).mean())
        mv.append(p["vz"].mean())
    assert np.mean(ke) == pytest.approx(1.5 * KB * tg, rel=0.01)
    assert abs(np.mean(mv)) < 0.02 * math.sqrt(KB * tg / m)


def _drift(p, tg, ez, dt, steps, langevin, n=2000):
    f = _box(p, tg, ez=ez)
    ion = synth.Ion(500.0, 1, 2e-18, 150, alpha=0.0)
    op = synth.Operating(dt=dt, z_det=f.grid.L, r_det=f.grid.R, collisions_on=1, langevin_on=int(langevin),
                         lv_switch=0.05)
    s = _sim(f, ion, op)
    s.write_packs(_snap(n, 2e-3))
    s.step(steps // 10)
    z0 = s.read_packs()["z"].mean()
    rest = steps - steps // 10
    s.step(rest)
    t = s.read_tallies()
    assert (t["n_langevin"] > 0) == bool(langevin)
    return (s.read_packs()["z"].mean() - z0) / (rest * dt)


def test_drift_in_uniform_field_splitting_factor():
    """Push then relax: per step v -> v + a dt, then (v - u) e^{-x}; the
    steady drift over the push is (a / gamma) (x/2) coth(x/2), x = gamma dt,
    the factor the explicit branch shows at the same step."""
    p, tg, ez, dt = 1e5, 300.0, 1e5, 1e-9
    m = 500 * DA
    g = O.langevin_gamma(m, MG, p / (KB * tg) * 2e-18, tg)
    x = g * dt
    vd = _drift(p, tg, ez, dt, 2000, True)
    assert vd == pytest.approx(QE * ez / (m * g) * (x / 2) / math.tanh(x / 2), rel=0.01)


def test_explicit_and_langevin_drift_agree():
    """Both branches at the same point and step: the explicit thinning and
    the aggregated relaxation give the same mean drift (first-approximation
    mobility of hard spheres, within the statistics of the explicit run)."""
    p, tg, ez, dt = 1e5, 300.0, 1e5, 1e-9
    ve = _drift(p, tg, ez, dt, 2000, False)
    vl = _drift(p, tg, ez, dt, 2000, True)
    assert vl == pytest.approx(ve, rel=0.04)


def test_window_and_switch_select_the_branch():
    tg = 300.0
    f = _box(1e5, tg)
    ion = synth.Ion(500.0, 1, 2e-18, 150)
    n = 3000
    snap = _snap(n, 0.0)
    snap["z"] = np.linspace(1e-3, 9e-3, n)
    base = dict(dt=1e-9, z_det=f.grid.L, r_det=f.grid.R, collisions_on=1, langevin_on=1)
    # window [4, 6) mm: exactly the packs whose post-push z lies inside
    s = _sim(f, ion, synth.Operating(**base, lv_z_lo=4e-3, lv_z_hi=6e-3, lv_switch=0.05))
    s.write_packs(snap)
    s.step(1)
    t, p = s.read_tallies(), s.read_packs()
    inside = int(((p["z"] >= 4e-3) & (p["z"] < 6e-3)).sum())
    assert t["n_langevin"] == inside and 0 < inside < n
    assert t["n_cand"] > 10 * (n - inside)
    # a switch above every pack's lambda dt (about 23 here): explicit everywhere
    s = _sim(f, ion, synth.Operating(**base, lv_switch=1e3))
    s.write_packs(snap)
    s.step(1)
    assert s.read_tallies()["n_langevin"] == 0
    # the branch off: explicit everywhere
    s = _sim(f, ion, synth.Operating(**{**base, "langevin_on": 0}))
    s.write_packs(snap)
    s.step(1)
    assert s.read_tallies()["n_langevin"] == 0
