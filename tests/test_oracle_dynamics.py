"""Oracle pins: push, classification, emission, collisions, dissociation,
tallies.  Closed forms, invariants and statistics that the mathematics fixes."""
import math

import numpy as np
import pytest

from oracle import binding as O
from paper_2609_31258_amd import synth

KB, QE, DA, EPS0 = 1.380649e-23, 1.602176634e-19, 1.66053906892e-27, 8.8541878188e-12
MG = 28.0134 * DA


def _snap(n, x, y, z, vx, vy, vz, e_int=1e-19, w=1.0, tag=0):
    full = lambda v: np.broadcast_to(np.asarray(v, dtype=float), (n,)).copy()
    return dict(x=full(x), y=full(y), z=full(z), vx=full(vx), vy=full(vy), vz=full(vz), e_int=full(e_int),
                h=np.zeros(n), w=full(w), id=np.arange(n, dtype=np.int64), tag=np.full(n, tag, np.int32))


def _sim(fields, ion, op, seed=7, sources=()):
    s = O.OracleSim(seed)
    s.setup(fields, [ion], list(sources), op)
    return s


# ----------------------------------------------------------------------------
# Push (RK4, Eqs. 3-4)
# ----------------------------------------------------------------------------

def test_uniform_field_drift_is_exact_and_energy_conserved():
    h = 5e-5
    ez = 2.0e4
    f = synth.uniform_fields(16, 400, h, ez=ez)
    ion = synth.Ion(500.0, 2, 2e-18, 150)
    dt = 1e-9
    op = synth.Operating(dt=dt, z_det=f.grid.L, r_det=f.grid.R, collisions_on=0)
    s = _sim(f, ion, op)
    rng = np.random.default_rng(2)
    n = 64
    v0 = rng.normal(0, 50, (n, 3))
    x0 = np.stack([rng.uniform(-2e-4, 2e-4, n), rng.uniform(-2e-4, 2e-4, n), np.full(n, 2e-3)], axis=1)
    s.write_packs(_snap(n, x0[:, 0], x0[:, 1], x0[:, 2], v0[:, 0], v0[:, 1], v0[:, 2]))
    steps = 1000
    s.step(steps)
    p = s.read_packs()
    t = steps * dt
    a = 2 * QE * ez / (500.0 * DA)
    assert np.allclose(p["z"], x0[:, 2] + v0[:, 2] * t + 0.5 * a * t * t, rtol=1e-12, atol=1e-15)
    assert np.allclose(p["x"], x0[:, 0] + v0[:, 0] * t, rtol=1e-12, atol=1e-15)
    assert np.allclose(p["vz"], v0[:, 2] + a * t, rtol=1e-12)
    m, q = 500.0 * DA, 2 * QE
    e0 = 0.5 * m * (v0 ** 2).sum(1) + q * (-ez * x0[:, 2])
    e1 = 0.5 * m * (p["vx"] ** 2 + p["vy"] ** 2 + p["vz"] ** 2) + q * (-ez * p["z"])
    assert np.allclose(e1, e0, rtol=1e-10)


def test_rf_field_closed_form():
    h = 5e-5
    e0 = 3.0e3  # RF basis field per volt
    f = synth.uniform_fields(16, 400, h, rf_ez=e0)
    ion = synth.Ion(500.0, 1, 2e-18, 150)
    dt, vrf, freq = 1e-9, 10.0, 1e6
    op = synth.Operating(dt=dt, v_rf=vrf, f_rf=freq, z_det=f.grid.L, r_det=f.grid.R, collisions_on=0)
    s = _sim(f, ion, op)
    s.write_packs(_snap(4, 0.0, 0.0, 5e-3, 0.0, 0.0, [0.0, 10.0, -20.0, 5.0]))
    steps = 1500
    s.step(steps)
    p = s.read_packs()
    t, w = steps * dt, 2 * math.pi * freq
    amp = QE * vrf * e0 / (500.0 * DA)
    vz0 = np.array([0.0, 10.0, -20.0, 5.0])
    z_exact = 5e-3 + vz0 * t + amp / w ** 2 * (1 - math.cos(w * t))
    v_exact = vz0 + amp / w * math.sin(w * t)
    assert np.allclose(p["z"], z_exact, rtol=0, atol=1e-12)
    assert np.allclose(p["vz"], v_exact, rtol=0, atol=1e-8)


def test_radial_projection_zero_on_axis():
    """E_x = E_r x/r, E_y = E_r y/r, no transverse force on the axis (Eq. 3)."""
    h = 5e-5
    f = synth.uniform_fields(16, 64, h)
    R = np.arange(16) * h
    f.phi_dc = np.ascontiguousarray(np.repeat((-4e6 * R ** 2)[None, :], 64, axis=0))  # E_r = 8e6 r
    ion = synth.Ion(500.0, 1, 2e-18, 150)
    dt = 1e-10
    op = synth.Operating(dt=dt, z_det=f.grid.L, r_det=f.grid.R, collisions_on=0)
    s = _sim(f, ion, op)
    s.write_packs(_snap(3, [0.0, 3 * h, 0.0], [0.0, 0.0, -5 * h], 1e-3, 0.0, 0.0, 0.0))
    s.step(1)
    p = s.read_packs()
    assert p["vx"][0] == 0.0 and p["vy"][0] == 0.0
    a_r = QE / (500 * DA) * 8e6
    assert p["vx"][1] == pytest.approx(a_r * 3 * h * dt, rel=1e-6) and abs(p["vy"][1]) < 1e-20
    assert p["vy"][2] == pytest.approx(-a_r * 5 * h * dt, rel=1e-6) and abs(p["vx"][2]) < 1e-20


# ----------------------------------------------------------------------------
# Terminal classification
# ----------------------------------------------------------------------------

def _class_sim(d_hit=1e-5):
    h = 2.0 ** -14  # exact binary spacing: half-node ties are exact
    nr, nz = 20, 40
    f = synth.uniform_fields(nr, nz, h)
    f.mask[30, 8] = 1
    ion = synth.Ion(500.0, 1, 2e-18, 150)
    op = synth.Operating(dt=1e-9, z_det=f.grid.L, r_det=0.5 * f.grid.R, collisions_on=0, d_hit=d_hit,
                         exit_bin_dt=1e-9, n_exit_bins=10)
    return _sim(f, ion, op), f, h


def test_classification_cases():
    s, f, h = _class_sim()
    L, R = f.grid.L, f.grid.R
    dt = 1e-9
    cases = [
        # (x, y, z, vx, vy, vz) -> class
        ((8 * h, 0, 30 * h, 0, 0, 0), 2),            # on the metal node
        ((7.5 * h, 0, 30 * h, 0, 0, 0), 2),          # tie in r rounds up onto the metal node
        ((8 * h, 0, 29.5 * h, 0, 0, 0), 2),          # tie in z rounds up onto the metal node
        ((7.49 * h, 0, 30 * h, 0, 0, 0), 0),         # nearest node is not metal
        ((8 * h, 0, 30.5 * h, 0, 0, 0), 0),          # tie rounds up away from the metal node
        ((0.0, 0.0, L - 0.25 * h, 0, 0, 0.5 * h / dt), 1),   # crosses the detector on axis
        ((0.9 * R, 0.0, L - 0.25 * h, 0, 0, 0.5 * h / dt), 4),  # crosses outside r_det
        ((0.0, 0.0, 0.25 * h, 0, 0, -0.5 * h / dt), 4),       # leaves upstream
        ((R - 0.1 * h, 0.0, 10 * h, 0.2 * h / dt, 0, 0), 3),  # radial loss
        ((0.0, R - 0.1 * h, 10 * h, 0, 0.2 * h / dt, 0), 3),
    ]
    n = len(cases)
    arr = np.array([c[0] for c in cases], dtype=float)
    s.write_packs(_snap(n, arr[:, 0], arr[:, 1], arr[:, 2], arr[:, 3], arr[:, 4], arr[:, 5]))
    s.step(1)
    p = s.read_packs()
    assert list(p["status"]) == [c[1] for c in cases]
    ex = s.read_exits()
    byid = {int(e["id"]): e for e in ex}
    for k in (0, 1, 2):
        assert (byid[k]["inode"], byid[k]["jnode"]) == (8, 30)
    # crossing point: linear interpolation to the plane, at half the step
    e = byid[5]
    assert e["t_cross"] == pytest.approx(0.5 * dt, rel=1e-9)
    assert e["r_cross"] == 0.0
    e = byid[6]
    assert e["r_cross"] == pytest.approx(0.9 * R, rel=1e-12)
    T = s.read_tallies()
    assert T["exit_bins"][0] == 2 ** 32  # Eq. 8: unit weight crossing in bin 0
    assert T["loss_map"][30, 8] == 3 * 2 ** 32
    assert T["class_n"].tolist() == [2, 1, 3, 2, 2, 0]


def test_hit_distance():
    h = 2.0 ** -14
    s, _, _ = _class_sim(d_hit=0.0)  # reach = h/2: the metal node only
    assert s.read_hit().sum() == 1
    s2, _, _ = _class_sim(d_hit=1.2 * h)  # reach = 1.7 h: 4- and 8-neighbours
    hit = s2.read_hit()
    assert hit.sum() == 9 and hit[29:32, 7:10].all()
    s3, _, _ = _class_sim(d_hit=0.95 * h)  # reach = 1.45 h: 4-neighbours and diagonals (1.414 h)
    assert s3.read_hit().sum() == 9
    s4, _, _ = _class_sim(d_hit=0.6 * h)  # reach = 1.1 h: 4-neighbours only
    assert s4.read_hit().sum() == 5


# ----------------------------------------------------------------------------
# Emission (Eq. 5 and the Gaussian source)
# ----------------------------------------------------------------------------

def test_current_accumulator_eq5():
    f = synth.uniform_fields(16, 64, 5e-5, t_gas=300.0)
    ion = synth.Ion(500.0, 3, 2e-18, 150)
    dt, cur, w = 1e-9, 7e-9, 0.37
    op = synth.Operating(dt=dt, z_det=f.grid.L, r_det=f.grid.R, collisions_on=0)
    src = synth.Source(kind=2, current_a=cur, weight=w, n_total=10 ** 9, sigma_r=1e-4, r_trunc=3e-4,
                       z_inj=1e-3)
    s = _sim(f, ion, op, sources=[src])
    for n in (1, 10, 137, 1000):
        s.step(n - s.current_step)
        T = s.read_tallies()
        real = cur * n * dt / (3 * QE)
        assert T["emitted_n"] * w <= real * (1 + 1e-12) and real < (T["emitted_n"] + 1) * w * (1 + 1e-12)
        assert T["emitted_w"] == T["emitted_n"] * round(w * 2 ** 32)
        assert T["class_w"].sum() == T["emitted_w"]  # emitted = active + terminal


def test_fixed_rate_source_and_weight():
    f = synth.uniform_fields(16, 64, 5e-5)
    ion = synth.Ion(5000.0, 5, 1.5e-17, 1500)
    dt = 0.5e-9
    op = synth.Operating(dt=dt, z_det=f.grid.L, r_det=f.grid.R, collisions_on=0)
    src = synth.Source(kind=1, current_a=10e-9, packs_per_step=500, n_total=1700, sigma_r=1e-4, r_trunc=3e-4)
    s = _sim(f, ion, op, sources=[src])
    s.step(2)
    assert s.n_packs == 1000
    s.step(3)
    assert s.n_packs == 1700
    p = s.read_packs()
    w = 10e-9 * dt / (5 * QE) / 500
    assert np.allclose(p["w"], w, rtol=1e-15)
    assert w == pytest.approx(0.012483, rel=1e-4)
    assert np.all(p["q"] == round(5 * w * 2 ** 32))


def test_injection_distribution():
    stats = pytest.importorskip("scipy.stats")
    f = synth.uniform_fields(32, 64, 5e-5, t_gas=400.0, uz=250.0, ur=0.0)
    ion = synth.Ion(500.0, 1, 2e-18, 150)
    op = synth.Operating(dt=1e-9, z_det=f.grid.L, r_det=f.grid.R, collisions_on=0)
    sig, rt = 1e-4, 2.5e-4
    src = synth.Source(kind=0, weight=1.0, sigma_r=sig, r_trunc=rt, z_inj=1e-3)
    s = _sim(f, ion, op, sources=[src])
    n = 40000
    s.inject(0, n)
    p = s.read_packs()
    r = np.hypot(p["x"], p["y"])
    assert r.max() <= rt
    cdf = lambda x: (1 - np.exp(-np.minimum(x, rt) ** 2 / (2 * sig ** 2))) / (1 - math.exp(-rt ** 2 / (2 * sig ** 2)))
    assert stats.kstest(r, cdf).pvalue > 1e-3
    assert stats.kstest(np.arctan2(p["y"], p["x"]), "uniform", args=(-math.pi, 2 * math.pi)).pvalue > 1e-3
    vth2 = KB * 400.0 / (500 * DA)
    for comp, mean in (("vx", 0.0), ("vy", 0.0), ("vz", 250.0)):
        v = p[comp]
        assert abs(v.mean() - mean) < 5 * math.sqrt(vth2 / n)
        assert v.var() == pytest.approx(vth2, rel=5 * math.sqrt(2 / n))
    assert np.all(p["z"] == 1e-3)
    assert np.allclose(p["e_int"], O.einstein_u(300.0, 150), rtol=0)


# ----------------------------------------------------------------------------
# Collisions (Eq. 6 and the explicit collision adapter)
# ----------------------------------------------------------------------------

def _gbar(s, a):
    """Mean relative speed |v - w| for a Maxwellian w of 1-D width a."""
    if s == 0.0:
        return a * math.sqrt(8 / math.pi)
    return a * math.sqrt(2 / math.pi) * math.exp(-s * s / (2 * a * a)) + (s + a * a / s) * math.erf(s / (math.sqrt(2) * a))


def _moment_g(k, s, a):
    """E|g|^k for g = s e_z - w, w Maxwellian: noncentral chi distribution."""
    from scipy.integrate import quad
    if s == 0.0:
        pdf = lambda r: math.sqrt(2 / math.pi) * r * r / a ** 3 * math.exp(-r * r / (2 * a * a))
    else:
        pdf = lambda r: r / (s * a * math.sqrt(2 * math.pi)) * (math.exp(-(r - s) ** 2 / (2 * a * a)) -
                                                                 math.exp(-(r + s) ** 2 / (2 * a * a)))
    return quad(lambda r: r ** k * pdf(r), 0, s + 12 * a, limit=200)[0]


@pytest.mark.parametrize("s_over_a", [0.0, 1.0, 4.0])
def test_collision_rate_and_partner_law(s_over_a):
    pytest.importorskip("scipy")
    p, tg, m_da, ccs, dt = 1e5, 300.0, 500.0, 2e-18, 1e-9
    a = math.sqrt(KB * tg / MG)
    u = np.array([10.0, -20.0, 300.0])
    v = u + np.array([0.0, 0.0, s_over_a * a])
    nsteps = 20000
    r = O.collision_probe(m_da, ccs, 28.0134, p, tg, u, v, dt, nsteps, 99)
    n_gas = p / (KB * tg)
    expect = n_gas * ccs * _gbar(s_over_a * a, a) * dt * nsteps
    assert r["n_acc"] == pytest.approx(expect, rel=5 / math.sqrt(expect))
    # accepted partners are distributed as |g| f(w): E[|g|^2 | accepted] = E|g|^3 / E|g|
    e3, e1 = _moment_g(3, s_over_a * a, a), _moment_g(1, s_over_a * a, a)
    assert e1 == pytest.approx(_gbar(s_over_a * a, a), rel=1e-8)
    assert r["sum_g2"] / r["n_acc"] == pytest.approx(e3 / e1, rel=0.01)
    if s_over_a == 0.0:
        assert e3 / e1 == pytest.approx(4 * a * a, rel=1e-8)


def test_iict_update_conserves_momentum_and_energy():
    rng = np.random.default_rng(8)
    m, mg = 500 * DA, MG
    for alpha in (0.0, 1.0):
        for _ in range(200):
            v = rng.normal(0, 300, 3)
            vg = rng.normal(0, 300, 3)
            e_int = rng.uniform(1e-20, 1e-18)
            uni = rng.uniform(0, 1, 5)
            vo, vgo, eo, cl, ex = O.iict_update(m, mg, v, vg, e_int, 450.0, alpha, uni)
            assert ex == (1 if alpha == 1.0 else 0)
            assert np.allclose(m * vo + mg * vgo, m * v + mg * vg, rtol=1e-12, atol=1e-30)
            ke0 = 0.5 * m * v @ v + 0.5 * mg * vg @ vg + e_int
            ke1 = 0.5 * m * vo @ vo + 0.5 * mg * vgo @ vgo + eo
            assert ke1 == pytest.approx(ke0, rel=1e-12)
            assert eo >= 0.0
            if alpha == 0.0:
                assert eo == e_int
                assert np.linalg.norm(vo - vgo) == pytest.approx(np.linalg.norm(v - vg), rel=1e-12)


def _gas_box(p, tg, ez=0.0, nr=16, nz=128):
    return synth.uniform_fields(nr, nz, 5e-5, ez=ez, p=p, t_gas=tg)


def _einstein_heat_capacity(t, n_atoms, theta=1100.0):
    """Textbook heat capacity of s = 3N - 6 Einstein oscillators,
    C = s kB x^2 e^x / (e^x - 1)^2 with x = theta / T."""
    x = theta / t
    return (3 * n_atoms - 6) * KB * x * x * math.exp(x) / math.expm1(x) ** 2


def test_thermalisation_to_gas_temperature():
    """Uniform gas at 500 K, packs starting at T_eff = 300 K: the translational
    energy goes to (3/2) kB T, the mean T_eff to T, and the spread of T_eff
    about it to that of a canonical bath, sqrt(kB T^2 / C) (C the heat
    capacity of the internal modes at T)."""
    tg = 500.0
    f = _gas_box(1e5, tg)
    ion = synth.Ion(500.0, 1, 2e-18, 150)
    op = synth.Operating(dt=1e-9, z_det=f.grid.L, r_det=f.grid.R, collisions_on=1)
    s = _sim(f, ion, op)
    n = 2000
    s.write_packs(_snap(n, 0.0, 0.0, 3e-3, 0.0, 0.0, 0.0, e_int=O.einstein_u(300.0, 150)))
    s.step(120)
    ke, te, var = [], [], []
    m = 500 * DA
    for _ in range(40):
        s.step(2)
        p = s.read_packs()
        assert np.all(p["status"] == 0)
        ke.append(0.5 * m * (p["vx"] ** 2 + p["vy"] ** 2 + p["vz"] ** 2).mean())
        t = np.array([O.einstein_t(e, 150) for e in p["e_int"]])
        te.append(t.mean())
        var.append(t.var())
    assert np.mean(ke) == pytest.approx(1.5 * KB * tg, rel=0.015)
    assert np.mean(te) == pytest.approx(tg, rel=0.01)
    sd_canonical = math.sqrt(KB * tg * tg / _einstein_heat_capacity(tg, 150))
    assert sd_canonical == pytest.approx(28.8, abs=0.1)
    assert math.sqrt(np.mean(var)) == pytest.approx(sd_canonical, rel=0.05)


def _head_on_transfer(m1, m2):
    """Share of the kinetic energy that a head-on elastic collision passes
    from a moving m1 to m2 at rest: the non-trivial root a = v1'/v1 of
    momentum and energy conservation, m1 = m1 a + m2 b and
    m1 = m1 a^2 + m2 b^2 (v1 = 1), solved numerically; the share is 1 - a^2."""
    k = m1 * m1 / m2
    roots = np.roots([m1 + k, -2 * k, k - m1]).real
    a = roots[np.argmax(np.abs(roots - 1.0))]
    return 1.0 - a * a


def _exchange_counts(alpha, m_da=500.0, n_atoms=150, n=4000, steps=20):
    f = _gas_box(1e5, 300.0)
    ion = synth.Ion(m_da, 1, 2e-18, n_atoms, alpha=alpha)
    op = synth.Operating(dt=1e-9, z_det=f.grid.L, r_det=f.grid.R, collisions_on=1)
    s = _sim(f, ion, op)
    s.write_packs(_snap(n, 0.0, 0.0, 3e-3, 0.0, 0.0, 0.0, e_int=O.einstein_u(300.0, n_atoms)))
    s.step(steps)
    t = s.read_tallies()
    return t["n_exchange"], t["n_coll"]


@pytest.mark.parametrize("alpha,m_da,n_atoms", [(0.0, 500.0, 150), (0.2, 500.0, 150), (1.0, 500.0, 150),
                                                 (-1.0, 500.0, 150), (-1.0, 10 * 28.0134, 10)])
def test_exchange_fraction_per_accepted_collision(alpha, m_da, n_atoms):
    """The internal-energy exchange happens on a fraction alpha of the
    accepted collisions (binomial, 5 sigma).  alpha < 0 selects the default:
    the head-on elastic transfer share between a gas molecule and one atom
    of the ion (mass m/N), 0.3801 for the 500 Da, 150-atom ion and exactly 1
    when an atom weighs as much as the gas molecule."""
    ex, acc = _exchange_counts(alpha, m_da, n_atoms)
    assert acc > 500_000
    want = alpha if alpha >= 0.0 else _head_on_transfer(28.0134, m_da / n_atoms)
    if alpha < 0.0 and n_atoms == 150:
        assert want == pytest.approx(0.3801, abs=1e-4)
    if want in (0.0, 1.0):
        assert ex == round(want * acc)
    else:
        assert abs(ex / acc - want) < 5 * math.sqrt(want * (1 - want) / acc), (ex / acc, want)


def test_internal_energy_relaxation_rate():
    """Initial heating of the internal modes by the gas: ion translation at
    the gas temperature T, internal modes at T0.  Accepted collisions come
    at nu = n sigma <|g|>, <|g|> = sqrt(8 kB T / (pi mu)); their relative
    energy is Gamma(2, kB T) (mean 2 kB T) and a fraction alpha of them
    redraw it from the bath, Gamma(2, kB T_eff) (mean 2 kB T_eff), the
    difference going to E_int:
        d<E_int>/dt = alpha nu 2 kB (T - T_eff),
    with T_eff relaxing at kappa = 2 kB alpha nu / C(T_eff), so over a short
    window t, <E_int(t)> - E0 = alpha nu 2 kB (T - T0) t (1 - kappa t / 2)
    to first order.  alpha is the default (head-on transfer) share."""
    tg, t0, p, n_atoms, m_da, ccs = 500.0, 300.0, 1e5, 150, 500.0, 2e-18
    dt, steps, n = 1e-10, 2, 100_000
    f = _gas_box(p, tg)
    ion = synth.Ion(m_da, 1, ccs, n_atoms)
    op = synth.Operating(dt=dt, z_det=f.grid.L, r_det=f.grid.R, collisions_on=1)
    s = _sim(f, ion, op)
    m = m_da * DA
    rng = np.random.default_rng(21)
    e0 = O.einstein_u(t0, n_atoms)
    snap = _snap(n, 0.0, 0.0, 3e-3, 0.0, 0.0, 0.0, e_int=e0)
    snap["vx"], snap["vy"], snap["vz"] = rng.normal(0.0, math.sqrt(KB * tg / m), (3, n))
    s.write_packs(snap)
    s.step(steps)
    de = s.read_packs()["e_int"] - e0
    t = steps * dt
    mu = m * MG / (m + MG)
    nu = p / (KB * tg) * ccs * math.sqrt(8 * KB * tg / (math.pi * mu))
    alpha = _head_on_transfer(28.0134, m_da / n_atoms)
    kappa = 2 * KB * alpha * nu / _einstein_heat_capacity(t0, n_atoms)
    want = alpha * nu * 2 * KB * (tg - t0) * t * (1 - 0.5 * kappa * t)
    sem = de.std() / math.sqrt(n)
    assert abs(de.mean() - want) < 5 * sem + 0.005 * want, (de.mean() / want, sem / want)


def _mason_schamp(m_da, ccs, p, tg, charge=1):
    """Mason-Schamp first approximation for hard spheres:
    K = (3 q / 16 N) sqrt(2 pi / (mu kB T)) / sigma."""
    mu = m_da * 28.0134 / (m_da + 28.0134) * DA
    N = p / (KB * tg)
    return 3 * charge * QE / (16 * N) * math.sqrt(2 * math.pi / (mu * KB * tg)) / ccs


def _drift(p, tg, ez, dt, steps, alpha, n=2000, m_da=500.0, ccs=2e-18):
    f = _gas_box(p, tg, ez=ez, nz=256)
    ion = synth.Ion(m_da, 1, ccs, 150, alpha=alpha)
    op = synth.Operating(dt=dt, z_det=f.grid.L, r_det=f.grid.R, collisions_on=1)
    s = _sim(f, ion, op)
    s.write_packs(_snap(n, 0.0, 0.0, 2e-3, 0.0, 0.0, 0.0, e_int=O.einstein_u(300.0, 150)))
    s.step(steps // 20)
    z0 = s.read_packs()["z"].mean()
    rest = steps - steps // 20
    s.step(rest)
    z1 = s.read_packs()["z"].mean()
    return (z1 - z0) / (rest * dt)


@pytest.mark.parametrize("alpha,tol", [(0.0, 0.02), (-1.0, 0.04)])
def test_low_field_mobility(alpha, tol):
    """Drift velocity v_d = K E in the low-field limit, at a step where the
    momentum relaxation rate times dt is small (0.07)."""
    p, tg, ez, dt = 2e3, 300.0, 2e3, 2e-9
    K = _mason_schamp(500.0, 2e-18, p, tg)
    abar = math.sqrt(8 * KB * tg / (math.pi * MG))
    assert K * ez < 0.05 * abar  # low-field regime
    vd = _drift(p, tg, ez, dt, 22000, alpha)
    assert vd == pytest.approx(K * ez, rel=tol)


def test_drift_splitting_factor_at_large_collision_number():
    """At 1e5 Pa and dt = 1 ns (about 29 collisions per step) the push-then-
    collide splitting applies the field kick before the step's momentum
    relaxation exp(-nu dt); the steady drift is then K E (x/2) coth(x/2),
    x = nu dt, nu = q/(m K).  Checks the thinning process and the step order
    together, far from the small-step limit."""
    p, tg, ez, dt = 1e5, 300.0, 1e5, 1e-9
    K = _mason_schamp(500.0, 2e-18, p, tg)
    nu = QE / (500.0 * DA * K)
    x = nu * dt
    vd = _drift(p, tg, ez, dt, 2000, 0.0)
    assert vd == pytest.approx(K * ez * (x / 2) / math.tanh(x / 2), rel=0.03)


# ----------------------------------------------------------------------------
# Dissociation (Eq. 7) and tallies
# ----------------------------------------------------------------------------

def test_survival_yield_constant_temperature():
    f = synth.uniform_fields(16, 64, 5e-5)
    dH, dS = 100e3, -80.0
    ion = synth.Ion(500.0, 1, 2e-18, 150, act_kind=1, act_p1=dH, act_p2=dS)
    dt = 1e-9
    op = synth.Operating(dt=dt, z_det=f.grid.L, r_det=f.grid.R, collisions_on=0)
    s = _sim(f, ion, op)
    temps = np.array([400.0, 700.0, 1100.0])
    e = np.array([O.einstein_u(t, 150) for t in temps])
    s.write_packs(_snap(3, 0.0, 0.0, 1e-3, 0.0, 0.0, 0.0, e_int=e))
    steps = 500
    s.step(steps)
    p = s.read_packs()
    Rg = 6.02214076e23 * KB
    k = KB * temps / 6.62607015e-34 * np.exp(dS / Rg - dH / (Rg * temps))
    assert np.allclose(p["h"], k * steps * dt, rtol=1e-9)
    assert np.allclose(np.exp(-p["h"]), np.exp(-k * steps * dt), rtol=1e-9)


def test_run_is_deterministic_and_conserves_weight():
    f, ions, srcs, op, _ = synth.config_c1t(300)
    srcs[0].z_inj = 2.0e-3
    op.v_rf = 300.0
    out = []
    for _ in range(2):
        s = O.OracleSim(7)
        s.setup(f, ions, srcs, op)
        s.inject(0, 300)
        s.step(400)
        out.append((s.read_packs(), s.read_tallies()))
    (p0, t0), (p1, t1) = out
    for k in p0:
        assert np.array_equal(p0[k], p1[k]), k
    for k in t0:
        assert np.array_equal(np.asarray(t0[k]), np.asarray(t1[k])), k
    assert t0["class_w"].sum() == t0["emitted_w"] == 300 * 2 ** 32
