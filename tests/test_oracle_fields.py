"""Oracle pins: random numbers, field bake, gather, heat capacity, rates,
sine transform, Poisson solve and CIC deposit.

Every check here compares the oracle with something other than itself: an
independent library implementation, a closed form, a textbook value, an
invariant, or brute force on a tiny input.
"""
import math

import numpy as np
import pytest

from oracle import binding as O
from paper_2609_31258_amd import synth

KB, QE, EPS0, HPL = 1.380649e-23, 1.602176634e-19, 8.8541878188e-12, 6.62607015e-34


# ----------------------------------------------------------------------------
# Philox4x32-10: bit-exact against an independent implementation (the Philox
# of the Triton language, run by its CPU interpreter), plus uniformity.
# ----------------------------------------------------------------------------

def _triton_philox(ctrs: np.ndarray, seed: int) -> np.ndarray:
    import os
    os.environ["TRITON_INTERPRET"] = "1"
    torch = pytest.importorskip("torch")
    triton = pytest.importorskip("triton")
    import triton.language as tl

    @triton.jit
    def kern(out, c0p, c1p, c2p, c3p, seed, N: tl.constexpr):
        i = tl.arange(0, N)
        a, b, c, d = tl.philox(seed, tl.load(c0p + i), tl.load(c1p + i), tl.load(c2p + i), tl.load(c3p + i))
        tl.store(out + 4 * i, a)
        tl.store(out + 4 * i + 1, b)
        tl.store(out + 4 * i + 2, c)
        tl.store(out + 4 * i + 3, d)

    n = ctrs.shape[0]
    cols = [torch.from_numpy(np.ascontiguousarray(ctrs[:, k]).view(np.int32)).view(torch.uint32) for k in range(4)]
    out = torch.zeros(4 * n, dtype=torch.uint32)
    kern[(1,)](out, *cols, seed, N=n)
    return out.view(torch.int32).numpy().view(np.uint32).reshape(n, 4)


def test_philox_matches_independent_implementation():
    rng = np.random.default_rng(1)
    ctrs = rng.integers(0, 2 ** 32, size=(16, 4), dtype=np.uint64).astype(np.uint32)
    ctrs[0] = 0
    ctrs[1] = 0xFFFFFFFF
    for seed in (0, 7, 0x243F6A8885A308D3):
        ref = _triton_philox(ctrs, seed)
        key = (seed & 0xFFFFFFFF, seed >> 32)
        got = np.stack([O.philox(c, key) for c in ctrs])
        assert np.array_equal(got, ref), f"seed {seed:#x}"


def test_philox_uniformity():
    key = (7, 0)
    words = np.concatenate([O.philox((i, 3, 1 << 24, 0), key) for i in range(8192)])
    u = (words.astype(np.float64) + 0.5) / 2 ** 32
    n = u.size
    assert abs(u.mean() - 0.5) < 5 * math.sqrt(1 / 12 / n)
    assert abs(u.var() - 1 / 12) < 5 * 0.0745 / math.sqrt(n)
    counts = np.bincount((words >> 24).astype(np.int64), minlength=256)
    chi2 = ((counts - n / 256) ** 2 / (n / 256)).sum()
    assert chi2 < 255 + 6 * math.sqrt(2 * 255)
    r = np.corrcoef(u[:-1], u[1:])[0, 1]
    assert abs(r) < 5 / math.sqrt(n)


# ----------------------------------------------------------------------------
# Field bake E = -grad(phi)
# ----------------------------------------------------------------------------

def test_bake_linear_and_quadratic():
    nr, nz, dr, dz = 9, 13, 1e-4, 2.5e-4  # dr != dz catches swapped spacings
    r = np.arange(nr) * dr
    z = np.arange(nz) * dz
    Z, R = np.meshgrid(z, r, indexing="ij")
    er, ez = O.bake(-3.0 * Z + 0.0 * R, dr, dz)
    assert np.allclose(ez, 3.0, rtol=1e-12, atol=0)
    assert np.all(er == 0.0)
    er, ez = O.bake(5.0 * R, dr, dz)
    assert np.all(er[:, 0] == 0.0)  # symmetry axis
    assert np.allclose(er[:, 1:], -5.0, rtol=1e-12)
    assert np.allclose(ez, 0.0, atol=1e-15)
    # quadratics: central differences are exact at interior nodes
    er, _ = O.bake(7.0 * R ** 2, dr, dz)
    assert np.allclose(er[:, 1:-1], -14.0 * R[:, 1:-1], rtol=1e-10)
    _, ez = O.bake(-2.0 * Z ** 2, dr, dz)
    assert np.allclose(ez[1:-1, :], 4.0 * Z[1:-1, :], rtol=1e-10)


# ----------------------------------------------------------------------------
# Bilinear gather
# ----------------------------------------------------------------------------

def test_gather_bilinear_exact_and_clamped():
    nr, nz, dr, dz = 7, 11, 2e-4, 3e-4
    r = np.arange(nr) * dr
    z = np.arange(nz) * dz
    Z, R = np.meshgrid(z, r, indexing="ij")
    f = lambda rr, zz: 1.5 + 2e3 * rr - 4e3 * zz + 3e6 * rr * zz
    tab = f(R, Z)
    rng = np.random.default_rng(3)
    for _ in range(200):
        rr, zz = rng.uniform(0, r[-1]), rng.uniform(0, z[-1])
        assert O.gather(tab, dr, dz, rr, zz) == pytest.approx(f(rr, zz), rel=1e-12, abs=1e-12)
    for i in range(nr):
        for j in range(nz):
            assert O.gather(tab, dr, dz, r[i], z[j]) == pytest.approx(tab[j, i], rel=1e-13, abs=1e-13)
    # outside: constant extension from the nearest edge
    assert O.gather(tab, dr, dz, 10 * r[-1], z[3]) == pytest.approx(tab[3, -1], rel=1e-13)
    assert O.gather(tab, dr, dz, r[2], -5 * dz) == pytest.approx(tab[0, 2], rel=1e-13)


# ----------------------------------------------------------------------------
# Einstein heat capacity
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("n_atoms", [3, 64, 150, 1500])
def test_einstein_inverse_and_limits(n_atoms):
    s = 3 * n_atoms - 6
    th = 1100.0
    for t in (50.0, 300.0, 411.0, 2000.0, 1e5):
        assert O.einstein_t(O.einstein_u(t, n_atoms, th), n_atoms, th) == pytest.approx(t, rel=1e-12)
    # classical limit: U = s kB (T - theta/2 + theta^2/(12 T) - ...)
    t = 1e6
    assert O.einstein_u(t, n_atoms, th) == pytest.approx(s * KB * (t - th / 2 + th * th / (12 * t)), rel=1e-9)
    # low-temperature limit: U = s kB theta exp(-theta/T)
    t = 40.0
    assert O.einstein_u(t, n_atoms, th) == pytest.approx(s * KB * th * math.exp(-th / t), rel=1e-10)
    # heat capacity C = dU/dT positive and below the classical s kB
    c = (O.einstein_u(501.0, n_atoms, th) - O.einstein_u(499.0, n_atoms, th)) / 2.0
    assert 0 < c < s * KB


# ----------------------------------------------------------------------------
# Dissociation rates (Eq. 7)
# ----------------------------------------------------------------------------

def test_rate_eyring_textbook_and_slopes():
    # with dH = dS = 0 the Eyring rate is kB T / h = 6.2124e12 1/s at 298.15 K
    assert O.rate(1, 0.0, 0.0, 298.15) == pytest.approx(6.2124e12, rel=1e-4)
    dH, dS = 100e3, -80.0  # Rhodamine B proxy parameters of Table S3
    Rg = 6.02214076e23 * KB  # molar gas constant, exact in SI
    t1, t2 = 400.0, 800.0
    l1 = math.log(O.rate(1, dH, dS, t1) / t1)
    l2 = math.log(O.rate(1, dH, dS, t2) / t2)
    assert (l2 - l1) / (1 / t2 - 1 / t1) == pytest.approx(-dH / Rg, rel=1e-9)
    assert l1 + dH / (Rg * t1) == pytest.approx(math.log(KB / HPL) + dS / Rg, rel=1e-12)
    assert O.rate(1, dH, dS, 0.0) == 0.0
    assert O.rate(0, dH, dS, 500.0) == 0.0


def test_rate_arrhenius_slope():
    A, ea = 1e12, 1.2
    t1, t2 = 500.0, 1500.0
    slope = (math.log(O.rate(2, A, ea, t2)) - math.log(O.rate(2, A, ea, t1))) / (1 / t2 - 1 / t1)
    assert slope == pytest.approx(-ea * QE / KB, rel=1e-10)
    assert O.rate(2, A, ea, 1e9) == pytest.approx(A, rel=1e-4)


# ----------------------------------------------------------------------------
# DST-I and the Poisson solve
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("m", [1, 2, 7, 30, 62])
def test_dst1_against_library_and_involution(m):
    scipy_fft = pytest.importorskip("scipy.fft")
    x = np.random.default_rng(m).normal(size=m)
    y = O.dst1(x)
    assert np.allclose(y, scipy_fft.dst(x, type=1) / 2.0, rtol=1e-12, atol=1e-12)
    assert np.allclose(O.dst1(y) * 2.0 / (m + 1), x, rtol=1e-11, atol=1e-12)


def _fv_volumes(nr, dr, dz):
    """Finite-volume control volumes of the radial operator: disk of radius
    dr/2 on the axis, annuli of width dr elsewhere."""
    v = 2 * math.pi * np.arange(nr) * dr * dr * dz
    v[0] = math.pi * (dr / 2) ** 2 * dz
    return v


def test_poisson_gauss_law_uniform_cylinder():
    nr, nz, h = 48, 768, 5e-5  # long: L/R ~ 16, end effects ~exp(-2.4*8)
    ia = 9
    rho0 = 1e-4
    rho = np.zeros((nz, nr))
    rho[:, : ia + 1] = rho0
    phi = O.poisson(rho, h, h)
    assert O.poisson_residual(rho, phi, h, h) < 1e-11
    jm = nz // 2
    vol = _fv_volumes(nr, h, h)
    qenc = np.cumsum(rho0 * vol * (np.arange(nr) <= ia))
    for i in range(0, nr - 1):
        r_face = (i + 0.5) * h
        flux = 2 * math.pi * r_face * h * (phi[jm, i] - phi[jm, i + 1]) / h
        assert flux == pytest.approx(qenc[i] / EPS0, rel=1e-7), i
    # nodal E_r against the analytic field of a cylinder of radius (ia+1/2) h
    er, _ = O.bake(phi, h, h)
    a = (ia + 0.5) * h
    for i in (3, 6, 15, 25):
        r = i * h
        exact = rho0 * r / (2 * EPS0) if r < a else rho0 * a * a / (2 * EPS0 * r)
        assert er[jm, i] == pytest.approx(exact, rel=2e-3), i
    # symmetric charge -> potential symmetric in z
    assert np.allclose(phi, phi[::-1, :], rtol=1e-9, atol=1e-12 * np.abs(phi).max())


def test_poisson_manufactured_solution():
    nr, nz, dr, dz = 12, 20, 1e-4, 2e-4
    rng = np.random.default_rng(5)
    phi = np.zeros((nz, nr))
    phi[1:-1, :-1] = rng.normal(size=(nz - 2, nr - 1))
    # apply the finite-volume operator by brute force on each node (flux form)
    lap = np.zeros_like(phi)
    vol = _fv_volumes(nr, dr, dz)
    for j in range(1, nz - 1):
        for i in range(nr - 1):
            out = 0.0
            if i > 0:
                out += 2 * math.pi * (i - 0.5) * dr * dz * (phi[j, i - 1] - phi[j, i]) / dr
            out += 2 * math.pi * (i + 0.5) * dr * dz * (phi[j, i + 1] - phi[j, i]) / dr
            area = vol[i] / dz
            out += area * (phi[j + 1, i] - 2 * phi[j, i] + phi[j - 1, i]) / dz
            lap[j, i] = out / vol[i]
    rho = -EPS0 * lap
    got = O.poisson(rho, dr, dz)
    assert np.allclose(got, phi, rtol=1e-9, atol=1e-9 * np.abs(phi).max())


# ----------------------------------------------------------------------------
# Deposit and charge density
# ----------------------------------------------------------------------------

def _charge_sim(snap, nr=24, nz=40, h=5e-5, charge=3):
    f = synth.uniform_fields(nr, nz, h)
    s = O.OracleSim(7)
    s.setup(f, [synth.Ion(500.0, charge, 2e-18, 150)], [], synth.Operating(dt=1e-9, z_det=f.grid.L,
                                                                           r_det=f.grid.R, collisions_on=0))
    s.write_packs(snap)
    s.pic_update()
    return s, f


def _snap(x, y, z, w):
    n = len(x)
    return dict(x=np.asarray(x, float), y=np.asarray(y, float), z=np.asarray(z, float), vx=np.zeros(n),
                vy=np.zeros(n), vz=np.zeros(n), e_int=np.full(n, 1e-19), h=np.zeros(n), w=np.asarray(w, float),
                id=np.arange(n, dtype=np.int64), tag=np.zeros(n, np.int32))


def test_deposit_exact_total_and_moments():
    rng = np.random.default_rng(11)
    n = 5000
    h = 5e-5
    r = rng.uniform(0, 20 * h, n)
    ph = rng.uniform(0, 2 * math.pi, n)
    z = rng.uniform(0, 35 * h, n)
    w = rng.uniform(0.01, 3.0, n)
    s, f = _charge_sim(_snap(r * np.cos(ph), r * np.sin(ph), z, w))
    q = s.read_charge()
    p = s.read_packs()
    assert q.sum() == p["q"].sum()  # exact
    assert np.all(p["q"] == np.array([round(3 * wi * 2 ** 32) for wi in w]))
    # first moments: linear weights reproduce the pack position (to rounding of the split)
    one = _snap([3.3 * h], [0.0], [7.6 * h], [1.0])
    s1, _ = _charge_sim(one)
    q1 = s1.read_charge()
    ri = np.arange(f.grid.nr) * h
    zj = np.arange(f.grid.nz) * h
    Q = q1.sum()
    assert (q1 * ri[None, :]).sum() / Q == pytest.approx(3.3 * h, rel=1e-9)
    assert (q1 * zj[:, None]).sum() / Q == pytest.approx(7.6 * h, rel=1e-9)
    assert np.count_nonzero(q1) == 4


def test_deposit_pack_on_node():
    h = 5e-5
    s, _ = _charge_sim(_snap([0.0, 4 * h], [0.0, 0.0], [0.0, 9 * h], [1.0, 2.0]))
    q = s.read_charge()
    assert q[0, 0] == round(3 * 2 ** 32) and q[9, 4] == round(6 * 2 ** 32)
    assert np.count_nonzero(q) == 2


def test_rho_from_uniform_density():
    """Packs uniform in a cylinder volume: the CIC charge of each off-axis
    node over its annular control volume 2 pi r_i dr dz (which is also the
    volume its CIC weight covers) is the true density.  On the axis the
    control volume is the disk pi (dr/2)^2 dz while the CIC weight covers
    pi dr^2 dz / 3, so that node reads 4/3 of the density."""
    h = 5e-5
    nr, nz = 24, 40
    rng = np.random.default_rng(4)
    n = 2_000_000
    rmax, z0, z1 = 15 * h, 5 * h, 30 * h
    r = rmax * np.sqrt(rng.uniform(0, 1, n))
    ph = rng.uniform(0, 2 * math.pi, n)
    z = rng.uniform(z0, z1, n)
    s, f = _charge_sim(_snap(r * np.cos(ph), r * np.sin(ph), z, np.ones(n)), nr=nr, nz=nz, charge=1)
    rho = O.rho_from_charge(s.read_charge(), h, h)
    true = n * QE / (math.pi * rmax ** 2 * (z1 - z0))
    j0, j1, imax = 7, 28, 12
    est = rho[j0:j1, :imax].mean(axis=0) / true
    vhat = np.array([math.pi * h ** 3 / 3] + [2 * math.pi * i * h ** 3 for i in range(1, imax)])
    per_node = n * vhat / (math.pi * rmax ** 2 * (z1 - z0)) * (j1 - j0)
    sd = 1.0 / np.sqrt(per_node)
    expect = np.ones(imax)
    expect[0] = 4.0 / 3.0
    assert np.all(np.abs(est - expect) < 5 * sd * expect + 1e-3), (est, sd)


def test_deposited_charge_gauss_flux_through_first_faces():
    """Deposit, solve and field as one chain: packs on every interior row of a
    long grid (L/R ~ 16, end effects ~exp(-2.4 * 8)) at r = 0.3 dr and 2.6 dr,
    CIC-deposited, divided by the control volumes and solved.  In the middle
    row the potential no longer varies along z, so the discrete Gauss law
    holds face by face: the flux 2 pi r_{i+1/2} dz (Phi_i - Phi_{i+1}) / dr
    through the cylinder face r_{i+1/2} equals the deposited charge of the
    row's nodes 0..i over eps0 -- the axis node's charge in full."""
    nr, nz, h = 48, 768, 5e-5
    rows = np.arange(1, nz - 1, dtype=float)
    rad = np.concatenate([np.full(rows.size, 0.3 * h), np.full(rows.size, 2.6 * h)])
    zz = np.concatenate([rows, rows]) * h
    ph = np.linspace(0.0, 2 * math.pi, rad.size, endpoint=False)
    s, f = _charge_sim(_snap(rad * np.cos(ph), rad * np.sin(ph), zz, np.full(rad.size, 1000.0)), nr=nr, nz=nz,
                       charge=1)
    q = s.read_charge()
    phi, _, _ = s.read_sc()
    jm = nz // 2
    assert q[jm, 0] > 0 and q[jm, 1] > 0 and q[jm, 2] > 0 and q[jm, 3] > 0 and np.all(q[jm, 4:] == 0)
    qenc = np.cumsum(q[jm].astype(float)) * QE * 2.0 ** -32
    for i in range(0, 8):
        flux = 2 * math.pi * (i + 0.5) * h * h * (phi[jm, i] - phi[jm, i + 1]) / h
        assert flux == pytest.approx(qenc[i] / EPS0, rel=1e-7), i


