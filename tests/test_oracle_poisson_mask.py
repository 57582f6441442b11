"""Oracle pins for the Poisson solve with the metal-mask Dirichlet condition
(space-charge section: zero perturbation potential on metal-mask nodes).

The masked solver (preconditioned conjugate gradients on the symmetric form
of the finite-volume operator) is pinned against the mask-free direct solver
where the two problems coincide, against the direct solver on two separate
boxes when the mask fills a whole z-plane, by its own residual, and by the
discrete maximum principle."""
import numpy as np
import pytest

from oracle import binding as O
from paper_2609_31258_amd import synth

EPS0 = 8.8541878188e-12


def _rho(nr, nz, seed, lo=0.0):
    rng = np.random.default_rng(seed)
    rho = np.zeros((nz, nr))
    # a few Gaussian blobs of positive charge density [C/m^3]
    r = np.arange(nr)[None, :]
    z = np.arange(nz)[:, None]
    for _ in range(4):
        i0, j0 = rng.uniform(0, nr * 0.6), rng.uniform(nz * 0.1, nz * 0.9)
        rho += 1e-6 * np.exp(-((r - i0) ** 2 + (z - j0) ** 2) / (2 * rng.uniform(2, 6) ** 2))
    return rho + lo


def _masked_residual(rho, phi, mask, dr, dz):
    """max |L phi + rho/eps0| over the non-mask unknowns / max |rho/eps0|."""
    nz, nr = rho.shape
    i = np.arange(nr, dtype=np.float64)
    pj = phi[1:-1]
    ar = np.empty((nz - 2, nr - 1))
    ar[:, 0] = 4.0 * (pj[:, 1] - pj[:, 0]) / dr ** 2
    ri = i[1:nr - 1] * dr
    ar[:, 1:] = ((ri + 0.5 * dr) * (pj[:, 2:] - pj[:, 1:-1]) - (ri - 0.5 * dr) * (pj[:, 1:-1] - pj[:, :-2])) / (
        ri * dr * dr)
    az = (phi[2:, :nr - 1] - 2.0 * phi[1:-1, :nr - 1] + phi[:-2, :nr - 1]) / dz ** 2
    b = -rho[1:-1, :nr - 1] / EPS0
    free = mask[1:-1, :nr - 1] == 0
    return np.abs((ar + az - b)[free]).max() / np.abs(b).max()


def test_empty_mask_reproduces_the_direct_solver():
    nr, nz, h = 48, 160, 5e-5
    rho = _rho(nr, nz, 1)
    ref = O.poisson(rho, h, h)
    phi, it = O.poisson_masked(rho, np.zeros((nz, nr), np.uint8), h, h)
    assert 0 < it <= 3
    assert np.abs(phi - ref).max() <= 1e-11 * np.abs(ref).max()


def test_ring_mask_dirichlet_and_residual():
    f = synth.ring_fields(64, 256)
    g = f.grid
    rho = _rho(g.nr, g.nz, 2)
    phi, it = O.poisson_masked(rho, f.mask, g.dr, g.dz)
    assert 0 < it < 300
    m = f.mask.astype(bool)
    assert m.sum() > 100
    assert np.all(phi[m] == 0.0)
    assert _masked_residual(rho, phi, f.mask, g.dr, g.dz) <= 1e-9
    # the conductors change the potential: images of the charge
    ref = O.poisson(rho, g.dr, g.dz)
    assert np.abs(phi - ref).max() > 1e-3 * np.abs(ref).max()


def test_full_plane_mask_splits_into_two_boxes():
    nr, nz, h, j0 = 40, 200, 5e-5, 83
    rho = _rho(nr, nz, 3)
    mask = np.zeros((nz, nr), np.uint8)
    mask[j0, :] = 1
    phi, it = O.poisson_masked(rho, mask, h, h)
    assert it > 0
    lo = O.poisson(np.ascontiguousarray(rho[: j0 + 1]), h, h)
    hi = O.poisson(np.ascontiguousarray(rho[j0:]), h, h)
    s = np.abs(phi).max()
    assert np.abs(phi[: j0 + 1] - lo).max() <= 1e-10 * s
    assert np.abs(phi[j0:] - hi).max() <= 1e-10 * s


def test_grounded_conductors_lower_the_potential_of_positive_charge():
    f = synth.ring_fields(64, 256)
    g = f.grid
    rho = _rho(g.nr, g.nz, 4)
    free = O.poisson(rho, g.dr, g.dz)
    phi, _ = O.poisson_masked(rho, f.mask, g.dr, g.dz)
    s = np.abs(free).max()
    assert phi.min() >= -1e-12 * s
    assert np.all(phi <= free + 1e-12 * s)


def test_simulation_pic_update_uses_the_mask():
    f, ions, _, op, _ = synth.config_c1(1000)
    op.sc_on, op.sc_mask = 1, 1
    s = O.OracleSim(7)
    s.setup(f, ions, [], op)
    snap = synth.pack_snapshot(20000, f, seed=5, z_lo=1e-3, z_hi=f.grid.L * 0.8, r_hi=f.grid.R * 0.8, weight=50.0)
    s.write_packs(snap)
    s.pic_update()
    phi, er, ez = s.read_sc()
    assert np.abs(phi).max() > 0 and np.all(phi[f.mask.astype(bool)] == 0.0)
    g = f.grid
    q = s.read_charge()
    i = np.arange(g.nr)
    rho = O.rho_from_charge(q, g.dr, g.dz)
    assert _masked_residual(rho, phi, f.mask, g.dr, g.dz) <= 1e-9
