"""Seeded synthetic inputs for the ion-pack propagation path.

This module builds the *inputs* of a run -- field tables, ion templates,
source definitions, operating conditions, pack snapshots and serving
queries -- and nothing else.  It contains none of the method's arithmetic
(no field bake, gather, push, collision, deposit or Poisson step): both the
HIP library and the CPU oracle receive the same arrays and parameters from
here and compute everything else with their own code.

The paper's production fields (SIMION potential arrays, Fluent CFD exports,
electrode geometry) are not available, so a synthetic generator stands in:
an axisymmetric (r, z) node grid with a linear DC ramp plus eight Gaussian
ring bumps, an RF basis that is +/-1 V at alternating rings (the RF basis
convention of the paper's field section, Eq. 4), an exponentially decaying
gas pressure and axial gas velocity, and an eight-ring electrode mask.

Array layout: every table is a C-contiguous float64 (or uint8 for the mask)
array of shape (nz, nr): element [j, i] is node (r_i = i*dr, z_j = j*dz).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

# Physical constants (exact SI definitions; CODATA 2022 for Da and eps0).
K_B = 1.380649e-23
E_CHARGE = 1.602176634e-19
DALTON = 1.66053906892e-27
M_N2_DA = 28.0134

SEED = 7  # the paper's production random seed (Table S2)


@dataclasses.dataclass
class Grid:
    nr: int
    nz: int
    dr: float
    dz: float

    @property
    def R(self) -> float:
        return (self.nr - 1) * self.dr

    @property
    def L(self) -> float:
        return (self.nz - 1) * self.dz


@dataclasses.dataclass
class Ion:
    """Ion template (the paper's ion template: mass, charge, CCS, atom count,
    heat-capacity profile and activation parameters)."""
    mass_da: float
    charge_z: int
    ccs_m2: float
    n_atoms: int
    theta_e: float = 1100.0        # Einstein temperature of the heat-capacity profile [K]
    alpha: float = -1.0            # internal-exchange probability; <0 selects the default
    t_eff0: float = 300.0          # initial effective temperature [K] (Table S3)
    act_kind: int = 0              # 0 none, 1 Eyring (dH J/mol, dS J/mol/K), 2 Arrhenius (A 1/s, Ea eV)
    act_p1: float = 0.0
    act_p2: float = 0.0


@dataclasses.dataclass
class Source:
    """Source definition (current, spatial profile, injection plane)."""
    kind: int                      # 0 burst (explicit inject), 1 fixed packs per step, 2 current accumulator (Eq. 5)
    ion: int = 0
    current_a: float = 0.0
    weight: float = 1.0            # burst / accumulator: target pack weight (real ions per pack)
    packs_per_step: int = 0
    n_total: int = 0
    sigma_r: float = 1e-4
    r_trunc: float = 3e-4
    z_inj: float = 0.0
    step_start: int = 0


@dataclasses.dataclass
class Operating:
    dt: float
    v_rf: float = 0.0
    f_rf: float = 1e6
    phase_rf: float = 0.0
    v_off: float = 0.0
    gas_mass_da: float = M_N2_DA
    collisions_on: int = 1
    sc_on: int = 0
    sc_every: int = 10
    z_det: float = 0.0
    r_det: float = 0.0
    d_hit: float = 1e-5
    exit_bin_dt: float = 1e-7
    n_exit_bins: int = 1000
    langevin_on: int = 0          # hybrid Langevin branch
    lv_z_lo: float = 0.0          # axial window [lv_z_lo, lv_z_hi); none when lv_z_hi <= lv_z_lo
    lv_z_hi: float = 0.0
    lv_switch: float = 0.05       # switch when lambda dt >= lv_switch
    sc_mask: int = 0              # space charge: Phi = 0 on the metal-mask nodes
    sample_every: int = 0         # trajectory samples every sample_every steps (0 = off)
    sample_stride: int = 0        # ... of the packs whose id is a multiple of sample_stride
    adaptive: int = 0             # Eq. 1 adaptive step (dt is then the largest step)
    lv_dt_max: float = 0.0        # adaptive: step cap while any pack is on the Langevin branch
    sort_every: int = 0           # reorder the slots by species and cell every sort_every steps (0 = never)


@dataclasses.dataclass
class Fields:
    grid: Grid
    phi_dc: np.ndarray
    phi_off: np.ndarray
    phi_rf: np.ndarray
    gas_ur: np.ndarray
    gas_uz: np.ndarray
    gas_p: np.ndarray
    gas_t: np.ndarray
    mask: np.ndarray


def _smoothstep(x: np.ndarray, a: float, b: float) -> np.ndarray:
    t = np.clip((x - a) / (b - a), 0.0, 1.0)
    return t * t * (3.0 - 2.0 * t)


def ring_fields(nr: int, nz: int, h: float = 5e-5, *, p0: float = 1e5, p1: float = 200.0,
                r_in: Optional[float] = None, u0: float = 300.0, t_gas: float = 300.0,
                v_ramp: float = -50.0, v_bump: float = 20.0, sigma_bump: float = 3e-4,
                n_rings: int = 8) -> Fields:
    """Ring-electrode field set on an (nr x nz) node grid of spacing h.

    DC potential: linear ramp 0 -> v_ramp along z plus n_rings Gaussian ring
    bumps of alternating sign (+/- v_bump, sigma 0.3 mm) centred on the ring
    inner radius; RF basis: the same bumps with unit alternating amplitude;
    DC-offset basis: a smoothstep from 0 to 1 V over z in [0.85 L, 0.95 L];
    gas: p(z) = p0 (p1/p0)^(z/L), u_z = u0 exp(-4 z / L), u_r = 0, T = t_gas;
    mask: rings of radial extent [r_in, r_in + 0.5 mm] and half-length 0.25 mm.
    """
    g = Grid(nr, nz, h, h)
    R, L = g.R, g.L
    if r_in is None:
        r_in = R / 4.0
    r = np.arange(nr, dtype=np.float64) * h
    z = np.arange(nz, dtype=np.float64) * h
    Z, Rr = np.meshgrid(z, r, indexing="ij")  # shape (nz, nr)
    phi_dc = v_ramp * Z / L
    phi_rf = np.zeros_like(Z)
    mask = np.zeros((nz, nr), dtype=np.uint8)
    for k in range(n_rings):
        zk = L * (k + 1) / (n_rings + 1)
        bump = np.exp(-((Rr - r_in) ** 2 + (Z - zk) ** 2) / (2.0 * sigma_bump ** 2))
        sign = 1.0 if k % 2 == 0 else -1.0
        phi_dc = phi_dc + sign * v_bump * bump
        phi_rf = phi_rf + sign * bump
        ring = (Rr >= r_in - 1e-12) & (Rr <= r_in + 5e-4 + 1e-12) & (np.abs(Z - zk) <= 2.5e-4 + 1e-12)
        mask[ring] = 1
    phi_off = _smoothstep(Z, 0.85 * L, 0.95 * L)
    gas_p = p0 * (p1 / p0) ** (Z / L)
    gas_uz = u0 * np.exp(-Z / (L / 4.0))
    gas_ur = np.zeros_like(Z)
    gas_t = np.full_like(Z, t_gas)
    c = np.ascontiguousarray
    return Fields(g, c(phi_dc), c(phi_off), c(phi_rf), c(gas_ur), c(gas_uz), c(gas_p), c(gas_t), c(mask))


def uniform_fields(nr: int, nz: int, h: float, *, ez: float = 0.0, p: float = 0.0, t_gas: float = 300.0,
                   uz: float = 0.0, ur: float = 0.0, rf_ez: float = 0.0) -> Fields:
    """Closed-form test fields: phi_dc = -ez * z (uniform axial field ez),
    RF basis phi_rf = -rf_ez * z, uniform gas (p, T, u), no electrodes."""
    g = Grid(nr, nz, h, h)
    z = np.arange(nz, dtype=np.float64) * h
    Z = np.repeat(z[:, None], nr, axis=1)
    full = lambda v: np.full((nz, nr), float(v))
    c = np.ascontiguousarray
    return Fields(g, c(-ez * Z), c(np.zeros((nz, nr))), c(-rf_ez * Z), c(full(ur)), c(full(uz)),
                  c(full(p)), c(full(t_gas)), c(np.zeros((nz, nr), dtype=np.uint8)))


# ---------------------------------------------------------------------------
# Workload configurations.  Each returns (fields, [ions], [sources], operating).
# ---------------------------------------------------------------------------

def _n_atoms_from_mass(m_da: float) -> int:
    return int(round(0.3 * m_da))


def config_c1(n_packs: int = 10_000):
    """Plain FP64, CPU-sized: 128x512 grid (0.05 mm), 1e4 packs of m=500 Da,
    z=+1, CCS 200 A^2, 150 atoms, N2 gas; Gaussian injection (sigma 0.1 mm)
    at z=0 with thermal velocities; dt = 1 ns, 2000 steps, collisions on,
    space charge off."""
    f = ring_fields(128, 512)
    ion = Ion(500.0, 1, 200e-20, 150, act_kind=1, act_p1=100e3, act_p2=-80.0)
    src = Source(kind=0, ion=0, weight=1.0, n_total=n_packs, sigma_r=1e-4, r_trunc=3e-4, z_inj=0.0)
    op = Operating(dt=1e-9, v_rf=100.0, f_rf=1e6, z_det=f.grid.L, r_det=f.grid.R, sc_on=0,
                   exit_bin_dt=1e-7, n_exit_bins=1000)
    return f, [ion], [src], op, {"steps": 2000, "burst": n_packs}


def config_c1t(n_packs: int = 10_000):
    """Low-pressure variant of C1 that transmits and loses packs: pressure
    1000 -> 20 Pa, ring inner radius 0.25 mm (parity of transmission and
    loss maps)."""
    f = ring_fields(128, 512, p0=1000.0, p1=20.0, r_in=2.5e-4)
    ion = Ion(500.0, 1, 200e-20, 150, act_kind=1, act_p1=100e3, act_p2=-80.0)
    src = Source(kind=0, ion=0, weight=1.0, n_total=n_packs, sigma_r=1e-4, r_trunc=3e-4, z_inj=0.0)
    op = Operating(dt=1e-9, v_rf=100.0, f_rf=1e6, z_det=f.grid.L, r_det=f.grid.R, sc_on=0,
                   exit_bin_dt=1e-6, n_exit_bins=1000)
    return f, [ion], [src], op, {"steps": 100_000, "burst": n_packs}


def config_c1x(n_transmit: int = 16_000, n_ring: int = 8_000):
    """Terminal-event variant of the low-pressure fields (1000 -> 20 Pa, ring
    inner radius 0.25 mm) on a narrow 20 x 512 grid (R = 0.95 mm), built so
    that every terminal class occurs within about 1000 steps: a burst
    source 1.5 mm before the detector plane (packs cross it within the
    detector radius of 0.3 mm -> transmitted, outside it -> axial, or leave
    through r = R -> radial) and a burst source between the last two rings
    (electrode hits on the last ring).  Ion: 500 Da, z = +1, 200 A^2,
    150 atoms, Arrhenius dissociation with A = 1e12 1/s and Ea = 0.42 eV
    (about 1e5 1/s at 300 K, so survival yields are well inside (0, 1));
    RF 100 V at 1 MHz; dt = 5 ns (lambda dt <= 0.05)."""
    f = ring_fields(20, 512, p0=1000.0, p1=20.0, r_in=2.5e-4)
    ion = Ion(500.0, 1, 200e-20, 150, act_kind=2, act_p1=1e12, act_p2=0.42)
    srcs = [Source(kind=0, ion=0, weight=1.0, n_total=n_transmit, sigma_r=3e-4, r_trunc=9e-4, z_inj=24.0e-3),
            Source(kind=0, ion=0, weight=0.5, n_total=n_ring, sigma_r=3e-4, r_trunc=9e-4, z_inj=21.3e-3)]
    op = Operating(dt=5e-9, v_rf=100.0, f_rf=1e6, z_det=f.grid.L, r_det=3e-4, sc_on=0,
                   exit_bin_dt=1e-7, n_exit_bins=100)
    return f, [ion], srcs, op, {"steps": 1200, "bursts": [n_transmit, n_ring]}


def config_c2(n_packs: int = 1_000_000, packs_per_step: int = 500, current_a: float = 10e-9):
    """256x1024 grid with space charge: packs injected continuously at
    packs_per_step, weighted to a 10 nA current; m = 5000 Da, z = +5,
    CCS 1500 A^2; CIC deposit + Poisson every 10 steps; dt = 0.5 ns,
    2e4 steps."""
    f = ring_fields(256, 1024)
    m = 5000.0
    ion = Ion(m, 5, 1500e-20, _n_atoms_from_mass(m), act_kind=1, act_p1=100e3, act_p2=-80.0)
    src = Source(kind=1, ion=0, current_a=current_a, packs_per_step=packs_per_step, n_total=n_packs,
                 sigma_r=1e-4, r_trunc=3e-4, z_inj=0.0)
    op = Operating(dt=0.5e-9, v_rf=100.0, f_rf=1e6, z_det=f.grid.L, r_det=f.grid.R, sc_on=1, sc_every=10,
                   exit_bin_dt=1e-7, n_exit_bins=1000)
    return f, [ion], [src], op, {"steps": 20_000}


def config_c5_species(n_species: int = 10):
    """Ten species for the large configuration: masses log-spaced 200 -> 5e4 Da,
    atoms log-spaced 100 -> 5000, charge round(1 + 24 k / 9), CCS scaled as
    m^(2/3), Arrhenius activation with A = 1e12 1/s and Ea 0.8 -> 1.6 eV."""
    ions = []
    for k in range(n_species):
        t = k / max(n_species - 1, 1)
        m = 200.0 * (5e4 / 200.0) ** t
        na = int(round(100.0 * (5000.0 / 100.0) ** t))
        zq = int(round(1 + 24 * k / 9))
        ccs = 200e-20 * (m / 500.0) ** (2.0 / 3.0)
        ea = 0.8 + 0.8 * t
        ions.append(Ion(m, zq, ccs, na, act_kind=2, act_p1=1e12, act_p2=ea))
    return ions


def config_c5(n_packs: int = 16_000_000, emit_steps: int = 10_000, current_a: float = 50e-9,
              nr: int = 1024, nz: int = 8192):
    """Large: 1024x8192 grid (0.05 mm), ten species sharing the packs and the
    current equally (5 nA each), each emitted at n_packs / (10 emit_steps)
    packs per step over the first emit_steps steps; Einstein heat capacity
    and Arrhenius dissociation per species; space charge every 5 steps;
    dt = 0.25 ns, 1e5 steps; run in the FP32 precision form."""
    f = ring_fields(nr, nz)
    ions = config_c5_species(10)
    per = n_packs // len(ions)
    srcs = [Source(kind=1, ion=k, current_a=current_a / len(ions), packs_per_step=max(1, per // emit_steps),
                   n_total=per, sigma_r=1e-4, r_trunc=3e-4, z_inj=0.0) for k in range(len(ions))]
    op = Operating(dt=0.25e-9, v_rf=100.0, f_rf=1e6, z_det=f.grid.L, r_det=f.grid.R, sc_on=1, sc_every=5,
                   exit_bin_dt=1e-7, n_exit_bins=1000)
    return f, ions, srcs, op, {"steps": 100_000, "emit_steps": emit_steps}


def config_c5_pack_weights(ions, srcs, op) -> List[float]:
    """Each species' pack weight in the large configuration: its share of the
    current over its packs per step (ions per pack)."""
    return [src.current_a * op.dt / (ion.charge_z * E_CHARGE) / src.packs_per_step for src, ion in zip(srcs, ions)]


def c5_post_ramp_snapshot(f: Fields, ions, weights, n: int, seed: int = SEED) -> Dict[str, np.ndarray]:
    """The large configuration's packs after its emission ramp, as a seeded
    snapshot: the ten species in equal shares (round robin), positions within
    3 mm of the injection plane and 0.3 mm of the axis, velocities thermal
    about the gas flow, internal energies of an Einstein solid at 300-1500 K."""
    snap = pack_snapshot(n, f, seed=seed, z_hi=3e-3, r_hi=3e-4, v_sigma=50.0, v_drift=300.0)
    tag = (np.arange(n) % len(ions)).astype(np.int32)
    snap["tag"] = tag
    snap["w"] = np.asarray(weights, dtype=np.float64)[tag]
    dof = np.array([3 * i.n_atoms - 6 for i in ions], dtype=np.float64)[tag]
    snap["e_int"] = dof * K_B * 300.0 * np.random.default_rng(seed + 1).uniform(0.3, 1.5, n)
    return snap


def serving_queries(n_queries: int = 256, rate_hz: float = 20.0, seed: int = SEED,
                    pack_lo: float = 1e3, pack_hi: float = 1e6) -> List[Dict]:
    """Design queries with Poisson arrivals: RF amplitude U(50, 300) V, DC
    offset U(-80, 0) V, current log-U(0.1, 20) nA, pack count log-U, ion
    mass log-U(200, 5e4) Da, charge U{1..25}, CCS = 200 A^2 (m/500)^(2/3)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=n_queries)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for q in range(n_queries):
        m = float(np.exp(rng.uniform(math.log(200.0), math.log(5e4))))
        out.append(dict(
            arrival_s=float(t[q]),
            v_rf=float(rng.uniform(50.0, 300.0)),
            v_off=float(rng.uniform(-80.0, 0.0)),
            current_a=float(np.exp(rng.uniform(math.log(0.1e-9), math.log(20e-9)))),
            n_packs=int(round(np.exp(rng.uniform(math.log(pack_lo), math.log(pack_hi))))),
            mass_da=m,
            charge_z=int(rng.integers(1, 26)),
            ccs_m2=200e-20 * (m / 500.0) ** (2.0 / 3.0),
            n_atoms=_n_atoms_from_mass(m),
            seed=int(rng.integers(1, 2 ** 62)),
        ))
    return out


def pack_snapshot(n: int, fields: Fields, *, seed: int = SEED, z_lo: float = 0.0, z_hi: Optional[float] = None,
                  r_hi: Optional[float] = None, v_sigma: float = 200.0, v_drift: float = 300.0,
                  e_lo: float = 1e-19, e_hi: float = 6e-19, weight: float = 1.0, ion: int = 0) -> Dict[str, np.ndarray]:
    """A synthetic population of active packs for single-step parity:
    positions uniform in a sub-volume of the grid, velocities Gaussian about
    an axial drift, internal energies uniform in [e_lo, e_hi] J."""
    g = fields.grid
    rng = np.random.default_rng(seed)
    z_hi = g.L * 0.9 if z_hi is None else z_hi
    r_hi = g.R * 0.9 if r_hi is None else r_hi
    r = r_hi * np.sqrt(rng.uniform(0.0, 1.0, n))
    ph = rng.uniform(0.0, 2 * math.pi, n)
    snap = dict(
        x=r * np.cos(ph), y=r * np.sin(ph), z=rng.uniform(z_lo, z_hi, n),
        vx=rng.normal(0.0, v_sigma, n), vy=rng.normal(0.0, v_sigma, n), vz=v_drift + rng.normal(0.0, v_sigma, n),
        e_int=rng.uniform(e_lo, e_hi, n), h=np.zeros(n), w=np.full(n, float(weight)),
        id=np.arange(n, dtype=np.int64), tag=np.full(n, ion, dtype=np.int32),
    )
    return {k: np.ascontiguousarray(v) for k, v in snap.items()}
