"""Mutation checks of the oracle's pins (CPU).  Each case plants one plausible
mistake in a copy of the oracle's source, builds the copy and runs the pins
that should catch it against that build (in a child process, through the
binding's MC_ORACLE_LIB); the pins must fail.  A mistake no pin catches would
go unnoticed in the parity tests as well, since the GPU path is compared with
the oracle.

Mistakes:
  - internal-energy exchange selected by the acceptance uniform itself instead
    of the acceptance residual u (s + |w|) / |g| (uniform given acceptance);
  - the default exchange share 2 instead of 4 mg ma / (mg + ma)^2;
  - the axis control volume pi dr^2 dz / 3 (the area its CIC weight covers)
    instead of the finite-volume disk pi (dr/2)^2 dz;
  - a dropped factor 2 in the internal-energy heating (the relative energy
    redrawn from Gamma(1) instead of Gamma(2), one logarithm instead of two);
  - Langevin branch: the friction prefactor 8/3 instead of 16/3; the variance
    1 - f instead of 1 - f^2; a Box-Muller radius without its factor 2; the
    second normal drawn from the third word's angle (correlated normals); the
    hazard accumulated in an aggregated step;
  - adaptive step (Eq. 1): the CFL limit a full spacing instead of half; the
    acceleration limit without the thermal speed; the collision limit 1/lambda
    instead of 0.1/lambda; the RF limit a tenth of a period instead of a
    twentieth; no stop at the next space-charge update;
  - masked Poisson solve: the lower axial neighbour taken from the radial
    row (o - 1 for o - nr); a preconditioner that does not vanish on the mask.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "mc_oracle.c")

MUTANTS = {
    "exchange_select_by_acceptance_uniform": (
        "double ui[5] = {u01(wc[0]), u01(wc[1]), uacc * (s + wn) / gn, u01(wc[2]), u01(wc[3])};",
        "double ui[5] = {u01(wc[0]), u01(wc[1]), uacc, u01(wc[2]), u01(wc[3])};",
        ["tests/test_oracle_dynamics.py::test_exchange_fraction_per_accepted_collision"]),
    "default_share_halved": (
        "4.0 * mg * ma / ((mg + ma) * (mg + ma))",
        "2.0 * mg * ma / ((mg + ma) * (mg + ma))",
        ["tests/test_oracle_dynamics.py::test_exchange_fraction_per_accepted_collision"]),
    "axis_volume_of_the_cic_weight": (
        "double v = (i == 0) ? PI * (0.5 * dr) * (0.5 * dr) * dz : 2.0 * PI * (i * dr) * dr * dz;",
        "double v = (i == 0) ? PI * dr * dr * dz / 3.0 : 2.0 * PI * (i * dr) * dr * dz;",
        ["tests/test_oracle_fields.py::test_deposited_charge_gauss_flux_through_first_faces"]),
    "bath_energy_gamma1": (
        "etp = -KB * t_eff * log(u[3] * u[4]);",
        "etp = -KB * t_eff * log(u[3]);",
        ["tests/test_oracle_dynamics.py::test_internal_energy_relaxation_rate",
         "tests/test_oracle_dynamics.py::test_thermalisation_to_gas_temperature"]),
    "langevin_friction_prefactor": (
        "return (16.0 / 3.0) * n_sigma * sqrt(",
        "return (8.0 / 3.0) * n_sigma * sqrt(",
        ["tests/test_oracle_langevin.py"]),
    "langevin_variance_form": (
        "double sd = sqrt((KB * t_gas / m) * (1.0 - f * f));",
        "double sd = sqrt((KB * t_gas / m) * (1.0 - f));",
        ["tests/test_oracle_langevin.py"]),
    "langevin_box_muller_radius": (
        "double r0 = sqrt(-2.0 * log(u01(w[0]))), r1 = sqrt(-2.0 * log(u01(w[2])));",
        "double r0 = sqrt(-log(u01(w[0]))), r1 = sqrt(-2.0 * log(u01(w[2])));",
        ["tests/test_oracle_langevin.py"]),
    "langevin_angle_word": (
        "xi[1] = r0 * sin(2.0 * PI * u01(w[1]));",
        "xi[1] = r0 * sin(2.0 * PI * u01(w[3]));",
        ["tests/test_oracle_langevin.py"]),
    "langevin_hazard_not_frozen": (
        "if (lv) return; /* no T_eff or hazard update in an aggregated step */",
        "/* (hazard accumulated in every step) */",
        ["tests/test_oracle_langevin.py"]),
    "adaptive_cfl_full_spacing": (
        "if (vn > 0.0) lim = fmin(lim, 0.5 * fmin(s->dr, s->dz) / vn);",
        "if (vn > 0.0) lim = fmin(lim, fmin(s->dr, s->dz) / vn);",
        ["tests/test_oracle_adaptive.py"]),
    "adaptive_acceleration_without_thermal_speed": (
        "0.1 * (sv + vth) / an",
        "0.1 * sv / an",
        ["tests/test_oracle_adaptive.py"]),
    "adaptive_collision_limit": (
        "else if (lam > 0.0) lim = fmin(lim, 0.1 / lam);",
        "else if (lam > 0.0) lim = fmin(lim, 1.0 / lam);",
        ["tests/test_oracle_adaptive.py"]),
    "adaptive_rf_tenth": (
        "dt = fmin(dt, 0.05 / s->op.f_rf);",
        "dt = fmin(dt, 0.1 / s->op.f_rf);",
        ["tests/test_oracle_adaptive.py"]),
    "adaptive_no_stop_at_space_charge": (
        "if (s->op.sc_on) dt = fmin(dt, s->t_next_pic - t0);",
        "/* (no stop at the next space-charge update) */",
        ["tests/test_oracle_adaptive.py"]),
    "masked_wrong_axial_neighbour": (
        "double az = (x[o + nr] - 2.0 * p[i] + x[o - nr]) / (dz * dz);",
        "double az = (x[o + nr] - 2.0 * p[i] + x[o - 1]) / (dz * dz);",
        ["tests/test_oracle_poisson_mask.py"]),
    "masked_preconditioner_not_on_subspace": (
        "        if (mask[o]) z[o] = 0.0;\n}",
        "        (void)0;\n}",
        ["tests/test_oracle_poisson_mask.py"]),
}


def _build(tmp, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"{name}: the text to mutate is not in the oracle exactly once"
    path = os.path.join(tmp, f"mc_oracle_{name}.c")
    open(path, "w").write(src.replace(old, new))
    lib = os.path.join(tmp, f"libmc_oracle_{name}.so")
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c11", "-shared", "-fPIC",
                    "-I" + os.path.dirname(SRC),
                    "-o", lib, path, "-lm"], check=True)
    return lib


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_its_pins(tmp_path, name):
    old, new, pins = MUTANTS[name]
    lib = _build(str(tmp_path), name, old, new)
    env = dict(os.environ, MC_ORACLE_LIB=lib, OMP_NUM_THREADS=os.environ.get("OMP_NUM_THREADS", "4"))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *pins], cwd=ROOT,
                       env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, f"{name}: the pins passed against the mutated oracle\n{r.stdout[-2000:]}"
    assert "failed" in r.stdout


def test_unmutated_copy_passes_the_same_pins(tmp_path):
    """Control: the same build recipe on the unchanged source passes them."""
    src = open(SRC).read()
    path = os.path.join(str(tmp_path), "mc_oracle_copy.c")
    open(path, "w").write(src)
    lib = os.path.join(str(tmp_path), "libmc_oracle_copy.so")
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c11", "-shared", "-fPIC",
                    "-I" + os.path.dirname(SRC),
                    "-o", lib, path, "-lm"], check=True)
    pins = sorted({p for _, _, ps in MUTANTS.values() for p in ps})
    env = dict(os.environ, MC_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", *pins], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:]
