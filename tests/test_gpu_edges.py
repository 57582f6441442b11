"""Edge cases on the GPU: hand-placed packs at the boundaries of every
terminal class (against the oracle: classes, nodes, tallies and exit-time
bins exactly, crossing time and radius within 1e-12), collision-free steps
within 1e-12 (RK4 with four bilinear gathers, rounding apart), exit-buffer
overflow, capacity and argument errors, empty steps, and gas regions where
the collision rate vanishes (vacuum, zero gas temperature)."""
import sys

import numpy as np
import pytest

from paper_2609_31258_amd import synth
from tests.parity_util import by_id, make_pair

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _edge_snapshot(f):
    g = f.grid
    R, L = g.R, g.L
    r_ring, z_ring = R / 4 + 1e-4, L / 9  # inside the first ring's metal
    rows = [  # x, y, z, vx, vy, vz
        (0.0, 0.0, 2e-3, 0.0, 0.0, 0.0),             # on the axis at rest
        (0.0, 0.0, 2e-3, 0.0, 0.0, 300.0),           # on the axis moving
        (R - 1e-6, 0.0, 3e-3, 2000.0, 0.0, 0.0),     # leaves radially
        (0.0, R - 1e-6, 3e-3, 0.0, 2000.0, 0.0),     # leaves radially along y
        (2e-4, 0.0, L - 1e-7, 0.0, 0.0, 1000.0),     # crosses the detector inside r_det
        (2e-3, 0.0, L - 1e-7, 0.0, 0.0, 1000.0),     # crosses the detector plane outside r_det
        (1e-4, 1e-4, 1e-7, 0.0, 0.0, -1000.0),       # leaves upstream through z = 0
        (r_ring, 0.0, z_ring, 0.0, 0.0, 0.0),        # sits in metal
        (0.0, r_ring, z_ring, 0.0, 0.0, 0.0),        # the same node, other azimuth
        (r_ring * 0.7071067811865476, r_ring * 0.7071067811865476, z_ring, 0.0, 0.0, 0.0),
        (R / 4 - 2e-4, 0.0, z_ring, 0.0, 0.0, 0.0),  # just off the metal, inside the ring
    ]
    a = np.array(rows)
    n = len(a)
    return dict(x=a[:, 0].copy(), y=a[:, 1].copy(), z=a[:, 2].copy(), vx=a[:, 3].copy(), vy=a[:, 4].copy(),
                vz=a[:, 5].copy(), e_int=np.full(n, 3e-19), h=np.zeros(n), w=np.linspace(0.5, 2.0, n),
                id=np.arange(n, dtype=np.int64), tag=np.zeros(n, np.int32))


@pytest.mark.parametrize("precision,collisions", [(0, 1), (0, 0), (1, 1)])
def test_boundary_packs_classify_like_the_oracle(precision, collisions):
    f, ions, _, op, _ = synth.config_c1(100)
    op.r_det = 1e-3
    op.collisions_on = collisions
    snap = _edge_snapshot(f)
    _say("boundary packs, precision", precision, "collisions", collisions)
    g, o = make_pair(f, ions, [], op, cap=64, precision=precision)
    g.write_packs(snap)
    o.write_packs(snap)
    g.step(1)
    o.step(1)
    a, b = by_id(g.read_packs()), by_id(o.read_packs())
    _say("  classes", a["status"].tolist())
    assert np.array_equal(a["status"], b["status"])
    assert sorted(set(b["status"].tolist())) == [0, 1, 2, 3, 4]  # active, transmitted, axial, radial, electrode
    ea, eb = g.read_exits(), o.read_exits()
    assert np.array_equal(ea["id"], eb["id"]) and np.array_equal(ea["cls"], eb["cls"])
    assert np.array_equal(ea["inode"], eb["inode"]) and np.array_equal(ea["jnode"], eb["jnode"])
    tol = 1e-12 if precision == 0 else 1e-6
    assert np.allclose(ea["t_cross"], eb["t_cross"], rtol=tol, atol=0)
    assert np.allclose(ea["r_cross"], eb["r_cross"], rtol=tol, atol=1e-18)
    ta, tb = g.read_tallies(), o.read_tallies()
    assert np.array_equal(ta["class_n"], tb["class_n"]) and np.array_equal(ta["class_w"], tb["class_w"])
    assert np.array_equal(ta["loss_map"], tb["loss_map"])
    assert np.array_equal(ta["exit_bins"], tb["exit_bins"])
    if precision == 0 and not collisions:
        keep = a["status"] == 0
        for k in ("x", "y", "z", "vx", "vy", "vz"):
            assert np.allclose(a[k][keep], b[k][keep], rtol=1e-12, atol=1e-12), k
    g.close()


def test_exit_buffer_overflow_counts_every_exit():
    from paper_2609_31258_amd import mucite
    f, ions, _, op, _ = synth.config_c1(100)
    n = 20
    snap = dict(x=np.zeros(n), y=np.zeros(n), z=np.full(n, 1e-7), vx=np.zeros(n), vy=np.zeros(n),
                vz=np.full(n, -1000.0), e_int=np.full(n, 3e-19), h=np.zeros(n), w=np.ones(n),
                id=np.arange(n, dtype=np.int64), tag=np.zeros(n, np.int32))
    g = mucite.Sim(seed=7, pack_capacity=n, exit_capacity=5, precision=0)
    g.setup(f, ions, [], op)
    g.write_packs(snap)
    g.step(1)
    t = g.read_tallies()
    e = g.read_exits()
    assert t["class_n"][4] == n and len(e) == 5 and t["exit_dropped"] == n - 5  # class 4: axial exit
    g.close()


def test_capacity_and_argument_errors_leave_the_context_usable():
    from paper_2609_31258_amd import mucite
    f, ions, srcs, op, _ = synth.config_c1(1000)
    g = mucite.Sim(seed=7, pack_capacity=500, precision=0)
    g.setup(f, ions, srcs, op)
    with pytest.raises(mucite.MucateError) as e:
        g.inject(0, 1000)  # more than the capacity
    assert e.value.code == mucite.MC_ENOMEM
    g.inject(0, 400)
    bad = synth.Operating(**{**op.__dict__, "dt": 0.0})
    with pytest.raises(mucite.MucateError) as e:
        g.set_operating(bad)
    assert e.value.code == mucite.MC_EINVAL
    snap = synth.pack_snapshot(10, f, seed=1)
    snap["vx"][3] = np.nan
    with pytest.raises(mucite.MucateError) as e:
        g.write_packs(snap)
    assert e.value.code == mucite.MC_EINVAL
    g.step(0)
    g.step(2)
    t = g.read_tallies()
    assert t["emitted_n"] == 400 and t["class_n"].sum() == 400 and t["pack_steps"] == 800
    g.close()


def test_non_finite_field_tables_are_refused():
    from paper_2609_31258_amd import mucite
    f, ions, srcs, op, _ = synth.config_c1(100)
    for name, value in (("phi_dc", np.nan), ("gas_uz", np.inf), ("gas_p", -1.0)):
        bad = synth.Fields(**{**f.__dict__, name: getattr(f, name).copy()})
        getattr(bad, name)[7, 3] = value
        g = mucite.Sim(seed=7, pack_capacity=16, precision=0)
        with pytest.raises(mucite.MucateError) as e:
            g.load_fields(bad)
        assert e.value.code == mucite.MC_EINVAL, name
        g.load_fields(f)  # the context is still usable
        g.close()


def _degenerate_gas_fields():
    """The C1 field set with a vacuum third (gas pressure 0), a third at zero
    gas temperature (pressure kept), and gas beyond: the collision rate is
    zero in the first two, where a pack must fly free."""
    f, ions, _, op, _ = synth.config_c1(100)
    g = f.grid
    p = f.gas_p.reshape(g.nz, g.nr).copy()
    t = f.gas_t.reshape(g.nz, g.nr).copy()
    p[: g.nz // 3, :] = 0.0
    t[g.nz // 3: 2 * g.nz // 3, :] = 0.0
    f.gas_p, f.gas_t = p.reshape(-1), t.reshape(-1)
    return f, ions, op


@pytest.mark.parametrize("precision", [0, 1])
def test_vacuum_and_zero_temperature_gas_match_the_oracle(precision):
    """Packs spread over the three regions: one step against the oracle
    (statuses exactly; FP64: state within 1e-6 and candidate count within
    1e-3; FP32 form: candidate count within 1 %).  Packs only in the vacuum
    third: three steps with collisions on equal the collision-free steps bit
    for bit and draw no candidate."""
    from paper_2609_31258_amd import mucite
    from tests.parity_util import step_errors, thermal_speed
    f, ions, op = _degenerate_gas_fields()
    g = f.grid
    n = 6000
    snap = synth.pack_snapshot(n, f, seed=23, z_lo=0.05 * g.L, z_hi=0.95 * g.L, r_hi=0.2 * g.R, v_sigma=300.0)
    _say("degenerate gas regions, precision", precision)
    gp, orc = make_pair(f, ions, [], op, cap=n, precision=precision)
    gp.write_packs(snap)
    orc.write_packs(snap)
    gp.step(1)
    orc.step(1)
    a, b = by_id(gp.read_packs()), by_id(orc.read_packs())
    assert np.array_equal(a["status"], b["status"])
    ta, tb = gp.read_tallies(), orc.read_tallies()
    _say(f"  candidates gpu {ta['n_cand']} oracle {tb['n_cand']}")
    assert tb["n_cand"] > 0
    if precision == 0:
        r = step_errors(gp.read_packs(), orc.read_packs(), g.dr, thermal_speed(), snap["h"])
        assert r["ok"].sum() >= n - max(1, n // 10_000)
        assert abs(ta["n_cand"] - tb["n_cand"]) <= max(2, tb["n_cand"] // 1000)
    else:
        assert abs(ta["n_cand"] - tb["n_cand"]) <= 0.01 * tb["n_cand"]
    gp.close()

    zv = (g.nz // 3 - 2) * g.dz  # below it every gather reads only vacuum nodes
    snap_v = synth.pack_snapshot(2000, f, seed=29, z_lo=0.1 * zv, z_hi=0.5 * zv, r_hi=0.2 * g.R, v_sigma=300.0)
    runs = []
    for coll in (1, 0):
        op.collisions_on = coll
        s = mucite.Sim(seed=synth.SEED, pack_capacity=2000, precision=precision)
        s.setup(f, ions, [], op)
        s.write_packs(snap_v)
        s.step(3)
        runs.append((s.read_packs(), s.read_tallies()))
        s.close()
    (pa, ta), (pb, tb) = runs
    assert ta["n_cand"] == 0 and tb["n_cand"] == 0
    for k in ("x", "y", "z", "vx", "vy", "vz", "e_int", "h", "status"):
        assert np.array_equal(pa[k], pb[k]), k
