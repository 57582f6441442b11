"""Oracle pins for time-resolved snapshots (trajectory samples): the records
of a collision-free run in a uniform field follow the closed-form motion,
the sampled set is exactly the active packs with id % stride == 0 at every
sampled step, and the step-0 record is the written state."""
import numpy as np

from oracle import binding as O
from paper_2609_31258_amd import synth

QE, DA = 1.602176634e-19, 1.66053906892e-27


def test_samples_follow_the_uniform_field_motion():
    ez, dt, m = 2e3, 1e-9, 500.0
    f = synth.uniform_fields(16, 512, 5e-5, ez=ez)
    ion = synth.Ion(m, 1, 2e-18, 150)
    op = synth.Operating(dt=dt, z_det=f.grid.L, r_det=f.grid.R, collisions_on=0, sample_every=4, sample_stride=3)
    s = O.OracleSim(7)
    s.setup(f, [ion], [], op)
    n = 50
    rng = np.random.default_rng(1)
    z0 = rng.uniform(1e-3, 2e-3, n)
    vz0 = rng.uniform(-50, 50, n)
    snap = dict(x=np.zeros(n), y=np.zeros(n), z=z0, vx=np.zeros(n), vy=np.zeros(n), vz=vz0, e_int=np.full(n, 1e-19),
                h=np.zeros(n), w=np.ones(n), id=np.arange(n, dtype=np.int64), tag=np.zeros(n, np.int32))
    s.write_packs(snap)
    s.step(21)
    r = s.read_samples()
    ids = np.arange(0, n, 3)
    steps = np.arange(0, 21, 4)
    assert len(r) == len(ids) * len(steps)
    assert np.array_equal(r["step"], np.repeat(steps, len(ids)))
    assert np.array_equal(r["id"], np.tile(ids, len(steps)))
    a = QE * ez / (m * DA)
    t = r["step"] * dt
    assert np.allclose(r["z"], z0[r["id"]] + vz0[r["id"]] * t + 0.5 * a * t * t, rtol=1e-13, atol=1e-18)
    assert np.allclose(r["vz"], vz0[r["id"]] + a * t, rtol=1e-12, atol=1e-9)
    ke = 0.5 * m * DA * r["vz"] ** 2 / QE
    assert np.allclose(r["ke_ev"], ke, rtol=1e-12, atol=0)
    first = r[r["step"] == 0]
    assert np.array_equal(first["z"], z0[ids]) and np.array_equal(first["vz"], vz0[ids])


def test_samples_skip_terminal_packs():
    f = synth.uniform_fields(16, 64, 5e-5, ez=-1e5)  # pushes packs upstream, out through z = 0
    ion = synth.Ion(500.0, 1, 2e-18, 150)
    op = synth.Operating(dt=1e-9, z_det=f.grid.L, r_det=f.grid.R, collisions_on=0, sample_every=1, sample_stride=1)
    s = O.OracleSim(7)
    s.setup(f, [ion], [], op)
    n = 20
    z0 = np.linspace(1e-6, 4e-5, n)
    snap = dict(x=np.zeros(n), y=np.zeros(n), z=z0, vx=np.zeros(n), vy=np.zeros(n), vz=np.zeros(n),
                e_int=np.full(n, 1e-19), h=np.zeros(n), w=np.ones(n), id=np.arange(n, dtype=np.int64),
                tag=np.zeros(n, np.int32))
    s.write_packs(snap)
    s.step(40)
    r = s.read_samples()
    p = s.read_packs()
    ex = s.read_exits()
    assert len(ex) > 0
    for k in range(40):
        rk = r[r["step"] == k]
        # sampled at step k: exactly the packs that had not exited before step k
        alive = set(int(i) for i in p["id"] if i not in set(ex["id"][ex["step"] < k]))
        assert set(rk["id"].tolist()) == alive
