"""Main mode with collisions, ejections and N_min (Sec. 3.2.7, 3.2.8, 3.4.6)
against the oracle: the events (kind, bodies, step, part of the step), the
bodies left and their row order, the states (1e-12 relative), and the
internal energy U; a run that falls below nmin stops."""
import numpy as np
import pytest

import oracle as O
from paper_1404_2324_amd import genga as G
from paper_1404_2324_amd import workloads as W

pytestmark = pytest.mark.gpu
REL = 1e-12


def _say(*a):
    print(*a, flush=True)


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return (np.linalg.norm(a - b, axis=-1) / np.maximum(np.linalg.norm(b, axis=-1), 1e-300)).max(
        initial=0.0)


def _op(gp):
    return O.params(G=gp.G, m0=gp.m0, dt=gp.dt, n1=gp.n1, n2=gp.n2, pf=gp.pf, bs_tol=gp.bs_tol,
                    bs_max_depth=gp.bs_max_depth, kepler_max_iter=gp.kepler_max_iter)


def _headon(mA, mB, d=0.01, w=1.0, phase=0.0):
    c, s = np.cos(phase), np.sin(phase)
    rot = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])
    x = np.array([[1.0, 0.0, 0.0], [1.0 + d, 0.0, 0.0]]) @ rot.T
    u = np.array([[0.0, 1.0, 0.0], [-w, 1.0, 0.0]]) @ rot.T
    return np.array([mA, mB]), x, u, np.array([4e-4, 6e-4])


def _with_background(m, x, u, R, k=5, seed=70):
    """The given bodies after k quiet planetesimals (rows 0 .. k-1), radii
    that never touch, so rows move when bodies leave."""
    q = W.planetesimals(k, seed_index=seed)
    return (np.concatenate([q.m, m]), np.concatenate([q.x, x]), np.concatenate([q.u, u]),
            np.concatenate([np.full(k, 1e-7), R]))


def _run(m, x, u, R, gp, steps, nmin=0):
    sim = G.Simulation(m, x, u, gp, coords="helio")
    sim.set_radii(R)
    for _ in range(steps):
        sim.step(1)
    orc = O.MassiveSim(_op(gp), m, x, u, coords="helio", radii=R, rcut=gp.rcut,
                       rcut_sun=gp.rcut_sun, nmin=nmin)
    orc.step(steps)
    return sim, orc


def _compare(sim, orc):
    xg, vg = [t.cpu().numpy() for t in sim.state("dem")]
    ids, nl, U = sim.bodies()
    evs = sim.events()
    _say("gpu: n", nl[0], "ids", ids.tolist(), "U", U[0],
         "events", [(e.kind, e.id_i, e.id_j, e.step, e.frac) for e in evs])
    _say("oracle: n", orc.n, "ids", orc.id.tolist(), "U", orc.U,
         "events", [(e.kind, e.id_i, e.id_j, e.step, e.frac) for e in orc.events])
    k = min(orc.n, nl[0])
    _say("rel x", _rel(xg[:k], orc.x[:k]), "v", _rel(vg[:k], orc.v[:k]))
    assert nl[0] == orc.n, (nl[0], orc.n)
    np.testing.assert_array_equal(ids[:orc.n], orc.id)
    assert np.all(ids[orc.n:] == -1)
    assert np.all(np.isnan(xg[orc.n:]))
    e1, e2 = _rel(xg[:orc.n], orc.x), _rel(vg[:orc.n], orc.v)
    assert e1 < REL and e2 < REL, (e1, e2)
    assert U[0] == pytest.approx(orc.U, rel=1e-12, abs=1e-300)
    ge = sorted((e.kind, e.id_i, e.id_j, e.step, e.frac) for e in evs)
    oe = sorted((e.kind, e.id_i, e.id_j, e.step, e.frac) for e in orc.events)
    assert ge == oe, (ge, oe)
    for e in (e for e in evs if e.kind == G.EV_MERGE):
        oe1 = [f for f in orc.events if f.id_i == e.id_i and f.step == e.step][0]
        assert e.U == pytest.approx(oe1.U, rel=1e-10)
        assert _rel([e.x_i], [list(oe1.x_i)]) < REL
    return max(e1, e2), evs


@pytest.mark.parametrize("masses", [(1e-10, 2e-10), (1e-10, 1e-10)])
def test_headon_merger_matches_oracle(masses):
    """A head-on pair behind five quiet bodies: the heavier (or, on equal
    masses, the lower row) survives; the rows after it move."""
    m, x, u, R = _with_background(*_headon(*masses))
    gp = G.default_params()
    sim, orc = _run(m, x, u, R, gp, 3)
    sim.check()
    worst, evs = _compare(sim, orc)
    _say("head-on", masses, [(e.kind, e.id_i, e.id_j, e.step, e.frac) for e in evs], worst)
    assert [e.kind for e in evs] == [G.EV_MERGE]


def test_merger_inside_a_group_of_three():
    m, x, u, R = _headon(3e-10, 2e-10, phase=2.0)
    x = np.vstack([x, x[1] + [0.004, 0.003, 0.0]])
    u = np.vstack([u, u[1]])
    m, x, u, R = _with_background(np.append(m, 1e-10), x, u, np.append(R, 3e-4), k=4, seed=71)
    gp = G.default_params()
    sim, orc = _run(m, x, u, R, gp, 3)
    sim.check()
    worst, evs = _compare(sim, orc)
    _say("group of three", [(e.kind, e.id_i, e.id_j, e.step, e.frac) for e in evs], worst)
    assert sum(e.kind == G.EV_MERGE for e in evs) >= 1


def test_ejections_far_and_sun():
    s = W.planetesimals(8, seed_index=61)
    x, u = s.x.copy(), s.u.copy()
    x[1] *= 30.0 / np.linalg.norm(x[1])
    u[1] *= 0.0
    x[3] *= 0.01 / np.linalg.norm(x[3])
    u[3] *= 0.0
    gp = G.default_params(rcut=20.0, rcut_sun=0.05)
    sim, orc = _run(s.m, x, u, np.zeros(8), gp, 2)
    sim.check()
    worst, evs = _compare(sim, orc)
    assert sorted(e.kind for e in evs) == [G.EV_EJECT_FAR, G.EV_EJECT_SUN]


def test_nmin_stops_the_run():
    m, x, u, R = _headon(1e-10, 2e-10)
    gp = G.default_params(nmin=2)
    sim = G.Simulation(m, x, u, gp, coords="helio")
    sim.set_radii(R)
    sim.step(1)
    assert sim.check() == G.WNMIN
    x1, v1 = sim.state("dem")
    sim.step(3)                       # stopped: the state stays
    assert sim.check() == G.WNMIN
    x2, v2 = sim.state("dem")
    assert bool((x1.isnan() == x2.isnan()).all())
    assert bool((x1[~x1.isnan()] == x2[~x2.isnan()]).all())
    orc = O.MassiveSim(_op(gp), m, x, u, coords="helio", radii=R, nmin=2)
    orc.step(4)
    assert orc.stopped and orc.n == 1
    _compare(sim, orc)


def test_radii_that_never_touch_on_planetesimals():
    """300 planetesimals with radii far below their separations: the
    collision path runs every step and changes nothing the oracle does not."""
    s = W.planetesimals(300, seed_index=3)
    gp = G.default_params(rcut=100.0)
    sim, orc = _run(s.m, s.x, s.u, np.full(300, 1e-9), gp, 10)
    sim.check()
    worst, evs = _compare(sim, orc)
    assert evs == []
    assert sim.stats()["enc_total"] > 0
