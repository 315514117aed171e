"""Fourth- and sixth-order composed steps (Sec. 2.3) on the GPU against the
oracle's: each sub-step the full hybrid scheme with its own critical radii,
the encounter search over all pairs; positions and velocities within 1e-12
relative after the steps, encounter counts equal."""
import numpy as np
import pytest

import oracle as O
from paper_1404_2324_amd import genga as G
from paper_1404_2324_amd import workloads as W

pytestmark = pytest.mark.gpu
REL = 1e-12


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return (np.linalg.norm(a - b, axis=-1) / np.maximum(np.linalg.norm(b, axis=-1), 1e-300)).max()


def _op(gp):
    return O.params(G=gp.G, m0=gp.m0, dt=gp.dt, n1=gp.n1, n2=gp.n2, pf=gp.pf,
                    bs_tol=gp.bs_tol, bs_max_depth=gp.bs_max_depth,
                    kepler_max_iter=gp.kepler_max_iter, encounter_free=gp.encounter_free)


@pytest.mark.parametrize("order", [4, 6])
def test_composed_plain_n16(order):
    s = W.plain_n16()
    gp = G.default_params(order=order)
    sim = G.Simulation(s.m, s.x, s.u, gp, coords="helio")
    print("order", order, flush=True)
    sim.step(10)
    sim.check()
    xg, vg = [t.cpu().numpy() for t in sim.state("dem")]
    v0 = O.helio_to_dem(_op(gp), s.m, s.u)
    xo, vo, _, st = O.step_order(_op(gp), order, s.m, s.x, v0, 10)
    print("order", order, "rel x", _rel(xg, xo), "v", _rel(vg, vo), "enc", st["enc_total"],
          sim.stats()["enc_total"], flush=True)
    assert _rel(xg, xo) < REL and _rel(vg, vo) < REL
    assert sim.stats()["enc_total"] == st["enc_total"]


def test_composed_dense_encounters_order4():
    """Strongly interacting bodies (the dense small system of the main-mode
    tests): encounters and BS groups in every sub-step."""
    rng = np.random.default_rng(31)
    n = 24
    m = rng.uniform(1e-6, 1e-5, n)
    a = rng.uniform(0.95, 1.05, n)
    ang = rng.uniform(0, 0.6, n)
    x = np.stack([a * np.cos(ang), a * np.sin(ang), rng.normal(0, 0.002, n)], 1)
    u = np.stack([-np.sin(ang), np.cos(ang), np.zeros(n)], 1) / np.sqrt(a)[:, None]
    gp = G.default_params(n2=1.5, order=4)
    sim = G.Simulation(m, x, u, gp, coords="helio")
    sim.step(2)
    sim.check()
    xg, vg = [t.cpu().numpy() for t in sim.state("dem")]
    v0 = O.helio_to_dem(_op(gp), m, u)
    xo, vo, _, st = O.step_order(_op(gp), 4, m, x, v0, 2)
    print("dense order 4: rel x", _rel(xg, xo), "v", _rel(vg, vo), "enc", st["enc_total"], flush=True)
    assert st["enc_total"] > 0 and st["max_group"] >= 2
    assert sim.stats()["enc_total"] == st["enc_total"]
    assert _rel(xg, xo) < REL and _rel(vg, vo) < REL


def test_composed_planetesimals_n2048_order4():
    s = W.planetesimals()
    gp = G.default_params(order=4)
    sim = G.Simulation(s.m, s.x, s.u, gp, coords="helio")
    sim.step(3)
    sim.check()
    xg, vg = [t.cpu().numpy() for t in sim.state("dem")]
    v0 = O.helio_to_dem(_op(gp), s.m, s.u)
    xo, vo, _, st = O.step_order(_op(gp), 4, s.m, s.x, v0, 3)
    gs = sim.stats()
    print("n2048 order 4: rel x", _rel(xg, xo), "v", _rel(vg, vo), "enc", st["enc_total"],
          gs["enc_total"], "full kicks", gs["full_kicks"], flush=True)
    assert st["enc_total"] > 0
    assert _rel(xg, xo) < REL and _rel(vg, vo) < REL
    assert gs["enc_total"] == st["enc_total"]


def test_composed_encounter_free_reversible():
    s = W.plain_n16()
    gp = G.default_params(order=6, encounter_free=1)
    sim = G.Simulation(s.m, s.x, s.u, gp, coords="helio")
    x0, v0 = sim.state()
    sim.step(20)
    x1, v1 = sim.state()
    back = G.Simulation(s.m, x1, v1, G.default_params(order=6, encounter_free=1, dt=-gp.dt),
                        coords="dem")
    back.step(20)
    x2, v2 = back.state()
    assert _rel(x2.cpu().numpy(), x0.cpu().numpy()) < 1e-13
    assert _rel(v2.cpu().numpy(), v0.cpu().numpy()) < 1e-13
    xo, vo, _, _ = O.step_order(_op(gp), 6, s.m, x0.cpu().numpy(), v0.cpu().numpy(), 20)
    assert _rel(x1.cpu().numpy(), xo) < REL


def test_composed_order_limits():
    s = W.plain_n16()
    with pytest.raises(G.GengaError):
        G.Simulation(s.m, s.x, s.u, G.default_params(order=3))
    sim = G.Simulation(s.m, s.x, s.u, G.default_params(order=4))
    with pytest.raises(G.GengaError):
        sim.step_kernel_us(2)
    planets, xt, ut = W.test_particles(ntp=10)
    with pytest.raises(G.GengaError):
        G.TestParticleSimulation(planets.m, planets.x, planets.u, xt, ut,
                                 G.default_params(order=4))
