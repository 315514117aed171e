"""GPU parity of test-particle mode (Sec. 3.3) against the oracle.  Particles
do not act on anything, so the oracle can follow any subset of them one by
one with the same planets."""
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
    num = np.linalg.norm(np.asarray(a) - np.asarray(b), axis=-1)
    den = np.maximum(np.linalg.norm(np.asarray(b), axis=-1), 1e-300)
    return num / den


def _op(gp):
    return O.params(G=gp.G, m0=gp.m0, dt=gp.dt, n1=gp.n1, n2=gp.n2, pf=gp.pf,
                    bs_tol=gp.bs_tol, bs_max_depth=gp.bs_max_depth,
                    kepler_max_iter=gp.kepler_max_iter, encounter_free=gp.encounter_free)


def _sample(ntp_total, sel, seed_index=3):
    planets, xt, ut = W.test_particles(ntp=ntp_total, seed_index=seed_index)
    return planets, xt[sel], ut[sel]


def _tp_sets_close(sim, orc, sel=None, band=1e-10):
    """The last step's particle-planet encounter pairs (Sec. 3.3) of the GPU
    run against the oracle's, as sets: equal except pairs whose Hermite
    minimum lies within `band` (relative) of r_crit,ij^2 on either side.
    Pairs in both sets carry the same threshold and minimum (to the rounding
    of states that agree to 1e-12).  sel: the GPU particle index of each
    oracle particle when the oracle follows a subset.  Returns the count."""
    ij_g, d2_g, rc2_g = sim.tp_encounters()
    assert np.all(d2_g < rc2_g)
    if sel is not None:
        pos = {int(g): o for o, g in enumerate(sel)}
        keep = np.array([int(k) in pos for k in ij_g[:, 0]], dtype=bool)
        ij_g, d2_g, rc2_g = ij_g[keep], d2_g[keep], rc2_g[keep]
        ij_g = np.stack([np.array([pos[int(k)] for k in ij_g[:, 0]], dtype=np.int64),
                         ij_g[:, 1]], 1)
    ij_o, d2_o, rc2_o = orc.tp_encounters()
    A = {tuple(q): (v, t) for q, v, t in zip(ij_g.tolist(), d2_g, rc2_g)}
    B = {tuple(q): (v, t) for q, v, t in zip(ij_o.tolist(), d2_o, rc2_o)}
    for k in set(A) ^ set(B):
        seen = [A.get(k), B.get(k), (orc.tp_d2[k], orc.tp_rc2[k])]
        assert any(c is not None and np.isfinite(c[0]) and abs(c[0] - c[1]) <= band * c[1]
                   for c in seen), f"pair {k} differs and is not in the band: {seen}"
    for k in set(A) & set(B):
        (vg, tg), (vo, to) = A[k], B[k]
        assert abs(tg - to) <= 1e-11 * to, k
        assert abs(vg - vo) <= 1e-8 * to, k
    return len(B)


@pytest.mark.parametrize("ntp", [0, 1, 63, 2000])
def test_tp_ten_steps(ntp):
    _say("tp parity ntp", ntp)
    planets, xt, ut = W.test_particles(ntp=max(ntp, 1), seed_index=3)
    xt, ut = xt[:ntp], ut[:ntp]
    gp = G.default_params()
    sim = G.TestParticleSimulation(planets.m, planets.x, planets.u, xt, ut, gp, coords="helio")
    orc = O.TPSim(_op(gp), planets.m, planets.x, planets.u, xt, ut, coords="helio")
    enc_o = 0
    for _ in range(10):
        sim.step(1)
        st = orc.step(1)
        enc_o += st["tp_enc"]
        # the step's encounter set, pair by pair, every step
        assert _tp_sets_close(sim, orc) == st["tp_enc"]
    sim.check()
    gs = sim.stats()
    xp, vp, xg, vg = [t.cpu().numpy() for t in sim.split_state()]
    assert _rel(xp, orc.x).max() < REL and _rel(vp, orc.v).max() < REL
    # every drift of the 10 steps is in the Kepler-iteration histogram
    assert sum(gs["kepler_hist"]) == 10 * (planets.m.size + ntp)
    assert max(k for k, c in enumerate(gs["kepler_hist"]) if c) == gs["kepler_iter_max"]
    if ntp:
        ex, ev = _rel(xg, orc.xt), _rel(vg, orc.vt)
        _say("tp", ntp, "enc gpu total", gs["tp_enc_total"], "oracle", enc_o, "max rel x",
             ex.max(), "v", ev.max())
        assert ex.max() < REL and ev.max() < REL
    if ntp == 2000:
        assert enc_o > 50


def test_tp_million_sampled():
    """10^6 particles on the GPU for 3 steps; the oracle follows every 997th
    particle (plus all of the first 500) with the same planets, held to the
    1e-12 bar, and every particle with an encounter in the last step, whose
    encounter pairs are compared as sets.  Deep passages by a planet amplify
    rounding differences (nothing removes a particle here), so the particles
    of the encounter sample are held to 10 times the oracle's own spread
    under 1-ulp input changes, measured here."""
    planets, xt, ut = W.test_particles(ntp=1_000_000, seed_index=3)
    gp = G.default_params()
    sim = G.TestParticleSimulation(planets.m, planets.x, planets.u, xt, ut, gp, coords="helio")
    sim.step(3)
    sim.check()
    st = sim.stats()
    _say("1e6 tp stats", st)
    assert st["tp_enc"] > 1000  # the workload exercises the particle BS path
    _, _, xg, vg = [t.cpu().numpy() for t in sim.split_state()]
    base = np.unique(np.concatenate([np.arange(500), np.arange(0, 1_000_000, 997)]))
    ij, _, _ = sim.tp_encounters()
    assert len(ij) == st["tp_enc"]
    sel = np.unique(np.concatenate([base, ij[:, 0]]))
    inb = np.isin(sel, base)
    orc = O.TPSim(_op(gp), planets.m, planets.x, planets.u, xt[sel], ut[sel], coords="helio")
    orc.step(3)
    ex, ev = _rel(xg[sel], orc.xt), _rel(vg[sel], orc.vt)
    _say("sampled", int(inb.sum()), "max rel x", ex[inb].max(), "v", ev[inb].max())
    assert ex[inb].max() < REL and ev[inb].max() < REL
    spread = 0.0
    for seed in (1, 2):
        pr = np.random.default_rng(seed)
        xp = xt[sel] * (1 + 2.0 ** -52 * pr.choice([-1.0, 1.0], (len(sel), 3)))
        o2 = O.TPSim(_op(gp), planets.m, planets.x, planets.u, xp, ut[sel], coords="helio")
        o2.step(3)
        spread = max(spread, _rel(o2.xt, orc.xt).max(), _rel(o2.vt, orc.vt).max())
    _say("encounter sample", int((~inb).sum()), "max rel x", ex.max(), "v", ev.max(),
         "oracle 1-ulp spread", spread)
    assert max(ex.max(), ev.max()) < max(REL, 10 * spread)
    n_o = _tp_sets_close(sim, orc, sel=sel)
    _say("sampled encounter pairs (last step)", n_o)
    assert n_o > 1000


def test_tp_encounter_sets_5000():
    """The prechecker masks and the Hermite test of 5000 particles, through
    the encounter pairs of each of 5 steps."""
    planets, xt, ut = W.test_particles(ntp=5000, seed_index=3)
    gp = G.default_params()
    orc = O.TPSim(_op(gp), planets.m, planets.x, planets.u, xt, ut, coords="helio")
    sim = G.TestParticleSimulation(planets.m, planets.x, planets.u, xt, ut, gp, coords="helio")
    total = 0
    for _ in range(5):
        sim.step(1)
        so = orc.step(1)
        total += _tp_sets_close(sim, orc)
        assert sim.stats()["tp_enc"] == len(sim.tp_encounters()[0])
    assert total > 100


def test_tp_encounter_free_equals_massive_free():
    """K = 1: particles follow the planets' Newtonian field; same map as the
    main mode with zero-mass bodies."""
    planets, xt, ut = W.test_particles(ntp=300, seed_index=3)
    gp = G.default_params(encounter_free=1)
    sim = G.TestParticleSimulation(planets.m, planets.x, planets.u, xt, ut, gp, coords="helio")
    sim.step(20)
    _, _, xg, vg = [t.cpu().numpy() for t in sim.split_state()]
    orc = O.TPSim(_op(gp), planets.m, planets.x, planets.u, xt, ut, coords="helio")
    orc.step(20)
    assert _rel(xg, orc.xt).max() < REL


def _coll_spread(planets, xt, ut, rad, gp, orc, steps, seeds=(1, 2, 3)):
    """The oracle against itself with the particles' positions moved by 1 ulp
    (random signs): the removal sets, the agreement of the collision
    fractions, and the relative spread of the reports and of the survivors.
    Close passages amplify any rounding difference, so this is the yardstick
    for the GPU-oracle difference in the same run."""
    out = {"frac_equal": 1.0, "dfrac": 0.0, "report": 0.0, "x": 0.0, "v": 0.0}
    gone = orc.removed()
    for seed in seeds:
        pr = np.random.default_rng(seed)
        xp = xt * (1 + 2.0 ** -52 * pr.choice([-1.0, 1.0], xt.shape))
        o2 = O.TPSim(_op(gp), planets.m, planets.x, planets.u, xp, ut, coords="helio", radii=rad)
        o2.step(steps)
        assert np.array_equal(o2.removed(), gone)
        eq = o2.coll_frac[gone] == orc.coll_frac[gone]
        out["frac_equal"] = min(out["frac_equal"], float(eq.mean()) if len(gone) else 1.0)
        out["dfrac"] = max(out["dfrac"], float(np.abs(o2.coll_frac[gone] - orc.coll_frac[gone]).max(initial=0)))
        out["report"] = max(out["report"], float(_rel(o2.coll_xv[gone][eq], orc.coll_xv[gone][eq]).max(initial=0)))
        alive = np.setdiff1d(np.arange(len(xt)), gone)
        out["x"] = max(out["x"], float(_rel(o2.xt[alive], orc.xt[alive]).max(initial=0)))
        out["v"] = max(out["v"], float(_rel(o2.vt[alive], orc.vt[alive]).max(initial=0)))
    return out


def _coll_parity(sim, orc, ntp, spread):
    """Removal reports and surviving states of the GPU run against the
    oracle's.  Unique and compared exactly: which particles are removed, by
    which planet, in which step.  The part of the step at which a collision is
    reported is resolved to the BS substep; where the two sides take an
    accept/reject decision on different sides of the tolerance (their forces
    differ in the last bits) the substep partition differs.  The bounds for
    those are the oracle's own spread under 1-ulp input changes (`spread`):
    the share of equal fractions at least 0.9 of the oracle's own, their
    largest difference at most 4 times the oracle's, report states of equal
    fraction within 10 times the oracle's report spread."""
    rep = sim.collisions()
    gone_o = orc.removed()
    _say("removed gpu", len(rep["tp"]), "oracle", len(gone_o), "oracle spread", spread)
    order = np.argsort(rep["tp"], kind="stable")
    np.testing.assert_array_equal(rep["tp"][order], gone_o)
    np.testing.assert_array_equal(rep["planet"][order], orc.coll_planet[gone_o])
    np.testing.assert_array_equal(rep["step"][order], orc.coll_step[gone_o])
    fg, fo = rep["frac"][order], orc.coll_frac[gone_o]
    same = fg == fo
    _say("frac equal", int(same.sum()), "gpu earlier", int((fg < fo).sum()),
         "gpu later", int((fg > fo).sum()), "max |dfrac|", float(np.abs(fg - fo).max(initial=0)))
    assert same.mean() >= 0.9 * spread["frac_equal"]
    assert np.abs(fg - fo).max(initial=0) <= 4 * max(spread["dfrac"], 2.0 ** -20)
    if len(gone_o):
        xg_r, xo_r = rep["xv"][order], orc.coll_xv[gone_o]
        dx = _rel(xg_r[same, :3], xo_r[same, :3]).max(initial=0)
        dv = _rel(xg_r[same, 3:], xo_r[same, 3:]).max(initial=0)
        _say("reports with equal frac: max rel x", dx, "v", dv)
        tol = max(REL, 10 * spread["report"])
        assert dx < tol and dv < tol
    _, _, xg, vg = [t.cpu().numpy() for t in sim.split_state(coords="dem")]
    alive = np.setdiff1d(np.arange(ntp), gone_o)
    assert np.all(np.isnan(xg[gone_o])) and np.all(np.isnan(vg[gone_o]))
    assert np.all(np.isfinite(xg[alive]))
    return xg, vg, alive


def _flyby_inputs(n_bg=2000, n_fly=2000):
    """The workload's planets and particles plus particles aimed at the
    planets inside 4 planet radii; physical radii (bulk density 2 g/cm^3)."""
    planets, xt, ut = W.test_particles(ntp=n_bg, seed_index=3)
    xf, uf = W.tp_flybys(planets, W.tp_radii(planets.m, 0), n_fly)
    xt, ut = np.concatenate([xt, xf]), np.concatenate([ut, uf])
    return planets, xt, ut, W.tp_radii(planets.m, len(xt))


def test_tp_collisions_match_oracle():
    """Sec. 3.3 removal: about 900 of 4000 particles hit a planet in 12 steps.
    Passages within a few planet radii amplify differences (the BS tolerance
    is ~1e-10 of the particle-planet distance there), so the survivors of
    these passages are held to 10 times the oracle's own 1-ulp spread,
    measured here; the background particles hold the 1e-12 bar."""
    planets, xt, ut, rad = _flyby_inputs()
    ntp = len(xt)
    gp = G.default_params()
    sim = G.TestParticleSimulation(planets.m, planets.x, planets.u, xt, ut, gp, coords="helio",
                                   radii=rad)
    orc = O.TPSim(_op(gp), planets.m, planets.x, planets.u, xt, ut, coords="helio", radii=rad)
    sub_o = 0
    for _ in range(3):
        sim.step(4)
        sub_o += orc.step(4)["bs_substeps"]
    sim.check()
    st = sim.stats()
    _say("bs substeps gpu", st["bs_substeps"], "oracle", sub_o)
    assert abs(st["bs_substeps"] - sub_o) <= 0.01 * sub_o
    assert st["tp_removed"] == len(orc.removed()) > 500
    spread = _coll_spread(planets, xt, ut, rad, gp, orc, 12)
    xg, vg, alive = _coll_parity(sim, orc, ntp, spread)
    ex, ev = _rel(xg[alive], orc.xt[alive]), _rel(vg[alive], orc.vt[alive])
    _say("survivors max rel x", ex.max(), "v", ev.max(), "beyond 1e-12:", int((ex > 1e-12).sum()))
    assert ex.max() < max(REL, 10 * spread["x"]) and ev.max() < max(REL, 10 * spread["v"])
    # the background particles (no aimed passage) hold the 1e-12 bar
    bg = alive[alive < 2000]
    assert ex[: len(bg)].max() < REL and ev[: len(bg)].max() < REL


def test_tp_million_with_radii_sampled_and_all_removals():
    """The 10^6-particle workload with its physical radii for 10 steps: every
    removal matches the oracle's (which follows all particles), and the
    survivors match on a sample."""
    planets, xt, ut = W.test_particles(ntp=1_000_000, seed_index=3)
    rad = W.tp_radii(planets.m, len(xt))
    gp = G.default_params()
    sim = G.TestParticleSimulation(planets.m, planets.x, planets.u, xt, ut, gp, coords="helio",
                                   radii=rad)
    sim.step(10)
    sim.check()
    orc = O.TPSim(_op(gp), planets.m, planets.x, planets.u, xt, ut, coords="helio", radii=rad)
    orc.step(10)
    rep = sim.collisions()
    gone_o = orc.removed()
    _say("1e6 removals gpu", len(rep["tp"]), "oracle", len(gone_o))
    np.testing.assert_array_equal(np.sort(rep["tp"]), gone_o)
    _, _, xg, vg = [t.cpu().numpy() for t in sim.split_state(coords="dem")]
    sel = np.setdiff1d(np.arange(0, 1_000_000, 499), gone_o)
    assert _rel(xg[sel], orc.xt[sel]).max() < REL and _rel(vg[sel], orc.vt[sel]).max() < REL


def test_tp_radii_errors_and_removed_rows_round_trip():
    planets, xt, ut, rad = _flyby_inputs(1000, 500)
    gp = G.default_params()
    sim = G.TestParticleSimulation(planets.m, planets.x, planets.u, xt, ut, gp, coords="helio")
    bad = rad.copy()
    bad[3] = -1.0
    with pytest.raises(G.GengaError) as ei:
        sim.set_radii(bad)
    assert ei.value.code == G.EINVAL
    sim.set_radii(rad)
    sim.step(4)
    sim.check()
    gone = sim.collisions()["tp"]
    assert len(gone) > 0
    # a removed particle's row is six NaN; set_state takes it back as removed
    x, v = sim.state("dem")
    sim2 = G.TestParticleSimulation(planets.m, planets.x, planets.u, xt, ut, gp, coords="helio")
    sim2.set_state(x, v, coords="dem")
    x2, v2 = sim2.state("dem")
    assert torch_equal_nan(x, x2) and torch_equal_nan(v, v2)
    sim2.step(2)
    sim2.check()
    x3, _ = sim2.state("dem")
    assert bool(x3[planets.m.size + gone].isnan().all())
    # a half-NaN particle row is rejected
    x[planets.m.size, 0] = float("nan")
    x[planets.m.size + gone[0]] = 0.5
    with pytest.raises(G.GengaError):
        sim2.set_state(x, v, coords="dem")
    # main mode takes radii only with encounters (the K = 1 map has no BS)
    import torch
    ms = G.Simulation(planets.m, planets.x, planets.u, G.default_params(encounter_free=1),
                      coords="helio")
    r = torch.zeros(planets.m.size, dtype=torch.float64, device="cuda")
    assert G.lib().genga_set_radii(ms._ctx, r.data_ptr()) == G.EINVAL
    ms.close()


def torch_equal_nan(a, b):
    import torch
    return bool(torch.equal(torch.nan_to_num(a, nan=1e300), torch.nan_to_num(b, nan=1e300)))
