"""GPU parity: the gfx950 library (through its C ABI) against the CPU oracle
on the same seeded inputs.  Tolerances: positions and velocities within
1e-12 relative (per body) after 10 steps; encounter and candidate sets equal
except pairs within 1e-10 (relative) of their threshold."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1404_2324_amd import genga as G
from paper_1404_2324_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda"
REL = 1e-12


def _say(*a):
    print(*a, flush=True)


def _rel_body(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    num = np.linalg.norm(a - b, axis=-1)
    den = np.maximum(np.linalg.norm(b, axis=-1), 1e-300)
    return (num / den).max()


def _gparams(**kw):
    return G.default_params(**kw)


def _oparams(gp):
    return O.params(G=gp.G, m0=gp.m0, dt=gp.dt, n1=gp.n1, n2=gp.n2, pf=gp.pf,
                    bs_tol=gp.bs_tol, bs_max_depth=gp.bs_max_depth,
                    kepler_max_iter=gp.kepler_max_iter, encounter_free=gp.encounter_free)


def _pairs_close(a_ij, b_ij, a_val, a_thr, b_val, b_thr, band=1e-10):
    """Sets equal except pairs whose value is within `band` of its threshold."""
    A = {tuple(p): (v, t) for p, v, t in zip(map(tuple, a_ij), a_val, a_thr)}
    B = {tuple(p): (v, t) for p, v, t in zip(map(tuple, b_ij), b_val, b_thr)}
    for k in set(A) ^ set(B):
        v, t = A.get(k) or B.get(k)
        assert abs(v - t) <= band * t, f"pair {k} differs and is not in the band"


def _cand_sets_close(cg, co, orc, band=1e-10, r2g=None):
    """Candidate sets equal except pairs within `band` of pf r_crit,ij; with
    r2g (the GPU's r_ij^2 per pair of cg), those agree with r_ij^2 from the
    oracle's positions to what the 1e-12 position bar allows:
    |d r^2| <= 2 r |d(x_j - x_i)| with |dx| <= 1e-12 |x| per body."""
    diff = set(map(tuple, cg)) ^ set(map(tuple, co))
    for i, j in diff:
        r = np.linalg.norm(orc.x[j] - orc.x[i])
        t = orc.p.pf * max(orc.rc[i], orc.rc[j])
        assert abs(r - t) <= band * t, f"candidate {(i, j)} differs and is not in the band"
    if r2g is not None and len(cg):
        xi, xj = orc.x[cg[:, 0]], orc.x[cg[:, 1]]
        ro2 = np.sum((xj - xi) ** 2, axis=1)
        dx = 1e-12 * (np.linalg.norm(xi, axis=1) + np.linalg.norm(xj, axis=1))
        assert np.all(np.abs(r2g - ro2) <= 2 * np.sqrt(ro2) * dx + 1e-15 * ro2)


# ------------------------------------------------------------- components --
def test_kepler_drift_parity():
    rng = np.random.default_rng(21)
    n = 5000
    x0 = rng.uniform(-3, 3, (n, 3))
    r = np.linalg.norm(x0, axis=1, keepdims=True)
    # bound, near-parabolic and hyperbolic orbits
    vfac = rng.uniform(0.2, 1.6, (n, 1))
    v0 = rng.standard_normal((n, 3))
    v0 *= vfac * np.sqrt(2.0 / r) / np.linalg.norm(v0, axis=1, keepdims=True)
    for dt in (0.0628, -0.0628, 0.7):
        _say("kepler parity dt", dt)
        x, v, it = G.kepler(1.0, x0, v0, dt)
        x, v, it = x.cpu().numpy(), v.cpu().numpy(), it.cpu().numpy()
        assert (it > 0).all()
        xo = np.zeros_like(x0)
        vo = np.zeros_like(v0)
        for k in range(0, n, 7):
            xo[k], vo[k], _ = O.kepler(1.0, x0[k], v0[k], dt)
        sel = np.arange(0, n, 7)
        assert _rel_body(x[sel], xo[sel]) < 1e-13
        assert _rel_body(v[sel], vo[sel]) < 1e-13


def test_kepler_nonconvergence_reported():
    # eccentric orbit: the first guess s = dt/r0 is not the root
    x, v, it = G.kepler(1.0, [[1.0, 0, 0]], [[0, 1.2, 0.1]], 0.5, max_iter=1)
    assert int(it.cpu()[0]) < 0
    x, v, it = G.kepler(1.0, [[1.0, 0, 0]], [[0, 1.2, 0.1]], 0.5, max_iter=40)
    assert 0 < int(it.cpu()[0]) <= 6


def test_hermite_parity():
    rng = np.random.default_rng(22)
    n = 20000
    q = rng.standard_normal((n, 12))
    dt = 0.0628
    got = G.hermite(dt, q).cpu().numpy()
    ref = np.array([O.hermite_dmin2(dt, r[0:3], r[3:6], r[6:9], r[9:12]) for r in q[:2000]])
    np.testing.assert_allclose(got[:2000], ref, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("n", [1, 2, 16, 63, 64, 65, 300, 1000, 2048])
def test_accel_parity(n):
    _say("accel parity n", n)
    rng = np.random.default_rng(100 + n)
    m = rng.uniform(1e-9, 1e-6, n)
    x = rng.uniform(-1, 1, (n, 3)) * np.array([1, 1, 0.05]) + np.array([1.5, 0, 0])
    rc = rng.uniform(0.01, 0.08, n)  # many pairs in the changeover band
    gp = _gparams()
    a = G.accel(gp, m, x, rc).cpu().numpy()
    ao = O.accel(_oparams(gp), m, x, rc)
    scale = np.abs(ao).max() + 1e-300
    assert np.abs(a - ao).max() <= 1e-13 * scale
    gp1 = _gparams(encounter_free=1)
    a1 = G.accel(gp1, m, x).cpu().numpy()
    ao1 = O.accel(_oparams(gp1), m, x)
    assert np.abs(a1 - ao1).max() <= 1e-13 * (np.abs(ao1).max() + 1e-300)


def test_accel_parity_maximum_size():
    """The largest system the library takes (65,536 bodies, encounter-free):
    the pair sum per body against the oracle's, relative to each body's own
    acceleration (the far-field sums of 65,535 terms cancel strongly)."""
    n = 65536
    s = W.planetesimals(n, seed_index=2)
    gp = _gparams(encounter_free=1)
    a = G.accel(gp, s.m, s.x).cpu().numpy()
    ao = O.accel(_oparams(gp), s.m, s.x)
    rel = np.linalg.norm(a - ao, axis=1) / np.linalg.norm(ao, axis=1)
    _say("n 65536 accel: max rel", rel.max(), "median", np.median(rel))
    assert rel.max() < 1e-11 and np.median(rel) < 1e-13


def test_encounter_free_16384_ten_steps():
    """The capability run of the pair kernel (16,384 bodies, K = 1) for ten
    steps against the oracle's encounter-free map."""
    s = W.planetesimals(16384, seed_index=2)
    gp = _gparams(encounter_free=1)
    sim = G.Simulation(s.m, s.x, s.u, gp, coords="helio")
    sim.step(10)
    sim.check()
    xg, vg = [t.cpu().numpy() for t in sim.state("dem")]
    op = _oparams(gp)
    v0 = O.helio_to_dem(op, s.m, s.u)
    xo, vo = O.free_step(op, s.m, s.x, v0, 10)
    assert _rel_body(xg, xo) < REL and _rel_body(vg, vo) < REL


# --------------------------------------------------------------- full step --
def _run_pair(sysm, x, u, gp, steps):
    sim = G.Simulation(sysm, x, u, gp, coords="helio")
    orc = O.MassiveSim(_oparams(gp), sysm, x, u, coords="helio")
    sim.step(steps)
    orc.step(steps)
    xg, vg = sim.state("dem")
    return sim, orc, xg.cpu().numpy(), vg.cpu().numpy()


def test_plain_n16_ten_steps():
    s = W.plain_n16()
    gp = _gparams()
    sim, orc, xg, vg = _run_pair(s.m, s.x, s.u, gp, 10)
    assert _rel_body(xg, orc.x) < REL
    assert _rel_body(vg, orc.v) < REL
    sim.check()


def test_plain_n16_with_encounters_1000_steps():
    """Energy error statistics of a long run with encounters; states are
    compared over the first 200 steps (before chaotic divergence)."""
    s = W.plain_n16()
    gp = _gparams()
    sim = G.Simulation(s.m, s.x, s.u, gp, coords="helio")
    orc = O.MassiveSim(_oparams(gp), s.m, s.x, s.u, coords="helio")
    E0, _ = sim.energy()
    Eo0, _ = orc.energy()
    assert E0 == pytest.approx(Eo0, rel=1e-14)
    errs, oerrs, enc = [], [], 0
    for k in range(10):
        sim.step(100)
        st = orc.step(100)
        enc += st["enc_total"]
        E, _ = sim.energy()
        Eo, _ = orc.energy()
        errs.append(abs((E - E0) / E0))
        oerrs.append(abs((Eo - Eo0) / Eo0))
        if k == 1:
            xg, vg = sim.state()
            assert _rel_body(xg.cpu().numpy(), orc.x) < 1e-10
    sim.check()
    gs = sim.stats()
    assert gs["enc_total"] > 0 and enc > 0
    assert max(errs) < 1e-8
    _say("n16 |dE/E| gpu max", max(errs), "oracle max", max(oerrs))


def test_planetesimals_n2048_ten_steps_and_sets():
    s = W.planetesimals()
    gp = _gparams()
    sim = G.Simulation(s.m, s.x, s.u, gp, coords="helio")
    orc = O.MassiveSim(_oparams(gp), s.m, s.x, s.u, coords="helio")
    # candidate sets of the initial precheck
    cg, r2g = sim.candidates(with_r2=True)
    co = orc.candidates()
    _say("n2048 candidates gpu/oracle", len(cg), len(co))
    _cand_sets_close(cg, co, orc, r2g=r2g)
    for k in range(10):
        sim.step(1)
        orc.step(1)
        ij, d2, rc2 = sim.encounters()
        _pairs_close(ij, orc.enc, d2, rc2, orc.enc_d2, orc.enc_rc2)
    cg, r2g = sim.candidates(with_r2=True)
    _cand_sets_close(cg, orc.candidates(), orc, r2g=r2g)
    xg, vg = sim.state()
    assert _rel_body(xg.cpu().numpy(), orc.x) < REL
    assert _rel_body(vg.cpu().numpy(), orc.v) < REL
    st = sim.stats()
    # every body's drift of the 10 steps is in the Kepler-iteration histogram
    assert sum(st["kepler_hist"]) == 10 * 2048
    assert max(k for k, c in enumerate(st["kepler_hist"]) if c) == st["kepler_iter_max"]
    _say("n2048 stats", st, "oracle", orc.stats.as_dict())
    if set(map(tuple, ij)) == set(map(tuple, orc.enc)):
        assert st["n_enc"] == orc.stats.n_enc
        assert st["max_group"] == orc.stats.max_group
        assert st["n_groups"] == orc.stats.n_groups
    assert orc.stats.miss_total == 0


@pytest.mark.parametrize("n", [2, 3, 300])
def test_ragged_sizes_ten_steps(n):
    s = W.planetesimals(n, seed_index=40 + n)
    gp = _gparams()
    sim, orc, xg, vg = _run_pair(s.m, s.x, s.u, gp, 10)
    assert _rel_body(xg, orc.x) < REL
    assert _rel_body(vg, orc.v) < REL


def test_dense_encounters_small_system():
    """Strongly interacting bodies: many candidates, groups, BS every step."""
    rng = np.random.default_rng(31)
    n = 24
    m = rng.uniform(1e-6, 1e-5, n)
    a = rng.uniform(0.95, 1.05, n)
    ang = rng.uniform(0, 0.6, n)
    x = np.stack([a * np.cos(ang), a * np.sin(ang), rng.normal(0, 0.002, n)], 1)
    u = np.stack([-np.sin(ang), np.cos(ang), np.zeros(n)], 1) / np.sqrt(a)[:, None]
    gp = _gparams(n2=1.5)
    sim = G.Simulation(m, x, u, gp, coords="helio")
    orc = O.MassiveSim(_oparams(gp), m, x, u, coords="helio")
    for k in range(10):
        sim.step(1)
        orc.step(1)
        ij, d2, rc2 = sim.encounters()
        _pairs_close(ij, orc.enc, d2, rc2, orc.enc_d2, orc.enc_rc2)
    st = sim.stats()
    _say("dense stats", st)
    assert st["enc_total"] > 0 and st["max_group"] >= 3
    # A dense group is chaotic: rounding differences grow over the steps.  The
    # bound is the oracle's own spread under 1-ulp perturbations of the input.
    spread = 0.0
    for seed in (1, 2, 3):
        pr = np.random.default_rng(seed)
        xp = x * (1 + 2.0 ** -52 * pr.choice([-1.0, 1.0], x.shape))
        o2 = O.MassiveSim(_oparams(gp), m, xp, u, coords="helio")
        o2.step(10)
        spread = max(spread, _rel_body(o2.x, orc.x), _rel_body(o2.v, orc.v))
    xg, vg = sim.state()
    dx = _rel_body(xg.cpu().numpy(), orc.x)
    dv = _rel_body(vg.cpu().numpy(), orc.v)
    _say("dense: gpu-oracle", dx, dv, "oracle 1-ulp spread", spread)
    assert max(dx, dv) < max(REL, 10 * spread)


def test_long_candidate_rows():
    """A 5 x 5 x 5 lattice of co-orbiting bodies 1.1 r_crit apart: no
    encounters, but candidate rows of every length class (up to 8, 9-32 and
    beyond 32 partners), so the opening kick sums every kind of row."""
    gp = _gparams(cand_per_body=96)
    rc = gp.n2 * gp.dt * 1.0
    g = (np.arange(5) - 2.0) * 1.1 * rc
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    x = np.stack([1.0 + X.ravel(), Y.ravel(), Z.ravel()], 1)
    r = np.linalg.norm(x[:, :2], axis=1)
    u = np.stack([-x[:, 1], x[:, 0], np.zeros(len(r))], 1) / r[:, None] ** 1.5
    m = np.full(len(r), 1e-9)
    sim = G.Simulation(m, x, u, gp, coords="helio")
    orc = O.MassiveSim(_oparams(gp), m, x, u, coords="helio")
    cnt = np.bincount(orc.candidates()[:, 0], minlength=len(m))
    assert (cnt <= 8).any() and ((cnt > 8) & (cnt <= 32)).any() and (cnt > 32).any()
    for _ in range(4):
        sim.step(1)
        orc.step(1)
        _cand_sets_close(sim.candidates(), orc.candidates(), orc)
    sim.check()
    xg, vg = sim.state()
    assert _rel_body(xg.cpu().numpy(), orc.x) < REL
    assert _rel_body(vg.cpu().numpy(), orc.v) < REL
    assert sim.stats()["full_kicks"] == 0


def test_encounter_free_reversible_on_gpu():
    s = W.plain_n16()
    gp = _gparams(encounter_free=1)
    sim = G.Simulation(s.m, s.x, s.u, gp, coords="helio")
    x0, v0 = sim.state()
    sim.step(40)
    x1, v1 = sim.state()
    gb = _gparams(encounter_free=1, dt=-gp.dt)
    back = G.Simulation(s.m, x1, v1, gb, coords="dem")
    back.step(40)
    x2, v2 = back.state()
    assert _rel_body(x2.cpu().numpy(), x0.cpu().numpy()) < 1e-13
    assert _rel_body(v2.cpu().numpy(), v0.cpu().numpy()) < 1e-13
    # same map as the oracle
    xo, vo = O.free_step(_oparams(gp), s.m, x0.cpu().numpy(), v0.cpu().numpy(), 40)
    assert _rel_body(x1.cpu().numpy(), xo) < REL


def test_energy_and_state_conversions():
    s = W.planetesimals(500, seed_index=7)
    gp = _gparams()
    sim = G.Simulation(s.m, s.x, s.u, gp, coords="helio")
    orc = O.MassiveSim(_oparams(gp), s.m, s.x, s.u, coords="helio")
    E, L = sim.energy()
    Eo, Lo = orc.energy()
    assert E == pytest.approx(Eo, rel=1e-13)
    np.testing.assert_allclose(L, Lo, rtol=1e-13)
    xh, uh = sim.state("helio")
    np.testing.assert_allclose(xh.cpu().numpy(), s.x, rtol=0, atol=1e-15)
    np.testing.assert_allclose(uh.cpu().numpy(), s.u, rtol=0, atol=1e-15)
    # set_state round trip keeps the trajectory
    sim.step(3)
    x3, v3 = sim.state()
    sim.set_state(x3, v3)
    sim.step(2)
    orc.step(5)
    xg, _ = sim.state()
    assert _rel_body(xg.cpu().numpy(), orc.x) < REL


def test_determinism_two_runs():
    s = W.planetesimals(2048)
    gp = _gparams()
    outs = []
    for _ in range(2):
        sim = G.Simulation(s.m, s.x, s.u, gp, coords="helio")
        sim.step(20)
        x, v = sim.state()
        outs.append((x.cpu().numpy(), v.cpu().numpy(), sim.encounters()[0]))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
    assert np.array_equal(outs[0][2], outs[1][2])


def test_profiled_steps_match_graph_steps():
    """The measurement path (kernels launched one by one, the pair kernel
    timed by its own dispatch timestamps) computes the same steps bit for bit."""
    s = W.planetesimals(2048)
    gp = _gparams()
    a = G.Simulation(s.m, s.x, s.u, gp, coords="helio")
    b = G.Simulation(s.m, s.x, s.u, gp, coords="helio")
    a.step(12)
    us = b.step_profiled(12)
    _say("profiled pair kernel us", us)
    assert 0.0 < us < 1e5
    xa, va = a.state()
    xb, vb = b.state()
    assert torch.equal(xa, xb) and torch.equal(va, vb)
    assert a.stats()["steps"] == b.stats()["steps"] == 12


def test_kernel_timed_steps_match_graph_steps():
    """Every kernel of the step timed by its own dispatch timestamps: the
    same steps bit for bit, a positive time for each kernel the mode
    launches, and none for those it does not (encounter-free)."""
    s = W.planetesimals(2048)
    gp = _gparams()
    a = G.Simulation(s.m, s.x, s.u, gp, coords="helio")
    b = G.Simulation(s.m, s.x, s.u, gp, coords="helio")
    a.step(10)
    us = b.step_kernel_us(10)
    _say("kernel us", us)
    assert all(0.0 < v < 1e5 for v in us.values())
    xa, va = a.state()
    xb, vb = b.state()
    assert torch.equal(xa, xb) and torch.equal(va, vb)
    f = G.Simulation(s.m, s.x, s.u, _gparams(encounter_free=1), coords="helio")
    uf = f.step_kernel_us(3)
    assert uf["k_encounter"] == uf["k_group_bs"] == 0.0
    assert uf["k_pair_part"] > 0.0 and uf["k_pair_finish"] > 0.0 and uf["k_open_drift"] > 0.0
    with pytest.raises(G.GengaError):
        f.step_kernel_us(513)


# ----------------------------------------------------------- error paths --
def test_nan_input_rejected():
    s = W.plain_n16()
    x = s.x.copy()
    x[3, 1] = np.nan
    with pytest.raises(G.GengaError) as ei:
        G.Simulation(s.m, x, s.u, _gparams())
    assert ei.value.code == G.EINVAL


def test_candidate_overflow_reported():
    rng = np.random.default_rng(5)
    n = 12
    m = np.full(n, 1e-5)
    x = np.stack([np.ones(n), np.linspace(-0.01, 0.01, n), np.zeros(n)], 1)
    u = np.tile([0.0, 1.0, 0.0], (n, 1))
    gp = _gparams(cand_per_body=1)
    sim = G.Simulation(m, x, u, gp)
    assert sim.sync() == G.EOVERFLOW


def test_kepler_cap_reported():
    s = W.plain_n16()
    sim = G.Simulation(s.m, s.x, s.u, _gparams(kepler_max_iter=1))
    sim.step(1)
    assert sim.sync() == G.EKEPLER


def test_bs_depth_reported():
    rng = np.random.default_rng(6)
    n = 6
    m = np.full(n, 1e-6)
    x = np.stack([np.ones(n), np.linspace(0, 0.02, n), np.zeros(n)], 1)
    u = np.tile([0.0, 1.0, 0.0], (n, 1))
    sim = G.Simulation(m, x, u, _gparams(bs_tol=-1.0, bs_max_depth=2))
    sim.step(1)
    assert sim.sync() == G.EBS


def _cluster(k, spacing, seed):
    """k co-orbiting bodies on an arc `spacing` rad apart (a chain of
    encounters: one group of k members)."""
    rng = np.random.default_rng(seed)
    m = np.full(k, 3e-7)
    ang = 0.3 + spacing * np.arange(k)
    a = 1.0 + 0.0005 * rng.standard_normal(k)
    x = np.stack([a * np.cos(ang), a * np.sin(ang), 1e-4 * rng.standard_normal(k)], 1)
    u = np.stack([-np.sin(ang), np.cos(ang), np.zeros(k)], 1) / np.sqrt(a)[:, None]
    return m, x, u


@pytest.mark.parametrize("k", [2, 7, 8, 9, 12, 64, 65, 100])
def test_bs_group_size_boundaries(k):
    """A tight cluster of k bodies forms one group of k members: groups of up
    to 8 take the all-columns BS path, up to 64 the lane-per-member path,
    larger ones the members-in-chunks path (Sec. 3.2.6's large groups)."""
    m, x, u = _cluster(k, 0.004, 50 + k)
    gp = _gparams(cand_per_body=96 if k >= 64 else 32)
    sim = G.Simulation(m, x, u, gp, coords="helio")
    orc = O.MassiveSim(_oparams(gp), m, x, u, coords="helio")
    osub = 0
    for _ in range(3):
        sim.step(1)
        osub += orc.step(1)["bs_substeps"]
    st = sim.stats()
    _say("group", k, st, orc.stats.as_dict())
    assert st["max_group"] == orc.stats.max_group
    xg, vg = sim.state()
    assert _rel_body(xg.cpu().numpy(), orc.x) < REL
    assert _rel_body(vg.cpu().numpy(), orc.v) < REL
    assert st["bs_substeps"] == osub


def test_many_encounter_pairs_one_large_group():
    """200 bodies 0.002 rad apart on an arc: about 2,300 encounter pairs per
    step (beyond the 2,048 the grouping holds in LDS) chaining into one group
    of 200 members; encounter sets, group size, BS substeps and states against
    the oracle over two steps (a tighter arc makes the oracle's BS exhaust its
    depth in the second step)."""
    m, x, u = _cluster(200, 0.002, 250)
    gp = _gparams(cand_per_body=160)
    sim = G.Simulation(m, x, u, gp, coords="helio")
    orc = O.MassiveSim(_oparams(gp), m, x, u, coords="helio")
    osub = 0
    for _ in range(2):
        sim.step(1)
        osub += orc.step(1)["bs_substeps"]
        ij, d2, rc2 = sim.encounters()
        _say("many pairs: gpu", len(ij), sim.stats(), "oracle", len(orc.enc), orc.stats.as_dict())
        xg, vg = sim.state()
        _say("rel x", _rel_body(xg.cpu().numpy(), orc.x), "v", _rel_body(vg.cpu().numpy(), orc.v))
        _pairs_close(ij, orc.enc, d2, rc2, orc.enc_d2, orc.enc_rc2)
        assert len(ij) > 2048
    st = sim.stats()
    _say("many pairs", st, orc.stats.as_dict())
    assert st["max_group"] == orc.stats.max_group == 200 and st["n_groups"] == 1
    assert st["bs_substeps"] == osub
    xg, vg = sim.state()
    assert _rel_body(xg.cpu().numpy(), orc.x) < REL
    assert _rel_body(vg.cpu().numpy(), orc.v) < REL
