"""GPU reverse-mode gradient of the encounter-free map (K = 1) against the
oracle: its forward map, its adjoint (built from its tangent-linear model),
the dot-product identity with that model (2e-12 relative; observed at most
7e-13), and central finite differences through the GPU forward map.
Gradients: 1e-9 of the largest component (the two sides accumulate
thousands of rounding steps in different orders; observed 2e-13); states:
1e-12 relative."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1404_2324_amd import genga as G
from paper_1404_2324_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _systems(nsys, seed_index=5):
    m, x, u = W.adjoint_systems(nsys=nsys, nplanets=8, seed_index=seed_index)
    p = O.params(encounter_free=1)
    v = np.stack([O.helio_to_dem(p, m[s], u[s]) for s in range(nsys)])
    off = np.arange(0, 8 * nsys + 1, 8, dtype=np.int32)
    return off, np.ones(nsys), m.reshape(-1), x.reshape(-1, 3), v.reshape(-1, 3)


def _gp():
    return G.default_params(encounter_free=1)


def test_adjoint_forward_and_gradients_match_oracle():
    nsys, T, K = 12, 100, 32          # ragged last segment: 3 x 32 + 4
    off, m0s, m, x, v = _systems(nsys)
    rng = np.random.default_rng(21)
    gxT = rng.standard_normal(x.shape)
    gvT = rng.standard_normal(v.shape)
    sim = G.BatchedSimulation(off, m0s, m, x, v, _gp(), coords="dem")
    sim.adj_forward(T, K)
    sim.check()
    xT, vT = [t.cpu().numpy() for t in sim.state("dem")]
    gx0, gv0, gm = [t.cpu().numpy() for t in sim.adj_backward(gxT, gvT)]
    sim.check()
    p = O.params(encounter_free=1)
    worst = 0.0
    for s in range(nsys):
        a, b = off[s], off[s + 1]
        xo, vo = O.free_step(p, m[a:b], x[a:b], v[a:b], T)
        assert np.abs(xT[a:b] - xo).max() <= 1e-12 * np.abs(xo).max()
        assert np.abs(vT[a:b] - vo).max() <= 1e-12 * np.abs(vo).max()
        ox, ov, om = O.free_adjoint(p, m[a:b], x[a:b], v[a:b], T, gxT[a:b], gvT[a:b])
        for g, o in ((gx0[a:b], ox), (gv0[a:b], ov), (gm[a:b], om)):
            err = np.abs(g - o).max() / np.abs(o).max()
            worst = max(worst, err)
            assert err < 1e-9, f"system {s}: {err:.3e}"
    _say("adjoint vs oracle worst", worst)


def test_adjoint_dot_product_with_oracle_tlm():
    nsys, T, K = 4, 64, 16
    off, m0s, m, x, v = _systems(nsys, seed_index=6)
    rng = np.random.default_rng(22)
    lx, lv = rng.standard_normal(x.shape), rng.standard_normal(v.shape)
    dx, dv = rng.standard_normal(x.shape), rng.standard_normal(v.shape)
    dm = rng.standard_normal(m.shape) * m
    sim = G.BatchedSimulation(off, m0s, m, x, v, _gp(), coords="dem")
    sim.adj_forward(T, K)
    gx0, gv0, gm = [t.cpu().numpy() for t in sim.adj_backward(lx, lv)]
    p = O.params(encounter_free=1)
    for s in range(nsys):
        a, b = off[s], off[s + 1]
        _, _, dxT, dvT = O.free_tlm(p, m[a:b], x[a:b], v[a:b], dm[a:b], dx[a:b], dv[a:b], T)
        lhs = np.sum(dxT * lx[a:b]) + np.sum(dvT * lv[a:b])
        rhs = np.sum(dx[a:b] * gx0[a:b]) + np.sum(dv[a:b] * gv0[a:b]) + np.sum(dm[a:b] * gm[a:b])
        rel = abs(lhs - rhs) / max(abs(lhs), 1e-300)
        _say("dot product system", s, "relative difference", rel)
        assert rel <= 2e-12, (s, lhs, rhs)


def test_autograd_loss_against_finite_differences():
    """L = sum |x_T - x_target|^2 through torch.autograd; directional
    derivatives by central differences of the GPU forward map (h = 1e-8
    relative: the residual x_T - x_target is only ~1e-6, so a step of that
    size would leave a truncation error of order h^2 / 1e-6), over 200
    steps with a checkpoint every 32."""
    nsys, T = 8, 200
    off, m0s, m, x, v = _systems(nsys, seed_index=7)
    rng = np.random.default_rng(23)
    # the target: the map run from initial conditions perturbed by 1e-6
    # (relative, normal) in position and velocity
    xp = x * (1.0 + 1e-6 * rng.standard_normal(x.shape))
    vp = v * (1.0 + 1e-6 * rng.standard_normal(v.shape))
    with torch.no_grad():
        tgt, _ = G.encounter_free_map(torch.tensor(xp, device="cuda"), torch.tensor(vp, device="cuda"),
                                      torch.tensor(m, device="cuda"), off, m0s, T, 32)
    tgt = tgt.detach().clone()
    x0 = torch.tensor(x, device="cuda", requires_grad=True)
    v0 = torch.tensor(v, device="cuda", requires_grad=True)
    mm = torch.tensor(m, device="cuda", requires_grad=True)

    def loss(xa, va, ma):
        xT, _ = G.encounter_free_map(xa, va, ma, off, m0s, T, 32)
        return ((xT - tgt) ** 2).sum()

    L = loss(x0, v0, mm)
    L.backward()
    grads = (x0.grad.cpu().numpy(), v0.grad.cpu().numpy(), mm.grad.cpu().numpy())
    with torch.no_grad():
        for k in range(3):
            d = [rng.standard_normal(x.shape) * np.abs(x), rng.standard_normal(v.shape) * np.abs(v),
                 rng.standard_normal(m.shape) * m]
            if k < 2:
                d[2] = np.zeros_like(m)      # position / velocity directions
            if k == 0:
                d[1] = np.zeros_like(v)
            h = 1e-8
            args_p = [torch.tensor(b + h * e, device="cuda") for b, e in zip((x, v, m), d)]
            args_m = [torch.tensor(b - h * e, device="cuda") for b, e in zip((x, v, m), d)]
            fd = (float(loss(*args_p)) - float(loss(*args_m))) / (2 * h)
            an = sum(float(np.sum(g * e)) for g, e in zip(grads, d))
            _say("direction", k, "adjoint", an, "fd", fd)
            assert abs(an - fd) <= 1e-5 * max(abs(fd), 1e-30)


def test_adjoint_flags_pairs_inside_rcrit():
    off, m0s, m, x, v = _systems(2, seed_index=8)
    x = x.copy()
    x[1] = x[0] * (1.0 + 1e-3)       # two planets of system 0 almost together
    sim = G.BatchedSimulation(off, m0s, m, x, v, _gp(), coords="dem")
    sim.adj_forward(4, 2)
    with pytest.raises(G.GengaError) as ei:
        sim.check()
    assert ei.value.code == G.EADJ_ENCOUNTER


def test_adjoint_full_workload_sampled():
    """1024 systems x 8 planets, 1000 steps, checkpoint every 32; the oracle's
    adjoint for four of the systems."""
    nsys, T, K = 1024, 1000, 32
    off, m0s, m, x, v = _systems(nsys)
    rng = np.random.default_rng(24)
    gxT = rng.standard_normal(x.shape)
    gvT = np.zeros_like(v)
    sim = G.BatchedSimulation(off, m0s, m, x, v, _gp(), coords="dem")
    sim.adj_forward(T, K)
    gx0, gv0, gm = [t.cpu().numpy() for t in sim.adj_backward(gxT, gvT)]
    sim.check()
    p = O.params(encounter_free=1)
    for s in (0, 333, 700, 1023):
        a, b = off[s], off[s + 1]
        ox, ov, om = O.free_adjoint(p, m[a:b], x[a:b], v[a:b], T, gxT[a:b], gvT[a:b])
        for g, o in ((gx0[a:b], ox), (gv0[a:b], ov), (gm[a:b], om)):
            assert np.abs(g - o).max() / np.abs(o).max() < 1e-8


def test_encounter_free_map_reuses_its_context():
    """Two forward/backward passes of the autograd map on different inputs
    take the same context (no new init) and give the same bits as fresh
    contexts; the caller's parameters are left as they were."""
    nsys, T = 6, 70
    off, m0s, m, x, v = _systems(nsys, seed_index=9)
    rng = np.random.default_rng(25)
    gp = G.default_params()
    G._EF_IDLE.clear()
    seen = []
    for scale in (1.0, 1.0 + 1e-7):
        xs, vs, ms = x * scale, v, m * scale
        x0 = torch.tensor(xs, device="cuda", requires_grad=True)
        v0 = torch.tensor(vs, device="cuda", requires_grad=True)
        m0 = torch.tensor(ms, device="cuda", requires_grad=True)
        gxT = torch.tensor(rng.standard_normal(x.shape), device="cuda")
        xT, vT = G.encounter_free_map(x0, v0, m0, off, m0s, T, 16, gp)
        (xT * gxT).sum().backward()
        pool = [s for lst in G._EF_IDLE.values() for s in lst]
        assert len(pool) == 1
        seen.append(id(pool[0]))
        ref = G.BatchedSimulation(off, m0s, ms, xs, vs, G.default_params(encounter_free=1),
                                  coords="dem")
        ref.adj_forward(T, 16)
        rx, rv = ref.state("dem")
        gx, gv, gm = ref.adj_backward(gxT, torch.zeros_like(gxT))
        ref.check()
        assert torch.equal(xT.detach(), rx) and torch.equal(vT.detach(), rv)
        assert torch.equal(x0.grad, gx) and torch.equal(v0.grad, gv) and torch.equal(m0.grad, gm)
        ref.close()
    assert seen[0] == seen[1]
    assert gp.encounter_free == 0
