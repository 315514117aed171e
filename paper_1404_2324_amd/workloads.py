"""Seeded synthetic workloads (initial conditions) for the hybrid symplectic
step.  This module only draws inputs: orbital elements from the stated
distributions, converted to heliocentric Cartesian positions and velocities.
It holds none of the integrator's arithmetic and serves both the GPU library
and the CPU oracle.

Units: G = 1, central mass m0 = 1, lengths in AU-like units, so an orbit at
a = 1 has period 2*pi.  The time step is 0.01 of that period.

Element -> Cartesian convention: heliocentric osculating elements with
mu = G (m0 + m_i) for massive bodies and mu = G m0 for test particles.
Random numbers: numpy PCG64 at seed 1404232400 + workload index; angles
(node, argument of pericentre, mean anomaly) uniform on [0, 2 pi);
Rayleigh(sigma) drawn as sigma * sqrt(-2 ln(1 - u)).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 1404232400
TWO_PI = 2.0 * np.pi
DT = 0.01 * TWO_PI


def rng_for(index: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + index))


def rayleigh(rng, sigma, n):
    u = rng.random(n)
    return sigma * np.sqrt(-2.0 * np.log1p(-u))


def _solve_kepler_elliptic(M, e):
    """Eccentric anomaly from the mean anomaly (elliptic orbits, e < 1)."""
    E = np.where(e < 0.8, M, np.pi * np.ones_like(M))
    for _ in range(60):
        dE = (E - e * np.sin(E) - M) / (1.0 - e * np.cos(E))
        E = E - dE
        if np.all(np.abs(dE) < 1e-15):
            break
    return E


def elements_to_cartesian(mu, a, e, inc, node, peri, M):
    """Heliocentric position and velocity from osculating elements
    (elliptic orbits).  All arguments broadcast; returns (x, u) as n x 3."""
    mu = np.broadcast_to(np.asarray(mu, dtype=np.float64), np.shape(a))
    E = _solve_kepler_elliptic(np.mod(M, TWO_PI), e)
    cE, sE = np.cos(E), np.sin(E)
    sq = np.sqrt(1.0 - e * e)
    nmean = np.sqrt(mu / a ** 3)
    xp = a * (cE - e)
    yp = a * sq * sE
    den = 1.0 - e * cE
    vxp = -a * nmean * sE / den
    vyp = a * nmean * sq * cE / den
    cO, sO = np.cos(node), np.sin(node)
    cw, sw = np.cos(peri), np.sin(peri)
    ci, si = np.cos(inc), np.sin(inc)
    # rotation R3(node) R1(inc) R3(peri) applied to the perifocal frame
    P = np.stack([cO * cw - sO * sw * ci, sO * cw + cO * sw * ci, sw * si], -1)
    Q = np.stack([-cO * sw - sO * cw * ci, -sO * sw + cO * cw * ci, cw * si], -1)
    x = xp[:, None] * P + yp[:, None] * Q
    u = vxp[:, None] * P + vyp[:, None] * Q
    return x, u


def _angles(rng, n):
    return rng.random(n) * TWO_PI, rng.random(n) * TWO_PI, rng.random(n) * TWO_PI


@dataclass
class System:
    """One planetary system: heliocentric x, heliocentric velocities u."""
    m: np.ndarray
    x: np.ndarray
    u: np.ndarray
    m0: float = 1.0
    meta: dict = field(default_factory=dict)


def _draw_system(rng, m, a, e, inc, m0=1.0, G=1.0):
    node, peri, M = _angles(rng, len(m))
    x, u = elements_to_cartesian(G * (m0 + m), a, e, inc, node, peri, M)
    return x, u


def plain_n16(seed_index: int = 1) -> System:
    """Main mode, N = 16 equal masses 1e-7, a ~ U(0.5, 1.5), e ~ Ray(0.01),
    i ~ Ray(0.005)."""
    rng = rng_for(seed_index)
    n = 16
    m = np.full(n, 1e-7)
    a = rng.uniform(0.5, 1.5, n)
    e = rayleigh(rng, 0.01, n)
    inc = rayleigh(rng, 0.005, n)
    x, u = _draw_system(rng, m, a, e, inc)
    return System(m, x, u, meta={"workload": "plain_n16", "n": n})


def planetesimals(n: int = 2048, seed_index: int = 2) -> System:
    """Main mode planetesimal disk: masses from dN/dm ~ m^-2 on
    [1e-9, 1e-7] by inverse CDF, a ~ U(0.5, 4), e ~ Ray(0.02),
    i ~ Ray(0.01)."""
    rng = rng_for(seed_index)
    mmin, mmax = 1e-9, 1e-7
    u = rng.random(n)
    m = 1.0 / (1.0 / mmin - u * (1.0 / mmin - 1.0 / mmax))
    a = rng.uniform(0.5, 4.0, n)
    e = rayleigh(rng, 0.02, n)
    inc = rayleigh(rng, 0.01, n)
    x, uu = _draw_system(rng, m, a, e, inc)
    return System(m, x, uu, meta={"workload": f"planetesimals_n{n}", "n": n})


def _planets_tp_mode(rng, n):
    m = np.exp(rng.uniform(np.log(1e-7), np.log(1e-3), n))
    a = rng.uniform(0.4, 5.0, n)
    e = rng.uniform(0.0, 0.05, n)
    inc = rng.uniform(0.0, 0.05, n)
    return m, a, e, inc


def test_particles(ntp: int = 1_000_000, nplanets: int = 8, seed_index: int = 3):
    """Test-particle mode: planets with log-uniform masses in [1e-7, 1e-3],
    a ~ U(0.4, 5), e ~ U(0, 0.05), i ~ U(0, 0.05); massless particles with
    a ~ U(0.3, 5), e ~ U(0, 0.3), i ~ U(0, 0.1).  Returns (planets, xt, ut)
    with heliocentric particle velocities (mu = G m0)."""
    rng = rng_for(seed_index)
    m, a, e, inc = _planets_tp_mode(rng, nplanets)
    x, u = _draw_system(rng, m, a, e, inc)
    at = rng.uniform(0.3, 5.0, ntp)
    et = rng.uniform(0.0, 0.3, ntp)
    it = rng.uniform(0.0, 0.1, ntp)
    node, peri, M = _angles(rng, ntp)
    xt, ut = elements_to_cartesian(1.0, at, et, it, node, peri, M)
    planets = System(m, x, u, meta={"workload": f"tp_{nplanets}p_{ntp}", "n": nplanets})
    return planets, xt, ut


MSUN_G = 1.98847e33
AU_CM = 1.495978707e13


def tp_radii(m, ntp: int, rho_cgs: float = 2.0, r_tp_km: float = 10.0):
    """Physical radii for test-particle mode, planets first: a planet of mass
    m (solar masses) gets the radius of a sphere of bulk density rho_cgs
    (g/cm^3); every particle gets r_tp_km.  Lengths in AU."""
    m = np.asarray(m, dtype=np.float64)
    rp = np.cbrt(3.0 * m * MSUN_G / (4.0 * np.pi * rho_cgs)) / AU_CM
    return np.concatenate([rp, np.full(ntp, r_tp_km * 1e5 / AU_CM)])


def tp_flybys(planets: System, radii, n: int, seed_index: int = 6, d0: float = 0.02,
              bmax: float = 4.0):
    """Test particles aimed at the planets (particle k at planet k mod nm):
    heliocentric start d0 before the planet along a random direction, offset
    sideways by an impact parameter b ~ U(0, bmax) x the planet's radius,
    relative speed ~ U(0.2, 1).  Returns (xt, ut)."""
    rng = rng_for(seed_index)
    nm = len(planets.m)
    j = np.arange(n) % nm
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    e = np.cross(d, rng.standard_normal((n, 3)))
    e /= np.linalg.norm(e, axis=1, keepdims=True)
    b = rng.uniform(0.0, bmax, n) * np.asarray(radii)[j]
    s = rng.uniform(0.2, 1.0, n)
    xt = planets.x[j] - d0 * d + b[:, None] * e
    ut = planets.u[j] + s[:, None] * d
    return xt, ut


def batched(nsys: int = 4096, seed_index: int = 4, nmin: int = 2, nmax: int = 32):
    """Independent systems with N ~ U{nmin..nmax} bodies, masses
    log-uniform in [1e-8, 1e-4], a ~ U(0.3, 3), e, i ~ Ray(0.02).
    Returns (offsets, m0s, m, x, u) with bodies of system s in
    [offsets[s], offsets[s+1])."""
    rng = rng_for(seed_index)
    sizes = rng.integers(nmin, nmax + 1, nsys)
    offsets = np.zeros(nsys + 1, dtype=np.int32)
    offsets[1:] = np.cumsum(sizes)
    nb = int(offsets[-1])
    m = np.exp(rng.uniform(np.log(1e-8), np.log(1e-4), nb))
    a = rng.uniform(0.3, 3.0, nb)
    e = rayleigh(rng, 0.02, nb)
    inc = rayleigh(rng, 0.02, nb)
    node, peri, M = _angles(rng, nb)
    x, u = elements_to_cartesian(1.0 + m, a, e, inc, node, peri, M)
    m0s = np.ones(nsys)
    return offsets, m0s, m, x, u


def adjoint_systems(nsys: int = 1024, nplanets: int = 8, seed_index: int = 5,
                    min_spacing_hill: float = 8.0, min_gap: float = 0.1):
    """Systems of planets drawn as in the test-particle workload, one planet
    at a time: a planet is redrawn until its orbit keeps apart from every
    planet already placed: the inner apocentre and the outer pericentre at
    least `min_spacing_hill` mutual Hill radii and `min_gap` AU apart (so
    that no pair comes near its critical radius and K = 1 holds).  Returns
    (m, x, u) of shape (nsys, nplanets[, 3])."""
    rng = rng_for(seed_index)
    ms, xs, us = [], [], []
    while len(ms) < nsys:
        m = np.zeros(nplanets)
        a = np.zeros(nplanets)
        e = np.zeros(nplanets)
        inc = np.zeros(nplanets)
        k, tries = 0, 0
        while k < nplanets and tries < 200:
            tries += 1
            # 64 candidates at a time; the first that fits is placed
            mc, ac, ec, ic = _planets_tp_mode(rng, 64)
            A, E, Mm = a[None, :k], e[None, :k], m[None, :k]
            inner = A < ac[:, None]
            apo = np.where(inner, A * (1.0 + E), (ac * (1.0 + ec))[:, None])
            peri = np.where(inner, (ac * (1.0 - ec))[:, None], A * (1.0 - E))
            rh = 0.5 * (A + ac[:, None]) * np.cbrt((Mm + mc[:, None]) / 3.0)
            ok = np.all(peri - apo >= np.maximum(min_spacing_hill * rh, min_gap), axis=1)
            hit = np.flatnonzero(ok)
            if hit.size == 0:
                continue
            c = hit[0]
            m[k], a[k], e[k], inc[k] = mc[c], ac[c], ec[c], ic[c]
            k += 1
        if k < nplanets:
            continue
        x, u = _draw_system(rng, m, a, e, inc)
        ms.append(m)
        xs.append(x)
        us.append(u)
    return np.stack(ms), np.stack(xs), np.stack(us)


def encounter_systems(nsys: int = 1024, nplanets: int = 8, seed_index: int = 7,
                      da: float = 0.01, dphase: float = 0.06):
    """Systems of planets packed so that close encounters happen from the
    first step: masses log-uniform in [1e-8, 1e-7], a ~ U(1 - da, 1 + da),
    e ~ Ray(0.005), i ~ Ray(0.001), random node and pericentre, and mean
    longitudes within dphase rad of each other (the radii of Eq. 6 are
    ~0.025 AU, the velocity term, so most pairs start inside their changeover
    zone).  Returns (m, x, u) of shape (nsys, nplanets[, 3])."""
    rng = rng_for(seed_index)
    n = nsys * nplanets
    m = np.exp(rng.uniform(np.log(1e-8), np.log(1e-7), n))
    a = rng.uniform(1.0 - da, 1.0 + da, n)
    e = rayleigh(rng, 0.005, n)
    inc = rayleigh(rng, 0.001, n)
    node = rng.uniform(0.0, 2.0 * np.pi, n)
    peri = rng.uniform(0.0, 2.0 * np.pi, n)
    lam = rng.uniform(0.0, dphase, n)
    M = np.mod(lam - node - peri, 2.0 * np.pi)
    x, u = elements_to_cartesian(1.0 + m, a, e, inc, node, peri, M)
    return (m.reshape(nsys, nplanets), x.reshape(nsys, nplanets, 3),
            u.reshape(nsys, nplanets, 3))


def perturbed(x, u, rel: float = 1e-6, seed_index: int = 1005):
    """Relative Gaussian perturbation of a state (for adjoint targets)."""
    rng = rng_for(seed_index)
    return (x * (1.0 + rel * rng.standard_normal(x.shape)),
            u * (1.0 + rel * rng.standard_normal(u.shape)))
