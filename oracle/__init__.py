"""Plain FP64 CPU oracle for the hybrid symplectic N-body step of Grimm &
Stadel, "The GENGA Code" (arXiv:1404.2324).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  It shares no
code with the GPU library: the arithmetic lives in ``genga_oracle.c``
(compiled with gcc, -ffp-contract=off), this module only marshals numpy
arrays.

Parity status (see the C source for the passage each routine follows):
  changeover K, kick, Sun kick, Kepler drift, Hermite test, grouping,
  energy / angular momentum, tangent-linear model: pinned by closed forms,
  invariants and brute force in ``tests/test_oracle_pins.py``.
  BS sequence / error norm / tolerance, the Hill-radius reading and the
  strictness of the encounter threshold: parity unpinned against the paper
  (readings), pinned only by the physics invariants.
  Derivative of the hybrid step (``genga_cstep.c``, complex step): pinned by
  its real parts (equal to the main-mode step), the tangent-linear model of
  the encounter-free map and central differences of the main-mode step.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "genga_oracle.c")
_SRC_CS = os.path.join(_HERE, "genga_cstep.c")
_LIB = os.path.join(_HERE, "libgenga_oracle.so")

GO_OK, GO_EINVAL, GO_EOVERFLOW, GO_EKEPLER, GO_EBS, GO_EADJ_ENCOUNTER = 0, -1, -3, -4, -5, -6


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/libgenga_oracle.so``."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, _SRC_CS, "-lm"]
        subprocess.check_call(cmd, cwd=_HERE)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [("G", ctypes.c_double), ("m0", ctypes.c_double),
                ("dt", ctypes.c_double), ("n1", ctypes.c_double),
                ("n2", ctypes.c_double), ("pf", ctypes.c_double),
                ("bs_tol", ctypes.c_double), ("bs_max_depth", ctypes.c_int),
                ("kepler_max_iter", ctypes.c_int),
                ("encounter_free", ctypes.c_int), ("pad_", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "steps", "n_cand", "n_enc", "n_miss", "n_groups", "max_group",
        "bs_substeps", "enc_total", "miss_total", "kepler_iter_max",
        "tp_enc", "tp_enc_total", "tp_removed")]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class Event(ctypes.Structure):
    """A merger or an ejection (Sec. 3.2.7, 3.2.8)."""
    _fields_ = [("kind", ctypes.c_int32), ("id_i", ctypes.c_int32), ("id_j", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("step", ctypes.c_int64), ("frac", ctypes.c_double),
                ("m_i", ctypes.c_double), ("m_j", ctypes.c_double), ("R_i", ctypes.c_double),
                ("R_j", ctypes.c_double)] + [
        (f"{q}_{b}", ctypes.c_double * 3) for b in "ij" for q in ("x", "v", "s")] + [
        ("U", ctypes.c_double)]


EV_MERGE, EV_EJECT_FAR, EV_EJECT_SUN = 1, 2, 3
GO_STOPPED = 2


def params(G=1.0, m0=1.0, dt=0.01 * 2 * np.pi, n1=3.0, n2=0.4, pf=3.0,
           bs_tol=1e-13, bs_max_depth=20, kepler_max_iter=40,
           encounter_free=0) -> Params:
    return Params(G, m0, dt, n1, n2, pf, bs_tol, bs_max_depth, kepler_max_iter,
                  encounter_free, 0)


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)
_I64 = ctypes.POINTER(ctypes.c_int64)
_U8 = ctypes.POINTER(ctypes.c_uint8)
_P = ctypes.POINTER(Params)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        i64, i32 = ctypes.c_int64, ctypes.c_int
        sig = {
            "go_set_threads": (None, [i32]),
            "go_threads": (i32, []),
            "go_changeover": (None, [ctypes.c_double, _D, _D]),
            "go_rcrit": (None, [_P, i32, _D, _D, _D, _D]),
            "go_accel": (None, [_P, i32, _D, _D, _D, _D]),
            "go_sun_drift": (None, [_P, i32, _D, _D, _D, ctypes.c_double]),
            "go_kepler": (i32, [ctypes.c_double, _D, _D, ctypes.c_double, _D, _D,
                                i32, ctypes.POINTER(ctypes.c_int)]),
            "go_stumpff": (None, [ctypes.c_double, _D]),
            "go_hermite_dmin2": (ctypes.c_double, [ctypes.c_double, _D, _D, _D, _D]),
            "go_groups": (i32, [i32, i32, _I32, _I32]),
            "go_bs_group": (i32, [_P, i32, _D, _D, _D, _D, ctypes.c_double,
                                  ctypes.POINTER(i64)]),
            "go_energy": (None, [_P, i32, _D, _D, _D, _D, _D]),
            "go_helio_to_dem": (None, [_P, i32, _D, _D]),
            "go_dem_to_helio": (None, [_P, i32, _D, _D]),
            "go_massive_init": (i32, [_P, i32, _D, _D, _D, _D, _U8]),
            "go_massive_step": (i32, [_P, i32, _D, _D, _D, _D, _U8, i64,
                                      ctypes.POINTER(Stats), i32, _I32, _D, _D,
                                      ctypes.POINTER(ctypes.c_int)]),
            "go_tp_init": (i32, [_P, i32, _D, _D, _D, _D, _U8, i64, _D, _D, _U8]),
            "go_tp_step": (i32, [_P, i32, _D, _D, _D, _D, _U8, i64, _D, _D, _U8,
                                 i64, ctypes.POINTER(Stats), _D, i64, _I32, _I64, _D,
                                 _D, _D, _D]),
            "go_massive_step_phys": (i32, [_P, ctypes.POINTER(ctypes.c_int), _D, _D, _D, _D, _U8,
                                           i64, ctypes.POINTER(Stats), _D, _D, _I32,
                                           ctypes.c_double, ctypes.c_double, i32, i64,
                                           ctypes.POINTER(Event), i32,
                                           ctypes.POINTER(ctypes.c_int),
                                           ctypes.POINTER(ctypes.c_double)]),
            "go_merge": (ctypes.c_double, [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                           _D, _D, ctypes.c_double, ctypes.c_double, _D, _D,
                                           _D, _D, _D, _D]),
            "go_composition": (i32, [i32, _D]),
            "go_massive_step_order": (i32, [_P, i32, i32, _D, _D, _D, _D, i64,
                                            ctypes.POINTER(Stats)]),
            "go_free_step": (i32, [_P, i32, _D, _D, _D, i64]),
            "go_free_tlm": (i32, [_P, i32, _D, _D, _D, _D, _D, _D, i64, _D, _D,
                                  _D, _D]),
            "go_free_adjoint": (i32, [_P, i32, _D, _D, _D, i64, _D, _D, _D, _D,
                                      _D]),
            "go_cs_massive": (i32, [_P, i32, _D, _D, _D, _D, _D, _D, ctypes.c_double, i64,
                                    _D, _D, _D, _D, ctypes.POINTER(Stats)]),
            "go_kepler_root": (i32, [ctypes.c_double, _D, _D, ctypes.c_double, i32, _D,
                                     ctypes.POINTER(ctypes.c_int)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_D)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _check(code, what):
    if code != GO_OK:
        raise OracleError(code, what)


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle error {code}")
        self.code = code


def set_threads(n):
    """Threads of the oracle's OpenMP loops; returns the number now used."""
    lib().go_set_threads(int(n))
    return int(lib().go_threads())


def threads():
    return int(lib().go_threads())


# ---------------------------------------------------------------- blocks ---
def changeover(y: float):
    K, dK = ctypes.c_double(), ctypes.c_double()
    lib().go_changeover(float(y), ctypes.byref(K), ctypes.byref(dK))
    return K.value, dK.value


def rcrit(p: Params, m, x, v):
    m, x, v = _f64(m), _f64(x, (-1, 3)), _f64(v, (-1, 3))
    rc = np.zeros(len(m))
    lib().go_rcrit(ctypes.byref(p), len(m), _d(m), _d(x), _d(v), _d(rc))
    return rc


def accel(p: Params, m, x, rc=None):
    m, x = _f64(m), _f64(x, (-1, 3))
    rc = np.zeros(len(m)) if rc is None else _f64(rc)
    acc = np.zeros_like(x)
    lib().go_accel(ctypes.byref(p), len(m), _d(m), _d(x), _d(rc), _d(acc))
    return acc


def sun_drift(p: Params, m, x, v, h):
    m, v = _f64(m), _f64(v, (-1, 3))
    x = _f64(x, (-1, 3)).copy()
    lib().go_sun_drift(ctypes.byref(p), len(m), _d(m), _d(x), _d(v), float(h))
    return x


def kepler(mu, x0, v0, dt, max_iter=40):
    x0, v0 = _f64(x0, (3,)), _f64(v0, (3,))
    x, v = np.zeros(3), np.zeros(3)
    it = ctypes.c_int()
    code = lib().go_kepler(float(mu), _d(x0), _d(v0), float(dt), _d(x), _d(v),
                           int(max_iter), ctypes.byref(it))
    _check(code, "kepler")
    return x, v, it.value


def stumpff(z):
    c = np.zeros(4)
    lib().go_stumpff(float(z), _d(c))
    return c


def hermite_dmin2(dt, dx0, dv0, dx1, dv1):
    a = [_f64(t, (3,)) for t in (dx0, dv0, dx1, dv1)]
    return lib().go_hermite_dmin2(float(dt), *[_d(t) for t in a])


def groups(n, pairs):
    pairs = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    label = np.zeros(n, dtype=np.int32)
    ng = lib().go_groups(int(n), len(pairs), pairs.ctypes.data_as(_I32),
                         label.ctypes.data_as(_I32))
    return ng, label


def bs_group(p: Params, m, rc, x, v, H):
    m, rc = _f64(m), _f64(rc)
    x, v = _f64(x, (-1, 3)).copy(), _f64(v, (-1, 3)).copy()
    sub = ctypes.c_int64()
    code = lib().go_bs_group(ctypes.byref(p), len(m), _d(m), _d(rc), _d(x), _d(v),
                             float(H), ctypes.byref(sub))
    _check(code, "bs_group")
    return x, v, sub.value


def energy(p: Params, m, x, v):
    m, x, v = _f64(m), _f64(x, (-1, 3)), _f64(v, (-1, 3))
    E = ctypes.c_double()
    L = np.zeros(3)
    lib().go_energy(ctypes.byref(p), len(m), _d(m), _d(x), _d(v), ctypes.byref(E), _d(L))
    return E.value, L


def helio_to_dem(p: Params, m, u):
    m, v = _f64(m), _f64(u, (-1, 3)).copy()
    lib().go_helio_to_dem(ctypes.byref(p), len(m), _d(m), _d(v))
    return v


def dem_to_helio(p: Params, m, v):
    m, u = _f64(m), _f64(v, (-1, 3)).copy()
    lib().go_dem_to_helio(ctypes.byref(p), len(m), _d(m), _d(u))
    return u


def merge(G, mi, mj, yi, yj, Ri, Rj, si, sj):
    """The merger of Sec. 3.2.7: (m, y = x and v of the new body, R, spin, U)."""
    yi, yj, si, sj = _f64(yi, (6,)), _f64(yj, (6,)), _f64(si, (3,)), _f64(sj, (3,))
    mo, Ro = ctypes.c_double(), ctypes.c_double()
    yo, so = np.zeros(6), np.zeros(3)
    U = lib().go_merge(float(G), float(mi), float(mj), _d(yi), _d(yj), float(Ri), float(Rj),
                       _d(si), _d(sj), ctypes.byref(mo), _d(yo), ctypes.byref(Ro), _d(so))
    return mo.value, yo, Ro.value, so, U


# ------------------------------------------------------------ main mode ---
class MassiveSim:
    """One planetary system in main mode; state in democratic coordinates.

    radii (optional, one per body) turns on collisions between massive
    bodies (Sec. 3.2.7), rcut / rcut_sun on ejections (Sec. 3.2.8) and nmin
    the stop below that many bodies (Sec. 3.4.6).  Bodies then leave the
    arrays (the last moves into a freed row); ``id`` holds each row's original
    index, ``S`` the spins, ``U`` the internal energy of the mergers and
    ``events`` every merger and ejection."""

    def __init__(self, p: Params, m, x, v, coords="dem", radii=None, rcut=0.0, rcut_sun=0.0,
                 nmin=0):
        self.p = p
        self.m = _f64(m).copy()
        self.x = _f64(x, (-1, 3)).copy()
        v = _f64(v, (-1, 3)).copy()
        if coords == "helio":
            v = helio_to_dem(p, self.m, v)
        self.v = v
        n = len(self.m)
        self.rc = np.zeros(n)
        self.cand = np.zeros((n, n), dtype=np.uint8)
        _check(lib().go_massive_init(ctypes.byref(p), n, _d(self.m), _d(self.x),
                                     _d(self.v), _d(self.rc),
                                     self.cand.ctypes.data_as(_U8)), "massive_init")
        self.stats = Stats()
        self.enc = np.zeros((0, 2), dtype=np.int32)
        self.enc_d2 = np.zeros(0)
        self.enc_rc2 = np.zeros(0)
        self.phys = radii is not None or rcut > 0.0 or rcut_sun > 0.0
        self.R = np.zeros(n) if radii is None else _f64(radii).copy()
        self.S = np.zeros((n, 3))
        self.id = np.arange(n, dtype=np.int32)
        self.rcut, self.rcut_sun, self.nmin = float(rcut), float(rcut_sun), int(nmin)
        self.U = 0.0
        self.events = []
        self.nstep = 0
        self.stopped = False

    @property
    def n(self):
        return len(self.m)

    def _step_phys(self, nsteps):
        n0 = self.n
        nn = ctypes.c_int(n0)
        m, x, v, rc = self.m.copy(), self.x.copy(), self.v.copy(), self.rc.copy()
        R, S, idv = self.R.copy(), self.S.copy(), self.id.copy()
        cap = 4 * n0 + 16
        ev = (Event * cap)()
        nev = ctypes.c_int()
        U = ctypes.c_double(self.U)
        st = Stats()
        code = lib().go_massive_step_phys(
            ctypes.byref(self.p), ctypes.byref(nn), _d(m), _d(x), _d(v), _d(rc),
            self.cand.ctypes.data_as(_U8), int(nsteps), ctypes.byref(st), _d(R), _d(S),
            idv.ctypes.data_as(_I32), self.rcut, self.rcut_sun, self.nmin, self.nstep, ev, cap,
            ctypes.byref(nev), ctypes.byref(U))
        k = nn.value
        self.m, self.x, self.v, self.rc = m[:k], x[:k], v[:k], rc[:k]
        self.R, self.S, self.id = R[:k], S[:k], idv[:k]
        self.cand = np.ascontiguousarray(self.cand.reshape(-1)[:k * k].reshape(k, k))
        self.U = U.value
        self.events += [ev[i] for i in range(min(nev.value, cap))]
        self.nstep += int(st.steps)
        self.stats = st
        if code == GO_STOPPED:
            self.stopped = True
            return st.as_dict()
        _check(code, "massive_step_phys")
        return st.as_dict()

    def candidates(self):
        i, j = np.nonzero(self.cand)
        return np.stack([i, j], 1).astype(np.int32)

    def step(self, nsteps=1, enc_cap=None):
        if self.phys:
            return self._step_phys(nsteps)
        n = self.n
        cap = n * (n - 1) // 2 if enc_cap is None else enc_cap
        ij = np.zeros((max(cap, 1), 2), dtype=np.int32)
        d2 = np.zeros(max(cap, 1))
        rc2 = np.zeros(max(cap, 1))
        ne = ctypes.c_int()
        st = Stats()
        code = lib().go_massive_step(ctypes.byref(self.p), n, _d(self.m), _d(self.x),
                                     _d(self.v), _d(self.rc),
                                     self.cand.ctypes.data_as(_U8), int(nsteps),
                                     ctypes.byref(st), int(cap),
                                     ij.ctypes.data_as(_I32), _d(d2), _d(rc2),
                                     ctypes.byref(ne))
        self.stats = st
        k = min(ne.value, cap)
        self.enc, self.enc_d2, self.enc_rc2 = ij[:k].copy(), d2[:k].copy(), rc2[:k].copy()
        _check(code, "massive_step")
        return st.as_dict()

    def energy(self):
        return energy(self.p, self.m, self.x, self.v)

    def helio_v(self):
        return dem_to_helio(self.p, self.m, self.v)


# --------------------------------------------------- test-particle mode ---
class TPSim:
    """Main-mode massive bodies plus massless test particles.  radii (optional,
    nm + ntp values, planets first) enables collisions: a removed particle's
    x and v become NaN and coll_planet / coll_step / coll_frac / coll_xv hold
    its report (coll_planet = -1 while it is present)."""

    def __init__(self, p: Params, m, x, v, xt, vt, coords="dem", radii=None):
        self.p = p
        self.m = _f64(m).copy()
        self.x = _f64(x, (-1, 3)).copy()
        v = _f64(v, (-1, 3)).copy()
        vt = _f64(vt, (-1, 3)).copy()
        if coords == "helio":
            # barycentric shift of the massive bodies applies to the particles
            u = v.copy()
            v = helio_to_dem(p, self.m, u)
            vt = vt + (v[0] - u[0])
        self.v = v
        self.xt = _f64(xt, (-1, 3)).copy()
        self.vt = vt
        nm, ntp = len(self.m), len(self.xt)
        self.rad = None if radii is None else _f64(radii).copy()
        if self.rad is not None and self.rad.shape != (nm + ntp,):
            raise ValueError("radii: nm + ntp values")
        self.coll_planet = np.full(ntp, -1, dtype=np.int32)
        self.coll_step = np.zeros(ntp, dtype=np.int64)
        self.coll_frac = np.zeros(ntp)
        self.coll_xv = np.zeros((ntp, 6))
        # last step: Hermite minimum and threshold of every tested pair
        self.tp_d2 = np.full((ntp, nm), np.nan)
        self.tp_rc2 = np.full((ntp, nm), np.nan)
        self.nstep = 0
        self.rc = np.zeros(nm)
        self.cand = np.zeros((nm, nm), dtype=np.uint8)
        self.cand_tp = np.zeros((ntp, nm), dtype=np.uint8)
        _check(lib().go_tp_init(ctypes.byref(p), nm, _d(self.m), _d(self.x), _d(self.v),
                                _d(self.rc), self.cand.ctypes.data_as(_U8), ntp,
                                _d(self.xt), _d(self.vt),
                                self.cand_tp.ctypes.data_as(_U8)), "tp_init")
        self.stats = Stats()

    def step(self, nsteps=1):
        st = Stats()
        rad = None if self.rad is None else _d(self.rad)
        code = lib().go_tp_step(ctypes.byref(self.p), len(self.m), _d(self.m), _d(self.x),
                                _d(self.v), _d(self.rc), self.cand.ctypes.data_as(_U8),
                                len(self.xt), _d(self.xt), _d(self.vt),
                                self.cand_tp.ctypes.data_as(_U8), int(nsteps),
                                ctypes.byref(st), rad, self.nstep,
                                self.coll_planet.ctypes.data_as(_I32),
                                self.coll_step.ctypes.data_as(_I64), _d(self.coll_frac),
                                _d(self.coll_xv), _d(self.tp_d2), _d(self.tp_rc2))
        self.stats = st
        self.nstep += int(st.steps)
        _check(code, "tp_step")
        return st.as_dict()

    def removed(self):
        """Indices of the removed particles, ascending."""
        return np.nonzero(self.coll_planet >= 0)[0]

    def tp_encounters(self):
        """Test-particle encounters of the last step (Sec. 3.3): rows
        (particle, planet) with d2 < r_crit,ij^2, sorted, and their d2, rc2."""
        with np.errstate(invalid="ignore"):
            k, j = np.nonzero(self.tp_d2 < self.tp_rc2)
        return (np.stack([k, j], 1).astype(np.int64), self.tp_d2[k, j].copy(),
                self.tp_rc2[k, j].copy())


# ------------------------------------------------------------- batched ---
def batched_run(p: Params, offsets, m0s, m, x, v, nsteps):
    """Independent systems, each run as its own main-mode system with its own
    central mass (the multi-simulation mode of Sec. 3.4)."""
    x = _f64(x, (-1, 3)).copy()
    v = _f64(v, (-1, 3)).copy()
    m = _f64(m)
    stats = []
    for s in range(len(offsets) - 1):
        a, b = int(offsets[s]), int(offsets[s + 1])
        q = Params.from_buffer_copy(p)
        q.m0 = float(m0s[s])
        sim = MassiveSim(q, m[a:b], x[a:b], v[a:b])
        stats.append(sim.step(nsteps))
        x[a:b], v[a:b] = sim.x, sim.v
    return x, v, stats


# ---------------------------------------------------- higher orders ---
def composition(order):
    """Sub-step coefficients w_k of the composed step (Sec. 2.3)."""
    w = np.zeros(7)
    k = lib().go_composition(int(order), _d(w))
    if k == 0:
        raise OracleError(GO_EINVAL, "composition")
    return w[:k].copy()


def step_order(p: Params, order, m, x, v, nsteps):
    """nsteps composed steps of the given order (2, 4, 6) from democratic
    (x, v): each sub-step the full hybrid step with every pair Hermite-tested.
    Returns x, v, the radii of the last sub-step and the counters."""
    m = _f64(m)
    x, v = _f64(x, (-1, 3)).copy(), _f64(v, (-1, 3)).copy()
    rc = np.zeros(len(m))
    st = Stats()
    _check(lib().go_massive_step_order(ctypes.byref(p), int(order), len(m), _d(m), _d(x), _d(v),
                                       _d(rc), int(nsteps), ctypes.byref(st)), "step_order")
    return x, v, rc, st.as_dict()


# ------------------------------------------- encounter-free map + adjoint ---
def free_step(p: Params, m, x, v, nsteps):
    m = _f64(m)
    x, v = _f64(x, (-1, 3)).copy(), _f64(v, (-1, 3)).copy()
    _check(lib().go_free_step(ctypes.byref(p), len(m), _d(m), _d(x), _d(v), int(nsteps)),
           "free_step")
    return x, v


def free_tlm(p: Params, m, x0, v0, dm, dx0, dv0, nsteps):
    m, dm = _f64(m), _f64(dm)
    x0, v0 = _f64(x0, (-1, 3)), _f64(v0, (-1, 3))
    dx0, dv0 = _f64(dx0, (-1, 3)), _f64(dv0, (-1, 3))
    xT, vT = np.zeros_like(x0), np.zeros_like(v0)
    dxT, dvT = np.zeros_like(x0), np.zeros_like(v0)
    _check(lib().go_free_tlm(ctypes.byref(p), len(m), _d(m), _d(x0), _d(v0), _d(dm),
                             _d(dx0), _d(dv0), int(nsteps), _d(xT), _d(vT), _d(dxT),
                             _d(dvT)), "free_tlm")
    return xT, vT, dxT, dvT


def free_adjoint(p: Params, m, x0, v0, nsteps, gxT, gvT):
    m = _f64(m)
    x0, v0 = _f64(x0, (-1, 3)), _f64(v0, (-1, 3))
    gxT, gvT = _f64(gxT, (-1, 3)), _f64(gvT, (-1, 3))
    gx0, gv0, gm = np.zeros_like(x0), np.zeros_like(v0), np.zeros_like(m)
    _check(lib().go_free_adjoint(ctypes.byref(p), len(m), _d(m), _d(x0), _d(v0),
                                 int(nsteps), _d(gxT), _d(gvT), _d(gx0), _d(gv0),
                                 _d(gm)), "free_adjoint")
    return gx0, gv0, gm


# ------------------- derivative of the hybrid step (complex step) ---
def cs_massive(p: Params, m, x0, v0, dm, dx0, dv0, nsteps, h=1e-30):
    """nsteps steps of the main-mode step (as MassiveSim.step, no collisions)
    from democratic (x0, v0) and their derivative along (dm, dx0, dv0), with
    every decision of the run (candidates, encounters, groups, BS acceptance
    and halving, Kepler stopping) held fixed: the complex-step derivative of
    genga_cstep.c.  Returns xT, vT (equal to the real run's), dxT, dvT and
    the counters."""
    m = _f64(m)
    x0, v0 = _f64(x0, (-1, 3)), _f64(v0, (-1, 3))
    dm = _f64(dm) if dm is not None else np.zeros_like(m)
    dx0 = _f64(dx0, (-1, 3)) if dx0 is not None else np.zeros_like(x0)
    dv0 = _f64(dv0, (-1, 3)) if dv0 is not None else np.zeros_like(v0)
    xT, vT = np.zeros_like(x0), np.zeros_like(v0)
    dxT, dvT = np.zeros_like(x0), np.zeros_like(v0)
    st = Stats()
    _check(lib().go_cs_massive(ctypes.byref(p), len(m), _d(m), _d(x0), _d(v0), _d(dm), _d(dx0),
                               _d(dv0), float(h), int(nsteps), _d(xT), _d(vT), _d(dxT), _d(dvT),
                               ctypes.byref(st)), "cs_massive")
    return xT, vT, dxT, dvT, st.as_dict()


def cs_gradient(p: Params, m, x0, v0, nsteps, gxT, gvT):
    """Gradient of L with dL/dx_T = gxT, dL/dv_T = gvT with respect to
    (x0, v0, m) through nsteps hybrid steps, one directional derivative per
    input coordinate (7 n runs of cs_massive: small systems only)."""
    m = _f64(m)
    x0, v0 = _f64(x0, (-1, 3)), _f64(v0, (-1, 3))
    gxT, gvT = _f64(gxT, (-1, 3)), _f64(gvT, (-1, 3))
    n = len(m)
    gx, gv, gm = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros(n)
    for which, out in ((0, gx), (1, gv), (2, gm)):
        for idx in np.ndindex(out.shape):
            d = [None, None, None]
            e = np.zeros(out.shape)
            e[idx] = 1.0
            d[which] = e
            _, _, dxT, dvT, _ = cs_massive(p, m, x0, v0, d[2], d[0], d[1], nsteps)
            out[idx] = np.sum(gxT * dxT) + np.sum(gvT * dvT)
    return gx, gv, gm
