"""ctypes binding of the C ABI in ``include/genga.h``.

Argument marshalling only: every step of the integration runs in the gfx950
kernels of ``libgenga.so``.  PyTorch supplies device memory and the stream.
If the library is missing this module raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgenga.so")

GENGA_MASSIVE, GENGA_TEST, GENGA_BATCH = 0, 1, 2
GENGA_HELIO, GENGA_DEMOCRATIC = 0, 1
OK, EINVAL, EHIP, EOVERFLOW, EKEPLER, EBS, EADJ_ENCOUNTER, ENOMEM, EGROUP = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
WSTOPPED = 1  # warning: batched systems stopped after a failed step
KEPLER_BINS = 16  # GENGA_KEPLER_BINS


class GengaError(RuntimeError):
    def __init__(self, code, what):
        msg = lib().genga_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("G", ctypes.c_double), ("m0", ctypes.c_double), ("dt", ctypes.c_double),
                ("n1", ctypes.c_double), ("n2", ctypes.c_double), ("pf", ctypes.c_double),
                ("bs_tol", ctypes.c_double), ("bs_max_depth", ctypes.c_int32),
                ("kepler_max_iter", ctypes.c_int32), ("encounter_free", ctypes.c_int32),
                ("cand_per_body", ctypes.c_int32), ("enc_cap", ctypes.c_int32),
                ("order", ctypes.c_int32), ("rcut", ctypes.c_double),
                ("rcut_sun", ctypes.c_double), ("nmin", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Event(ctypes.Structure):
    """A merger or an ejection (genga_event)."""
    _fields_ = [("kind", ctypes.c_int32), ("sys", ctypes.c_int32), ("id_i", ctypes.c_int32),
                ("id_j", ctypes.c_int32), ("step", ctypes.c_int64), ("frac", ctypes.c_double),
                ("m_i", ctypes.c_double), ("m_j", ctypes.c_double), ("R_i", ctypes.c_double),
                ("R_j", ctypes.c_double)] + [
        (f"{q}_{b}", ctypes.c_double * 3) for b in "ij" for q in ("x", "v", "s")] + [
        ("U", ctypes.c_double)]


EV_MERGE, EV_EJECT_FAR, EV_EJECT_SUN = 1, 2, 3
WNMIN = 2  # batched system status: fewer than nmin bodies left


class Stats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("n_cand", ctypes.c_int32),
                ("n_enc", ctypes.c_int32), ("n_groups", ctypes.c_int32),
                ("max_group", ctypes.c_int32), ("kepler_iter_max", ctypes.c_int32),
                ("tp_enc", ctypes.c_int32), ("bs_substeps", ctypes.c_int64),
                ("enc_total", ctypes.c_int64), ("full_kicks", ctypes.c_int64),
                ("tp_enc_total", ctypes.c_int64), ("tp_removed", ctypes.c_int64),
                ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32),
                ("kepler_hist", ctypes.c_int64 * KEPLER_BINS)]

    def as_dict(self):
        d = {k: int(getattr(self, k)) for k, _ in self._fields_
             if k not in ("reserved", "kepler_hist")}
        d["kepler_hist"] = [int(v) for v in self.kepler_hist]
        return d


# every symbol the header declares, with its ctypes signature
_vp, _i32, _i64, _d, _sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
_PP = ctypes.POINTER(Params)
SIGNATURES = {
    "genga_params_default": (None, [_PP]),
    "genga_workspace_bytes": (_sz, [_i32, _PP, _i32, _i64, _i32, _i64]),
    "genga_init": (_i32, [ctypes.POINTER(_vp), _i32, _PP, _i32, _i64, _i32, _vp, _vp, _vp, _vp,
                          _vp, _i32, _vp, _sz, _vp]),
    "genga_step": (_i32, [_vp, _i64]),
    "genga_sync": (_i32, [_vp]),
    "genga_step_profiled": (_i32, [_vp, _i64, ctypes.POINTER(ctypes.c_double)]),
    "genga_step_kernel_us": (_i32, [_vp, _i64, ctypes.POINTER(ctypes.c_double)]),
    "genga_get_state": (_i32, [_vp, _vp, _vp, _i32]),
    "genga_set_state": (_i32, [_vp, _vp, _vp, _i32]),
    "genga_set_masses": (_i32, [_vp, _vp]),
    "genga_energy": (_i32, [_vp, _vp, _vp]),
    "genga_accel_state": (_i32, [_vp, _vp]),
    "genga_encounters": (_i32, [_vp, _vp, _vp, _vp, _i32, ctypes.POINTER(_i32)]),
    "genga_candidates": (_i32, [_vp, _vp, _vp, _i32, ctypes.POINTER(_i32)]),
    "genga_tp_encounters": (_i32, [_vp, _vp, _vp, _vp, _vp, _i64, ctypes.POINTER(_i64)]),
    "genga_stats": (_i32, [_vp, ctypes.POINTER(Stats)]),
    "genga_set_radii": (_i32, [_vp, _vp]),
    "genga_tune": (_i32, [_vp, _i32, _vp, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "genga_tune_variant": (ctypes.c_char_p, [_i32]),
    "genga_batch_set_variant": (_i32, [_vp, _i32]),
    "genga_batch_status": (_i32, [_vp, _vp, _vp, _i32]),
    "genga_events": (_i32, [_vp, ctypes.POINTER(Event), _i64, ctypes.POINTER(_i64)]),
    "genga_bodies": (_i32, [_vp, _vp, _i64, _vp, _vp, _i32]),
    "genga_adj_buffer_bytes": (_sz, [_vp, _i64, _i32]),
    "genga_adj_forward": (_i32, [_vp, _i64, _i32, _vp, _sz]),
    "genga_adj_backward": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "genga_collisions": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _i64, ctypes.POINTER(_i64)]),
    "genga_strerror": (ctypes.c_char_p, [_i32]),
    "genga_destroy": (_i32, [_vp]),
    "genga_accel_workspace_bytes": (_sz, [_i32]),
    "genga_accel": (_i32, [_PP, _i32, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "genga_accel_noalloc": (_i32, [_PP, _i32, _vp, _vp, _vp, _vp, _vp]),
    "genga_kepler": (_i32, [_d, _i64, _vp, _vp, _d, _vp, _vp, _i32, _vp, _vp]),
    "genga_hermite": (_i32, [_i64, _d, _vp, _vp, _vp]),
}

_lib = None


def lib():
    """Load libgenga.so (raises when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(code, what):
    """Errors are negative; positive codes are warnings (see check())."""
    if code < 0:
        raise GengaError(code, what)


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev(a, device, dtype=torch.float64):
    t = torch.as_tensor(a, dtype=dtype)
    return t.to(device).contiguous()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def default_params(**kw) -> Params:
    p = Params()
    lib().genga_params_default(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


class Simulation:
    """Main-mode system on one GPU.  State stays in the library's workspace;
    ``state()`` returns fresh device tensors."""

    def __init__(self, m, x, v, params: Params | None = None, coords: str = "helio",
                 device="cuda", stream=None):
        self.p = params if params is not None else default_params()
        self.device = torch.device(device)
        self.stream = stream
        m = _dev(m, self.device)
        x = _dev(x, self.device).reshape(-1, 3)
        v = _dev(v, self.device).reshape(-1, 3)
        self.n = int(m.numel())
        nbytes = lib().genga_workspace_bytes(GENGA_MASSIVE, ctypes.byref(self.p), self.n, 0, 0, 0)
        if nbytes == 0:
            raise GengaError(EINVAL, "genga_workspace_bytes")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._ctx = ctypes.c_void_p()
        code = lib().genga_init(ctypes.byref(self._ctx), GENGA_MASSIVE, ctypes.byref(self.p),
                                self.n, 0, 0, None, None, _ptr(m), _ptr(x), _ptr(v),
                                GENGA_HELIO if coords == "helio" else GENGA_DEMOCRATIC,
                                _ptr(self.ws), nbytes, _stream(stream))
        _check(code, "genga_init")

    def step(self, nsteps: int = 1):
        _check(lib().genga_step(self._ctx, int(nsteps)), "genga_step")

    def step_profiled(self, nsteps: int):
        """Run nsteps steps launch by launch; returns the closing-kick pair
        kernel's average duration in microseconds (HIP events)."""
        us = ctypes.c_double()
        _check(lib().genga_step_profiled(self._ctx, int(nsteps), ctypes.byref(us)),
               "genga_step_profiled")
        return us.value

    STEP_KERNELS = ("k_open_drift", "k_encounter", "k_group_bs", "k_pair_part",
                    "k_pair_finish")

    def step_kernel_us(self, nsteps: int) -> dict:
        """Run nsteps steps with every kernel timed (HIP events on the
        dispatches); returns each kernel's average duration in microseconds,
        in launch order."""
        us = (ctypes.c_double * len(self.STEP_KERNELS))()
        _check(lib().genga_step_kernel_us(self._ctx, int(nsteps), us), "genga_step_kernel_us")
        return dict(zip(self.STEP_KERNELS, list(us)))

    def sync(self):
        return lib().genga_sync(self._ctx)

    def check(self):
        """Raise on a latched error; return the status (warnings are > 0)."""
        code = self.sync()
        if code < 0:
            _check(code, "device status")
        return code

    def state(self, coords: str = "dem"):
        x = torch.empty((self.n, 3), dtype=torch.float64, device=self.device)
        v = torch.empty_like(x)
        code = lib().genga_get_state(self._ctx, _ptr(x), _ptr(v),
                                     GENGA_HELIO if coords == "helio" else GENGA_DEMOCRATIC)
        _check(code, "genga_get_state")
        return x, v

    def set_state(self, x, v, coords: str = "dem"):
        x = _dev(x, self.device).reshape(-1, 3)
        v = _dev(v, self.device).reshape(-1, 3)
        code = lib().genga_set_state(self._ctx, _ptr(x), _ptr(v),
                                     GENGA_HELIO if coords == "helio" else GENGA_DEMOCRATIC)
        _check(code, "genga_set_state")

    def energy(self):
        E = torch.empty(1, dtype=torch.float64, device=self.device)
        L = torch.empty(3, dtype=torch.float64, device=self.device)
        _check(lib().genga_energy(self._ctx, _ptr(E), _ptr(L)), "genga_energy")
        torch.cuda.synchronize(self.device)
        return float(E[0]), L.cpu().numpy()

    def accel_state(self, out=None):
        """H_B acceleration of the current state (pair kernel only)."""
        if out is None:
            out = torch.empty((self.n, 3), dtype=torch.float64, device=self.device)
        _check(lib().genga_accel_state(self._ctx, _ptr(out)), "genga_accel_state")
        return out

    def encounters(self):
        n = ctypes.c_int()
        code = lib().genga_encounters(self._ctx, None, None, None, 0, ctypes.byref(n))
        if code not in (OK, EOVERFLOW):
            _check(code, "genga_encounters")
        cap = max(n.value, 1)
        ij = np.zeros((cap, 2), dtype=np.int32)
        d2 = np.zeros(cap)
        rc2 = np.zeros(cap)
        code = lib().genga_encounters(self._ctx, ij.ctypes.data_as(_vp), d2.ctypes.data_as(_vp),
                                      rc2.ctypes.data_as(_vp), cap, ctypes.byref(n))
        _check(code, "genga_encounters")
        k = n.value
        return ij[:k], d2[:k], rc2[:k]

    def candidates(self, with_r2: bool = False):
        """Prechecker pairs i < j entering the next step (and r_ij^2)."""
        n = ctypes.c_int()
        code = lib().genga_candidates(self._ctx, None, None, 0, ctypes.byref(n))
        if code not in (OK, EOVERFLOW):
            _check(code, "genga_candidates")
        cap = max(n.value, 1)
        ij = np.zeros((cap, 2), dtype=np.int32)
        r2 = np.zeros(cap)
        _check(lib().genga_candidates(self._ctx, ij.ctypes.data_as(_vp), r2.ctypes.data_as(_vp),
                                      cap, ctypes.byref(n)), "genga_candidates")
        k = n.value
        return (ij[:k], r2[:k]) if with_r2 else ij[:k]

    def stats(self, check: bool = True):
        s = Stats()
        code = lib().genga_stats(self._ctx, ctypes.byref(s))
        if check:
            _check(code, "genga_stats")
        return s.as_dict()

    def set_radii(self, radii):
        """Physical radii, one per row: collisions between massive bodies
        (Sec. 3.2.7; main and batched mode)."""
        r = _dev(radii, self.device).reshape(-1).contiguous()
        if r.numel() != self.n:
            raise ValueError("radii: one per row")
        _check(lib().genga_set_radii(self._ctx, _ptr(r)), "genga_set_radii")

    def events(self):
        """Every merger and ejection since init, sorted (list of Event)."""
        n = ctypes.c_int64()
        code = lib().genga_events(self._ctx, None, 0, ctypes.byref(n))
        if code not in (OK, EOVERFLOW) and code < 0:
            _check(code, "genga_events")
        k = int(n.value)
        buf = (Event * max(k, 1))()
        _check(lib().genga_events(self._ctx, buf, max(k, 1), ctypes.byref(n)), "genga_events")
        return [buf[i] for i in range(k)]

    def bodies(self):
        """(original row per row, -1 past a system's count; bodies left per
        system; internal energy U of each system's mergers)."""
        nsys = getattr(self, "nsys", 1)
        ids = np.zeros(self.n, dtype=np.int32)
        nl = np.zeros(nsys, dtype=np.int32)
        U = np.zeros(nsys)
        _check(lib().genga_bodies(self._ctx, ids.ctypes.data, self.n, nl.ctypes.data,
                                  U.ctypes.data, nsys), "genga_bodies")
        return ids, nl, U

    def close(self):
        if getattr(self, "_ctx", None):
            lib().genga_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def accel(params: Params, m, x, rc=None, device="cuda", stream=None):
    """H_B acceleration of every body (the kick's pair sum)."""
    dev = torch.device(device)
    m = _dev(m, dev)
    x = _dev(x, dev).reshape(-1, 3)
    n = int(m.numel())
    rct = _dev(rc, dev) if rc is not None else None
    out = torch.empty((n, 3), dtype=torch.float64, device=dev)
    nb = lib().genga_accel_workspace_bytes(n)
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
    _check(lib().genga_accel(ctypes.byref(params), n, _ptr(m), _ptr(x), _ptr(rct), _ptr(out),
                             _ptr(ws), nb, _stream(stream)), "genga_accel")
    return out


def kepler(mu, x0, v0, dt, max_iter=40, device="cuda", stream=None):
    """Kepler drift of independent bodies; returns x, v, iteration counts."""
    dev = torch.device(device)
    x0 = _dev(x0, dev).reshape(-1, 3)
    v0 = _dev(v0, dev).reshape(-1, 3)
    n = x0.shape[0]
    x = torch.empty_like(x0)
    v = torch.empty_like(v0)
    it = torch.empty(n, dtype=torch.int32, device=dev)
    _check(lib().genga_kepler(float(mu), n, _ptr(x0), _ptr(v0), float(dt), _ptr(x), _ptr(v),
                              int(max_iter), _ptr(it), _stream(stream)), "genga_kepler")
    return x, v, it


def hermite(dt, q, device="cuda", stream=None):
    """Hermite minimum squared separation for rows (dx0, dv0, dx1, dv1)."""
    dev = torch.device(device)
    q = _dev(q, dev).reshape(-1, 12)
    out = torch.empty(q.shape[0], dtype=torch.float64, device=dev)
    _check(lib().genga_hermite(q.shape[0], float(dt), _ptr(q), _ptr(out), _stream(stream)),
           "genga_hermite")
    return out


class TestParticleSimulation(Simulation):
    """Test-particle mode: up to 32 massive bodies plus massless particles
    (row order: massive bodies first, then particles).  radii (optional,
    n_massive + n_test values) turns on removal by collision."""

    def __init__(self, m, x, v, xt, vt, params: Params | None = None, coords: str = "helio",
                 device="cuda", stream=None, radii=None):
        self.p = params if params is not None else default_params()
        self.device = torch.device(device)
        self.stream = stream
        m = _dev(m, self.device)
        self.nm = int(m.numel())
        xa = torch.cat([_dev(x, self.device).reshape(-1, 3), _dev(xt, self.device).reshape(-1, 3)])
        va = torch.cat([_dev(v, self.device).reshape(-1, 3), _dev(vt, self.device).reshape(-1, 3)])
        self.ntp = xa.shape[0] - self.nm
        self.n = xa.shape[0]
        nbytes = lib().genga_workspace_bytes(GENGA_TEST, ctypes.byref(self.p), self.nm, self.ntp, 0, 0)
        if nbytes == 0:
            raise GengaError(EINVAL, "genga_workspace_bytes")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._ctx = ctypes.c_void_p()
        code = lib().genga_init(ctypes.byref(self._ctx), GENGA_TEST, ctypes.byref(self.p), self.nm,
                                self.ntp, 0, None, None, _ptr(m), _ptr(xa.contiguous()),
                                _ptr(va.contiguous()),
                                GENGA_HELIO if coords == "helio" else GENGA_DEMOCRATIC,
                                _ptr(self.ws), nbytes, _stream(stream))
        _check(code, "genga_init")
        if radii is not None:
            self.set_radii(radii)

    def set_radii(self, radii):
        r = _dev(radii, self.device).reshape(-1).contiguous()
        if r.numel() != self.n:
            raise ValueError("radii: n_massive + n_test values")
        _check(lib().genga_set_radii(self._ctx, _ptr(r)), "genga_set_radii")

    def collisions(self):
        """Removal reports since init, sorted by (step, particle): a dict of
        numpy arrays tp, planet, step, frac and xv (n x 6, democratic)."""
        n = ctypes.c_int64()
        code = lib().genga_collisions(self._ctx, None, None, None, None, None, 0, ctypes.byref(n))
        if code not in (OK, EOVERFLOW):
            _check(code, "genga_collisions")
        k = int(n.value)
        tp = np.zeros(k, dtype=np.int64)
        pl = np.zeros(k, dtype=np.int32)
        stp = np.zeros(k, dtype=np.int64)
        fr = np.zeros(k)
        xv = np.zeros((k, 6))
        if k:
            _check(lib().genga_collisions(self._ctx, tp.ctypes.data, pl.ctypes.data, stp.ctypes.data,
                                          fr.ctypes.data, xv.ctypes.data, k, ctypes.byref(n)),
                   "genga_collisions")
        return {"tp": tp, "planet": pl, "step": stp, "frac": fr, "xv": xv}

    def tp_encounters(self):
        """Particle-planet encounters of the last step: rows (particle,
        planet) sorted, with the Hermite minimum d2 and r_crit,ij^2."""
        n = ctypes.c_int64()
        code = lib().genga_tp_encounters(self._ctx, None, None, None, None, 0, ctypes.byref(n))
        if code not in (OK, EOVERFLOW):
            _check(code, "genga_tp_encounters")
        k = int(n.value)
        tp = np.zeros(max(k, 1), dtype=np.int64)
        pl = np.zeros(max(k, 1), dtype=np.int32)
        d2 = np.zeros(max(k, 1))
        rc2 = np.zeros(max(k, 1))
        _check(lib().genga_tp_encounters(self._ctx, tp.ctypes.data, pl.ctypes.data, d2.ctypes.data,
                                         rc2.ctypes.data, max(k, 1), ctypes.byref(n)),
               "genga_tp_encounters")
        return np.stack([tp[:k], pl[:k].astype(np.int64)], 1), d2[:k], rc2[:k]

    def split_state(self, coords: str = "dem"):
        x, v = self.state(coords)
        return x[:self.nm], v[:self.nm], x[self.nm:], v[self.nm:]


class BatchedSimulation(Simulation):
    """Independent systems (Sec. 3.4), system s in rows
    [offsets[s], offsets[s+1]), each with its own central mass m0s[s]; every
    call to ``step(n)`` is one launch (a captured HIP graph) that advances
    every system n steps.  The tuner runs before the first steps."""

    def __init__(self, offsets, m0s, m, x, v, params: Params | None = None,
                 coords: str = "helio", device="cuda", stream=None):
        self.p = params if params is not None else default_params()
        self.device = torch.device(device)
        self.stream = stream
        off = torch.as_tensor(np.asarray(offsets, dtype=np.int32)).to(self.device).contiguous()
        m0 = None if m0s is None else _dev(m0s, self.device)
        m = _dev(m, self.device)
        x = _dev(x, self.device).reshape(-1, 3)
        v = _dev(v, self.device).reshape(-1, 3)
        self.nsys = int(off.numel()) - 1
        self.n = int(m.numel())
        self.offsets = np.asarray(offsets, dtype=np.int64)
        nbytes = lib().genga_workspace_bytes(GENGA_BATCH, ctypes.byref(self.p), 0, 0, self.nsys,
                                             self.n)
        if nbytes == 0:
            raise GengaError(EINVAL, "genga_workspace_bytes")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._ctx = ctypes.c_void_p()
        code = lib().genga_init(ctypes.byref(self._ctx), GENGA_BATCH, ctypes.byref(self.p), 0, 0,
                                self.nsys, _ptr(off), _ptr(m0), _ptr(m), _ptr(x), _ptr(v),
                                GENGA_HELIO if coords == "helio" else GENGA_DEMOCRATIC,
                                _ptr(self.ws), nbytes, _stream(stream))
        _check(code, "genga_init")

    def energy(self):
        E = torch.empty(self.nsys, dtype=torch.float64, device=self.device)
        L = torch.empty(3 * self.nsys, dtype=torch.float64, device=self.device)
        _check(lib().genga_energy(self._ctx, _ptr(E), _ptr(L)), "genga_energy")
        torch.cuda.synchronize(self.device)
        return E.cpu().numpy(), L.cpu().numpy().reshape(-1, 3)

    def status(self):
        """Per system: (status code, steps completed since init)."""
        st = np.zeros(self.nsys, dtype=np.int32)
        ns = np.zeros(self.nsys, dtype=np.int64)
        _check(lib().genga_batch_status(self._ctx, st.ctypes.data, ns.ctypes.data, self.nsys),
               "genga_batch_status")
        return st, ns

    def set_masses(self, m):
        """New masses, one per row; positions and velocities stay."""
        m = _dev(m, self.device).reshape(-1).contiguous()
        if m.numel() != self.n:
            raise ValueError("masses: one per row")
        _check(lib().genga_set_masses(self._ctx, _ptr(m)), "genga_set_masses")

    def tune(self, nsteps: int = 4):
        """Re-run the tuner; returns ({variant: microseconds}, chosen variant)."""
        us = (ctypes.c_double * 16)()
        n, ch = ctypes.c_int(), ctypes.c_int()
        _check(lib().genga_tune(self._ctx, int(nsteps), us, 16, ctypes.byref(n), ctypes.byref(ch)),
               "genga_tune")
        names = {v: lib().genga_tune_variant(v).decode() for v in range(n.value)}
        return {names[v]: us[v] for v in range(n.value) if us[v] >= 0.0}, names[ch.value]

    def set_variant(self, v: int):
        """Use kernel variant v (numbered as by the tuner) for later steps."""
        _check(lib().genga_batch_set_variant(self._ctx, int(v)), "genga_batch_set_variant")

    # ---- adjoint of the encounter-free map (contexts with encounter_free=1) --
    def adj_forward(self, nsteps: int, ckpt_every: int = 32):
        """Advance nsteps steps keeping checkpoints for adj_backward."""
        nb = lib().genga_adj_buffer_bytes(self._ctx, int(nsteps), int(ckpt_every))
        if nb == 0:
            raise GengaError(EINVAL, "genga_adj_buffer_bytes")
        self._adj_buf = torch.empty(nb, dtype=torch.uint8, device=self.device)
        _check(lib().genga_adj_forward(self._ctx, int(nsteps), int(ckpt_every),
                                       _ptr(self._adj_buf), nb), "genga_adj_forward")

    def adj_backward(self, gxT, gvT):
        """(dL/dx0, dL/dv0, dL/dm) from dL/dxT, dL/dvT (democratic rows)."""
        gxT = _dev(gxT, self.device).reshape(-1, 3)
        gvT = _dev(gvT, self.device).reshape(-1, 3)
        gx0 = torch.empty_like(gxT)
        gv0 = torch.empty_like(gvT)
        gm = torch.empty(self.n, dtype=torch.float64, device=self.device)
        _check(lib().genga_adj_backward(self._ctx, _ptr(gxT), _ptr(gvT), _ptr(gx0), _ptr(gv0),
                                        _ptr(gm)), "genga_adj_backward")
        return gx0, gv0, gm


# Idle adjoint contexts by (device, system layout, central masses,
# parameters): a forward takes one (or makes one), its backward gives it back,
# so repeated calls re-use the workspace instead of a new init each time.
_EF_IDLE: dict = {}


def _ef_key(device, offsets, m0s, p):
    off = tuple(int(q) for q in np.asarray(offsets).reshape(-1))
    m0 = None if m0s is None else tuple(float(q) for q in np.asarray(
        m0s.detach().cpu() if torch.is_tensor(m0s) else m0s, dtype=np.float64).reshape(-1))
    return (str(device), off, m0, bytes(p))


def _ef_take(x0, v0, m, offsets, m0s, p):
    key = _ef_key(x0.device, offsets, m0s, p)
    idle = _EF_IDLE.get(key)
    if idle:
        sim = idle.pop()
        sim.set_masses(m.detach())
        sim.set_state(x0.detach(), v0.detach(), "dem")
    else:
        sim = BatchedSimulation(offsets, m0s, m.detach(), x0.detach(), v0.detach(), p,
                                coords="dem", device=x0.device)
    sim._ef_key = key
    return sim


def _ef_give_back(sim):
    sim._adj_buf = None
    _EF_IDLE.setdefault(sim._ef_key, []).append(sim)


def _map_forward(ctx, x0, v0, m, offsets, m0s, nsteps, ckpt_every, params, encounter_free):
    p = Params()
    ctypes.memmove(ctypes.byref(p), ctypes.byref(params if params is not None
                                                 else default_params()), ctypes.sizeof(p))
    p.encounter_free = encounter_free
    sim = _ef_take(x0, v0, m, offsets, m0s, p)
    try:
        sim.adj_forward(nsteps, ckpt_every)
        xT, vT = sim.state("dem")
        sim.check()
    except Exception:
        sim.close()
        raise
    ctx.sim = sim
    return xT, vT


def _map_backward(ctx, gxT, gvT):
    sim = ctx.sim
    ctx.sim = None
    if gxT is None:
        gxT = torch.zeros(sim.n, 3, dtype=torch.float64, device=sim.device)
    if gvT is None:
        gvT = torch.zeros(sim.n, 3, dtype=torch.float64, device=sim.device)
    try:
        gx0, gv0, gm = sim.adj_backward(gxT.contiguous(), gvT.contiguous())
        sim.check()
    except Exception:
        sim.close()
        raise
    _ef_give_back(sim)
    return gx0, gv0, gm, None, None, None, None, None


class EncounterFreeMap(torch.autograd.Function):
    """(x_T, v_T) = nsteps steps of the encounter-free map (K = 1) of every
    system from democratic (x0, v0) with masses m; backward runs the library's
    adjoint with a checkpoint every ckpt_every steps.  Contexts are re-used
    across calls of the same shape and parameters."""

    @staticmethod
    def forward(ctx, x0, v0, m, offsets, m0s, nsteps, ckpt_every=32, params=None):
        return _map_forward(ctx, x0, v0, m, offsets, m0s, nsteps, ckpt_every, params, 1)

    @staticmethod
    def backward(ctx, gxT, gvT):
        return _map_backward(ctx, gxT, gvT)


class HybridMap(torch.autograd.Function):
    """(x_T, v_T) = nsteps hybrid steps (Eq. 7: changeover, encounter groups
    integrated by BS) of every system from democratic (x0, v0) with masses
    m; backward runs the library's encounter-aware adjoint, which holds every
    decision of the run fixed (candidates, encounters, groups, accepted BS
    substeps).  The first step's candidates are the precheck of (x0, v0)."""

    @staticmethod
    def forward(ctx, x0, v0, m, offsets, m0s, nsteps, ckpt_every=32, params=None):
        return _map_forward(ctx, x0, v0, m, offsets, m0s, nsteps, ckpt_every, params, 0)

    @staticmethod
    def backward(ctx, gxT, gvT):
        return _map_backward(ctx, gxT, gvT)


def hybrid_map(x0, v0, m, offsets, m0s, nsteps, ckpt_every=32, params=None):
    return HybridMap.apply(x0, v0, m, offsets, m0s, nsteps, ckpt_every, params)


def encounter_free_map(x0, v0, m, offsets, m0s, nsteps, ckpt_every=32, params=None):
    return EncounterFreeMap.apply(x0, v0, m, offsets, m0s, nsteps, ckpt_every, params)
