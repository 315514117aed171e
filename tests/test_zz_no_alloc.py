"""The no-allocation form of the pair kernel's acceleration call against the
workspace form, through the C ABI: the same bits on two calls in a row (the
second with fewer bodies, so rows left in the library's fixed scratch by the
first call would show), with the changeover and with K = 1, and the size
limit."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1404_2324_amd import genga as G

pytestmark = pytest.mark.gpu


def _bodies(n, seed):
    rng = np.random.default_rng(seed)
    m = rng.uniform(1e-9, 1e-6, n)
    x = rng.uniform(-1, 1, (n, 3)) * np.array([1, 1, 0.05]) + np.array([1.5, 0, 0])
    rc = rng.uniform(0.01, 0.08, n)     # many pairs inside the changeover band
    return [torch.tensor(a, dtype=torch.float64, device="cuda").contiguous() for a in (m, x, rc)]


def _noalloc(gp, m, x, rc, n=None):
    n = int(m.numel()) if n is None else n
    out = torch.full((max(n, 1), 3), float("nan"), dtype=torch.float64, device="cuda")
    code = G.lib().genga_accel_noalloc(ctypes.byref(gp), n, G._ptr(m), G._ptr(x), G._ptr(rc),
                                       G._ptr(out), G._stream())
    return code, out


@pytest.mark.parametrize("encounter_free", [0, 1])
def test_noalloc_accel_equals_workspace_accel_twice(encounter_free):
    gp = G.default_params(encounter_free=encounter_free)
    for n, seed in ((5000, 31), (1203, 32)):
        print("no-alloc accel: n", n, "encounter_free", encounter_free, flush=True)
        m, x, rc = _bodies(n, seed)
        code, a = _noalloc(gp, m, x, rc)
        assert code == G.OK
        ref = G.accel(gp, m, x, rc if not encounter_free else None)
        torch.cuda.synchronize()
        assert torch.isfinite(a).all()
        assert torch.equal(a, ref), float((a - ref).abs().max())


def test_noalloc_accel_size_limit_and_arguments():
    gp = G.default_params()
    nmax = 16384                        # GENGA_ACCEL_NOALLOC_MAX
    m, x, rc = _bodies(nmax, 33)
    code, a = _noalloc(gp, m, x, rc)
    assert code == G.OK
    ref = G.accel(gp, m, x, rc)
    torch.cuda.synchronize()
    assert torch.equal(a, ref)
    m1, x1, rc1 = _bodies(nmax + 1, 34)
    assert _noalloc(gp, m1, x1, rc1)[0] == G.EINVAL
    assert _noalloc(gp, m, x, rc, n=0)[0] == G.EINVAL
    out = torch.empty((4, 3), dtype=torch.float64, device="cuda")
    assert G.lib().genga_accel_noalloc(ctypes.byref(gp), 4, G._ptr(m), G._ptr(x), None,
                                       G._ptr(out), G._stream()) == G.EINVAL
