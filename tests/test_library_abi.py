"""Host-side checks of the C ABI (no GPU needed): the built library loads,
exports every function include/genga.h declares, and its host-only calls
(defaults, workspace sizing, messages) behave as documented."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "genga.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(genga_[a-z_]+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def G():
    from paper_1404_2324_amd import genga
    return genga


def test_library_exports_every_declared_symbol(G):
    L = G.lib()
    declared = _declared_functions()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(L, name), f"{name} declared in genga.h but not exported"
        assert name in G.SIGNATURES, f"{name} has no binding signature"


def test_struct_layouts_match_header(G, tmp_path):
    """The binding's structs have the C compiler's size and field offsets."""
    import subprocess
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "genga.h"', "int main(void) {"]
    for cname, cls in (("genga_params", G.Params), ("genga_stats_t", G.Stats)):
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                        text=True).stdout.splitlines())
    for cname, cls in (("genga_params", G.Params), ("genga_stats_t", G.Stats)):
        assert int(out[cname]) == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert int(out[f"{cname}.{f}"]) == getattr(cls, f).offset, f"{cname}.{f}"


def test_default_params(G):
    p = G.default_params()
    assert p.G == 1.0 and p.m0 == 1.0
    assert p.n1 == 3.0 and p.n2 == 0.4 and p.pf == 3.0
    assert abs(p.dt - 0.02 * 3.141592653589793) < 1e-16
    assert p.bs_tol == 1e-13 and p.bs_max_depth == 20 and p.kepler_max_iter == 40


def test_workspace_sizing_and_limits(G):
    L = G.lib()
    p = G.default_params()
    b16 = L.genga_workspace_bytes(G.GENGA_MASSIVE, ctypes.byref(p), 16, 0, 0, 0)
    b2k = L.genga_workspace_bytes(G.GENGA_MASSIVE, ctypes.byref(p), 2048, 0, 0, 0)
    assert 0 < b16 < b2k
    assert b2k < 64 << 20
    # encounter mode is limited by the one-workgroup grouping
    assert L.genga_workspace_bytes(G.GENGA_MASSIVE, ctypes.byref(p), 2049, 0, 0, 0) == 0
    assert L.genga_workspace_bytes(G.GENGA_MASSIVE, ctypes.byref(p), 0, 0, 0, 0) == 0
    q = G.default_params(encounter_free=1)
    assert L.genga_workspace_bytes(G.GENGA_MASSIVE, ctypes.byref(q), 16384, 0, 0, 0) > 0
    bad = G.default_params(pf=0.5)
    assert L.genga_workspace_bytes(G.GENGA_MASSIVE, ctypes.byref(bad), 16, 0, 0, 0) == 0
    bad = G.default_params(m0=-1.0)
    assert L.genga_workspace_bytes(G.GENGA_MASSIVE, ctypes.byref(bad), 16, 0, 0, 0) == 0
    # composed steps (Sec. 2.3): orders 2, 4, 6, main mode only
    for order, ok in ((0, True), (2, True), (4, True), (6, True), (3, False), (8, False)):
        q = G.default_params(order=order)
        assert (L.genga_workspace_bytes(G.GENGA_MASSIVE, ctypes.byref(q), 16, 0, 0, 0) > 0) == ok
    q4 = G.default_params(order=4)
    assert L.genga_workspace_bytes(G.GENGA_TEST, ctypes.byref(q4), 8, 100, 0, 0) == 0
    assert L.genga_workspace_bytes(G.GENGA_BATCH, ctypes.byref(q4), 0, 0, 4, 8) == 0


def test_argument_errors_without_device(G):
    L = G.lib()
    assert L.genga_step(None, 1) == G.EINVAL
    assert L.genga_sync(None) == G.EINVAL
    assert L.genga_destroy(None) == G.EINVAL
    us = (ctypes.c_double * 6)()
    assert L.genga_step_kernel_us(None, 4, us) == G.EINVAL
    assert L.genga_step_profiled(None, 4, us) == G.EINVAL
    ctx = ctypes.c_void_p()
    p = G.default_params()
    # null arrays are rejected before any device work
    assert L.genga_init(ctypes.byref(ctx), G.GENGA_MASSIVE, ctypes.byref(p), 16, 0, 0, None,
                        None, None, None, None, G.GENGA_HELIO, None, 0, None) == G.EINVAL
    for code in (G.OK, G.EINVAL, G.EHIP, G.EOVERFLOW, G.EKEPLER, G.EBS, G.ENOMEM, G.EGROUP):
        assert L.genga_strerror(code)


def test_batch_workspace_sizing_and_tuner_names(G):
    L = G.lib()
    p = G.default_params()
    b1 = L.genga_workspace_bytes(G.GENGA_BATCH, ctypes.byref(p), 0, 0, 4096, 69632)
    b2 = L.genga_workspace_bytes(G.GENGA_BATCH, ctypes.byref(p), 0, 0, 8192, 2 * 69632)
    assert 0 < b1 < b2
    # 1..64 bodies per system
    assert L.genga_workspace_bytes(G.GENGA_BATCH, ctypes.byref(p), 0, 0, 10, 9) == 0
    assert L.genga_workspace_bytes(G.GENGA_BATCH, ctypes.byref(p), 0, 0, 10, 641) == 0
    assert L.genga_workspace_bytes(G.GENGA_BATCH, ctypes.byref(p), 0, 0, 0, 0) == 0
    assert L.genga_tune(None, 4, None, 0, None, None) == G.EINVAL
    assert L.genga_batch_status(None, None, None, 0) == G.EINVAL
    assert b"stopped" in L.genga_strerror(G.WSTOPPED)
    assert L.genga_batch_set_variant(None, 0) == G.EINVAL
    names = {L.genga_tune_variant(v).decode() for v in range(9)}
    assert len(names) == 9 and L.genga_tune_variant(9).decode() == "?"
    assert L.genga_tune_variant(-1).decode() == "?"
