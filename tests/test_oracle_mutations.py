"""Mutation check of the oracle's pins: each case plants one plausible
mistake (a dropped term, a wrong sign, a wrong index or factor) in a copy of
the oracle source, builds it on the CPU and runs the pins against it.  Every
mutant must fail at least one pin."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "hermite_a_sign": ("3.0 * dt * (Pd0 + Pd1)", "3.0 * dt * (Pd0 - Pd1)"),
    "drop_Kprime": ("f = K / (r2 * r) - dK / r2;", "f = K / (r2 * r);"),
    "kprime_sign": ("f = K / (r2 * r) - dK / r2;", "f = K / (r2 * r) + dK / r2;"),
    "ha_kprime_sign": ("f = (1.0 - K) / (q2 * q) + dK / q2;", "f = (1.0 - K) / (q2 * q) - dK / q2;"),
    "sun_sign": ("x[3 * i + k] += h * P[k] / p->m0;", "x[3 * i + k] -= h * P[k] / p->m0;"),
    "stumpff_c3": ("double n3 = 0.25 * (c2 + c0 * c3);", "double n3 = 0.25 * (c2 + c1 * c3);"),
    "kepler_gdot": ("double gd = 1.0 - mu * G[2] / r;", "double gd = 1.0 - mu * G[2] / r0;"),
    "rcrit_hill": ("cbrt(m[i] / (3.0 * p->m0))", "cbrt(m[i] / (p->m0))"),
    "y_scale": ("double y = (r - 0.1 * rcij) / (0.9 * rcij);", "double y = (r - 0.1 * rcij) / (rcij);"),
    "mmid_smoothing": ("yout[k] = 0.5 * (ym[k] + yn[k] + hs * d[k]);",
                       "yout[k] = 0.5 * (ym[k] + yn[k] + 2.0 * hs * d[k]);"),
    "neville_h2": ("double den = ratio * ratio - 1.0;", "double den = ratio - 1.0;"),
    "tlm_kick": ("3.0 * d[k] * ddot * ir3 / r2", "2.0 * d[k] * ddot * ir3 / r2"),
    "tlm_dbeta": ("- 2.0 * dot3(v0, dv0);", "- 2.0 * dot3(x0, dv0);"),
    "helio_dem_mass": ("v[3 * i + k] -= S[k] / (p->m0 + M);", "v[3 * i + k] -= S[k] / (p->m0);"),
    "groups_max_label": ("int l = label[a] < label[b] ? label[a] : label[b];",
                         "int l = label[a] > label[b] ? label[a] : label[b];"),
    "energy_sun_term": ("*E = kin + dot3(P, P) / (2.0 * p->m0) + pot;", "*E = kin + pot;"),
    "precheck_factor": ("cand[(size_t)i * n + j] = r < p->pf * rcij;", "cand[(size_t)i * n + j] = r < rcij;"),
    "sun_kick_m0": ("for (int k = 0; k < 3; ++k) x[3 * i + k] += h * P[k] / p->m0;",
                    "for (int k = 0; k < 3; ++k) x[3 * i + k] += h * P[k];"),
    "coll_particle_radius": ("double R = s->rad[0] + s->rad[j];", "double R = s->rad[j];"),
    "coll_end_points_only": ("if (go_hermite_dmin2(h, dx0, dv0, dx1, dv1) < R * R) return j;",
                             "if (dot3(dx1, dx1) < R * R) return j;"),
    "coll_report_after": ("                    rcode = BS_COLLIDED;\n",
                          "                    memcpy(y, ynew, sizeof(double) * dim);\n"
                          "                    rcode = BS_COLLIDED;\n"),
    "coll_frac_after": ("*coll_frac = ldexp((double)pos, -D);",
                        "*coll_frac = ldexp((double)(pos + ((int64_t)1 << (D - d))), -D);"),
    "merge_survivor_tie": ("int sv = m[cb] > m[ca] ? cb : ca", "int sv = m[cb] >= m[ca] ? cb : ca"),
    "merge_U_sign": ("- G * mi * mj / sqrt(dot3(dx, dx));", "+ G * mi * mj / sqrt(dot3(dx, dx));"),
    "merge_spin_orbital": ("s_out[k] = si[k] + sj[k] + mi * li[k] + mj * lj[k];",
                           "s_out[k] = si[k] + sj[k];"),
    "merge_report_after": ("                    *coll_b = cb;\n",
                           "                    *coll_b = cb;\n"
                           "                    memcpy(y, ynew, sizeof(double) * dim);\n"),
    "compaction_ascending": ("for (int h = n - 1; h >= 0; --h) {", "for (int h = 0; h < n; ++h) {"),
    "yoshida_w0": ("w[1] = 1.0 - 2.0 * w[0];", "w[1] = 1.0 - w[0];"),
    "yoshida_w1": ("w[0] = w[2] = 1.0 / (2.0 - c);", "w[0] = w[2] = 1.0 / (2.0 + c);"),
    "eject_rcut_sun_off": ("if (ph->rcut_sun > 0.0 && r < ph->rcut_sun) kind = GO_EV_EJECT_SUN;",
                           "if (ph->rcut_sun > 0.0 && r > ph->rcut_sun) kind = GO_EV_EJECT_SUN;"),
}


# the complex-step derivative of the hybrid step (genga_cstep.c)
CS_MUTANTS = {
    "cs_kepler_root_fixed": ("cplx sc = CMPLX(s, -cimag(F) / creal(Fp));", "cplx sc = s;"),
    "cs_sqrt_slope": ("return CMPLX(s, cimag(z) / (2.0 * s));", "return CMPLX(s, cimag(z) / s);"),
    "cs_cbrt_slope": ("return CMPLX(c, cimag(z) / (3.0 * c * c));",
                      "return CMPLX(c, cimag(z) / (3.0 * c));"),
    "cs_radius_fixed": ("cplx y = (r - 0.1 * rcij) / (0.9 * rcij);",
                        "cplx y = (r - 0.1 * creal(rcij)) / (0.9 * creal(rcij));"),
    "cs_bs_mass_fixed": ("cplx sj = s->p->G * s->m[j] * f;",
                         "cplx sj = s->p->G * creal(s->m[j]) * f;"),
    "cs_ha_kprime_sign": ("cplx f = (1.0 - K) / (q2 * q) + dK / q2;",
                          "cplx f = (1.0 - K) / (q2 * q) - dK / q2;"),
    "cs_sun_mass_fixed": ("P[k] += m[j] * v[3 * j + k];", "P[k] += creal(m[j]) * v[3 * j + k];"),
}


def _run_mutant(tmp_path, fname, a, b, pins_filter=None):
    src = open(os.path.join(ROOT, "oracle", fname)).read()
    assert a in src, "mutation pattern no longer present in the oracle"
    pkg = tmp_path / "oracle"
    shutil.copytree(os.path.join(ROOT, "oracle"), pkg,
                    ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    (pkg / fname).write_text(src.replace(a, b, 1))
    args = ['-q', '-x', '-p', 'no:cacheprovider']
    if pins_filter:
        args += ['-k', pins_filter]
    code = ("import sys; sys.path.insert(0, %r); sys.path.insert(1, %r); import pytest; "
            "sys.exit(pytest.main(%r + [%r]))"
            % (str(tmp_path), ROOT, args, os.path.join(ROOT, "tests", "test_oracle_pins.py")))
    env = dict(os.environ, OMP_NUM_THREADS="1", OMP_WAIT_POLICY="passive")
    return subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                          cwd=str(tmp_path), timeout=600, env=env)


@pytest.mark.parametrize("name", sorted(CS_MUTANTS))
def test_cs_pins_catch_mutant(name, tmp_path):
    a, b = CS_MUTANTS[name]
    r = _run_mutant(tmp_path, "genga_cstep.c", a, b, pins_filter="cs_")
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    a, b = MUTANTS[name]
    src = open(os.path.join(ROOT, "oracle", "genga_oracle.c")).read()
    assert a in src, "mutation pattern no longer present in the oracle"
    pkg = tmp_path / "oracle"
    shutil.copytree(os.path.join(ROOT, "oracle"), pkg,
                    ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    (pkg / "genga_oracle.c").write_text(src.replace(a, b, 1))
    code = ("import sys; sys.path.insert(0, %r); sys.path.insert(1, %r); import pytest; "
            "sys.exit(pytest.main(['-q', '-x', '-p', 'no:cacheprovider', %r]))"
            % (str(tmp_path), ROOT, os.path.join(ROOT, "tests", "test_oracle_pins.py")))
    # the pins are small: one OpenMP thread keeps parallel test workers from
    # oversubscribing the cores
    env = dict(os.environ, OMP_NUM_THREADS="1", OMP_WAIT_POLICY="passive")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       cwd=str(tmp_path), timeout=600, env=env)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
