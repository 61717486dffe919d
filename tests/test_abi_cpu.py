"""CPU-side checks of the C-ABI library: it loads, exports every declared
symbol, its host-only pieces (scheme tables, closed-form stage coefficients,
argument validation) agree with the oracle and the header.  No GPU compute."""
import ctypes
import math
import os
import re
from dataclasses import replace

import numpy as np
import pytest

import oracle
import paper_1007_3470_amd as pkg
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hfgpe.h")


def declared_symbols():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"\b(hfgpe_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = pkg.load()
    names = declared_symbols()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(pkg.SYMBOLS)


def test_header_is_plain_c99(tmp_path):
    """The boundary compiles and links from strict C99 (the C driver of the GPU
    test suite, linked against the library; not run here)."""
    import subprocess
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    libdir = os.path.join(ROOT, "paper_1007_3470_amd")
    pkg.load()
    subprocess.check_call(["gcc", "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror",
                           "-fsyntax-only", "-x", "c", HEADER])
    subprocess.check_call(["gcc", "-std=c99", "-O2", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(rocm, "include"), "-D__HIP_PLATFORM_AMD__",
                           os.path.join(ROOT, "tests", "c_abi_driver.c"), "-o", str(tmp_path / "drv"),
                           "-L", libdir, "-lhfgpe", "-L", os.path.join(rocm, "lib"), "-lamdhip64", "-lm"])


def test_version_and_status_strings():
    lib = pkg.load()
    ma, mi = ctypes.c_int(), ctypes.c_int()
    assert lib.hfgpe_version(ctypes.byref(ma), ctypes.byref(mi)) == 0
    assert (ma.value, mi.value) == (0, 3)
    for code in range(-8, 1):
        assert lib.hfgpe_status_string(code).decode() != "unknown status"
    assert lib.hfgpe_status_string(-99).decode() == "unknown status"


@pytest.mark.parametrize("name", ["leapfrog", "lie", "srkn6_4", "ni4_82", "ni5_84"])
def test_scheme_presets_match_oracle_tables(name):
    a, b = pkg.scheme_preset(name)
    oa, ob = oracle.scheme_coefficients(name)
    assert np.array_equal(a, oa) and np.array_equal(b, ob)


def test_unknown_scheme_rejected():
    with pytest.raises(pkg.HfgpeError) as e:
        pkg.scheme_preset("nope")
    assert e.value.code == -1


RULES = ["exact_const", "cf4", "magnus6"]


@pytest.mark.parametrize("rule", RULES)
@pytest.mark.parametrize("scheme", ["leapfrog", "ni5_84", "srkn6_4", "ni4_82"])
@pytest.mark.parametrize("dt", [1e-3, 0.05, -0.02])
def test_closed_forms_match_oracle_matrix_route(rule, scheme, dt):
    rng = np.random.default_rng(abs(hash((rule, scheme, dt))) % 2 ** 32)
    for _ in range(5):
        mu = float(rng.uniform(0.5, 2.0))
        amp = 0.0 if rule == "exact_const" else float(rng.uniform(0, 0.5))
        om = (float(rng.uniform(0.5, 2.0)), amp, float(rng.uniform(0.5, 3)), float(rng.uniform(0, 6)))
        inst = W.Instance(2, (8, 8, 1), (-1, -1, 0), (1, 1, 1), mu=mu,
                          omega=(om, (1.3, 0.0, 0.0, 0.0), W.CONST_OMEGA))
        tn = float(rng.uniform(0, 10))
        lib_c = pkg.stage_coeffs_params(inst, scheme, rule, dt, tn)
        orc_c = oracle.stage_coeffs(inst, scheme, rule, dt, tn)
        assert np.allclose(lib_c, orc_c, rtol=1e-12, atol=0), np.abs(lib_c / orc_c - 1).max()


FORMS = {"sin": (1.4, 0.3, 3.0, 0.2, 0), "sq_sin": W.TIMEDEP_OMEGA["cos"],
         "pulse": W.TIMEDEP_OMEGA["pulse"]}


@pytest.mark.parametrize("form", sorted(FORMS))
@pytest.mark.parametrize("rule", ["cf4", "magnus6", "fundamental", "fundamental:5", "fsplit"])
@pytest.mark.parametrize("scheme,dt", [("leapfrog", 0.05), ("ni5_84", -0.03), ("srkn6_4", 0.1)])
def test_time_forms_and_fundamental_rule_match_oracle(form, rule, scheme, dt):
    """The library's (f, g, e) under the trap forms of Sec. 4.2 and the
    fundamental-matrix rule agree with the oracle's 2x2 route."""
    for mu, tn in ((1.0, 0.0), (1.7, 1.85), (0.6, 2.3)):
        inst = W.Instance(1, (8, 1, 1), (-1, 0, 0), (1, 1, 1), mu=mu,
                          omega=(FORMS[form], W.CONST_OMEGA, W.CONST_OMEGA))
        lib_c = pkg.stage_coeffs_params(inst, scheme, rule, dt, tn)
        if rule == "fsplit":   # free drift: g = a_i dt / mu, no chirps
            a, _ = oracle.scheme_coefficients(scheme)
            assert np.allclose(lib_c[:, 0, 1], np.array(a) * dt / mu, rtol=1e-15, atol=0)
            assert not lib_c[:, 0, 0].any() and not lib_c[:, 0, 2].any()
            continue
        orc_c = oracle.stage_coeffs(inst, scheme, rule, dt, tn)
        assert np.allclose(lib_c, orc_c, rtol=1e-12, atol=0), np.abs(lib_c / orc_c - 1).max()


def test_time_form_validation():
    base = W.gpe_1d(n=64, nsteps=0).instances[0]
    pulse = replace(base, omega=(W.TIMEDEP_OMEGA["pulse"],) + base.omega[1:])
    cosq = replace(base, omega=(W.TIMEDEP_OMEGA["cos"],) + base.omega[1:])
    for inst in (pulse, cosq):
        for rule in ("cf4", "magnus6", "fundamental", "fsplit"):
            assert _gpu_or_nodevice(_create([inst], rule=rule, dt=1e-2)), rule
    assert _create([replace(base, sigma=(1.0, 0.1, 1.0, 0.0, 1))]) == -1     # sigma: no squared form
    assert _gpu_or_nodevice(_create([replace(base, sigma=(1.0, 0.1, 1.0, 0.0, 2))]))
    assert _create([replace(base, omega=((4.0, 0.2, 0.0, 2.0, 2),) + base.omega[1:])]) == -1
    assert _create([replace(base, omega=((1.0, 0.0, 0.0, 0.0, 7),) + base.omega[1:])]) == -1
    # pulse driving omega through zero: 1 - 2 * max|t sech^2| < 0
    neg = replace(base, omega=((4.0, -2.0, 2.0, 2.0, 2),) + base.omega[1:])
    assert _create([neg]) == -4
    assert _create([replace(base, omega=((1.0, 1.2, 1.0, 0.0, 1),) + base.omega[1:])]) == -4
    # constant squared form is a constant frequency sqrt(v0) for the exact rule
    const_sq = replace(base, omega=((2.25, 0.0, 0.0, 0.0, 1),) + base.omega[1:])
    assert _gpu_or_nodevice(_create([const_sq], rule="exact_const", dt=2.0))   # 1.5 * 2 < pi
    assert _create([const_sq], rule="exact_const", dt=2.2) == -3              # 1.5 * 2.2 > pi
    assert _create([pulse], rule="exact_const") == -1
    assert _gpu_or_nodevice(_create([pulse], rule="fundamental:256", dt=1e-2))
    assert _create([pulse], rule="fundamental:257", dt=1e-2) == -1


def test_exact_const_matches_oracle_for_constant_squared_form():
    inst = W.Instance(1, (8, 1, 1), (-1, 0, 0), (1, 1, 1), mu=1.3,
                      omega=((2.25, 0.0, 0.0, 0.0, 1), W.CONST_OMEGA, W.CONST_OMEGA))
    lib_c = pkg.stage_coeffs_params(inst, "leapfrog", "exact_const", 0.7, 0.0)
    mu, w, t = 1.3, 1.5, 0.7
    assert np.allclose(lib_c[0, 0], [mu * w * math.tan(w * t / 2), math.sin(w * t) / (mu * w),
                                     mu * w * math.tan(w * t / 2)], rtol=1e-14, atol=0)


def _create(instances, scheme="leapfrog", rule="cf4", dtype=1, dt=1e-3, m=None, a=None, b=None, opts=None):
    lib = pkg.load()
    if a is None:
        a, b = pkg.scheme_preset(scheme)
    ca, cb = (ctypes.c_double * len(a))(*a), (ctypes.c_double * len(b))(*b)
    sch = pkg.Scheme(len(a) if m is None else m, ca, cb, *pkg.parse_rule(rule))
    n = len(instances)
    g = (pkg.Grid * max(1, n))(*[pkg.make_grid(i) for i in instances])
    p = (pkg.Params * max(1, n))(*[pkg.make_params(i) for i in instances])
    h = ctypes.c_void_p()
    rc = lib.hfgpe_plan_create(ctypes.byref(h), n, g, p, ctypes.byref(sch), dtype, dt,
                               None if opts is None else ctypes.byref(opts), None)
    if rc == 0:
        lib.hfgpe_plan_destroy(h)
    return rc


def _gpu_or_nodevice(rc):
    # valid arguments: OK on a gfx950 box, NO_DEVICE without one
    return rc in (0, -8)


def test_plan_validation_codes():
    base = W.gpe_1d(n=64, nsteps=0).instances[0]
    assert _gpu_or_nodevice(_create([base]))
    # options: chunk_steps >= 0, in_kernel_records 0 or 1
    assert _gpu_or_nodevice(_create([base], opts=pkg.Options(in_kernel_records=1)))
    assert _create([base], opts=pkg.Options(in_kernel_records=2)) == -1
    assert _create([base], opts=pkg.Options(in_kernel_records=-1)) == -1
    assert _create([base], opts=pkg.Options(chunk_steps=-1)) == -1
    assert _create([replace(base, n=(48, 1, 1))]) == -2              # not a power of two
    assert _create([replace(base, n=(8192, 1, 1))]) == -2            # beyond the 1-D limit
    assert _create([replace(base, n=(64, 2, 1))]) == -2              # unused axis not 1
    assert _create([replace(base, mu=0.0)]) == -1
    assert _create([replace(base, hi=(-20.0, 1.0, 1.0))]) == -1      # empty box
    assert _create([base], dt=0.0) == -1
    assert _create([base], dt=float("nan")) == -1
    assert _create([base], dtype=7) == -1
    assert _create([base], m=0) == -1
    assert _create([base], a=[0.0], b=[0.5, 0.5]) == -1              # zero stage
    assert _create([base], rule="exact_const") == -1                 # omega varies in time
    assert _create([base], dt=3.0) == -3                             # beyond the first zero of g
    neg = replace(base, omega=((-1.0, 0.0, 0.0, 0.0),) + base.omega[1:])
    assert _create([neg]) == -4
    assert _create([replace(base, omega=((1.0, 1.2, 1.0, 0.0),) + base.omega[1:])]) == -4
    two = [base, replace(base, ndim=2, n=(64, 64, 1))]
    assert _create(two) == -1                                        # mixed dimensions


def test_exact_rule_singularity_bound():
    c1 = W.coherent_1d().instances[0]
    assert _gpu_or_nodevice(_create([c1], rule="exact_const", dt=3.1))
    assert _create([c1], rule="exact_const", dt=3.2) == -3
    assert _gpu_or_nodevice(_create([c1], rule="exact_const", dt=-3.1))


def test_empty_plan_is_valid_without_device():
    lib = pkg.load()
    a, b = pkg.scheme_preset("leapfrog")
    ca, cb = (ctypes.c_double * 1)(*a), (ctypes.c_double * 2)(*b)
    sch = pkg.Scheme(1, ca, cb, 1)
    h = ctypes.c_void_p()
    assert lib.hfgpe_plan_create(ctypes.byref(h), 0, None, None, ctypes.byref(sch), 0, 1e-3,
                                 None, None) == 0
    off = (ctypes.c_int64 * 1)()
    assert lib.hfgpe_instance_offsets(h, off) == 0 and off[0] == 0
    assert lib.hfgpe_evolve(h, None, 0.0, 10) == 0
    assert lib.hfgpe_norm(h, None, None) == 0
    assert lib.hfgpe_plan_destroy(h) == 0
    assert lib.hfgpe_plan_destroy(None) == 0


def test_null_arguments_rejected():
    lib = pkg.load()
    assert lib.hfgpe_plan_create(None, 0, None, None, None, 0, 1e-3, None, None) == -1
    assert lib.hfgpe_evolve(None, None, 0.0, 1) == -1
    assert lib.hfgpe_norm(None, None, None) == -1
    assert lib.hfgpe_instance_offsets(None, None) == -1
    assert lib.hfgpe_stage_coeffs(None, 0, 0.0, None) == -1


# ---------------------------------------------------------------------------
# coupled trap (off-diagonal W): library factor triples vs the oracle's 2d x 2d route
# ---------------------------------------------------------------------------
def _coupled_inst(d, mu=1.2, const=False, wc=(0.3, 0.2, -0.25)):
    om = ((1.2, 0.0 if const else 0.2, 1.5, 0.3), (0.9, 0.0, 0.0, 0.0),
          (1.4, 0.0 if const else 0.1, 0.7, 0.0))
    nn = tuple([8] * d + [1] * (3 - d))
    return W.Instance(d, nn, tuple([-2.0] * d + [0.0] * (3 - d)), tuple([2.0] * d + [1.0] * (3 - d)),
                      mu=mu, omega=om, wcross=wc)


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("rule", ["exact_const", "cf4"])
@pytest.mark.parametrize("scheme,dt", [("leapfrog", 0.05), ("ni5_84", -0.1), ("srkn6_4", 0.2)])
def test_coupled_triples_match_oracle(d, rule, scheme, dt):
    for mu, tn in ((1.0, 0.0), (1.7, 1.3)):
        inst = _coupled_inst(d, mu=mu, const=(rule == "exact_const"))
        lib_t = pkg.stage_coeffs_coupled(inst, scheme, rule, dt, tn)
        orc_t = oracle.stage_coeffs_full(inst, scheme, rule, dt, tn)
        assert lib_t.shape == orc_t.shape
        scale = np.abs(orc_t).max()
        assert np.abs(lib_t - orc_t).max() < 1e-13 * scale, np.abs(lib_t - orc_t).max()


def test_coupled_fsplit_triples():
    inst = _coupled_inst(2, mu=1.5)
    t = pkg.stage_coeffs_coupled(inst, "ni4_82", "fsplit", 0.1, 0.4)
    a, _ = oracle.scheme_coefficients("ni4_82")
    assert t.shape == (4, 3, 2, 2)
    for k in range(4):
        assert not t[k, 0].any() and not t[k, 2].any()
        assert np.array_equal(t[k, 1], np.eye(2) * (a[k] * 0.1 / 1.5))


def test_coupled_validation():
    base = W.gpe_2d(n=16, n_inst=1, nsteps=0).instances[0]
    cpl = replace(base, wcross=(0.2, 0.0, 0.0))
    assert _gpu_or_nodevice(_create([cpl], rule="cf4"))
    assert _gpu_or_nodevice(_create([cpl], rule="fsplit"))
    assert _create([cpl], rule="magnus6") == -1                      # rule not written for coupled W
    assert _create([cpl], rule="fundamental") == -1
    assert _create([cpl], rule="exact_const") == -1                  # omega_y varies in time
    const = replace(cpl, omega=((1.0, 0.0, 0.0, 0.0), (1.5, 0.0, 0.0, 0.0), W.CONST_OMEGA))
    assert _gpu_or_nodevice(_create([const], rule="exact_const", dt=1.0))
    assert _create([const], rule="exact_const", dt=3.0) == -3        # beyond the first zero of G
    assert _create([cpl, base], rule="cf4") == -1                    # mixed coupled / diagonal plan
    assert _create([replace(cpl, wcross=(5.0, 0.0, 0.0))], rule="cf4") == -4   # W indefinite
    assert _create([replace(cpl, wcross=(float("nan"), 0.0, 0.0))], rule="cf4") == -1
    # a 1-D instance ignores wcross
    c1 = replace(W.gpe_1d(n=64, nsteps=0).instances[0], wcross=(0.5, 0.0, 0.0))
    assert _gpu_or_nodevice(_create([c1]))


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built HIP library the binding raises; there is no CPU
    fallback anywhere on the product path."""
    monkeypatch.setattr(pkg, "_lib", None)
    monkeypatch.setattr(pkg, "LIB_PATH", str(tmp_path / "libhfgpe.so"))
    with pytest.raises(ImportError):
        pkg.load()
    w = W.gpe_1d(n=64, nsteps=1)
    with pytest.raises(ImportError):
        pkg.Plan(w.instances, w.scheme, w.ho_rule, "c128", w.dt)
    with pytest.raises(ImportError):
        pkg.scheme_preset("leapfrog")


# modulated cross terms W_ij(t) and a time factor of eps V_I
WMOD = ((0.5, 2.3, 0.4, 0), (0.8, 2.0, 0.6, 2), (-0.4, 1.1, 0.0, 0))


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("scheme,dt", [("leapfrog", 0.05), ("ni5_84", -0.1), ("srkn6_4", 0.2)])
def test_modulated_coupled_triples_match_oracle(d, scheme, dt):
    for mu, tn in ((1.0, 0.0), (1.7, 1.3)):
        inst = replace(_coupled_inst(d, mu=mu), wmod=WMOD)
        lib_t = pkg.stage_coeffs_coupled(inst, scheme, "cf4", dt, tn)
        orc_t = oracle.stage_coeffs_full(inst, scheme, "cf4", dt, tn)
        scale = np.abs(orc_t).max()
        assert np.abs(lib_t - orc_t).max() < 1e-13 * scale, np.abs(lib_t - orc_t).max()
        # and the modulation is not a no-op
        plain = pkg.stage_coeffs_coupled(_coupled_inst(d, mu=mu), scheme, "cf4", dt, tn)
        assert np.abs(plain - lib_t).max() > 1e-6 * scale


def test_modulation_validation():
    base = W.gpe_2d(n=16, n_inst=1, nsteps=0).instances[0]
    cpl = replace(base, wcross=(0.2, 0.0, 0.0), wmod=((0.5, 1.0, 0.0, 0),) + ((0.0, 0.0, 0.0, 0),) * 2)
    assert _gpu_or_nodevice(_create([cpl], rule="cf4"))
    assert _gpu_or_nodevice(_create([cpl], rule="fsplit"))
    const = replace(cpl, omega=((1.0, 0.0, 0.0, 0.0), (1.5, 0.0, 0.0, 0.0), W.CONST_OMEGA))
    assert _create([const], rule="exact_const", dt=1.0) == -1          # W(t) not constant
    unmod = replace(const, wmod=((0.0, 0.0, 0.0, 0),) * 3)
    assert _gpu_or_nodevice(_create([unmod], rule="exact_const", dt=1.0))
    # |W_xy| reaches 0.2 * 1.5 = 0.3; with wcross 0.6 it reaches 0.9 > omega_x^2 - ... (indefinite)
    assert _create([replace(cpl, wcross=(1.2, 0.0, 0.0))], rule="cf4") == -4
    assert _create([replace(cpl, wmod=((0.5, 1.0, 0.0, 1),) + cpl.wmod[1:])], rule="cf4") == -1   # no kind 1
    assert _create([replace(cpl, wmod=((0.5, 0.0, 0.0, 2),) + cpl.wmod[1:])], rule="cf4") == -1   # pulse freq 0
    assert _create([replace(base, vmod=(float("inf"), 1.0, 0.0, 0))]) == -1
    assert _gpu_or_nodevice(_create([replace(base, vmod=(0.5, 1.0, 0.0, 2))]))


def test_tune_cache_save_load(tmp_path):
    """The pass-tuning cache round-trips through its text form; a malformed
    file is rejected whole."""
    lib = pkg.load()
    good = tmp_path / "tune.txt"
    good.write_text("# comment\n2 512 512 1 1 0 2 0 2 256\n2 512 512 1 1 0 2 1 3 512\n")
    assert lib.hfgpe_tune_load(str(good).encode()) == 0
    out = tmp_path / "out.txt"
    assert lib.hfgpe_tune_save(str(out).encode()) == 0
    rows = [l for l in out.read_text().splitlines() if not l.startswith("#")]
    assert "2 512 512 1 1 0 2 0 2 256" in rows and "2 512 512 1 1 0 2 1 3 512" in rows
    bad = tmp_path / "bad.txt"
    bad.write_text("2 512 512 1 1 0 2 0 2 256\n2 512 512 1 1 0 2 5 2 256\n")   # position 5 of 2
    assert lib.hfgpe_tune_load(str(bad).encode()) == -1
    assert lib.hfgpe_tune_load(str(tmp_path / "missing.txt").encode()) == -1
    assert lib.hfgpe_tune_save(None) == -1
