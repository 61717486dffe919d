"""MI355X Hermite-Fourier GPE time stepping: Python binding of libhfgpe.so.

Thin ctypes binding of the C ABI declared in ``include/hfgpe.h``: argument
marshalling only.  Every step of the method runs in the library's gfx950 HIP
kernels; PyTorch provides device memory and the stream.  There is no CPU
fallback: if the shared library is missing or no gfx950 device is present the
calls raise.

Method: P. Bader and S. Blanes, "Fourier methods for the perturbed harmonic
oscillator in linear and nonlinear Schroedinger equations", arXiv:1007.3470.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhfgpe.so")

HFGPE_C64, HFGPE_C128 = 0, 1
HO_RULES = {"exact_const": 0, "cf4": 1, "magnus6": 2, "fsplit": 3, "fundamental": 4}
TF_KINDS = {"sin": 0, "sq_sin": 1, "pulse": 2}
STATUS = {0: "ok", -1: "invalid argument", -2: "unsupported grid shape", -3: "singular stage",
          -4: "non-positive frequency", -5: "allocation failed", -6: "HIP error",
          -7: "non-finite coefficient", -8: "no gfx950 device"}
SYMBOLS = ["hfgpe_plan_create", "hfgpe_plan_destroy", "hfgpe_instance_offsets", "hfgpe_evolve",
           "hfgpe_norm", "hfgpe_norm_noalloc", "hfgpe_energy", "hfgpe_stage_coeffs", "hfgpe_stage_coeffs_params",
           "hfgpe_stage_coeffs_coupled", "hfgpe_set_potential", "hfgpe_set_potential_f32", "hfgpe_set_stage_callback",
           "hfgpe_set_coef_callback",
           "hfgpe_scheme_preset",
           "hfgpe_device_status", "hfgpe_profile", "hfgpe_autotune", "hfgpe_tune_get", "hfgpe_tune_save",
           "hfgpe_tune_load", "hfgpe_status_string", "hfgpe_version", "hfgpe_last_hip_error"]


class HfgpeError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__("%s failed: %s (%d)" % (where, STATUS.get(code, "?"), code))


class Grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("n", ctypes.c_int * 3), ("lo", ctypes.c_double * 3),
                ("hi", ctypes.c_double * 3)]


class TFunc(ctypes.Structure):
    _fields_ = [("v0", ctypes.c_double), ("amp", ctypes.c_double), ("freq", ctypes.c_double),
                ("phase", ctypes.c_double), ("kind", ctypes.c_int)]


class VFactor(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("c0", "c2", "c4", "gs", "k", "phi")]


class TMod(ctypes.Structure):
    _fields_ = [("amp", ctypes.c_double), ("freq", ctypes.c_double), ("phase", ctypes.c_double),
                ("kind", ctypes.c_int)]


class Params(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("omega", TFunc * 3), ("sigma", TFunc),
                ("eps", ctypes.c_double), ("v", VFactor * 3), ("wcross", ctypes.c_double * 3),
                ("vmod", TMod), ("wmod", TMod * 3)]


class Scheme(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int), ("a", ctypes.POINTER(ctypes.c_double)),
                ("b", ctypes.POINTER(ctypes.c_double)), ("ho_rule", ctypes.c_int),
                ("ho_substeps", ctypes.c_int)]


def parse_rule(name: str):
    """HO rule name -> (hfgpe_ho_rule, ho_substeps).  "fundamental:q" selects
    q Magnus sub-steps per stage ("fundamental" alone: the library default)."""
    base, _, q = name.partition(":")
    return HO_RULES[base], int(q) if q else 0


class Options(ctypes.Structure):
    _fields_ = [("steps_per_launch", ctypes.c_int), ("plain", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("profile", ctypes.c_int),
                ("nd_workgroups", ctypes.c_int), ("nd_generic", ctypes.c_int),
                ("chunk_steps", ctypes.c_int), ("in_kernel_records", ctypes.c_int)]


# int fn(void *user, int inst, int axis, double t0, double tau, double mu, double *fge)
STAGE_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                            ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_double))
# double fn(void *user, int inst, int which, double t)
COEF_FN = ctypes.CFUNCTYPE(ctypes.c_double, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double)

_lib = None


def load() -> ctypes.CDLL:
    """Load libhfgpe.so (built by ``__graft_entry__.build()``); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libhfgpe.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp, dp, i64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)
    lib.hfgpe_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(Grid),
                                      ctypes.POINTER(Params), ctypes.POINTER(Scheme), ctypes.c_int,
                                      ctypes.c_double, ctypes.POINTER(Options), vp]
    lib.hfgpe_plan_destroy.argtypes = [vp]
    lib.hfgpe_instance_offsets.argtypes = [vp, i64p]
    lib.hfgpe_evolve.argtypes = [vp, vp, ctypes.c_double, ctypes.c_int64]
    lib.hfgpe_norm.argtypes = [vp, vp, dp]
    lib.hfgpe_norm_noalloc.argtypes = [vp, vp, vp]
    lib.hfgpe_set_potential.argtypes = [vp, vp]
    lib.hfgpe_set_potential_f32.argtypes = [vp, vp]
    lib.hfgpe_set_stage_callback.argtypes = [vp, STAGE_FN, vp]
    lib.hfgpe_set_coef_callback.argtypes = [vp, COEF_FN, vp]
    lib.hfgpe_energy.argtypes = [vp, vp, ctypes.c_double, dp]
    lib.hfgpe_stage_coeffs.argtypes = [vp, ctypes.c_int, ctypes.c_double, dp]
    lib.hfgpe_stage_coeffs_params.argtypes = [ctypes.POINTER(Params), ctypes.c_int,
                                              ctypes.POINTER(Scheme), ctypes.c_double,
                                              ctypes.c_double, dp]
    lib.hfgpe_stage_coeffs_coupled.argtypes = [ctypes.POINTER(Params), ctypes.c_int,
                                               ctypes.POINTER(Scheme), ctypes.c_double,
                                               ctypes.c_double, dp, ctypes.POINTER(ctypes.c_int)]
    lib.hfgpe_scheme_preset.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int), dp, dp]
    lib.hfgpe_device_status.argtypes = [vp]
    lib.hfgpe_profile.argtypes = [vp, dp, dp, i64p]
    lib.hfgpe_autotune.argtypes = [vp, vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int)]
    ip = ctypes.POINTER(ctypes.c_int)
    lib.hfgpe_tune_get.argtypes = [vp, ctypes.c_int, ip, ip, ip]
    lib.hfgpe_tune_save.argtypes = [ctypes.c_char_p]
    lib.hfgpe_tune_load.argtypes = [ctypes.c_char_p]
    lib.hfgpe_status_string.argtypes = [ctypes.c_int]
    lib.hfgpe_status_string.restype = ctypes.c_char_p
    lib.hfgpe_version.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    _lib = lib
    return lib


def _check(rc: int, where: str) -> None:
    if rc != 0:
        raise HfgpeError(rc, where)


def _check_device_buffer(buf, dtype, need: int, what: str) -> None:
    """A tensor handed to the library as a device pointer: on the GPU, of the
    plan's element type, contiguous and holding at least `need` elements."""
    if not getattr(buf, "is_cuda", False):
        raise TypeError("%s must be a CUDA (HIP) tensor" % what)
    if buf.dtype != dtype:
        raise TypeError("%s has dtype %s, the plan needs %s" % (what, buf.dtype, dtype))
    if not buf.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    if buf.numel() < need:
        raise ValueError("%s holds %d elements, the plan needs %d" % (what, buf.numel(), need))


def scheme_preset(name: str):
    """(a, b) of a named composition as held by the library."""
    lib = load()
    m = ctypes.c_int(0)
    a = (ctypes.c_double * 16)()
    b = (ctypes.c_double * 17)()
    _check(lib.hfgpe_scheme_preset(name.encode(), ctypes.byref(m), a, b), "hfgpe_scheme_preset")
    return list(a[: m.value]), list(b[: m.value + 1])


def stage_coeffs_params(inst, scheme: str, ho_rule: str, dt: float, tn: float) -> np.ndarray:
    """(f, g, e) per stage and axis by the library's closed forms (host only)."""
    lib = load()
    a, b = scheme_preset(scheme)
    ca, cb = (ctypes.c_double * len(a))(*a), (ctypes.c_double * len(b))(*b)
    sch = Scheme(len(a), ca, cb, *parse_rule(ho_rule))
    out = (ctypes.c_double * (len(a) * inst.ndim * 3))()
    p = make_params(inst)
    _check(lib.hfgpe_stage_coeffs_params(ctypes.byref(p), inst.ndim, ctypes.byref(sch), float(dt),
                                         float(tn), out), "hfgpe_stage_coeffs_params")
    return np.array(out[:]).reshape(len(a), inst.ndim, 3)


def stage_coeffs_coupled(inst, scheme: str, ho_rule: str, dt: float, tn: float) -> np.ndarray:
    """Factor triples (F, G, E) of a coupled-trap step by the library (host
    only): shape (triples, 3, d, d), in the order they act."""
    lib = load()
    a, b = scheme_preset(scheme)
    ca, cb = (ctypes.c_double * len(a))(*a), (ctypes.c_double * len(b))(*b)
    sch = Scheme(len(a), ca, cb, *parse_rule(ho_rule))
    d = inst.ndim
    out = (ctypes.c_double * (2 * len(a) * 3 * d * d))()
    nt = ctypes.c_int(0)
    p = make_params(inst)
    _check(lib.hfgpe_stage_coeffs_coupled(ctypes.byref(p), d, ctypes.byref(sch), float(dt), float(tn),
                                          out, ctypes.byref(nt)), "hfgpe_stage_coeffs_coupled")
    return np.array(out[: nt.value * 3 * d * d]).reshape(nt.value, 3, d, d)


def make_grid(inst) -> Grid:
    g = Grid()
    g.ndim = inst.ndim
    for j in range(3):
        g.n[j] = int(inst.n[j])
        g.lo[j] = float(inst.lo[j])
        g.hi[j] = float(inst.hi[j])
    return g


def make_tfunc(spec) -> TFunc:
    """(v0, amp, freq, phase[, kind]) -> hfgpe_tfunc (kind 0 when omitted)."""
    kind = int(spec[4]) if len(spec) > 4 else 0
    return TFunc(*[float(v) for v in spec[:4]], kind)


def make_params(inst) -> Params:
    p = Params()
    p.mu = float(inst.mu)
    for j in range(3):
        p.omega[j] = make_tfunc(inst.omega[j])
        p.v[j] = VFactor(*[float(v) for v in inst.vfac[j]])
    p.sigma = make_tfunc(inst.sigma)
    p.eps = float(inst.eps)
    for j, v in enumerate(getattr(inst, "wcross", (0.0, 0.0, 0.0))):
        p.wcross[j] = float(v)
    vm = getattr(inst, "vmod", (0.0, 0.0, 0.0, 0))
    p.vmod = TMod(float(vm[0]), float(vm[1]), float(vm[2]), int(vm[3]))
    for j, m in enumerate(getattr(inst, "wmod", ((0.0, 0.0, 0.0, 0),) * 3)):
        p.wmod[j] = TMod(float(m[0]), float(m[1]), float(m[2]), int(m[3]))
    return p


class Plan:
    """A batch of instances sharing scheme, dtype and step (hfgpe_plan)."""

    def __init__(self, instances: Sequence, scheme: str = "leapfrog", ho_rule: str = "cf4",
                 dtype: str = "c128", dt: float = 1e-3, steps_per_launch: int = 0,
                 plain: bool = False, use_graph: bool = False, profile: int = 0,
                 nd_workgroups: int = 0, nd_generic: bool = False, chunk_steps: int = 0,
                 in_kernel_records: bool = False, stream=None,
                 a: Optional[Sequence[float]] = None, b: Optional[Sequence[float]] = None):
        import torch
        self.lib = load()
        self.n_inst = len(instances)
        self.dtype = dtype
        self.torch_dtype = torch.complex64 if dtype == "c64" else torch.complex128
        if a is None:
            a, b = scheme_preset(scheme)
        self._a = (ctypes.c_double * len(a))(*a)
        self._b = (ctypes.c_double * len(b))(*b)
        sch = Scheme(len(a), self._a, self._b, *parse_rule(ho_rule))
        grids = (Grid * max(1, self.n_inst))(*[make_grid(i) for i in instances])
        params = (Params * max(1, self.n_inst))(*[make_params(i) for i in instances])
        opts = Options(int(steps_per_launch), int(bool(plain)), int(bool(use_graph)),
                       int(profile), int(nd_workgroups), int(bool(nd_generic)), int(chunk_steps),
                       int(bool(in_kernel_records)))
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        handle = ctypes.c_void_p()
        _check(self.lib.hfgpe_plan_create(ctypes.byref(handle), self.n_inst, grids, params,
                                          ctypes.byref(sch), HFGPE_C64 if dtype == "c64" else HFGPE_C128,
                                          float(dt), ctypes.byref(opts),
                                          ctypes.c_void_p(stream.cuda_stream)), "hfgpe_plan_create")
        self.handle = handle
        off = (ctypes.c_int64 * (self.n_inst + 1))()
        _check(self.lib.hfgpe_instance_offsets(self.handle, off), "hfgpe_instance_offsets")
        self.offsets = np.array(off[:], dtype=np.int64)
        self.shapes = [tuple(reversed(i.n[: i.ndim])) for i in instances]

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.hfgpe_plan_destroy(h)
            self.handle = None

    # -- buffers ----------------------------------------------------------
    def pack(self, psis: Iterable[np.ndarray]):
        """Host arrays (one per instance) -> packed device tensor."""
        import torch
        flat = np.concatenate([np.asarray(p, dtype=np.complex128).ravel() for p in psis]) \
            if self.n_inst else np.zeros(0, np.complex128)
        if flat.size != self.offsets[-1]:
            raise ValueError("pack: %d points given, the plan holds %d" % (flat.size, self.offsets[-1]))
        return torch.from_numpy(flat).to(self.torch_dtype).to("cuda")

    def unpack(self, buf) -> List[np.ndarray]:
        host = buf.detach().to("cpu").to(__import__("torch").complex128).numpy()
        return [host[self.offsets[k]:self.offsets[k + 1]].reshape(self.shapes[k])
                for k in range(self.n_inst)]

    def _ptr(self, buf) -> ctypes.c_void_p:
        """Device address of a state buffer, after checking that the kernels
        stay inside it (explicit checks: they must hold under python -O)."""
        _check_device_buffer(buf, self.torch_dtype, int(self.offsets[-1]), "state buffer")
        return ctypes.c_void_p(buf.data_ptr())

    # -- the hot path -----------------------------------------------------
    def evolve(self, buf, t0: float, nsteps: int) -> None:
        self._stage_exc = None
        rc = self.lib.hfgpe_evolve(self.handle, self._ptr(buf), float(t0), int(nsteps))
        if rc != 0:
            exc, self._stage_exc = self._stage_exc, None
            raise HfgpeError(rc, "hfgpe_evolve") from exc

    def set_stage_callback(self, fn) -> None:
        """Harmonic-oscillator stages from a Python function
        fn(inst, axis, t0, tau, mu) -> (f, g, e), the K(f) D(g) K(e) factors of
        that axis's flow over [t0, t0 + tau]; None restores the plan's rule."""
        if fn is None:
            self._stage_cb = None
            _check(self.lib.hfgpe_set_stage_callback(self.handle, STAGE_FN(), None),
                   "hfgpe_set_stage_callback")
            return

        def tramp(user, inst, axis, t0, tau, mu, out):
            try:
                f, g, e = fn(inst, axis, t0, tau, mu)
                out[0], out[1], out[2] = float(f), float(g), float(e)
                return 0
            except Exception as exc:  # noqa: BLE001 - reported to the library as a failed stage
                self._stage_exc = exc  # re-raised by evolve() as the cause
                return 1

        self._stage_cb = STAGE_FN(tramp)
        self._coef_cb = None
        _check(self.lib.hfgpe_set_stage_callback(self.handle, self._stage_cb, None),
               "hfgpe_set_stage_callback")

    def set_coef_callback(self, fn) -> None:
        """Time dependence from a Python function fn(inst, which, t): omega_j(t)
        for which = j < ndim, sigma(t) for which = 3, sampled by the plan's HO
        rule on the host; None restores the parameters' forms.  Setting it
        clears a stage callback (and the other way round)."""
        if fn is None:
            self._coef_cb = None
            _check(self.lib.hfgpe_set_coef_callback(self.handle, COEF_FN(), None), "hfgpe_set_coef_callback")
            return

        def tramp(user, inst, which, t):
            try:
                return float(fn(inst, which, t))
            except Exception as exc:  # noqa: BLE001 - a NaN makes the library fail the chunk
                self._stage_exc = exc  # re-raised by evolve() as the cause
                return float("nan")

        self._coef_cb = COEF_FN(tramp)
        self._stage_cb = None
        _check(self.lib.hfgpe_set_coef_callback(self.handle, self._coef_cb, None), "hfgpe_set_coef_callback")

    def set_potential(self, vi) -> None:
        """Use a device tensor of eps V_I per point (float64 or float32, the
        state's packed layout) instead of the factor form; None restores it.
        The tensor is kept referenced by the plan."""
        if vi is None:
            self._vi = None
            _check(self.lib.hfgpe_set_potential(self.handle, None), "hfgpe_set_potential")
            return
        import torch
        if vi.dtype == torch.float32:
            _check_device_buffer(vi, torch.float32, int(self.offsets[-1]), "potential")
            self._vi = vi
            _check(self.lib.hfgpe_set_potential_f32(self.handle, ctypes.c_void_p(vi.data_ptr())),
                   "hfgpe_set_potential_f32")
            return
        _check_device_buffer(vi, torch.float64, int(self.offsets[-1]), "potential")
        self._vi = vi
        _check(self.lib.hfgpe_set_potential(self.handle, ctypes.c_void_p(vi.data_ptr())),
               "hfgpe_set_potential")

    def pack_real(self, arrays):
        """Host real arrays (one per instance) -> packed float64 device tensor."""
        import torch
        flat = np.concatenate([np.asarray(a, dtype=np.float64).ravel() for a in arrays])
        if flat.size != self.offsets[-1]:
            raise ValueError("pack_real: %d points given, the plan holds %d" % (flat.size, self.offsets[-1]))
        return torch.from_numpy(flat).to("cuda")

    def norm(self, buf) -> np.ndarray:
        out = (ctypes.c_double * max(1, self.n_inst))()
        _check(self.lib.hfgpe_norm(self.handle, self._ptr(buf), out), "hfgpe_norm")
        return np.array(out[: self.n_inst])

    def energy(self, buf, t: float) -> np.ndarray:
        out = (ctypes.c_double * max(4, 4 * self.n_inst))()
        _check(self.lib.hfgpe_energy(self.handle, self._ptr(buf), float(t), out), "hfgpe_energy")
        return np.array(out[: 4 * self.n_inst]).reshape(self.n_inst, 4)

    def stage_coeffs(self, inst: int, tn: float, m: int, ndim: int) -> np.ndarray:
        out = (ctypes.c_double * (m * ndim * 3))()
        _check(self.lib.hfgpe_stage_coeffs(self.handle, int(inst), float(tn), out),
               "hfgpe_stage_coeffs")
        return np.array(out[:]).reshape(m, ndim, 3)

    def profile(self):
        """(step-kernel ms, coefficient-kernel ms, step-kernel launches) since
        the last call, from HIP events on the plan's stream."""
        sm, cm, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        _check(self.lib.hfgpe_profile(self.handle, ctypes.byref(sm), ctypes.byref(cm),
                                      ctypes.byref(n)), "hfgpe_profile")
        return sm.value, cm.value, n.value

    def autotune(self, psis, trial_steps: int = 20) -> int:
        """Time the candidate schedules on a scratch copy of ``psis`` and keep
        the fastest; returns the chosen setting."""
        scratch = self.pack(psis)
        c = ctypes.c_int(0)
        _check(self.lib.hfgpe_autotune(self.handle, self._ptr(scratch), int(trial_steps),
                                       ctypes.byref(c)), "hfgpe_autotune")
        return c.value

    def tune_settings(self):
        """[(workgroups per CU, threads per group)] of every d-D pass position
        (0 = the default policy); [] for 1-D plans."""
        n = ctypes.c_int(0)
        self.lib.hfgpe_tune_get(self.handle, -1, None, None, ctypes.byref(n))
        out = []
        for pp in range(n.value):
            a, b = ctypes.c_int(0), ctypes.c_int(0)
            _check(self.lib.hfgpe_tune_get(self.handle, pp, ctypes.byref(a), ctypes.byref(b), None),
                   "hfgpe_tune_get")
            out.append((a.value, b.value))
        return out

    def device_status(self) -> int:
        return int(self.lib.hfgpe_device_status(self.handle))
