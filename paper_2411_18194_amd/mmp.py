"""ctypes binding of libmmp (include/mmp.h): argument marshalling only.

Every computation runs in the HIP library; this module converts a problem
dict (see ``inputs``) into ``mmp_params``, NumPy arrays into pointers, and
error codes into exceptions.  It raises ``MMPError`` if the library cannot
be loaded: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmmp.so")

FP32, FP64 = 0, 1
T_DEMAG, T_EXCH, T_AFM_NN, T_AFM_CELL, T_DMI = 1, 2, 4, 8, 16
T_ANIS_U, T_ANIS_C, T_ZEEMAN, T_MEL = 32, 64, 128, 256
T_ALL = 0x1FF
T_ZL = 1 << 9
OUT_TORQUE = 1 << 16
TERM_BITS = {"demag": T_DEMAG, "exch": T_EXCH, "afm_nn": T_AFM_NN, "afm_cell": T_AFM_CELL,
             "dmi": T_DMI, "anis_u": T_ANIS_U, "anis_c": T_ANIS_C, "zeeman": T_ZEEMAN,
             "mel": T_MEL}
ENERGY_NAMES = ("demag", "exch", "afm_nn", "afm_cell", "dmi", "anis_u", "anis_c", "zeeman",
                "mel", "elastic")
PENDING = 1
# embedded Runge-Kutta pairs (MMP_RK_*)
SOLVERS = {"dp45": 0, "heun": 1, "bs23": 2, "cashkarp": 3, "rkf45": 4}


class MMPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mmp error {code}: {msg}")
        self.code = code


class Sub(C.Structure):
    _fields_ = [("Ms", C.c_double), ("A11", C.c_double), ("alpha", C.c_double),
                ("Ku1", C.c_double), ("Ku2", C.c_double), ("anis_u", C.c_double * 3),
                ("Kc1", C.c_double), ("cub_c1", C.c_double * 3), ("cub_c2", C.c_double * 3),
                ("Dint", C.c_double), ("B1", C.c_double), ("B2", C.c_double),
                ("zl_P", C.c_double), ("zl_xi", C.c_double)]


class Params(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("precision", C.c_int32), ("nsub", C.c_int32),
                ("demag", C.c_int32), ("gamma", C.c_double), ("sub", Sub * 3),
                ("A0", C.c_double), ("A12", C.c_double), ("latcon", C.c_double),
                ("B_ext", C.c_double * 3), ("j", C.c_double * 3), ("dmi_layer", C.c_int32),
                ("ngrains", C.c_int32), ("grain", C.POINTER(C.c_uint16)),
                ("grain_axes", C.POINTER(C.c_double)), ("elastic", C.c_int32),
                ("pad0", C.c_int32), ("rho", C.c_double), ("C11", C.c_double),
                ("C12", C.c_double), ("C44", C.c_double), ("eta", C.c_double),
                ("trac_amp", C.c_double), ("trac_freq", C.c_double), ("tol", C.c_double),
                ("dt0", C.c_double), ("dt_min", C.c_double), ("solver", C.c_int32),
                ("pbc", C.c_int32 * 3), ("rayleigh", C.c_double),
                ("dmi_homo", C.c_double * 3), ("bc_eq6", C.c_int32), ("pad2", C.c_int32),
                ("dmi_W", ((C.c_double * 3) * 3) * 2), ("dmi_W12", (C.c_double * 3) * 3),
                ("grain_exch_reduction", C.c_double), ("dt_max", C.c_double),
                ("safety", C.c_double), ("fac_min", C.c_double), ("fac_max", C.c_double)]


class StepInfo(C.Structure):
    _fields_ = [("t", C.c_double), ("dt", C.c_double), ("err", C.c_double),
                ("steps", C.c_int64), ("rejects", C.c_int64)]


class RunOpts(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("max_samples", C.c_int32),
                ("sample_every", C.c_double), ("sample_t", C.POINTER(C.c_double)),
                ("sample_m", C.POINTER(C.c_double)), ("max_steps", C.c_int64)]


class RunInfo(C.Structure):
    _fields_ = [("t", C.c_double), ("dt", C.c_double), ("steps", C.c_int64),
                ("rejects", C.c_int64), ("nsamples", C.c_int32), ("status", C.c_int32)]


class ServerOpts(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("hbm_budget", C.c_int64),
                ("max_active", C.c_int32), ("precision", C.c_int32), ("batch", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("nz", C.c_int32), ("cellsize", C.c_double * 3), ("params", Params),
                ("m0", C.POINTER(C.c_double)), ("t_relax", C.c_double)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("nsub", C.c_int32), ("m_avg", (C.c_double * 3) * 3),
                ("energy", C.c_double), ("steps", C.c_int64), ("rejects", C.c_int64),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double)]


class Plan(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("pad", C.c_int32 * 3), ("x_rows", C.c_int32 * 2),
                ("y_lines", C.c_int32 * 2), ("xy_cols", C.c_int32), ("z_cols", C.c_int32),
                ("z_lanes", C.c_int32), ("z_waves", C.c_int32), ("z_threads", C.c_int32),
                ("z_mode", C.c_int32), ("field_zplanes", C.c_int32), ("kinds", C.c_uint32), ("lds_axes", C.c_int32),
                ("demag_ms", C.c_double), ("field_ms", C.c_double)]


PLAN_KEYS = ("pad", "x_rows", "y_lines", "xy_cols", "z_cols", "z_lanes", "z_waves",
             "z_threads", "z_mode", "field_zplanes", "lds_axes")


def _plan_dict(pl: Plan) -> dict:
    d = {}
    for k, _ in Plan._fields_[1:]:
        v = getattr(pl, k)
        d[k] = list(v) if hasattr(v, "__len__") else v
    return d


EXPORTS = ("mmp_grid_create", "mmp_grid_destroy", "mmp_set_params", "mmp_set_state",
           "mmp_get_state", "mmp_eval_heff", "mmp_step", "mmp_run_fixed", "mmp_run",
           "mmp_set_stream", "mmp_set_graphs", "mmp_synchronize", "mmp_grid_bytes", "mmp_get_demag_tensor",
           "mmp_get_plan", "mmp_set_plan", "mmp_autotune", "mmp_stray_field",
           "mmp_stray_field_noalloc", "mmp_prof_enable", "mmp_prof_count", "mmp_prof_read", "mmp_prof_reset",
           "mmp_server_create", "mmp_submit", "mmp_poll", "mmp_server_destroy",
           "mmp_server_clock", "mmp_last_error", "mmp_set_state_device", "mmp_get_state_device",
           "mmp_eval_heff_device")

_lib = None


def load(path: str = LIB_PATH):
    """Load libmmp.so (raises MMPError if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise MMPError(-3, f"{path} not built; run python -m paper_2411_18194_amd.build")
    lib = C.CDLL(path)
    dp = C.POINTER(C.c_double)
    vp = C.c_void_p
    sig = {
        "mmp_grid_create": ([C.c_int32, C.c_int32, C.c_int32, dp, C.POINTER(vp)], C.c_int32),
        "mmp_grid_destroy": ([vp], C.c_int32),
        "mmp_set_params": ([vp, C.POINTER(Params)], C.c_int32),
        "mmp_set_state": ([vp, dp, dp, dp, C.c_double], C.c_int32),
        "mmp_get_state": ([vp, dp, dp, dp, dp, dp], C.c_int32),
        "mmp_eval_heff": ([vp, C.c_uint32, dp, dp], C.c_int32),
        "mmp_set_state_device": ([vp, vp, vp, vp, C.c_double], C.c_int32),
        "mmp_get_state_device": ([vp, vp, vp, vp, vp], C.c_int32),
        "mmp_eval_heff_device": ([vp, C.c_uint32, vp], C.c_int32),
        "mmp_step": ([vp, C.c_double, C.POINTER(StepInfo)], C.c_int32),
        "mmp_run_fixed": ([vp, C.c_double, C.c_int64, C.POINTER(StepInfo)], C.c_int32),
        "mmp_run": ([vp, C.c_double, C.POINTER(RunOpts), C.POINTER(RunInfo)], C.c_int32),
        "mmp_set_stream": ([vp, vp], C.c_int32),
        "mmp_set_graphs": ([vp, C.c_int32], C.c_int32),
        "mmp_synchronize": ([vp], C.c_int32),
        "mmp_grid_bytes": ([vp, C.POINTER(C.c_int64)], C.c_int32),
        "mmp_get_demag_tensor": ([vp, dp], C.c_int32),
        "mmp_stray_field": ([vp, C.c_double, dp], C.c_int32),
        "mmp_stray_field_noalloc": ([vp, C.c_double, vp], C.c_int32),
        "mmp_get_plan": ([vp, C.POINTER(Plan)], C.c_int32),
        "mmp_set_plan": ([vp, C.POINTER(Plan)], C.c_int32),
        "mmp_autotune": ([vp, C.POINTER(Plan)], C.c_int32),
        "mmp_prof_enable": ([vp, C.c_int32], C.c_int32),
        "mmp_prof_count": ([], C.c_int32),
        "mmp_prof_read": ([vp, C.c_int32, C.POINTER(C.c_char_p), dp, C.POINTER(C.c_int64)],
                          C.c_int32),
        "mmp_prof_reset": ([vp], C.c_int32),
        "mmp_server_create": ([C.POINTER(ServerOpts), C.POINTER(vp)], C.c_int32),
        "mmp_submit": ([vp, C.POINTER(Request), C.POINTER(C.c_uint64)], C.c_int32),
        "mmp_poll": ([vp, C.c_uint64, C.POINTER(Result)], C.c_int32),
        "mmp_server_destroy": ([vp], C.c_int32),
        "mmp_server_clock": ([vp], C.c_double),
        "mmp_last_error": ([], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(rc):
    if rc < 0:
        raise MMPError(rc, load().mmp_last_error().decode())
    return rc


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _dev_buf(x, n, name):
    """Address of a caller's FP64 device buffer of n elements: a tensor
    (checked to be float64, on a GPU, contiguous, of n elements) or a raw
    device address (int); None stays NULL."""
    if x is None:
        return None
    if isinstance(x, int):
        return C.c_void_p(x)
    if (str(getattr(x, "dtype", "")) != "torch.float64" or not getattr(x, "is_cuda", False)
            or not x.is_contiguous() or x.numel() != n):
        raise MMPError(-1, f"{name}: need a contiguous float64 GPU tensor of {n} elements")
    return C.c_void_p(x.data_ptr())


def make_params(p: dict, precision=FP32, tol=1e-5, dt0=1e-14, dt_min=1e-20):
    """mmp_params from a problem dict; returns (Params, keepalive)."""
    P = Params()
    P.struct_size = C.sizeof(Params)
    P.precision = precision
    P.nsub = p["nsub"]
    P.demag = 1 if p["demag"] else 0
    P.gamma = p["gamma"]
    for s in range(p["nsub"]):
        S = P.sub[s]
        S.Ms = p["Ms"][s]; S.A11 = p["A11"][s]; S.alpha = p["alpha"][s]
        S.Ku1 = p["Ku1"][s]; S.Ku2 = p["Ku2"][s]
        S.anis_u[:] = list(p["anis_u"][s])
        S.Kc1 = p["Kc1"][s]
        S.cub_c1[:] = list(p["cub_c1"][s]); S.cub_c2[:] = list(p["cub_c2"][s])
        S.Dint = p["Dint"][s]; S.B1 = p["B1"][s]; S.B2 = p["B2"][s]
        S.zl_P = p["zl_P"][s]; S.zl_xi = p["zl_xi"][s]
    P.A0 = p["A0"]; P.A12 = p["A12"]; P.latcon = p["latcon"]
    P.B_ext[:] = list(p["B_ext"]); P.j[:] = list(p["j"])
    P.dmi_layer = -1 if p.get("dmi_layer") is None else int(p["dmi_layer"])
    keep = []
    if p.get("grain") is not None:
        g = np.ascontiguousarray(p["grain"], dtype=np.uint16)
        ax = np.ascontiguousarray(p["grain_axes"], dtype=np.float64)
        keep += [g, ax]
        P.ngrains = ax.shape[0]
        P.grain = g.ctypes.data_as(C.POINTER(C.c_uint16))
        P.grain_axes = _dptr(ax)
        P.grain_exch_reduction = 1.0 - float(p.get("grain_exchange_scale", 1.0))
    el = p.get("elastic")
    if el is not None:
        P.elastic = 1
        P.rho = el["rho"]; P.C11 = el["C11"]; P.C12 = el["C12"]; P.C44 = el["C44"]
        P.eta = el["eta"]; P.trac_amp = el["trac_amp"]; P.trac_freq = el["trac_freq"]
        P.rayleigh = el.get("rayleigh", 0.0)
    P.tol, P.dt0, P.dt_min = tol, dt0, dt_min
    P.dt_max = float(p.get("dt_max") or 0.0)
    P.safety = float(p.get("safety") or 0.0)
    P.fac_min = float(p.get("fac_min") or 0.0)
    P.fac_max = float(p.get("fac_max") or 0.0)
    P.solver = SOLVERS[p.get("solver", "dp45")]
    P.pbc[:] = [int(v) for v in p.get("pbc", (0, 0, 0))]
    P.dmi_homo[:] = [float(v) for v in p.get("dmi_homo", (0.0, 0.0, 0.0))]
    P.bc_eq6 = 1 if p.get("bc", "open") == "eq6" else 0
    if p.get("dmi_W") is not None:
        W = np.asarray(p["dmi_W"], dtype=np.float64)
        for s_ in range(W.shape[0]):
            for i in range(3):
                for c in range(3):
                    P.dmi_W[s_][i][c] = float(W[s_, i, c])
    if p.get("dmi_W12") is not None:
        W = np.asarray(p["dmi_W12"], dtype=np.float64)
        for i in range(3):
            for c in range(3):
                P.dmi_W12[i][c] = float(W[i, c])
    return P, keep


class Grid:
    """One simulation grid in the HIP library."""

    def __init__(self, p: dict, precision=FP32, **solver):
        self.lib = load()
        self.p = p
        self.n = tuple(p["n"])
        self.nsub = p["nsub"]
        self.N = self.n[0] * self.n[1] * self.n[2]
        h = C.c_void_p()
        cs = np.array(p["cell"], dtype=np.float64)
        _check(self.lib.mmp_grid_create(*self.n, _dptr(cs), C.byref(h)))
        self.h = h
        self.set_params(p, precision, **solver)

    def set_params(self, p, precision=FP32, **solver):
        P, keep = make_params(p, precision, **solver)
        _check(self.lib.mmp_set_params(self.h, C.byref(P)))
        self.precision = precision
        self.p = p

    def close(self):
        if getattr(self, "h", None):
            self.lib.mmp_grid_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def shape_m(self):
        nx, ny, nz = self.n
        return (self.nsub, 3, nz, ny, nx)

    def set_state(self, m, u=None, v=None, t=0.0):
        m = np.ascontiguousarray(m, dtype=np.float64).reshape(self.shape_m())
        u = None if u is None else np.ascontiguousarray(u, dtype=np.float64)
        v = None if v is None else np.ascontiguousarray(v, dtype=np.float64)
        _check(self.lib.mmp_set_state(self.h, _dptr(m), _dptr(u), _dptr(v), t))

    def get_state(self):
        m = np.empty(self.shape_m())
        nx, ny, nz = self.n
        u = np.empty((3, nz, ny, nx))
        v = np.empty((3, nz, ny, nx))
        t = C.c_double()
        dt = C.c_double()
        _check(self.lib.mmp_get_state(self.h, _dptr(m), _dptr(u), _dptr(v), C.byref(t),
                                      C.byref(dt)))
        return m, u, v, t.value, dt.value

    def eval_heff(self, mask=T_ALL, want_b=True):
        b = np.empty(self.shape_m()) if want_b else None
        e = np.empty(10)
        _check(self.lib.mmp_eval_heff(self.h, mask, _dptr(b), _dptr(e)))
        return b, dict(zip(ENERGY_NAMES, e))

    # device-pointer variants: buffers are FP64 GPU tensors (or raw device
    # addresses) in the layouts of set_state / get_state / eval_heff; the
    # work is enqueued on the grid's stream and the calls return at once
    def set_state_device(self, m, u=None, v=None, t=0.0):
        n = int(np.prod(self.shape_m()))
        n3 = n // self.nsub
        _check(self.lib.mmp_set_state_device(self.h, _dev_buf(m, n, "m"), _dev_buf(u, n3, "u"),
                                             _dev_buf(v, n3, "v"), float(t)))

    def get_state_device(self, m=None, u=None, v=None, t_dt=None):
        n = int(np.prod(self.shape_m()))
        n3 = n // self.nsub
        _check(self.lib.mmp_get_state_device(self.h, _dev_buf(m, n, "m"), _dev_buf(u, n3, "u"),
                                             _dev_buf(v, n3, "v"), _dev_buf(t_dt, 2, "t_dt")))

    def eval_heff_device(self, b, mask=T_ALL):
        n = int(np.prod(self.shape_m()))
        _check(self.lib.mmp_eval_heff_device(self.h, mask, _dev_buf(b, n, "b")))

    def step(self, dt_fixed=0.0):
        info = StepInfo()
        _check(self.lib.mmp_step(self.h, dt_fixed, C.byref(info)))
        return info

    def run_fixed(self, dt, nsteps, sync=True):
        info = StepInfo()
        _check(self.lib.mmp_run_fixed(self.h, dt, nsteps, C.byref(info) if sync else None))
        return info

    def run(self, t_end, sample_every=0.0, max_samples=0, max_steps=0):
        info = RunInfo()
        o = RunOpts()
        o.struct_size = C.sizeof(RunOpts)
        o.sample_every = sample_every
        o.max_samples = max_samples
        o.max_steps = max_steps
        st = sm = None
        if sample_every > 0:
            st = np.zeros(max_samples)
            sm = np.zeros((max_samples, self.nsub, 3))
            o.sample_t = _dptr(st)
            o.sample_m = _dptr(sm)
        _check(self.lib.mmp_run(self.h, t_end, C.byref(o), C.byref(info)))
        if sample_every > 0:
            k = min(info.nsamples, max_samples)
            return info, st[:k], sm[:k]
        return info, None, None

    def set_stream(self, stream_ptr):
        _check(self.lib.mmp_set_stream(self.h, C.c_void_p(stream_ptr)))

    def set_graphs(self, on=True):
        """Replay captured HIP graphs in the step loops (default on)."""
        _check(self.lib.mmp_set_graphs(self.h, 1 if on else 0))

    def synchronize(self):
        _check(self.lib.mmp_synchronize(self.h))

    def nbytes(self):
        b = C.c_int64()
        _check(self.lib.mmp_grid_bytes(self.h, C.byref(b)))
        return b.value

    def demag_tensor(self):
        nx, ny, nz = self.n
        n6 = np.empty((6, nz, ny, nx))
        _check(self.lib.mmp_get_demag_tensor(self.h, _dptr(n6)))
        return n6

    def stray_field(self, height):
        """Stray field (3, ny, nx) in tesla in the layer of cells centred
        `height` above the top surface."""
        nx, ny, nz = self.n
        b = np.empty((3, ny, nx))
        _check(self.lib.mmp_stray_field(self.h, float(height), _dptr(b)))
        return b

    def stray_field_noalloc(self, height, out_dev_ptr):
        """Enqueue the stray field into the caller's device buffer at address
        out_dev_ptr (3*nx*ny doubles) on the grid's stream, with no device
        allocation; synchronise before reading it."""
        _check(self.lib.mmp_stray_field_noalloc(self.h, float(height),
                                                C.c_void_p(int(out_dev_ptr))))

    def plan(self) -> dict:
        """The demag plan: pads and launch shapes (see mmp_plan)."""
        pl = Plan(struct_size=C.sizeof(Plan))
        _check(self.lib.mmp_get_plan(self.h, C.byref(pl)))
        return _plan_dict(pl)

    def set_plan(self, **changes) -> dict:
        """Install the current plan with the given fields replaced."""
        cur = self.plan()
        cur.update(changes)
        pl = Plan(struct_size=C.sizeof(Plan))
        for k in PLAN_KEYS:
            v = cur[k]
            if isinstance(v, (list, tuple)):
                arr = getattr(pl, k)
                for i, x in enumerate(v):
                    arr[i] = int(x)
            else:
                setattr(pl, k, int(v))
        _check(self.lib.mmp_set_plan(self.h, C.byref(pl)))
        return self.plan()

    def autotune(self) -> dict:
        """Time candidate pads and launch shapes and install the fastest."""
        pl = Plan(struct_size=C.sizeof(Plan))
        _check(self.lib.mmp_autotune(self.h, C.byref(pl)))
        return _plan_dict(pl)

    def prof_enable(self, on=True):
        _check(self.lib.mmp_prof_enable(self.h, 1 if on else 0))

    def prof_reset(self):
        _check(self.lib.mmp_prof_reset(self.h))

    def prof_read(self):
        out = {}
        for i in range(self.lib.mmp_prof_count()):
            name = C.c_char_p()
            ms = C.c_double()
            cnt = C.c_int64()
            _check(self.lib.mmp_prof_read(self.h, i, C.byref(name), C.byref(ms), C.byref(cnt)))
            out[name.value.decode()] = (ms.value, cnt.value)
        return out


class Server:
    """Continuous-batching request server in the HIP library."""

    def __init__(self, hbm_budget, max_active=8, precision=FP32, batch=True):
        self.lib = load()
        o = ServerOpts()
        o.struct_size = C.sizeof(ServerOpts)
        o.hbm_budget = int(hbm_budget)
        o.max_active = max_active
        o.precision = precision
        o.batch = 1 if batch else 0
        h = C.c_void_p()
        _check(self.lib.mmp_server_create(C.byref(o), C.byref(h)))
        self.h = h
        self._keep = {}

    def submit(self, p, m0, t_relax, tol=1e-5):
        r = Request()
        r.struct_size = C.sizeof(Request)
        r.nx, r.ny, r.nz = p["n"]
        r.cellsize[:] = list(p["cell"])
        P, keep = make_params(p, FP32, tol=tol)
        r.params = P
        m0 = np.ascontiguousarray(m0, dtype=np.float64)
        r.m0 = _dptr(m0)
        r.t_relax = t_relax
        t = C.c_uint64()
        _check(self.lib.mmp_submit(self.h, C.byref(r), C.byref(t)))
        return t.value

    def poll(self, ticket):
        res = Result()
        rc = _check(self.lib.mmp_poll(self.h, ticket, C.byref(res)))
        if rc == PENDING:
            return None
        return res

    def wait(self, ticket, timeout=600.0, interval=1e-3):
        """Poll until the request is done; returns its Result."""
        t_end = time.monotonic() + timeout
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if time.monotonic() > t_end:
                raise MMPError(PENDING, f"request {ticket} not done after {timeout} s")
            time.sleep(interval)

    def clock(self):
        return self.lib.mmp_server_clock(self.h)

    def close(self):
        if getattr(self, "h", None):
            self.lib.mmp_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
