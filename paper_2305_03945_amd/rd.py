"""ctypes binding of librdpdhg (the C ABI in include/rd.h).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch supplies device memory (float64 CUDA tensors) and the current HIP stream.
Importing this module raises if the built library is missing; there is no
fallback path.
"""
import ctypes
import os
import weakref

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librdpdhg.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("librdpdhg.so is not built (run `python -m paper_2305_03945_amd.build`): %s" % LIB_PATH)

_lib = ctypes.CDLL(LIB_PATH)

# ---------------------------------------------------------------- enums (values of rd.h)
RD_OK, RD_E_INVALID, RD_E_NOCONV, RD_E_NONFINITE, RD_E_NOMEM, RD_E_DEVICE, RD_E_BUSY = 0, -1, -2, -3, -4, -5, -6
RD_BC_PERIODIC, RD_BC_NEUMANN = 0, 1
RD_OP_LAP5, RD_OP_BIHARM13, RD_OP_FCH6 = 0, 1, 2
RD_RX_NONE, RD_RX_ALLEN_CAHN, RD_RX_CAHN_HILLIARD, RD_RX_SCHNAKENBERG, RD_RX_FCH = 0, 1, 2, 3, 4
RD_FP64, RD_FP32_MIXED = 0, 1
RD_INIT_PREV, RD_INIT_PROX = 0, 1

STATUS_NAMES = {RD_OK: "ok", RD_E_INVALID: "invalid", RD_E_NOCONV: "noconv", RD_E_NONFINITE: "nonfinite",
                RD_E_NOMEM: "nomem", RD_E_DEVICE: "device", RD_E_BUSY: "busy"}

# Every C-ABI symbol include/rd.h declares.
EXPORTED = ("rd_create", "rd_destroy", "rd_default_opts", "rd_footprint_bytes", "rd_step", "rd_step_noalloc",
            "rd_residual",
            "rd_precond_solve", "rd_prox", "rd_profile_iteration", "rd_serve_set_budget", "rd_traj_open", "rd_traj_submit",
            "rd_serve_pump", "rd_poll", "rd_traj_read", "rd_traj_close", "rd_serve_stats", "rd_adapt_next",
            "rd_advance", "rd_status_str")


class Problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("lx", ctypes.c_double), ("ly", ctypes.c_double),
                ("bc", ctypes.c_int32), ("op", ctypes.c_int32), ("rx", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("diff", ctypes.c_double * 2), ("p", ctypes.c_double * 4)]


class Opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("max_outer", ctypes.c_int32),
                ("tau_u", ctypes.c_double), ("tau_p", ctypes.c_double), ("omega", ctypes.c_double),
                ("precision", ctypes.c_int32), ("init", ctypes.c_int32), ("inner_rtol", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("outer", ctypes.c_int32), ("residual_l2", ctypes.c_double),
                ("residual0", ctypes.c_double), ("mass_drift", ctypes.c_double), ("status", ctypes.c_int32),
                ("pad0", ctypes.c_int32)]

    def as_dict(self):
        return dict(iters=self.iters, outer=self.outer, residual=self.residual_l2, residual0=self.residual0,
                    mass_drift=self.mass_drift, status=STATUS_NAMES.get(self.status, str(self.status)),
                    status_code=self.status)


class ServeInfo(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("resident_bytes", ctypes.c_uint64), ("admitted", ctypes.c_int32),
                ("queued", ctypes.c_int32), ("running", ctypes.c_int32), ("pending_steps", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Adapt(ctypes.Structure):
    _fields_ = [("ht0", ctypes.c_double), ("eta", ctypes.c_double), ("n_hi", ctypes.c_int32), ("n_lo", ctypes.c_int32),
                ("ht_min", ctypes.c_double), ("max_rejects", ctypes.c_int32), ("pad0", ctypes.c_int32)]


class AdaptInfo(ctypes.Structure):
    _fields_ = [("accepted", ctypes.c_int32), ("rejected", ctypes.c_int32), ("shrinks", ctypes.c_int32),
                ("enlarges", ctypes.c_int32), ("pdhg_iters", ctypes.c_int64), ("t", ctypes.c_double),
                ("ht", ctypes.c_double), ("status", ctypes.c_int32), ("pad0", ctypes.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "pad0"}
        d["status"] = STATUS_NAMES.get(self.status, str(self.status))
        return d


def make_adapt(ht0, eta=0.75, n_hi=100, n_lo=20, ht_min=1e-12, max_rejects=30):
    return Adapt(ht0=float(ht0), eta=float(eta), n_hi=int(n_hi), n_lo=int(n_lo), ht_min=float(ht_min),
                 max_rejects=int(max_rejects))


def adapt_next(adapt, h, iters, status_code):
    """The step-size rule (host logic of the library): (next h, accepted)."""
    nxt, acc = ctypes.c_double(), ctypes.c_int32()
    _check(_lib.rd_adapt_next(ctypes.byref(adapt), float(h), int(iters), int(status_code), ctypes.byref(nxt),
                              ctypes.byref(acc)), "rd_adapt_next")
    return nxt.value, bool(acc.value)


_vp = ctypes.c_void_p
_P = ctypes.POINTER
_sig = {
    "rd_create": (ctypes.c_int, [ctypes.c_int, _P(_vp)]),
    "rd_destroy": (ctypes.c_int, [_vp]),
    "rd_default_opts": (None, [_P(Opts)]),
    "rd_footprint_bytes": (ctypes.c_size_t, [_P(Problem), _P(Opts)]),
    "rd_step": (ctypes.c_int, [_vp, _P(Problem), _P(Opts), ctypes.c_double, _vp, _vp, _vp, _P(Info)]),
    "rd_step_noalloc": (ctypes.c_int, [_vp, _P(Problem), _P(Opts), ctypes.c_double, _vp, _vp, _vp, _P(Info)]),
    "rd_residual": (ctypes.c_int, [_vp, _P(Problem), ctypes.c_double, _vp, _vp, _vp, _vp, _P(ctypes.c_double)]),
    "rd_precond_solve": (ctypes.c_int, [_vp, _P(Problem), ctypes.c_double, ctypes.c_int32, _vp, _vp, _vp]),
    "rd_prox": (ctypes.c_int, [_vp, _P(Problem), ctypes.c_double, _vp, _vp, _vp]),
    "rd_profile_iteration": (ctypes.c_int, [_vp, _P(Problem), _P(Opts), ctypes.c_double, _vp, ctypes.c_int32, _vp,
                                            _P(ctypes.c_double)]),
    "rd_serve_set_budget": (ctypes.c_int, [_vp, ctypes.c_size_t]),
    "rd_traj_open": (ctypes.c_int, [_vp, _P(Problem), _P(Opts), _vp, _vp, _P(_vp)]),
    "rd_traj_submit": (ctypes.c_int, [_vp, ctypes.c_double, _P(ctypes.c_uint64)]),
    "rd_serve_pump": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "rd_poll": (ctypes.c_int, [_vp, ctypes.c_uint64, _P(Info)]),
    "rd_traj_read": (ctypes.c_int, [_vp, _vp, _vp]),
    "rd_traj_close": (ctypes.c_int, [_vp]),
    "rd_serve_stats": (ctypes.c_int, [_vp, _P(ServeInfo)]),
    "rd_adapt_next": (ctypes.c_int, [_P(Adapt), ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                     _P(ctypes.c_double), _P(ctypes.c_int32)]),
    "rd_advance": (ctypes.c_int, [_vp, _P(Problem), _P(Opts), _P(Adapt), ctypes.c_double, ctypes.c_double, _vp, _vp,
                                  _P(AdaptInfo), _P(ctypes.c_double), _P(ctypes.c_int32), _P(ctypes.c_int32),
                                  ctypes.c_int32]),
    "rd_status_str": (ctypes.c_char_p, [ctypes.c_int]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class RDError(RuntimeError):
    def __init__(self, code, what):
        super().__init__("%s failed: %s (%d)" % (what, _lib.rd_status_str(code).decode(), code))
        self.code = code


def _check(code, what, allowed=(RD_OK,)):
    if code not in allowed:
        raise RDError(code, what)
    return code


# ---------------------------------------------------------------- argument builders
_KIND_TO_ABI = {
    "allen_cahn": (RD_OP_LAP5, RD_RX_ALLEN_CAHN),
    "heat": (RD_OP_LAP5, RD_RX_NONE),
    "cahn_hilliard": (RD_OP_BIHARM13, RD_RX_CAHN_HILLIARD),
    "biharmonic": (RD_OP_BIHARM13, RD_RX_NONE),
    "schnakenberg": (RD_OP_LAP5, RD_RX_SCHNAKENBERG),
    "fch": (RD_OP_FCH6, RD_RX_FCH),
}


def make_problem(kind, N, L=1.0, bc="periodic", diff=(1.0,), b=1.0, a=0.0, sb=0.0, kappa=1.0, dim=2):
    op, rx = _KIND_TO_ABI[kind]
    p = Problem()
    p.nx = p.ny = int(N)
    p.nz = int(N) if dim == 3 else 0
    p.lx = p.ly = float(L)
    p.bc = RD_BC_PERIODIC if bc == "periodic" else RD_BC_NEUMANN
    p.op, p.rx = op, rx
    d = tuple(diff) + (0.0,) * (2 - len(diff))
    p.diff[0], p.diff[1] = float(d[0]), float(d[1])
    if rx in (RD_RX_ALLEN_CAHN, RD_RX_CAHN_HILLIARD):
        p.p[0] = float(b)
    elif rx == RD_RX_SCHNAKENBERG:
        p.p[0], p.p[1], p.p[2] = float(a), float(sb), float(kappa)
    return p


def problem_from_config(cfg, N=None, bc=None):
    return make_problem(cfg["kind"], N or cfg["N"], cfg.get("L", 1.0), bc or cfg["bc"], cfg["diff"],
                        b=cfg.get("b", 1.0), a=cfg.get("a", 0.0), sb=cfg.get("sb", 0.0),
                        kappa=cfg.get("kappa", 1.0), dim=cfg.get("dim", 2))


def make_opts(tol=1e-10, max_iter=10000, tau_u=0.9, tau_p=0.9, omega=1.0, precision="fp64", init="prev",
              inner_rtol=3e-2, max_outer=20):
    o = Opts()
    _lib.rd_default_opts(ctypes.byref(o))
    o.tol = float(tol)
    o.max_iter = int(max_iter)
    o.max_outer = int(max_outer)
    o.tau_u, o.tau_p, o.omega = float(tau_u), float(tau_p), float(omega)
    o.precision = RD_FP64 if precision == "fp64" else RD_FP32_MIXED
    o.init = RD_INIT_PREV if init == "prev" else RD_INIT_PROX
    o.inner_rtol = float(inner_rtol)
    return o


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def field_size(problem):
    """FP64 values of one field of the problem: components x grid points."""
    ncomp = 2 if problem.rx == RD_RX_SCHNAKENBERG else 1
    return ncomp * problem.nx * problem.ny * (problem.nz if problem.nz > 1 else 1)


def _dptr(t, problem=None, numel=None):
    """The device address of a contiguous float64 tensor, after checking that it holds
    exactly one field of `problem` (or `numel` values): the library reads and writes
    whole fields through the pointer and cannot check the size itself."""
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 device tensor")
    want = field_size(problem) if problem is not None else numel
    if want is not None and t.numel() != want:
        raise ValueError("tensor holds %d values, the problem's field %d" % (t.numel(), want))
    return ctypes.c_void_p(t.data_ptr())


def footprint_bytes(problem, opts):
    return int(_lib.rd_footprint_bytes(ctypes.byref(problem), ctypes.byref(opts)))


class Context:
    """An rd_ctx on one HIP device."""

    def __init__(self, device=0):
        h = ctypes.c_void_p()
        _check(_lib.rd_create(int(device), ctypes.byref(h)), "rd_create")
        self._h = h
        self.device = device
        self._trajs = weakref.WeakSet()   # open trajectories: rd_destroy frees them

    def close(self):
        if self._h:
            for t in list(self._trajs):
                t._h = None
            _lib.rd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------- one implicit step
    def step(self, u, ht, problem, opts, out=None, stream=None, raise_on=(RD_E_INVALID, RD_E_DEVICE, RD_E_NOMEM)):
        import torch
        if out is None:
            out = torch.empty_like(u)
        info = Info()
        code = _lib.rd_step(self._h, ctypes.byref(problem), ctypes.byref(opts), float(ht), _dptr(u, problem), _dptr(out, problem),
                            _stream_ptr(stream), ctypes.byref(info))
        if code in raise_on:
            raise RDError(code, "rd_step")
        return out, info.as_dict()

    def step_noalloc(self, u, ht, problem, opts, out, stream=None, raise_on=(RD_E_INVALID, RD_E_DEVICE)):
        """rd_step_noalloc: one step whose workspace is the library's device scratch array
        (the caller passes the output buffer; the call allocates nothing).  Returns
        (info dict, status code); RD_E_NOMEM for problems beyond the scratch array."""
        info = Info()
        code = _lib.rd_step_noalloc(self._h, ctypes.byref(problem), ctypes.byref(opts), float(ht), _dptr(u, problem),
                                    _dptr(out, problem), _stream_ptr(stream), ctypes.byref(info))
        if code in raise_on:
            raise RDError(code, "rd_step_noalloc")
        return info.as_dict(), code

    # ---------------------------------------------------------- kernel-level calls
    def residual(self, u, uk, ht, problem, stream=None):
        import torch
        w = torch.empty_like(u)
        res = ctypes.c_double()
        _check(_lib.rd_residual(self._h, ctypes.byref(problem), float(ht), _dptr(u, problem), _dptr(uk, problem), _dptr(w, problem),
                                _stream_ptr(stream), ctypes.byref(res)), "rd_residual")
        return w, res.value

    def precond_solve(self, w, ht, problem, precision="fp64", stream=None):
        import torch
        y = torch.empty_like(w)
        prec = RD_FP64 if precision == "fp64" else RD_FP32_MIXED
        _check(_lib.rd_precond_solve(self._h, ctypes.byref(problem), float(ht), prec, _dptr(w, problem), _dptr(y, problem),
                                     _stream_ptr(stream)), "rd_precond_solve")
        return y

    def prox(self, c, ht, problem, stream=None):
        import torch
        u = torch.empty_like(c)
        _check(_lib.rd_prox(self._h, ctypes.byref(problem), float(ht), _dptr(c, problem), _dptr(u, problem), _stream_ptr(stream)),
               "rd_prox")
        return u

    def profile_iteration(self, u, ht, problem, opts, reps=20, stream=None):
        """Mean launch duration (ms) of each kernel of one iteration, HIP events on `stream`."""
        out = (ctypes.c_double * 6)()
        _check(_lib.rd_profile_iteration(self._h, ctypes.byref(problem), ctypes.byref(opts), float(ht), _dptr(u, problem),
                                         int(reps), _stream_ptr(stream), out), "rd_profile_iteration")
        names = ("yfwd", "zsym", "yinv", "rowinv", "upd", "rowfwd") if problem.nz > 1 else \
            ("cols", "rowinv", "upd", "rowfwd")
        return dict(zip(names, list(out)))

    def advance(self, u, t_end, problem, opts, adapt, t0=0.0, trace_cap=4096, stream=None):
        """Advance u in place from t0 to t_end with the adaptive step-size rule.
        Returns (info dict, trace list of (h, iterations, accepted))."""
        info = AdaptInfo()
        th = (ctypes.c_double * max(trace_cap, 1))()
        ti = (ctypes.c_int32 * max(trace_cap, 1))()
        tk = (ctypes.c_int32 * max(trace_cap, 1))()
        code = _lib.rd_advance(self._h, ctypes.byref(problem), ctypes.byref(opts), ctypes.byref(adapt), float(t0),
                               float(t_end), _dptr(u, problem), _stream_ptr(stream), ctypes.byref(info), th, ti, tk,
                               int(trace_cap))
        _check(code, "rd_advance", allowed=(RD_OK, RD_E_NOCONV))
        n = min(trace_cap, info.accepted + info.rejected)
        return info.as_dict(), [(th[i], ti[i], bool(tk[i])) for i in range(n)]

    # ---------------------------------------------------------- serving
    def set_budget(self, nbytes):
        _check(_lib.rd_serve_set_budget(self._h, int(nbytes)), "rd_serve_set_budget")

    def open(self, problem, opts, u0, stream=None):
        h = ctypes.c_void_p()
        _check(_lib.rd_traj_open(self._h, ctypes.byref(problem), ctypes.byref(opts), _dptr(u0, problem),
                                 _stream_ptr(stream), ctypes.byref(h)), "rd_traj_open")
        t = Trajectory(self, h, tuple(u0.shape))
        self._trajs.add(t)
        return t

    def pump(self, max_wait_us=0):
        _check(_lib.rd_serve_pump(self._h, int(max_wait_us)), "rd_serve_pump")

    def serve_stats(self):
        out = ServeInfo()
        _check(_lib.rd_serve_stats(self._h, ctypes.byref(out)), "rd_serve_stats")
        return out.as_dict()

    def poll(self, ticket):
        info = Info()
        code = _lib.rd_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(info))
        if code == RD_E_BUSY:
            return None
        if code == RD_E_INVALID:
            raise RDError(code, "rd_poll")
        return info.as_dict()


class Trajectory:
    def __init__(self, ctx, handle, shape):
        self.ctx = ctx
        self._h = handle
        self.shape = shape
        self.numel = 1
        for n in shape:
            self.numel *= int(n)

    def _handle(self, what):
        # a trajectory closed, or freed with its context, has no handle left
        if not self._h:
            raise RDError(RD_E_INVALID, what)
        return self._h

    def submit(self, ht):
        h = self._handle("rd_traj_submit")
        t = ctypes.c_uint64()
        _check(_lib.rd_traj_submit(h, float(ht), ctypes.byref(t)), "rd_traj_submit")
        return t.value

    def read(self, out=None, stream=None):
        import torch
        h = self._handle("rd_traj_read")
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device="cuda")
        _check(_lib.rd_traj_read(h, _dptr(out, numel=self.numel), _stream_ptr(stream)), "rd_traj_read")
        return out

    def close(self):
        if self._h:
            _check(_lib.rd_traj_close(self._h), "rd_traj_close")
            self._h = None


def status_str(code):
    return _lib.rd_status_str(int(code)).decode()
