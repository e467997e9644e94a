"""Python binding of the C ABI in include/nlte.h (ctypes).

Argument marshalling only: every step of the residual, the Jacobian-vector
product and the solve runs in the HIP library.  Device memory and streams come
from PyTorch tensors (``torch.float64`` on a HIP device).  The library must
have been built (``python -m paper_2406_17234_amd.build``); loading fails
loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnlte.so")

NLTE_OK, NLTE_E_INVALID, NLTE_E_NOMEM, NLTE_E_DEVICE = 0, -1, -2, -3
NLTE_E_NOCONV, NLTE_E_NONFINITE, NLTE_E_BUSY = -4, -5, -6
DEPTH_SCAN = 0x100  # OR into a column's precision: depth-parallel formal solution
FP64, FP32_FORM = 0, 1
PROBE_FMA_F32, PROBE_FMA_F64, PROBE_EXP_F32, PROBE_RCP_F32 = 0, 1, 2, 3
KRYLOV_GMRES, KRYLOV_BICGSTAB = 0, 1  # nlte_solve_opts.krylov_method
JV_FD, JV_TANGENT = 0, 1               # nlte_solve_opts.jv_method
STATUS_NAMES = {0: "OK", -1: "INVALID", -2: "NOMEM", -3: "DEVICE", -4: "NOCONV",
                -5: "NONFINITE", -6: "BUSY"}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class NLTEError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class AtmosDesc(C.Structure):
    _fields_ = [("nz", C.c_int32), ("z", _dp), ("T", _dp), ("ne", _dp), ("ntot", _dp),
                ("chi_c", _dp), ("chi_sca", _dp), ("eta_c", _dp), ("vlos", _dp)]


class AtomDesc(C.Structure):
    _fields_ = [("nlev", C.c_int32), ("E", _dp), ("g", _dp), ("stage", _ip),
                ("nline", C.c_int32), ("line_lo", _ip), ("line_up", _ip), ("A_ul", _dp),
                ("a_damp", _dp), ("mass_amu", C.c_double), ("vturb", C.c_double),
                ("nbf", C.c_int32), ("bf_lo", _ip), ("bf_ptr", _ip), ("bf_nu", _dp),
                ("bf_alpha", _dp)]


class GridDesc(C.Structure):
    _fields_ = [("nnu", C.c_int32), ("nu", _dp), ("win_lo", _ip), ("win_hi", _ip),
                ("nmu", C.c_int32), ("mu", _dp), ("w_mu", _dp), ("w_nu", _dp)]


class SolveOpts(C.Structure):
    _fields_ = [("ftol", C.c_double), ("rtol", C.c_double), ("maxiter", C.c_int32),
                ("max_krylov", C.c_int32), ("restart", C.c_int32),
                ("max_halvings", C.c_int32), ("init", C.c_int32), ("eps_scale", C.c_double),
                ("max_krylov_total", C.c_int32), ("fp64_fallback", C.c_int32),
                ("krylov_method", C.c_int32),
                ("jv_method", C.c_int32), ("krylov_x0", C.c_int32), ("launch", C.c_int32)]


class SolveStats(C.Structure):
    _fields_ = [("status", C.c_int32), ("newton_iters", C.c_int32),
                ("krylov_iters", C.c_int32), ("f_calls", C.c_int32), ("stalls", C.c_int32),
                ("precond_calls", C.c_int32), ("rho_inf", C.c_double), ("dn_inf", C.c_double),
                ("precision", C.c_int32), ("fp64_evals", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Profile(C.Structure):
    _fields_ = [("steps", C.c_int64), ("formal_launches", C.c_int64), ("formal_ms", C.c_double),
                ("depth_ms", C.c_double), ("assemble_ms", C.c_double), ("solver_ms", C.c_double),
                ("opacity_ms", C.c_double), ("formal_f_launches", C.c_int64),
                ("formal_f_ms", C.c_double), ("last_graph", C.c_int32),
                ("last_formal_wpb", C.c_int32), ("last_tune_ms", C.c_double * 3),
                ("last_captures", C.c_int32), ("pad_profile", C.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("last_tune_ms", "pad_profile")}
        d["last_tune_ms"] = list(self.last_tune_ms)
        return d


NLTE_SOLVE_GRAPH, NLTE_SOLVE_TUNE = 1, 2


class PlanInfo(C.Structure):
    _fields_ = [("ncol", C.c_int32), ("opac_depths", C.c_int32), ("formal_wpb", C.c_int32),
                ("graph", C.c_int32), ("depth_points", C.c_int64), ("tune_ms", C.c_double * 9)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "tune_ms"}
        d["tune_ms"] = list(self.tune_ms)
        return d


NLTE_PLAN_GRAPH, NLTE_PLAN_TUNE = 1, 2


class ServerResult(C.Structure):
    _fields_ = [("stats", SolveStats), ("t_submit_ms", C.c_double), ("t_admit_ms", C.c_double),
                ("t_done_ms", C.c_double)]

    def as_dict(self):
        d = self.stats.as_dict()
        d.update(t_submit_ms=self.t_submit_ms, t_admit_ms=self.t_admit_ms, t_done_ms=self.t_done_ms)
        return d


class ServerInfo(C.Structure):
    _fields_ = [("steps", C.c_int64), ("submitted", C.c_int64), ("completed", C.c_int64),
                ("active", C.c_int32), ("queued", C.c_int32), ("active_bytes", C.c_int64),
                ("busy_ms", C.c_double), ("peak_active_bytes", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libnlte.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch brings its own HIP runtime with the same soname as the system
        # one; loading torch first makes the library bind to that runtime, so
        # one runtime serves both (device pointers, streams).
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} missing: run `python -m paper_2406_17234_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.nlte_last_error.restype = C.c_char_p
        L.nlte_ctx_create.argtypes = [C.c_int, C.POINTER(vp)]
        L.nlte_ctx_destroy.argtypes = [vp]
        L.nlte_ctx_destroy.restype = None
        L.nlte_column_create.argtypes = [vp, C.POINTER(AtmosDesc), C.POINTER(AtomDesc),
                                         C.POINTER(GridDesc), _dp, C.c_int, vp, C.POINTER(vp)]
        L.nlte_column_destroy.argtypes = [vp]
        L.nlte_column_destroy.restype = None
        L.nlte_column_dims.argtypes = [vp, _ip]
        L.nlte_column_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
        L.nlte_column_plan_bytes.argtypes = [C.POINTER(AtmosDesc), C.POINTER(AtomDesc),
                                             C.POINTER(GridDesc), _dp, C.c_int,
                                             C.POINTER(C.c_size_t)]
        L.nlte_lte_populations.argtypes = [vp, vp, vp]
        L.nlte_zero_radiation_populations.argtypes = [vp, vp, vp]
        L.nlte_residual.argtypes = [vp, vp, vp, vp, vp, vp, vp, C.c_int, vp]
        L.nlte_residual_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, vp, C.c_int, vp]
        L.nlte_jvp.argtypes = [vp, vp, vp, C.c_double, vp, vp]
        L.nlte_jvp_tangent.argtypes = [vp, vp, vp, vp, vp]
        L.nlte_solve.argtypes = [vp, vp, vp, C.POINTER(SolveOpts), vp, vp, C.POINTER(SolveStats),
                                 vp]
        L.nlte_solve_batch.argtypes = [vp, C.POINTER(vp), C.c_int32, C.POINTER(vp), C.POINTER(vp),
                                       C.POINTER(SolveOpts), C.POINTER(vp),
                                       C.POINTER(SolveStats), vp]
        L.nlte_solve_opts_default.argtypes = [C.POINTER(SolveOpts)]
        L.nlte_solve_opts_default.restype = None
        L.nlte_voigt_host.argtypes = [C.c_double, _dp, C.c_int32, _dp]
        L.nlte_issue_rate.argtypes = [vp, C.c_int32, C.c_int32, _dp]
        L.nlte_struct_size.argtypes = [C.c_char_p]
        L.nlte_struct_size.restype = C.c_int32
        L.nlte_plan_create.argtypes = [vp, C.POINTER(vp), C.c_int32, C.POINTER(vp), C.POINTER(vp),
                                       C.c_int32, vp, C.POINTER(vp)]
        L.nlte_plan_run.argtypes = [vp, vp]
        L.nlte_plan_info_get.argtypes = [vp, C.POINTER(PlanInfo)]
        L.nlte_plan_destroy.argtypes = [vp]
        L.nlte_plan_destroy.restype = None
        L.nlte_server_create.argtypes = [vp, C.c_size_t, C.c_int32, C.POINTER(SolveOpts),
                                         C.POINTER(vp)]
        L.nlte_server_submit.argtypes = [vp, vp, vp, C.POINTER(C.c_uint64)]
        L.nlte_server_submit_problem.argtypes = [vp, C.POINTER(AtmosDesc), C.POINTER(AtomDesc),
                                                 C.POINTER(GridDesc), _dp, C.c_int, vp,
                                                 C.POINTER(C.c_uint64)]
        L.nlte_server_poll.argtypes = [vp, C.c_uint64, vp, C.POINTER(ServerResult)]
        L.nlte_server_drain.argtypes = [vp, C.c_double]
        L.nlte_server_info_get.argtypes = [vp, C.POINTER(ServerInfo)]
        L.nlte_server_destroy.argtypes = [vp]
        L.nlte_server_destroy.restype = None
        L.nlte_profile_enable.argtypes = [vp, C.c_int]
        L.nlte_profile_read.argtypes = [vp, C.POINTER(Profile)]
        _lib = L
    return _lib


def _check(st):
    if st != NLTE_OK:
        raise NLTEError(st, lib().nlte_last_error().decode())
    return st


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_ip)


def voigt_host(a, v):
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.empty_like(v)
    _check(lib().nlte_voigt_host(float(a), v.ctypes.data_as(_dp), v.size, out.ctypes.data_as(_dp)))
    return out


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    lib().nlte_solve_opts_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


class Context:
    def __init__(self, device: int = 0):
        self.device = device
        h = C.c_void_p()
        _check(lib().nlte_ctx_create(device, C.byref(h)))
        self.h = h

    def profile(self, on: bool = True):
        """Turn kernel timing of solves on/off (clears the accumulators)."""
        _check(lib().nlte_profile_enable(self.h, int(on)))

    def issue_rate(self, op: int, iters: int = 16384) -> float:
        """Lane operations per second of one vector operation (nlte_issue_rate)."""
        r = C.c_double()
        _check(lib().nlte_issue_rate(self.h, op, iters, C.byref(r)))
        return r.value

    def read_profile(self) -> dict:
        p = Profile()
        _check(lib().nlte_profile_read(self.h, C.byref(p)))
        return p.as_dict()

    def close(self):
        if self.h:
            lib().nlte_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _descriptors(problem):
    """Descriptor structs of a problem (any object with ``atom``, ``atmos``,
    ``grid`` and ``C_up`` shaped like the synthetic generator's ``Problem``)
    and the arrays they point into (keep them alive while the structs are
    used)."""
    a, m, g = problem.atmos, problem.atom, problem.grid
    keep = []

    def D(x):
        arr, p = _d(x)
        keep.append(arr)
        return p

    def I(x):
        arr, p = _i(x)
        keep.append(arr)
        return p

    eta_c = getattr(a, "eta_c", None)
    vlos = getattr(a, "vlos", None)
    atm = AtmosDesc(len(a.z), D(a.z), D(a.T), D(a.ne), D(a.ntot), D(a.chi_c),
                    D(a.chi_sca) if a.chi_sca is not None else None,
                    D(eta_c) if eta_c is not None else None,
                    D(vlos) if vlos is not None else None)
    bf_ptr = np.concatenate([[0], np.cumsum([len(x) for x in g.bf_nu])]).astype(np.int32)
    bf_nu = np.concatenate(g.bf_nu) if len(g.bf_nu) else np.zeros(1)
    bf_al = np.concatenate(g.bf_alpha) if len(g.bf_alpha) else np.zeros(1)
    atom = AtomDesc(m.nlev, D(m.E), D(m.g), I(m.stage), m.nline, I(m.line_lo), I(m.line_up),
                    D(m.A_ul), D(m.a_damp), float(m.mass_amu), float(m.vturb), m.nbf,
                    I(m.bf_lo), I(bf_ptr), D(bf_nu), D(bf_al))
    w_nu = getattr(g, "w_nu", None)
    grid = GridDesc(len(g.nu), D(g.nu), I(g.win_lo), I(g.win_hi), len(g.mu), D(g.mu), D(g.w_mu),
                    D(w_nu) if w_nu is not None else None)
    cup = D(np.ascontiguousarray(problem.C_up))
    return atm, atom, grid, cup, keep


class Prepared:
    """The descriptor structs of a problem and the arrays behind them, built
    once (e.g. before a timed window) and passed to calls that take
    descriptors."""

    def __init__(self, problem):
        self.atm, self.atom, self.grid, self.cup, self._keep = _descriptors(problem)


def plan_bytes(problem, precision: int = FP64) -> int:
    """Device bytes a column of this problem would own (host-only validation
    and sizing, nlte_column_plan_bytes); raises NLTEError on bad input."""
    atm, atom, grid, cup, keep = _descriptors(problem)
    nb = C.c_size_t()
    _check(lib().nlte_column_plan_bytes(C.byref(atm), C.byref(atom), C.byref(grid), cup,
                                        int(precision), C.byref(nb)))
    return nb.value


class Column:
    """One column: model atmosphere + model atom + grids (+ collision rates).

    ``problem`` is any object with ``atom``, ``atmos``, ``grid`` and ``C_up``
    attributes shaped like the synthetic generator's ``Problem``.
    """

    def __init__(self, ctx: Context, problem, precision: int = FP64, stream=None):
        import torch
        self.ctx = ctx
        atm, atom, grid, cup, keep = _descriptors(problem)
        h = C.c_void_p()
        torch.cuda.set_device(ctx.device)
        _check(lib().nlte_column_create(ctx.h, C.byref(atm), C.byref(atom), C.byref(grid),
                                        cup, int(precision), _stream(stream), C.byref(h)))
        self.h = h
        dims = (C.c_int32 * 8)()
        _check(lib().nlte_column_dims(h, dims))
        self.nz, self.nlev, self.ntr, self.nline, self.nbf, self.nnu, self.nmu, pf = list(dims)
        self.precision = pf & ~DEPTH_SCAN
        self.depth_scan = bool(pf & DEPTH_SCAN)
        self.device = torch.device("cuda", ctx.device)
        nb = C.c_size_t()
        _check(lib().nlte_column_bytes(h, C.byref(nb)))
        self.bytes = nb.value

    def close(self):
        if getattr(self, "h", None):
            lib().nlte_column_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _empty(self, *shape):
        import torch
        return torch.empty(*shape, dtype=torch.float64, device=self.device)

    def lte(self, stream=None):
        n = self._empty(self.nz, self.nlev)
        _check(lib().nlte_lte_populations(self.h, _ptr(n), _stream(stream)))
        return n

    def zero_radiation(self, stream=None):
        n = self._empty(self.nz, self.nlev)
        _check(lib().nlte_zero_radiation_populations(self.h, _ptr(n), _stream(stream)))
        return n

    def residual(self, n, want_J=False, want_R=False, want_Jbar=False, want_P=False,
                 update_J=False, stream=None, noalloc=False):
        """F(n) and optional outputs (nlte_residual; with noalloc, the
        allocation-free nlte_residual_noalloc)."""
        n = n.contiguous()
        out = {"F": self._empty(self.nz, self.nlev)}
        if want_J:
            out["J"] = self._empty(self.nz, self.nnu)
        if want_R:
            out["R"] = self._empty(self.nz, self.ntr, 2)
        if want_Jbar:
            out["Jbar"] = self._empty(self.nz, max(self.nline, 1))
        if want_P:
            out["P"] = self._empty(self.nz, self.nlev, self.nlev)
        fn = lib().nlte_residual_noalloc if noalloc else lib().nlte_residual
        _check(fn(self.h, _ptr(n), _ptr(out["F"]), _ptr(out.get("J")), _ptr(out.get("R")),
                  _ptr(out.get("Jbar")), _ptr(out.get("P")), int(update_J), _stream(stream)))
        return out

    def jvp(self, n, v, eps, stream=None):
        out = self._empty(self.nz, self.nlev)
        _check(lib().nlte_jvp(self.h, _ptr(n.contiguous()), _ptr(v.contiguous()), float(eps),
                              _ptr(out), _stream(stream)))
        return out

    def jvp_tangent(self, n, v, stream=None):
        out = self._empty(self.nz, self.nlev)
        _check(lib().nlte_jvp_tangent(self.h, _ptr(n.contiguous()), _ptr(v.contiguous()),
                                      _ptr(out), _stream(stream)))
        return out

    def solve(self, n0=None, opts: SolveOpts | None = None, want_J=False, J0=None, stream=None,
              **kw):
        if opts is None:
            opts = default_opts(**kw)
        n = self._empty(self.nz, self.nlev)
        J = self._empty(self.nz, self.nnu) if want_J else None
        st = SolveStats()
        rc = lib().nlte_solve(self.h, _ptr(n0), _ptr(None if J0 is None else J0.contiguous()),
                              C.byref(opts), _ptr(n), _ptr(J), C.byref(st), _stream(stream))
        if rc not in (NLTE_OK, NLTE_E_NOCONV):
            _check(rc)
        return n, J, st.as_dict(), rc


def solve_batch(ctx: Context, columns, opts: SolveOpts | None = None, n0=None, J0=None,
                stream=None, **kw):
    """Solve many columns in shared launches; returns (list of n, stats list, status).
    n0, J0: optional lists of device tensors (entries of J0 may be None)."""
    import torch
    if opts is None:
        opts = default_opts(**kw)
    nc = len(columns)
    outs = [torch.empty(c.nz, c.nlev, dtype=torch.float64, device=c.device) for c in columns]
    cols = (C.c_void_p * nc)(*[c.h for c in columns])
    outp = (C.c_void_p * nc)(*[o.data_ptr() for o in outs])
    n0p = None
    if n0 is not None:
        n0p = (C.c_void_p * nc)(*[x.data_ptr() for x in n0])
    J0p = None
    if J0 is not None:
        J0p = (C.c_void_p * nc)(*[0 if x is None else x.data_ptr() for x in J0])
    stats = (SolveStats * nc)()
    rc = lib().nlte_solve_batch(ctx.h, cols, nc, n0p, J0p, C.byref(opts), outp, stats,
                                _stream(stream))
    if rc not in (NLTE_OK, NLTE_E_NOCONV):
        _check(rc)
    return outs, [s.as_dict() for s in stats], rc


class Server:
    """Continuous-batching solve server (nlte_server_*): submit columns, poll
    tickets.  Columns stay owned by the caller and must not be touched until
    their ticket has been polled."""

    def __init__(self, ctx: Context, hbm_budget: int, max_active: int = 4096,
                 opts: SolveOpts | None = None, **kw):
        if opts is None:
            opts = default_opts(**kw)
        self.ctx = ctx
        h = C.c_void_p()
        _check(lib().nlte_server_create(ctx.h, int(hbm_budget), int(max_active), C.byref(opts),
                                        C.byref(h)))
        self.h = h
        self._keep = {}

    def submit(self, column: Column, n0=None) -> int:
        t = C.c_uint64()
        _check(lib().nlte_server_submit(self.h, column.h, _ptr(n0), C.byref(t)))
        self._keep[t.value] = (column, n0)
        return t.value

    def submit_problem(self, problem, n_out, precision: int = FP64) -> int:
        """Queue a problem whose column the server creates at admission and
        destroys at retirement; the populations land in ``n_out`` (a device
        tensor [nz][nlev] kept alive until the ticket is polled).  ``problem``
        may be a Prepared (descriptors built beforehand)."""
        prep = problem if isinstance(problem, Prepared) else Prepared(problem)
        t = C.c_uint64()
        _check(lib().nlte_server_submit_problem(self.h, C.byref(prep.atm), C.byref(prep.atom),
                                                C.byref(prep.grid), prep.cup, int(precision),
                                                _ptr(n_out), C.byref(t)))
        self._keep[t.value] = (n_out,)
        return t.value

    def poll(self, ticket: int, out=None):
        """(populations or None, result dict) once finished, else None."""
        res = ServerResult()
        st = lib().nlte_server_poll(self.h, C.c_uint64(ticket), _ptr(out), C.byref(res))
        if st == NLTE_E_BUSY:
            return None
        _check(st)
        self._keep.pop(ticket, None)
        return out, res.as_dict()

    def drain(self, timeout_s: float = 600.0):
        _check(lib().nlte_server_drain(self.h, float(timeout_s)))

    def info(self) -> dict:
        i = ServerInfo()
        _check(lib().nlte_server_info_get(self.h, C.byref(i)))
        return i.as_dict()

    def close(self):
        if getattr(self, "h", None):
            lib().nlte_server_destroy(self.h)
            self.h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Residual plan (nlte_plan_*): F(n) of a fixed set of columns in shared
    launches; each run reads n_list[c] and writes F_list[c] (device tensors
    [nz][nlev] that must stay alive with the plan)."""

    def __init__(self, ctx: Context, columns, n_list, F_list, graph: bool = True,
                 tune: bool = False, stream=None):
        nc = len(columns)
        cols = (C.c_void_p * nc)(*[c.h for c in columns])
        ns = (C.c_void_p * nc)(*[x.data_ptr() for x in n_list])
        Fs = (C.c_void_p * nc)(*[x.data_ptr() for x in F_list])
        flags = (NLTE_PLAN_GRAPH if graph else 0) | (NLTE_PLAN_TUNE if tune else 0)
        h = C.c_void_p()
        _check(lib().nlte_plan_create(ctx.h, cols, nc, ns, Fs, flags, _stream(stream), C.byref(h)))
        self.h = h
        self._keep = (list(columns), list(n_list), list(F_list))

    def run(self, stream=None):
        _check(lib().nlte_plan_run(self.h, _stream(stream)))

    def info(self) -> dict:
        i = PlanInfo()
        _check(lib().nlte_plan_info_get(self.h, C.byref(i)))
        return i.as_dict()

    def close(self):
        if getattr(self, "h", None):
            lib().nlte_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
