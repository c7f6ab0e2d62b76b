"""Python binding of the l1ls HIP library (``include/l1ls.h``).

Argument marshalling only: every step of the solver runs in the HIP kernels
of ``libl1ls.so``.  PyTorch supplies device memory (output tensors) and
streams.  Importing this package never falls back to another
implementation: if the shared library is missing, ``lib()`` raises.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libl1ls.so")

L1LS_OK = 0
L1LS_NOT_CONVERGED = 1
F32, F64 = 0, 1
OP_STORED, OP_MATRIX_FREE, OP_BLOCKED = 0, 1, 2
STORE_F32, STORE_F64, STORE_BLK32, STORE_MF_WINDOWS, STORE_WINDOWS = 1, 2, 4, 8, 32
REQ_FP64_FINISH = 1
SIGMA_ALTERNATING, SIGMA_UNIFORM = 0, 1
XSTAR_TABLE1, XSTAR_OSGEN, XSTAR_OSGEN3 = 0, 1, 2

_STATUS = {0: "ok", 1: "not converged", -1: "invalid argument", -2: "device allocation failed",
           -3: "HIP runtime error", -4: "non-finite value", -5: "invalid state", -6: "unsupported"}


class L1lsError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: l1ls status {status} ({_STATUS.get(status, '?')})")


LAYOUT_NATURAL, LAYOUT_STAGE = 0, 1


class GenOpts(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("storage", ctypes.c_uint32), ("stream", ctypes.c_void_p),
                ("layout", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("s", ctypes.c_int64), ("nnz", ctypes.c_int64),
        ("rounds", ctypes.c_int32), ("storage", ctypes.c_uint32), ("layout", ctypes.c_int32),
        ("kappa", ctypes.c_double), ("tau", ctypes.c_double), ("L", ctypes.c_double),
        ("f_star", ctypes.c_double), ("seed", ctypes.c_uint64),
        ("b_dev", ctypes.c_void_p), ("x_star_dev", ctypes.c_void_p), ("g_dev", ctypes.c_void_p),
        ("e_dev", ctypes.c_void_p), ("sigma_dev", ctypes.c_void_p), ("support_dev", ctypes.c_void_p),
        ("perm_n_dev", ctypes.c_void_p), ("perm_m_dev", ctypes.c_void_p),
        ("cs_n_dev", ctypes.c_void_p * 2), ("cs_m_dev", ctypes.c_void_p * 2),
        ("csr_ptr_dev", ctypes.c_void_p), ("csr_col_dev", ctypes.c_void_p),
        ("csr_val32_dev", ctypes.c_void_p), ("csr_val64_dev", ctypes.c_void_p),
        ("csc_ptr_dev", ctypes.c_void_p), ("csc_row_dev", ctypes.c_void_p),
        ("csc_val32_dev", ctypes.c_void_p), ("csc_val64_dev", ctypes.c_void_p),
    ]


class SolveOpts(ctypes.Structure):
    _fields_ = [
        ("tau", ctypes.c_double), ("rel_gap_tol", ctypes.c_double), ("max_iter", ctypes.c_int64),
        ("check_every", ctypes.c_int32), ("precision", ctypes.c_int32), ("op", ctypes.c_int32),
        ("polish", ctypes.c_int32), ("L", ctypes.c_double), ("x0_dev", ctypes.c_void_p),
        ("stream", ctypes.c_void_p), ("time_kernels", ctypes.c_int32),
        ("mu", ctypes.c_double), ("pcg_rtol", ctypes.c_double), ("max_backtrack", ctypes.c_int32),
        ("pcg_maxit", ctypes.c_int32), ("hessian", ctypes.c_int32), ("tile_chunk", ctypes.c_int32),
        ("f_target", ctypes.c_double), ("pcdm_p", ctypes.c_double), ("graph", ctypes.c_int32),
        ("persist_rows", ctypes.c_int32), ("pcdm_tau_nice", ctypes.c_int32),
    ]


class Report(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int64), ("inner", ctypes.c_int64), ("primal", ctypes.c_double),
        ("dual", ctypes.c_double), ("rel_gap", ctypes.c_double), ("rel_err", ctypes.c_double),
        ("seconds", ctypes.c_double), ("converged", ctypes.c_int32), ("polish_rounds", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Request(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("kappa", ctypes.c_double), ("s", ctypes.c_int64),
        ("tau", ctypes.c_double), ("seed", ctypes.c_uint64), ("rounds", ctypes.c_int32), ("flags", ctypes.c_int32),
        ("rel_gap_tol", ctypes.c_double), ("max_iter", ctypes.c_int64),
    ]


class SgtParams(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("m", ctypes.c_int64), ("s", ctypes.c_int64), ("theta", ctypes.c_double),
        ("sigma_odd", ctypes.c_double), ("sigma_even", ctypes.c_double), ("x_neg", ctypes.c_double),
        ("x_pos", ctypes.c_double), ("tau", ctypes.c_double), ("seed", ctypes.c_uint64),
        ("sigma_law", ctypes.c_int32), ("xstar_law", ctypes.c_int32), ("sigma_scale", ctypes.c_double),
        ("sigma_shift", ctypes.c_double), ("gamma", ctypes.c_double), ("s1", ctypes.c_int64), ("s2", ctypes.c_int64),
    ]


class SgtDesc(ctypes.Structure):
    _fields_ = [
        ("params", SgtParams), ("L", ctypes.c_double), ("f_star", ctypes.c_double), ("c", ctypes.c_double),
        ("s_rot", ctypes.c_double), ("b_dev", ctypes.c_void_p), ("sigma_min", ctypes.c_double),
        ("sigma_max", ctypes.c_double), ("colscale_dev", ctypes.c_void_p),
    ]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", ctypes.c_void_p)]


# Every symbol include/l1ls.h declares, with (restype, argtypes).
_P = ctypes.c_void_p
_SIGS = {
    "l1ls_generate": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_int64,
                                     ctypes.c_double, ctypes.c_uint64, ctypes.POINTER(_P)]),
    "l1ls_generate_ex": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_int64,
                                        ctypes.c_double, ctypes.c_uint64, ctypes.POINTER(GenOpts),
                                        ctypes.POINTER(_P)]),
    "l1ls_set_allocator": (ctypes.c_int, [ctypes.POINTER(Allocator)]),
    "l1ls_instance_info": (ctypes.c_int, [_P, ctypes.POINTER(Info)]),
    "l1ls_instance_bytes": (ctypes.c_size_t, [_P]),
    "l1ls_free": (None, [_P]),
    "l1ls_apply": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P, _P]),
    "l1ls_power_iteration": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P, ctypes.POINTER(ctypes.c_double),
                                            _P]),
    "l1ls_objective_gap": (ctypes.c_int, [_P, ctypes.c_double, _P, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), _P]),
    "l1ls_objective_gap_noalloc": (ctypes.c_int, [_P, ctypes.c_double, _P, ctypes.POINTER(ctypes.c_double),
                                                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                                  _P]),
    "l1ls_solve_opts_default": (None, [ctypes.POINTER(SolveOpts)]),
    "l1ls_solve_fista": (ctypes.c_int, [_P, ctypes.POINTER(SolveOpts), _P, ctypes.POINTER(Report)]),
    "l1ls_solve_cg_newton": (ctypes.c_int, [_P, ctypes.POINTER(SolveOpts), _P, ctypes.POINTER(Report)]),
    "l1ls_solve_pcdm": (ctypes.c_int, [_P, ctypes.POINTER(SolveOpts), _P, ctypes.POINTER(Report)]),
    "l1ls_fista_create": (ctypes.c_int, [_P, ctypes.POINTER(SolveOpts), ctypes.POINTER(_P)]),
    "l1ls_fista_iterate": (ctypes.c_int, [_P, ctypes.c_int64]),
    "l1ls_fista_report": (ctypes.c_int, [_P, ctypes.POINTER(Report)]),
    "l1ls_fista_get_x": (ctypes.c_int, [_P, _P]),
    "l1ls_fista_kernel_times": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double),
                                               ctypes.POINTER(ctypes.c_int64)]),
    "l1ls_fista_kernel_times_ex": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                                  ctypes.POINTER(ctypes.c_int64)]),
    "l1ls_fista_destroy": (None, [_P]),
    "l1ls_batch_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_size_t, ctypes.POINTER(SolveOpts),
                                         ctypes.POINTER(_P)]),
    "l1ls_batch_add": (ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.POINTER(ctypes.c_int32)]),
    "l1ls_batch_add_ex": (ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                         ctypes.POINTER(ctypes.c_int32)]),
    "l1ls_batch_iterate": (ctypes.c_int, [_P, ctypes.c_int64]),
    "l1ls_batch_poll": (ctypes.c_int, [_P, ctypes.POINTER(Report), ctypes.POINTER(ctypes.c_int32)]),
    "l1ls_batch_get_x": (ctypes.c_int, [_P, ctypes.c_int32, _P]),
    "l1ls_batch_remove": (ctypes.c_int, [_P, ctypes.c_int32]),
    "l1ls_batch_destroy": (None, [_P]),
    "l1ls_instance_footprint": (ctypes.c_size_t, [_P]),
    "l1ls_server_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32, _P,
                                          ctypes.POINTER(_P)]),
    "l1ls_server_submit": (ctypes.c_int, [_P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_int64)]),
    "l1ls_server_tick": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "l1ls_server_completed": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]),
    "l1ls_server_take": (ctypes.c_int, [_P, ctypes.c_int64, _P, ctypes.POINTER(Report)]),
    "l1ls_server_stats": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_size_t)]),
    "l1ls_server_destroy": (None, [_P]),
    "l1ls_request_footprint": (ctypes.c_size_t, [ctypes.POINTER(Request)]),
    "l1ls_solve_fista_batched": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                                ctypes.POINTER(SolveOpts), ctypes.POINTER(_P),
                                                ctypes.POINTER(Report)]),
    "l1ls_solve_fista_path": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                             ctypes.POINTER(SolveOpts), _P, ctypes.POINTER(Report)]),
    "l1ls_sgt_params_default": (None, [ctypes.c_int64, ctypes.c_uint64, ctypes.POINTER(SgtParams)]),
    "l1ls_sgt_bytes": (ctypes.c_size_t, [ctypes.c_int64]),
    "l1ls_sgt_solve_bytes": (ctypes.c_size_t, [ctypes.c_int64]),
    "l1ls_sgt_generate": (ctypes.c_int, [ctypes.POINTER(SgtParams), _P, ctypes.POINTER(_P)]),
    "l1ls_sgt_describe": (ctypes.c_int, [_P, ctypes.POINTER(SgtDesc)]),
    "l1ls_sgt_free": (None, [_P]),
    "l1ls_sgt_planted": (ctypes.c_int, [_P, _P, _P, _P]),
    "l1ls_sgt_apply": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P]),
    "l1ls_sgt_objective_gap": (ctypes.c_int, [_P, ctypes.c_double, _P, ctypes.POINTER(ctypes.c_double),
                                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                               _P]),
    "l1ls_sgt_solve_cg_newton": (ctypes.c_int, [_P, ctypes.POINTER(SolveOpts), _P, ctypes.POINTER(Report)]),
    "l1ls_sgt_kappa_rho": (ctypes.c_int, [_P, ctypes.c_double, ctypes.POINTER(ctypes.c_double), _P]),
    "l1ls_sgt_solve_fista": (ctypes.c_int, [_P, ctypes.POINTER(SolveOpts), _P, ctypes.POINTER(Report)]),
    "l1ls_sgt_solve_pcdm": (ctypes.c_int, [_P, ctypes.POINTER(SolveOpts), _P, ctypes.POINTER(Report)]),
    "l1ls_sgt_newton_create": (ctypes.c_int, [_P, ctypes.POINTER(SolveOpts), _P, ctypes.POINTER(_P)]),
    "l1ls_sgt_newton_step": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.POINTER(Report)]),
    "l1ls_sgt_newton_destroy": (None, [_P]),
    "l1ls_sgt_kernel_times": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
    "l1ls_tune_get": (ctypes.c_int32, [ctypes.c_char_p]),
    "l1ls_tune_set": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_int32]),
    "l1ls_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
    "l1ls_version": (ctypes.c_int32, []),
}
EXPORTED = tuple(_SIGS)

_lib = None


def lib():
    """The loaded libl1ls.so (raises if it was not built).  On first load it
    installs PyTorch's caching allocator as the library's device-memory
    source (l1ls_set_allocator), unless L1LS_HIP_MALLOC=1."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
        if os.environ.get("L1LS_HIP_MALLOC") != "1":
            use_torch_allocator()
    return _lib


# State of the PyTorch allocator shim.  The callbacks are kept alive for the
# life of the process (blocks made through them may be returned while the
# interpreter shuts down); after exit handlers ran, returns are dropped, since
# the process releases the device memory anyway.
_torch_alloc = {"installed": False, "live": True, "keep": None}


def _make_torch_callbacks():
    import torch
    raw_alloc = torch._C._cuda_cudaCachingAllocator_raw_alloc
    raw_delete = torch._C._cuda_cudaCachingAllocator_raw_delete
    current_stream = torch.cuda.current_stream

    def alloc(ctx, nbytes):
        try:
            return raw_alloc(int(nbytes), current_stream().cuda_stream)
        except Exception:
            return None  # the library reports L1LS_E_NOMEM

    def free(ctx, ptr, nbytes):
        if _torch_alloc["live"] and ptr:
            try:
                raw_delete(ptr)
            except Exception:
                pass

    return _ALLOC_FN(alloc), _FREE_FN(free)


def use_torch_allocator():
    """Route the library's device memory through PyTorch's caching allocator
    (torch.cuda.memory_allocated then counts it)."""
    if _torch_alloc["installed"]:
        return
    try:
        fa, ff = _make_torch_callbacks()
    except ImportError:
        return
    spec = Allocator(fa, ff, None)
    _check(_lib.l1ls_set_allocator(ctypes.byref(spec)), "l1ls_set_allocator")
    # one reference that is never dropped: the trampolines outlive every object
    ctypes.pythonapi.Py_IncRef(ctypes.py_object(fa))
    ctypes.pythonapi.Py_IncRef(ctypes.py_object(ff))
    _torch_alloc.update(installed=True, keep=(fa, ff, spec))
    import atexit
    atexit.register(_torch_alloc.__setitem__, "live", False)


def use_hip_malloc():
    """New device blocks from hipMalloc again (blocks made through PyTorch go
    back to it)."""
    _check(lib().l1ls_set_allocator(None), "l1ls_set_allocator")
    _torch_alloc["installed"] = False


def _check(status, where, allow=(L1LS_OK,)):
    if status not in allow:
        raise L1lsError(status, where)
    return status


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class Instance:
    """Owns an l1ls_instance (l1ls_generate / l1ls_generate_ex)."""

    def __init__(self, handle, params):
        self._h = handle
        self.params = params

    @property
    def handle(self):
        return self._h

    def nbytes(self):
        """Device bytes the instance holds (l1ls_instance_bytes)."""
        return int(lib().l1ls_instance_bytes(self._h))

    def info(self):
        inf = Info()
        _check(lib().l1ls_instance_info(self._h, ctypes.byref(inf)), "l1ls_instance_info")
        return inf

    def free(self):
        if self._h:
            lib().l1ls_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def l1ls_generate(m, n, kappa, s, tau, seed, rounds=1, storage=STORE_F32 | STORE_F64, stream=None,
                  layout=LAYOUT_STAGE):
    h = ctypes.c_void_p()
    o = GenOpts(rounds, storage, _stream(stream), layout)
    _check(lib().l1ls_generate_ex(m, n, kappa, s, tau, seed, ctypes.byref(o), ctypes.byref(h)),
           "l1ls_generate_ex")
    return Instance(h, dict(m=m, n=n, kappa=kappa, s=s, tau=tau, seed=seed, rounds=rounds, storage=storage,
                            layout=layout))


generate = l1ls_generate


def solve_opts(**kw):
    o = SolveOpts()
    lib().l1ls_solve_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if k == "stream":
            o.stream = _stream(v)
        elif k == "x0":
            o.x0_dev = _ptr(v)
        else:
            setattr(o, k, v)
    if "stream" not in kw:
        o.stream = _stream(None)
    return o


def l1ls_apply(inst, trans, op, prec, x_in, x_out, stream=None):
    _check(lib().l1ls_apply(inst.handle, trans, op, prec, _ptr(x_in), _ptr(x_out), _stream(stream)),
           "l1ls_apply")


def l1ls_power_iteration(inst, iters, op=OP_STORED, v0=None, stream=None):
    """lambda_max(A^T A) by the FP64 power method (l1ls_power_iteration)."""
    lam = ctypes.c_double()
    _check(lib().l1ls_power_iteration(inst.handle, op, int(iters), _ptr(v0), ctypes.byref(lam), _stream(stream)),
           "l1ls_power_iteration")
    return lam.value


def l1ls_objective_gap(inst, tau, x, stream=None):
    P, D, g = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().l1ls_objective_gap(inst.handle, tau, _ptr(x), ctypes.byref(P), ctypes.byref(D),
                                    ctypes.byref(g), _stream(stream)), "l1ls_objective_gap")
    return P.value, D.value, g.value


def l1ls_objective_gap_noalloc(inst, tau, x, stream=None):
    P, D, g = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().l1ls_objective_gap_noalloc(inst.handle, tau, _ptr(x), ctypes.byref(P), ctypes.byref(D),
                                            ctypes.byref(g), _stream(stream)), "l1ls_objective_gap_noalloc")
    return P.value, D.value, g.value


def _solve(fn, name, inst, x_out, kw):
    import torch
    n = inst.params["n"]
    if x_out is None:
        x_out = torch.empty(n, dtype=torch.float64, device="cuda")
    o = solve_opts(**kw)
    rep = Report()
    st = _check(fn(inst.handle, ctypes.byref(o), _ptr(x_out), ctypes.byref(rep)), name,
                allow=(L1LS_OK, L1LS_NOT_CONVERGED))
    return x_out, rep.as_dict(), st


def l1ls_solve_fista(inst, x_out=None, **kw):
    return _solve(lib().l1ls_solve_fista, "l1ls_solve_fista", inst, x_out, kw)


def l1ls_solve_cg_newton(inst, x_out=None, **kw):
    return _solve(lib().l1ls_solve_cg_newton, "l1ls_solve_cg_newton", inst, x_out, kw)


def l1ls_solve_pcdm(inst, x_out=None, **kw):
    kw.setdefault("precision", F64)
    return _solve(lib().l1ls_solve_pcdm, "l1ls_solve_pcdm", inst, x_out, kw)


class Fista:
    """The stepping interface (l1ls_fista_create / iterate / report / get_x)."""

    def __init__(self, inst, **kw):
        self.inst = inst
        self._opts = solve_opts(**kw)
        self._keep = kw.get("x0")
        h = ctypes.c_void_p()
        _check(lib().l1ls_fista_create(inst.handle, ctypes.byref(self._opts), ctypes.byref(h)),
               "l1ls_fista_create")
        self._h = h

    def iterate(self, iters):
        _check(lib().l1ls_fista_iterate(self._h, int(iters)), "l1ls_fista_iterate")

    def report(self):
        rep = Report()
        _check(lib().l1ls_fista_report(self._h, ctypes.byref(rep)), "l1ls_fista_report")
        return rep.as_dict()

    def get_x(self, x_out=None):
        import torch
        if x_out is None:
            x_out = torch.empty(self.inst.params["n"], dtype=torch.float64, device="cuda")
        _check(lib().l1ls_fista_get_x(self._h, _ptr(x_out)), "l1ls_fista_get_x")
        return x_out

    def kernel_times(self, slots=3):
        ms = (ctypes.c_double * slots)()
        cnt = (ctypes.c_int64 * slots)()
        _check(lib().l1ls_fista_kernel_times_ex(self._h, slots, ms, cnt), "l1ls_fista_kernel_times_ex")
        return list(ms), list(cnt)

    def destroy(self):
        if self._h:
            lib().l1ls_fista_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


# --------------------------------------------------------------------------
# device -> host copies of raw device pointers (instance arrays)
# --------------------------------------------------------------------------
_hip = None


def _hiprt():
    global _hip
    if _hip is None:
        import torch  # noqa: F401  (loads the HIP runtime torch was built with)
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.restype = ctypes.c_int
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipDeviceSynchronize.restype = ctypes.c_int
    return _hip


def device_to_numpy(ptr, count, dtype):
    """Copy `count` elements of numpy `dtype` from a raw device pointer."""
    import numpy as np
    out = np.empty(int(count), dtype=dtype)
    if count == 0:
        return out
    rt = _hiprt()
    if rt.hipDeviceSynchronize() != 0:
        raise RuntimeError("hipDeviceSynchronize failed")
    rc = rt.hipMemcpy(out.ctypes.data, ptr, out.nbytes, 2)  # hipMemcpyDeviceToHost
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed ({rc})")
    return out


class Batch:
    """Continuous batching of FISTA solves (l1ls_batch_*)."""

    def __init__(self, capacity, hbm_budget_bytes=0, **kw):
        self.capacity = int(capacity)
        self._opts = solve_opts(**kw)
        h = ctypes.c_void_p()
        _check(lib().l1ls_batch_create(self.capacity, int(hbm_budget_bytes), ctypes.byref(self._opts),
                                       ctypes.byref(h)), "l1ls_batch_create")
        self._h = h
        self._inst = {}

    def add(self, inst, tau=0.0, rel_gap_tol=None, max_iter=0):
        slot = ctypes.c_int32(-1)
        if rel_gap_tol is None and not max_iter:
            st = lib().l1ls_batch_add(self._h, inst.handle, float(tau), ctypes.byref(slot))
        else:
            tol = -1.0 if rel_gap_tol is None else float(rel_gap_tol)
            st = lib().l1ls_batch_add_ex(self._h, inst.handle, float(tau), tol, int(max_iter), ctypes.byref(slot))
        if st != L1LS_OK:
            raise L1lsError(st, "l1ls_batch_add")
        self._inst[slot.value] = inst
        return slot.value

    def try_add(self, inst, tau=0.0):
        """Slot index, or None when the budget or the slots are exhausted."""
        slot = ctypes.c_int32(-1)
        st = lib().l1ls_batch_add(self._h, inst.handle, float(tau), ctypes.byref(slot))
        if st in (-2, -5):
            return None
        _check(st, "l1ls_batch_add")
        self._inst[slot.value] = inst
        return slot.value

    def iterate(self, iters):
        _check(lib().l1ls_batch_iterate(self._h, int(iters)), "l1ls_batch_iterate")

    def poll(self):
        reps = (Report * self.capacity)()
        act = ctypes.c_int32(0)
        _check(lib().l1ls_batch_poll(self._h, reps, ctypes.byref(act)), "l1ls_batch_poll")
        return [r.as_dict() for r in reps], act.value

    def get_x(self, slot, x_out=None):
        import torch
        if x_out is None:
            x_out = torch.empty(self._inst[slot].params["n"], dtype=torch.float64, device="cuda")
        _check(lib().l1ls_batch_get_x(self._h, int(slot), _ptr(x_out)), "l1ls_batch_get_x")
        return x_out

    def remove(self, slot):
        _check(lib().l1ls_batch_remove(self._h, int(slot)), "l1ls_batch_remove")
        self._inst.pop(slot, None)

    def destroy(self):
        if self._h:
            lib().l1ls_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Server:
    """FIFO request queue in front of a batch (l1ls_server_*)."""

    def __init__(self, max_slots, hbm_budget_bytes=0, iters_per_tick=16, check_every=16, stream=None):
        h = ctypes.c_void_p()
        _check(lib().l1ls_server_create(int(max_slots), int(hbm_budget_bytes), int(iters_per_tick),
                                        int(check_every), _stream(stream), ctypes.byref(h)), "l1ls_server_create")
        self._h = h
        self._n = {}

    def submit(self, m, n, kappa, s, tau, seed, rounds=2, rel_gap_tol=1e-5, max_iter=100000, fp64_finish=False):
        r = Request(int(m), int(n), float(kappa), int(s), float(tau), int(seed), int(rounds),
                    REQ_FP64_FINISH if fp64_finish else 0, float(rel_gap_tol), int(max_iter))
        rid = ctypes.c_int64(-1)
        _check(lib().l1ls_server_submit(self._h, ctypes.byref(r), ctypes.byref(rid)), "l1ls_server_submit")
        self._n[rid.value] = int(n)
        return rid.value

    def tick(self):
        a = ctypes.c_int32(0)
        c = ctypes.c_int32(0)
        _check(lib().l1ls_server_tick(self._h, ctypes.byref(a), ctypes.byref(c)), "l1ls_server_tick")
        return a.value, c.value

    def completed(self, cap=4096):
        ids = (ctypes.c_int64 * cap)()
        k = lib().l1ls_server_completed(self._h, ids, cap)
        return list(ids[:k])

    def take(self, rid, want_x=True):
        import torch
        n = self._n.get(rid)
        x = torch.empty(n, dtype=torch.float64, device="cuda") if (want_x and n) else None
        rep = Report()
        _check(lib().l1ls_server_take(self._h, int(rid), _ptr(x), ctypes.byref(rep)), "l1ls_server_take")
        self._n.pop(rid, None)
        return x, rep.as_dict()

    def stats(self):
        q = ctypes.c_int32(0)
        r = ctypes.c_int32(0)
        u = ctypes.c_size_t(0)
        _check(lib().l1ls_server_stats(self._h, ctypes.byref(q), ctypes.byref(r), ctypes.byref(u)),
               "l1ls_server_stats")
        return q.value, r.value, u.value

    def destroy(self):
        if self._h:
            lib().l1ls_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def request_footprint(m, n, rounds=2, kappa=1e2, s=0, tau=1.0, rel_gap_tol=1e-6, max_iter=1, fp64_finish=False):
    """Admission estimate of a serving request (bytes; 0 if the request is invalid)."""
    r = Request(int(m), int(n), float(kappa), int(s), float(tau), 0, int(rounds),
                REQ_FP64_FINISH if fp64_finish else 0, float(rel_gap_tol), int(max_iter))
    return int(lib().l1ls_request_footprint(ctypes.byref(r)))


def instance_footprint(inst):
    return int(lib().l1ls_instance_footprint(inst.handle))


def l1ls_solve_fista_batched(insts, taus=None, **kw):
    import torch
    count = len(insts)
    handles = (ctypes.c_void_p * count)(*[i.handle.value for i in insts])
    tv = (ctypes.c_double * count)(*(taus if taus is not None else [0.0] * count))
    xs = [torch.empty(i.params["n"], dtype=torch.float64, device="cuda") for i in insts]
    xp = (ctypes.c_void_p * count)(*[x.data_ptr() for x in xs])
    reps = (Report * count)()
    o = solve_opts(**kw)
    st = _check(lib().l1ls_solve_fista_batched(handles, tv, count, ctypes.byref(o), xp, reps),
                "l1ls_solve_fista_batched", allow=(L1LS_OK, L1LS_NOT_CONVERGED))
    return xs, [r.as_dict() for r in reps], st


def l1ls_solve_fista_path(inst, taus, **kw):
    """Solutions for every tau in `taus` (<= 64): an n x k FP64 tensor (column c for taus[c])."""
    import torch
    k = len(taus)
    n = inst.params["n"]
    X = torch.empty((k, n), dtype=torch.float64, device="cuda")   # row c = column c of the n x k output
    tv = (ctypes.c_double * k)(*[float(t) for t in taus])
    reps = (Report * k)()
    o = solve_opts(**kw)
    st = _check(lib().l1ls_solve_fista_path(inst.handle, tv, k, ctypes.byref(o), _ptr(X), reps),
                "l1ls_solve_fista_path", allow=(L1LS_OK, L1LS_NOT_CONVERGED))
    return X, [r.as_dict() for r in reps], st


# ---- A = Sigma G^T instance class (sections 8.4 to 8.9) ----------------------
def sgt_params(n, seed, **kw):
    """The section 8.9 parameters for n (l1ls_sgt_params_default), with
    overrides; s1 and s2 follow an overridden s unless given."""
    p = SgtParams()
    lib().l1ls_sgt_params_default(n, seed, ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    if "s" in kw and "s1" not in kw:
        p.s1 = p.s // 2
    if "s" in kw and "s2" not in kw:
        p.s2 = p.s - p.s1
    return p


class SgtInstance:
    """Owns an l1ls_sgt (l1ls_sgt_generate)."""

    def __init__(self, params, stream=None):
        h = ctypes.c_void_p()
        _check(lib().l1ls_sgt_generate(ctypes.byref(params), _stream(stream), ctypes.byref(h)),
               "l1ls_sgt_generate")
        self._h = h
        self.params = {f: getattr(params, f) for f, _ in SgtParams._fields_}

    @property
    def handle(self):
        return self._h

    def describe(self):
        d = SgtDesc()
        _check(lib().l1ls_sgt_describe(self._h, ctypes.byref(d)), "l1ls_sgt_describe")
        return d

    def planted(self, x_star=None, g=None, stream=None):
        _check(lib().l1ls_sgt_planted(self._h, _ptr(x_star), _ptr(g), _stream(stream)), "l1ls_sgt_planted")

    def apply(self, trans, x_in, x_out, stream=None):
        _check(lib().l1ls_sgt_apply(self._h, trans, _ptr(x_in), _ptr(x_out), _stream(stream)), "l1ls_sgt_apply")

    def objective_gap(self, tau, x, stream=None):
        P, D, g = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(lib().l1ls_sgt_objective_gap(self._h, tau, _ptr(x), ctypes.byref(P), ctypes.byref(D),
                                             ctypes.byref(g), _stream(stream)), "l1ls_sgt_objective_gap")
        return P.value, D.value, g.value

    def kappa_rho(self, rho, stream=None):
        k = ctypes.c_double()
        _check(lib().l1ls_sgt_kappa_rho(self._h, rho, ctypes.byref(k), _stream(stream)), "l1ls_sgt_kappa_rho")
        return k.value

    def solve_fista(self, x_out=None, **kw):
        import torch
        if x_out is None:
            x_out = torch.empty(self.params["n"], dtype=torch.float64, device="cuda")
        o = solve_opts(**kw)
        rep = Report()
        st = _check(lib().l1ls_sgt_solve_fista(self._h, ctypes.byref(o), _ptr(x_out), ctypes.byref(rep)),
                    "l1ls_sgt_solve_fista", allow=(L1LS_OK, L1LS_NOT_CONVERGED))
        return x_out, rep.as_dict(), st

    def solve_pcdm(self, x_out=None, **kw):
        import torch
        if x_out is None:
            x_out = torch.empty(self.params["n"], dtype=torch.float64, device="cuda")
        o = solve_opts(**kw)
        rep = Report()
        st = _check(lib().l1ls_sgt_solve_pcdm(self._h, ctypes.byref(o), _ptr(x_out), ctypes.byref(rep)),
                    "l1ls_sgt_solve_pcdm", allow=(L1LS_OK, L1LS_NOT_CONVERGED))
        return x_out, rep.as_dict(), st

    def solve_cg_newton(self, x_out=None, **kw):
        import torch
        if x_out is None:
            x_out = torch.empty(self.params["n"], dtype=torch.float64, device="cuda")
        o = solve_opts(**kw)
        rep = Report()
        st = _check(lib().l1ls_sgt_solve_cg_newton(self._h, ctypes.byref(o), _ptr(x_out), ctypes.byref(rep)),
                    "l1ls_sgt_solve_cg_newton", allow=(L1LS_OK, L1LS_NOT_CONVERGED))
        return x_out, rep.as_dict(), st

    def newton(self, x_out=None, **kw):
        """A SgtNewton stepping object (l1ls_sgt_newton_create)."""
        return SgtNewton(self, x_out, **kw)

    def kernel_times(self):
        """{pass: (total ms, launches)} of the last solve with time_kernels=1."""
        ms = (ctypes.c_double * 3)()
        calls = (ctypes.c_int64 * 3)()
        _check(lib().l1ls_sgt_kernel_times(self._h, ms, calls), "l1ls_sgt_kernel_times")
        return {k: (ms[q], calls[q]) for q, k in enumerate(("pcg_iteration", "line_search", "newton_setup"))}

    def fista_kernel_times(self):
        """{pass: (total ms, launches)} of the last FISTA solve with time_kernels=1."""
        t = self.kernel_times()
        return {"iteration": t["pcg_iteration"], "gap": t["line_search"]}

    def free(self):
        if self._h:
            lib().l1ls_sgt_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def sgt_bytes(n):
    return lib().l1ls_sgt_bytes(n)


def sgt_solve_bytes(n):
    return lib().l1ls_sgt_solve_bytes(n)


class SgtNewton:
    """CG-Newton on a SgtInstance one call at a time (l1ls_sgt_newton_*)."""

    def __init__(self, inst, x_out=None, **kw):
        import torch
        self.inst = inst
        self.x = x_out if x_out is not None else torch.empty(inst.params["n"], dtype=torch.float64, device="cuda")
        self._o = solve_opts(**kw)
        h = ctypes.c_void_p()
        _check(lib().l1ls_sgt_newton_create(inst.handle, ctypes.byref(self._o), _ptr(self.x), ctypes.byref(h)),
               "l1ls_sgt_newton_create")
        self._h = h

    def step(self, steps=1):
        rep = Report()
        st = _check(lib().l1ls_sgt_newton_step(self._h, steps, ctypes.byref(rep)), "l1ls_sgt_newton_step",
                    allow=(L1LS_OK, L1LS_NOT_CONVERGED))
        return rep.as_dict(), st

    def destroy(self):
        if self._h:
            lib().l1ls_sgt_newton_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def tune_get(key):
    """The autotuner's cached choice for `key` (l1ls_tune_get), -1 if none."""
    return int(lib().l1ls_tune_get(key.encode()))


def tune_set(key, choice):
    _check(lib().l1ls_tune_set(key.encode(), int(choice)), "l1ls_tune_set")
