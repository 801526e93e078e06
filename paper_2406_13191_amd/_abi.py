"""ctypes binding of libdcopf_dual.so (argument marshalling only).

Every step of the ascent runs in the library's HIP kernels; this module only
converts numpy arrays to the C structs of ``include/dcopf_dual.h`` and back.
Importing it raises if the library has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdcopf_dual.so")

DCOPF_OK = 0
STATUS_NAMES = {0: "OK", -1: "E_INVALID", -2: "E_NOMEM", -3: "E_HIP", -4: "E_NONFINITE",
                -5: "E_INFEASIBLE", -7: "E_STATE"}
RULES = {"gdm": 0, "adam": 1, "adagrad": 2}
PRECISIONS = {"fp64": 0, "fp32": 1}
PANELS = {"genbus": 0, "allbus": 1}


class DcopfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Problem_C(C.Structure):
    _fields_ = [("n_bus", C.c_int32), ("n_line", C.c_int32), ("n_gen", C.c_int32),
                ("slack", C.c_int32), ("H", C.POINTER(C.c_double)),
                ("gen_bus", C.POINTER(C.c_int32)), ("c", C.POINTER(C.c_double)),
                ("q", C.POINTER(C.c_double)), ("p_min", C.POINTER(C.c_double)),
                ("p_max", C.POINTER(C.c_double)), ("d", C.POINTER(C.c_double)),
                ("f_max", C.POINTER(C.c_double))]


class Opts_C(C.Structure):
    _fields_ = [("rule", C.c_int32), ("literal", C.c_int32), ("alpha", C.c_double),
                ("rho", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double), ("decay", C.c_double), ("precision", C.c_int32),
                ("panel", C.c_int32), ("graph_iters", C.c_int32), ("qp_dual", C.c_int32),
                ("scheme", C.c_int32)]


class Primal_C(C.Structure):
    _fields_ = [("cost", C.c_double), ("balance", C.c_double), ("max_overload", C.c_double),
                ("sum_overload", C.c_double), ("iterations", C.c_int64),
                ("n_overloaded", C.c_int32)]


class Repair_C(C.Structure):
    _fields_ = [("cost", C.c_double), ("balance", C.c_double), ("max_overload", C.c_double),
                ("max_shift", C.c_double), ("feasible", C.c_int32), ("rounds", C.c_int32),
                ("n_active", C.c_int32), ("pad", C.c_int32)]


class Result_C(C.Structure):
    _fields_ = [("bound", C.c_double), ("gamma_last", C.c_double), ("gap", C.c_double),
                ("iters", C.c_int64), ("iter_of_bound", C.c_int64), ("status", C.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -m paper_2406_13191_amd.build)")
    # PyTorch ships its own HIP runtime under the same soname as ROCm's.  Load
    # it first (when installed) so that this library binds to the same
    # runtime and stream handles from torch are valid here; loading ours first
    # would leave torch with a second, conflicting runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER
    sig = {
        "dcopf_dual_create": (C.c_int, [P(Problem_C), P(Opts_C), C.c_void_p, P(C.c_void_p)]),
        "dcopf_dual_step": (C.c_int, [C.c_void_p, C.c_int64]),
        "dcopf_dual_bound": (C.c_int, [C.c_void_p, P(C.c_double), P(C.c_double),
                                       P(C.c_double), P(C.c_double)]),
        "dcopf_dual_best": (C.c_int, [C.c_void_p, P(C.c_double), P(C.c_int64)]),
        "dcopf_dual_solve": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_double,
                                       C.c_int64, C.c_int64, P(Result_C)]),
        "dcopf_dual_gammas": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, P(C.c_double)]),
        "dcopf_dual_state_len": (C.c_size_t, [C.c_void_p]),
        "dcopf_dual_get_state": (C.c_int, [C.c_void_p, P(C.c_double), C.c_size_t]),
        "dcopf_dual_set_state": (C.c_int, [C.c_void_p, P(C.c_double), C.c_size_t]),
        "dcopf_dual_info": (C.c_int, [C.c_void_p, P(C.c_int32), P(C.c_int64)]),
        "dcopf_dual_scheme": (C.c_int, [C.c_void_p, P(C.c_int32), P(C.c_int32)]),
        "dcopf_dual_average": (C.c_int, [C.c_void_p, C.c_int32]),
        "dcopf_dual_primal": (C.c_int, [C.c_void_p, P(Primal_C), P(C.c_double)]),
        "dcopf_dual_repair": (C.c_int, [C.c_void_p, P(C.c_double), C.c_int32, P(Repair_C),
                                        P(C.c_double)]),
        "dcopf_dual_time_phases": (C.c_int, [C.c_void_p, C.c_int64, P(C.c_double)]),
        "dcopf_dual_destroy": (None, [C.c_void_p]),
        "dcopf_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


# ---------------------------------------------------------------------------
# Device memory from PyTorch's caching allocator (dcopf_set_allocator): the
# handles' buffers then come from, and go back to, torch's pool on the
# handle's stream.  Installed for the importing thread when a GPU is
# present; other threads call use_torch_allocator() themselves.
# ---------------------------------------------------------------------------
_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
lib.dcopf_set_allocator.restype = C.c_int
lib.dcopf_set_allocator.argtypes = [_ALLOC_FN, _FREE_FN, C.c_void_p]
_exiting = False


def _torch_alloc(nbytes, stream, ctx):
    import torch
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
    except Exception:  # noqa: BLE001  (out of memory: the library reports E_NOMEM)
        return None


def _torch_free(ptr, nbytes, stream, ctx):
    if _exiting or not ptr:
        return  # at interpreter exit torch may be gone; the process frees all
    import torch
    torch.cuda.caching_allocator_delete(int(ptr))


_TORCH_ALLOC = _ALLOC_FN(_torch_alloc)
_TORCH_FREE = _FREE_FN(_torch_free)


def use_torch_allocator():
    """Handles created from now on by this thread take their device memory
    from torch's caching allocator."""
    check(lib.dcopf_set_allocator(_TORCH_ALLOC, _TORCH_FREE, None))


def use_hip_allocator():
    """Handles created from now on by this thread use hipMalloc / hipFree."""
    check(lib.dcopf_set_allocator(_ALLOC_FN(), _FREE_FN(), None))


def _mark_exit():
    global _exiting
    _exiting = True


def last_error() -> str:
    return lib.dcopf_last_error().decode()


def check(status: int):
    if status != DCOPF_OK:
        raise DcopfError(status, last_error())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


QP_DUALS = {"closed": 0, "iterated": 1}
SCHEMES = {"auto": 0, "two_pass": 1, "read_once": 2}


def make_opts(rule="gdm", alpha=1e-3, rho=0.9, beta1=0.9, beta2=0.999, eps=1e-8,
              decay=0.0, literal=False, precision="fp32", panel="genbus",
              graph_iters=0, qp_dual="closed", scheme="auto") -> Opts_C:
    return Opts_C(RULES[rule], int(bool(literal)), float(alpha), float(rho), float(beta1),
                  float(beta2), float(eps), float(decay), PRECISIONS[precision],
                  PANELS[panel], int(graph_iters), QP_DUALS[qp_dual], SCHEMES[scheme])


class DualSolver:
    """One DCOPF instance on the GPU (``dcopf_dual_*``).

    ``prob`` has the fields of the paper's statement: H [n_line, n_bus],
    gen_bus, c, q, p_min, p_max, d, f_max, slack.  ``stream`` is a
    hipStream_t handle as an int (e.g. torch.cuda.current_stream().cuda_stream)
    or None for the null stream.
    """

    def __init__(self, prob, stream=None, **opts):
        self._arrays = dict(
            H=_f64(prob.H), gen_bus=np.ascontiguousarray(np.asarray(prob.gen_bus, np.int32)),
            c=_f64(prob.c), q=None if prob.q is None else _f64(prob.q),
            p_min=_f64(prob.p_min), p_max=_f64(prob.p_max), d=_f64(prob.d),
            f_max=_f64(prob.f_max))
        a = self._arrays
        n_line, n_bus = a["H"].shape if a["H"].ndim == 2 else (len(a["f_max"]), len(a["d"]))
        self.n_line, self.n_bus, self.n_gen = int(n_line), int(n_bus), int(a["c"].size)
        pc = Problem_C(self.n_bus, self.n_line, self.n_gen, int(prob.slack), _dptr(a["H"]),
                       a["gen_bus"].ctypes.data_as(C.POINTER(C.c_int32)), _dptr(a["c"]),
                       _dptr(a["q"]) if a["q"] is not None else None, _dptr(a["p_min"]),
                       _dptr(a["p_max"]), _dptr(a["d"]), _dptr(a["f_max"]))
        self.opts = make_opts(**opts)
        h = C.c_void_p()
        check(lib.dcopf_dual_create(C.byref(pc), C.byref(self.opts),
                                    C.c_void_p(stream or 0), C.byref(h)))
        self._h = h
        self._arrays = None  # inputs were copied by create

    # -- lifecycle ---------------------------------------------------------
    def close(self, _destroy=lib.dcopf_dual_destroy):
        # the destroy function is bound at class creation, so that a handle
        # closed while the interpreter shuts down still finds it
        if getattr(self, "_h", None):
            _destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- calls -------------------------------------------------------------
    def step(self, n: int):
        check(lib.dcopf_dual_step(self._h, int(n)))

    def bound(self, want_multipliers=False):
        v = C.c_double()
        if want_multipliers:
            lam = C.c_double()
            mp = np.empty(self.n_line)
            mm = np.empty(self.n_line)
            check(lib.dcopf_dual_bound(self._h, C.byref(v), C.byref(lam), _dptr(mp), _dptr(mm)))
            return v.value, lam.value, mp, mm
        check(lib.dcopf_dual_bound(self._h, C.byref(v), None, None, None))
        return v.value

    def best(self):
        v = C.c_double()
        k = C.c_int64()
        check(lib.dcopf_dual_best(self._h, C.byref(v), C.byref(k)))
        return v.value, k.value

    def solve(self, opt=math.nan, gap_tol=1e-3, dgamma_tol=0.0, max_iters=20000,
              check_every=100):
        r = Result_C()
        check(lib.dcopf_dual_solve(self._h, float(opt), float(gap_tol), float(dgamma_tol),
                                   int(max_iters), int(check_every), C.byref(r)))
        return dict(bound=r.bound, gamma_last=r.gamma_last, gap=r.gap, iters=r.iters,
                    iter_of_bound=r.iter_of_bound, status=r.status)

    def gammas(self, first: int, count: int) -> np.ndarray:
        out = np.empty(int(count))
        check(lib.dcopf_dual_gammas(self._h, int(first), int(count), _dptr(out)))
        return out

    def state_len(self) -> int:
        return int(lib.dcopf_dual_state_len(self._h))

    def get_state(self) -> np.ndarray:
        buf = np.empty(self.state_len())
        check(lib.dcopf_dual_get_state(self._h, _dptr(buf), buf.size))
        return buf

    def set_state(self, buf):
        buf = _f64(buf)
        check(lib.dcopf_dual_set_state(self._h, _dptr(buf), buf.size))

    def average(self, enable: bool = True):
        """Restart (True) or stop (False) the primal average of p*."""
        check(lib.dcopf_dual_average(self._h, 1 if enable else 0))

    def primal(self):
        """The averaged dispatch (generator order) with its cost and residuals."""
        r = Primal_C()
        p = np.zeros(self.n_gen)
        check(lib.dcopf_dual_primal(self._h, C.byref(r), _dptr(p)))
        return dict(cost=r.cost, balance=r.balance, max_overload=r.max_overload,
                    sum_overload=r.sum_overload, iterations=r.iterations,
                    n_overloaded=r.n_overloaded, p=p)

    def repair(self, p=None, max_rounds: int = 32):
        """A feasible dispatch near p (generator order), or near the current
        primal average when p is None; its cost and residuals."""
        r = Repair_C()
        out = np.zeros(self.n_gen)
        pin = None if p is None else _f64(p)
        check(lib.dcopf_dual_repair(self._h, None if pin is None else _dptr(pin),
                                    int(max_rounds), C.byref(r), _dptr(out)))
        return dict(cost=r.cost, balance=r.balance, max_overload=r.max_overload,
                    max_shift=r.max_shift, feasible=bool(r.feasible), rounds=r.rounds,
                    n_active=r.n_active, p=out)

    def time_phases(self, n: int):
        """Average (column pass, line pass) kernel durations in ms over n
        real iterations, each dispatch timed by events attached to it; the
        iterate is restored afterwards."""
        ms = np.zeros(2)
        check(lib.dcopf_dual_time_phases(self._h, int(n), _dptr(ms)))
        return float(ms[0]), float(ms[1])

    def info(self):
        nc = C.c_int32()
        it = C.c_int64()
        check(lib.dcopf_dual_info(self._h, C.byref(nc), C.byref(it)))
        return dict(n_cols=nc.value, iters=it.value)

    def scheme(self):
        sc = C.c_int32()
        g = C.c_int32()
        check(lib.dcopf_dual_scheme(self._h, C.byref(sc), C.byref(g)))
        return dict(scheme={v: k for k, v in SCHEMES.items()}[sc.value], line_groups=g.value)

    # -- state helpers -------------------------------------------------------
    def split_state(self, buf):
        nl = self.n_line
        return dict(k=int(buf[0]), lam=buf[1], v_lam=buf[2], s_lam=buf[3],
                    mu_p=buf[5:5 + nl], mu_m=buf[5 + nl:5 + 2 * nl],
                    v_p=buf[5 + 2 * nl:5 + 3 * nl], v_m=buf[5 + 3 * nl:5 + 4 * nl],
                    s_p=buf[5 + 4 * nl:5 + 5 * nl], s_m=buf[5 + 5 * nl:5 + 6 * nl])


# ---------------------------------------------------------------------------
# Batched instances (dcopf_batch.h)
# ---------------------------------------------------------------------------
class BatchNet_C(C.Structure):
    _fields_ = [("n_bus", C.c_int32), ("n_line", C.c_int32), ("n_gen", C.c_int32),
                ("slack", C.c_int32), ("H", C.POINTER(C.c_double)),
                ("gen_bus", C.POINTER(C.c_int32)), ("p_min", C.POINTER(C.c_double)),
                ("p_max", C.POINTER(C.c_double)), ("f_max", C.POINTER(C.c_double)),
                ("n_inst", C.c_int32), ("d", C.POINTER(C.c_double)),
                ("c", C.POINTER(C.c_double)), ("q", C.POINTER(C.c_double)),
                ("alpha", C.c_double), ("rho", C.c_double)]


class BatchOpts_C(C.Structure):
    _fields_ = [("rule", C.c_int32), ("literal", C.c_int32), ("beta1", C.c_double),
                ("beta2", C.c_double), ("eps", C.c_double), ("decay", C.c_double),
                ("lolo", C.c_int32), ("graph_iters", C.c_int32), ("autotune", C.c_int32),
                ("gamma_cap", C.c_int32)]


def _bind_batch():
    P = C.POINTER
    sig = {
        "dcopf_batch_create": (C.c_int, [P(BatchNet_C), C.c_int32, P(BatchOpts_C), C.c_void_p,
                                         P(C.c_void_p)]),
        "dcopf_batch_step": (C.c_int, [C.c_void_p, C.c_int64]),
        "dcopf_batch_state_len": (C.c_size_t, [C.c_void_p, C.c_int32]),
        "dcopf_batch_get_state": (C.c_int, [C.c_void_p, C.c_int32, P(C.c_double), C.c_size_t]),
        "dcopf_batch_set_state": (C.c_int, [C.c_void_p, C.c_int32, P(C.c_double), C.c_size_t]),
        "dcopf_batch_bound": (C.c_int, [C.c_void_p, P(C.c_double)]),
        "dcopf_batch_best": (C.c_int, [C.c_void_p, P(C.c_double), P(C.c_int64)]),
        "dcopf_batch_solve": (C.c_int, [C.c_void_p, P(C.c_double), C.c_double, C.c_int64,
                                        C.c_int64, P(C.c_int64)]),
        "dcopf_batch_gammas": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, P(C.c_double)]),
        "dcopf_batch_get_multipliers": (C.c_int, [C.c_void_p, C.c_int32, P(C.c_double),
                                                  P(C.c_double), P(C.c_double)]),
        "dcopf_batch_set_multipliers": (C.c_int, [C.c_void_p, C.c_int32, P(C.c_double),
                                                  P(C.c_double), P(C.c_double)]),
        "dcopf_batch_info": (C.c_int, [C.c_void_p, C.c_int32, P(C.c_int32), P(C.c_int64)]),
        "dcopf_batch_set_tiles": (C.c_int, [C.c_void_p, C.c_int32, P(C.c_int32)]),
        "dcopf_batch_set_start_dev": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32]),
        "dcopf_batch_adopt_better": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32,
                                               C.POINTER(C.c_int32)]),
        "dcopf_batch_average": (C.c_int, [C.c_void_p, C.c_int32]),
        "dcopf_batch_primal": (C.c_int, [C.c_void_p, C.c_int32, P(Primal_C), P(C.c_double)]),
        "dcopf_batch_repair": (C.c_int, [C.c_void_p, C.c_int32, P(C.c_double), C.c_int32,
                                         P(Repair_C), P(C.c_double)]),
        "dcopf_batch_time_phases": (C.c_int, [C.c_void_p, C.c_int64, P(C.c_double)]),
        "dcopf_batch_destroy": (None, [C.c_void_p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args


_bind_batch()


class BatchNetwork:
    """One network and its instances: ``base`` has the network fields
    (H, gen_bus, p_min, p_max, f_max, slack); D [B, n_bus] loads,
    Cc [B, n_gen] linear costs, Q [B, n_gen] quadratic costs (or None)."""

    def __init__(self, base, D, Cc, Q=None, alpha=1e-4, rho=0.99):
        self.base, self.alpha, self.rho = base, float(alpha), float(rho)
        self.D = _f64(np.atleast_2d(D))
        self.Cc = _f64(np.atleast_2d(Cc))
        self.Q = None if Q is None else _f64(np.atleast_2d(Q))
        self.B = self.D.shape[0]


class BatchSolver:
    """Many instances advanced together (``dcopf_batch_*``)."""

    def __init__(self, networks, stream=None, rule="gdm", literal=False, beta1=0.9,
                 beta2=0.999, eps=1e-8, decay=0.0, lolo=False, graph_iters=0, autotune=False,
                 gamma_cap=4096):
        self.networks = list(networks)
        keep = []
        arr = (BatchNet_C * len(self.networks))()
        for k, n in enumerate(self.networks):
            b = n.base
            H = _f64(b.H)
            gb = np.ascontiguousarray(np.asarray(b.gen_bus, np.int32))
            pmin, pmax, fmax = _f64(b.p_min), _f64(b.p_max), _f64(b.f_max)
            keep += [H, gb, pmin, pmax, fmax, n.D, n.Cc, n.Q]
            arr[k] = BatchNet_C(H.shape[1], H.shape[0], gb.size, int(b.slack), _dptr(H),
                                gb.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(pmin),
                                _dptr(pmax), _dptr(fmax), n.B, _dptr(n.D), _dptr(n.Cc),
                                _dptr(n.Q) if n.Q is not None else None, n.alpha, n.rho)
        self.opts = BatchOpts_C(RULES[rule], int(bool(literal)), float(beta1), float(beta2),
                                float(eps), float(decay), int(bool(lolo)), int(graph_iters),
                                int(bool(autotune)), int(gamma_cap))
        h = C.c_void_p()
        check(lib.dcopf_batch_create(arr, len(self.networks), C.byref(self.opts),
                                     C.c_void_p(stream or 0), C.byref(h)))
        self._h = h
        self.sizes = [n.B for n in self.networks]
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)]).astype(int)
        self.n_total = int(self.offsets[-1])

    def close(self, _destroy=lib.dcopf_batch_destroy):
        # the destroy function is bound at class creation, so that a handle
        # closed while the interpreter shuts down still finds it
        if getattr(self, "_h", None):
            _destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def step(self, n: int):
        check(lib.dcopf_batch_step(self._h, int(n)))

    def bound(self) -> np.ndarray:
        out = np.empty(self.n_total)
        check(lib.dcopf_batch_bound(self._h, _dptr(out)))
        return out

    def best(self):
        v = np.empty(self.n_total)
        k = np.empty(self.n_total, np.int64)
        check(lib.dcopf_batch_best(self._h, _dptr(v), k.ctypes.data_as(C.POINTER(C.c_int64))))
        return v, k

    def solve(self, opt, gap_tol=1e-3, max_iters=5000, check_every=100) -> np.ndarray:
        opt = _f64(opt)
        hit = np.empty(self.n_total, np.int64)
        check(lib.dcopf_batch_solve(self._h, _dptr(opt), float(gap_tol), int(max_iters),
                                    int(check_every), hit.ctypes.data_as(C.POINTER(C.c_int64))))
        return hit

    def gammas(self, first: int, count: int) -> np.ndarray:
        out = np.empty((int(count), self.n_total))
        check(lib.dcopf_batch_gammas(self._h, int(first), int(count), _dptr(out)))
        return out

    def get_multipliers(self, net: int):
        n = self.networks[net]
        nl = np.asarray(n.base.f_max).size
        lam = np.empty(n.B)
        mp = np.empty((n.B, nl))
        mm = np.empty((n.B, nl))
        check(lib.dcopf_batch_get_multipliers(self._h, int(net), _dptr(lam), _dptr(mp),
                                              _dptr(mm)))
        return lam, mp, mm

    def set_multipliers(self, net: int, lam, mu_p, mu_m):
        lam, mu_p, mu_m = _f64(lam), _f64(mu_p), _f64(mu_m)
        check(lib.dcopf_batch_set_multipliers(self._h, int(net), _dptr(lam), _dptr(mu_p),
                                              _dptr(mu_m)))

    def get_state(self, net: int) -> np.ndarray:
        """Network `net`'s whole ascent state (dcopf_batch_get_state layout)."""
        buf = np.empty(lib.dcopf_batch_state_len(self._h, int(net)))
        check(lib.dcopf_batch_get_state(self._h, int(net), _dptr(buf), buf.size))
        return buf

    def set_state(self, net: int, buf):
        buf = _f64(buf)
        check(lib.dcopf_batch_set_state(self._h, int(net), _dptr(buf), buf.size))

    def split_state(self, net: int, buf) -> dict:
        """The fields of a state buffer: k, lam, v_lam, s_lam [B] and mu_p,
        mu_m, v_p, v_m, s_p, s_m [B, n_line]."""
        n = self.networks[net]
        B, nl = n.B, np.asarray(n.base.f_max).size
        out = dict(k=int(buf[0]), lam=buf[1:1 + B], v_lam=buf[1 + B:1 + 2 * B],
                   s_lam=buf[1 + 2 * B:1 + 3 * B])
        o = 1 + 3 * B
        for name in ("mu_p", "mu_m", "v_p", "v_m", "s_p", "s_m"):
            out[name] = buf[o:o + B * nl].reshape(B, nl)
            o += B * nl
        return out

    @staticmethod
    def pack_state(k, lam, v_lam, s_lam, mu_p, mu_m, v_p, v_m, s_p, s_m) -> np.ndarray:
        """Inverse of split_state."""
        parts = [[float(k)], lam, v_lam, s_lam, mu_p, mu_m, v_p, v_m, s_p, s_m]
        return np.concatenate([np.ravel(np.asarray(x, dtype=np.float64)) for x in parts])

    def set_start_dev(self, net: int, y_ptr: int, ld: int):
        """Start multipliers from a device FP32 array [n_inst, ld] laid out
        [mu+, mu-, lambda] (e.g. a torch tensor's data_ptr())."""
        check(lib.dcopf_batch_set_start_dev(self._h, int(net), C.c_void_p(y_ptr), int(ld)))

    def adopt_better(self, net: int, other: "BatchSolver", other_net: int):
        """Where an instance of `other` (the same instances from another
        start, at the same iteration) has the larger exact bound, its state
        replaces this batch's (dcopf_batch_adopt_better).  Returns the
        per-instance flags (1: taken from `other`)."""
        kept = np.zeros(self.sizes[net], np.int32)
        check(lib.dcopf_batch_adopt_better(self._h, int(net), other._h, int(other_net),
                                           kept.ctypes.data_as(C.POINTER(C.c_int32))))
        return kept

    def info(self, net: int):
        cfg = np.zeros(4, np.int32)
        it = C.c_int64()
        check(lib.dcopf_batch_info(self._h, int(net), cfg.ctypes.data_as(C.POINTER(C.c_int32)),
                                   C.byref(it)))
        return dict(w_tile=(int(cfg[0]), int(cfg[1])), w_split=int(cfg[2]),
                    f_tile=(int(cfg[3]) // 1000, int(cfg[3]) % 1000), iters=it.value)

    def set_tiles(self, net: int, w_tile, w_split: int, f_tile):
        """Pin network `net`'s tile shapes, e.g. an earlier ``info(net)``."""
        cfg = np.array([w_tile[0], w_tile[1], w_split, f_tile[0] * 1000 + f_tile[1]], np.int32)
        check(lib.dcopf_batch_set_tiles(self._h, int(net),
                                        cfg.ctypes.data_as(C.POINTER(C.c_int32))))

    def average(self, enable: bool = True):
        """Restart (True) or stop (False) every instance's primal average."""
        check(lib.dcopf_batch_average(self._h, 1 if enable else 0))

    def primal(self, net: int):
        """Network `net`'s averaged dispatches [n_inst, n_gen] (generator
        order) with per-instance cost and residuals, as arrays."""
        n = self.networks[net]
        ng = np.asarray(n.base.gen_bus).size
        r = (Primal_C * n.B)()
        p = np.zeros((n.B, ng))
        check(lib.dcopf_batch_primal(self._h, int(net), r, _dptr(p)))
        f = lambda k: np.array([getattr(x, k) for x in r])
        return dict(cost=f("cost"), balance=f("balance"), max_overload=f("max_overload"),
                    sum_overload=f("sum_overload"), iterations=int(r[0].iterations),
                    n_overloaded=f("n_overloaded"), p=p)

    def repair(self, net: int, p=None, max_rounds: int = 32):
        """Feasible dispatches near p [n_inst, n_gen] (generator order), or
        near the current primal averages when p is None, for network `net`."""
        n = self.networks[net]
        ng = np.asarray(n.base.gen_bus).size
        r = (Repair_C * n.B)()
        out = np.zeros((n.B, ng))
        pin = None if p is None else _f64(np.reshape(p, (n.B, ng)))
        check(lib.dcopf_batch_repair(self._h, int(net), None if pin is None else _dptr(pin),
                                     int(max_rounds), r, _dptr(out)))
        f = lambda k: np.array([getattr(x, k) for x in r])
        return dict(cost=f("cost"), balance=f("balance"), max_overload=f("max_overload"),
                    max_shift=f("max_shift"), feasible=f("feasible").astype(bool),
                    rounds=f("rounds"), n_active=f("n_active"), p=out)

    def time_phases(self, n: int):
        ms = np.zeros(3)
        check(lib.dcopf_batch_time_phases(self._h, int(n), _dptr(ms)))
        return tuple(float(v) for v in ms)


# ---------------------------------------------------------------------------
# Warm-start network (dcopf_mlp.h)
# ---------------------------------------------------------------------------
class MlpConfig_C(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("h1", C.c_int32), ("h2", C.c_int32),
                ("n_out", C.c_int32), ("max_batch", C.c_int32), ("beta1", C.c_double),
                ("beta2", C.c_double), ("eps", C.c_double)]


def _bind_mlp():
    P = C.POINTER
    sig = {
        "dcopf_mlp_create": (C.c_int, [P(MlpConfig_C), C.c_void_p, P(C.c_void_p)]),
        "dcopf_mlp_param_count": (C.c_size_t, [C.c_void_p]),
        "dcopf_mlp_get_params": (C.c_int, [C.c_void_p, P(C.c_float), C.c_size_t]),
        "dcopf_mlp_set_params": (C.c_int, [C.c_void_p, P(C.c_float), C.c_size_t]),
        "dcopf_mlp_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
        "dcopf_mlp_train_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                           C.c_double, P(C.c_double)]),
        "dcopf_mlp_get_grads": (C.c_int, [C.c_void_p, P(C.c_float), C.c_size_t]),
        "dcopf_mlp_time_train": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                           C.c_int32, P(C.c_double)]),
        "dcopf_mlp_column_stats": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                            C.c_void_p, C.c_void_p]),
        "dcopf_mlp_standardize": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                           C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
        "dcopf_mlp_fold_standardizers": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p,
                                                  C.c_void_p, C.c_void_p]),
        "dcopf_mlp_destroy": (None, [C.c_void_p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args


_bind_mlp()


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_float))


class MLP:
    """Warm-start network on the GPU.  Data arguments of forward/train_step
    are device addresses (ints, e.g. torch_tensor.data_ptr()) of contiguous
    FP32 arrays."""

    def __init__(self, n_in, h1, h2, n_out, max_batch=256, beta1=0.9, beta2=0.999, eps=1e-8,
                 stream=None):
        self.dims = (n_in, h1, h2, n_out)
        cfg = MlpConfig_C(n_in, h1, h2, n_out, max_batch, beta1, beta2, eps)
        h = C.c_void_p()
        check(lib.dcopf_mlp_create(C.byref(cfg), C.c_void_p(stream or 0), C.byref(h)))
        self._h = h
        self.n_params = int(lib.dcopf_mlp_param_count(h))

    def close(self, _destroy=lib.dcopf_mlp_destroy):
        # the destroy function is bound at class creation, so that a handle
        # closed while the interpreter shuts down still finds it
        if getattr(self, "_h", None):
            _destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def shapes(self):
        n_in, h1, h2, n_out = self.dims
        return [(h1, n_in), (h1,), (h2, h1), (h2,), (n_out, h2), (n_out,)]

    def pack(self, params):
        return np.ascontiguousarray(np.concatenate([np.asarray(p, np.float32).ravel()
                                                    for p in params]))

    def unpack(self, flat):
        out, o = [], 0
        for s in self.shapes():
            n = int(np.prod(s))
            out.append(flat[o:o + n].reshape(s))
            o += n
        return out

    def set_params(self, params):
        flat = self.pack(params)
        check(lib.dcopf_mlp_set_params(self._h, _fptr(flat), flat.size))

    def get_params(self):
        flat = np.empty(self.n_params, np.float32)
        check(lib.dcopf_mlp_get_params(self._h, _fptr(flat), flat.size))
        return self.unpack(flat)

    def get_grads(self):
        flat = np.empty(self.n_params, np.float32)
        check(lib.dcopf_mlp_get_grads(self._h, _fptr(flat), flat.size))
        return self.unpack(flat)

    def forward(self, x_ptr: int, batch: int, y_ptr: int):
        check(lib.dcopf_mlp_forward(self._h, C.c_void_p(x_ptr), int(batch), C.c_void_p(y_ptr)))

    def train_step(self, x_ptr: int, t_ptr: int, batch: int, lr: float, want_loss=False):
        loss = C.c_double()
        check(lib.dcopf_mlp_train_step(self._h, C.c_void_p(x_ptr), C.c_void_p(t_ptr), int(batch),
                                       float(lr), C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def time_train(self, x_ptr: int, t_ptr: int, batch: int, n: int) -> float:
        ms = C.c_double()
        check(lib.dcopf_mlp_time_train(self._h, C.c_void_p(x_ptr), C.c_void_p(t_ptr),
                                       int(batch), int(n), C.byref(ms)))
        return ms.value

    def column_stats(self, a_ptr: int, rows: int, cols: int, mean_ptr: int, std_ptr: int):
        check(lib.dcopf_mlp_column_stats(self._h, C.c_void_p(a_ptr), int(rows), int(cols),
                                         C.c_void_p(mean_ptr), C.c_void_p(std_ptr)))

    def standardize(self, a_ptr: int, rows: int, cols: int, mean_ptr: int, std_ptr: int,
                    out_ptr: int, inverse=False):
        check(lib.dcopf_mlp_standardize(self._h, C.c_void_p(a_ptr), int(rows), int(cols),
                                        C.c_void_p(mean_ptr), C.c_void_p(std_ptr),
                                        int(bool(inverse)), C.c_void_p(out_ptr)))

    def fold_standardizers(self, xm_ptr: int, xs_ptr: int, ym_ptr: int, ys_ptr: int):
        check(lib.dcopf_mlp_fold_standardizers(self._h, C.c_void_p(xm_ptr), C.c_void_p(xs_ptr),
                                               C.c_void_p(ym_ptr), C.c_void_p(ys_ptr)))


# ---------------------------------------------------------------------------
# PTDF construction (dcopf_ptdf.h)
# ---------------------------------------------------------------------------
lib.dcopf_ptdf.restype = C.c_int
lib.dcopf_ptdf.argtypes = [C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                           C.POINTER(C.c_double), C.c_int32, C.c_void_p, C.c_void_p]


def ptdf(n_bus: int, fbus, tbus, b, slack: int, H_ptr: int, stream=None):
    """H_a of the network into the device buffer at H_ptr (n_line * n_bus
    doubles, row-major, e.g. a torch tensor's data_ptr())."""
    fb = np.ascontiguousarray(np.asarray(fbus, np.int32))
    tb = np.ascontiguousarray(np.asarray(tbus, np.int32))
    bb = _f64(b)
    check(lib.dcopf_ptdf(int(n_bus), int(fb.size), fb.ctypes.data_as(C.POINTER(C.c_int32)),
                         tb.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(bb), int(slack),
                         C.c_void_p(stream or 0), C.c_void_p(H_ptr)))


lib.dcopf_ptdf_noalloc.restype = C.c_int
lib.dcopf_ptdf_noalloc.argtypes = lib.dcopf_ptdf.argtypes
PTDF_NOALLOC_MAX_BUS = 2049
PTDF_NOALLOC_MAX_LINE = 16384


def ptdf_noalloc(n_bus: int, fbus, tbus, b, slack: int, H_ptr: int, stream=None):
    """As ptdf(), through the entry point that allocates no device memory
    (fixed workspace inside the library; at most PTDF_NOALLOC_MAX_BUS buses
    and PTDF_NOALLOC_MAX_LINE lines)."""
    fb = np.ascontiguousarray(np.asarray(fbus, np.int32))
    tb = np.ascontiguousarray(np.asarray(tbus, np.int32))
    bb = _f64(b)
    check(lib.dcopf_ptdf_noalloc(int(n_bus), int(fb.size),
                                 fb.ctypes.data_as(C.POINTER(C.c_int32)),
                                 tb.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(bb), int(slack),
                                 C.c_void_p(stream or 0), C.c_void_p(H_ptr)))


def _install_default_allocator():
    import atexit
    atexit.register(_mark_exit)
    try:
        import torch
    except ImportError:
        return
    # DCOPF_ALLOCATOR=hip keeps hipMalloc / hipFree (for tools that do not
    # follow memory handed out by torch's pool)
    if torch.cuda.is_available() and os.environ.get("DCOPF_ALLOCATOR", "torch") != "hip":
        use_torch_allocator()


_install_default_allocator()
