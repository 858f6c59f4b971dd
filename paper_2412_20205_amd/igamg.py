"""Thin ctypes binding of libigamg.so (include/igamg.h, include/igamg_host.h).

Argument marshalling only: every step of the solver runs in the HIP library.
Device vectors are contiguous float64 torch tensors on the GPU; their data
pointers are passed through.  The current torch stream is handed to the
library at setup so that torch and the solver share one stream.

The library must be built (paper_2412_20205_amd/build.py); loading fails loudly
when it is missing -- there is no fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libigamg.so")

OK, EINVAL, ENOMEM, EHIP, ENOTSPD, EBREAKDOWN, ENOCONV, ENONFINITE = 0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENOTSPD",
                -5: "EBREAKDOWN", -6: "ENOCONV", -7: "ENONFINITE"}
UNIT_SQUARE, QUARTER_ANNULUS, UNIT_CUBE, QUARTER_ANNULUS_EXACT = 0, 1, 2, 3
PDE_POISSON, PDE_ELLIPTIC_1, PDE_ELLIPTIC_2, PDE_ADVECTION_DIFFUSION = 0, 1, 2, 3
SMOOTH_MCGS, SMOOTH_LEXGS, SMOOTH_JACOBI, SMOOTH_LEARNED = 0, 1, 2, 3
EXTRAP_NONE, RRE, MPE = 0, 1, 2
PRECOND_VCYCLE, PRECOND_RRE, PRECOND_MPE = 0, 1, 2
FP64, FP32_IR = 0, 1


class Geometry(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("n_el", ctypes.c_int), ("r_in", ctypes.c_double),
                ("r_out", ctypes.c_double)]


class Options(ctypes.Structure):
    _fields_ = [("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("smoother", ctypes.c_int),
                ("omega", ctypes.c_double), ("precision", ctypes.c_int),
                ("n_el_coarsest", ctypes.c_int), ("use_graphs", ctypes.c_int),
                ("tail_items", ctypes.c_int), ("stored_stencil", ctypes.c_int),
                ("mu", ctypes.c_int), ("monitor", ctypes.c_int), ("pde", ctypes.c_int),
                ("row_sweeps", ctypes.c_int),
                ("stream", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("restarts", ctypes.c_int), ("vcycles", ctypes.c_int),
                ("breakdowns", ctypes.c_int), ("learned_fallbacks", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("gen_residual", ctypes.c_double),
                ("residual_checks", ctypes.c_int), ("setup_ms", ctypes.c_double),
                ("solve_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class State(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int), ("q", ctypes.c_int), ("restarts", ctypes.c_int),
                ("vcycles", ctypes.c_int), ("breakdowns", ctypes.c_int),
                ("learned_fallbacks", ctypes.c_int), ("residual_checks", ctypes.c_int),
                ("learned_off", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("gen_scale", ctypes.c_double), ("monitor_ratio", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Tuning(ctypes.Structure):
    _fields_ = [("tail_items", ctypes.c_int), ("tail_top", ctypes.c_int), ("num_levels", ctypes.c_int),
                ("row_class", ctypes.c_int * 16), ("learned_kernel", ctypes.c_int * 16),
                ("vcycle_ms", ctypes.c_double)]

    def as_dict(self):
        n = self.num_levels
        return {"tail_items": self.tail_items, "tail_top": self.tail_top, "num_levels": n,
                "row_class": list(self.row_class)[:n], "learned_kernel": list(self.learned_kernel)[:n],
                "vcycle_ms": self.vcycle_ms}


class TrainOptions(ctypes.Structure):
    _fields_ = [("n_rhs", ctypes.c_int), ("modes", ctypes.c_void_p), ("n_modes", ctypes.c_int),
                ("vcycles_per_rhs", ctypes.c_int), ("epochs", ctypes.c_int), ("batch", ctypes.c_int),
                ("lr", ctypes.c_double), ("seed", ctypes.c_ulonglong), ("val_modes", ctypes.c_void_p),
                ("val_n_modes", ctypes.c_int), ("val_vcycles", ctypes.c_int),
                ("solve_tol", ctypes.c_double), ("per_level_accept", ctypes.c_int)]


class TrainReport(ctypes.Structure):
    _fields_ = [("levels_trained", ctypes.c_int), ("patches", ctypes.c_int),
                ("loss_first", ctypes.c_double * 16), ("loss_last", ctypes.c_double * 16),
                ("rho_plain", ctypes.c_double), ("rho_learned", ctypes.c_double),
                ("accepted", ctypes.c_int), ("train_ms", ctypes.c_double),
                ("rho_plain_level", ctypes.c_double * 16), ("rho_learned_level", ctypes.c_double * 16),
                ("accepted_level", ctypes.c_int * 16)]

    def as_dict(self):
        return {"levels_trained": self.levels_trained, "patches": self.patches,
                "loss_first": list(self.loss_first), "loss_last": list(self.loss_last),
                "rho_plain": self.rho_plain, "rho_learned": self.rho_learned,
                "accepted": self.accepted, "train_ms": self.train_ms,
                "rho_plain_level": list(self.rho_plain_level),
                "rho_learned_level": list(self.rho_learned_level),
                "accepted_level": list(self.accepted_level)}


class IgamgError(RuntimeError):
    def __init__(self, status, func, msg):
        super().__init__("%s failed: %s (%s)" % (func, STATUS_NAMES.get(status, status), msg))
        self.status = status


_lib = None
_P = ctypes.c_void_p
class Problem1D(ctypes.Structure):
    _fields_ = [("n_el", ctypes.c_int), ("degree", ctypes.c_int), ("levels", ctypes.c_int),
                ("smoother", ctypes.c_int), ("nu1", ctypes.c_int), ("nu2", ctypes.c_int),
                ("mu", ctypes.c_int), ("omega", ctypes.c_double), ("method", ctypes.c_int),
                ("q", ctypes.c_int)]


class Stats1D(ctypes.Structure):
    _fields_ = [("restarts", ctypes.c_int), ("vcycles", ctypes.c_int),
                ("breakdowns", ctypes.c_int), ("converged", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("l2_error", ctypes.c_double),
                ("solve_ms", ctypes.c_double)]


_i = ctypes.c_int
_d = ctypes.c_double
_ll = ctypes.c_longlong

_SIGNATURES = {
    "igamg_options_default": (None, [ctypes.POINTER(Options)]),
    "igamg_setup": (_i, [ctypes.POINTER(Geometry), _i, _i, ctypes.POINTER(Options),
                         ctypes.POINTER(_P)]),
    "igamg_destroy": (None, [_P]),
    "igamg_ndof": (_i, [_P, ctypes.POINTER(_ll)]),
    "igamg_num_levels": (_i, [_P, ctypes.POINTER(_i)]),
    "igamg_level_ndof": (_i, [_P, _i, ctypes.POINTER(_ll)]),
    "igamg_set_rhs": (_i, [_P, _P, _i]),
    "igamg_set_rhs_field": (_i, [_P, _P, _i]),
    "igamg_set_rhs_builtin": (_i, [_P]),
    "igamg_get_rhs": (_i, [_P, _P]),
    "igamg_vcycle": (_i, [_P, _P]),
    "igamg_set_precision": (_i, [_P, _i]),
    "igamg_extrapolate": (_i, [_P, _i, _i, _P, _P, _P]),
    "igamg_generalized_residual": (_i, [_P, ctypes.POINTER(_d)]),
    "igamg_solve_fgmres": (_i, [_P, _d, _i, _i, _i, _i, _P, ctypes.POINTER(Stats)]),
    "igamg_solve": (_i, [_P, _d, _i, _i, _i, _P, ctypes.POINTER(Stats)]),
    "igamg_residual": (_i, [_P, _P, ctypes.POINTER(_d)]),
    "igamg_get_state": (_i, [_P, _P, ctypes.POINTER(State)]),
    "igamg_set_state": (_i, [_P, ctypes.POINTER(State)]),
    "igamg_get_operator_rows": (_i, [_P, _i, _P, _i, _P]),
    "igamg_apply": (_i, [_P, _i, _P, _P]),
    "igamg_smooth": (_i, [_P, _i, _P, _P, _i]),
    "igamg_restrict": (_i, [_P, _i, _P, _P]),
    "igamg_prolong_add": (_i, [_P, _i, _P, _P]),
    "igamg_coarse_solve": (_i, [_P, _P, _P]),
    "igamg_extrap_coeffs": (_i, [_P, _i, _i, _P, _P, ctypes.POINTER(_i)]),
    "igamg_extrap_coeffs_noalloc": (_i, [_P, _i, _i, _P, _P, ctypes.POINTER(_i)]),
    "igamg_profile_smoother": (_i, [_P, _i, _i, _i, ctypes.POINTER(_d), ctypes.POINTER(_d),
                                    ctypes.POINTER(_i)]),
    "igamg_train_options_default": (None, [ctypes.POINTER(TrainOptions)]),
    "igamg_train_smoother": (_i, [_P, ctypes.POINTER(TrainOptions), ctypes.POINTER(TrainReport)]),
    "igamg_set_learned": (_i, [_P, _i]),
    "igamg_get_smoother_weights": (_i, [_P, _i, _P, ctypes.c_size_t]),
    "igamg_set_smoother_weights": (_i, [_P, _i, _P, ctypes.c_size_t]),
    "igamg_smoother_forward": (_i, [_P, _i, _P, _P]),
    "igamg_smoother_loss_grad": (_i, [_P, _i, _P, _P, ctypes.POINTER(_d), _P]),
    "igamg_setup_batch": (_i, [_i, _P, _P, ctypes.POINTER(Options), ctypes.POINTER(_P)]),
    "igamg_destroy_batch": (None, [_P]),
    "igamg_batch_instance": (_i, [_P, _i, ctypes.POINTER(_P)]),
    "igamg_solve_batch": (_i, [_P, _d, _i, _i, _P, _P]),
    "igamg_autotune": (_i, [_P, ctypes.POINTER(_i), ctypes.POINTER(_d)]),
    "igamg_get_tuning": (_i, [_P, ctypes.POINTER(Tuning)]),
    "igamg_set_tuning": (_i, [_P, ctypes.POINTER(Tuning)]),
    "igamg_problem1d_default": (None, [ctypes.POINTER(Problem1D)]),
    "igamg_setup_1d": (_i, [_i, ctypes.POINTER(Problem1D), _P, ctypes.POINTER(_P)]),
    "igamg_destroy_1d": (None, [_P]),
    "igamg_ndof_1d": (_ll, [_P, _i]),
    "igamg_set_rhs_1d": (_i, [_P, _i, _P]),
    "igamg_get_rhs_1d": (_i, [_P, _i, _P]),
    "igamg_cycles_1d": (_i, [_P, _i, _P]),
    "igamg_solve_1d": (_i, [_P, _d, _i, _P, ctypes.POINTER(Stats1D)]),
    "igamg_last_error": (ctypes.c_char_p, []),
    "igamg_host_gauss_legendre": (_i, [_i, _P, _P]),
    "igamg_host_basis": (_i, [_i, _i, _d, _P, _P, ctypes.POINTER(_i)]),
    "igamg_host_prolongation_1d": (_i, [_i, _i, _P]),
    "igamg_host_bands": (_i, [_i, _i, _i, _i, _P, _P]),
    "igamg_host_coarse_inverse": (_i, [_i, _P, _i, _P]),
}


def lib():
    """Load libigamg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libigamg.so is not built: run paper_2412_20205_amd/build.py "
                              "(or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status, func):
    if status != OK:
        raise IgamgError(status, func, lib().igamg_last_error().decode())


def _check_len(t, n, what):
    if n is not None and t.numel() != n:
        raise ValueError("%s has %d entries, the call reads/writes %d" % (what, t.numel(), n))


def _ptr(t, n=None, what="vector"):
    """Device pointer of a contiguous float64 CUDA tensor of n entries (or None).

    The length is checked first (the library reads and writes exactly n
    values).  Work already queued by torch on its current stream is completed
    first, so the library's stream sees the tensor's final contents."""
    if t is None:
        return None
    _check_len(t, n, what)
    import torch
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 device tensor")
    torch.cuda.current_stream().synchronize()
    return ctypes.c_void_p(t.data_ptr())


def _ptr32(t, n=None, what="vector"):
    """Device pointer of a contiguous float32 CUDA tensor of n entries."""
    _check_len(t, n, what)
    import torch
    if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError("expected a contiguous float32 device tensor")
    torch.cuda.current_stream().synchronize()
    return ctypes.c_void_p(t.data_ptr())


def _ptrs(*specs):
    """Pointers of several (tensor, length, name) vectors: every length is
    checked before any tensor is inspected further."""
    for t, n, what in specs:
        if t is not None:
            _check_len(t, n, what)
    return [_ptr(t, n, what) for t, n, what in specs]


def _ptrs32(*specs):
    for t, n, what in specs:
        _check_len(t, n, what)
    return [_ptr32(t, n, what) for t, n, what in specs]


def _ptr_list(xs, lengths, what):
    """ctypes array of the device pointers of xs (one per problem)."""
    if len(xs) != len(lengths):
        raise ValueError("%d %s given for %d problems" % (len(xs), what, len(lengths)))
    for x, n in zip(xs, lengths):
        _check_len(x, n, what)
    return (ctypes.c_void_p * len(xs))(*[_ptr(x, n, what).value for x, n in zip(xs, lengths)])


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def default_options(**kw):
    o = Options()
    lib().igamg_options_default(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Solver:
    """One solver context (owns its device data; see include/igamg.h)."""

    def __init__(self, geometry, n_el, degree, levels=0, stream=None, radii=(0.0, 0.0), **opts):
        import torch
        if stream is None:
            cs = torch.cuda.current_stream()
            # the legacy default stream cannot be captured into graphs: let the
            # library create its own (blocking) stream in that case
            stream = None if cs.cuda_stream == 0 else cs.cuda_stream
        o = default_options(**opts)
        o.stream = stream
        self._stream_ptr = stream
        g = Geometry(geometry, n_el, radii[0], radii[1])
        h = _P()
        _check(lib().igamg_setup(ctypes.byref(g), degree, levels, ctypes.byref(o),
                                 ctypes.byref(h)), "igamg_setup")
        self._h = h
        self.geometry, self.n_el, self.degree = geometry, n_el, degree
        self.options = o

    def close(self):
        if getattr(self, "_h", None):
            lib().igamg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def ndof(self):
        n = _ll()
        _check(lib().igamg_ndof(self._h, ctypes.byref(n)), "igamg_ndof")
        return n.value

    @property
    def num_levels(self):
        n = _i()
        _check(lib().igamg_num_levels(self._h, ctypes.byref(n)), "igamg_num_levels")
        return n.value

    def level_ndof(self, level):
        n = _ll()
        _check(lib().igamg_level_ndof(self._h, level, ctypes.byref(n)), "igamg_level_ndof")
        return n.value

    def set_rhs(self, b):
        """b: float64 device tensor or host numpy array of ndof entries."""
        if isinstance(b, np.ndarray):
            b = np.ascontiguousarray(b, dtype=np.float64)
            if b.size != self.ndof:
                raise ValueError("wrong length")
            _check(lib().igamg_set_rhs(self._h, _np_ptr(b), 0), "igamg_set_rhs")
        else:
            _check(lib().igamg_set_rhs(self._h, _ptr(b, self.ndof, "b"), 1), "igamg_set_rhs")

    def set_rhs_field(self, modes):
        """modes: one row (a, k, l, phi) per sine mode in 2D, (a, k, l, m, phi) in 3D."""
        modes = np.ascontiguousarray(modes, dtype=np.float64)
        width = 5 if self.geometry == UNIT_CUBE else 4
        if modes.ndim != 2 or modes.shape[1] != width or modes.shape[0] < 1:
            raise ValueError("mode table must have shape (n_modes, %d)" % width)
        _check(lib().igamg_set_rhs_field(self._h, _np_ptr(modes), modes.shape[0]),
               "igamg_set_rhs_field")

    def set_rhs_builtin(self):
        _check(lib().igamg_set_rhs_builtin(self._h), "igamg_set_rhs_builtin")

    def get_rhs(self, out):
        _check(lib().igamg_get_rhs(self._h, _ptr(out, self.ndof, "out")), "igamg_get_rhs")
        return out

    def set_precision(self, precision):
        _check(lib().igamg_set_precision(self._h, precision), "igamg_set_precision")

    def vcycle(self, x):
        _check(lib().igamg_vcycle(self._h, _ptr(x, self.ndof, "x")), "igamg_vcycle")
        return x

    def extrapolate(self, method, q, x, iterates=None):
        gamma = np.zeros(q + 1)
        n = self.ndof
        px, pit = _ptrs((x, n, "x"), (iterates, (q + 2) * n, "iterates"))
        st = lib().igamg_extrapolate(self._h, method, q, px, pit, _np_ptr(gamma))
        _check(st, "igamg_extrapolate")
        return gamma

    def solve_fgmres(self, x, tol=1e-10, max_iters=200, m=20, precond=PRECOND_RRE, q=3, check=True):
        """Flexible GMRES(m) preconditioned by the multigrid cycle; x is the
        initial guess and the result.  Returns (stats, status)."""
        st = Stats()
        status = lib().igamg_solve_fgmres(self._h, tol, max_iters, m, precond, q, _ptr(x, self.ndof, "x"),
                                          ctypes.byref(st))
        if check:
            _check(status, "igamg_solve_fgmres")
        return st, status

    def generalized_residual(self):
        """||t~ - t|| of the last extrapolation (from its R factor)."""
        g = _d()
        _check(lib().igamg_generalized_residual(self._h, ctypes.byref(g)), "igamg_generalized_residual")
        return g.value

    def solve(self, x, tol=1e-10, max_restarts=100, method=RRE, q=5, check=True):
        st = Stats()
        status = lib().igamg_solve(self._h, tol, max_restarts, method, q, _ptr(x, self.ndof, "x"),
                                   ctypes.byref(st))
        if check:
            _check(status, "igamg_solve")
        return st, status

    def get_state(self, x=None):
        """Checkpoint of the last solve: its accepted iterate goes to x (if
        given) and its counts and adaptive settings are returned."""
        state = State()
        _check(lib().igamg_get_state(self._h, _ptr(x, self.ndof, "x"), ctypes.byref(state)),
               "igamg_get_state")
        return state

    def set_state(self, state):
        """Loads a checkpoint for the next solve (which starts from its x)."""
        _check(lib().igamg_set_state(self._h, ctypes.byref(state)), "igamg_set_state")

    def residual(self, x):
        r = _d()
        _check(lib().igamg_residual(self._h, _ptr(x, self.ndof, "x"), ctypes.byref(r)), "igamg_residual")
        return r.value

    def operator_rows(self, level, rows):
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        W = 2 * self.degree + 1
        S = W ** (3 if self.geometry == UNIT_CUBE else 2)
        out = np.zeros((len(rows), S))
        _check(lib().igamg_get_operator_rows(self._h, level, _np_ptr(rows), len(rows),
                                             _np_ptr(out)), "igamg_get_operator_rows")
        return out

    def apply(self, level, x, y):
        n = self.level_ndof(level)
        _check(lib().igamg_apply(self._h, level, *_ptrs((x, n, "x"), (y, n, "y"))), "igamg_apply")
        return y

    def smooth(self, level, b, x, nsweeps=1):
        n = self.level_ndof(level)
        _check(lib().igamg_smooth(self._h, level, *_ptrs((b, n, "b"), (x, n, "x")), nsweeps), "igamg_smooth")
        return x

    def restrict(self, level, r, rc):
        _check(lib().igamg_restrict(self._h, level, *_ptrs((r, self.level_ndof(level), "r"),
                                                           (rc, self.level_ndof(level - 1), "rc"))),
               "igamg_restrict")
        return rc

    def prolong_add(self, level, e, x):
        _check(lib().igamg_prolong_add(self._h, level, *_ptrs((e, self.level_ndof(level - 1), "e"),
                                                              (x, self.level_ndof(level), "x"))),
               "igamg_prolong_add")
        return x

    def coarse_solve(self, b, x):
        n = self.level_ndof(0)
        _check(lib().igamg_coarse_solve(self._h, *_ptrs((b, n, "b"), (x, n, "x"))), "igamg_coarse_solve")
        return x

    def profile_smoother(self, level, precision, nsweeps=4):
        """(mean ms per colour launch, algorithmic bytes per launch, launches)."""
        ms, by, n = _d(), _d(), _i()
        _check(lib().igamg_profile_smoother(self._h, level, precision, nsweeps, ctypes.byref(ms),
                                            ctypes.byref(by), ctypes.byref(n)),
               "igamg_profile_smoother")
        return ms.value, by.value, n.value

    def autotune(self):
        """(chosen tail_items, V-cycle ms); the per-level choices via tuning()."""
        t, ms = _i(), _d()
        _check(lib().igamg_autotune(self._h, ctypes.byref(t), ctypes.byref(ms)), "igamg_autotune")
        return t.value, ms.value

    def tuning(self):
        """The launch shapes in use (dict: split, per-level sweep and learned kernels)."""
        t = Tuning()
        _check(lib().igamg_get_tuning(self._h, ctypes.byref(t)), "igamg_get_tuning")
        return t.as_dict()

    def set_tuning(self, d):
        """Sets the launch shapes from a dict as tuning() returns."""
        n = int(d["num_levels"])
        if len(d["row_class"]) != n or len(d["learned_kernel"]) != n or n > 16:
            raise ValueError("per-level lists must have num_levels <= 16 entries")
        t = Tuning()
        t.tail_items, t.num_levels = int(d["tail_items"]), n
        for l in range(n):
            t.row_class[l] = int(d["row_class"][l])
            t.learned_kernel[l] = int(d["learned_kernel"][l])
        _check(lib().igamg_set_tuning(self._h, ctypes.byref(t)), "igamg_set_tuning")

    # ---- learned smoother
    def train_smoother(self, modes_list, val_modes=None, **kw):
        o = TrainOptions()
        lib().igamg_train_options_default(ctypes.byref(o))
        tab = np.ascontiguousarray(np.concatenate([np.asarray(m, dtype=np.float64) for m in modes_list]))
        o.n_rhs = len(modes_list)
        o.n_modes = int(np.asarray(modes_list[0]).shape[0])
        o.modes = _np_ptr(tab)
        vm = None
        if val_modes is not None:
            vm = np.ascontiguousarray(val_modes, dtype=np.float64)
            o.val_modes = _np_ptr(vm)
            o.val_n_modes = vm.shape[0]
        for k, v in kw.items():
            setattr(o, k, v)
        rep = TrainReport()
        _check(lib().igamg_train_smoother(self._h, ctypes.byref(o), ctypes.byref(rep)),
               "igamg_train_smoother")
        del tab, vm
        return rep.as_dict()

    def set_learned(self, enabled):
        _check(lib().igamg_set_learned(self._h, int(enabled)), "igamg_set_learned")

    def get_smoother_weights(self, level):
        w = np.zeros(2592, dtype=np.uint16)
        _check(lib().igamg_get_smoother_weights(self._h, level, _np_ptr(w), w.size),
               "igamg_get_smoother_weights")
        return w

    def set_smoother_weights(self, level, w):
        w = np.ascontiguousarray(w, dtype=np.uint16)
        _check(lib().igamg_set_smoother_weights(self._h, level, _np_ptr(w), w.size),
               "igamg_set_smoother_weights")

    def smoother_forward(self, level, z, y):
        n = self.level_ndof(level)
        _check(lib().igamg_smoother_forward(self._h, level, *_ptrs32((z, n, "z"), (y, n, "y"))),
               "igamg_smoother_forward")
        return y

    def smoother_loss_grad(self, level, z, t):
        g = np.zeros(2592, dtype=np.float32)
        loss = _d()
        n = self.level_ndof(level)
        _check(lib().igamg_smoother_loss_grad(self._h, level, *_ptrs32((z, n, "z"), (t, n, "t")),
                                              ctypes.byref(loss), _np_ptr(g)),
               "igamg_smoother_loss_grad")
        return loss.value, g

    def extrap_coeffs(self, method, q, iterates, noalloc=False):
        """gamma_0..gamma_q and the breakdown code for q+2 stored iterates;
        noalloc=True takes igamg_extrap_coeffs_noalloc (fixed device scratch)."""
        gamma = np.zeros(q + 1)
        info = _i()
        name = "igamg_extrap_coeffs_noalloc" if noalloc else "igamg_extrap_coeffs"
        _check(getattr(lib(), name)(self._h, method, q, _ptr(iterates, (q + 2) * self.ndof, "iterates"),
                                    _np_ptr(gamma), ctypes.byref(info)), name)
        return gamma, info.value


class _Borrowed(Solver):
    """A problem owned by a batch, addressed with the single-problem calls."""

    def __init__(self, handle, geometry, n_el, degree):
        self._h = handle
        self._owned = False
        self.geometry, self.n_el, self.degree = geometry, n_el, degree

    def close(self):
        self._h = None


class Batch:
    """A batch of independent 2D problems (include/igamg.h, igamg_setup_batch)."""

    def __init__(self, problems, stream=None, tail_items=32, row_sweeps=1):
        """problems: list of (geometry, n_el, degree); tail_items < 0 autotunes;
        row_sweeps 0 sweeps one colour per launch instead of one row class."""
        import torch
        if stream is None:
            cs = torch.cuda.current_stream()
            stream = None if cs.cuda_stream == 0 else cs.cuda_stream
        n = len(problems)
        geoms = (Geometry * n)(*[Geometry(g, e, 0.0, 0.0) for g, e, _ in problems])
        degs = (ctypes.c_int * n)(*[d for _, _, d in problems])
        o = default_options()
        o.stream = stream
        o.tail_items = tail_items
        o.row_sweeps = row_sweeps
        h = _P()
        _check(lib().igamg_setup_batch(n, ctypes.cast(geoms, _P), ctypes.cast(degs, _P),
                                       ctypes.byref(o), ctypes.byref(h)), "igamg_setup_batch")
        self._h = h
        self.problems = list(problems)
        self.instances = []
        for i, (g, e, d) in enumerate(problems):
            ih = _P()
            _check(lib().igamg_batch_instance(h, i, ctypes.byref(ih)), "igamg_batch_instance")
            self.instances.append(_Borrowed(ih, g, e, d))

    def close(self):
        if getattr(self, "_h", None):
            for s in self.instances:
                s.close()
            lib().igamg_destroy_batch(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, xs, tol=1e-10, max_restarts=100, q=5, check=True):
        n = len(xs)
        ptrs = _ptr_list(xs, [inst.ndof for inst in self.instances], "initial guesses")
        stats = (Stats * n)()
        st = lib().igamg_solve_batch(self._h, tol, max_restarts, q, ctypes.cast(ptrs, _P),
                                     ctypes.cast(stats, _P))
        if check:
            _check(st, "igamg_solve_batch")
        return [stats[i] for i in range(n)], st


class Set1D:
    """A set of independent 1D model problems (include/igamg.h, igamg_setup_1d),
    each solved by one workgroup of one launch."""

    def __init__(self, problems, stream=None):
        """problems: list of dicts with any igamg_problem1d fields (others keep
        igamg_problem1d_default's values)."""
        import torch
        if stream is None:
            cs = torch.cuda.current_stream()
            stream = None if cs.cuda_stream == 0 else cs.cuda_stream
        n = len(problems)
        arr = (Problem1D * n)()
        for k, pr in enumerate(problems):
            lib().igamg_problem1d_default(ctypes.byref(arr[k]))
            for key, val in pr.items():
                if not hasattr(arr[k], key):
                    raise KeyError(key)
                setattr(arr[k], key, val)
        h = _P()
        _check(lib().igamg_setup_1d(n, arr, stream, ctypes.byref(h)), "igamg_setup_1d")
        self._h = h
        self.problems = [dict((f, getattr(arr[k], f)) for f, _ in Problem1D._fields_) for k in range(n)]

    def close(self):
        if getattr(self, "_h", None):
            lib().igamg_destroy_1d(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def ndof(self, i):
        return int(lib().igamg_ndof_1d(self._h, i))

    def set_rhs(self, i, b):
        _check(lib().igamg_set_rhs_1d(self._h, i, _ptr(b, self.ndof(i), "b")), "igamg_set_rhs_1d")

    def get_rhs(self, i, out):
        _check(lib().igamg_get_rhs_1d(self._h, i, _ptr(out, self.ndof(i), "out")), "igamg_get_rhs_1d")
        return out

    def cycles(self, xs, ncycles=1):
        ptrs = _ptr_list(xs, [self.ndof(i) for i in range(len(self.problems))], "initial guesses")
        _check(lib().igamg_cycles_1d(self._h, ncycles, ctypes.cast(ptrs, _P)), "igamg_cycles_1d")
        return xs

    def solve(self, xs, tol=1e-12, max_iters=1000, check=True):
        n = len(xs)
        ptrs = _ptr_list(xs, [self.ndof(i) for i in range(len(self.problems))], "initial guesses")
        stats = (Stats1D * n)()
        st = lib().igamg_solve_1d(self._h, tol, max_iters, ctypes.cast(ptrs, _P), stats)
        if check:
            _check(st, "igamg_solve_1d")
        return [stats[i] for i in range(n)], st


# ---- host-only helpers (no GPU needed)

def host_gauss_legendre(m):
    x, w = np.zeros(m), np.zeros(m)
    if lib().igamg_host_gauss_legendre(m, _np_ptr(x), _np_ptr(w)) != 0:
        raise ValueError("bad m")
    return x, w


def host_basis(ne, p, u):
    N, D = np.zeros(p + 1), np.zeros(p + 1)
    first = _i()
    if lib().igamg_host_basis(ne, p, float(u), _np_ptr(N), _np_ptr(D), ctypes.byref(first)) != 0:
        raise ValueError("bad arguments")
    return first.value, N, D


def host_prolongation_1d(ne_coarse, p):
    out = np.zeros((2 * ne_coarse + p, ne_coarse + p))
    if lib().igamg_host_prolongation_1d(ne_coarse, p, _np_ptr(out)) != 0:
        raise ValueError("bad arguments")
    return out


def host_bands(ne, ne_coarsest, level, p):
    n = (ne_coarsest << level) + p - 2
    K, M = np.zeros((n, 2 * p + 1)), np.zeros((n, 2 * p + 1))
    if lib().igamg_host_bands(ne, ne_coarsest, level, p, _np_ptr(K), _np_ptr(M)) != 0:
        raise ValueError("bad arguments")
    return K, M


def host_coarse_inverse(A, symmetric=True):
    """(status, inverse) of a dense coarsest operator, as the setup forms it."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    if A.shape != (n, n):
        raise ValueError("square matrix expected")
    inv = np.zeros((n, n))
    st = lib().igamg_host_coarse_inverse(n, _np_ptr(A), int(symmetric), _np_ptr(inv))
    return st, inv
