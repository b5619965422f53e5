"""ctypes binding of libabsorber.so: one Python method per C entry point.

Device arrays are passed as raw pointers (``tensor.data_ptr()`` of contiguous
float64 CUDA tensors); every computation happens in the HIP library.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libabsorber.so")

ABS_OK = 0
ERRORS = {
    -1: "ABS_ERR_ARG", -2: "ABS_ERR_HIP", -3: "ABS_ERR_OOM", -4: "ABS_ERR_STATE",
    -10: "ABS_ERR_INERTIA", -11: "ABS_ERR_LS", -12: "ABS_ERR_MAXITER", -13: "ABS_ERR_NAN",
    -14: "ABS_ERR_DIVERGE",
}

c_double_p = ctypes.POINTER(ctypes.c_double)
c_int64_p = ctypes.POINTER(ctypes.c_int64)
c_float_p = ctypes.POINTER(ctypes.c_float)


class AbsorberError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class AbsorberParams(ctypes.Structure):
    _fields_ = [
        ("nu", ctypes.c_double * 5 * 11),
        ("lnK_A", ctypes.c_double * 5), ("lnK_B", ctypes.c_double * 5),
        ("lnK_C", ctypes.c_double * 5), ("lnK_D", ctypes.c_double * 5),
        ("psat_a", ctypes.c_double), ("psat_b", ctypes.c_double),
        ("henry_lnH298", ctypes.c_double), ("henry_kappa", ctypes.c_double),
        ("henry_Tref", ctypes.c_double), ("henry_ln_ratio_MEA", ctypes.c_double),
        ("Tref", ctypes.c_double),
        ("hL_ref", ctypes.c_double * 9), ("cpL_a", ctypes.c_double * 9), ("cpL_b", ctypes.c_double * 9),
        ("hV_ref", ctypes.c_double * 4), ("cpV_a", ctypes.c_double * 4), ("cpV_b", ctypes.c_double * 4),
        ("R", ctypes.c_double), ("u_max", ctypes.c_double),
        ("x_lo", ctypes.c_double), ("x_hi", ctypes.c_double), ("y_lo", ctypes.c_double), ("y_hi", ctypes.c_double),
        ("L_lo", ctypes.c_double), ("L_hi", ctypes.c_double), ("V_lo", ctypes.c_double), ("V_hi", ctypes.c_double),
        ("T_lo", ctypes.c_double), ("T_hi", ctypes.c_double), ("d_lo", ctypes.c_double), ("d_hi", ctypes.c_double),
        ("x0", ctypes.c_double * 21), ("d0", ctypes.c_double), ("dp_stage", ctypes.c_double),
        ("op_weight", ctypes.c_double), ("op_loss_coef", ctypes.c_double), ("op_molar_mass", ctypes.c_double * 4),
    ]


class Dims(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("n_var_total", "n_var_free", "n_eq", "n_fixed", "n_ineq",
                                               "nnz_jac", "nnz_hess", "kkt_dim")]


class IpmOptions(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("warm_start", ctypes.c_int32),
        ("mu_init", ctypes.c_double), ("warm_mu_init", ctypes.c_double), ("bound_push", ctypes.c_double),
        ("warm_bound_push", ctypes.c_double), ("nlp_scaling_max_gradient", ctypes.c_double),
        ("print_level", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("feasibility_restart", ctypes.c_int32),
        ("autotune", ctypes.c_int32), ("delta_w_max", ctypes.c_double),
    ]


class IpmResult(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32), ("iterations", ctypes.c_int32), ("E0", ctypes.c_double),
        ("inf_pr", ctypes.c_double), ("inf_du", ctypes.c_double), ("compl_", ctypes.c_double),
        ("d", ctypes.c_double), ("seconds", ctypes.c_double), ("n_inertia_corrections", ctypes.c_int32),
        ("n_factorizations", ctypes.c_int32), ("max_lin_resid", ctypes.c_double),
        ("feasibility_restarts", ctypes.c_int32), ("graph_replays", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class IpmLogEntry(ctypes.Structure):
    _fields_ = [
        ("iteration", ctypes.c_int32), ("n_factorizations", ctypes.c_int32), ("n_trials", ctypes.c_int32),
        ("pad", ctypes.c_int32), ("mu", ctypes.c_double), ("theta", ctypes.c_double), ("alpha", ctypes.c_double),
        ("alpha_z", ctypes.c_double), ("delta_w", ctypes.c_double), ("delta_c", ctypes.c_double),
        ("d", ctypes.c_double), ("E0", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


class Profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 4), ("calls", ctypes.c_int64 * 4), ("bytes_factor_slots", ctypes.c_int64)]


class MlpConfig(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("n_in", "n_hidden", "n_layers", "n_out", "max_batch")]


class MlpTrainOptions(ctypes.Structure):
    _fields_ = [
        ("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_double),
        ("beta1", ctypes.c_double), ("beta2", ctypes.c_double), ("eps", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("cosine", ctypes.c_int32),
    ]


class MlpTrainResult(ctypes.Structure):
    _fields_ = [("final_loss", ctypes.c_double), ("seconds", ctypes.c_double), ("steps", ctypes.c_int64)]


class Tuning(ctypes.Structure):
    _fields_ = [("tuned", ctypes.c_int32), ("factor_waves_per_simd", ctypes.c_int32),
                ("factor_row_split", ctypes.c_int32),
                ("solve_waves_per_simd", ctypes.c_int32), ("eval_block", ctypes.c_int32),
                ("factor_ms", ctypes.c_float * 3 * 2), ("solve_ms", ctypes.c_float * 3),
                ("eval_ms", ctypes.c_float * 3)]


PROFILE_CLASSES = ("factor", "solve", "eval", "residual")

_lib = None


def lib():
    """Load libabsorber.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2607_15420_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sig = {
            "absorber_create": (ctypes.c_int, [ctypes.POINTER(AbsorberParams), i32, i32, c_double_p,
                                               ctypes.POINTER(vp)]),
            "absorber_destroy": (None, [vp]),
            "absorber_create_batch": (ctypes.c_int, [ctypes.POINTER(AbsorberParams), i32, ctypes.POINTER(i32),
                                                     ctypes.POINTER(i32), c_double_p, ctypes.POINTER(vp)]),
            "absorber_create_sections": (ctypes.c_int, [ctypes.POINTER(AbsorberParams), i32, i32, i32, c_double_p,
                                                        ctypes.POINTER(vp)]),
            "absorber_batch_solve": (ctypes.c_int, [vp, ctypes.POINTER(IpmOptions), vp, vp, vp, vp,
                                                    ctypes.POINTER(IpmResult)]),
            "absorber_get_dims": (ctypes.c_int, [vp, ctypes.POINTER(Dims)]),
            "absorber_initial_point": (ctypes.c_int, [vp, vp, vp]),
            "absorber_set_scaling": (ctypes.c_int, [vp, c_double_p, vp]),
            "absorber_eval_cons": (ctypes.c_int, [vp, vp, vp, vp]),
            "absorber_eval_obj": (ctypes.c_int, [vp, vp, c_double_p, vp, vp]),
            "absorber_jac_structure": (ctypes.c_int, [vp, c_int64_p, c_int64_p]),
            "absorber_eval_jac": (ctypes.c_int, [vp, vp, vp, vp]),
            "absorber_hess_structure": (ctypes.c_int, [vp, c_int64_p, c_int64_p]),
            "absorber_eval_hess": (ctypes.c_int, [vp, vp, vp, dbl, vp, vp]),
            "absorber_kkt_factor": (ctypes.c_int, [vp, vp, vp, vp, vp, dbl, dbl, c_int64_p, vp]),
            "absorber_kkt_solve": (ctypes.c_int, [vp, vp, vp, c_double_p, vp]),
            "absorber_ipm_default_options": (None, [ctypes.POINTER(IpmOptions)]),
            "absorber_ipm_solve": (ctypes.c_int, [vp, ctypes.POINTER(IpmOptions), vp, vp, vp, vp,
                                                  ctypes.POINTER(IpmResult)]),
            "absorber_ipm_log_get": (ctypes.c_int, [vp, i32, i32, ctypes.POINTER(IpmLogEntry),
                                                    ctypes.POINTER(i32)]),
            "absorber_profile_enable": (ctypes.c_int, [vp, i32]),
            "absorber_profile_get": (ctypes.c_int, [vp, ctypes.POINTER(Profile)]),
            "absorber_tuning_get": (ctypes.c_int, [vp, ctypes.POINTER(Tuning)]),
            "absorber_tuning_set": (ctypes.c_int, [vp, ctypes.POINTER(Tuning)]),
            "absorber_last_error": (ctypes.c_char_p, []),
            "absorber_mlp_default_config": (None, [ctypes.POINTER(MlpConfig)]),
            "absorber_mlp_default_train_options": (None, [ctypes.POINTER(MlpTrainOptions)]),
            "absorber_mlp_create": (ctypes.c_int, [ctypes.POINTER(MlpConfig), ctypes.c_uint64, ctypes.POINTER(vp)]),
            "absorber_mlp_destroy": (None, [vp]),
            "absorber_mlp_get_config": (ctypes.c_int, [vp, ctypes.POINTER(MlpConfig)]),
            "absorber_mlp_num_params": (i64, [vp]),
            "absorber_mlp_set_params": (ctypes.c_int, [vp, c_float_p]),
            "absorber_mlp_get_params": (ctypes.c_int, [vp, c_float_p]),
            "absorber_mlp_set_normalization": (ctypes.c_int, [vp, c_float_p, c_float_p, c_float_p, c_float_p]),
            "absorber_mlp_get_normalization": (ctypes.c_int, [vp, c_float_p, c_float_p, c_float_p, c_float_p]),
            "absorber_mlp_fit_normalization": (ctypes.c_int, [vp, vp, vp, i64, vp]),
            "absorber_mlp_forward": (ctypes.c_int, [vp, vp, i64, vp, vp]),
            "absorber_mlp_loss_grad": (ctypes.c_int, [vp, vp, vp, i64, vp, c_double_p, vp]),
            "absorber_mlp_adam_step": (ctypes.c_int, [vp, vp, ctypes.POINTER(MlpTrainOptions), dbl, vp]),
            "absorber_mlp_train": (ctypes.c_int, [vp, vp, vp, i64, ctypes.POINTER(MlpTrainOptions),
                                                  ctypes.POINTER(MlpTrainResult)]),
            "absorber_simulate": (ctypes.c_int, [vp, vp, dbl, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
            "absorber_warm_features": (ctypes.c_int, [vp, vp, vp]),
            "absorber_warm_targets": (ctypes.c_int, [vp, vp, vp, vp, vp]),
            "absorber_warm_point": (ctypes.c_int, [vp, vp, i32, dbl, vp, vp, vp]),
            "absorber_warm_start": (ctypes.c_int, [vp, vp, vp, vp, dbl, vp, vp, vp]),
            "absorber_warm_start_noalloc": (ctypes.c_int, [vp, vp, dbl, vp, vp, vp]),
            "absorber_warm_solve": (ctypes.c_int, [vp, vp, ctypes.POINTER(IpmOptions), dbl, vp, vp,
                                                   ctypes.POINTER(IpmResult), ctypes.POINTER(ctypes.c_int32)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != ABS_OK:
        raise AbsorberError(rc, lib().absorber_last_error().decode())
    return rc


def _check_call(rc):
    """Raise on a failed call (bad argument, HIP error, allocation, call
    order); solver outcomes (-10 and below) are returned in the results."""
    if -10 < rc < ABS_OK:
        _check(rc)
    return rc


def params_struct(p: dict) -> AbsorberParams:
    """Fill the C parameter struct from the problem-data dict (params.json)."""
    s = AbsorberParams()
    for i in range(11):
        for r in range(5):
            s.nu[i][r] = p["nu"][i][r]
    for f in ("lnK_A", "lnK_B", "lnK_C", "lnK_D"):
        for r in range(5):
            getattr(s, f)[r] = p[f][r]
    for f in ("psat_a", "psat_b", "henry_lnH298", "henry_kappa", "henry_Tref", "henry_ln_ratio_MEA", "Tref",
              "R", "u_max"):
        setattr(s, f, float(p[f]))
    for f in ("hL_ref", "cpL_a", "cpL_b"):
        for i in range(9):
            getattr(s, f)[i] = p[f][i]
    for f in ("hV_ref", "cpV_a", "cpV_b"):
        for j in range(4):
            getattr(s, f)[j] = p[f][j]
    b = p["bounds"]
    s.x_lo, s.x_hi = b["x"]
    s.y_lo, s.y_hi = b["y"]
    s.L_lo, s.L_hi = b["L"]
    s.V_lo, s.V_hi = b["V"]
    s.T_lo, s.T_hi = b["T"]
    s.d_lo, s.d_hi = b["d"]
    ip = p["initial_point"]
    z = list(ip["x"]) + list(ip["y"]) + [ip["L"], ip["V"], ip["T"]] + [ip["eps"]] * 5
    for k in range(21):
        s.x0[k] = float(z[k])
    s.d0 = float(ip["d"])
    s.dp_stage = float(p.get("dp_stage", 0.0))
    op = p.get("operating_cost", {})
    s.op_weight = float(op.get("weight", 0.0))
    s.op_loss_coef = float(op.get("loss_coef", 0.0))
    for j, m in enumerate(op.get("molar_mass", [0.0] * 4)):
        s.op_molar_mass[j] = float(m)
    return s


def _ptr(t):
    """Device pointer of a contiguous float64/int tensor (or None)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        return None
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


class Absorber:
    """Handle of one problem instance (S scenarios, N stages) on the current GPU,
    or of a batch of independent problems (Absorber.batch)."""

    def __init__(self, params: dict, n_stages: int, feeds: np.ndarray):
        feeds = np.ascontiguousarray(feeds, dtype=np.float64)
        if feeds.ndim != 2 or feeds.shape[1] != 18:
            raise ValueError("feeds must be (S, 18)")
        self._p = params_struct(params)
        h = ctypes.c_void_p()
        _check(lib().absorber_create(ctypes.byref(self._p), int(n_stages), int(feeds.shape[0]),
                                     feeds.ctypes.data_as(c_double_p), ctypes.byref(h)))
        self.h = h
        self.P = 1
        self.npar = 1
        self.N, self.S = int(n_stages), int(feeds.shape[0])
        self._sizes()

    @classmethod
    def sections(cls, params: dict, n_stages: int, feeds: np.ndarray, n_sections: int) -> "Absorber":
        """One problem whose column has n_sections diameters theta_k (the design
        vector of eq. 8): stage n belongs to section n * n_sections // n_stages;
        x ends with the n_sections diameters."""
        feeds = np.ascontiguousarray(feeds, dtype=np.float64)
        if feeds.ndim != 2 or feeds.shape[1] != 18:
            raise ValueError("feeds must be (S, 18)")
        self = cls.__new__(cls)
        self._p = params_struct(params)
        h = ctypes.c_void_p()
        _check(lib().absorber_create_sections(ctypes.byref(self._p), int(n_stages), int(feeds.shape[0]),
                                              int(n_sections), feeds.ctypes.data_as(c_double_p), ctypes.byref(h)))
        self.h = h
        self.P = 1
        self.npar = int(n_sections)
        self.N, self.S = int(n_stages), int(feeds.shape[0])
        self._sizes()
        return self

    def _sizes(self):
        d = self.dims()
        self.nx = d["n_var_free"]
        self.nc = d["n_eq"] + d["n_ineq"]
        self.nkkt = d["kkt_dim"]
        self.nst = d["n_ineq"]

    @classmethod
    def batch(cls, params: dict, problems) -> "Absorber":
        """Batch of independent problems; problems = [(n_stages, feeds (S_p, 18)), ...]."""
        self = cls.__new__(cls)
        Ns = np.array([int(n) for n, _ in problems], dtype=np.int32)
        Ss = np.array([np.asarray(f).shape[0] for _, f in problems], dtype=np.int32)
        feeds = np.ascontiguousarray(np.concatenate([np.asarray(f, dtype=np.float64) for _, f in problems]))
        if feeds.ndim != 2 or feeds.shape[1] != 18:
            raise ValueError("feeds must be (S_p, 18) per problem")
        self._p = params_struct(params)
        h = ctypes.c_void_p()
        i32p = ctypes.POINTER(ctypes.c_int32)
        _check(lib().absorber_create_batch(ctypes.byref(self._p), len(problems), Ns.ctypes.data_as(i32p),
                                           Ss.ctypes.data_as(i32p), feeds.ctypes.data_as(c_double_p),
                                           ctypes.byref(h)))
        self.h = h
        self.P = len(problems)
        self.npar = 1
        self.N, self.S = int(Ns.max()), int(Ss.sum())
        self.pN, self.pS = Ns, Ss
        self._sizes()
        return self

    def batch_solve(self, opts: IpmOptions | None = None, x0=None, lam0=None, x_out=None, lam_out=None):
        """Interior-point solve of every problem of the handle; returns (rc, [IpmResult] * P)."""
        o = opts if opts is not None else self.default_options()
        res = (IpmResult * self.P)()
        rc = lib().absorber_batch_solve(self.h, ctypes.byref(o), _ptr(x0), _ptr(lam0), _ptr(x_out), _ptr(lam_out),
                                        res)
        _check_call(rc)
        return rc, list(res)

    def close(self):
        if getattr(self, "h", None):
            lib().absorber_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def dims(self) -> dict:
        d = Dims()
        _check(lib().absorber_get_dims(self.h, ctypes.byref(d)))
        return {k: getattr(d, k) for k, _ in d._fields_}

    def initial_point(self, x, stream=None):
        _check(lib().absorber_initial_point(self.h, _ptr(x), _stream(stream)))

    def set_scaling(self, var_scale=None, row_scale=None):
        vs = None
        if var_scale is not None:
            arr = np.ascontiguousarray(var_scale, dtype=np.float64)
            if arr.size != 22:
                raise ValueError("var_scale must have 22 entries")
            self._vs = arr
            vs = arr.ctypes.data_as(c_double_p)
        _check(lib().absorber_set_scaling(self.h, vs, _ptr(row_scale)))

    def eval_cons(self, x, c, stream=None):
        _check(lib().absorber_eval_cons(self.h, _ptr(x), _ptr(c), _stream(stream)))

    def eval_obj(self, x, grad=None, stream=None):
        f = ctypes.c_double()
        _check(lib().absorber_eval_obj(self.h, _ptr(x), ctypes.byref(f), _ptr(grad), _stream(stream)))
        return f.value

    def jac_structure(self):
        n = self.dims()["nnz_jac"]
        rows, cols = np.empty(n, np.int64), np.empty(n, np.int64)
        _check(lib().absorber_jac_structure(self.h, rows.ctypes.data_as(c_int64_p), cols.ctypes.data_as(c_int64_p)))
        return rows, cols

    def eval_jac(self, x, vals, stream=None):
        _check(lib().absorber_eval_jac(self.h, _ptr(x), _ptr(vals), _stream(stream)))

    def hess_structure(self):
        n = self.dims()["nnz_hess"]
        rows, cols = np.empty(n, np.int64), np.empty(n, np.int64)
        _check(lib().absorber_hess_structure(self.h, rows.ctypes.data_as(c_int64_p),
                                             cols.ctypes.data_as(c_int64_p)))
        return rows, cols

    def eval_hess(self, x, lam, vals, obj_factor=1.0, stream=None):
        _check(lib().absorber_eval_hess(self.h, _ptr(x), _ptr(lam), float(obj_factor), _ptr(vals),
                                        _stream(stream)))

    def profile_enable(self, on=True, mask=0xF):
        """Time the kernel classes in mask (bit 0 factor, 1 solve, 2 eval, 3 residual)."""
        _check(lib().absorber_profile_enable(self.h, int(mask) if on else 0))

    def ipm_log(self, problem: int = 0) -> list:
        """Accepted iterations of problem `problem` in the last solve (list of dicts)."""
        n = ctypes.c_int32()
        _check(lib().absorber_ipm_log_get(self.h, int(problem), 0, None, ctypes.byref(n)))
        buf = (IpmLogEntry * max(n.value, 1))()
        _check(lib().absorber_ipm_log_get(self.h, int(problem), n.value, buf, ctypes.byref(n)))
        return [buf[i].as_dict() for i in range(n.value)]

    def tuning(self) -> dict:
        t = Tuning()
        _check(lib().absorber_tuning_get(self.h, ctypes.byref(t)))
        return {"tuned": bool(t.tuned), "factor_waves_per_simd": t.factor_waves_per_simd,
                "factor_row_split": t.factor_row_split,
                "solve_waves_per_simd": t.solve_waves_per_simd, "eval_block": t.eval_block,
                "factor_ms": [list(r) for r in t.factor_ms], "solve_ms": list(t.solve_ms),
                "eval_ms": list(t.eval_ms)}

    def set_tuning(self, factor_waves_per_simd=3, factor_row_split=0, solve_waves_per_simd=3, eval_block=128):
        """Pin the launch shapes (the autotuner then does not run)."""
        t = Tuning()
        t.factor_waves_per_simd, t.factor_row_split = factor_waves_per_simd, factor_row_split
        t.solve_waves_per_simd, t.eval_block = solve_waves_per_simd, eval_block
        _check(lib().absorber_tuning_set(self.h, ctypes.byref(t)))

    def profile(self) -> dict:
        p = Profile()
        _check(lib().absorber_profile_get(self.h, ctypes.byref(p)))
        out = {c: {"ms": p.ms[i], "calls": p.calls[i]} for i, c in enumerate(PROFILE_CLASSES)}
        out["bytes_factor_slots"] = p.bytes_factor_slots
        return out

    def kkt_factor(self, x, lam, sigma_x, sigma_s, delta_w=0.0, delta_c=0.0, stream=None):
        inert = np.zeros(3, np.int64)
        _check(lib().absorber_kkt_factor(self.h, _ptr(x), _ptr(lam), _ptr(sigma_x), _ptr(sigma_s),
                                         float(delta_w), float(delta_c), inert.ctypes.data_as(c_int64_p),
                                         _stream(stream)))
        return tuple(int(v) for v in inert)

    def kkt_solve(self, rhs, sol, stream=None):
        rel = ctypes.c_double()
        _check(lib().absorber_kkt_solve(self.h, _ptr(rhs), _ptr(sol), ctypes.byref(rel), _stream(stream)))
        return rel.value

    def simulate(self, x, tol=1e-12, max_iter=100):
        """Process simulation of every scenario from x (in/out); returns (converged per problem, iterations)."""
        conv = np.zeros(self.P, np.int32)
        it = ctypes.c_int32()
        _check(lib().absorber_simulate(self.h, _ptr(x), float(tol), int(max_iter),
                                       conv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(it)))
        return conv.astype(bool), it.value

    def warm_features(self, X, stream=None):
        """X: float32 (S, 3) device tensor <- (gas flow, CO2 fraction, gas temperature) per scenario."""
        _check(lib().absorber_warm_features(self.h, _ptr(X), _stream(stream)))

    def warm_targets(self, x, T, lam=None, stream=None):
        """T: float32 (S, 21 N) or, with lam, (S, 43 N) <- network encoding of x (float64, nx) [and lam (nc)]."""
        _check(lib().absorber_warm_targets(self.h, _ptr(x), _ptr(lam), _ptr(T), _stream(stream)))

    def warm_point(self, Y, x0, lam0=None, d_margin=1e-3, stream=None):
        """x0 (float64, nx) [and lam0 (nc)] <- decoded network rows Y (float32, (S, n_out))."""
        _check(lib().absorber_warm_point(self.h, _ptr(Y), int(Y.shape[1]), float(d_margin), _ptr(x0), _ptr(lam0),
                                         _stream(stream)))

    def warm_start(self, net: "Mlp", X_work, Y_work, x0, lam0=None, d_margin=1e-3, stream=None):
        _check(lib().absorber_warm_start(self.h, net.h, _ptr(X_work), _ptr(Y_work), float(d_margin), _ptr(x0),
                                         _ptr(lam0), _stream(stream)))

    def warm_start_noalloc(self, net: "Mlp", x0, lam0=None, d_margin=1e-3, stream=None):
        """absorber_warm_start with the library's static workspace (no device allocation)."""
        _check(lib().absorber_warm_start_noalloc(self.h, net.h, float(d_margin), _ptr(x0), _ptr(lam0),
                                                 _stream(stream)))

    def warm_solve(self, net: "Mlp", opts: IpmOptions | None = None, d_margin=1e-3, x_out=None, lam_out=None):
        """Warm-started solve with cold fallback; returns (result, used_warm)."""
        o = opts if opts is not None else self.default_options()
        r = IpmResult()
        used = ctypes.c_int32()
        _check(lib().absorber_warm_solve(self.h, net.h, ctypes.byref(o), float(d_margin), _ptr(x_out), _ptr(lam_out),
                                         ctypes.byref(r), ctypes.byref(used)))
        return r, bool(used.value)

    @staticmethod
    def default_options(**kw) -> IpmOptions:
        o = IpmOptions()
        lib().absorber_ipm_default_options(ctypes.byref(o))
        for k, v in kw.items():
            setattr(o, k, v)
        return o

    def ipm_solve(self, opts: IpmOptions | None = None, x0=None, lam0=None, x_out=None, lam_out=None,
                  check=False) -> IpmResult:
        """Run the interior-point method; returns the result struct (status in .status)."""
        o = opts if opts is not None else self.default_options()
        r = IpmResult()
        rc = lib().absorber_ipm_solve(self.h, ctypes.byref(o), _ptr(x0), _ptr(lam0), _ptr(x_out), _ptr(lam_out),
                                      ctypes.byref(r))
        if check:
            _check(rc)
        _check_call(rc)
        return r


def absorber_create(params: dict, n_stages: int, feeds: np.ndarray) -> Absorber:
    return Absorber(params, n_stages, feeds)


class Mlp:
    """Warm-start network on the current GPU (see absorber.h)."""

    def __init__(self, n_in=3, n_hidden=256, n_layers=3, n_out=210, max_batch=512, seed=0):
        c = MlpConfig()
        lib().absorber_mlp_default_config(ctypes.byref(c))
        c.n_in, c.n_hidden, c.n_layers, c.n_out, c.max_batch = n_in, n_hidden, n_layers, n_out, max_batch
        h = ctypes.c_void_p()
        _check(lib().absorber_mlp_create(ctypes.byref(c), int(seed), ctypes.byref(h)))
        self.h, self.cfg = h, c
        self.n_params = int(lib().absorber_mlp_num_params(h))

    def close(self):
        if getattr(self, "h", None):
            lib().absorber_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def default_train_options(**kw) -> MlpTrainOptions:
        o = MlpTrainOptions()
        lib().absorber_mlp_default_train_options(ctypes.byref(o))
        for k, v in kw.items():
            setattr(o, k, v)
        return o

    def set_params(self, flat: np.ndarray):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        if a.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters")
        _check(lib().absorber_mlp_set_params(self.h, a.ctypes.data_as(c_float_p)))

    def get_params(self) -> np.ndarray:
        a = np.empty(self.n_params, np.float32)
        _check(lib().absorber_mlp_get_params(self.h, a.ctypes.data_as(c_float_p)))
        return a

    def set_normalization(self, in_mean, in_std, out_mean, out_std):
        arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in (in_mean, in_std, out_mean, out_std)]
        self._norm = arrs
        _check(lib().absorber_mlp_set_normalization(self.h, *[a.ctypes.data_as(c_float_p) for a in arrs]))

    def get_normalization(self):
        arrs = [np.empty(n, np.float32) for n in (self.cfg.n_in, self.cfg.n_in, self.cfg.n_out, self.cfg.n_out)]
        _check(lib().absorber_mlp_get_normalization(self.h, *[a.ctypes.data_as(c_float_p) for a in arrs]))
        return arrs

    def fit_normalization(self, X, T, stream=None):
        _check(lib().absorber_mlp_fit_normalization(self.h, _ptr(X), _ptr(T), int(X.shape[0]), _stream(stream)))

    def forward(self, X, Y, stream=None):
        _check(lib().absorber_mlp_forward(self.h, _ptr(X), int(X.shape[0]), _ptr(Y), _stream(stream)))

    def loss_grad(self, X, T, grad, stream=None) -> float:
        loss = ctypes.c_double()
        _check(lib().absorber_mlp_loss_grad(self.h, _ptr(X), _ptr(T), int(X.shape[0]), _ptr(grad),
                                            ctypes.byref(loss), _stream(stream)))
        return loss.value

    def adam_step(self, grad, lr, opts: MlpTrainOptions | None = None, stream=None):
        o = opts if opts is not None else self.default_train_options()
        _check(lib().absorber_mlp_adam_step(self.h, _ptr(grad), ctypes.byref(o), float(lr), _stream(stream)))

    def train(self, X, T, opts: MlpTrainOptions | None = None) -> MlpTrainResult:
        o = opts if opts is not None else self.default_train_options()
        r = MlpTrainResult()
        _check(lib().absorber_mlp_train(self.h, _ptr(X), _ptr(T), int(X.shape[0]), ctypes.byref(o), ctypes.byref(r)))
        return r
