"""Thin Python binding of libfastlsq (ctypes; argument marshalling only).

Every function here forwards to the C entry point of the same name in
``include/fastlsq.h``; all arithmetic runs in the library's HIP kernels.  Device
arrays are torch tensors on the context's GPU (float64, contiguous); host arrays
are numpy arrays or Python sequences.  PyTorch provides device memory and the
stream only.  There is no fallback: if the library is missing or the GPU is
absent, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfastlsq.so")

FLSQ_OK, FLSQ_EINVAL, FLSQ_ENOTSPD, FLSQ_ENOCONV, FLSQ_EHIP, FLSQ_ENOMEM, FLSQ_ENONFINITE = range(7)
STATUS_NAMES = {0: "FLSQ_OK", 1: "FLSQ_EINVAL", 2: "FLSQ_ENOTSPD", 3: "FLSQ_ENOCONV", 4: "FLSQ_EHIP",
                5: "FLSQ_ENOMEM", 6: "FLSQ_ENONFINITE"}
PREC_FP64, PREC_FP32_REFINE, PREC_BF16X3_REFINE, PREC_INT8_CRT = 0, 1, 2, 3
MAX_DIM = 8

# Every symbol the header declares (checked by the CPU test suite).
EXPORTS = (
    "flsq_create", "flsq_destroy", "flsq_last_error", "flsq_build_info", "flsq_assemble", "flsq_gram",
    "flsq_solve_linear", "flsq_factorize", "flsq_factor_free", "flsq_factor_shape", "flsq_factor_solve",
    "flsq_factor_solve_normal", "flsq_apply_A", "flsq_apply_At", "flsq_evaluate", "flsq_evaluate_noalloc", "flsq_solve_newton",
    "flsq_inverse_loss_grad", "flsq_inverse_prepare", "flsq_bandwidth_loss_grad", "flsq_adam_step",
    "flsq_assemble_var",
    "flsq_solve_linear_var", "flsq_solve_newton_var",
)


class FlsqError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class flsq_term(C.Structure):
    _fields_ = [("coef", C.c_double), ("alpha", C.c_uint8 * MAX_DIM)]


class flsq_op(C.Structure):
    _fields_ = [("terms", C.POINTER(flsq_term)), ("n_terms", C.c_int32)]


class flsq_basis(C.Structure):
    _fields_ = [("d", C.c_int32), ("n_feat", C.c_int32), ("W", C.c_void_p), ("b", C.c_void_p),
                ("normalize", C.c_int32)]


class flsq_rows(C.Structure):
    _fields_ = [("n_rows", C.c_int64), ("x", C.c_void_p), ("op", flsq_op), ("weight", C.c_double),
                ("rhs", C.c_void_p)]


class flsq_solve_opts(C.Structure):
    _fields_ = [("mu", C.c_double), ("prec", C.c_int32), ("max_refine", C.c_int32), ("refine_tol", C.c_double),
                ("shift_rel", C.c_double), ("report_grad", C.c_int32), ("second_pass", C.c_int32),
                ("pivot_boost", C.c_double), ("store_matrix", C.c_int32)]


class flsq_solve_info(C.Structure):
    _fields_ = [("refine_iters", C.c_int32), ("chol_retries", C.c_int32), ("shift", C.c_double),
                ("grad_norm0", C.c_double), ("grad_norm", C.c_double), ("last_step_rel", C.c_double),
                ("t_gram_ms", C.c_double), ("t_chol_ms", C.c_double), ("t_refine_ms", C.c_double),
                ("t_total_ms", C.c_double), ("t_gram_kernel_ms", C.c_double), ("second_pass", C.c_int32),
                ("t_second_pass_ms", C.c_double), ("boosted_pivots", C.c_int32),
                ("shift_recalled", C.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class flsq_nonlin(C.Structure):
    _fields_ = [("n_poly", C.c_int32), ("poly", C.POINTER(C.c_double))]


class flsq_channel(C.Structure):
    _fields_ = [("op", flsq_op), ("coef", C.c_void_p)]


class flsq_vrows(C.Structure):
    _fields_ = [("n_rows", C.c_int64), ("x", C.c_void_p), ("weight", C.c_double), ("rhs", C.c_void_p),
                ("n_channels", C.c_int32), ("channels", C.POINTER(flsq_channel))]


class flsq_nonlin_grad(C.Structure):
    _fields_ = [("n_poly", C.c_int32), ("poly", C.POINTER(C.c_double)), ("n_adv", C.c_int32),
                ("adv_coef", C.POINTER(C.c_double)), ("adv_pow", C.POINTER(C.c_int32)),
                ("adv_axis", C.POINTER(C.c_int32)), ("exp_coef", C.c_double)]


class flsq_newton_opts(C.Structure):
    _fields_ = [("lin", flsq_solve_opts), ("tol_dbeta", C.c_double), ("max_iter", C.c_int32),
                ("armijo_c", C.c_double), ("max_halvings", C.c_int32), ("warm_start", C.c_int32),
                ("refactor_iters", C.c_int32)]


class flsq_newton_trace(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("res_norm", C.c_double * 64),
                ("alpha", C.c_double * 64), ("step_norm", C.c_double * 64), ("du_rel", C.c_double * 64),
                ("halvings", C.c_int32 * 64), ("t_total_ms", C.c_double), ("refine_iters", C.c_int32 * 64),
                ("shift", C.c_double * 64), ("t_solve_ms", C.c_double * 64), ("factored", C.c_int32 * 64)]

    def as_list(self):
        return [dict(it=i, res_norm=self.res_norm[i], alpha=self.alpha[i], step_norm=self.step_norm[i],
                     du_rel=self.du_rel[i], halvings=self.halvings[i], refine_iters=self.refine_iters[i],
                     shift=self.shift[i], t_solve_ms=self.t_solve_ms[i], factored=self.factored[i])
                for i in range(self.iters)]


_lib = None


def load(path: str = LIB_PATH):
    """Load the in-tree library; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: run __graft_entry__.build() (hipcc, gfx950) first")
    lib = C.CDLL(path)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    st = C.c_int
    sig = {
        "flsq_create": (st, [C.POINTER(vp), C.c_int, vp]),
        "flsq_destroy": (None, [vp]),
        "flsq_last_error": (C.c_char_p, [vp]),
        "flsq_build_info": (C.c_char_p, []),
        "flsq_assemble": (st, [vp, C.POINTER(flsq_basis), C.POINTER(flsq_rows), i32, i32, vp, vp]),
        "flsq_gram": (st, [vp, C.POINTER(flsq_basis), C.POINTER(flsq_rows), i32, i32, vp, vp]),
        "flsq_solve_linear": (st, [vp, C.POINTER(flsq_basis), C.POINTER(flsq_rows), i32,
                                   C.POINTER(flsq_solve_opts), vp, C.POINTER(flsq_solve_info)]),
        "flsq_factorize": (st, [vp, C.POINTER(flsq_basis), C.POINTER(flsq_rows), i32, C.POINTER(flsq_solve_opts),
                                C.POINTER(vp), C.POINTER(flsq_solve_info)]),
        "flsq_factor_free": (None, [vp]),
        "flsq_factor_shape": (st, [vp, C.POINTER(i64), C.POINTER(i32)]),
        "flsq_factor_solve": (st, [vp, vp, vp, i32, vp, C.POINTER(flsq_solve_info)]),
        "flsq_factor_solve_normal": (st, [vp, vp, vp, i32, vp]),
        "flsq_apply_A": (st, [vp, vp, vp, i32, vp]),
        "flsq_apply_At": (st, [vp, vp, vp, i32, vp]),
        "flsq_evaluate": (st, [vp, C.POINTER(flsq_basis), vp, i64, vp, i32, C.POINTER(C.c_uint8), i32, vp]),
        "flsq_evaluate_noalloc": (st, [vp, C.POINTER(flsq_basis), vp, i64, vp, i32, C.POINTER(C.c_uint8), i32, vp]),
        "flsq_solve_newton": (st, [vp, C.POINTER(flsq_basis), C.POINTER(flsq_rows), i32, i32,
                                   C.POINTER(flsq_nonlin), C.POINTER(flsq_newton_opts), vp,
                                   C.POINTER(flsq_newton_trace)]),
        "flsq_inverse_loss_grad": (st, [vp, vp, i64, dbl, i32, vp, i32, i64, vp, vp, vp, vp, vp]),
        "flsq_inverse_prepare": (st, [vp, vp, i64, i64, vp]),
        "flsq_bandwidth_loss_grad": (st, [vp, C.POINTER(flsq_basis), C.POINTER(dbl), C.POINTER(flsq_rows), i32,
                                          C.POINTER(flsq_solve_opts), vp, C.POINTER(dbl), C.POINTER(dbl)]),
        "flsq_adam_step": (st, [vp, vp, vp, vp, vp, i32, i32, i32, dbl, dbl, dbl, dbl, i32, dbl, dbl]),
        "flsq_assemble_var": (st, [vp, C.POINTER(flsq_basis), C.POINTER(flsq_vrows), i32, vp, vp]),
        "flsq_solve_linear_var": (st, [vp, C.POINTER(flsq_basis), C.POINTER(flsq_vrows), i32,
                                       C.POINTER(flsq_solve_opts), vp, C.POINTER(flsq_solve_info)]),
        "flsq_solve_newton_var": (st, [vp, C.POINTER(flsq_basis), C.POINTER(flsq_vrows), i32, i32,
                                       C.POINTER(flsq_nonlin_grad), C.POINTER(flsq_newton_opts), dbl, vp,
                                       C.POINTER(flsq_newton_trace)]),
    }
    missing = [name for name in sig if not hasattr(lib, name)]
    if missing:
        raise RuntimeError(f"{path} does not export {missing}: rebuild it")
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(t):
    """Device pointer of a contiguous torch tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _check_f64(t, name):
    import torch
    if t is not None and (t.dtype != torch.float64 or not t.is_cuda):
        raise ValueError(f"{name} must be a float64 GPU tensor")


class Context:
    """flsq_create / flsq_destroy around torch's current stream on ``device``."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the HIP library needs a ROCm device")
        self.device = device
        torch.cuda.set_device(device)
        s = stream if stream is not None else torch.cuda.current_stream(device)
        self.stream = s
        h = C.c_void_p()
        st = self.lib.flsq_create(C.byref(h), device, C.c_void_p(s.cuda_stream))
        if st != FLSQ_OK:
            raise FlsqError(st, "flsq_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.flsq_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, st):
        if st != FLSQ_OK:
            raise FlsqError(st, self.lib.flsq_last_error(self.h).decode())
        return st

    def last_error(self):
        return self.lib.flsq_last_error(self.h).decode()


# ---------------------------------------------------------------------------- argument marshalling

@dataclass
class Basis:
    struct: flsq_basis
    W: object
    b: object


def make_basis(W, b, normalize=True) -> Basis:
    _check_f64(W, "W")
    _check_f64(b, "b")
    n, d = W.shape
    return Basis(flsq_basis(d, n, W.data_ptr(), b.data_ptr(), int(bool(normalize))), W, b)


def make_terms(terms, d):
    arr = (flsq_term * len(terms))()
    for i, (c, a) in enumerate(terms):
        arr[i].coef = float(c)
        a = list(a)
        if len(a) > MAX_DIM:
            raise ValueError("multi-index longer than the ABI supports")
        for k, v in enumerate(a):
            arr[i].alpha[k] = int(v)
    return arr


@dataclass
class Rows:
    array: object          # ctypes array of flsq_rows
    keep: list             # objects that must outlive the call
    n_blocks: int


def make_rows(blocks, d) -> Rows:
    """blocks: sequence of (x [n x d float64 GPU tensor], terms, weight, rhs tensor or None)."""
    arr = (flsq_rows * len(blocks))()
    keep = []
    for i, (x, terms, weight, rhs) in enumerate(blocks):
        _check_f64(x, "x")
        _check_f64(rhs, "rhs")
        t = make_terms(terms, d)
        keep += [x, rhs, t]
        arr[i].n_rows = int(x.shape[0])
        arr[i].x = x.data_ptr() if x.numel() else None
        arr[i].op = flsq_op(C.cast(t, C.POINTER(flsq_term)), len(terms))
        arr[i].weight = float(weight)
        arr[i].rhs = rhs.data_ptr() if (rhs is not None and rhs.numel()) else None
    return Rows(arr, keep, len(blocks))


@dataclass
class VRows:
    array: object          # ctypes array of flsq_vrows
    keep: list
    n_blocks: int


def make_vrows(blocks, d) -> VRows:
    """blocks: sequence of (x [n x d float64 GPU tensor], channels, weight, rhs tensor or None), each
    channel a (terms, coef GPU tensor of n float64 or None) pair."""
    arr = (flsq_vrows * len(blocks))()
    keep = []
    for i, (x, channels, weight, rhs) in enumerate(blocks):
        _check_f64(x, "x")
        _check_f64(rhs, "rhs")
        ch = (flsq_channel * len(channels))()
        for t, (terms, coef) in enumerate(channels):
            _check_f64(coef, "channel coefficient")
            tt = make_terms(terms, d)
            keep += [tt, coef]
            ch[t].op = flsq_op(C.cast(tt, C.POINTER(flsq_term)), len(terms))
            ch[t].coef = coef.data_ptr() if (coef is not None and coef.numel()) else None
        keep += [x, rhs, ch]
        arr[i].n_rows = int(x.shape[0])
        arr[i].x = x.data_ptr() if x.numel() else None
        arr[i].weight = float(weight)
        arr[i].rhs = rhs.data_ptr() if (rhs is not None and rhs.numel()) else None
        arr[i].n_channels = len(channels)
        arr[i].channels = C.cast(ch, C.POINTER(flsq_channel))
    return VRows(arr, keep, len(blocks))


def solve_opts(mu, prec=PREC_FP64, max_refine=10, refine_tol=1e-12, shift_rel=0.0, report_grad=False,
               second_pass=0, pivot_boost=0.0, store_matrix=False):
    return flsq_solve_opts(float(mu), int(prec), int(max_refine), float(refine_tol), float(shift_rel),
                           1 if report_grad else 0, int(second_pass), float(pivot_boost), 1 if store_matrix else 0)


# ---------------------------------------------------------------------------- entry points

def flsq_build_info():
    return load().flsq_build_info().decode()


def flsq_assemble(ctx, basis: Basis, rows: Rows, A_out, rhs_out=None, fp32=False):
    return ctx.check(ctx.lib.flsq_assemble(ctx.h, C.byref(basis.struct), rows.array, rows.n_blocks, int(fp32),
                                           _ptr(A_out), _ptr(rhs_out)))


def flsq_gram(ctx, basis: Basis, rows: Rows, prec, G_out, c_out=None):
    return ctx.check(ctx.lib.flsq_gram(ctx.h, C.byref(basis.struct), rows.array, rows.n_blocks, int(prec),
                                       _ptr(G_out), _ptr(c_out)))


def flsq_solve_linear(ctx, basis: Basis, rows: Rows, opts: flsq_solve_opts, beta_out, check=True):
    info = flsq_solve_info()
    st = ctx.lib.flsq_solve_linear(ctx.h, C.byref(basis.struct), rows.array, rows.n_blocks, C.byref(opts),
                                   _ptr(beta_out), C.byref(info))
    if check and st not in (FLSQ_OK, FLSQ_ENOCONV):
        ctx.check(st)
    return st, info


class Factor:
    def __init__(self, ctx, handle, info):
        self.ctx, self.h, self.info = ctx, handle, info

    def shape(self):
        P, n = C.c_int64(), C.c_int32()
        self.ctx.check(self.ctx.lib.flsq_factor_shape(self.h, C.byref(P), C.byref(n)))
        return P.value, n.value

    def free(self):
        if self.h:
            self.ctx.lib.flsq_factor_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def flsq_factorize(ctx, basis: Basis, rows: Rows, opts: flsq_solve_opts) -> Factor:
    h = C.c_void_p()
    info = flsq_solve_info()
    ctx.check(ctx.lib.flsq_factorize(ctx.h, C.byref(basis.struct), rows.array, rows.n_blocks, C.byref(opts),
                                     C.byref(h), C.byref(info)))
    return Factor(ctx, h, info)


def flsq_factor_solve(ctx, F: Factor, rhs_rows, beta_out):
    K = 1 if rhs_rows.dim() == 1 else rhs_rows.shape[1]
    info = flsq_solve_info()
    ctx.check(ctx.lib.flsq_factor_solve(ctx.h, F.h, _ptr(rhs_rows), K, _ptr(beta_out), C.byref(info)))
    return info


def flsq_factor_solve_normal(ctx, F: Factor, V, out):
    K = 1 if V.dim() == 1 else V.shape[1]
    return ctx.check(ctx.lib.flsq_factor_solve_normal(ctx.h, F.h, _ptr(V), K, _ptr(out)))


def flsq_apply_A(ctx, F: Factor, V, out):
    K = 1 if V.dim() == 1 else V.shape[1]
    return ctx.check(ctx.lib.flsq_apply_A(ctx.h, F.h, _ptr(V), K, _ptr(out)))


def flsq_apply_At(ctx, F: Factor, Y, out):
    K = 1 if Y.dim() == 1 else Y.shape[1]
    return ctx.check(ctx.lib.flsq_apply_At(ctx.h, F.h, _ptr(Y), K, _ptr(out)))


def flsq_evaluate(ctx, basis: Basis, beta, xq, alphas, out):
    import torch
    d = basis.struct.d
    al = np.ascontiguousarray(np.array([list(a) for a in alphas], dtype=np.uint8).reshape(len(alphas), d))
    fp32 = xq.dtype == torch.float32
    return ctx.check(ctx.lib.flsq_evaluate(ctx.h, C.byref(basis.struct), _ptr(beta), int(xq.shape[0]), _ptr(xq),
                                           int(fp32), al.ctypes.data_as(C.POINTER(C.c_uint8)), len(alphas),
                                           _ptr(out)))


def flsq_evaluate_noalloc(ctx, basis: Basis, beta, xq, alphas, out):
    """flsq_evaluate with its staging in the library's static per-device scratch (no device allocation)."""
    import torch
    d = basis.struct.d
    al = np.ascontiguousarray(np.array([list(a) for a in alphas], dtype=np.uint8).reshape(len(alphas), d))
    fp32 = xq.dtype == torch.float32
    return ctx.check(ctx.lib.flsq_evaluate_noalloc(ctx.h, C.byref(basis.struct), _ptr(beta), int(xq.shape[0]),
                                                   _ptr(xq), int(fp32), al.ctypes.data_as(C.POINTER(C.c_uint8)),
                                                   len(alphas), _ptr(out)))


def newton_opts(mu, max_iter=15, tol_dbeta=1e-10, armijo_c=1e-4, max_halvings=10, warm_start=True,
                prec=PREC_FP64, max_refine=60, refine_tol=1e-14, refactor_iters=16):
    """Defaults: each Gauss-Newton step refined until u changes by < 1e-14 relative (at most 60 CG
    steps), preconditioned by the last factor formed while it converges within 16 CG steps
    (refactor_iters=0: a Gram and factor at every step)."""
    return flsq_newton_opts(solve_opts(mu, prec, max_refine, refine_tol), float(tol_dbeta), int(max_iter),
                            float(armijo_c), int(max_halvings), int(bool(warm_start)), int(refactor_iters))


def flsq_solve_newton(ctx, basis: Basis, rows: Rows, nonlin_block, poly, opts: flsq_newton_opts, beta_inout,
                      check=True):
    p = (C.c_double * len(poly))(*[float(v) for v in poly])
    nl = flsq_nonlin(len(poly), C.cast(p, C.POINTER(C.c_double)))
    tr = flsq_newton_trace()
    st = ctx.lib.flsq_solve_newton(ctx.h, C.byref(basis.struct), rows.array, rows.n_blocks, int(nonlin_block),
                                   C.byref(nl), C.byref(opts), _ptr(beta_inout), C.byref(tr))
    if check and st not in (FLSQ_OK, FLSQ_ENOCONV):
        ctx.check(st)
    return st, tr


def flsq_assemble_var(ctx, basis: Basis, rows: VRows, A_out, rhs_out=None):
    return ctx.check(ctx.lib.flsq_assemble_var(ctx.h, C.byref(basis.struct), rows.array, rows.n_blocks, _ptr(A_out),
                                               _ptr(rhs_out)))


def flsq_solve_linear_var(ctx, basis: Basis, rows: VRows, opts: flsq_solve_opts, beta_out, check=True):
    info = flsq_solve_info()
    st = ctx.lib.flsq_solve_linear_var(ctx.h, C.byref(basis.struct), rows.array, rows.n_blocks, C.byref(opts),
                                       _ptr(beta_out), C.byref(info))
    if check and st not in (FLSQ_OK, FLSQ_ENOCONV):
        ctx.check(st)
    return st, info


def flsq_solve_newton_var(ctx, basis: Basis, rows: VRows, nonlin_block, poly, adv, opts: flsq_newton_opts, tol_du,
                          beta_inout, check=True, exp_coef=0.0):
    """adv: sequence of (coef, power, axis) for the terms coef u^power d_axis u; exp_coef: + exp_coef e^u."""
    poly = list(poly or ())
    p = (C.c_double * max(1, len(poly)))(*[float(v) for v in poly])
    ac = (C.c_double * max(1, len(adv)))(*[float(c) for c, _, _ in adv])
    ap = (C.c_int32 * max(1, len(adv)))(*[int(m) for _, m, _ in adv])
    ax = (C.c_int32 * max(1, len(adv)))(*[int(a) for _, _, a in adv])
    nl = flsq_nonlin_grad(len(poly), C.cast(p, C.POINTER(C.c_double)), len(adv), C.cast(ac, C.POINTER(C.c_double)),
                          C.cast(ap, C.POINTER(C.c_int32)), C.cast(ax, C.POINTER(C.c_int32)), float(exp_coef))
    tr = flsq_newton_trace()
    st = ctx.lib.flsq_solve_newton_var(ctx.h, C.byref(basis.struct), rows.array, rows.n_blocks, int(nonlin_block),
                                       C.byref(nl), C.byref(opts), float(tol_du), _ptr(beta_inout), C.byref(tr))
    if check and st not in (FLSQ_OK, FLSQ_ENOCONV):
        ctx.check(st)
    return st, tr


def flsq_inverse_loss_grad(ctx, F: Factor, n_src_rows, src_weight, n_lap_dims, thetas, x_obs, data, loss_out,
                           grad_theta_out, grad_kappa_out=None):
    return ctx.check(ctx.lib.flsq_inverse_loss_grad(
        ctx.h, F.h, int(n_src_rows), float(src_weight), int(n_lap_dims), _ptr(thetas), int(thetas.shape[0]),
        int(x_obs.shape[0]), _ptr(x_obs), _ptr(data), _ptr(loss_out), _ptr(grad_theta_out),
        _ptr(grad_kappa_out)))


def flsq_inverse_prepare(ctx, F: Factor, n_src_rows, x_obs):
    """Keep the observation operator R = H (A^T A + mu I)^{-1} A_src^T on the factor (keyed by
    n_src_rows and the x_obs tensor's device pointer)."""
    return ctx.check(ctx.lib.flsq_inverse_prepare(ctx.h, F.h, int(n_src_rows), int(x_obs.shape[0]), _ptr(x_obs)))


def flsq_bandwidth_loss_grad(ctx, base: Basis, L, rows: Rows, opts: flsq_solve_opts, beta_out):
    """Outer loss ||A(L) beta* - b||^2 and its gradient in the lower-triangular L (packed row by row),
    with W_j = L What_j for the frozen draws in `base`.  L: host d x d (any array-like)."""
    import numpy as np
    Lh = np.ascontiguousarray(np.asarray(L, dtype=np.float64))
    d = Lh.shape[0]
    loss = C.c_double()
    grad = (C.c_double * (d * (d + 1) // 2))()
    ctx.check(ctx.lib.flsq_bandwidth_loss_grad(
        ctx.h, C.byref(base.struct), Lh.ctypes.data_as(C.POINTER(C.c_double)), rows.array, rows.n_blocks,
        C.byref(opts), _ptr(beta_out), C.byref(loss), grad))
    return loss.value, np.array(grad[:], dtype=np.float64)


def flsq_adam_step(ctx, params, grads, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8, clamp_col=-1, clamp_min=0.0,
                   weight_decay=0.0):
    """Adam (AdamW when weight_decay > 0) on device arrays of shape K x P (a 1-D array is 1 x P)."""
    K, P = (1, params.shape[0]) if params.dim() == 1 else params.shape
    return ctx.check(ctx.lib.flsq_adam_step(ctx.h, _ptr(params), _ptr(grads), _ptr(m), _ptr(v), int(K), int(P),
                                            int(t), float(lr), float(b1), float(b2), float(eps), int(clamp_col),
                                            float(clamp_min), float(weight_decay)))


# ---------------------------------------------------------------------------- workload helpers

class DeviceProblem:
    """A workloads.Problem moved to the GPU with its ABI structures."""

    def __init__(self, prob, device="cuda"):
        import torch
        self.prob = prob
        f64 = dict(dtype=torch.float64, device=device)
        self.W = torch.tensor(prob.W, **f64).contiguous()
        self.b = torch.tensor(prob.b, **f64).contiguous()
        self.basis = make_basis(self.W, self.b, prob.normalize)
        self.xs = [torch.tensor(bl.x, **f64).contiguous() for bl in prob.blocks]
        self.rhs = [torch.tensor(bl.rhs, **f64).contiguous() for bl in prob.blocks]
        self.rows = make_rows([(x, bl.terms, bl.weight, r) for x, bl, r in zip(self.xs, prob.blocks, self.rhs)],
                              prob.d)
        self.n_rows = sum(int(x.shape[0]) for x in self.xs)

    def rows_with_terms(self, terms_per_block):
        return make_rows([(x, t, bl.weight, r) for x, t, bl, r in
                          zip(self.xs, terms_per_block, self.prob.blocks, self.rhs)], self.prob.d)


class DeviceVarProblem:
    """A workloads.Problem whose blocks carry row-dependent channels, moved to the GPU."""

    def __init__(self, prob, device="cuda"):
        import torch
        self.prob = prob
        f64 = dict(dtype=torch.float64, device=device)
        self.W = torch.tensor(prob.W, **f64).contiguous()
        self.b = torch.tensor(prob.b, **f64).contiguous()
        self.basis = make_basis(self.W, self.b, prob.normalize)
        self.xs = [torch.tensor(bl.x, **f64).contiguous() for bl in prob.blocks]
        self.rhs = [torch.tensor(bl.rhs, **f64).contiguous() for bl in prob.blocks]
        self.coefs = [[None if a is None else torch.tensor(a, **f64).contiguous() for _, a in bl.channels]
                      for bl in prob.blocks]
        self.rows = make_vrows([(x, [(t, a) for (t, _), a in zip(bl.channels, cs)], bl.weight, r)
                                for x, bl, cs, r in zip(self.xs, prob.blocks, self.coefs, self.rhs)], prob.d)
        self.n_rows = sum(int(x.shape[0]) for x in self.xs)
