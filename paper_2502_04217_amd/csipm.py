"""Thin ctypes binding of libcsipm.so (include/csipm.h).

Argument marshalling only: device memory and streams come from torch, every
operation runs in the library's HIP kernels.  Importing this module without
the built library raises (there is no fallback path).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcsipm.so")
MLP_PARAMS = 1249
KAPPLY_PASSES = 5

FP64, FP32 = 0, 1
PC_PLAIN, PC_LEARNED, PC_SCALED = 0, 1, 2
KRYLOV_CG, KRYLOV_CR, KRYLOV_CAR = 0, 1, 2
BETA, Z, NU1, NU2, XI, DIAG_H, PC_C = range(7)

STATUS = {0: "OK", 1: "NOT_CONVERGED", 2: "STALLED", 3: "FELL_BACK", -1: "EINVAL", -2: "ENOMEM",
          -3: "EHIP", -4: "ENONFINITE", -5: "EUNSUPPORTED", -6: "ESTATE"}


class CsipmError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"csipm status {status} ({STATUS.get(status, '?')}): {msg}")
        self.status = status


class Options(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int), ("cg_max", C.c_int), ("cg_rtol", C.c_double),
                ("cg_atol", C.c_double), ("sigma", C.c_double), ("tau", C.c_double), ("precision", C.c_int),
                ("pc", C.c_int), ("refine_max", C.c_int), ("refine_inner_rtol", C.c_double),
                ("refine_trust", C.c_double), ("pc_min_cg", C.c_int), ("krylov", C.c_int),
                ("pc_rho", C.c_double), ("pc_max_relevant", C.c_double), ("mehrotra", C.c_int),
                ("build_next", C.c_int), ("graphs", C.c_int), ("pc_min_missing", C.c_double)]


class Info(C.Structure):
    _fields_ = [("status", C.c_int), ("ipm_iters", C.c_int), ("cg_iters_max", C.c_int),
                ("cg_iters_total", C.c_longlong), ("refine_steps_total", C.c_int), ("fallbacks", C.c_int),
                ("rel_kkt", C.c_double), ("res_beta_inf", C.c_double), ("res_z_inf", C.c_double),
                ("compl_max", C.c_double), ("mu", C.c_double), ("lambda_", C.c_double), ("xi_inf", C.c_double),
                ("solve_seconds", C.c_double), ("objective", C.c_double), ("dual_objective", C.c_double),
                ("rel_dual_gap", C.c_double), ("natural_residual", C.c_double), ("g_inf", C.c_double),
                ("setup_seconds", C.c_double)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["lambda"] = d.pop("lambda_")
        return d


class KernelTime(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("calls", C.c_int), ("working_calls", C.c_int), ("total_ms", C.c_double),
                ("working_ms", C.c_double), ("dropped", C.c_longlong)]


class IterLog(C.Structure):
    _fields_ = [("iter", C.c_int), ("cg_iters", C.c_int), ("refine_steps", C.c_int), ("fell_back", C.c_int),
                ("learned", C.c_int), ("mu", C.c_double), ("rel_kkt", C.c_double), ("alpha", C.c_double),
                ("relevant", C.c_double)]


def load_library(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_2502_04217_amd.build`")
    # torch first: it brings its own HIP runtime, which the library must share
    # (loaded the other way round, the process can hold two runtimes and
    # torch's device memory is then invalid for the library's calls)
    import torch  # noqa: F401
    lib = C.CDLL(path)
    P, I, D, S, F = C.c_void_p, C.c_int, C.c_double, C.c_size_t, C.c_float
    sig = {
        "csipm_default_options": (None, [C.POINTER(Options)]),
        "csipm_workspace_bytes": (S, [I, I, I]),
        "csipm_create": (I, [C.POINTER(P), I, I, I, P, P, P, S, P]),
        "csipm_set_lambda": (I, [P, D]),
        "csipm_lambda_rule": (I, [P, D, C.POINTER(D)]),
        "csipm_solve": (I, [P, C.POINTER(Options), C.POINTER(Info)]),
        "csipm_get_iterate": (I, [P, I, P]),
        "csipm_get_residuals": (I, [P, C.POINTER(Info)]),
        "csipm_get_log": (I, [P, C.POINTER(IterLog), I, C.POINTER(I)]),
        "csipm_apply_A": (I, [P, P, P, I]),
        "csipm_apply_At": (I, [P, P, P, I]),
        "csipm_apply_H": (I, [P, P, P, I]),
        "csipm_apply_K": (I, [P, P, P, P, P, I]),
        "csipm_apply_Pinv": (I, [P, P, P, P, P, I]),
        "csipm_set_barrier": (I, [P, P, P]),
        "csipm_set_pc_params": (I, [P, P, I]),
        "csipm_mlp_scratch_bytes": (S, [I]),
        "csipm_mlp_forward": (I, [P, P, P, I, P]),
        "csipm_mlp_backward": (I, [P, P, P, P, I, P, S, P]),
        "csipm_mlp_loss_grad": (I, [P, P, P, I, P, P, P, S, P]),
        "csipm_mlp_adam": (I, [P, P, P, P, I, F, P]),
        "csipm_mlp_train_step": (I, [P, P, P, I, F, P, P, I, P, P, P, S, P]),
        "csipm_mlp_loss_grad_noalloc": (I, [P, P, P, I, P, P, P]),
        "csipm_capture": (I, [P, I, P, P, I, I, C.c_ulonglong]),
        "csipm_captured": (I, [P, C.POINTER(I), P, I]),
        "csipm_features": (I, [P, P]),
        "csipm_pc_correction": (I, [P, P]),
        "csipm_profile_kapply": (I, [P, I, I, C.POINTER(D)]),
        "csipm_timing": (I, [P, I]),
        "csipm_timing_report": (I, [P, D, C.POINTER(KernelTime), I, C.POINTER(I)]),
        "csipm_destroy": (I, [P]),
        "csipm_status_string": (C.c_char_p, [I]),
        "csipm_last_error": (C.c_char_p, [P]),
        "csipm_small_workspace_bytes": (S, [I, I, I, I]),
        "csipm_solve_small_batch": (I, [I, I, I, I, P, P, P, D, C.POINTER(Options), P, P, P, S, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def default_options(**kw) -> Options:
    o = Options()
    lib().csipm_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def solve_batch(problems, opts: Options | None = None, max_threads: int = 0, **kw) -> list:
    """csipm_solve_batch: solves distinct problems concurrently (each on its
    own host thread and on the stream its Problem was created with); returns
    one info dict per problem."""
    o = opts if opts is not None else default_options(**kw)
    k = len(problems)
    ctxs = (C.c_void_p * k)(*[p._ctx.value for p in problems])
    infos = (Info * k)()
    sts = (C.c_int * k)()
    st = lib().csipm_solve_batch(ctxs, k, C.byref(o), infos, sts, int(max_threads))
    if st < 0:
        raise CsipmError(st, "solve_batch")
    out = []
    for i in range(k):
        d = infos[i].as_dict()
        d["status"] = sts[i]
        d["status_name"] = STATUS.get(sts[i], "?")
        out.append(d)
    return out


SMALL_INFO = 6
SMALL_STATUS = {0: "OK", 1: "NOT_CONVERGED", -2: "NONFINITE"}


def small_workspace_bytes(shape, count: int) -> int:
    return int(lib().csipm_small_workspace_bytes(*[int(s) for s in shape], int(count)))


def solve_small_batch(signals, observed, lambdas=None, lambda_frac: float = 0.05, opts: Options | None = None,
                      **kw):
    """csipm_solve_small_batch: count problems of one small grid (each
    extent <= 64) solved by one kernel, one workgroup per problem.
    signals: [count, N1, N2, N3] float64, observed: the same shape, nonzero =
    observed (numpy or torch); lambdas: [count] or None (lambda_frac times
    ||M_perp^T b||_inf).  Returns (beta [count, N1, N2, N3] float64 on the
    device, info [count, SMALL_INFO] on the host: status, interior-point
    iterations, PCG iterations, rel_kkt, mu, lambda)."""
    import torch
    o = opts if opts is not None else default_options(**kw)
    sig = torch.as_tensor(signals, dtype=torch.float64).to("cuda").contiguous()
    obs = (torch.as_tensor(observed) != 0).to(torch.uint8).to("cuda").contiguous()
    if sig.dim() != 4 or obs.shape != sig.shape:
        raise ValueError("signals and observed must be [count, N1, N2, N3]")
    count, shape = sig.shape[0], tuple(sig.shape[1:])
    lam = None
    if lambdas is not None:
        lam = torch.as_tensor(lambdas, dtype=torch.float64).to("cuda").contiguous()
    beta = torch.empty_like(sig)
    info = torch.empty((count, SMALL_INFO), dtype=torch.float64, device="cuda")
    nb = small_workspace_bytes(shape, count)
    if nb == 0:
        raise CsipmError(-5, "solve_small_batch: extents must lie in [1, 64]")
    ws = torch.empty(nb // 8 + 64, dtype=torch.float64, device="cuda")
    base = ws.data_ptr()
    off = (-base) % 256
    st = lib().csipm_solve_small_batch(*[int(v) for v in shape], int(count), _ptr(sig), _ptr(obs),
                                       _ptr(lam) if lam is not None else None, float(lambda_frac), C.byref(o),
                                       _ptr(beta), _ptr(info), C.c_void_p(base + off), nb, _stream())
    if st < 0:
        msg = lib().csipm_last_error(None)
        raise CsipmError(st, f"solve_small_batch: {msg.decode() if msg else ''}")
    torch.cuda.current_stream().synchronize()
    return beta, info.cpu().numpy()


def workspace_bytes(shape) -> int:
    return int(lib().csipm_workspace_bytes(*[int(s) for s in shape]))


class Problem:
    """One recovery problem on the current HIP device (csipm_create)."""

    def __init__(self, signal, observed, device="cuda", stream=None):
        """`stream` (a torch.cuda.Stream, optional): the stream every call of
        this problem queues on (default: the current stream); problems on
        distinct streams overlap in solve_batch."""
        import torch
        self.shape = tuple(int(s) for s in signal.shape)
        self.n = int(np.prod(self.shape))
        self.device = torch.device(device)
        self.signal = torch.as_tensor(signal, dtype=torch.float64).to(self.device).contiguous()
        self.observed = torch.as_tensor(observed, dtype=torch.uint8).to(self.device).contiguous()
        nbytes = workspace_bytes(self.shape)
        if nbytes == 0:
            raise CsipmError(-5, f"unsupported grid {self.shape}")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self._ws_ptr = C.c_void_p(base + off)
        self._ctx = C.c_void_p()
        self.stream = stream
        if stream is not None:
            torch.cuda.current_stream(self.device).synchronize()   # inputs copied before the context reads them
        handle = C.c_void_p(stream.cuda_stream) if stream is not None else _stream()
        st = lib().csipm_create(C.byref(self._ctx), *self.shape, _ptr(self.signal), _ptr(self.observed),
                                self._ws_ptr, nbytes, handle)
        if st != 0:
            msg = lib().csipm_last_error(None)
            raise CsipmError(st, f"csipm_create: {msg.decode() if msg else ''}")

    # -- helpers
    def _check(self, st, what):
        if st < 0:
            msg = lib().csipm_last_error(self._ctx)
            raise CsipmError(st, f"{what}: {msg.decode() if msg else ''}")
        return st

    def _vec(self, dtype=None):
        import torch
        return torch.empty(self.shape, dtype=dtype or torch.float64, device=self.device)

    def close(self):
        if self._ctx:
            lib().csipm_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- problem data
    def set_lambda(self, lam: float):
        self._check(lib().csipm_set_lambda(self._ctx, float(lam)), "set_lambda")

    def lambda_rule(self, frac: float = 0.05) -> float:
        out = C.c_double()
        self._check(lib().csipm_lambda_rule(self._ctx, float(frac), C.byref(out)), "lambda_rule")
        return out.value

    def solve(self, opts: Options | None = None, **kw) -> dict:
        o = opts if opts is not None else default_options(**kw)
        info = Info()
        st = self._check(lib().csipm_solve(self._ctx, C.byref(o), C.byref(info)), "solve")
        d = info.as_dict()
        d["status_name"] = STATUS.get(st, "?")
        return d

    def get(self, which: int):
        out = self._vec()
        self._check(lib().csipm_get_iterate(self._ctx, which, _ptr(out)), "get_iterate")
        if self.stream is not None:
            self.stream.synchronize()
        return out

    def residuals(self) -> dict:
        info = Info()
        self._check(lib().csipm_get_residuals(self._ctx, C.byref(info)), "get_residuals")
        return info.as_dict()

    def log(self) -> list:
        n = C.c_int()
        self._check(lib().csipm_get_log(self._ctx, None, 0, C.byref(n)), "get_log")
        buf = (IterLog * max(1, n.value))()
        self._check(lib().csipm_get_log(self._ctx, buf, n.value, C.byref(n)), "get_log")
        return [{f: getattr(buf[i], f) for f, _ in IterLog._fields_} for i in range(n.value)]

    # -- operators
    def _prec(self, t):
        import torch
        if t.dtype == torch.float64:
            return FP64
        if t.dtype == torch.float32:
            return FP32
        raise TypeError(t.dtype)

    def apply_A(self, beta):
        x = self._vec(beta.dtype)
        self._check(lib().csipm_apply_A(self._ctx, _ptr(beta), _ptr(x), self._prec(beta)), "apply_A")
        return x

    def apply_At(self, x):
        b = self._vec(x.dtype)
        self._check(lib().csipm_apply_At(self._ctx, _ptr(x), _ptr(b), self._prec(x)), "apply_At")
        return b

    def apply_H(self, beta):
        y = self._vec(beta.dtype)
        self._check(lib().csipm_apply_H(self._ctx, _ptr(beta), _ptr(y), self._prec(beta)), "apply_H")
        return y

    def apply_K(self, pb, pz):
        qb, qz = self._vec(pb.dtype), self._vec(pb.dtype)
        self._check(lib().csipm_apply_K(self._ctx, _ptr(pb), _ptr(pz), _ptr(qb), _ptr(qz), self._prec(pb)),
                    "apply_K")
        return qb, qz

    def apply_Pinv(self, rb, rz):
        zb, zz = self._vec(rb.dtype), self._vec(rb.dtype)
        self._check(lib().csipm_apply_Pinv(self._ctx, _ptr(rb), _ptr(rz), _ptr(zb), _ptr(zz), self._prec(rb)),
                    "apply_Pinv")
        return zb, zz

    def set_barrier(self, sig1, sig2):
        self._b1, self._b2 = sig1.contiguous(), sig2.contiguous()
        self._check(lib().csipm_set_barrier(self._ctx, _ptr(self._b1), _ptr(self._b2)), "set_barrier")

    # -- learned preconditioner
    def set_pc_params(self, params):
        self._params = params.contiguous()
        self._check(lib().csipm_set_pc_params(self._ctx, _ptr(self._params), self._params.numel()),
                    "set_pc_params")

    def capture(self, feat, rec, n_per_iter: int, max_iters: int, seed: int = 0, policy: bool = False):
        """csipm_capture; policy=True is mode 2 (iterations and coefficients
        where the learned form applies the correction)."""
        self._cap = (feat, rec)
        self._check(lib().csipm_capture(self._ctx, 2 if policy else 1, _ptr(feat), _ptr(rec), n_per_iter,
                                        max_iters, seed), "capture")

    def capture_off(self):
        self._check(lib().csipm_capture(self._ctx, 0, None, None, 0, 0, 0), "capture")

    def captured(self, max_iters: int = 1024):
        n = C.c_int()
        cg = (C.c_int * max_iters)()
        self._check(lib().csipm_captured(self._ctx, C.byref(n), cg, max_iters), "captured")
        return n.value, list(cg[:n.value])

    def profile_kapply(self, precision: int, reps: int = 20, direct: bool = False):
        """Average milliseconds of each of the KAPPLY_PASSES K-apply kernels
        (events around each), and of one whole K-apply among `reps` back to
        back (one event pair; replayed from a HIP graph, or launched directly
        with direct=True): (list, float)."""
        ms, graph, launched = self.profile_kapply_all(precision, reps)
        return ms, launched if direct else graph

    def profile_kapply_all(self, precision: int, reps: int = 20):
        """csipm_profile_kapply: (per-kernel ms, whole K-apply from a graph
        replay, whole K-apply launched directly)."""
        out = (C.c_double * (KAPPLY_PASSES + 2))()
        self._check(lib().csipm_profile_kapply(self._ctx, precision, reps, out), "profile_kapply")
        return list(out[:KAPPLY_PASSES]), out[KAPPLY_PASSES], out[KAPPLY_PASSES + 1]

    def timing(self, enable: bool):
        """Start (clearing earlier records) or stop per-kernel event timing."""
        self._check(lib().csipm_timing(self._ctx, 1 if enable else 0), "timing")

    def timing_report(self, min_us: float = 8.0) -> list:
        """Per-kernel aggregates of the recorded launches: name, calls,
        working_calls (those lasting >= min_us), total_ms, working_ms."""
        n = C.c_int(0)
        self._check(lib().csipm_timing_report(self._ctx, min_us, None, 0, C.byref(n)), "timing_report")
        buf = (KernelTime * max(1, n.value))()
        self._check(lib().csipm_timing_report(self._ctx, min_us, buf, n.value, C.byref(n)), "timing_report")
        return [{"name": r.name.decode(), "calls": r.calls, "working_calls": r.working_calls,
                 "total_ms": r.total_ms, "working_ms": r.working_ms, "dropped": r.dropped} for r in buf[:n.value]]

    def pc_correction(self):
        out = self._vec()
        self._check(lib().csipm_pc_correction(self._ctx, _ptr(out)), "pc_correction")
        return out

    def features(self):
        import torch
        out = torch.empty((self.n, 4), dtype=torch.float32, device=self.device)
        self._check(lib().csipm_features(self._ctx, _ptr(out)), "features")
        return out


def _check(st, what):
    if st != 0:
        raise CsipmError(st, what)


def mlp_forward(params, feat):
    import torch
    c = torch.empty(feat.shape[0], dtype=torch.float32, device=feat.device)
    _check(lib().csipm_mlp_forward(_ptr(params), _ptr(feat), _ptr(c), feat.shape[0], _stream()), "mlp_forward")
    return c


def _scratch(n, device):
    import torch
    nb = int(lib().csipm_mlp_scratch_bytes(n))
    return torch.empty(nb // 8 + 1, dtype=torch.float64, device=device), nb


def mlp_backward(params, feat, dc, grad=None):
    import torch
    g = torch.zeros(MLP_PARAMS, dtype=torch.float32, device=feat.device) if grad is None else grad
    sc, nb = _scratch(feat.shape[0], feat.device)
    _check(lib().csipm_mlp_backward(_ptr(params), _ptr(feat), _ptr(dc), _ptr(g), feat.shape[0], _ptr(sc), nb,
                                    _stream()), "mlp_backward")
    return g


def mlp_loss_grad(params, feat, rec, scratch=None):
    import torch
    n = feat.shape[0]
    g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=feat.device)
    loss = torch.empty(1, dtype=torch.float64, device=feat.device)
    sc, nb = scratch if scratch is not None else _scratch(n, feat.device)
    _check(lib().csipm_mlp_loss_grad(_ptr(params), _ptr(feat), _ptr(rec), n, _ptr(loss), _ptr(g), _ptr(sc), nb,
                                     _stream()), "mlp_loss_grad")
    return loss, g


NOALLOC_MAX_REC = 65536


def mlp_loss_grad_noalloc(params, feat, rec, loss, grad):
    """csipm_mlp_loss_grad_noalloc into caller-given loss (1 double) and grad
    (1249 floats) tensors: nothing is allocated on the device by the call."""
    st = lib().csipm_mlp_loss_grad_noalloc(_ptr(params), _ptr(feat), _ptr(rec), int(feat.shape[0]), _ptr(loss),
                                           _ptr(grad), _stream())
    if st != 0:
        msg = lib().csipm_last_error(None)
        raise CsipmError(st, f"mlp_loss_grad_noalloc: {msg.decode() if msg else ''}")


def mlp_train_step(params, m, v, t, lr, feat, rec, scratch=None):
    """csipm_mlp_train_step: loss and gradient at params, then one Adam step
    (params, m, v updated in place); returns (loss, grad)."""
    import torch
    n = feat.shape[0]
    g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=feat.device)
    loss = torch.empty(1, dtype=torch.float64, device=feat.device)
    sc, nb = scratch if scratch is not None else _scratch(n, feat.device)
    _check(lib().csipm_mlp_train_step(_ptr(params), _ptr(m), _ptr(v), int(t), float(lr), _ptr(feat), _ptr(rec), n,
                                      _ptr(loss), _ptr(g), _ptr(sc), nb, _stream()), "mlp_train_step")
    return loss, g


def mlp_adam(params, grad, m, v, t, lr):
    _check(lib().csipm_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(t), float(lr), _stream()),
           "mlp_adam")
