"""Python binding of libopengrape.so (ctypes; argument marshalling only).

Every step of the propagation, cost and gradient runs in the library's HIP
kernels.  PyTorch provides device memory and the stream.  There is no CPU
fallback: creating a Problem without the built library, or without a GPU,
raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("OPENGRAPE_LIB") or os.path.join(_HERE, "libopengrape.so")

PREC = {"f64": 0, "f32": 1, "bf16x3": 2, "f16x3": 3}
GMODE = {"grape1": 0, "exact": 1}
PATH = {"auto": 0, "dense": 1, "banded": 2}
PATH_NAMES = {1: "dense", 2: "banded"}

STATUS = {
    0: "OG_OK",
    -1: "OG_ERR_ARG",
    -2: "OG_ERR_SHAPE",
    -3: "OG_ERR_NOT_HERMITIAN",
    -4: "OG_ERR_UNSTABLE_DT",
    -5: "OG_ERR_WORKSPACE",
    -6: "OG_ERR_ORDER",
    -7: "OG_ERR_NONFINITE",
    -8: "OG_ERR_DEVICE",
}

# Every symbol declared in include/opengrape.h.
EXPORTS = (
    "og_default_options", "og_create", "og_destroy", "og_path_used", "og_workspace_bytes",
    "og_forward", "og_cost", "og_adjoint", "og_gradient", "og_profile", "og_profile_read",
    "og_server_create", "og_server_submit", "og_server_step", "og_server_active", "og_server_completed",
    "og_server_destroy", "og_status_string", "og_last_error", "og_gradient_sum", "og_set_penalty",
    "og_filter_apply", "og_filter_grad", "og_create_banded", "og_set_adaptive", "og_adaptive_stats",
    "og_set_resident", "og_generation", "og_set_fused", "og_fused_used", "og_evaluate_static",
)
STATIC_WS_BYTES = 256 << 20  # OG_STATIC_WS_BYTES


class OgRequest(ctypes.Structure):
    _fields_ = [("n_t", ctypes.c_int), ("dt", ctypes.c_double), ("u", ctypes.c_void_p), ("rho0", ctypes.c_void_p),
                ("sigma", ctypes.c_void_p), ("phi", ctypes.c_void_p), ("grad", ctypes.c_void_p),
                ("ws", ctypes.c_void_p), ("ws_bytes", ctypes.c_size_t), ("tag", ctypes.c_long)]


class OgOptions(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int), ("gmode", ctypes.c_int), ("path", ctypes.c_int),
                ("n_sub", ctypes.c_int), ("ckpt_stride", ctypes.c_int), ("validate", ctypes.c_int)]


class OgError(RuntimeError):
    def __init__(self, status: int, detail: str):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__(f"{self.name}: {detail}")


_LIB = None


def load_library(path: str = LIB_PATH):
    """Load libopengrape.so and declare the C signatures (no GPU needed)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    lib.og_default_options.argtypes = [ctypes.POINTER(OgOptions)]
    lib.og_default_options.restype = None
    lib.og_create.argtypes = [ctypes.POINTER(vp), i, i, i, vp, vp, vp, vp, ctypes.POINTER(OgOptions)]
    lib.og_create.restype = i
    lib.og_create_banded.argtypes = [ctypes.POINTER(vp), i, i, i, i, vp, vp, vp, vp, vp, ctypes.POINTER(OgOptions)]
    lib.og_create_banded.restype = i
    lib.og_destroy.argtypes = [vp]
    lib.og_destroy.restype = i
    lib.og_path_used.argtypes = [vp]
    lib.og_path_used.restype = i
    lib.og_workspace_bytes.argtypes = [vp, i, i]
    lib.og_workspace_bytes.restype = sz
    lib.og_forward.argtypes = [vp, i, i, d, vp, vp, vp, vp, sz, vp]
    lib.og_forward.restype = i
    lib.og_cost.argtypes = [vp, vp, vp, vp]
    lib.og_cost.restype = i
    lib.og_adjoint.argtypes = [vp, vp, vp]
    lib.og_adjoint.restype = i
    lib.og_gradient.argtypes = [vp, vp, vp]
    lib.og_gradient.restype = i
    lib.og_profile.argtypes = [vp, i]
    lib.og_profile.restype = i
    lib.og_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_long)]
    lib.og_profile_read.restype = i
    lib.og_gradient_sum.argtypes = [vp, vp, i, vp]
    lib.og_gradient_sum.restype = i
    lib.og_set_penalty.argtypes = [vp, vp, d]
    lib.og_set_penalty.restype = i
    lib.og_set_adaptive.argtypes = [vp, d, d]
    lib.og_set_adaptive.restype = i
    lib.og_adaptive_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_long)]
    lib.og_adaptive_stats.restype = i
    lib.og_set_resident.argtypes = [vp, i]
    lib.og_set_resident.restype = i
    lib.og_evaluate_static.argtypes = [vp, i, i, d, vp, vp, vp, vp, vp, vp]
    lib.og_evaluate_static.restype = i
    lib.og_set_fused.argtypes = [vp, i]
    lib.og_set_fused.restype = i
    lib.og_fused_used.argtypes = [vp]
    lib.og_fused_used.restype = i
    lib.og_generation.argtypes = [vp]
    lib.og_generation.restype = ctypes.c_ulonglong
    lib.og_filter_apply.argtypes = [i, i, i, i, d, d, d, vp, vp, vp]
    lib.og_filter_apply.restype = i
    lib.og_filter_grad.argtypes = [i, i, i, i, d, d, d, i, vp, vp, vp]
    lib.og_filter_grad.restype = i
    lib.og_server_create.argtypes = [ctypes.POINTER(vp), vp, i]
    lib.og_server_create.restype = i
    lib.og_server_submit.argtypes = [vp, ctypes.POINTER(OgRequest), vp]
    lib.og_server_submit.restype = i
    lib.og_server_step.argtypes = [vp, i, vp]
    lib.og_server_step.restype = i
    lib.og_server_active.argtypes = [vp]
    lib.og_server_active.restype = i
    lib.og_server_completed.argtypes = [vp, ctypes.POINTER(ctypes.c_long), i]
    lib.og_server_completed.restype = i
    lib.og_server_destroy.argtypes = [vp]
    lib.og_server_destroy.restype = i
    lib.og_status_string.argtypes = [i]
    lib.og_status_string.restype = ctypes.c_char_p
    lib.og_last_error.argtypes = []
    lib.og_last_error.restype = ctypes.c_char_p
    _LIB = lib
    return lib


def _check(status: int):
    if status != 0:
        detail = _LIB.og_last_error().decode() if _LIB is not None else ""
        raise OgError(status, detail)


def _host_c128(x, shape):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.complex128))
    if a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _stream_ptr(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Problem:
    """One operator set (H0, H_k, c_m, gamma_m) on one GPU.

    Methods mirror the C ABI: forward -> cost -> adjoint -> gradient.  All
    tensors are on the Problem's device; controls are float64 [B, N_t, K],
    states complex128 [B, d, d]."""

    def __init__(self, H0, Hk, c_ops, gammas, *, prec="f64", gmode="grape1", path="auto", n_sub=1,
                 ckpt_stride=0, validate=True, device=None, _banded=None):
        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("opengrape needs a ROCm GPU; no device is visible")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        if _banded is not None:
            self._init_banded(lib, _banded, gammas, prec, gmode, path, n_sub, ckpt_stride, validate)
            return
        H0 = np.asarray(H0)
        d = H0.shape[0]
        Hk = np.asarray(Hk, dtype=np.complex128).reshape(-1, d, d) if len(Hk) else np.zeros((0, d, d), np.complex128)
        c_ops = (np.asarray(c_ops, dtype=np.complex128).reshape(-1, d, d) if len(c_ops)
                 else np.zeros((0, d, d), np.complex128))
        self.d, self.K, self.J = d, Hk.shape[0], c_ops.shape[0]
        self._h0 = _host_c128(H0, (d, d))
        self._hk = np.ascontiguousarray(Hk)
        self._c = np.ascontiguousarray(c_ops)
        self._g = np.ascontiguousarray(np.asarray(gammas, dtype=np.float64).reshape(-1))
        if self._g.shape[0] != self.J:
            raise ValueError("one rate per collapse operator")
        opt = OgOptions()
        lib.og_default_options(ctypes.byref(opt))
        opt.prec, opt.gmode, opt.path = PREC[prec], GMODE[gmode], PATH[path]
        opt.n_sub, opt.ckpt_stride, opt.validate = int(n_sub), int(ckpt_stride), int(bool(validate))
        self.prec, self.gmode, self.n_sub = prec, gmode, int(n_sub)
        ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.og_create(ctypes.byref(ctx), d, self.K, self.J, self._h0.ctypes.data,
                                 self._hk.ctypes.data if self.K else None,
                                 self._c.ctypes.data if self.J else None,
                                 self._g.ctypes.data if self.J else None, ctypes.byref(opt)))
        self._ctx = ctx
        self._lib = lib
        self._keep = {}

    @classmethod
    def from_workload(cls, w, **kw):
        return cls(w.H0, w.Hk, w.c_ops, w.gammas, **kw)

    @classmethod
    def from_banded(cls, offsets, H0_diags, Hk_diags, c_diags, gammas, **kw):
        """Operators in diagonal storage on one offset list (og_create_banded):
        H0_diags [n_diag, d], Hk_diags [K, n_diag, d], c_diags [J, n_diag, d],
        entry [t, i] = operator[i, i + offsets[t]]."""
        return cls(None, None, None, gammas, _banded=(offsets, H0_diags, Hk_diags, c_diags), **kw)

    def _init_banded(self, lib, banded, gammas, prec, gmode, path, n_sub, ckpt_stride, validate):
        offsets, H0d, Hkd, cd = banded
        self._offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.int32).reshape(-1))
        n_diag = self._offs.shape[0]
        self._h0 = np.ascontiguousarray(np.asarray(H0d, dtype=np.complex128))
        if self._h0.ndim != 2 or self._h0.shape[0] != n_diag:
            raise ValueError("H0_diags must be [n_diag, d]")
        d = self._h0.shape[1]
        self._hk = np.ascontiguousarray(np.asarray(Hkd, dtype=np.complex128).reshape(-1, n_diag, d))
        self._c = np.ascontiguousarray(np.asarray(cd, dtype=np.complex128).reshape(-1, n_diag, d))
        self.d, self.K, self.J = d, self._hk.shape[0], self._c.shape[0]
        self._g = np.ascontiguousarray(np.asarray(gammas, dtype=np.float64).reshape(-1))
        if self._g.shape[0] != self.J:
            raise ValueError("one rate per collapse operator")
        opt = OgOptions()
        lib.og_default_options(ctypes.byref(opt))
        opt.prec, opt.gmode, opt.path = PREC[prec], GMODE[gmode], PATH[path]
        opt.n_sub, opt.ckpt_stride, opt.validate = int(n_sub), int(ckpt_stride), int(bool(validate))
        self.prec, self.gmode, self.n_sub = prec, gmode, int(n_sub)
        ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.og_create_banded(ctypes.byref(ctx), d, self.K, self.J, n_diag, self._offs.ctypes.data,
                                        self._h0.ctypes.data, self._hk.ctypes.data if self.K else None,
                                        self._c.ctypes.data if self.J else None,
                                        self._g.ctypes.data if self.J else None, ctypes.byref(opt)))
        self._ctx = ctx
        self._lib = lib
        self._keep = {}

    @property
    def path(self) -> str:
        return PATH_NAMES[self._lib.og_path_used(self._ctx)]

    def workspace_bytes(self, B: int, n_t: int) -> int:
        return int(self._lib.og_workspace_bytes(self._ctx, int(B), int(n_t)))

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.og_destroy(self._ctx)
            self._ctx = None
        self._keep = {}  # the workspace and inputs of the last evaluation

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- C ABI calls -------------------------------------------------------
    def _as_u(self, u):
        if not (isinstance(u, torch.Tensor) and u.is_cuda and u.dtype == torch.float64):
            raise TypeError("u must be a float64 CUDA tensor")
        if u.dim() == 2:
            u = u.unsqueeze(0)
        if u.dim() != 3 or u.shape[2] != self.K:
            raise ValueError(f"u must be [B, N_t, {self.K}]")
        return u.contiguous()

    def _as_states(self, r, B):
        if not (isinstance(r, torch.Tensor) and r.is_cuda and r.dtype == torch.complex128):
            raise TypeError("states must be complex128 CUDA tensors")
        if r.dim() == 2:
            r = r.unsqueeze(0)
        if r.shape[1:] != (self.d, self.d):
            raise ValueError(f"states must be [B, {self.d}, {self.d}]")
        if r.shape[0] == 1 and B > 1:
            r = r.expand(B, self.d, self.d)
        return r.contiguous()

    def forward(self, u, rho0, dt, want_rho_T=False, workspace=None):
        u = self._as_u(u)
        B, n_t = u.shape[0], u.shape[1]
        rho0 = self._as_states(rho0, B)
        need = self.workspace_bytes(B, n_t)
        if workspace is None or workspace.numel() < need:
            old = self._keep.get("ws")
            if old is not None and old.numel() >= need:
                workspace = old  # the previous evaluation's workspace, reused
            else:
                self._keep = {}  # release it before allocating a larger one
                workspace = torch.empty(need, dtype=torch.uint8, device=self.device)
        rhoT = torch.empty((B, self.d, self.d), dtype=torch.complex128, device=self.device) if want_rho_T else None
        self._keep = dict(u=u, rho0=rho0, ws=workspace, B=B, n_t=n_t)
        with torch.cuda.device(self.device):
            _check(self._lib.og_forward(self._ctx, B, n_t, float(dt), u.data_ptr(), rho0.data_ptr(),
                                        rhoT.data_ptr() if rhoT is not None else None,
                                        workspace.data_ptr(), need, _stream_ptr(self.device)))
        return rhoT

    @property
    def generation(self) -> int:
        """Number of forward sweeps run on this Problem (og_generation)."""
        return int(self._lib.og_generation(self._ctx))

    def cost(self, sigma):
        sigma = self._as_states(sigma, 1)[0].contiguous()
        phi = torch.empty(self._keep.get("B", 1), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check(self._lib.og_cost(self._ctx, sigma.data_ptr(), phi.data_ptr(), _stream_ptr(self.device)))
        self._keep["sigma"] = sigma
        return phi

    def adjoint(self, sigma):
        sigma = self._as_states(sigma, 1)[0].contiguous()
        self._keep["sigma_adj"] = sigma
        with torch.cuda.device(self.device):
            _check(self._lib.og_adjoint(self._ctx, sigma.data_ptr(), _stream_ptr(self.device)))

    def gradient(self):
        B, n_t = self._keep.get("B", 1), self._keep.get("n_t", 1)
        g = torch.empty((B, n_t, self.K), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check(self._lib.og_gradient(self._ctx, g.data_ptr(), _stream_ptr(self.device)))
        return g

    def profile(self, every: int):
        """Sample one right-hand-side kernel launch in `every` with HIP events (0 = off)."""
        _check(self._lib.og_profile(self._ctx, int(every)))

    def profile_read(self):
        """(mean device duration in microseconds, number of samples) of the sampled launches."""
        mean = ctypes.c_double()
        cnt = ctypes.c_long()
        with torch.cuda.device(self.device):
            _check(self._lib.og_profile_read(self._ctx, ctypes.byref(mean), ctypes.byref(cnt)))
        return mean.value, cnt.value

    def cost_and_grad(self, u, rho0, sigma, dt, workspace=None):
        """Phi[b] and dPhi/du[b] for a batch of control arrays."""
        self.forward(u, rho0, dt, workspace=workspace)
        phi = self.cost(sigma)
        self.adjoint(sigma)
        return phi, self.gradient()

    def evaluate_static(self, u, rho0, sigma, dt):
        """Phi[b] and dPhi/du[b] like cost_and_grad, with the library's static
        workspace (og_evaluate_static: no device allocation by the library,
        no synchronisation).  The output tensors are allocated here by torch;
        callers that cannot allocate call the C ABI with their own buffers."""
        u = self._as_u(u)
        B, n_t = u.shape[0], u.shape[1]
        rho0 = self._as_states(rho0, B)
        sigma = self._as_states(sigma, 1)[0].contiguous()
        phi = torch.empty(B, dtype=torch.float64, device=self.device)
        g = torch.empty((B, n_t, self.K), dtype=torch.float64, device=self.device)
        self._keep = dict(u=u, rho0=rho0, sigma=sigma, B=B, n_t=n_t)
        with torch.cuda.device(self.device):
            _check(self._lib.og_evaluate_static(self._ctx, B, n_t, float(dt), u.data_ptr(), rho0.data_ptr(),
                                                sigma.data_ptr(), phi.data_ptr(), g.data_ptr(),
                                                _stream_ptr(self.device)))
        return phi, g

    def gradient_sum(self, out=None):
        """sum_b dPhi_b/du (multi-state index, Eq. (22)); adds into `out` if given."""
        n_t = self._keep.get("n_t", 1)
        acc = out is not None
        if out is None:
            out = torch.empty((n_t, self.K), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check(self._lib.og_gradient_sum(self._ctx, out.data_ptr(), int(acc), _stream_ptr(self.device)))
        return out

    def set_adaptive(self, rtol, atol=0.0):
        """Adaptive Dormand-Prince 5(4) steps with the given tolerances
        (rtol = 0: fixed RK4 steps again).  Query workspace_bytes afterwards."""
        with torch.cuda.device(self.device):
            _check(self._lib.og_set_adaptive(self._ctx, float(rtol), float(atol)))

    def set_resident(self, n_slices):
        """Keep the states of the last n_slices slices of the forward sweep
        in the workspace (no checkpoint recompute for them; 0: none).
        Query workspace_bytes afterwards."""
        with torch.cuda.device(self.device):
            _check(self._lib.og_set_resident(self._ctx, int(n_slices)))

    def set_fused(self, enable: bool):
        """Fused RK4 steps (four stages per launch) where the operator
        structure allows (default on), or always the four stage kernels."""
        _check(self._lib.og_set_fused(self._ctx, int(bool(enable))))

    @property
    def fused(self) -> bool:
        """True when the fixed RK4 steps of this Problem run fused."""
        return bool(self._lib.og_fused_used(self._ctx))

    def resident_for_budget(self, B, n_t, budget_bytes):
        """A number of resident slices (up to n_t) whose workspace fits in
        budget_bytes, 0 when none fits; leaves the setting at 0.  The
        workspace grows with the resident count except near n_t, where the
        checkpoints it replaces can outweigh packed resident states: n_t
        itself is tried first, then the largest count found by bisection."""
        def ws(r):
            self.set_resident(r)
            return self.workspace_bytes(B, n_t)
        lo, hi = 0, int(n_t)
        if ws(hi) <= budget_bytes:
            lo = hi
        elif ws(0) > budget_bytes:
            lo = 0
        else:
            while lo < hi:  # ws(lo) <= budget throughout
                mid = (lo + hi + 1) // 2
                if ws(mid) <= budget_bytes:
                    lo = mid
                else:
                    hi = mid - 1
        self.set_resident(0)
        return lo

    def adaptive_stats(self, B):
        """[B, 4] numpy int64: accepted / rejected steps of the forward and
        adjoint sweeps of the last evaluation."""
        out = np.zeros((int(B), 4), dtype=np.int64)
        with torch.cuda.device(self.device):
            _check(self._lib.og_adaptive_stats(self._ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_long))))
        return out

    def set_penalty(self, A, beta):
        """Phi -= beta dt sum_n Tr(A rho_n) (Eqs. (24)-(25)); beta = 0 removes it."""
        a = None if A is None else _host_c128(A, (self.d, self.d))
        with torch.cuda.device(self.device):
            _check(self._lib.og_set_penalty(self._ctx, None if a is None else a.ctypes.data, float(beta)))


def filter_apply(u, N, M, dtu, dts, omega0):
    """Subpixel controls s = T u of the Gaussian filter (App. A); u [B, N, K] float64 CUDA."""
    lib = load_library()
    u = u.contiguous()
    B, K = (u.shape[0], u.shape[2]) if u.dim() == 3 else (1, u.shape[1])
    s = torch.empty((B, M, K), dtype=torch.float64, device=u.device)
    with torch.cuda.device(u.device):
        _check(lib.og_filter_apply(B, N, M, K, float(dtu), float(dts), float(omega0), u.data_ptr(), s.data_ptr(),
                                   _stream_ptr(u.device)))
    return s if u.dim() == 3 else s[0]


def filter_grad(g_s, N, M, dtu, dts, omega0, fix_ends=True):
    """Chain rule dPhi/du = T^T dPhi/ds (Eq. (A2)); first / last control held fixed."""
    lib = load_library()
    g_s = g_s.contiguous()
    B, K = (g_s.shape[0], g_s.shape[2]) if g_s.dim() == 3 else (1, g_s.shape[1])
    g_u = torch.empty((B, N, K), dtype=torch.float64, device=g_s.device)
    with torch.cuda.device(g_s.device):
        _check(lib.og_filter_grad(B, N, M, K, float(dtu), float(dts), float(omega0), int(bool(fix_ends)),
                                  g_s.data_ptr(), g_u.data_ptr(), _stream_ptr(g_s.device)))
    return g_u if g_s.dim() == 3 else g_u[0]


class OpenGrapeCost(torch.autograd.Function):
    """Phi(u) = Tr(sigma rho_T(u)) as a differentiable torch function.

    forward: og_forward + og_cost; backward: og_adjoint + og_gradient, which
    must run in the exact mode (the first-order Eq. (13) gradient is not the
    derivative of the computed Phi).  The workspace of a Problem holds the
    states of its last forward sweep only: when another application of the
    same Problem ran a forward sweep in between (og_generation changed),
    backward runs this application's forward sweep again before the adjoint,
    so every application gets its own gradient."""

    @staticmethod
    def forward(ctx, u, problem, rho0, sigma, dt):
        if problem.gmode != "exact":
            raise ValueError("OpenGrapeCost needs a Problem created with gmode='exact'")
        u_in = u.detach()
        problem.forward(u_in, rho0, dt)
        phi = problem.cost(sigma)
        ctx.problem = problem
        ctx.sigma = sigma
        ctx.inputs = (u_in, rho0, dt)
        ctx.generation = problem.generation
        ctx.squeeze = u.dim() == 2
        return phi[0] if ctx.squeeze else phi

    @staticmethod
    def backward(ctx, gphi):
        if ctx.problem.generation != ctx.generation:
            u_in, rho0, dt = ctx.inputs
            ctx.problem.forward(u_in, rho0, dt)
        ctx.problem.adjoint(ctx.sigma)
        g = ctx.problem.gradient()
        if ctx.squeeze:
            return gphi * g[0], None, None, None, None
        return gphi[:, None, None] * g, None, None, None, None


def open_grape_cost(u, problem, rho0, sigma, dt):
    return OpenGrapeCost.apply(u, problem, rho0, sigma, dt)


class Server:
    """Continuous-batching front end of og_server_* for one Problem (banded
    path, first-order gradient).  Each admitted request owns its inputs, its
    outputs and its workspace (a torch allocation, so the HBM budget is the
    caller's); they are kept alive here until the request is retired."""

    def __init__(self, problem: Problem, max_active: int = 1024):
        self.problem = problem
        self._lib = problem._lib
        srv = ctypes.c_void_p()
        _check(self._lib.og_server_create(ctypes.byref(srv), problem._ctx, int(max_active)))
        self._srv = srv
        self._live = {}
        self.max_active = max_active

    def request_bytes(self, n_t: int) -> int:
        """Device bytes a request of n_t slices holds while in flight."""
        p = self.problem
        return p.workspace_bytes(1, n_t) + 8 * (n_t * p.K + 1)

    def submit(self, tag: int, u, rho0, sigma, dt: float):
        """Admit one request; u [N_t, K] float64, rho0 / sigma [d, d]
        complex128, all on the problem's device.  Returns False when the
        server is full."""
        p = self.problem
        u = u.contiguous()
        n_t = u.shape[0]
        ws_bytes = p.workspace_bytes(1, n_t)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=p.device)
        phi = torch.empty(1, dtype=torch.float64, device=p.device)
        grad = torch.empty((n_t, p.K), dtype=torch.float64, device=p.device)
        req = OgRequest(n_t, float(dt), u.data_ptr(), rho0.data_ptr(), sigma.data_ptr(), phi.data_ptr(),
                        grad.data_ptr(), ws.data_ptr(), ws_bytes, int(tag))
        with torch.cuda.device(p.device):
            st = self._lib.og_server_submit(self._srv, ctypes.byref(req), _stream_ptr(p.device))
        if st == -5 and b"server full" in self._lib.og_last_error():
            return False
        _check(st)
        self._live[int(tag)] = dict(u=u, rho0=rho0, sigma=sigma, ws=ws, phi=phi, grad=grad, n_t=n_t)
        return True

    def step(self, max_slices: int = 8):
        with torch.cuda.device(self.problem.device):
            _check(self._lib.og_server_step(self._srv, int(max_slices), _stream_ptr(self.problem.device)))

    @property
    def active(self) -> int:
        return int(self._lib.og_server_active(self._srv))

    def completed(self):
        """Retired requests as {tag: (phi tensor, grad tensor)}; valid once the
        work enqueued on the stream has finished."""
        out = {}
        buf = (ctypes.c_long * 256)()
        while True:
            n = self._lib.og_server_completed(self._srv, buf, 256)
            for i in range(n):
                rec = self._live.pop(int(buf[i]))
                out[int(buf[i])] = (rec["phi"], rec["grad"])
            if n < 256:
                return out

    def close(self):
        if getattr(self, "_srv", None):
            self._lib.og_server_destroy(self._srv)
            self._srv = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
