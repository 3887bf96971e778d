"""Python binding of libcopa.so (ctypes). Argument marshalling only: every step of the fit and of
the gradient runs in the library's HIP kernels. PyTorch supplies device memory and the stream.

    plan = Plan.from_cohort(cohort, R=10, l=7)          # packs X, builds smoothing bases
    state = plan.new_state(H0, W0, V0)                   # FP32 device tensors
    rep, Qt = plan.fit(state, iters=20)                  # Algorithm 1, state updated in place
    loss, dH, dV, dW, dS = plan.loss_grad(H, V, W, Qt)   # adjoint of the reconstruction loss
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_int64, c_void_p

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcopa.so")

OK, EINVAL, ENOMEM, EDEVICE, ENUMERIC, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
PROX_NONE, PROX_NONNEG, PROX_L1, PROX_L0, PROX_NONNEG_L1 = 0, 1, 2, 3, 4
PREC_FP32, PREC_MIXED = 0, 1
ORDER_HWV, ORDER_WHV = 0, 1


def _order(order):
    """Block order as copa_order: "HWV" / "WHV" or the integer."""
    if isinstance(order, str):
        return {"HWV": ORDER_HWV, "WHV": ORDER_WHV}[order.upper()]
    return int(order)


# every function declared in include/copa.h
SYMBOLS = ("copa_workspace_bytes", "copa_plan_create", "copa_fit", "copa_mttkrp_last",
           "copa_plan_basis",
           "copa_loss_grad", "copa_plan_destroy", "copa_rank_supported", "copa_status_string",
           "copa_last_error", "copa_set_timing", "copa_read_timing", "copa_kernel_name",
           "copa_plan_query", "copa_set_graph", "copa_stationarity", "copa_loss_grad_static")
NUM_KERNELS = 14


class CopaTensor(ctypes.Structure):
    _fields_ = [("K", c_int64), ("J", c_int64), ("S", c_int64), ("nnz", c_int64),
                ("subj_ptr", c_void_p), ("row_ptr", c_void_p), ("col", c_void_p),
                ("val", c_void_p), ("days", c_void_p), ("l", c_int32), ("basis", c_void_p)]


class CopaOptions(ctypes.Structure):
    _fields_ = [("R", c_int32), ("inner_iters", c_int32), ("prox_H", c_int32),
                ("prox_W", c_int32), ("prox_V", c_int32), ("lambda_H", c_double),
                ("lambda_W", c_double), ("lambda_V", c_double), ("rank_rtol", c_double),
                ("basis_rtol", c_double), ("stop_tol", c_double), ("check_every", c_int32),
                ("precision", c_int32), ("mixed_refine", c_int32), ("deterministic", c_int32),
                ("adjoint", c_int32), ("autotune", c_int32), ("order", c_int32)]


class CopaState(ctypes.Structure):
    _fields_ = [("H", c_void_p), ("W", c_void_p), ("V", c_void_p), ("D_H", c_void_p),
                ("D_W", c_void_p), ("D_V", c_void_p), ("iter", c_int32)]


class CopaReport(ctypes.Structure):
    _fields_ = [("iters_done", c_int32), ("fail_iter", c_int32), ("fit", c_double),
                ("objective", c_double), ("sparsity_V", c_double), ("rank_deficient", c_int64),
                ("fit_history", POINTER(c_double)), ("objective_history", POINTER(c_double)),
                ("stationarity", c_double)]


class CopaError(RuntimeError):
    def __init__(self, status, where, message):
        super().__init__(f"{where}: {status_name(status)}: {message}")
        self.status = status


_lib = None


def lib():
    """Loads libcopa.so (built in-tree by paper_1803_04572_amd.build); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1803_04572_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.copa_workspace_bytes.argtypes = [POINTER(CopaTensor), POINTER(CopaOptions),
                                           POINTER(ctypes.c_size_t)]
        L.copa_plan_create.argtypes = [POINTER(CopaTensor), POINTER(CopaOptions), c_void_p,
                                       ctypes.c_size_t, c_void_p, POINTER(c_void_p)]
        L.copa_fit.argtypes = [c_void_p, POINTER(CopaState), c_int32, c_void_p,
                               POINTER(CopaReport), c_void_p]
        L.copa_mttkrp_last.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
        L.copa_plan_basis.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]
        L.copa_loss_grad.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                     c_void_p, c_void_p, c_void_p, POINTER(c_double), c_void_p]
        L.copa_stationarity.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                        POINTER(c_double), c_void_p]
        L.copa_loss_grad_static.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                            c_void_p, c_void_p, c_void_p, c_void_p,
                                            POINTER(c_double), c_void_p]
        L.copa_plan_destroy.argtypes = [c_void_p]
        L.copa_plan_destroy.restype = None
        L.copa_rank_supported.argtypes = [c_int32]
        L.copa_status_string.argtypes = [c_int32]
        L.copa_status_string.restype = ctypes.c_char_p
        L.copa_last_error.restype = ctypes.c_char_p
        L.copa_set_timing.argtypes = [c_void_p, c_int32]
        L.copa_set_graph.argtypes = [c_void_p, c_int32]
        L.copa_read_timing.argtypes = [c_void_p, POINTER(c_double), POINTER(c_int64)]
        L.copa_kernel_name.argtypes = [c_int32]
        L.copa_plan_query.argtypes = [c_void_p, c_int32, POINTER(c_int64)]
        L.copa_kernel_name.restype = ctypes.c_char_p
        for name in ("copa_loss_grad_static", "copa_workspace_bytes", "copa_plan_create", "copa_fit", "copa_mttkrp_last", "copa_plan_basis",
                     "copa_loss_grad", "copa_rank_supported", "copa_set_timing",
                     "copa_read_timing"):
            getattr(L, name).restype = c_int32
        _lib = L
    return _lib


def status_name(status):
    return lib().copa_status_string(int(status)).decode()


def last_error():
    return lib().copa_last_error().decode()


def _check(status, where):
    if status != OK:
        raise CopaError(status, where, last_error())


def _ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


def _stream():
    import torch
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, device):
    import torch
    return torch.as_tensor(np.ascontiguousarray(t)).to(device=device, dtype=dtype).contiguous()


class Plan:
    """A packed tensor plus fit options on one GPU (copa_plan_create)."""

    def __init__(self, subj_ptr, row_ptr, col, val, days, J, l, R, inner_iters=5,
                 prox=(PROX_NONE, PROX_NONNEG, PROX_L1), lam=(0.0, 0.0, 0.1), rank_rtol=1e-6,
                 basis_rtol=1e-10, stop_tol=0.0, check_every=10, basis=None,
                 precision=PREC_FP32, mixed_refine=1, deterministic=False, adjoint=False,
                 autotune=True, workspace="library", order="HWV"):
        """workspace: "library" (the library allocates it once) or "caller" (a torch uint8
        tensor of copa_workspace_bytes bytes, kept by this object). order: block order of an
        outer iteration, "HWV" (Algorithm 1) or "WHV"."""
        import torch
        K = subj_ptr.numel() - 1
        S = row_ptr.numel() - 1
        self.K, self.J, self.S, self.nnz, self.l, self.R = K, int(J), S, col.numel(), int(l), int(R)
        self.device = subj_ptr.device
        t = CopaTensor(K=K, J=self.J, S=S, nnz=self.nnz, subj_ptr=_ptr(subj_ptr),
                       row_ptr=_ptr(row_ptr), col=_ptr(col), val=_ptr(val),
                       days=_ptr(days) if days is not None else None, l=self.l,
                       basis=_ptr(basis) if basis is not None else None)
        o = CopaOptions(R=self.R, inner_iters=int(inner_iters), prox_H=int(prox[0]),
                        prox_W=int(prox[1]), prox_V=int(prox[2]), lambda_H=float(lam[0]),
                        lambda_W=float(lam[1]), lambda_V=float(lam[2]),
                        rank_rtol=float(rank_rtol), basis_rtol=float(basis_rtol),
                        stop_tol=float(stop_tol), check_every=int(check_every),
                        precision=int(precision), mixed_refine=int(mixed_refine),
                        deterministic=int(bool(deterministic)), adjoint=int(bool(adjoint)),
                        autotune=int(bool(autotune)), order=_order(order))
        self._ws = None
        ws_ptr, ws_bytes = None, 0
        if workspace == "caller":
            nb = ctypes.c_size_t(0)
            _check(lib().copa_workspace_bytes(ctypes.byref(t), ctypes.byref(o), ctypes.byref(nb)),
                   "copa_workspace_bytes")
            self._ws = torch.empty(max(1, nb.value), dtype=torch.uint8, device=self.device)
            ws_ptr, ws_bytes = c_void_p(self._ws.data_ptr()), nb.value
        elif workspace != "library":
            raise ValueError("workspace must be 'library' or 'caller'")
        h = c_void_p()
        _check(lib().copa_plan_create(ctypes.byref(t), ctypes.byref(o), ws_ptr, ws_bytes,
                                      _stream(), ctypes.byref(h)), "copa_plan_create")
        self._h = h

    @staticmethod
    def workspace_bytes(K, J, S, nnz, l, R, **opts):
        """copa_workspace_bytes for these shapes (no device memory is read)."""
        t = CopaTensor(K=K, J=J, S=S, nnz=nnz, l=l)
        o = CopaOptions(R=R, inner_iters=int(opts.get("inner_iters", 5)), prox_H=0, prox_W=1,
                        prox_V=2, lambda_V=0.1, precision=int(opts.get("precision", PREC_FP32)),
                        mixed_refine=int(opts.get("mixed_refine", 1)),
                        deterministic=int(bool(opts.get("deterministic", False))),
                        adjoint=int(bool(opts.get("adjoint", False))),
                        stop_tol=float(opts.get("stop_tol", 0.0)),
                        order=_order(opts.get("order", "HWV")))
        nb = ctypes.c_size_t(0)
        _check(lib().copa_workspace_bytes(ctypes.byref(t), ctypes.byref(o), ctypes.byref(nb)),
               "copa_workspace_bytes")
        return nb.value

    @classmethod
    def from_cohort(cls, coh, R, l, device="cuda", basis=None, **kw):
        """basis: optional host array (S x l) of the caller's basis rows M_k (instead of the
        spline basis at the visit days)."""
        import torch
        if basis is not None:
            kw["basis"] = _dev(np.asarray(basis, dtype=np.float64).reshape(coh.S, l),
                               torch.float64, device)
        return cls(_dev(coh.subj_ptr, torch.int64, device), _dev(coh.row_ptr, torch.int64, device),
                   _dev(coh.col, torch.int32, device), _dev(coh.val, torch.float32, device),
                   _dev(coh.days, torch.float64, device) if l > 0 and basis is None else None,
                   coh.J, l, R, **kw)

    def new_state(self, H0, W0, V0, D=None):
        """A fresh fit state (FP32 device tensors, duals zero unless given; "iter" = 0)."""
        import torch
        f = lambda a: _dev(a, torch.float32, self.device)  # noqa: E731
        st = {"H": f(H0), "W": f(W0), "V": f(V0)}
        if D is None:
            st.update(D_H=torch.zeros_like(st["H"]), D_W=torch.zeros_like(st["W"]),
                      D_V=torch.zeros_like(st["V"]))
        else:
            st.update(D_H=f(D[0]), D_W=f(D[1]), D_V=f(D[2]))
        st["iter"] = 0
        return st

    def fit(self, state, iters, qtilde=True, fresh=False):
        """Runs `iters` outer iterations (copa_fit) and advances state["iter"]; fresh=True (or
        state["iter"] == 0) marks the state as a new starting point. Returns (report dict,
        Qtilde or None). Raises CopaError on failure (the report is attached as `.report`)."""
        import torch
        for name, shape in (("H", (self.R, self.R)), ("W", (self.K, self.R)),
                            ("V", (self.J, self.R))):
            for key in (name, "D_" + name):
                t = state[key]
                if t.dtype != torch.float32 or not t.is_contiguous() or tuple(t.shape) != shape \
                        or t.device != self.device:
                    raise ValueError(f"state[{key}] must be contiguous float32 {shape} on "
                                     f"{self.device}")
        st = CopaState(**{k: _ptr(state[k]) for k in ("H", "W", "V", "D_H", "D_W", "D_V")},
                       iter=0 if fresh else int(state.get("iter", 0)))
        Qt = torch.empty((self.S, self.R), dtype=torch.float32, device=self.device) \
            if qtilde else None
        fh = (c_double * max(1, iters))()
        oh = (c_double * max(1, iters))()
        rep = CopaReport(fit_history=ctypes.cast(fh, POINTER(c_double)),
                         objective_history=ctypes.cast(oh, POINTER(c_double)))
        status = lib().copa_fit(self._h, ctypes.byref(st), int(iters), _ptr(Qt),
                                ctypes.byref(rep), _stream())
        state["iter"] = int(st.iter)
        out = dict(iters_done=rep.iters_done, fail_iter=rep.fail_iter, fit=rep.fit,
                   objective=rep.objective, sparsity_V=rep.sparsity_V,
                   rank_deficient=rep.rank_deficient, stationarity=rep.stationarity,
                   fit_history=list(fh)[:rep.iters_done],
                   objective_history=list(oh)[:rep.iters_done])
        if status != OK:
            err = CopaError(status, "copa_fit", last_error())
            err.report = out
            raise err
        return out, Qt

    def mttkrp_last(self):
        import torch
        FH = torch.empty((self.R, self.R), dtype=torch.float32, device=self.device)
        FW = torch.empty((self.K, self.R), dtype=torch.float32, device=self.device)
        FV = torch.empty((self.J, self.R), dtype=torch.float32, device=self.device)
        _check(lib().copa_mttkrp_last(self._h, _ptr(FH), _ptr(FW), _ptr(FV), _stream()),
               "copa_mttkrp_last")
        return FH, FW, FV

    def basis(self):
        import torch
        C = torch.empty((self.S, self.l), dtype=torch.float32, device=self.device)
        rk = torch.empty((self.K,), dtype=torch.int32, device=self.device)
        _check(lib().copa_plan_basis(self._h, _ptr(C), _ptr(rk), _stream()), "copa_plan_basis")
        return C, rk

    def loss_grad(self, H, V, W, Qt, want_dS=False):
        import torch
        dH, dV, dW = torch.empty_like(H), torch.empty_like(V), torch.empty_like(W)
        dS = torch.empty((self.K, self.R, self.R), dtype=torch.float32, device=self.device) \
            if want_dS else None
        loss = c_double()
        _check(lib().copa_loss_grad(self._h, _ptr(H), _ptr(V), _ptr(W), _ptr(Qt), _ptr(dH),
                                    _ptr(dV), _ptr(dW), _ptr(dS), ctypes.byref(loss), _stream()),
               "copa_loss_grad")
        return loss.value, dH, dV, dW, dS

    def loss_grad_static(self, H, V, W, Qt, want_dS=False):
        """copa_loss_grad_static: copa_loss_grad without any device allocation (the library's
        static 64 MiB work array); same return values as loss_grad."""
        import torch
        dH, dV, dW = torch.empty_like(H), torch.empty_like(V), torch.empty_like(W)
        dS = torch.empty((self.K, self.R, self.R), dtype=torch.float32, device=self.device) \
            if want_dS else None
        loss = c_double()
        _check(lib().copa_loss_grad_static(self._h, _ptr(H), _ptr(V), _ptr(W), _ptr(Qt),
                                           _ptr(dH), _ptr(dV), _ptr(dW), _ptr(dS),
                                           ctypes.byref(loss), _stream()),
               "copa_loss_grad_static")
        return loss.value, dH, dV, dW, dS

    def stationarity(self, H, V, W, Qt):
        """(r_H, r_W, r_V): stationarity residual of each factor block (copa_stationarity)."""
        res = (c_double * 3)()
        _check(lib().copa_stationarity(self._h, _ptr(H), _ptr(V), _ptr(W), _ptr(Qt), res,
                                       _stream()), "copa_stationarity")
        return tuple(res)

    def query(self, what):
        """Plan layout facts: 'compact' (pass 1 reads the lossless 4-byte nonzeros), 'chunks'
        (pass-2 chunks), 'waves' (pass-1 wave entries), 'pairs' (projected (subject, feature)
        pairs the passes stream; 0 when they stream nonzeros and basis rows)."""
        code = {"compact": 0, "chunks": 1, "waves": 2, "pairs": 3, "tuned": 4,
                "pass1_blocks_per_cu": 5, "procrustes_variant": 6, "gram_blocks": 7,
                "pass2_blocks": 8, "wfirst_blocks": 9, "mrows_blocks": 10}[what]
        out = c_int64(0)
        _check(lib().copa_plan_query(self._h, code, ctypes.byref(out)), "copa_plan_query")
        return int(out.value)

    def set_graph(self, enable=True):
        """Replay outer iterations from a captured hipGraph (default) or launch kernel by kernel."""
        _check(lib().copa_set_graph(self._h, int(bool(enable))), "copa_set_graph")

    def set_timing(self, enable=True):
        _check(lib().copa_set_timing(self._h, int(bool(enable))), "copa_set_timing")

    def read_timing(self):
        """{kernel name: (summed ms, launches)} since the previous read."""
        ms = (c_double * NUM_KERNELS)()
        n = (c_int64 * NUM_KERNELS)()
        _check(lib().copa_read_timing(self._h, ms, n), "copa_read_timing")
        return {lib().copa_kernel_name(i).decode(): (ms[i], n[i]) for i in range(NUM_KERNELS)}

    def close(self):
        if getattr(self, "_h", None):
            lib().copa_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _make_loss_fn():
    import torch

    class CopaLoss(torch.autograd.Function):
        """L(H, V, W) = 1/2 sum_k ||X_k - Qtilde_k H diag(W_k) V^T||^2 with Qtilde fixed; the
        backward pass returns the hand-written adjoint computed by copa_loss_grad."""

        @staticmethod
        def forward(ctx, H, V, W, plan, Qt):
            loss, dH, dV, dW, _ = plan.loss_grad(H.detach().contiguous(), V.detach().contiguous(),
                                                 W.detach().contiguous(), Qt)
            ctx.save_for_backward(dH, dV, dW)
            return torch.tensor(loss, dtype=torch.float64, device=H.device)

        @staticmethod
        def backward(ctx, g):
            dH, dV, dW = ctx.saved_tensors
            s = g.to(torch.float32)
            return dH * s, dV * s, dW * s, None, None

    return CopaLoss


_loss_cls = None


def copa_loss(H, V, W, plan, Qt):
    global _loss_cls
    if _loss_cls is None:
        _loss_cls = _make_loss_fn()
    return _loss_cls.apply(H, V, W, plan, Qt)
