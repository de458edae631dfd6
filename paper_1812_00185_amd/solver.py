"""Thin Python front end of the CGP HIP library.

torch is used only for device memory (the workspace and the field tensors) and
for the current HIP stream; every step of the method runs in the library's
kernels.  Methods mirror the C-ABI entry points one to one.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _native as N


def _ptr(t, dtype=None, numel=None, name="tensor"):
    """Device pointer of a contiguous tensor, after checking it (marshalling only)."""
    import torch

    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


class CGP:
    """One CGP problem (coarse mesh + k refinements) resident on one GPU."""

    def __init__(self, coarse_mesh: dict, levels: int, dt: float, nu: float, chi: int = 0,
                 precision: str = "fp64", restrict: str = "galerkin", pcg_tol: float = 1e-8,
                 inner_tol: float = 1e-5, mom_tol: float = 1e-12, mass_tol: float = 1e-12,
                 max_iter: int = 20000, mom_max_iter: int = 1000, mass_max_iter: int = 1000,
                 max_outer: int = 20, mass: str = "consistent", precond: str = "jacobi",
                 scheme: str = "incremental", device="cuda:0"):
        import torch

        self.lib = N.load()
        self.device = torch.device(device)
        xy = np.ascontiguousarray(coarse_mesh["xy"], np.float64)
        tri = np.ascontiguousarray(coarse_mesh["tri"], np.int32)
        bedge = np.ascontiguousarray(coarse_mesh["bedge"], np.int32)
        btag = np.ascontiguousarray(coarse_mesh["btag"], np.int32)
        self._host = (xy, tri, bedge, btag)
        mesh = N.Mesh(xy.shape[0], tri.shape[0], btag.shape[0],
                      xy.ctypes.data_as(C.POINTER(C.c_double)),
                      tri.ctypes.data_as(C.POINTER(C.c_int32)),
                      bedge.ctypes.data_as(C.POINTER(C.c_int32)),
                      btag.ctypes.data_as(C.POINTER(C.c_int32)))
        prec = {"fp64": N.CGP_FP64, "mixed": N.CGP_MIXED}[precision]
        rmode = {"galerkin": N.CGP_RESTRICT_GALERKIN, "inject": N.CGP_RESTRICT_INJECT}[restrict]
        mmode = {"consistent": N.CGP_MASS_CONSISTENT, "lumped_p": N.CGP_MASS_LUMPED_P,
                 "lumped": N.CGP_MASS_LUMPED, "mixed": N.CGP_MASS_CONSISTENT_MIXED}[mass]
        pmode = {"jacobi": N.CGP_PRECOND_JACOBI, "ndchol": N.CGP_PRECOND_NDCHOL,
                 "jacobi_s4": N.CGP_PRECOND_JACOBI_S4}[precond]
        smode = {"incremental": N.CGP_SCHEME_INCREMENTAL,
                 "nonincremental": N.CGP_SCHEME_NONINCREMENTAL}[scheme]
        self.problem = N.Problem(mesh, levels, chi, prec, rmode, dt, nu, pcg_tol, inner_tol,
                                 mom_tol, mass_tol, max_iter, mom_max_iter, mass_max_iter,
                                 max_outer, mmode, pmode, smode)
        ctx = C.c_void_p()
        N.check(self.lib.cgp_create(C.byref(self.problem), C.byref(ctx)))
        self.ctx = ctx
        sz = N.Sizes()
        N.check(self.lib.cgp_query(self.ctx, C.byref(sz)))
        self.sizes = sz
        nd = N.NdcholInfo()
        N.check(self.lib.cgp_query_ndchol(self.ctx, C.byref(nd)))
        self.ndchol = nd.as_dict()
        self.nf, self.nc = int(sz.n_fine), int(sz.n_coarse)
        self.ndir = int(sz.n_dirichlet)
        xyf = np.empty(2 * self.nf)
        N.check(self.lib.cgp_fine_nodes(self.ctx, xyf.ctypes.data_as(C.POINTER(C.c_double))))
        self.fine_xy = xyf.reshape(-1, 2)
        dn = np.empty(self.ndir, np.int32)
        N.check(self.lib.cgp_dirichlet_nodes(self.ctx, dn.ctypes.data_as(C.POINTER(C.c_int32))))
        self.dirichlet_nodes = dn
        self.workspace = None
        if self.device.type == "cuda":
            self.assemble()

    # -------------------------------------------------------------- set-up
    def _stream(self):
        import torch

        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def assemble(self):
        import torch

        nbytes = int(self.sizes.workspace_bytes)
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self._raw = raw
        self.workspace = raw[off:off + nbytes]
        # page-locked host memory the solver kernels mirror their flags into
        hbytes = int(self.sizes.host_bytes)
        hraw = torch.empty(hbytes + 64, dtype=torch.uint8, pin_memory=True)
        hoff = (-hraw.data_ptr()) % 64
        self._host_raw = hraw
        self.host_buffer = hraw[hoff:hoff + hbytes]
        N.check(self.lib.cgp_assemble(self.ctx, C.c_void_p(self.workspace.data_ptr()),
                                      nbytes, C.c_void_p(self.host_buffer.data_ptr()), hbytes,
                                      self._stream()))

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.cgp_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- fields
    def zeros(self, *shape):
        import torch

        return torch.zeros(*shape, dtype=torch.float64, device=self.device)

    def to_device(self, a):
        import torch

        return torch.as_tensor(np.ascontiguousarray(a, np.float64), device=self.device)

    # -------------------------------------------------------------- entry points
    def momentum(self, u_prev, u, p, u_dir, f=None, out=None, t_nat=None):
        import torch

        f64 = torch.float64
        out = self.zeros(2, self.nf) if out is None else out
        st = (N.SolveStats * 2)()
        rc = self.lib.cgp_momentum(
            self.ctx, _ptr(u_prev, f64, 2 * self.nf, "u_prev"), _ptr(u, f64, 2 * self.nf, "u"),
            _ptr(p, f64, self.nf, "p"), _ptr(u_dir, f64, 2 * self.ndir, "u_dir"),
            _ptr(f, f64, 2 * self.nf, "f"), _ptr(t_nat, f64, 2 * self.nf, "t_nat"),
            _ptr(out, f64, 2 * self.nf, "u_tilde"), st, self._stream())
        N.check(rc)
        return out, [s.as_dict() for s in st]

    def restrict(self, u_tilde, out=None):
        import torch

        out = self.zeros(self.nc) if out is None else out
        N.check(self.lib.cgp_restrict(self.ctx, _ptr(u_tilde, torch.float64, 2 * self.nf, "u_tilde"),
                                      _ptr(out, torch.float64, self.nc, "b_c"), self._stream()))
        return out

    def pcg_solve(self, b_c, phi_c):
        """Solves in place: phi_c holds the guess on entry and the solution on return."""
        import torch

        st = N.SolveStats()
        rc = self.lib.cgp_pcg_solve(self.ctx, _ptr(b_c, torch.float64, self.nc, "b_c"),
                                    _ptr(phi_c, torch.float64, self.nc, "phi_c"), C.byref(st),
                                    self._stream())
        N.check(rc)
        return st.as_dict()

    def pcg_solve_noalloc(self, b_c, phi_c):
        """pcg_solve through the entry point that allocates nothing (its
        Krylov vectors in the library's per-GPU scratch array)."""
        import torch

        st = N.SolveStats()
        rc = self.lib.cgp_pcg_solve_noalloc(
            self.ctx, _ptr(b_c, torch.float64, self.nc, "b_c"),
            _ptr(phi_c, torch.float64, self.nc, "phi_c"), C.byref(st), self._stream())
        N.check(rc)
        return st.as_dict()

    def prolong(self, phi_c, out=None):
        import torch

        out = self.zeros(self.nf) if out is None else out
        N.check(self.lib.cgp_prolong(self.ctx, _ptr(phi_c, torch.float64, self.nc, "phi_c"),
                                     _ptr(out, torch.float64, self.nf, "phi_f"), self._stream()))
        return out

    def correct(self, u_tilde, phi_f, p_in, u_out=None, p_out=None):
        import torch

        f64 = torch.float64
        u_out = self.zeros(2, self.nf) if u_out is None else u_out
        p_out = self.zeros(self.nf) if p_out is None else p_out
        st = (N.SolveStats * 3)()
        rc = self.lib.cgp_correct(self.ctx, _ptr(u_tilde, f64, 2 * self.nf, "u_tilde"),
                                  _ptr(phi_f, f64, self.nf, "phi_f"), _ptr(p_in, f64, self.nf, "p_in"),
                                  _ptr(u_out, f64, 2 * self.nf, "u_out"),
                                  _ptr(p_out, f64, self.nf, "p_out"), st, self._stream())
        N.check(rc)
        return u_out, p_out, [s.as_dict() for s in st]

    # -------------------------------------------------------------- time stepping
    def new_state(self, U_prev, U, P):
        return StepState(self, U_prev, U, P)

    def step(self, state: "StepState", u_dir, f=None, guess=None, stats=False, theta=None,
             t_nat=None):
        """One CGP step; with `theta` the coarse solve starts from the guarded
        learned guess; t_nat: nodal traction [2, N_f] on the natural edges."""
        import torch

        f64 = torch.float64
        st = N.StepStats() if stats else None
        tn = _ptr(t_nat, f64, 2 * self.nf, "t_nat")
        if theta is not None:
            rc = self.lib.cgp_project_step_net(
                self.ctx, C.byref(state.c), _ptr(u_dir, f64, 2 * self.ndir, "u_dir"),
                _ptr(f, f64, 2 * self.nf, "f"), tn,
                _ptr(theta, torch.float32, N.CGP_NET_PARAMS, "theta"),
                C.byref(st) if st is not None else None, self._stream())
        else:
            rc = self.lib.cgp_project_step(
                self.ctx, C.byref(state.c), _ptr(u_dir, f64, 2 * self.ndir, "u_dir"),
                _ptr(f, f64, 2 * self.nf, "f"), tn, _ptr(guess, f64, self.nc, "guess"),
                C.byref(st) if st is not None else None, self._stream())
        N.check(rc)
        state.sync_from_c()
        return st.as_dict() if st is not None else rc

    # -------------------------------------------------------------- learned guess
    def net_init(self, seed=0):
        """Device FP32 parameter vector, seeded by the library's initialiser."""
        import torch

        host = np.empty(N.CGP_NET_PARAMS, np.float32)
        N.check(self.lib.cgp_net_init(host.ctypes.data_as(C.POINTER(C.c_float)), seed))
        return torch.as_tensor(host, device=self.device)

    def _hist(self, hist):
        import torch

        if len(hist) != 4:
            raise ValueError("hist needs 4 increments, newest first")
        ptrs = [_ptr(h, torch.float64, self.nc, "hist") for h in hist]
        return (C.c_void_p * 4)(*[p.value for p in ptrs])

    def net_guess(self, theta, b_c, hist, out=None):
        import torch

        out = self.zeros(self.nc) if out is None else out
        N.check(self.lib.cgp_net_guess(
            self.ctx, _ptr(theta, torch.float32, N.CGP_NET_PARAMS, "theta"),
            _ptr(b_c, torch.float64, self.nc, "b_c"), self._hist(hist),
            _ptr(out, torch.float64, self.nc, "guess"), self._stream()))
        return out

    def net_grad(self, theta, b_c, hist, target):
        import torch

        grad = torch.empty(N.CGP_NET_PARAMS, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        N.check(self.lib.cgp_net_grad(
            self.ctx, _ptr(theta, torch.float32, N.CGP_NET_PARAMS, "theta"),
            _ptr(b_c, torch.float64, self.nc, "b_c"), self._hist(hist),
            _ptr(target, torch.float64, self.nc, "target"), _ptr(grad), _ptr(loss),
            self._stream()))
        return grad, loss

    def net_train_step(self, theta, m, v, step, lr, b_c, hist, target, loss=None):
        import torch

        f32 = torch.float32
        loss = torch.empty(1, dtype=f32, device=self.device) if loss is None else loss
        N.check(self.lib.cgp_net_train_step(
            self.ctx, _ptr(theta, f32, N.CGP_NET_PARAMS, "theta"),
            _ptr(m, f32, N.CGP_NET_PARAMS, "m"), _ptr(v, f32, N.CGP_NET_PARAMS, "v"),
            int(step), float(lr), _ptr(b_c, torch.float64, self.nc, "b_c"), self._hist(hist),
            _ptr(target, torch.float64, self.nc, "target"), _ptr(loss, f32, 1, "loss"),
            self._stream()))
        return loss

    def extrapolate(self, hist, out=None):
        """The quadratic extrapolation 3 h0 - 3 h1 + h2 of the newest three
        increments (the candidate the network refines)."""
        import torch

        out = self.zeros(self.nc) if out is None else out
        ptrs = [_ptr(h, torch.float64, self.nc, "hist") for h in hist[:3]]
        arr = (C.c_void_p * 3)(*[p.value for p in ptrs])
        N.check(self.lib.cgp_extrapolate(self.ctx, arr, _ptr(out, torch.float64, self.nc, "q"),
                                         self._stream()))
        return out

    def guess_guard(self, b_c, cand, prev, out=None):
        import torch

        f64 = torch.float64
        out = self.zeros(self.nc) if out is None else out
        chose = torch.zeros(1, dtype=torch.int32, device=self.device)
        N.check(self.lib.cgp_guess_guard(
            self.ctx, _ptr(b_c, f64, self.nc, "b_c"), _ptr(cand, f64, self.nc, "cand"),
            _ptr(prev, f64, self.nc, "prev"), _ptr(out, f64, self.nc, "out"),
            _ptr(chose, torch.int32, 1, "chose"), self._stream()))
        return out, chose

    def timing_enable(self, kernel_id: int):
        N.check(self.lib.cgp_timing_enable(self.ctx, kernel_id))

    def timing_read(self):
        ms, n = C.c_double(), C.c_int64()
        N.check(self.lib.cgp_timing_read(self.ctx, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def intermediates(self):
        a, b, c = C.c_void_p(), C.c_void_p(), C.c_void_p()
        N.check(self.lib.cgp_intermediates(self.ctx, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value


class StepState:
    """Device buffers of (U^{n-1}, U^n, P^n, Phi_c history).  The library
    rotates the buffer pointers each step; the tensors follow them."""

    def __init__(self, cgp: CGP, U_prev, U, P):
        self.bufs = {}
        t = [cgp.to_device(U_prev).reshape(2, cgp.nf).contiguous(),
             cgp.to_device(U).reshape(2, cgp.nf).contiguous(),
             cgp.to_device(P).reshape(cgp.nf).contiguous()]
        hist = [cgp.zeros(cgp.nc) for _ in range(4)]
        for x in t + hist:
            self.bufs[x.data_ptr()] = x
        self.c = N.State(t[0].data_ptr(), t[1].data_ptr(), t[2].data_ptr(),
                         (C.c_void_p * 4)(*[h.data_ptr() for h in hist]), 0)
        self.sync_from_c()

    def sync_from_c(self):
        self.U_prev = self.bufs[self.c.u_prev]
        self.U = self.bufs[self.c.u]
        self.P = self.bufs[self.c.p]
        self.phi_hist = [self.bufs[self.c.phi_hist[k]] for k in range(4)]
        self.step = int(self.c.step)
