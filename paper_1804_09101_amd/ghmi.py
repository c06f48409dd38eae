"""Python binding of libghmi.so (the C interface in include/ghmi.h).

Argument marshalling only: every step of the evolution runs in the HIP
library.  PyTorch supplies device memory (float64 CUDA tensors) and the
current HIP stream.  If the library has not been built, importing the
binding's entry points raises -- there is no CPU fallback.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libghmi.so")

GH_ERRORS = {
    -1: "GH_ERR_ARG", -2: "GH_ERR_SHAPE", -3: "GH_ERR_ORDER", -4: "GH_ERR_OOM",
    -5: "GH_ERR_NOT_OUTFLOW", -6: "GH_ERR_NONFINITE", -7: "GH_ERR_DEVICE",
}

# Every symbol declared in include/ghmi.h.
EXPORTS = [
    "gh_create", "gh_destroy", "gh_set_stream", "gh_set_domain", "gh_num_points",
    "gh_set_background", "gh_set_params", "gh_rhs", "gh_step", "gh_constraints",
    "gh_last_error", "gh_grid_coords", "gh_host_operator", "gh_set_timing", "gh_kernel_stats",
    "gh_query", "gh_rhs_vjp", "gh_step_vjp", "gh_constraints_vjp",
    "gh_set_graph", "gh_step_stages", "gh_step_vjp_stages", "gh_step_dp5", "gh_set_angular",
    "gh_filter", "gh_tensor_filter_matrix", "gh_set_interface", "gh_set_gemm_variant",
    "gh_constraints_static", "gh_set_outer_bc", "gh_set_gemm_plan",
]

NUM_GEMM_VARIANTS = 18

KERNEL_KINDS = {"deriv_gemm": 0, "filter_gemm": 1, "radial": 2, "pointwise": 3, "boundary": 4,
                "rk_combine_vjp": 5, "pointwise_vjp": 6, "deriv_gemm_T": 7,
                "angular_transform": 8, "tensor_coupling": 9}


class GHError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{GH_ERRORS.get(code, code)}: {msg}")
        self.code = code


class gh_shell(ctypes.Structure):
    _fields_ = [("instance", ctypes.c_int), ("n_r", ctypes.c_int), ("L", ctypes.c_int),
                ("r_in", ctypes.c_double), ("r_out", ctypes.c_double)]


_lib = None


def load_library(path=LIB_PATH):
    """Load libghmi.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"{path} not found: build it with __graft_entry__.build() "
                      "(paper_1804_09101_amd/_build.py); there is no fallback path")
    lib = ctypes.CDLL(path)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    pd = ctypes.POINTER(ctypes.c_double)
    pll = ctypes.POINTER(ctypes.c_longlong)
    psh = ctypes.POINTER(gh_shell)
    sig = {
        "gh_create": (i, [ctypes.POINTER(vp), i, vp]),
        "gh_destroy": (i, [vp]),
        "gh_set_stream": (i, [vp, vp]),
        "gh_set_domain": (i, [vp, i, i, psh, i, pd]),
        "gh_num_points": (i, [vp, pll, pll]),
        "gh_set_background": (i, [vp, vp, vp, vp]),
        "gh_set_params": (i, [vp, pd, pd]),
        "gh_rhs": (i, [vp, vp, vp]),
        "gh_step": (i, [vp, vp, i]),
        "gh_constraints": (i, [vp, vp, vp, vp]),
        "gh_constraints_static": (i, [vp, vp, vp, vp]),
        "gh_last_error": (ctypes.c_char_p, [vp]),
        "gh_grid_coords": (i, [i, psh, pd]),
        "gh_host_operator": (i, [i, i, pd, pd]),
        "gh_set_timing": (i, [vp, i]),
        "gh_kernel_stats": (i, [vp, i, pll, pd]),
        "gh_query": (i, [vp, i, pll]),
        "gh_rhs_vjp": (i, [vp, vp, vp, vp, vp]),
        "gh_step_vjp": (i, [vp, vp, vp, vp, vp]),
        "gh_constraints_vjp": (i, [vp, vp, vp, vp]),
        "gh_set_graph": (i, [vp, i]),
        "gh_step_stages": (i, [vp, vp, vp, vp, vp]),
        "gh_step_dp5": (i, [vp, vp, i, d, d, vp, vp, vp, vp, vp]),
        "gh_set_angular": (i, [vp, i]),
        "gh_step_vjp_stages": (i, [vp, vp, vp, vp, vp, vp, vp, vp]),
        "gh_filter": (i, [vp, vp, vp]),
        "gh_set_interface": (i, [vp, i]),
        "gh_set_outer_bc": (i, [vp, i]),
        "gh_set_gemm_plan": (i, [vp, i, i, i, i, i, i]),
        "gh_set_gemm_variant": (i, [vp, i, i, i]),
        "gh_tensor_filter_matrix": (i, [i, i, pd, i, pll, pll, ctypes.POINTER(ctypes.c_int), pd]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _shell_array(shells):
    arr = (gh_shell * len(shells))()
    for k, s in enumerate(shells):
        inst, n_r, L, r_in, r_out = s
        arr[k] = gh_shell(int(inst), int(n_r), int(L), float(r_in), float(r_out))
    return arr


def _dptr(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def grid_coords(shells):
    """Cartesian coordinates [3, P] of the collocation points (host-only call)."""
    lib = load_library()
    arr = _shell_array(shells)
    P = sum(int(s[1]) * 2 * (int(s[2]) + 1) ** 2 for s in shells)
    out = np.zeros((3, P))
    rc = lib.gh_grid_coords(len(shells), arr, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc:
        raise GHError(rc, "gh_grid_coords")
    return out


def host_operator(kind, n, params=None):
    """Dense operator as the library builds it (host-only call); see include/ghmi.h."""
    lib = load_library()
    if kind == 0:
        shape = (n, n)
    elif kind in (1, 2, 3, 7):
        S = 2 * (n + 1) ** 2
        shape = (S, S)
    elif kind == 6:
        S = 2 * (n + 1) ** 2
        shape = (S, 2 * S)
    elif kind == 4:
        shape = (n,)
    elif kind == 5:
        shape = (2, n + 1)
    else:
        raise ValueError("unknown operator kind")
    out = np.zeros(shape)
    keep, pp = _dptr(params if params is not None else [0.0, 0.0, 0.0])
    rc = lib.gh_host_operator(kind, n, pp, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc:
        raise GHError(rc, "gh_host_operator")
    return out


def tensor_filter_matrix(L, kind, params, transpose=False):
    """Coupling matrix of the tensor-coupled filter as CSR arrays (row_ptr,
    col, val) from the library's host builder (host-only call); kind 2
    ExpCheb (eta_c, alpha, order), 3 Heaviside (eta_c,); see include/ghmi.h."""
    lib = load_library()
    keep, pp = _dptr(list(params) + [0.0] * (3 - len(params)))
    nnz = ctypes.c_longlong(0)
    rc = lib.gh_tensor_filter_matrix(int(L), int(kind), pp, int(bool(transpose)), ctypes.byref(nnz), None, None, None)
    if rc:
        raise GHError(rc, "gh_tensor_filter_matrix")
    n = 50 * (L + 1) ** 2
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(nnz.value, dtype=np.int32)
    val = np.zeros(nnz.value)
    rc = lib.gh_tensor_filter_matrix(int(L), int(kind), pp, int(bool(transpose)), ctypes.byref(nnz),
                                     row_ptr.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)),
                                     col.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                     val.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc:
        raise GHError(rc, "gh_tensor_filter_matrix")
    return row_ptr, col, val


class GHSolver:
    """One context of the library: a domain, its background and parameters.

    shells: sequence of (instance, n_r, L, r_in, r_out).
    filter_params: None, or the parameters of the angular filter of kind
    filter_kind (1: exponential filter of every component, (eta_c, alpha,
    order); 2: tensor-coupled ExpCheb filter, (eta_c, alpha, order); 3:
    tensor-coupled Heaviside filter, (eta_c,)).
    """

    def __init__(self, shells, n_inst=None, filter_params=None, device=0, filter_kind=1):
        import torch
        self._torch = torch
        self.lib = load_library()
        self.shells = [tuple(s) for s in shells]
        self.n_inst = n_inst if n_inst is not None else 1 + max(int(s[0]) for s in self.shells)
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        rc = self.lib.gh_create(ctypes.byref(h), device, ctypes.c_void_p(self._stream()))
        if rc:
            raise GHError(rc, "gh_create failed (no HIP device?)")
        self.h = h
        arr = _shell_array(self.shells)
        kind = 0 if filter_params is None else int(filter_kind)
        fp = [0.0, 0.0, 0.0] if filter_params is None else list(filter_params) + [0.0] * (3 - len(filter_params))
        self._fp, fpp = _dptr(fp)
        self._check(self.lib.gh_set_domain(self.h, self.n_inst, len(self.shells), arr, kind, fpp))
        tot = ctypes.c_longlong()
        offs = (ctypes.c_longlong * (len(self.shells) + 1))()
        self._check(self.lib.gh_num_points(self.h, ctypes.byref(tot), offs))
        self.P = int(tot.value)
        self.offsets = np.array(list(offs), dtype=np.int64)

    # -- helpers -------------------------------------------------------------
    def _stream(self):
        return self._torch.cuda.current_stream().cuda_stream

    def _check(self, rc):
        if rc:
            msg = self.lib.gh_last_error(self.h)
            raise GHError(rc, msg.decode() if msg else "")

    def _sync_stream(self):
        self._check(self.lib.gh_set_stream(self.h, ctypes.c_void_p(self._stream())))

    def _dev(self, t, ncomp, name):
        torch = self._torch
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
            raise TypeError(f"{name} must be a float64 CUDA tensor")
        if not t.is_contiguous() or t.numel() != ncomp * self.P:
            raise ValueError(f"{name} must be contiguous with {ncomp}*P = {ncomp * self.P} elements")
        return ctypes.c_void_p(t.data_ptr())

    def new_field(self, ncomp=50):
        return self._torch.zeros(ncomp * self.P, dtype=self._torch.float64, device=self.device)

    # -- API ---------------------------------------------------------------------
    def set_background(self, H, dH, u_bg):
        self._sync_stream()
        self._check(self.lib.gh_set_background(self.h, self._dev(H, 4, "H"), self._dev(dH, 16, "dH"),
                                               self._dev(u_bg, 50, "u_bg")))

    def set_params(self, gamma, dt=None):
        g, gp = _dptr(np.asarray(gamma, dtype=float).reshape(self.n_inst, 3))
        if dt is None:
            self._check(self.lib.gh_set_params(self.h, gp, None))
        else:
            d, dp = _dptr(np.asarray(dt, dtype=float).reshape(self.n_inst))
            self._check(self.lib.gh_set_params(self.h, gp, dp))

    def rhs(self, u, out=None):
        out = self.new_field() if out is None else out
        self._sync_stream()
        self._check(self.lib.gh_rhs(self.h, self._dev(u, 50, "u"), self._dev(out, 50, "dudt")))
        return out

    def step(self, u, n_steps=1):
        self._sync_stream()
        self._check(self.lib.gh_step(self.h, self._dev(u, 50, "u"), int(n_steps)))
        return u

    def constraints(self, u, want_C=True):
        torch = self._torch
        C = self.new_field(64) if want_C else None
        norm = torch.zeros(self.n_inst, dtype=torch.float64, device=self.device)
        self._sync_stream()
        self._check(self.lib.gh_constraints(self.h, self._dev(u, 50, "u"),
                                            self._dev(C, 64, "C") if want_C else None,
                                            ctypes.c_void_p(norm.data_ptr())))
        return C, norm

    def constraints_static(self, u, C=None, norm=None):
        """gh_constraints_static: the caller supplies the outputs (C [64 P] or
        None, norm [n_inst] or None); nothing is allocated by the call."""
        self._sync_stream()
        self._check(self.lib.gh_constraints_static(
            self.h, self._dev(u, 50, "u"), self._dev(C, 64, "C") if C is not None else None,
            ctypes.c_void_p(norm.data_ptr()) if norm is not None else None))
        return C, norm

    def set_graph(self, enable=True):
        self._check(self.lib.gh_set_graph(self.h, 1 if enable else 0))

    def set_timing(self, enable=True):
        """True/1: events around every launch; 2: only around the angular
        derivative GEMM; False/0: off."""
        level = 2 if enable == 2 else (1 if enable else 0)
        self._check(self.lib.gh_set_timing(self.h, level))

    def kernel_stats(self, kind):
        """(launches, total_ms) of one kernel kind since timing was enabled or last queried."""
        n = ctypes.c_longlong()
        ms = ctypes.c_double()
        self._check(self.lib.gh_kernel_stats(self.h, KERNEL_KINDS[kind], ctypes.byref(n), ctypes.byref(ms)))
        return int(n.value), float(ms.value)

    def rhs_vjp(self, u, lam, g_gamma=None, out=None):
        """(d rhs/du)^T lam; g_gamma (float64 CUDA [n_inst*3]) is incremented if given."""
        out = self.new_field() if out is None else out
        self._sync_stream()
        g = ctypes.c_void_p(g_gamma.data_ptr()) if g_gamma is not None else None
        self._check(self.lib.gh_rhs_vjp(self.h, self._dev(u, 50, "u"), self._dev(lam, 50, "lam"),
                                        self._dev(out, 50, "lam_u"), g))
        return out

    def step_vjp(self, u_n, lam_np1, g_gamma=None, out=None):
        """(d step/du_n)^T lam_np1; g_gamma incremented if given."""
        out = self.new_field() if out is None else out
        self._sync_stream()
        g = ctypes.c_void_p(g_gamma.data_ptr()) if g_gamma is not None else None
        self._check(self.lib.gh_step_vjp(self.h, self._dev(u_n, 50, "u_n"), self._dev(lam_np1, 50, "lam_np1"),
                                         self._dev(out, 50, "lam_n"), g))
        return out

    def set_gemm_variant(self, plan, shape, order):
        """Pin the kernel variant and tile order of the derivative (plan 0) or
        filter (plan 1) GEMM instead of the autotuner's choice."""
        self._check(self.lib.gh_set_gemm_variant(self.h, int(plan), int(shape), int(order)))

    def set_gemm_plan(self, plan, shape, order, tail_shape=-1, tail_chunks=0, round_tiles=0):
        """Pin any GEMM plan, one launch (tail_shape -1) or split (gh_set_gemm_plan)."""
        self._check(self.lib.gh_set_gemm_plan(self.h, int(plan), int(shape), int(order), int(tail_shape),
                                              int(tail_chunks), int(round_tiles)))

    def set_outer_bc(self, mode):
        """0: Dirichlet outer boundary; 1: constraint-preserving (gh_set_outer_bc)."""
        self._check(self.lib.gh_set_outer_bc(self.h, int(mode)))

    def set_interface(self, mode):
        """0: interface projection from the background (frozen, default); 1: from
        the state at every boundary treatment (no reverse pass in this mode)."""
        self._check(self.lib.gh_set_interface(self.h, int(mode)))

    def filter(self, u, out=None):
        """The domain's angular filter applied once: out = F u (a new field if out is None)."""
        self._sync_stream()
        if out is None:
            out = self.new_field()
        self._check(self.lib.gh_filter(self.h, self._dev(u, 50, "u"), self._dev(out, 50, "out")))
        return out

    def set_angular(self, method):
        """0: dense angular operators (GEMM); 1: factorised by azimuthal order (transforms);
        2: the faster of the two for the derivatives and for the filter, timed on this domain."""
        self._check(self.lib.gh_set_angular(self.h, int(method)))

    def step_dp5(self, u, n_attempts, atol, rtol, t, dt, rejected=None, n_accepted=None, err=None):
        """n_attempts adaptive Dormand-Prince 5(4) attempts in place on u.

        t, dt: float64 CUDA [n_inst] (updated); rejected: int32 CUDA [n_inst]
        (in/out: last attempt rejected); n_accepted: int32 CUDA [n_inst]
        (incremented); err: float64 CUDA [n_inst] (last attempt's error norms).
        """
        torch = self._torch
        for name, x, dtype in (("t", t, torch.float64), ("dt", dt, torch.float64),
                               ("rejected", rejected, torch.int32),
                               ("n_accepted", n_accepted, torch.int32), ("err", err, torch.float64)):
            if x is None and name in ("t", "dt"):
                raise TypeError(f"{name} is required")
            if x is not None and (not x.is_cuda or x.dtype != dtype or x.numel() != self.n_inst
                                  or not x.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor with n_inst elements")
        self._sync_stream()
        ptr = lambda x: ctypes.c_void_p(x.data_ptr()) if x is not None else None
        self._check(self.lib.gh_step_dp5(self.h, self._dev(u, 50, "u"), int(n_attempts), float(atol), float(rtol),
                                         ptr(t), ptr(dt), ptr(rejected), ptr(n_accepted), ptr(err)))
        return u

    def step_stages(self, u, u1, u2, derivs=None):
        """One step in place on u, storing the stage states into u1, u2 and,
        if derivs (float64 CUDA [450 P]) is given, the derivatives of u, u1, u2."""
        self._sync_stream()
        d = self._dev(derivs, 450, "derivs") if derivs is not None else None
        self._check(self.lib.gh_step_stages(self.h, self._dev(u, 50, "u"), self._dev(u1, 50, "u1"),
                                            self._dev(u2, 50, "u2"), d))
        return u

    def step_vjp_stages(self, u_n, u1, u2, lam_np1, g_gamma=None, out=None, derivs=None):
        """step_vjp with the stage states (and optionally their derivatives) from step_stages."""
        out = self.new_field() if out is None else out
        self._sync_stream()
        g = ctypes.c_void_p(g_gamma.data_ptr()) if g_gamma is not None else None
        d = self._dev(derivs, 450, "derivs") if derivs is not None else None
        self._check(self.lib.gh_step_vjp_stages(self.h, self._dev(u_n, 50, "u_n"), self._dev(u1, 50, "u1"),
                                                self._dev(u2, 50, "u2"), d, self._dev(lam_np1, 50, "lam_np1"),
                                                self._dev(out, 50, "lam_n"), g))
        return out

    def constraints_vjp(self, u, lam_norm, out=None):
        """sum_i lam_norm[i] d||C||_i/du (lam_norm: float64 CUDA [n_inst])."""
        out = self.new_field() if out is None else out
        self._sync_stream()
        self._check(self.lib.gh_constraints_vjp(self.h, self._dev(u, 50, "u"), ctypes.c_void_p(lam_norm.data_ptr()),
                                                self._dev(out, 50, "lam_u")))
        return out

    def query(self, what):
        """0: derivative GEMM tile (BM*1000+BN), 1: filter GEMM tile, 2: derivative tiles, 3: points,
        4: derivative GEMM tile order, 5: filter GEMM tile order, 6: derivative GEMM kernel variant,
        7: filter GEMM kernel variant, 8: angular method, 9/10: derivative / filter in transform form."""
        v = ctypes.c_longlong()
        self._check(self.lib.gh_query(self.h, int(what), ctypes.byref(v)))
        return int(v.value)

    def close(self):
        if getattr(self, "h", None):
            self.lib.gh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
