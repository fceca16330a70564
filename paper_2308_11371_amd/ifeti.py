"""Python binding of libifeti (ctypes): argument marshalling only.

Every call goes straight to the C ABI declared in include/ifeti.h; device
arrays are torch float64 tensors on the GPU (their data pointers are passed),
host arrays are numpy.  No arithmetic of the method happens here.  If the
shared library is missing the import fails loudly: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libifeti.so")

IFETI_OK, IFETI_EINVAL, IFETI_ENOMEM, IFETI_ENOTSPD, IFETI_EBREAKDOWN, IFETI_EMAXIT, IFETI_EHIP = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "ENOTSPD", -4: "EBREAKDOWN", -5: "EMAXIT", -6: "EHIP"}
IFETI_FP64, IFETI_FP32_LOCAL, IFETI_BF16_LOCAL = 0, 1, 2

EXPORTED = ("ifeti_create", "ifeti_destroy", "ifeti_last_error", "ifeti_get_sizes", "ifeti_set_options",
            "ifeti_get_options",
            "ifeti_build_cells", "ifeti_get_rhs", "ifeti_build_reduced_basis", "ifeti_get_coefficients",
            "ifeti_apply_F", "ifeti_apply_MD", "ifeti_apply_MD_rom", "ifeti_apply_U", "ifeti_apply_Ut",
            "ifeti_apply_Kinv_rom",
            "ifeti_apply_A", "ifeti_solve_interface", "ifeti_recover_displacement", "ifeti_solve",
            "ifeti_get_stats", "ifeti_reset_stats", "ifeti_compliance_grad", "ifeti_update_widths",
            "ifeti_build_exact", "ifeti_exact_apply_F", "ifeti_exact_apply_MD", "ifeti_exact_solve",
            "ifeti_exact_cell_blocks", "ifeti_cell_displacements", "ifeti_apply_F_noalloc")


class LatticeDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("n_el", ctypes.c_int), ("degree", ctypes.c_int), ("h", ctypes.c_double),
                ("E_in", ctypes.c_double), ("E_out", ctypes.c_double), ("nu", ctypes.c_double),
                ("smooth_eps", ctypes.c_double), ("dirichlet_mask", ctypes.c_int), ("load_face", ctypes.c_int),
                ("u0_grad", ctypes.c_double * 9)]


class Sizes(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("dim", ctypes.c_int), ("n_ctrl", ctypes.c_int), ("n_dof", ctypes.c_int),
                ("n_i", ctypes.c_int), ("n_d", ctypes.c_int), ("n_p", ctypes.c_int), ("n_r", ctypes.c_int),
                ("L", ctypes.c_int), ("L_interface", ctypes.c_int), ("nP", ctypes.c_int),
                ("nU", ctypes.c_longlong), ("K", ctypes.c_int), ("nrhs", ctypes.c_int)]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("pcg_check_every", ctypes.c_int), ("fgmres_restart", ctypes.c_int),
                ("pcg_maxit", ctypes.c_int), ("timing", ctypes.c_int), ("timing_filter", ctypes.c_char * 256),
                ("timing_every", ctypes.c_int), ("use_graph", ctypes.c_int), ("autotune", ctypes.c_int),
                ("coarse_parts", ctypes.c_int), ("true_operator", ctypes.c_int), ("interface_block", ctypes.c_int),
                ("overlap_local", ctypes.c_int), ("local_iters", ctypes.c_int), ("md_precision", ctypes.c_int),
                ("tile_candidate", ctypes.c_int), ("coarse_approx", ctypes.c_int),
                ("block_cg", ctypes.c_int)]

OPTION_NAMES = tuple(name for name, _ in Options._fields_)
# the library's defaults (a new context starts with these)
DEFAULT_OPTIONS = dict(precision=IFETI_FP64, pcg_check_every=2, fgmres_restart=60, pcg_maxit=1000, timing=0,
                       timing_filter="", timing_every=1, use_graph=0, autotune=0, coarse_parts=0, true_operator=0,
                       interface_block=0, overlap_local=0, local_iters=1, md_precision=-1, tile_candidate=-1,
                       coarse_approx=0, block_cg=0)


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_longlong), ("total_ms", ctypes.c_double),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double), ("timed", ctypes.c_longlong)]


OP_NAMES = ("F", "MD", "U", "Ut", "Kinv_rom", "A")


class Stats(ctypes.Structure):
    _fields_ = [("applies", ctypes.c_longlong * 6), ("pcg_iterations", ctypes.c_longlong),
                ("fgmres_iterations", ctypes.c_longlong), ("n_kernels", ctypes.c_int),
                ("kernels", KernelStat * 32)]


class IfetiError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ifeti status {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libifeti.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with `python -m paper_2308_11371_amd.build`")
    lib = ctypes.CDLL(path)
    P, I, D, LL = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong
    lib.ifeti_last_error.restype = ctypes.c_char_p
    sig = {
        "ifeti_create": [ctypes.POINTER(P), ctypes.POINTER(LatticeDesc), P],
        "ifeti_destroy": [P],
        "ifeti_get_sizes": [P, ctypes.POINTER(Sizes)],
        "ifeti_set_options": [P, ctypes.POINTER(Options)],
        "ifeti_get_options": [P, ctypes.POINTER(Options)],
        "ifeti_build_cells": [P, P, P, P, I],
        "ifeti_get_rhs": [P, P, P],
        "ifeti_build_reduced_basis": [P, I, D, P, P, P],
        "ifeti_get_coefficients": [P, P, P, P],
        "ifeti_apply_F": [P, P, P, I],
        "ifeti_apply_F_noalloc": [P, P, P, I],
        "ifeti_apply_MD": [P, P, P, I],
        "ifeti_apply_MD_rom": [P, P, P, I],
        "ifeti_cell_displacements": [P, P, P, I],
        "ifeti_apply_U": [P, P, P, I],
        "ifeti_apply_Ut": [P, P, P, I],
        "ifeti_apply_Kinv_rom": [P, P, P, I],
        "ifeti_apply_A": [P, P, P, I],
        "ifeti_solve_interface": [P, P, P, I, D, I, P, P],
        "ifeti_recover_displacement": [P, P, P, P, I],
        "ifeti_solve": [P, P, P, P, P, I, D, I, D, P, P, P],
        "ifeti_get_stats": [P, ctypes.POINTER(Stats)],
        "ifeti_reset_stats": [P],
        "ifeti_compliance_grad": [P, P, P, P, P, I],
        "ifeti_update_widths": [P, P],
        "ifeti_build_exact": [P],
        "ifeti_exact_apply_F": [P, P, P, I],
        "ifeti_exact_apply_MD": [P, P, P, I],
        "ifeti_exact_solve": [P, P, P, P, P, I, D, I, P, P],
        "ifeti_exact_cell_blocks": [P, I, P, P, P, P, P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = None if name == "ifeti_destroy" else I
    _lib = lib
    return lib


def _ptr(t) -> int:
    """Device pointer of a contiguous float64/int tensor on the GPU."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a GPU torch tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _check(status: int):
    if status not in (IFETI_OK,):
        msg = load().ifeti_last_error().decode()
        raise IfetiError(status, msg)


def desc_from_problem(problem) -> LatticeDesc:
    """LatticeDesc of a latticegen.Problem (Dirichlet data u0(x) = u0_grad x on its Dirichlet faces)."""
    shape = tuple(problem.shape) + (1,) * (3 - len(problem.shape))
    mask = 0
    for f in problem.dirichlet_faces:
        mask |= 1 << f
    g = np.zeros(9)
    dim = problem.dim
    g[:dim * dim] = np.asarray(problem.u0_grad, dtype=np.float64).reshape(dim * dim)
    return LatticeDesc(problem.dim, shape[0], shape[1], shape[2], problem.n_el, problem.degree, problem.h,
                       problem.E_in, problem.E_out, problem.nu, problem.smooth_eps, mask, problem.load_face,
                       (ctypes.c_double * 9)(*g))


class Context:
    """One lattice on one GPU (wraps an ifeti_ctx)."""

    def __init__(self, desc: LatticeDesc, stream=None):
        import torch
        self.lib = load()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        _check(self.lib.ifeti_create(ctypes.byref(h), ctypes.byref(desc), ctypes.c_void_p(stream.cuda_stream)))
        self.h = h
        self.desc = desc

    @classmethod
    def from_problem(cls, problem, stream=None):
        return cls(desc_from_problem(problem), stream)

    def close(self):
        if getattr(self, "h", None):
            self.lib.ifeti_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ info
    @property
    def sizes(self) -> Sizes:
        s = Sizes()
        _check(self.lib.ifeti_get_sizes(self.h, ctypes.byref(s)))
        return s

    def get_options(self) -> dict:
        o = Options()
        _check(self.lib.ifeti_get_options(self.h, ctypes.byref(o)))
        out = {n: getattr(o, n) for n in OPTION_NAMES}
        out["timing_filter"] = o.timing_filter.decode()
        return out

    def set_options(self, **kw):
        """Change the named options (see ifeti_options); every other option keeps its current value."""
        unknown = set(kw) - set(OPTION_NAMES)
        if unknown:
            raise TypeError(f"unknown options {sorted(unknown)}")
        o = Options()
        _check(self.lib.ifeti_get_options(self.h, ctypes.byref(o)))
        for name, value in kw.items():
            if name == "timing_filter":
                value = value.encode()
                if len(value) > 255:
                    raise ValueError("timing_filter: at most 255 characters")
            setattr(o, name, value)
        _check(self.lib.ifeti_set_options(self.h, ctypes.byref(o)))

    def reset_options(self, **kw):
        """Every option back to the library default, then the named ones changed."""
        opts = dict(DEFAULT_OPTIONS)
        opts.update(kw)
        self.set_options(**opts)

    def stats(self) -> dict:
        s = Stats()
        _check(self.lib.ifeti_get_stats(self.h, ctypes.byref(s)))
        kern = {}
        for i in range(s.n_kernels):
            k = s.kernels[i]
            kern[k.name.decode()] = dict(launches=k.launches, timed=k.timed, total_ms=k.total_ms, flops=k.flops,
                                         bytes=k.bytes)
        return dict(applies={n: s.applies[i] for i, n in enumerate(OP_NAMES)}, pcg_iterations=s.pcg_iterations,
                    fgmres_iterations=s.fgmres_iterations, kernels=kern)

    def reset_stats(self):
        _check(self.lib.ifeti_reset_stats(self.h))

    # ------------------------------------------------------------ setup
    def build_cells(self, ctrl_pts, widths, tractions: np.ndarray):
        tr = np.ascontiguousarray(np.atleast_2d(tractions), dtype=np.float64)
        _check(self.lib.ifeti_build_cells(self.h, _ptr(ctrl_pts), _ptr(widths),
                                          tr.ctypes.data_as(ctypes.c_void_p), int(tr.shape[0])))

    def get_rhs(self):
        import torch
        s = self.sizes
        f = torch.empty(s.nrhs * s.nU, dtype=torch.float64, device="cuda")
        d = torch.empty(s.nrhs * s.L, dtype=torch.float64, device="cuda")
        _check(self.lib.ifeti_get_rhs(self.h, _ptr(f), _ptr(d)))
        return f, d

    def build_reduced_basis(self, n_principal: int, tol_rb: float = 1e-12,
                            principal_in: Optional[Sequence[int]] = None, theta_out=None):
        pin = None
        if principal_in is not None:
            pin = np.ascontiguousarray(principal_in, dtype=np.int32)
            n_principal = int(pin.size)
        pout = np.zeros(n_principal, dtype=np.int32)
        _check(self.lib.ifeti_build_reduced_basis(
            self.h, int(n_principal), float(tol_rb),
            pin.ctypes.data_as(ctypes.c_void_p) if pin is not None else None,
            pout.ctypes.data_as(ctypes.c_void_p), _ptr(theta_out) if theta_out is not None else None))
        self.sigma = pout[:self.sizes.K].copy()
        return self.sigma.copy()

    def get_coefficients(self):
        s = self.sizes
        a, p, d = (np.zeros((s.N, s.K)) for _ in range(3))
        _check(self.lib.ifeti_get_coefficients(self.h, a.ctypes.data_as(ctypes.c_void_p),
                                               p.ctypes.data_as(ctypes.c_void_p), d.ctypes.data_as(ctypes.c_void_p)))
        return a, p, d

    # ------------------------------------------------------------ operators
    def _apply(self, fn, x, n_out: int, nrhs: int, out=None):
        import torch
        if out is None:
            out = torch.empty(n_out * nrhs, dtype=torch.float64, device=x.device)
        _check(fn(self.h, _ptr(x), _ptr(out), int(nrhs)))
        return out

    def apply_F(self, lam, nrhs=1, out=None):
        return self._apply(self.lib.ifeti_apply_F, lam, self.sizes.L, nrhs, out)

    def apply_F_noalloc(self, lam, nrhs=1, out=None):
        """F̊ lam by the allocation-free entry point (its output tensor must be given or is made here)."""
        return self._apply(self.lib.ifeti_apply_F_noalloc, lam, self.sizes.L, nrhs, out)

    def apply_MD(self, r, nrhs=1, out=None):
        return self._apply(self.lib.ifeti_apply_MD, r, self.sizes.L, nrhs, out)

    def apply_MD_rom(self, r, nrhs=1, out=None):
        return self._apply(self.lib.ifeti_apply_MD_rom, r, self.sizes.L, nrhs, out)

    def cell_displacements(self, u, nrhs=1, out=None):
        """Per-cell (N, n_dof) view of u per load case (clamped corners zero)."""
        return self._apply(self.lib.ifeti_cell_displacements, u, self.sizes.N * self.sizes.n_dof, nrhs, out)

    def apply_U(self, v, nrhs=1, out=None):
        return self._apply(self.lib.ifeti_apply_U, v, self.sizes.L, nrhs, out)

    def apply_Ut(self, y, nrhs=1, out=None):
        return self._apply(self.lib.ifeti_apply_Ut, y, self.sizes.nU, nrhs, out)

    def apply_Kinv_rom(self, v, nrhs=1, out=None):
        return self._apply(self.lib.ifeti_apply_Kinv_rom, v, self.sizes.nU, nrhs, out)

    def apply_A(self, x, nrhs=1, out=None):
        s = self.sizes
        return self._apply(self.lib.ifeti_apply_A, x, s.nU + s.L, nrhs, out)

    def solve_interface(self, rhs, nrhs=1, tol=1e-11, maxit=1000, lam=None, check=True):
        import torch
        if lam is None:
            lam = torch.empty(self.sizes.L * nrhs, dtype=torch.float64, device=rhs.device)
        its = np.zeros(nrhs, dtype=np.int32)
        rel = np.zeros(nrhs)
        st = self.lib.ifeti_solve_interface(self.h, _ptr(rhs), _ptr(lam), int(nrhs), float(tol), int(maxit),
                                            its.ctypes.data_as(ctypes.c_void_p), rel.ctypes.data_as(ctypes.c_void_p))
        if check:
            _check(st)
        return lam, its, rel, st

    def recover_displacement(self, v, y, nrhs=1, out=None):
        import torch
        if out is None:
            out = torch.empty(self.sizes.nU * nrhs, dtype=torch.float64, device=v.device)
        _check(self.lib.ifeti_recover_displacement(self.h, _ptr(v), _ptr(y), _ptr(out), int(nrhs)))
        return out

    def solve(self, f, d, nrhs=1, tol=1e-8, maxit=60, inner_tol=1e-11, check=True):
        import torch
        s = self.sizes
        u = torch.empty(s.nU * nrhs, dtype=torch.float64, device=f.device)
        lam = torch.empty(s.L * nrhs, dtype=torch.float64, device=f.device)
        outer = np.zeros(nrhs, dtype=np.int32)
        inner = np.zeros(nrhs, dtype=np.int32)
        rel = np.zeros(nrhs)
        st = self.lib.ifeti_solve(self.h, _ptr(f), _ptr(d), _ptr(u), _ptr(lam), int(nrhs), float(tol), int(maxit),
                                  float(inner_tol), outer.ctypes.data_as(ctypes.c_void_p),
                                  inner.ctypes.data_as(ctypes.c_void_p), rel.ctypes.data_as(ctypes.c_void_p))
        if check:
            _check(st)
        return u, lam, dict(outer_its=outer, inner_its=inner, relres=rel, status=st)


def _compliance_grad(self, f, u, nrhs=1):
    """(compliance per load case as numpy, gradient tensor N x nrhs rhs-major)."""
    import torch
    g = torch.empty(self.sizes.N * nrhs, dtype=torch.float64, device=u.device)
    c = np.zeros(nrhs)
    _check(self.lib.ifeti_compliance_grad(self.h, _ptr(f), _ptr(u), _ptr(g), c.ctypes.data_as(ctypes.c_void_p),
                                          int(nrhs)))
    return c, g


def _update_widths(self, widths):
    _check(self.lib.ifeti_update_widths(self.h, _ptr(widths)))


Context.compliance_grad = _compliance_grad
Context.update_widths = _update_widths


# ---------------------------------------------------------------- standard (exact) FETI-DP
def _build_exact(self):
    """Factorise every cell (ifeti_build_exact); the exact operators and solve become available."""
    _check(self.lib.ifeti_build_exact(self.h))


def _exact_apply_F(self, lam, nrhs=1, out=None):
    return self._apply(self.lib.ifeti_exact_apply_F, lam, self.sizes.L, nrhs, out)


def _exact_apply_MD(self, r, nrhs=1, out=None):
    return self._apply(self.lib.ifeti_exact_apply_MD, r, self.sizes.L, nrhs, out)


def _exact_solve(self, f, d, nrhs=1, tol=1e-11, maxit=1000, check=True):
    import torch
    s = self.sizes
    u = torch.empty(s.nU * nrhs, dtype=torch.float64, device=f.device)
    lam = torch.empty(s.L * nrhs, dtype=torch.float64, device=f.device)
    its = np.zeros(nrhs, dtype=np.int32)
    rel = np.zeros(nrhs)
    st = self.lib.ifeti_exact_solve(self.h, _ptr(f), _ptr(d), _ptr(u), _ptr(lam), int(nrhs), float(tol), int(maxit),
                                    its.ctypes.data_as(ctypes.c_void_p), rel.ctypes.data_as(ctypes.c_void_p))
    if check:
        _check(st)
    return u, lam, dict(iters=its, relres=rel, status=st)


def _exact_cell_blocks(self, s):
    """(F_dd, S_dd, S_pp, U_d) of cell s as numpy arrays, and the device bytes of the exact form."""
    z = self.sizes
    F = np.zeros((z.n_d, z.n_d))
    S = np.zeros((z.n_d, z.n_d))
    P = np.zeros((z.n_p, z.n_p))
    U = np.zeros((z.n_d, z.n_p))
    b = ctypes.c_longlong(0)
    vp = ctypes.c_void_p
    _check(self.lib.ifeti_exact_cell_blocks(self.h, int(s), F.ctypes.data_as(vp), S.ctypes.data_as(vp),
                                            P.ctypes.data_as(vp), U.ctypes.data_as(vp), ctypes.byref(b)))
    return F, S, P, U, int(b.value)


Context.build_exact = _build_exact
Context.exact_apply_F = _exact_apply_F
Context.exact_apply_MD = _exact_apply_MD
Context.exact_solve = _exact_solve
Context.exact_cell_blocks = _exact_cell_blocks


def _autograd():
    import torch

    class ComplianceFn(torch.autograd.Function):
        """c(w) = f^T u(w); backward returns -u_s^T dK_s/dw_s u_s from the library (self-adjoint solve)."""

        @staticmethod
        def forward(fctx, widths, lattice, f, d, tol, inner_tol):
            lattice.update_widths(widths.detach().contiguous())
            u, lam, info = lattice.solve(f, d, tol=tol, inner_tol=inner_tol)
            c, g = lattice.compliance_grad(f, u)
            fctx.save_for_backward(g)
            return torch.tensor(c[0], dtype=torch.float64, device=widths.device)

        @staticmethod
        def backward(fctx, gout):
            (g,) = fctx.saved_tensors
            return gout * g, None, None, None, None, None

    return ComplianceFn


def compliance(widths, lattice, f, d, tol=1e-10, inner_tol=1e-11):
    """Differentiable compliance of the lattice for strut widths `widths` (torch, on the GPU)."""
    return _autograd().apply(widths, lattice, f, d, tol, inner_tol)


def setup(problem, n_principal=None, principal_in=None, stream=None) -> Context:
    """Create a context for a latticegen.Problem and run both offline calls."""
    import torch
    ctx = Context.from_problem(problem, stream)
    ctrl = torch.tensor(problem.ctrl, dtype=torch.float64, device="cuda").contiguous()
    w = torch.tensor(problem.widths, dtype=torch.float64, device="cuda")
    ctx.build_cells(ctrl, w, problem.tractions)
    ctx.build_reduced_basis(problem.n_principal if n_principal is None else n_principal,
                            principal_in=principal_in)
    return ctx
