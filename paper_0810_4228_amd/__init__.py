"""Python binding of libovsign (include/ovsign.h): sgn(gamma5 Dw(mu)) b on MI355X.

Argument marshalling only: every step runs in the HIP library.  PyTorch
supplies device memory and the stream; tensors are complex128 on the GPU in
the canonical layouts of the C header:
    links   [V, 4, 3, 3]            (site index x + Lx*(y + Ly*(z + Lz*t)))
    fields  [nrhs, V, 4, 3] or [nrhs, 12*V]

If the compiled library is missing this module raises on first use; there is
no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libovsign.so")

OVS_OK = 0
OVS_WARN_NOT_CONVERGED = 1
OVS_WARN_BREAKDOWN = 2
OVS_WARN_SIGN_AMBIGUOUS = 3
OVS_ERR_ARG = -1
OVS_ERR_HIP = -2
OVS_ERR_ALLOC = -3
OVS_ERR_STATE = -4

OVS_F64 = 0
OVS_F32_STORE = 1
OPS = {"Dw": 0, "Dw_dag": 1, "A": 2, "A_dag": 3}
METHODS = {"2sl": 0, "arnoldi": 1}
OVS_FLAG_TWO_PASS = 1
OVS_FLAG_GRAPH = 4
OVS_FLAG_OVERLAP = 8
OVS_FLAG_NO_SPLIT = 16
OVS_FLAG_PERSISTENT = 32
OVS_VJP_STORE_BASIS = 1
OVS_DEBUG_CHECKS = 1

EXPORTED = [
    "ovs_lattice_create", "ovs_lattice_destroy", "ovs_set_links", "ovs_set_params", "ovs_apply",
    "ovs_field_create", "ovs_field_destroy", "ovs_field_import", "ovs_field_export",
    "ovs_field_apply", "ovs_field_apply_timed", "ovs_dual_apply_timed", "ovs_autotune", "ovs_get_tuning", "ovs_get_tuning_ex", "ovs_set_tuning_ex",
    "ovs_deflation_set", "ovs_deflation_compute", "ovs_deflation_get", "ovs_deflation_destroy", "ovs_workspace_size", "ovs_sign_apply", "ovs_sign_apply_vjp", "ovs_link_force", "ovs_overlap_eigs", "ovs_last_coefficients",
    "ovs_inner_sign_tridiag", "ovs_inner_sign_hessenberg", "ovs_small_eig", "ovs_status_string", "ovs_last_error",
    "ovs_apply_noalloc", "ovs_set_debug", "ovs_workspace_held", "ovs_vjp_workspace_size",
]


class OvsError(RuntimeError):
    def __init__(self, status, what):
        detail = ""
        if status == OVS_ERR_HIP:
            try:
                detail = " [" + load().ovs_last_error().decode() + "]"
            except Exception:
                pass
        super().__init__(f"{what}: {status_string(status)} ({status}){detail}")
        self.status = status


class RhsInfo(ctypes.Structure):
    _fields_ = [
        ("k_used", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("est_rel_err", ctypes.c_double),
        ("quad_err", ctypes.c_double),
        ("n_b", ctypes.c_double),
        ("t_defl_ms", ctypes.c_double),
        ("t_krylov_ms", ctypes.c_double),
        ("t_inner_ms", ctypes.c_double),
        ("t_combine_ms", ctypes.c_double),
        ("fp64", ctypes.c_int32),
        ("escalated", ctypes.c_int32),
        ("min_abs_delta", ctypes.c_double),
        ("biorth_err", ctypes.c_double),
        ("ritz_min_re", ctypes.c_double),
        ("inner_check_err", ctypes.c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def load():
    """Load libovsign.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_0810_4228_amd.build")
    # PyTorch ships its own HIP runtime under the same soname as /opt/rocm's.
    # Loading torch first makes the library bind to that one, so a process
    # holds a single HIP runtime and device pointers and streams are shared.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    IP = ctypes.POINTER(ctypes.c_int32)
    DP = ctypes.POINTER(ctypes.c_double)
    sig = {
        "ovs_lattice_create": [IP, IP, I, P, ctypes.POINTER(P)],
        "ovs_lattice_destroy": [P],
        "ovs_set_links": [P, P, I],
        "ovs_set_params": [P, D, D],
        "ovs_set_debug": [P, I, I],
        "ovs_apply": [P, I, P, P, I],
        "ovs_apply_noalloc": [P, I, P, P, I],
        "ovs_field_create": [P, I, ctypes.POINTER(P)],
        "ovs_field_destroy": [P],
        "ovs_field_import": [P, P],
        "ovs_field_export": [P, P],
        "ovs_field_apply": [P, I, P, P],
        "ovs_field_apply_timed": [P, I, P, P, I, DP],
        "ovs_dual_apply_timed": [P, P, I, DP],
        "ovs_autotune": [P, I],
        "ovs_get_tuning": [P, I, IP, IP],
        "ovs_get_tuning_ex": [P, I, IP],
        "ovs_set_tuning_ex": [P, I, IP],
        "ovs_deflation_set": [P, I, DP, P, P, ctypes.POINTER(P)],
        "ovs_deflation_destroy": [P],
        "ovs_deflation_compute": [P, I, D, I, ctypes.POINTER(P)],
        "ovs_deflation_get": [P, DP, P, P, DP],
        "ovs_sign_apply": [P, P, I, P, P, I, I, DP, I, I, P, ctypes.c_size_t, ctypes.POINTER(RhsInfo)],
        "ovs_workspace_held": [P, ctypes.POINTER(ctypes.c_size_t)],
        "ovs_sign_apply_vjp": [P, P, I, P, P, I, I, I, P, P, DP, P, DP, P, ctypes.c_size_t],
        "ovs_vjp_workspace_size": [P, P, I, I, I, I, ctypes.POINTER(ctypes.c_size_t)],
        "ovs_overlap_eigs": [P, P, I, I, I, I, I, D, I, D, I, DP, P, DP],
        "ovs_link_force": [P, P, P, P],
        "ovs_workspace_size": [P, P, I, I, I, I, I, ctypes.POINTER(ctypes.c_size_t)],
        "ovs_last_coefficients": [P, DP, DP, DP, DP],
        "ovs_inner_sign_tridiag": [P, I, I, DP, DP, DP, DP, DP],
        "ovs_inner_sign_hessenberg": [P, I, I, DP, DP, DP],
        "ovs_small_eig": [I, DP, DP, DP],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int32
    lib.ovs_status_string.argtypes = [ctypes.c_int32]
    lib.ovs_status_string.restype = ctypes.c_char_p
    lib.ovs_last_error.argtypes = []
    lib.ovs_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def status_string(s: int) -> str:
    try:
        return load().ovs_status_string(int(s)).decode()
    except Exception:  # library not loadable: plain code
        return str(s)


def _check(status, what):
    if status < 0:
        raise OvsError(status, what)
    return status


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _torch():
    import torch
    return torch


def _dev_c128(t, what):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError(f"{what} must be a complex128 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return t


def _stream_handle():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Lattice:
    """ovs_lattice handle: geometry, boundary signs, links, m_w and mu."""

    def __init__(self, dims, bc=(1, 1, 1, -1), precision="f64"):
        lib = load()
        self.dims = tuple(int(d) for d in dims)
        self.V = int(np.prod(self.dims))
        self.N = 12 * self.V
        self.precision = precision
        prec = {"f64": OVS_F64, "f32": OVS_F32_STORE}[precision]
        d = (ctypes.c_int32 * 4)(*self.dims)
        b = (ctypes.c_int32 * 4)(*[int(x) for x in bc])
        h = ctypes.c_void_p()
        _check(lib.ovs_lattice_create(d, b, prec, _stream_handle(), ctypes.byref(h)), "ovs_lattice_create")
        self._h = h
        self._lib = lib

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ovs_lattice_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_links(self, U):
        """U: complex128 [V, 4, 3, 3] links, a CUDA tensor or a host numpy array."""
        if isinstance(U, np.ndarray):
            Uh = np.ascontiguousarray(U, dtype=np.complex128)
            if Uh.size != self.V * 36:
                raise ValueError("U must hold V*4*3*3 entries")
            _check(self._lib.ovs_set_links(self._h, Uh.ctypes.data_as(ctypes.c_void_p), 0),
                   "ovs_set_links")
            return
        U = _dev_c128(U, "U")
        if U.numel() != self.V * 36:
            raise ValueError("U must hold V*4*3*3 entries")
        _check(self._lib.ovs_set_links(self._h, ctypes.c_void_p(U.data_ptr()), 1), "ovs_set_links")

    def set_params(self, m_w, mu):
        _check(self._lib.ovs_set_params(self._h, float(m_w), float(mu)), "ovs_set_params")

    def set_debug(self, checks=False, breakdown_at=-1, progress=False, ranges=False):
        """Diagnostics of later sign_apply calls (ovs_set_debug): checks=True
        measures the 2sL biorthogonality and checks the inner sign against a
        dense eigensolve (results in the info records); breakdown_at >= 0
        forces delta = 0 in that iteration's beta step (a serious breakdown);
        progress=True prints the eigentriple solver's progress to stderr;
        ranges=True marks each call and its phases with roctx ranges."""
        flags = (OVS_DEBUG_CHECKS if checks else 0) | (2 if progress else 0) | (4 if ranges else 0)
        _check(self._lib.ovs_set_debug(self._h, flags, int(breakdown_at)), "ovs_set_debug")

    def _fields(self, x):
        x = _dev_c128(x, "x")
        if x.numel() % self.N:
            raise ValueError("field size must be a multiple of 12*V")
        return x, x.numel() // self.N

    def apply(self, op, x, out=None):
        torch = _torch()
        x, nrhs = self._fields(x)
        y = torch.empty_like(x) if out is None else _dev_c128(out, "out")
        _check(self._lib.ovs_apply(self._h, OPS[op], ctypes.c_void_p(x.data_ptr()),
                                   ctypes.c_void_p(y.data_ptr()), nrhs), "ovs_apply")
        return y

    def apply_noalloc(self, op, x, out):
        """y = op x like apply(), through ovs_apply_noalloc: the library's staging
        fields are its fixed per-device scratch (nothing is allocated); out is
        required.  Raises OvsError (OVS_ERR_ARG) when the staging does not fit."""
        x, nrhs = self._fields(x)
        y = _dev_c128(out, "out")
        _check(self._lib.ovs_apply_noalloc(self._h, OPS[op], ctypes.c_void_p(x.data_ptr()),
                                           ctypes.c_void_p(y.data_ptr()), nrhs), "ovs_apply_noalloc")
        return y

    def field_create(self, nrhs):
        return Field(self, nrhs)

    def autotune(self, nrhs):
        _check(self._lib.ovs_autotune(self._h, int(nrhs)), "ovs_autotune")

    def get_tuning(self, nrhs):
        b = ctypes.c_int32()
        w = ctypes.c_int32()
        _check(self._lib.ovs_get_tuning(self._h, int(nrhs), ctypes.byref(b), ctypes.byref(w)), "ovs_get_tuning")
        return b.value, w.value

    def get_tuning_raw(self, nrhs):
        out = (ctypes.c_int32 * 8)()
        _check(self._lib.ovs_get_tuning_ex(self._h, int(nrhs), out), "ovs_get_tuning_ex")
        return list(out)

    def set_tuning_raw(self, nrhs, cfg):
        arr = (ctypes.c_int32 * 8)(*[int(v) for v in cfg])
        _check(self._lib.ovs_set_tuning_ex(self._h, int(nrhs), arr), "ovs_set_tuning_ex")

    def get_tuning_ex(self, nrhs):
        out = (ctypes.c_int32 * 8)()
        _check(self._lib.ovs_get_tuning_ex(self._h, int(nrhs), out), "ovs_get_tuning_ex")
        keys = ("rhs_block", "wg", "lds_kb", "order")
        st = dict(zip(keys, out[0:4]))
        shape = st["rhs_block"]
        st.update(rhs_block=(shape // 100) % 10, lanes_per_site=(shape // 10) % 10,
                  streaming_store=shape % 10, staged_tile=shape // 1000)
        du = dict(zip(keys, out[4:8]))
        shape = du["rhs_block"]
        variants = {1: "one thread per site", 2: "lane pair", 3: "lane pair, LDS-staged tile",
                    4: "operator per workgroup", 5: "operator per workgroup, LDS-staged tile",
                    6: "operator per workgroup, marching along t"}
        du.update(rhs_block=shape // 100, variant=variants.get((shape // 10) % 10, "?"),
                  streaming_store=shape % 2, update_streaming_store=(shape % 10) // 2)
        return {"stencil": st, "dual": du}

    def deflation_set(self, lam, R, L):
        """lam: complex [m] (host); R, L: complex128 CUDA [m, 12V]."""
        lam = np.ascontiguousarray(np.asarray(lam, dtype=np.complex128))
        R = _dev_c128(R, "R")
        L = _dev_c128(L, "L")
        m = lam.shape[0]
        if R.numel() != m * self.N or L.numel() != m * self.N:
            raise ValueError("R and L must be [m, 12V]")
        lam_d = lam.view(np.float64)
        h = ctypes.c_void_p()
        _check(self._lib.ovs_deflation_set(self._h, m, _dptr(lam_d), ctypes.c_void_p(R.data_ptr()),
                                           ctypes.c_void_p(L.data_ptr()), ctypes.byref(h)),
               "ovs_deflation_set")
        return Deflation(self, h, m)

    def deflation_compute(self, m, tol=1e-10, max_iter=30):
        """Critical eigentriples computed on the GPU.  Returns (Deflation, status)."""
        h = ctypes.c_void_p()
        st = _check(self._lib.ovs_deflation_compute(self._h, int(m), float(tol), int(max_iter),
                                                    ctypes.byref(h)), "ovs_deflation_compute")
        return Deflation(self, h, int(m)), st

    def workspace_size(self, nrhs, k_max, defl=None, n_defl=None, method="2sl", two_pass=False,
                       split=True, persistent=False):
        """Bytes of device workspace a sign_apply with these arguments holds."""
        flags = (OVS_FLAG_TWO_PASS if two_pass else 0) | (0 if split else OVS_FLAG_NO_SPLIT) | \
                (OVS_FLAG_PERSISTENT if persistent else 0)
        dh = defl._h if defl is not None else None
        nd = (defl.m if n_defl is None else int(n_defl)) if defl is not None else 0
        out = ctypes.c_size_t()
        _check(self._lib.ovs_workspace_size(self._h, dh, nd, int(nrhs), int(k_max),
                                            METHODS[method], flags, ctypes.byref(out)),
               "ovs_workspace_size")
        return int(out.value)

    def workspace_held(self):
        """Bytes of device memory the handle holds for sign solves (ovs_workspace_held)."""
        out = ctypes.c_size_t()
        _check(self._lib.ovs_workspace_held(self._h, ctypes.byref(out)), "ovs_workspace_held")
        return int(out.value)

    def sign_apply(self, b, k_max, defl=None, n_defl=None, tol=None, method="2sl",
                   two_pass=False, graph=False, overlap=False, out=None, split=True,
                   persistent=False, workspace=None):
        """y = sgn(A) b (or D_ov b with overlap=True).  Returns (y, infos, status).
        split=False keeps a batch of 8 or more sources in one batch;
        persistent=True runs the Lanczos iterations in persistent launches.
        workspace: a CUDA tensor (any dtype, contiguous) the call uses as its
        workspace (at least workspace_size bytes), or None for the handle's own."""
        torch = _torch()
        b, nrhs = self._fields(b)
        y = torch.empty_like(b) if out is None else _dev_c128(out, "out")
        flags = (OVS_FLAG_TWO_PASS if two_pass else 0) | (OVS_FLAG_GRAPH if graph else 0) | \
                (OVS_FLAG_OVERLAP if overlap else 0) | (0 if split else OVS_FLAG_NO_SPLIT) | \
                (OVS_FLAG_PERSISTENT if persistent else 0)
        infos = (RhsInfo * nrhs)()
        tol_arr = None
        tol_p = None
        if tol is not None:
            tol_arr = np.ascontiguousarray(np.broadcast_to(np.asarray(tol, dtype=np.float64), (nrhs,)))
            tol_p = _dptr(tol_arr)
        dh = defl._h if defl is not None else None
        nd = (defl.m if n_defl is None else int(n_defl)) if defl is not None else 0
        ws_p, ws_n = None, 0
        if workspace is not None:
            if not workspace.is_cuda or not workspace.is_contiguous():
                raise ValueError("workspace must be a contiguous CUDA tensor")
            ws_p = ctypes.c_void_p(workspace.data_ptr())
            ws_n = workspace.numel() * workspace.element_size()
        st = self._lib.ovs_sign_apply(self._h, dh, nd, ctypes.c_void_p(b.data_ptr()),
                                      ctypes.c_void_p(y.data_ptr()), nrhs, int(k_max), tol_p,
                                      METHODS[method], flags, ws_p, ctypes.c_size_t(ws_n), infos)
        _check(st, "ovs_sign_apply")
        return y, [i.as_dict() for i in infos], st

    def link_force(self, U, grad_U):
        """su(3) force F = -TA(U grad_U^dagger) per link, [V, 4, 3, 3] complex128 on the
        GPU, for a real function of the links with gradient grad_U (as returned by
        sign_apply_vjp)."""
        torch = _torch()
        U = _dev_c128(U, "U").contiguous()
        G = _dev_c128(grad_U, "grad_U").contiguous()
        if U.numel() != 36 * self.V or G.numel() != 36 * self.V:
            raise ValueError("U and grad_U must hold V*4*3*3 complex entries")
        F = torch.empty((self.V, 4, 3, 3), dtype=torch.complex128, device=U.device)
        _check(self._lib.ovs_link_force(self._h, ctypes.c_void_p(U.data_ptr()),
                                        ctypes.c_void_p(G.data_ptr()),
                                        ctypes.c_void_p(F.data_ptr())), "ovs_link_force")
        return F

    def overlap_eigs(self, nev, ncv=None, block=1, k_inner=400, tol_inner=1e-10, tol=1e-8,
                     max_restarts=100, defl=None, n_defl=None, vectors=False, graph=False):
        """The nev eigenvalues of smallest magnitude of D_ov(mu) = 1 + gamma5 sgn(A)
        by block Arnoldi (block vectors per step, one batched sign solve each:
        two-sided Lanczos, k_inner, tol_inner; graph=True runs its iterations as
        graph replays).  Returns (lambda complex128 [nev] numpy, Ritz vectors
        [nev, V, 4, 3] or None, info dict, status)."""
        torch = _torch()
        block = int(block)
        if ncv is None:  # about 20 blocks per restart cycle, whole blocks
            ncv = max(2 * nev + 8, 20 * block, nev + 2 * block)
            ncv = min(-(-ncv // block) * block, 256 // block * block)
        ncv = int(ncv)
        lam = np.zeros(2 * nev, dtype=np.float64)
        info = np.zeros(4, dtype=np.float64)
        vecs = None
        if vectors:
            vecs = torch.empty((nev,) + tuple(reversed(self.dims)) + (4, 3), dtype=torch.complex128,
                               device="cuda")
        dh = defl._h if defl is not None else None
        nd = (defl.m if n_defl is None else int(n_defl)) if defl is not None else 0
        st = self._lib.ovs_overlap_eigs(self._h, dh, nd, int(nev), ncv, block, int(k_inner),
                                        float(tol_inner), OVS_FLAG_GRAPH if graph else 0,
                                        float(tol), int(max_restarts),
                                        _dptr(lam),
                                        ctypes.c_void_p(vecs.data_ptr()) if vecs is not None else None,
                                        _dptr(info))
        _check(st, "ovs_overlap_eigs")
        lam_c = lam[0::2] + 1j * lam[1::2]
        return lam_c, vecs, {"max_residual": info[0], "restarts": int(info[1]),
                             "sign_solves": int(info[2]), "inner_warnings": int(info[3])}, st

    def vjp_workspace_size(self, nrhs, k, store_basis=False, defl=None, n_defl=None):
        """Bytes of caller workspace a sign_apply_vjp call needs."""
        out = ctypes.c_size_t()
        dh = defl._h if defl is not None else None
        nd = (defl.m if n_defl is None else int(n_defl)) if defl is not None else 0
        _check(self._lib.ovs_vjp_workspace_size(self._h, dh, nd, int(nrhs), int(k),
                                                OVS_VJP_STORE_BASIS if store_basis else 0,
                                                ctypes.byref(out)), "ovs_vjp_workspace_size")
        return int(out.value)

    def sign_apply_vjp(self, b, chi, k, want_y=True, store_basis=False, workspace=None,
                       defl=None, n_defl=None):
        """Gradient of L = sum_r Re <chi_r, y_r> for the k-step two-sided Lanczos
        y_r ~ sgn(A) b_r (FP64 lattices), with LR deflation by `defl` (its
        first n_defl eigentriples, all by default) if given.  The reverse sweep
        recomputes the Lanczos vectors from checkpoints unless store_basis.
        Returns (y or None, grad_b, grad_mu, grad_U [V,4,3,3], quad_err [nrhs], status)."""
        torch = _torch()
        b, nrhs = self._fields(b)
        chi, n2 = self._fields(chi)
        if n2 != nrhs:
            raise ValueError("chi must hold as many fields as b")
        y = torch.empty_like(b) if want_y else None
        gb = torch.empty_like(b)
        gU = torch.empty((self.V, 4, 3, 3), dtype=torch.complex128, device=b.device)
        gmu = ctypes.c_double(0.0)
        qerr = np.zeros(nrhs, dtype=np.float64)
        ws_p, ws_n = None, 0
        if workspace is not None:
            if not workspace.is_cuda or not workspace.is_contiguous():
                raise ValueError("workspace must be a contiguous CUDA tensor")
            ws_p = ctypes.c_void_p(workspace.data_ptr())
            ws_n = workspace.numel() * workspace.element_size()
        dh = defl._h if defl is not None else None
        nd = (defl.m if n_defl is None else int(n_defl)) if defl is not None else 0
        st = self._lib.ovs_sign_apply_vjp(
            self._h, dh, nd, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(chi.data_ptr()), nrhs,
            int(k),
            OVS_VJP_STORE_BASIS if store_basis else 0,
            ctypes.c_void_p(y.data_ptr()) if y is not None else None,
            ctypes.c_void_p(gb.data_ptr()), ctypes.byref(gmu), ctypes.c_void_p(gU.data_ptr()),
            _dptr(qerr), ws_p, ctypes.c_size_t(ws_n))
        _check(st, "ovs_sign_apply_vjp")
        if st == OVS_WARN_BREAKDOWN:
            raise OvsError(st, "ovs_sign_apply_vjp")
        return y, gb, gmu.value, gU, qerr, st

    def last_coefficients(self, nrhs, k_max):
        a = np.zeros((nrhs, k_max), dtype=np.complex128)
        bb = np.zeros((nrhs, k_max), dtype=np.float64)
        g = np.zeros((nrhs, k_max), dtype=np.complex128)
        x = np.zeros((nrhs, k_max), dtype=np.complex128)
        _check(self._lib.ovs_last_coefficients(self._h, _dptr(a.view(np.float64)), _dptr(bb),
                                               _dptr(g.view(np.float64)), _dptr(x.view(np.float64))),
               "ovs_last_coefficients")
        return a, bb, g, x

    def inner_sign_tridiag(self, diag, sub, sup, return_status=False):
        """sgn(T) e_1 for a batch of tridiagonal T ([batch, k] complex arrays, host).
        Returns (x, err), or (x, err, status) with return_status: status is
        OVS_WARN_SIGN_AMBIGUOUS when the quadrature missed its target (an
        eigenvalue of T near the imaginary axis)."""
        diag = np.ascontiguousarray(np.atleast_2d(diag), dtype=np.complex128)
        sub = np.ascontiguousarray(np.atleast_2d(sub), dtype=np.complex128)
        sup = np.ascontiguousarray(np.atleast_2d(sup), dtype=np.complex128)
        batch, k = diag.shape
        x = np.zeros((batch, k), dtype=np.complex128)
        err = np.zeros(batch)
        st = _check(self._lib.ovs_inner_sign_tridiag(self._h, batch, k, _dptr(diag.view(np.float64)),
                                                     _dptr(sub.view(np.float64)),
                                                     _dptr(sup.view(np.float64)),
                                                     _dptr(x.view(np.float64)), _dptr(err)),
                    "ovs_inner_sign_tridiag")
        return (x, err, st) if return_status else (x, err)

    def inner_sign_hessenberg(self, H, return_status=False):
        """sgn(H) e_1 for a batch of upper Hessenberg H ([batch, k, k] complex, host).
        Returns (x, err), or (x, err, status) as inner_sign_tridiag."""
        H = np.asarray(H, dtype=np.complex128)
        if H.ndim == 2:
            H = H[None]
        batch, k, _ = H.shape
        Hc = np.ascontiguousarray(np.swapaxes(H, 1, 2))  # column-major per matrix
        x = np.zeros((batch, k), dtype=np.complex128)
        err = np.zeros(batch)
        st = _check(self._lib.ovs_inner_sign_hessenberg(self._h, batch, k, _dptr(Hc.view(np.float64)),
                                                        _dptr(x.view(np.float64)), _dptr(err)),
                    "ovs_inner_sign_hessenberg")
        return (x, err, st) if return_status else (x, err)


def small_eig(A):
    """Eigenvalues and unit right eigenvectors of a small complex matrix (host code of the library)."""
    A = np.asarray(A, dtype=np.complex128)
    n = A.shape[0]
    Ac = np.ascontiguousarray(A.T)  # column major
    lam = np.zeros(n, dtype=np.complex128)
    V = np.zeros((n, n), dtype=np.complex128)
    _check(load().ovs_small_eig(n, _dptr(Ac.view(np.float64)), _dptr(lam.view(np.float64)),
                                _dptr(V.view(np.float64))), "ovs_small_eig")
    return lam, V.T.copy()  # V was filled column major


class Field:
    """ovs_field: nrhs sources resident in the library's layout."""

    def __init__(self, lat: Lattice, nrhs: int):
        self.lat = lat
        self.nrhs = int(nrhs)
        h = ctypes.c_void_p()
        _check(lat._lib.ovs_field_create(lat._h, self.nrhs, ctypes.byref(h)), "ovs_field_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self.lat._lib.ovs_field_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def import_(self, x):
        x = _dev_c128(x, "x")
        if x.numel() != self.nrhs * self.lat.N:
            raise ValueError("size mismatch")
        _check(self.lat._lib.ovs_field_import(self._h, ctypes.c_void_p(x.data_ptr())), "ovs_field_import")

    def export(self, out=None):
        torch = _torch()
        y = out if out is not None else torch.empty((self.nrhs, self.lat.N), dtype=torch.complex128, device="cuda")
        _check(self.lat._lib.ovs_field_export(self._h, ctypes.c_void_p(y.data_ptr())), "ovs_field_export")
        return y

    def apply(self, op, out: "Field"):
        _check(self.lat._lib.ovs_field_apply(self.lat._h, OPS[op], self._h, out._h), "ovs_field_apply")

    def apply_timed(self, op, out: "Field", iters):
        ms = ctypes.c_double()
        _check(self.lat._lib.ovs_field_apply_timed(self.lat._h, OPS[op], self._h, out._h, int(iters),
                                                   ctypes.byref(ms)), "ovs_field_apply_timed")
        return ms.value

    def dual_timed(self, iters):
        """Average time (ms) of the tuned two-sided Lanczos dual stencil on this
        field's sources (v~ = the field, w~ = a copy of it in the workspace, so
        the two are read from distinct memory as in a solve), HIP events on the
        lattice stream."""
        ms = ctypes.c_double()
        _check(self.lat._lib.ovs_dual_apply_timed(self.lat._h, self._h, int(iters), ctypes.byref(ms)),
               "ovs_dual_apply_timed")
        return ms.value


class Deflation:
    def __init__(self, lat, h, m):
        self.lat = lat
        self._h = h
        self.m = m

    def get(self):
        """(lambda [m] host, R [m, 12V] CUDA, L [m, 12V] CUDA, info [3] host)."""
        torch = _torch()
        lam = np.zeros(self.m, dtype=np.complex128)
        info = np.zeros(3)
        R = torch.empty((self.m, self.lat.N), dtype=torch.complex128, device="cuda")
        L = torch.empty_like(R)
        _check(self.lat._lib.ovs_deflation_get(self._h, _dptr(lam.view(np.float64)),
                                               ctypes.c_void_p(R.data_ptr()),
                                               ctypes.c_void_p(L.data_ptr()), _dptr(info)),
               "ovs_deflation_get")
        return lam, R, L, info

    def close(self):
        if getattr(self, "_h", None):
            self.lat._lib.ovs_deflation_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_sign_fn = None


def _sign_function():
    global _sign_fn
    if _sign_fn is not None:
        return _sign_fn
    torch = _torch()

    class SignFunction(torch.autograd.Function):
        """y = k-step two-sided Lanczos sgn(gamma5 Dw(mu; U)) b, differentiable in
        (b, mu, U); the backward pass is ovs_sign_apply_vjp."""

        @staticmethod
        def forward(ctx, b, mu, U, lat, m_w, k, n_defl, defl_tol):
            lat.set_links(U)
            lat.set_params(m_w, float(mu))
            defl = None
            if n_defl > 0:  # the eigentriples of this (mu, U), kept for the backward pass
                defl, dst = lat.deflation_compute(n_defl, tol=defl_tol)
                if dst != OVS_OK:
                    defl.close()
                    raise OvsError(dst, "ovs_deflation_compute")
            y, _, st = lat.sign_apply(b, k, defl=defl)
            if st == OVS_WARN_BREAKDOWN:
                raise OvsError(st, "ovs_sign_apply")
            ctx.save_for_backward(b, mu, U)
            ctx.lat, ctx.m_w, ctx.k, ctx.defl = lat, m_w, k, defl
            return y

        @staticmethod
        def backward(ctx, gy):
            b, mu, U = ctx.saved_tensors
            lat = ctx.lat
            lat.set_links(U)
            lat.set_params(ctx.m_w, float(mu))
            _, gb, gmu, gU, _, _ = lat.sign_apply_vjp(b, gy.contiguous(), ctx.k, want_y=False,
                                                       defl=ctx.defl)
            if ctx.defl is not None:
                ctx.defl.close()
                ctx.defl = None
            gmu_t = torch.tensor(gmu, dtype=mu.dtype, device=mu.device)
            return gb.view_as(b), gmu_t, gU.view_as(U), None, None, None, None, None

    _sign_fn = SignFunction
    return _sign_fn


def sign_autograd(lat, b, mu, U, m_w, k, n_defl=0, defl_tol=1e-10):
    """Differentiable y = sgn(A) b by k-step two-sided Lanczos.

    lat: an FP64 Lattice of the right size; its links and parameters are set
    from U (complex128 [V,4,3,3], CUDA) and mu (real 0-dim tensor) on every
    call.  b: complex128 CUDA [nrhs, 12V] or [12V].  n_defl > 0: LR deflation
    by that many eigentriples, computed for this (mu, U) in the forward pass
    (ovs_deflation_compute to defl_tol) and differentiated through in the
    backward pass (the deflation-aware gradient)."""
    return _sign_function().apply(b, mu, U, lat, float(m_w), int(k), int(n_defl), float(defl_tol))
