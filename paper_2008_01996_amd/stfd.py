"""Python binding of the stfd C library (argument marshalling only).

Every computation happens in libstfd.so: host FP64 setup in C++, the hot path
in HIP kernels for gfx950.  PyTorch is used only to hold device memory and to
name the HIP stream; if the library is missing this module raises on import
of any entry point, there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstfd.so")

OK, EINVAL, ENOMEM, EHIP, ENUMERIC, ENOCONV, ESTATE = 0, -1, -2, -3, -4, -5, -6
PREC_FP64, PREC_FP32 = 0, 1
METHOD_FD, METHOD_BSC = 0, 1
MAX_HIST = 64

EXPORTED = [
    "stfd_opts_default", "stfd_last_error", "stfd_assemble_time", "stfd_space_create",
    "stfd_space_free", "stfd_space_info", "stfd_space_csr_size", "stfd_space_export_csr",
    "stfd_project_f", "stfd_assemble_load", "stfd_dirichlet_lift", "stfd_time_decompose", "stfd_time_schur", "stfd_fd_setup",
    "stfd_fd_setup_report", "stfd_fd_factor", "stfd_fd_solve", "stfd_kh_residual",
    "stfd_problem_free", "stfd_fd_apply", "stfd_spatial_solve", "stfd_system_lambdas",
    "stfd_profile", "stfd_profile_read", "stfd_batch_create", "stfd_batch_factor", "stfd_batch_solve",
    "stfd_batch_free",
]

STAGES = ["band_init", "band_ldl", "fwd1", "fwd2", "sweep_fwd", "sweep_bwd", "back", "spatial", "resid",
          "reduce", "inner", "band_inv"]


class StfdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"stfd error {code}: {msg}")
        self.code = code


class Opts(C.Structure):
    _fields_ = [("precision", C.c_int), ("fp64_transforms", C.c_int), ("rtol", C.c_double),
                ("max_refine", C.c_int), ("method", C.c_int), ("inner_refine", C.c_int),
                ("graph", C.c_int), ("nrhs_max", C.c_int), ("inner_refine_first", C.c_int)]


class Tuning(C.Structure):
    _fields_ = [("sweep_tile_min_rhs", C.c_int), ("gemm_tile_m_fp32", C.c_int), ("gemm_tile_m_fp64", C.c_int),
                ("gemm_n_fast", C.c_int), ("factor_kernel", C.c_int), ("factor_pack_real", C.c_int),
                ("gemm_tile_n_fp64", C.c_int), ("sweep_pack_real", C.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class SetupReport(C.Structure):
    _fields_ = [("min_re_lambda", C.c_double), ("max_abs_lambda", C.c_double),
                ("sigma_min", C.c_double), ("sigma_max", C.c_double), ("kappa2", C.c_double),
                ("eig_residual", C.c_double), ("n_real", C.c_int), ("n_pairs", C.c_int),
                ("n_sys", C.c_int), ("half_band", C.c_int), ("setup_seconds", C.c_double),
                ("factor_bytes", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class SolveReport(C.Structure):
    _fields_ = [("iterations", C.c_int), ("converged", C.c_int), ("nrhs", C.c_int),
                ("rel_residual", C.c_double * MAX_HIST), ("seconds", C.c_double)]

    def as_dict(self):
        return {"iterations": self.iterations, "converged": bool(self.converged), "nrhs": self.nrhs,
                "rel_residual": list(self.rel_residual[: self.iterations]), "seconds": self.seconds}


_LIB = None


def lib():
    """Load libstfd.so (built by paper_2008_01996_amd.build); raise if absent."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not found: build it with python -m paper_2008_01996_amd.build")
        # torch ships its own HIP runtime under the same soname as the one the
        # library links; loading torch first makes both use that one runtime
        # (the library loaded first left the library's HIP calls without a device)
        import torch  # noqa: F401

        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        vp = C.c_void_p
        L.stfd_last_error.restype = C.c_char_p
        L.stfd_opts_default.argtypes = [C.POINTER(Opts)]
        L.stfd_assemble_time.argtypes = [C.c_int, dp, dp, dp, dp]
        L.stfd_space_create.argtypes = [C.c_int, dp, C.c_int, ip, ip, C.POINTER(vp)]
        L.stfd_space_free.argtypes = [vp]
        L.stfd_space_free.restype = None
        L.stfd_space_info.argtypes = [vp, ip, ip, ip, C.POINTER(C.c_longlong)]
        L.stfd_space_csr_size.argtypes = [vp, C.c_int, ip, ip, C.POINTER(C.c_longlong)]
        L.stfd_space_export_csr.argtypes = [vp, C.c_int, ip, ip, dp]
        L.stfd_project_f.argtypes = [vp, C.c_int, dp, C.c_int, C.c_int, ip, ip, ip, dp, dp, dp]
        L.stfd_assemble_load.argtypes = [vp, C.c_int, dp, dp, dp]
        L.stfd_dirichlet_lift.argtypes = [vp, C.c_int, dp, dp, dp, dp]
        L.stfd_time_decompose.argtypes = [C.c_int, dp, dp, dp, dp, dp, dp, dp, C.POINTER(SetupReport)]
        L.stfd_time_schur.argtypes = [C.c_int, dp, dp, dp, dp]
        L.stfd_fd_setup.argtypes = [vp, C.c_int, dp, dp, C.POINTER(Opts), vp, C.POINTER(vp)]
        L.stfd_fd_setup_report.argtypes = [vp, C.POINTER(SetupReport)]
        L.stfd_fd_factor.argtypes = [vp, vp]
        L.stfd_get_tuning.argtypes = [vp, C.POINTER(Tuning)]
        L.stfd_kh_residual_noalloc.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp]
        L.stfd_kh_residual_noalloc_max_bytes.restype = C.c_size_t
        L.stfd_kh_residual_noalloc_max_bytes.argtypes = []
        L.stfd_set_tuning.argtypes = [vp, C.POINTER(Tuning)]
        L.stfd_fd_solve.argtypes = [vp, C.c_int, vp, vp, C.POINTER(SolveReport), vp]
        L.stfd_kh_residual.argtypes = [vp, C.c_int, vp, vp, vp, dp, vp]
        L.stfd_fd_apply.argtypes = [vp, C.c_int, vp, vp, vp]
        L.stfd_spatial_solve.argtypes = [vp, C.c_int, vp, vp, vp]
        L.stfd_system_lambdas.argtypes = [vp, dp]
        L.stfd_profile.argtypes = [vp, C.c_int]
        L.stfd_profile_read.argtypes = [vp, dp, C.POINTER(C.c_longlong)]
        L.stfd_problem_free.argtypes = [vp]
        L.stfd_problem_free.restype = None
        L.stfd_batch_create.argtypes = [C.c_int, C.POINTER(vp), C.POINTER(vp)]
        L.stfd_batch_factor.argtypes = [vp, vp]
        L.stfd_batch_solve.argtypes = [vp, ip, C.POINTER(vp), C.POINTER(vp), C.POINTER(SolveReport), vp]
        L.stfd_batch_free.argtypes = [vp]
        L.stfd_batch_free.restype = None
        _LIB = L
    return _LIB


def _check(rc):
    if rc != OK:
        raise StfdError(rc, lib().stfd_last_error().decode())
    return rc


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def assemble_time(t):
    """A_t, M_t, C_t (row = test index) on the time nodes t (Sec. 2)."""
    t = _f64(t)
    nt = len(t) - 1
    A = np.empty((nt, nt))
    M = np.empty((nt, nt))
    Cm = np.empty((nt, nt))
    _check(lib().stfd_assemble_time(nt, _dp(t), _dp(A), _dp(M), _dp(Cm)))
    return A, M, Cm


def time_decompose(At, Mt):
    """Host steps 1a/1b: eigenvalues (ordered pairs | conjugates | real),
    unit-norm eigenvectors X (columns), singular values of X, report."""
    At = _f64(At)
    Mt = _f64(Mt)
    n = At.shape[0]
    lr, li, s = np.empty(n), np.empty(n), np.empty(n)
    Xr, Xi = np.empty((n, n)), np.empty((n, n))
    rep = SetupReport()
    _check(lib().stfd_time_decompose(n, _dp(At), _dp(Mt), _dp(lr), _dp(li), _dp(Xr), _dp(Xi), _dp(s),
                                      C.byref(rep)))
    return lr + 1j * li, Xr + 1j * Xi, s, rep.as_dict()


def time_schur(At, Mt):
    """Host step 1 of Algorithm BSc: A_t^-1 M_t = W S W^* with W unitary and
    S upper triangular.  Returns (S, W)."""
    At = _f64(At)
    Mt = _f64(Mt)
    n = At.shape[0]
    S, W = np.empty(2 * n * n), np.empty(2 * n * n)
    _check(lib().stfd_time_schur(n, _dp(At), _dp(Mt), _dp(S), _dp(W)))
    return (S[0::2] + 1j * S[1::2]).reshape(n, n), (W[0::2] + 1j * W[1::2]).reshape(n, n)


class Space:
    """P1 space on a triangulation (mesh with xy, tri, dof, box attributes)."""

    def __init__(self, mesh):
        xy = _f64(mesh.xy).reshape(-1)
        tri = np.ascontiguousarray(mesh.tri, dtype=np.int32).reshape(-1)
        dof = np.ascontiguousarray(mesh.dof, dtype=np.int32)
        self._h = C.c_void_p()
        self.box = np.asarray(mesh.box, dtype=np.float64)
        _check(lib().stfd_space_create(len(dof), _dp(xy), len(tri) // 3, _ip(tri), _ip(dof), C.byref(self._h)))
        mx, nt, hb = C.c_int(), C.c_int(), C.c_int()
        nnz = C.c_longlong()
        _check(lib().stfd_space_info(self._h, C.byref(mx), C.byref(nt), C.byref(hb), C.byref(nnz)))
        self.Mx, self.ntri, self.half_band, self.nnz = mx.value, nt.value, hb.value, nnz.value
        self.nv = len(dof)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _LIB is not None:
            _LIB.stfd_space_free(h)
            self._h = None

    def csr(self, which):
        """(rowptr, col, val, shape) of M_x (0), A_x (1) or M10 (2)."""
        r, c = C.c_int(), C.c_int()
        nnz = C.c_longlong()
        _check(lib().stfd_space_csr_size(self._h, which, C.byref(r), C.byref(c), C.byref(nnz)))
        rp = np.empty(r.value + 1, np.int32)
        cl = np.empty(nnz.value, np.int32)
        vl = np.empty(nnz.value)
        _check(lib().stfd_space_export_csr(self._h, which, _ip(rp), _ip(cl), _dp(vl)))
        return rp, cl, vl, (r.value, c.value)

    def project_f(self, t, modes=None, kind=0):
        """Prism means F (ntri x Nt) of f: kind 0 random modes, kind 1 the
        manufactured time profile 2t + 2 pi^2 t^2, kind 2 the source of the
        L-shape example of Sec. 5 (modes not used)."""
        t = _f64(t)
        nt = len(t) - 1
        if kind == 2:
            F = np.empty((nt, self.ntri))
            _check(lib().stfd_project_f(self._h, nt, _dp(t), 2, 0, None, None, None, None, None, _dp(F)))
            return F.T
        a = np.ascontiguousarray(modes.a, np.int32)
        b = np.ascontiguousarray(modes.b, np.int32)
        d = np.ascontiguousarray(modes.d, np.int32)
        c = _f64(modes.c)
        F = np.empty((nt, self.ntri))           # column-major ntri x Nt
        _check(lib().stfd_project_f(self._h, nt, _dp(t), kind, len(a), _ip(a), _ip(b), _ip(d), _dp(c),
                                    _dp(self.box), _dp(F)))
        return F.T

    def assemble_load(self, Ct, F):
        """F~ = M10 F C_t^T as an (M_x, N_t) array."""
        Ct = _f64(Ct)
        nt = Ct.shape[0]
        Fc = np.ascontiguousarray(np.asarray(F, dtype=np.float64).T)      # column-major
        out = np.empty((nt, self.Mx))
        _check(lib().stfd_assemble_load(self._h, nt, _dp(Ct), _dp(Fc), _dp(out)))
        return out.T

    def dirichlet_lift(self, At, Mt, G, Ft):
        """Ft - (the coupling of the Dirichlet extension with nodal values
        G[v, k] at vertex v and time t_{k+1}) as a new (M_x, N_t) array;
        rows of G for interior vertices are ignored."""
        At = _f64(At)
        Mt = _f64(Mt)
        nt = At.shape[0]
        Gc = np.ascontiguousarray(np.asarray(G, dtype=np.float64).T)      # column-major nv x Nt
        out = np.ascontiguousarray(np.asarray(Ft, dtype=np.float64).T)    # column-major M_x x Nt
        if Gc.shape != (nt, self.nv) or out.shape != (nt, self.Mx) or Mt.shape != (nt, nt):
            raise ValueError("dirichlet_lift: shape mismatch")
        _check(lib().stfd_dirichlet_lift(self._h, nt, _dp(At), _dp(Mt), _dp(Gc), _dp(out)))
        return out.T


def _check_tensor(name, x, dtype, shape, device):
    """Raise ValueError unless x is a contiguous torch tensor of that dtype and
    shape on that device: the library reads and writes exactly that many
    elements at the pointer, so a mismatch must stop here, on the host."""
    import torch

    if not isinstance(x, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor, got {type(x).__name__}")
    if x.dtype != dtype:
        raise ValueError(f"{name}: dtype {x.dtype}, expected {dtype}")
    if x.device != device:
        raise ValueError(f"{name}: on {x.device}, expected {device}")
    if not x.is_contiguous():
        raise ValueError(f"{name}: not contiguous")
    if tuple(x.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(x.shape)}, expected {tuple(shape)}")


def _stream_ptr(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


class Problem:
    """Space-time solver (Algorithm FD, or BSc) for one (space, time mesh) pair on the current GPU."""

    def __init__(self, space: Space, At, Mt, precision="fp32", fp64_transforms=5, rtol=1e-10, max_refine=30,
                 stream=None, method="fd", inner_refine=-1, graph=True, nrhs_max=0, inner_refine_first=-1,
                 tuning="cache"):
        """fp64_transforms (FP32 form only): bit mask of the transform GEMMs run
        on FP64 matrix cores, bit 0 first forward, bit 1 second forward, bit 2
        back transform.  method "fd" (Algorithm FD) or "bsc" (Algorithm BSc,
        Bartels-Stewart with the complex Schur form; precision "fp64").
        inner_refine, graph, nrhs_max, inner_refine_first: the stfd_opts fields
        of those names.
        tuning: kernel variants, "cache" (the autotuner's entry for this
        shape, if any), None (library defaults) or a dict of stfd_tuning
        fields."""
        self.space = space        # keep alive: the problem refers to it
        At = _f64(At)
        Mt = _f64(Mt)
        self.Nt = At.shape[0]
        self.Mx = space.Mx
        o = Opts()
        _check(lib().stfd_opts_default(C.byref(o)))
        o.precision = {"fp32": PREC_FP32, "fp64": PREC_FP64}[precision]
        o.fp64_transforms = int(fp64_transforms)
        o.rtol = float(rtol)
        o.max_refine = int(max_refine)
        o.method = {"fd": METHOD_FD, "bsc": METHOD_BSC}[method]
        o.inner_refine = int(inner_refine)
        o.inner_refine_first = int(inner_refine_first)
        o.graph = int(bool(graph))
        o.nrhs_max = int(nrhs_max)
        self.precision = precision
        self.method = method
        import torch

        self.device = torch.device("cuda", torch.cuda.current_device())
        self._h = C.c_void_p()
        _check(lib().stfd_fd_setup(space._h, self.Nt, _dp(At), _dp(Mt), C.byref(o),
                                   C.c_void_p(_stream_ptr(stream)), C.byref(self._h)))
        rep = SetupReport()
        _check(lib().stfd_fd_setup_report(self._h, C.byref(rep)))
        self.setup_report = rep.as_dict()
        # kernel variants: the autotuner's cached choice for this shape
        # ("cache"), the library defaults (None), or explicit fields (dict)
        if tuning == "cache":
            from paper_2008_01996_amd import autotune
            autotune.apply(self)
        elif isinstance(tuning, dict):
            self.set_tuning(**tuning)
        elif tuning is not None:
            raise ValueError("tuning: 'cache', None or a dict of stfd_tuning fields")

    def tuning(self):
        """The kernel variants in use, as a dict (stfd_tuning)."""
        t = Tuning()
        _check(lib().stfd_get_tuning(self._h, C.byref(t)))
        return t.as_dict()

    def set_tuning(self, **kw):
        """Select kernel variants (stfd_tuning fields); effective from the
        next factor()."""
        t = Tuning()
        _check(lib().stfd_get_tuning(self._h, C.byref(t)))
        for k, v in kw.items():
            if k not in dict(Tuning._fields_):
                raise ValueError(f"unknown tuning field {k}")
            setattr(t, k, int(v))
        _check(lib().stfd_set_tuning(self._h, C.byref(t)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _LIB is not None:
            _LIB.stfd_problem_free(h)
            self._h = None

    def factor(self, stream=None):
        _check(lib().stfd_fd_factor(self._h, C.c_void_p(_stream_ptr(stream))))

    def _rhs_shape(self, X, name):
        import torch

        if not isinstance(X, torch.Tensor) or X.dim() != 3 or X.shape[0] < 1:
            raise ValueError(f"{name}: expected a (nrhs, N_t, M_x) tensor")
        return (X.shape[0], self.Nt, self.Mx)

    def _solve(self, fn, F, U, stream, check):
        import torch

        shape = self._rhs_shape(F, "F")
        _check_tensor("F", F, torch.float64, shape, self.device)
        _check_tensor("U", U, torch.float64, shape, self.device)
        rep = SolveReport()
        rc = fn(self._h, F.shape[0], C.c_void_p(F.data_ptr()), C.c_void_p(U.data_ptr()), C.byref(rep),
                C.c_void_p(_stream_ptr(stream)))
        out = rep.as_dict()
        out["status"] = rc
        if check:
            _check(rc)
        return out

    def solve(self, F, U, stream=None, check=True):
        """F, U: torch float64 CUDA tensors of shape (nrhs, N_t, M_x) (the
        [rhs][k][i] layout).  Returns the solve report as a dict."""
        return self._solve(lib().stfd_fd_solve, F, U, stream, check)

    def apply(self, X, U, stream=None):
        """One FD application without refinement: U = FD(X) (device tensors
        (nrhs, N_t, M_x) float64)."""
        import torch

        shape = self._rhs_shape(X, "X")
        _check_tensor("X", X, torch.float64, shape, self.device)
        _check_tensor("U", U, torch.float64, shape, self.device)
        _check(lib().stfd_fd_apply(self._h, X.shape[0], C.c_void_p(X.data_ptr()), C.c_void_p(U.data_ptr()),
                                   C.c_void_p(_stream_ptr(stream))))

    def spatial_solve(self, G, Z, stream=None):
        """Step 3 alone on device tensors of shape (nrhs, 2 n_sys, M_x) in the
        working precision (float32 for fp32, float64 for fp64)."""
        import torch

        dt = torch.float32 if self.precision == "fp32" else torch.float64
        if not isinstance(G, torch.Tensor) or G.dim() != 3 or G.shape[0] < 1:
            raise ValueError("G: expected a (nrhs, 2 n_sys, M_x) tensor")
        shape = (G.shape[0], 2 * self.setup_report["n_sys"], self.Mx)
        _check_tensor("G", G, dt, shape, self.device)
        _check_tensor("Z", Z, dt, shape, self.device)
        _check(lib().stfd_spatial_solve(self._h, G.shape[0], C.c_void_p(G.data_ptr()), C.c_void_p(Z.data_ptr()),
                                        C.c_void_p(_stream_ptr(stream))))

    def system_lambdas(self):
        n = self.setup_report["n_sys"]
        lam = np.empty(2 * n)
        _check(lib().stfd_system_lambdas(self._h, _dp(lam)))
        return lam[0::2] + 1j * lam[1::2]

    def profile(self, enable=True):
        """Enable (and clear) or disable per-stage event timing."""
        _check(lib().stfd_profile(self._h, int(bool(enable))))

    def profile_read(self):
        """{stage: (total ms, launches)} since the last clear."""
        ms = np.zeros(len(STAGES))
        cnt = (C.c_longlong * len(STAGES))()
        _check(lib().stfd_profile_read(self._h, _dp(ms), cnt))
        return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(STAGES)}

    def kh_residual(self, F, U, R, stream=None):
        """R = F - K_h U on the device; returns (||R||^2, ||F||^2) per RHS."""
        import torch

        shape = self._rhs_shape(F, "F")
        for name, x in (("F", F), ("U", U), ("R", R)):
            _check_tensor(name, x, torch.float64, shape, self.device)
        n = F.shape[0]
        norms = np.empty(2 * n)
        _check(lib().stfd_kh_residual(self._h, n, C.c_void_p(F.data_ptr()), C.c_void_p(U.data_ptr()),
                                      C.c_void_p(R.data_ptr()), _dp(norms), C.c_void_p(_stream_ptr(stream))))
        return norms.reshape(n, 2)


    def kh_residual_noalloc(self, F, U, R, norms=None, stream=None):
        """R = F - K_h U on the device, with no device allocation (the work
        memory is the library's fixed per-device array of
        kh_residual_noalloc_max_bytes() bytes); norms: None or a float64
        device tensor of 2 nrhs entries that receives (||R||^2, ||F||^2) per
        RHS.  Calls that overlap on one GPU race on that array."""
        import torch

        shape = self._rhs_shape(F, "F")
        for name, x in (("F", F), ("U", U), ("R", R)):
            _check_tensor(name, x, torch.float64, shape, self.device)
        if norms is not None:
            _check_tensor("norms", norms, torch.float64, (2 * F.shape[0],), self.device)
        _check(lib().stfd_kh_residual_noalloc(self._h, F.shape[0], C.c_void_p(F.data_ptr()),
                                              C.c_void_p(U.data_ptr()), C.c_void_p(R.data_ptr()),
                                              C.c_void_p(norms.data_ptr() if norms is not None else None),
                                              C.c_void_p(_stream_ptr(stream))))


def kh_residual_noalloc_max_bytes():
    """Size of the fixed work array of Problem.kh_residual_noalloc."""
    return int(lib().stfd_kh_residual_noalloc_max_bytes())

class Batch:
    """Independent problems solved together (lockstep refinement, one host
    synchronisation per round for all of them).  Keeps the problems alive."""

    def __init__(self, problems):
        self.problems = list(problems)
        arr = (C.c_void_p * len(self.problems))(*[p._h for p in self.problems])
        h = C.c_void_p()
        _check(lib().stfd_batch_create(len(self.problems), arr, C.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _LIB is not None:
            _LIB.stfd_batch_free(h)
            self._h = None

    def factor(self, stream=None):
        _check(lib().stfd_batch_factor(self._h, C.c_void_p(_stream_ptr(stream))))

    def solve(self, Fs, Us, stream=None, check=True):
        """Fs, Us: lists of torch float64 CUDA tensors (nrhs_i, N_t_i, M_x_i).
        Returns (status, list of per-problem report dicts)."""
        import torch

        n = len(self.problems)
        if len(Fs) != n or len(Us) != n:
            raise ValueError(f"batch solve: {n} problems, {len(Fs)} loads and {len(Us)} solutions")
        for i, (p, F, U) in enumerate(zip(self.problems, Fs, Us)):
            shape = p._rhs_shape(F, f"Fs[{i}]")
            _check_tensor(f"Fs[{i}]", F, torch.float64, shape, p.device)
            _check_tensor(f"Us[{i}]", U, torch.float64, shape, p.device)
        nr = (C.c_int * n)(*[F.shape[0] for F in Fs])
        fp = (C.c_void_p * n)(*[F.data_ptr() for F in Fs])
        up = (C.c_void_p * n)(*[U.data_ptr() for U in Us])
        reps = (SolveReport * n)()
        rc = lib().stfd_batch_solve(self._h, nr, fp, up, reps, C.c_void_p(_stream_ptr(stream)))
        if check:
            _check(rc)
        return rc, [r.as_dict() for r in reps]
