"""ctypes binding of libriga.so (include/riga.h).  Argument marshalling only:
every step of the solver runs in the library's HIP kernels.  PyTorch
provides device memory and the current stream.

The library must have been built (``python -m paper_2009_08167_amd.build``);
loading fails loudly otherwise -- there is no fallback path.
"""
import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libriga.so")

RIGA_OK, RIGA_EINVAL, RIGA_ENOMEM, RIGA_EDEVICE = 0, -1, -2, -3
RIGA_ENOCONV, RIGA_ESINGULAR, RIGA_EDEGENERATE, RIGA_EUNSUPPORTED = -4, -5, -6, -7
RIGA_FP64, RIGA_MIXED = 0, 1
RIGA_MAT_K, RIGA_MAT_M, RIGA_MAT_A = 0, 1, 2

EXPORTED = ["riga_set_allocator", "riga_analyze", "riga_assemble", "riga_update_coefficients",
            "riga_problem_info",
            "riga_tree_export", "riga_get_matrices", "riga_spmv", "riga_tune", "riga_factor", "riga_factor_batched", "riga_solve",
            "riga_solve_multi", "riga_project", "riga_project_noalloc", "riga_eigs", "riga_eigs_batched", "riga_eig_grad",
            "riga_mode_errors", "riga_exact_eigenvalues", "riga_destroy", "riga_status_string",
            "riga_last_error"]
RIGA_PROJECT_MAX_COLS = 8192


class MeshDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("ne", C.c_int32 * 3), ("p", C.c_int32),
                ("sep_spacing", C.c_int32), ("nquad", C.c_int32),
                ("kappa", C.c_void_p), ("rho", C.c_void_p), ("coeffs_on_device", C.c_int32),
                ("leaf_dofs", C.c_int32), ("stream", C.c_void_p), ("hermitian", C.c_int32),
                ("potential", C.c_double * 3)]


class EigsOpts(C.Structure):
    _fields_ = [("lo", C.c_double), ("hi", C.c_double), ("nev", C.c_int32),
                ("precision", C.c_int32), ("tol", C.c_double), ("max_basis", C.c_int32),
                ("max_restarts", C.c_int32), ("per_shift", C.c_int32), ("seed", C.c_uint64),
                ("stream", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [("n_shift", C.c_int32), ("n_fact", C.c_int32), ("n_fb", C.c_int32),
                ("n_mv", C.c_int32), ("n_it", C.c_int32), ("n_ir", C.c_int32),
                ("n_perturbed_pivots", C.c_int32), ("n_2x2_pivots", C.c_int32),
                ("t_fact", C.c_double), ("t_fb", C.c_double), ("t_mv", C.c_double),
                ("t_orth", C.c_double), ("t_proj", C.c_double), ("t_ritz", C.c_double),
                ("t_total", C.c_double), ("flops_fact", C.c_double), ("bytes_fb", C.c_double),
                ("n_thick", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ProblemInfo(C.Structure):
    _fields_ = [("n_dof", C.c_int64), ("n_elem", C.c_int64), ("nnz", C.c_int64),
                ("n1", C.c_int32 * 3), ("n_fronts", C.c_int32), ("tree_height", C.c_int32),
                ("max_front", C.c_int32), ("max_fs", C.c_int32), ("nnz_l", C.c_int64),
                ("flops_fact", C.c_double), ("front_pool", C.c_int64),
                ("nnz_l_exact", C.c_int64), ("flops_fact_exact", C.c_double),
                ("components", C.c_int32), ("sweep_bytes_stored", C.c_double),
                ("top_cut", C.c_int32), ("fused_heights", C.c_int32),
                ("fused_subtrees", C.c_int32), ("tuned", C.c_int32)]


class TuneResult(C.Structure):
    _fields_ = [("top_cut", C.c_int32), ("fused_heights", C.c_int32), ("candidates", C.c_int32),
                ("before_top_cut", C.c_int32), ("before_fused_heights", C.c_int32),
                ("sweep_us", C.c_double), ("fact_us", C.c_double),
                ("before_sweep_us", C.c_double), ("before_fact_us", C.c_double)]


class Allocator(C.Structure):
    _fields_ = [("ctx", C.c_void_p),
                ("alloc", C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)),
                ("free", C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p))]


class RigaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("riga status %d: %s" % (code, msg))
        self.code = code


_lib = None


def lib():
    """Load libriga.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libriga.so not built: run `python -m paper_2009_08167_amd.build`")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.riga_set_allocator.argtypes = [C.POINTER(Allocator)]
        L.riga_analyze.argtypes = [C.POINTER(MeshDesc), C.POINTER(P)]
        L.riga_assemble.argtypes = [C.POINTER(MeshDesc), C.POINTER(P)]
        L.riga_problem_info.argtypes = [P, C.POINTER(ProblemInfo)]
        L.riga_update_coefficients.argtypes = [P, P, P, C.c_int32, P]
        L.riga_tree_export.argtypes = [P] + [P] * 6
        L.riga_get_matrices.argtypes = [P, P, P, P, P]
        L.riga_spmv.argtypes = [P, C.c_int32, P, P, P]
        L.riga_factor.argtypes = [P, C.c_double, C.c_int32, C.POINTER(C.c_int64), C.POINTER(Stats)]
        L.riga_factor_batched.argtypes = [P, C.c_int32, P, C.c_int32, P, P]
        L.riga_tune.argtypes = [P, C.c_int32, C.c_int32, C.POINTER(TuneResult)]
        L.riga_solve.argtypes = [P, P, P, C.c_int32, P]
        L.riga_solve_multi.argtypes = [P, P, P, C.c_int32, C.c_int64, C.c_int32, P]
        L.riga_eigs.argtypes = [P, C.POINTER(EigsOpts), C.POINTER(C.c_int32), P, P, P,
                                C.POINTER(Stats)]
        L.riga_project.argtypes = [C.c_int64, C.c_int32, P, P, P, P, P]
        L.riga_project_noalloc.argtypes = [C.c_int64, C.c_int32, P, P, P, P, P]
        L.riga_eig_grad.argtypes = [P, C.c_int32, P, P, P, P, P, P]
        L.riga_mode_errors.argtypes = [P, C.c_int32, P, P, C.c_int32, P, C.c_int32, P, P, P, P, P, P]
        L.riga_exact_eigenvalues.argtypes = [C.c_int32, C.c_int32, P]
        L.riga_eigs_batched.argtypes = [P, C.c_int32, C.POINTER(EigsOpts), C.c_int32,
                                        C.POINTER(C.c_int32), P, P, P, P]
        L.riga_destroy.argtypes = [P]
        L.riga_destroy.restype = None
        L.riga_status_string.restype = C.c_char_p
        L.riga_last_error.restype = C.c_char_p
        for name in ["riga_analyze", "riga_assemble", "riga_update_coefficients",
                     "riga_problem_info", "riga_tree_export",
                     "riga_get_matrices", "riga_spmv", "riga_factor", "riga_solve", "riga_solve_multi",
                     "riga_eigs", "riga_eig_grad", "riga_set_allocator", "riga_eigs_batched",
                     "riga_mode_errors", "riga_exact_eigenvalues", "riga_project",
                     "riga_project_noalloc"]:
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(code, allow=()):
    if code != RIGA_OK and code not in allow:
        raise RigaError(code, lib().riga_last_error().decode())
    return code


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Problem:
    """An assembled (or only analysed) rIGA problem."""

    def __init__(self, handle, dim, ne, p, s, device):
        self._h = handle
        self.dim, self.ne, self.p, self.s = dim, ne, p, s
        self.device = device
        inf = ProblemInfo()
        _check(lib().riga_problem_info(self._h, C.byref(inf)))
        self.info = {f: (list(getattr(inf, f)) if f == "n1" else getattr(inf, f))
                     for f, _ in ProblemInfo._fields_}
        self.n_dof = int(inf.n_dof)
        self.n_elem = int(inf.n_elem)
        # a complex Hermitian pencil: n_dof real unknowns, n_dof / 2 complex DOFs
        self.hermitian = int(inf.components) == 2

    def refresh_info(self):
        """riga_problem_info again (its sweep bytes depend on the device set-up)."""
        inf = ProblemInfo()
        _check(lib().riga_problem_info(self._h, C.byref(inf)))
        self.info = {f: (list(getattr(inf, f)) if f == "n1" else getattr(inf, f))
                     for f, _ in ProblemInfo._fields_}
        return self.info

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            try:
                _lib.riga_destroy(h)
            except Exception:
                pass
        self._h = None

    def close(self):
        self.__del__()

    def update_coefficients(self, kappa, rho, stream=None):
        """Re-assemble K, M on the device for new per-element coefficients
        (torch device tensors or host arrays; None -> 1)."""
        keep = []
        on_dev = 0
        ptrs = []
        for v in (kappa, rho):
            if v is None:
                ptrs.append(None)
            elif hasattr(v, "is_cuda") and v.is_cuda:
                v = v.contiguous().double()
                keep.append(v)
                on_dev = 1
                ptrs.append(C.c_void_p(v.data_ptr()))
            else:
                a = np.ascontiguousarray(np.asarray(v, dtype=np.float64))
                keep.append(a)
                ptrs.append(C.c_void_p(a.ctypes.data))
        _check(lib().riga_update_coefficients(self._h, ptrs[0], ptrs[1], on_dev, _stream(stream)))

    def tree(self):
        """Symbolic analysis as numpy arrays."""
        nf = self.info["n_fronts"]
        perm = np.zeros(self.n_dof, np.int32)
        fk = np.zeros(nf, np.int32)
        ff = np.zeros(nf, np.int32)
        par = np.zeros(nf, np.int32)
        hgt = np.zeros(nf, np.int32)
        _check(lib().riga_tree_export(self._h, perm.ctypes.data, fk.ctypes.data, ff.ctypes.data,
                                      par.ctypes.data, hgt.ctypes.data, None))
        rows = np.zeros(int(ff.sum()), np.int32)
        _check(lib().riga_tree_export(self._h, None, None, None, None, None, rows.ctypes.data))
        return dict(perm=perm, k=fk, f=ff, parent=par, height=hgt, rows=rows)

    def pattern(self):
        nnz = self.info["nnz"]
        rp = np.zeros(self.n_dof + 1, np.int64)
        ci = np.zeros(nnz, np.int32)
        _check(lib().riga_get_matrices(self._h, rp.ctypes.data, ci.ctypes.data, None, None))
        return rp, ci

    def matrices(self):
        """(row_ptr, col_idx, K values, M values) copied from the device."""
        import scipy.sparse as sp
        nnz = self.info["nnz"]
        rp = np.zeros(self.n_dof + 1, np.int64)
        ci = np.zeros(nnz, np.int32)
        kv = np.zeros(nnz)
        mv = np.zeros(nnz)
        _check(lib().riga_get_matrices(self._h, rp.ctypes.data, ci.ctypes.data, kv.ctypes.data,
                                       mv.ctypes.data))
        shape = (self.n_dof, self.n_dof)
        return sp.csr_matrix((kv, ci, rp), shape=shape), sp.csr_matrix((mv, ci, rp), shape=shape)

    def spmv(self, which, x, y=None, stream=None):
        """y = K x, M x or (K - sigma M) x (queued on the stream)."""
        import torch
        if y is None:
            y = torch.empty_like(x)
        _check(lib().riga_spmv(self._h, which, _ptr(x), _ptr(y), _stream(stream)))
        return y

    def factor(self, sigma, precision=RIGA_FP64, allow_singular=False):
        """Factorise K - sigma M; returns (inertia, stats).  stats["status"]
        is RIGA_ESINGULAR (raised unless allow_singular) when a pivot had to
        be perturbed."""
        neg = C.c_int64(0)
        st = Stats()
        code = lib().riga_factor(self._h, float(sigma), precision, C.byref(neg), C.byref(st))
        _check(code, allow=(RIGA_ESINGULAR,) if allow_singular else ())
        d = st.as_dict()
        d["status"] = code
        return int(neg.value), d

    def tune(self, precision=RIGA_FP64, reps=0):
        """riga_tune: time the sweep decompositions of this problem, apply
        and cache the fastest; returns the result fields as a dict.  The
        factorisation is discarded (factor again before solve)."""
        r = TuneResult()
        _check(lib().riga_tune(self._h, precision, reps, C.byref(r)))
        self.refresh_info()
        return {f: getattr(r, f) for f, _ in TuneResult._fields_}

    def solve(self, b, max_ir=0, stream=None):
        import torch
        x = torch.empty_like(b)
        _check(lib().riga_solve(self._h, _ptr(b), _ptr(x), max_ir, _stream(stream)))
        return x

    def solve_multi(self, B, max_ir=0, stream=None):
        """Columns of X = A^{-1} B for B a contiguous [nrhs, n_dof] device
        tensor (one right-hand side per row), solved back to back."""
        import torch
        if B.dim() != 2 or B.shape[1] != self.n_dof or not B.is_contiguous():
            raise ValueError("B must be a contiguous [nrhs, n_dof] tensor")
        X = torch.empty_like(B)
        _check(lib().riga_solve_multi(self._h, _ptr(B), _ptr(X), B.shape[0], self.n_dof, max_ir,
                                      _stream(stream)))
        return X

    def eigs(self, nev, lo=0.0, hi=math.inf, precision=RIGA_FP64, tol=1e-9, max_basis=0,
             max_restarts=0, per_shift=0, seed=0, vectors=True, stream=None, allow_partial=False):
        """nev lowest eigenpairs in [lo, hi).  Returns (lam numpy, U torch
        [n_dof, nev] or None, resid numpy, stats dict); for a complex
        Hermitian problem U is complex128 [n_dof / 2, nev]."""
        import torch
        o = EigsOpts(lo=lo, hi=hi, nev=nev, precision=precision, tol=tol, max_basis=max_basis,
                     max_restarts=max_restarts, per_shift=per_shift, seed=seed,
                     stream=_stream(stream))
        lam = np.zeros(nev)
        res = np.zeros(nev)
        U = None
        if vectors:
            U = torch.zeros((nev, self.n_dof), dtype=torch.float64, device=self.device)
        nf = C.c_int32(0)
        st = Stats()
        code = lib().riga_eigs(self._h, C.byref(o), C.byref(nf), lam.ctypes.data,
                               _ptr(U) if U is not None else None, res.ctypes.data, C.byref(st))
        _check(code, allow=(RIGA_ENOCONV,) if allow_partial else ())
        n = int(nf.value)
        if U is not None:
            U = U[:n]
            if self.hermitian:
                U = torch.view_as_complex(U.reshape(n, self.n_dof // 2, 2))
            U = U.T
        d = st.as_dict()
        d["status"] = code
        return lam[:n], U, res[:n], d

    def eig_grad(self, lam, U, w, stream=None):
        """Gradient of sum_i w_i lam_i w.r.t. (kappa, rho); U: [n_dof, k]
        M-normalised eigenvectors on the device."""
        import torch
        k = len(lam)
        Uc = U.T.contiguous()  # column-major n_dof x k
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float64)
        gk = torch.empty(self.n_elem, dtype=torch.float64, device=self.device)
        gr = torch.empty(self.n_elem, dtype=torch.float64, device=self.device)
        _check(lib().riga_eig_grad(self._h, k, lam.ctypes.data, _ptr(Uc), w.ctypes.data,
                                   _ptr(gk), _ptr(gr), _stream(stream)))
        return gk, gr


    def mode_errors(self, lam, U, modes, nquad=0, stream=None):
        """Eigenfunction errors against the exact Laplace modes
        (riga_mode_errors).  lam [n] ascending; U [n_dof, n] M-normalised
        eigenvectors (as eigs returns them; a NumPy array is copied to the
        device); modes [n_modes, dim], 1-based.  Returns a dict of arrays:
        match, overlap, l2 (EFerr_L2), energy (EFerr_E), ev (EVerr)."""
        import torch
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        if isinstance(U, np.ndarray):
            U = torch.tensor(U, dtype=torch.float64, device=self.device)
        Uc = U.T.contiguous()  # [n][n_dof]
        modes = np.ascontiguousarray(np.atleast_2d(modes), dtype=np.int32)
        nm = modes.shape[0]
        out = {k: np.zeros(nm) for k in ("overlap", "l2", "energy", "ev")}
        match = np.zeros(nm, dtype=np.int32)
        _check(lib().riga_mode_errors(self._h, len(lam), lam.ctypes.data, _ptr(Uc), nm,
                                      modes.ctypes.data, nquad, match.ctypes.data,
                                      out["overlap"].ctypes.data, out["l2"].ctypes.data,
                                      out["energy"].ctypes.data, out["ev"].ctypes.data,
                                      _stream(stream)))
        out["match"] = match.astype(np.int64)
        return out


def project(W, B, x, c=None, noalloc=False, stream=None):
    """One Gram-Schmidt pass (riga_project, or riga_project_noalloc with
    noalloc=True): c = W^T x, x -= B c, with W, B contiguous float64 device
    tensors of shape [m, n] (row i = column i of the n x m block) and x [n]
    updated in place.  Returns c [m] (written into `c` if given)."""
    import torch
    m, n = B.shape
    if W.shape != B.shape or x.shape != (n,) or not (W.is_contiguous() and B.is_contiguous()
                                                     and x.is_contiguous()):
        raise ValueError("W, B: contiguous [m, n]; x: contiguous [n]")
    if c is None:
        c = torch.empty(m, dtype=torch.float64, device=x.device)
    fn = lib().riga_project_noalloc if noalloc else lib().riga_project
    _check(fn(n, m, _ptr(W), _ptr(B), _ptr(x), _ptr(c), _stream(stream)))
    return c


_alloc_keep = None


def set_allocator(alloc=None, free=None):
    """Route the library's device allocations through Python callables
    alloc(nbytes, stream_int) -> device pointer int (0 on failure) and
    free(ptr_int, stream_int); set_allocator() restores hipMalloc/hipFree.
    The callables stay referenced here until replaced (buffers made by a
    replaced hook are still released through it, so keep it alive while
    such problems live: see `keep`)."""
    global _alloc_keep
    if alloc is None:
        _check(lib().riga_set_allocator(None))
        return None

    def _a(ctx, nbytes, stream):
        try:
            return int(alloc(int(nbytes), int(stream or 0))) or None
        except Exception:
            return None

    def _f(ctx, ptr, stream):
        free(int(ptr), int(stream or 0))

    a = Allocator(None, Allocator._fields_[1][1](_a), Allocator._fields_[2][1](_f))
    _check(lib().riga_set_allocator(C.byref(a)))
    _alloc_keep = (a, _a, _f, alloc, free)
    return _alloc_keep


def use_torch_allocator():
    """Route the library's device allocations through torch's caching
    allocator (on the stream the library passes)."""
    import torch

    def alloc(nbytes, stream):
        return torch.cuda.caching_allocator_alloc(nbytes, stream=stream)

    def free(ptr, stream):
        torch.cuda.caching_allocator_delete(ptr)

    return set_allocator(alloc, free)


def exact_eigenvalues(dim, count):
    """The `count` smallest exact eigenvalues of the Dirichlet Laplacian on
    the unit square/cube, ascending with multiplicity (riga_exact_eigenvalues)."""
    out = np.zeros(count)
    _check(lib().riga_exact_eigenvalues(dim, count, out.ctypes.data))
    return out


def _desc(dim, ne, p, s, kappa, rho, nquad, leaf_dofs, stream, keep, potential=None):
    d = MeshDesc()
    d.dim = dim
    if potential is not None:
        pot = list(np.asarray(potential, dtype=np.float64).ravel())
        if len(pot) != dim:
            raise ValueError("potential needs one entry per direction")
        d.hermitian = 1
        for i in range(3):
            d.potential[i] = pot[i] if i < dim else 0.0
    nes = [ne] * dim if np.isscalar(ne) else list(ne)
    for i in range(3):
        d.ne[i] = nes[i] if i < dim else 1
    d.p, d.sep_spacing, d.nquad, d.leaf_dofs = p, s, nquad, leaf_dofs
    d.coeffs_on_device = 0
    for name in ("kappa", "rho"):
        v = kappa if name == "kappa" else rho
        if v is None:
            setattr(d, name, None)
            continue
        if hasattr(v, "is_cuda") and v.is_cuda:
            v = v.contiguous().double()
            d.coeffs_on_device = 1
            keep.append(v)
            setattr(d, name, v.data_ptr())
        else:
            a = np.ascontiguousarray(np.asarray(v, dtype=np.float64))
            keep.append(a)
            setattr(d, name, a.ctypes.data)
    if kappa is not None and rho is not None:
        on_dev = [hasattr(v, "is_cuda") and v.is_cuda for v in (kappa, rho)]
        if on_dev[0] != on_dev[1]:
            raise ValueError("kappa and rho must both be host arrays or both device tensors")
    d.stream = stream
    return d


def analyze(dim, ne, p, s, nquad=0, leaf_dofs=0, potential=None):
    """Host-only analysis (no device needed); `potential` (one entry per
    direction) selects the complex Hermitian (magnetic) pencil."""
    keep = []
    d = _desc(dim, ne, p, s, None, None, nquad, leaf_dofs, None, keep, potential)
    h = C.c_void_p()
    _check(lib().riga_analyze(C.byref(d), C.byref(h)))
    return Problem(h, dim, ne, p, s, None)


def assemble(dim, ne, p, s, kappa=None, rho=None, nquad=0, leaf_dofs=0, device="cuda:0",
             stream=None, potential=None):
    """Analyse and assemble K, M on the device.  `potential` (the constant
    vector potential A, one entry per direction) assembles the complex
    Hermitian pencil of the magnetic Laplacian instead (kappa = rho = 1)."""
    import torch
    dev = torch.device(device)
    with torch.cuda.device(dev):
        keep = []
        d = _desc(dim, ne, p, s, kappa, rho, nquad, leaf_dofs, _stream(stream), keep, potential)
        h = C.c_void_p()
        _check(lib().riga_assemble(C.byref(d), C.byref(h)))
        return Problem(h, dim, ne, p, s, dev)


def eigs(dim, ne, p, s, nev, kappa=None, rho=None, lo=0.0, hi=math.inf, precision=RIGA_FP64,
         **kw):
    pr = assemble(dim, ne, p, s, kappa, rho)
    return pr.eigs(nev, lo=lo, hi=hi, precision=precision, **kw)


def factor_batched(problems, sigmas, precision=RIGA_FP64, allow_singular=False):
    """Factorise K_i - sigma_i M_i of every problem (same device, each once)
    with every tree height of all of them in one launch per kernel; each
    problem keeps its factorisation for solve().  Returns [(inertia, stats)]
    as factor() does for each."""
    n = len(problems)
    if len(sigmas) != n:
        raise ValueError("one shift per problem")
    handles = (C.c_void_p * max(n, 1))(*[p._h for p in problems])
    sg = (C.c_double * max(n, 1))(*[float(x) for x in sigmas])
    neg = (C.c_int64 * max(n, 1))()
    sts = (Stats * max(n, 1))()
    code = lib().riga_factor_batched(handles, n, sg, precision, neg, sts)
    _check(code, allow=(RIGA_ESINGULAR,) if allow_singular else ())
    out = []
    for i in range(n):
        d = sts[i].as_dict()
        d["status"] = RIGA_ESINGULAR if d["n_perturbed_pivots"] > 0 else RIGA_OK
        out.append((int(neg[i]), d))
    return out


def eigs_batched(problems, nev, lo=0.0, hi=math.inf, precision=RIGA_FP64, tol=1e-9, workers=0,
                 per_shift=0, seed=0, vectors=True, allow_partial=False):
    """nev lowest pairs of every problem in `problems` (assembled on the same
    device), solved concurrently.  Returns a list of (lam, U, resid, stats)."""
    import torch
    n = len(problems)
    o = EigsOpts(lo=lo, hi=hi, nev=nev, precision=precision, tol=tol, max_basis=0,
                 max_restarts=0, per_shift=per_shift, seed=seed, stream=None)
    handles = (C.c_void_p * n)(*[p._h for p in problems])
    nf = (C.c_int32 * n)()
    lams = [np.zeros(nev) for _ in range(n)]
    ress = [np.zeros(nev) for _ in range(n)]
    Us = [torch.zeros((nev, p.n_dof), dtype=torch.float64, device=p.device) if vectors else None
          for p in problems]
    ev = (C.c_void_p * n)(*[a.ctypes.data for a in lams])
    rs = (C.c_void_p * n)(*[a.ctypes.data for a in ress])
    uv = (C.c_void_p * n)(*[u.data_ptr() for u in Us]) if vectors else None
    sts = (Stats * n)()
    torch.cuda.synchronize()  # output buffers were filled on torch's stream
    code = lib().riga_eigs_batched(handles, n, C.byref(o), workers, nf, ev, uv, rs, sts)
    _check(code, allow=(RIGA_ENOCONV,) if allow_partial else ())
    out = []
    for i in range(n):
        k = int(nf[i])
        out.append((lams[i][:k], Us[i][:k].T if vectors else None, ress[i][:k], sts[i].as_dict()))
    return out


def _autograd():
    import torch

    class EigSum(torch.autograd.Function):
        """L = sum_i w_i lambda_i(kappa, rho) for the nev lowest eigenvalues;
        backward through the adjoint kernel (riga_eig_grad)."""

        @staticmethod
        def forward(ctx, kappa, rho, w, dim, ne, p, s):
            nev = w.numel()
            pr = assemble(dim, ne, p, s, kappa.detach(), rho.detach(), device=kappa.device)
            # one pair more than the loss uses: a loss that cuts through a
            # multiple eigenvalue has no gradient (the sum depends on which
            # basis of the eigenspace the cut keeps)
            lam, U, _, _ = pr.eigs(min(nev + 1, pr.n_dof))
            if len(lam) > nev:
                a, b = lam[nev - 1], lam[nev]
                if abs(b - a) <= 1e-8 * max(abs(a), abs(b)):
                    raise RigaError(RIGA_EDEGENERATE, "eigenvalues %d and %d are not separated: "
                                    "the loss cuts through a multiple eigenvalue" % (nev - 1, nev))
            lam, U = lam[:nev], U[:, :nev]
            ctx.pr, ctx.U = pr, U
            ctx.lam = lam
            ctx.save_for_backward(w)
            lam_t = torch.as_tensor(lam, dtype=torch.float64, device=kappa.device)
            ctx.lam_t = lam_t
            return (w.to(torch.float64) * lam_t).sum()

        @staticmethod
        def backward(ctx, g):
            (w,) = ctx.saved_tensors
            wg = (w.detach().double() * g.detach().double()).cpu().numpy()
            gk, gr = ctx.pr.eig_grad(ctx.lam, ctx.U, wg)
            # d L / d w_i = lambda_i
            gw = (g.detach().double() * ctx.lam_t).to(w.dtype) if ctx.needs_input_grad[2] else None
            return gk, gr, gw, None, None, None, None

    return EigSum


class _Lazy:
    _cls = None

    def apply(self, *a):
        if _Lazy._cls is None:
            _Lazy._cls = _autograd()
        return _Lazy._cls.apply(*a)


EigSum = _Lazy()
