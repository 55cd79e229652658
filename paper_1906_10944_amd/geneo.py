"""Thin Python binding of libgeneo (ctypes).

Argument marshalling only: every step of the setup and of the solve runs in
the library's HIP kernels.  PyTorch supplies device memory and streams.
The functions carry the names of the C entry points declared in
``include/geneo.h``.  Loading fails loudly when the library is missing.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libgeneo.so")

GENEO_OK = 0
GENEO_PREC_FP64 = 0
GENEO_PREC_MIXED = 1
GENEO_POU_CONSTANT = 0
GENEO_POU_SARKIS = 1
GENEO_ELEM_Q1 = 0
GENEO_ELEM_S20 = 1
GENEO_LOCAL_AUTO = 0
GENEO_LOCAL_TRIANGULAR = 1
GENEO_LOCAL_INVERSE = 2

GENEO_ERR_ARG = 1
GENEO_ERR_OOM = 2
GENEO_ERR_LOCAL_NOT_SPD = 3
GENEO_ERR_EIGEN_NOCONV = 4
GENEO_ERR_COARSE_NOT_SPD = 5
GENEO_ERR_MAXIT = 6
GENEO_ERR_HIP = 7
GENEO_ERR_SHIFT_NOT_SPD = 8

ERRORS = {
    1: "GENEO_ERR_ARG", 2: "GENEO_ERR_OOM", 3: "GENEO_ERR_LOCAL_NOT_SPD",
    4: "GENEO_ERR_EIGEN_NOCONV", 5: "GENEO_ERR_COARSE_NOT_SPD",
    6: "GENEO_ERR_MAXIT", 7: "GENEO_ERR_HIP", 8: "GENEO_ERR_SHIFT_NOT_SPD",
}


class GeneoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code


class Grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("ncomp", C.c_int), ("ne", C.c_int * 3),
                ("h", C.c_double * 3), ("parts", C.c_int * 3), ("ovl", C.c_int),
                ("dirichlet", C.c_int), ("load", C.c_double * 3), ("pou", C.c_int),
                ("element", C.c_int)]


class Q1Sizes(C.Structure):
    _fields_ = [("ndof", C.c_int64), ("nnz", C.c_int64), ("nsub", C.c_int64),
                ("nloc", C.c_int64), ("nnz_loc", C.c_int64), ("nmax", C.c_int64)]


class Csr(C.Structure):
    _fields_ = [("n", C.c_int), ("nnz", C.c_int64), ("rowptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p)]


class Subdomains(C.Structure):
    _fields_ = [("nsub", C.c_int), ("nloc", C.c_int64), ("sub_ptr", C.c_void_p),
                ("sub_idx", C.c_void_p), ("sub_flags", C.c_void_p), ("pou", C.c_void_p)]


class CsrBatch(C.Structure):
    _fields_ = [("rowptr", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p)]


class Opts(C.Structure):
    _fields_ = [("nev", C.c_int), ("tau", C.c_double), ("nev_max", C.c_int),
                ("sigma", C.c_double), ("precision", C.c_int), ("pivot_tol", C.c_double),
                ("eig_tol", C.c_double), ("eig_maxit", C.c_int), ("eig_block", C.c_int),
                ("seed", C.c_uint64), ("coarse", C.c_int), ("eig_stall", C.c_int),
                ("eig_floor", C.c_double), ("eig_cheb", C.c_int), ("symv_tiles", C.c_int),
                ("refine", C.c_int), ("refine_rtol", C.c_double), ("eig_solve", C.c_int),
                ("eig_split", C.c_int), ("envelope", C.c_int), ("shifted_steps", C.c_int),
                ("local_solve", C.c_int), ("tau_sub", C.c_void_p)]


class SetupInfo(C.Structure):
    _fields_ = [("nsub", C.c_int), ("nc", C.c_int), ("fallback_fp64", C.c_int),
                ("eig_sweeps", C.c_int), ("eig_block", C.c_int),
                ("eig_max_resid", C.c_double), ("t_setup_ms", C.c_double),
                ("t_phase_ms", C.c_double * 8), ("bytes_local_factors", C.c_int64),
                ("eig_stalled", C.c_int), ("symv_tiles", C.c_int), ("eig_solve", C.c_int),
                ("eig_split", C.c_int), ("local_solve", C.c_int), ("eig_solve_split", C.c_int)]


class PcgInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("converged", C.c_int), ("relres", C.c_double),
                ("kappa_est", C.c_double), ("t_solve_ms", C.c_double), ("refine_iters", C.c_int),
                ("true_relres", C.c_double)]


_lib = None


def lib():
    """Load libgeneo.so (built in-tree by ``build.py``); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise RuntimeError("libgeneo.so is not built (%s); run "
                           "`python -m paper_1906_10944_amd.build`" % LIBPATH)
    # torch first: its HIP runtime is then the one the library binds to, so
    # that the library and torch share devices, streams and memory
    import torch  # noqa: F401
    L = C.CDLL(LIBPATH)
    vp, i, d, i64 = C.c_void_p, C.c_int, C.c_double, C.c_int64
    L.geneo_strerror.restype = C.c_char_p
    L.geneo_strerror.argtypes = [i]
    L.geneo_last_error.restype = C.c_char_p
    L.geneo_version.restype = C.c_char_p
    L.geneo_default_opts.argtypes = [C.POINTER(Opts)]
    L.geneo_default_opts.restype = None
    L.geneo_q1_sizes.argtypes = [C.POINTER(Grid), C.POINTER(Q1Sizes)]
    L.geneo_q1_thm1_tau.argtypes = [C.POINTER(Grid), vp]
    L.geneo_assemble_q1.argtypes = [C.POINTER(Grid)] + [vp] * 13 + [vp]
    L.geneo_setup.argtypes = [C.POINTER(Csr), C.POINTER(Subdomains), C.POINTER(CsrBatch),
                              C.POINTER(CsrBatch), C.POINTER(Opts), vp, C.POINTER(vp)]
    L.geneo_apply.argtypes = [vp, vp, vp, vp]
    L.geneo_destroy.argtypes = [vp]
    L.geneo_destroy.restype = None
    L.geneo_get_setup_info.argtypes = [vp, C.POINTER(SetupInfo)]
    L.geneo_get_eigenvalues.argtypes = [vp, vp, vp, i]
    L.geneo_get_coarse.argtypes = [vp, vp, vp, i64, vp]
    L.geneo_get_local_precision.argtypes = [vp, vp]
    L.pcg_solve.argtypes = [C.POINTER(Csr), vp, vp, vp, i, d, i, C.POINTER(PcgInfo), vp]
    L.pcg_solve_noalloc.argtypes = [C.POINTER(Csr), vp, vp, vp, i, d, i, C.POINTER(PcgInfo), vp]
    L.geneo_spmv.argtypes = [C.POINTER(Csr), vp, vp, vp]
    for f in ("geneo_q1_sizes", "geneo_q1_thm1_tau", "geneo_assemble_q1", "geneo_setup", "geneo_apply",
              "geneo_get_setup_info", "geneo_get_eigenvalues", "geneo_get_coarse",
              "pcg_solve", "pcg_solve_noalloc", "geneo_spmv"):
        getattr(L, f).restype = i
    _lib = L
    return L


def _check(rc):
    if rc != GENEO_OK:
        raise GeneoError(rc, lib().geneo_last_error().decode())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


# ------------------------------------------------------------------ grids
def grid_from_problem(prob):
    """geneo_grid_t of a ``synth.Problem``."""
    g = Grid()
    g.dim, g.ncomp = prob.dim, prob.ncomp
    for a in range(3):
        g.ne[a] = prob.ne[a] if a < prob.dim else 1
        g.h[a] = prob.h[a] if a < prob.dim else 1.0
        g.parts[a] = prob.parts[a] if a < prob.dim else 1
    g.ovl, g.dirichlet = prob.ovl, prob.dirichlet
    for c in range(prob.ncomp):
        g.load[c] = prob.load[c]
    g.pou = GENEO_POU_SARKIS if getattr(prob, "pou", "constant") == "sarkis" else GENEO_POU_CONSTANT
    g.element = GENEO_ELEM_S20 if getattr(prob, "element", "q1") == "s20" else GENEO_ELEM_Q1
    return g


def geneo_q1_sizes(grid):
    s = Q1Sizes()
    _check(lib().geneo_q1_sizes(C.byref(grid), C.byref(s)))
    return {k: int(getattr(s, k)) for k, _ in Q1Sizes._fields_}


def geneo_q1_thm1_tau(grid, nsub):
    """delta_j / H_j of every subdomain (Thm. 1), a float64 array."""
    t = np.zeros(nsub, dtype=np.float64)
    _check(lib().geneo_q1_thm1_tau(C.byref(grid), t.ctypes.data))
    return t


def with_tau_sub(opts, tau):
    """Options using the per-subdomain thresholds ``tau`` (kept alive with the
    options object until the setup has read them)."""
    arr = np.ascontiguousarray(tau, dtype=np.float64)
    opts._tau_keep = arr
    opts.tau_sub = arr.ctypes.data
    return opts


def geneo_default_opts(**kw):
    o = Opts()
    lib().geneo_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def opts_from_problem(prob, **kw):
    """Options of a ``synth.Problem`` (count or threshold rule, precision)."""
    o = geneo_default_opts()
    if prob.tau is not None:
        o.tau, o.nev_max = prob.tau, prob.nev_max
    else:
        o.nev = prob.nev
    o.precision = GENEO_PREC_MIXED if prob.precision == "mixed" else GENEO_PREC_FP64
    names = {f[0] for f in Opts._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError("geneo_opts_t has no field %r" % k)
        setattr(o, k, v)
    return o


class Q1System:
    """Device arrays written by geneo_assemble_q1 (torch tensors on cuda)."""

    def __init__(self, sizes, device):
        import torch
        s = sizes
        self.sizes = s
        I, D = torch.int32, torch.float64
        self.A_rowptr = torch.empty(s["ndof"] + 1, dtype=I, device=device)
        self.A_col = torch.empty(s["nnz"], dtype=I, device=device)
        self.A_val = torch.empty(s["nnz"], dtype=D, device=device)
        self.b = torch.empty(s["ndof"], dtype=D, device=device)
        self.sub_ptr = torch.empty(s["nsub"] + 1, dtype=I, device=device)
        self.sub_idx = torch.empty(s["nloc"], dtype=I, device=device)
        self.sub_flags = torch.empty(s["nloc"], dtype=torch.uint8, device=device)
        self.pou = torch.empty(s["nloc"], dtype=D, device=device)
        self.loc_rowptr = torch.empty(s["nloc"] + 1, dtype=I, device=device)
        self.loc_col = torch.empty(s["nnz_loc"], dtype=I, device=device)
        self.an_val = torch.empty(s["nnz_loc"], dtype=D, device=device)
        self.ao_val = torch.empty(s["nnz_loc"], dtype=D, device=device)

    def csr(self):
        return Csr(int(self.sizes["ndof"]), int(self.sizes["nnz"]), self.A_rowptr.data_ptr(),
                   self.A_col.data_ptr(), self.A_val.data_ptr())

    def subdomains(self):
        return Subdomains(int(self.sizes["nsub"]), int(self.sizes["nloc"]),
                          self.sub_ptr.data_ptr(), self.sub_idx.data_ptr(),
                          self.sub_flags.data_ptr(), self.pou.data_ptr())

    def neumann(self):
        return CsrBatch(self.loc_rowptr.data_ptr(), self.loc_col.data_ptr(),
                        self.an_val.data_ptr())

    def overlap(self):
        return CsrBatch(self.loc_rowptr.data_ptr(), self.loc_col.data_ptr(),
                        self.ao_val.data_ptr())


def geneo_assemble_q1(grid, coeff, device="cuda", stream=None):
    """Assemble a structured Q1 problem on the device; ``coeff`` is a float64
    tensor or array (nelem or nelem*21)."""
    import torch
    sizes = geneo_q1_sizes(grid)
    sysm = Q1System(sizes, device)
    if isinstance(coeff, torch.Tensor):
        coeff = coeff.to(device=device, dtype=torch.float64).contiguous()
    else:
        coeff = torch.as_tensor(np.ascontiguousarray(coeff), dtype=torch.float64).to(device)
    sysm.coeff = coeff
    args = [sysm.A_rowptr, sysm.A_col, sysm.A_val, sysm.b, sysm.sub_ptr, sysm.sub_idx,
            sysm.sub_flags, sysm.pou, sysm.loc_rowptr, sysm.loc_col, sysm.an_val, sysm.ao_val]
    _check(lib().geneo_assemble_q1(C.byref(grid), _ptr(coeff), *[_ptr(a) for a in args],
                                   _stream(stream)))
    return sysm


# ----------------------------------------------------------- preconditioner
class Handle:
    def __init__(self, h, keep):
        self.h = h
        self._keep = keep

    def __del__(self):
        self.close()

    def close(self):
        if getattr(self, "h", None):
            lib().geneo_destroy(self.h)
            self.h = None

    @property
    def value(self):
        if not self.h:
            raise RuntimeError("handle destroyed")
        return self.h


def geneo_setup(A, subs, An, Ao, opts=None, stream=None):
    h = C.c_void_p()
    _check(lib().geneo_setup(C.byref(A), C.byref(subs), C.byref(An) if An is not None else None,
                             C.byref(Ao) if Ao is not None else None,
                             C.byref(opts) if opts is not None else None, _stream(stream),
                             C.byref(h)))
    return Handle(h, None)


def geneo_apply(handle, r, z, stream=None):
    _check(lib().geneo_apply(handle.value, _ptr(r), _ptr(z), _stream(stream)))


def geneo_destroy(handle):
    handle.close()


def geneo_trim():
    """Return the device blocks the library keeps for reuse to the driver."""
    _check(lib().geneo_trim())


def geneo_get_setup_info(handle):
    info = SetupInfo()
    _check(lib().geneo_get_setup_info(handle.value, C.byref(info)))
    out = {k: getattr(info, k) for k, _ in SetupInfo._fields_ if k != "t_phase_ms"}
    out["t_phase_ms"] = list(info.t_phase_ms)
    return out


def geneo_get_eigenvalues(handle, nsub, ldl=64):
    m = np.zeros(nsub, dtype=np.int32)
    lam = np.zeros((nsub, ldl), dtype=np.float64)
    _check(lib().geneo_get_eigenvalues(handle.value, m.ctypes.data, lam.ctypes.data, ldl))
    return m, lam


def geneo_get_local_precision(handle, nsub):
    """1 where subdomain j's local inverse is FP64, 0 where it is FP32."""
    f = np.zeros(nsub, dtype=np.int32)
    _check(lib().geneo_get_local_precision(handle.value, f.ctypes.data))
    return f


def geneo_get_coarse(handle, nsub, with_ah=True):
    zoff = np.zeros(nsub + 1, dtype=np.int64)
    _check(lib().geneo_get_coarse(handle.value, zoff.ctypes.data, None, 0, None))
    z = np.zeros(max(int(zoff[-1]), 1), dtype=np.float64)
    info = geneo_get_setup_info(handle)
    nc = info["nc"]
    ah = np.zeros((max(nc, 1), max(nc, 1)), dtype=np.float64) if with_ah else None
    _check(lib().geneo_get_coarse(handle.value, zoff.ctypes.data, z.ctypes.data, z.size,
                                  ah.ctypes.data if ah is not None else None))
    return zoff, z, (ah[:nc, :nc] if ah is not None else None)


def pcg_solve(A, handle, b, x, rtol=1e-10, maxit=2000, nrhs=1, stream=None, check=True):
    infos = (PcgInfo * nrhs)()
    rc = lib().pcg_solve(C.byref(A), handle.value, _ptr(b), _ptr(x), nrhs, rtol, maxit, infos,
                         _stream(stream))
    out = [{k: getattr(inf, k) for k, _ in PcgInfo._fields_} for inf in infos]
    if check and rc not in (GENEO_OK,):
        _check(rc)
    return out if nrhs > 1 else out[0]


def pcg_solve_noalloc(A, handle, b, x, rtol=1e-10, maxit=2000, nrhs=1, stream=None, check=True):
    """pcg_solve with the library's fixed device work array (no allocation)."""
    infos = (PcgInfo * nrhs)()
    rc = lib().pcg_solve_noalloc(C.byref(A), handle.value, _ptr(b), _ptr(x), nrhs, rtol, maxit,
                                 infos, _stream(stream))
    out = [{k: getattr(inf, k) for k, _ in PcgInfo._fields_} for inf in infos]
    if check and rc not in (GENEO_OK,):
        _check(rc)
    return out if nrhs > 1 else out[0]


def geneo_spmv(A, x, y, stream=None):
    _check(lib().geneo_spmv(C.byref(A), _ptr(x), _ptr(y), _stream(stream)))


def geneo_strerror(code):
    return lib().geneo_strerror(code).decode()


def geneo_version():
    return lib().geneo_version().decode()
