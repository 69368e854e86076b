"""Python binding of libhelmdefl, the MI355X (gfx950) implementation of the
matrix-free multilevel deflation preconditioner (MADP) inside FGMRES for the
heterogeneous 2-D Helmholtz equation (Chen, Dwarka, Vuik, arXiv 2412.04980).

This module only marshals arguments: every step of the preconditioner and the
solver runs in the library's HIP kernels.  PyTorch provides device memory and
the stream.  The entry points carry the names of the C ABI in include/helmdefl.h:

    cfg = default_config(nx, ny, h)
    prob = create_problem(cfg, k)            # k: torch.float64 on the GPU, nx*ny
    x = precond_apply(prob, v)               # complex128
    u, info = fgmres_solve(prob, b)
    y = apply_operator(prob, level, which, x, sub=0)
    destroy_problem(prob)

    bt = create_batch(cfg, [k0, k1, k2])     # one configuration, several media
    us, infos = batch_solve(bt, [b0, b1, b2])  # lockstep: one launch per sweep
    destroy_batch(bt)

The library is loaded from libhelmdefl.so next to this file (built by
paper_2412_04980_amd.build); importing this module fails loudly when it is
missing.  There is no CPU fallback.
"""
import ctypes
import os

import torch  # loads the HIP runtime first, so the library binds to the same one

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhelmdefl.so")

HM_OK, HM_NOT_CONVERGED = 0, 1
HM_ERR_ARG, HM_ERR_NOMEM, HM_ERR_HIP, HM_ERR_STATE, HM_ERR_BASIS = -1, -2, -3, -4, -5
HM_FP64, HM_MIXED_FP32, HM_MIXED_FP32_ALL = 0, 1, 2
HM_BC_SOMMERFELD, HM_BC_DIRICHLET = 0, 1
HM_ORTH_CLASSICAL, HM_ORTH_MODIFIED = 0, 1

HM_OP_A, HM_OP_M, HM_OP_ZT, HM_OP_Z, HM_OP_VCYCLE, HM_OP_CSLP, HM_OP_PRECOND = range(7)
HM_OP_MG_M, HM_OP_MG_JACOBI, HM_OP_MG_RESTRICT, HM_OP_MG_PROLONG = 7, 8, 9, 10

KIND_LEVEL2, KIND_CSLP, KIND_MG_COARSE, KIND_OUTER = 0, 1, 2, 3

# kernel classes of hm_set_timing / hm_get_timing
HM_TK_CGS_DOT, HM_TK_CGS_UPDATE, HM_TK_WIDE, HM_TK_FIVE_POINT, HM_TK_MGS = range(5)
TIMING_CLASSES = {HM_TK_CGS_DOT: "cgs_dot", HM_TK_CGS_UPDATE: "cgs_update_norm",
                  HM_TK_WIDE: "wide_stencil_apply", HM_TK_FIVE_POINT: "five_point_apply",
                  HM_TK_MGS: "mgs_step"}

EXPORTED = ["hm_default_config", "hm_workspace_bytes", "hm_create_problem", "hm_precond_apply",
            "hm_fgmres_solve", "hm_apply_operator", "hm_level_shape", "hm_set_replay",
            "hm_get_counts", "hm_reset_counts", "hm_set_timing", "hm_get_timing",
            "hm_set_basis_cache", "hm_set_small_krylov", "hm_set_krylov_steps",
            "hm_destroy_problem", "hm_matfree_apply", "hm_csr_assemble", "hm_csr_spmv",
            "hm_batch_workspace_bytes", "hm_create_batch", "hm_batch_solve", "hm_batch_member",
            "hm_destroy_batch", "hm_residual_workspace_bytes", "hm_residual",
            "hm_residual_noalloc",
            "hm_status_string", "hm_last_error"]

MAX_BATCH = 16


class HmConfig(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("h", ctypes.c_double),
                ("bc", ctypes.c_int), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("levels", ctypes.c_int), ("tol_outer", ctypes.c_double),
                ("tol_level2", ctypes.c_double), ("tol_cslp", ctypes.c_double),
                ("maxit_coef", ctypes.c_double), ("outer_restart", ctypes.c_int),
                ("outer_maxit", ctypes.c_int), ("level2_maxit", ctypes.c_int),
                ("mg_nu_pre", ctypes.c_int), ("mg_nu_post", ctypes.c_int),
                ("precision", ctypes.c_int), ("coarse_steps", ctypes.c_int),
                ("tol_levels", ctypes.c_int), ("cslp_orth", ctypes.c_int),
                ("level2_basis", ctypes.c_int), ("reserved", ctypes.c_int * 4)]

    def replace(self, **kw):
        c = HmConfig()
        ctypes.pointer(c)[0] = self
        for key, val in kw.items():
            setattr(c, key, val)
        return c


class HmSolveInfo(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int), ("level2_iters_total", ctypes.c_int),
                ("cslp_iters_total", ctypes.c_int), ("mg_coarse_iters_total", ctypes.c_int),
                ("rel_res_estimate", ctypes.c_double), ("rel_res_true", ctypes.c_double),
                ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class HelmDeflError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("helmdefl status %d: %s" % (status, message))
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libhelmdefl.so is not built (expected at %s); run "
                          "`python paper_2412_04980_amd/build.py`" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P, V, I, D = ctypes.c_void_p, None, ctypes.c_int, ctypes.c_double
    sig = {
        "hm_default_config": (V, [ctypes.POINTER(HmConfig), I, I, D]),
        "hm_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(HmConfig)]),
        "hm_create_problem": (I, [ctypes.POINTER(HmConfig), P, P, ctypes.c_size_t, P,
                                  ctypes.POINTER(P)]),
        "hm_precond_apply": (I, [P, P, P, P]),
        "hm_fgmres_solve": (I, [P, P, P, ctypes.POINTER(HmSolveInfo), P]),
        "hm_apply_operator": (I, [P, I, I, I, P, P, P]),
        "hm_level_shape": (I, [P, I, I, ctypes.POINTER(I), ctypes.POINTER(I)]),
        "hm_set_replay": (I, [P, I, ctypes.POINTER(I), I]),
        "hm_get_counts": (I, [P, I, ctypes.POINTER(I), I, ctypes.POINTER(I)]),
        "hm_reset_counts": (I, [P]),
        "hm_set_timing": (I, [P, ctypes.c_uint, I]),
        "hm_get_timing": (I, [P, I, ctypes.POINTER(D), ctypes.POINTER(D),
                              ctypes.POINTER(ctypes.c_long)]),
        "hm_set_basis_cache": (I, [P, D, D]),
        "hm_set_small_krylov": (I, [P, I]),
        "hm_set_krylov_steps": (I, [P, I]),
        "hm_destroy_problem": (I, [P]),
        "hm_matfree_apply": (I, [I, I, D, P, P, P, P]),
        "hm_csr_assemble": (I, [I, I, D, P, P, P, P, P]),
        "hm_csr_spmv": (I, [I, I, P, P, P, P, P, P]),
        "hm_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(HmConfig), I]),
        "hm_create_batch": (I, [ctypes.POINTER(HmConfig), I, ctypes.POINTER(P), P,
                                ctypes.c_size_t, P, ctypes.POINTER(P)]),
        "hm_batch_solve": (I, [P, ctypes.POINTER(P), ctypes.POINTER(P),
                               ctypes.POINTER(HmSolveInfo), P]),
        "hm_batch_member": (P, [P, I]),
        "hm_destroy_batch": (I, [P]),
        "hm_residual_workspace_bytes": (ctypes.c_size_t, []),
        "hm_residual": (I, [I, I, D, I, P, P, P, P, P, P, ctypes.c_size_t, P]),
        "hm_residual_noalloc": (I, [I, I, D, I, P, P, P, P, P, P]),
        "hm_status_string": (ctypes.c_char_p, [I]),
        "hm_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()


class BasisExhausted(HelmDeflError):
    """A level-2 solve needed more basis vectors than the problem reserves
    (config level2_basis): re-create the problem with a larger basis."""


def _check(status):
    if status == HM_ERR_BASIS:
        raise BasisExhausted(status, _lib.hm_last_error().decode())
    if status < 0:
        raise HelmDeflError(status, _lib.hm_last_error().decode())
    return status


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _ordered(x, stream):
    """x was produced on torch's current stream; a call on another stream must
    not read it before that work is done."""
    if stream is not None and stream != torch.cuda.current_stream(x.device):
        stream.wait_stream(torch.cuda.current_stream(x.device))
    return x


def default_config(nx, ny, h, **overrides):
    c = HmConfig()
    _lib.hm_default_config(ctypes.byref(c), int(nx), int(ny), float(h))
    for key, val in overrides.items():
        setattr(c, key, val)
    return c


def workspace_bytes(cfg):
    n = _lib.hm_workspace_bytes(ctypes.byref(cfg))
    if n == 0:
        raise HelmDeflError(HM_ERR_ARG, _lib.hm_last_error().decode())
    return n


class Problem:
    """A problem hierarchy resident in a caller-owned (torch) workspace."""

    def __init__(self, handle, cfg, workspace, device, owned=True):
        self.handle = handle
        self.cfg = cfg
        self.workspace = workspace
        self.device = device
        self.owned = owned          # False: a batch member, freed with its batch
        self.N = cfg.nx * cfg.ny

    def close(self):
        if self.handle:
            if self.owned:
                _lib.hm_destroy_problem(self.handle)
            self.handle = None
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def create_problem(cfg, k, stream=None, workspace=None):
    """k: nodal wavenumber, torch.float64 CUDA tensor with nx*ny entries."""
    if not (k.is_cuda and k.dtype == torch.float64 and k.numel() == cfg.nx * cfg.ny):
        raise ValueError("k must be a float64 GPU tensor with nx*ny entries")
    k = _ordered(k.contiguous(), stream)
    nbytes = workspace_bytes(cfg)
    if workspace is None:
        workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=k.device)
    _same_device(workspace, k.device, "workspace")
    base = workspace.data_ptr()
    off = (-base) % 256
    handle = ctypes.c_void_p()
    _check(_lib.hm_create_problem(ctypes.byref(cfg), _ptr(k), ctypes.c_void_p(base + off),
                                  ctypes.c_size_t(workspace.numel() - off), _stream(stream),
                                  ctypes.byref(handle)))
    return Problem(handle, cfg, workspace, k.device)


def _same_device(x, device, name):
    """The library's kernels take every buffer of a call on one device: the
    problem's (or the call's first buffer's) device."""
    if device is not None and x.device != device:
        raise ValueError("%s is on %s, the call's other buffers on %s" % (name, x.device, device))


def _c128(x, n, name, device=None):
    if not (x.is_cuda and x.dtype == torch.complex128 and x.numel() == n and x.is_contiguous()):
        raise ValueError("%s must be a contiguous complex128 GPU tensor with %d entries" % (name, n))
    _same_device(x, device, name)
    return x


def precond_apply(prob, v, out=None, stream=None):
    _c128(v, prob.N, "v", prob.device)
    x = torch.empty_like(v) if out is None else _c128(out, prob.N, "out", prob.device)
    _check(_lib.hm_precond_apply(prob.handle, _ptr(v), _ptr(x), _stream(stream)))
    return x


def fgmres_solve(prob, b, out=None, stream=None):
    _c128(b, prob.N, "b", prob.device)
    u = torch.empty_like(b) if out is None else _c128(out, prob.N, "out", prob.device)
    info = HmSolveInfo()
    st = _check(_lib.hm_fgmres_solve(prob.handle, _ptr(b), _ptr(u), ctypes.byref(info),
                                     _stream(stream)))
    d = info.as_dict()
    d["status"] = st
    return u, d


def level_shape(prob, level, sub=0):
    nx, ny = ctypes.c_int(), ctypes.c_int()
    _check(_lib.hm_level_shape(prob.handle, level, sub, ctypes.byref(nx), ctypes.byref(ny)))
    return nx.value, ny.value


def apply_operator(prob, level, which, x, sub=0, stream=None):
    """Applies one building block (HM_OP_*) to the complex128 vector x."""
    nin = nout = None
    if which in (HM_OP_A, HM_OP_M, HM_OP_VCYCLE, HM_OP_CSLP, HM_OP_PRECOND):
        nx, ny = level_shape(prob, level)
        nin = nout = nx * ny
    elif which in (HM_OP_ZT, HM_OP_Z):
        f = level_shape(prob, level)
        c = level_shape(prob, level + 1)
        nin, nout = (f[0] * f[1], c[0] * c[1]) if which == HM_OP_ZT else (c[0] * c[1], f[0] * f[1])
    else:
        f = level_shape(prob, level, sub)
        nin = nout = f[0] * f[1]
        if which in (HM_OP_MG_RESTRICT, HM_OP_MG_PROLONG):
            c = level_shape(prob, level, sub + 1)
            if which == HM_OP_MG_RESTRICT:
                nout = c[0] * c[1]
            else:
                nin = c[0] * c[1]
    _c128(x, nin, "x", prob.device)
    out = torch.empty(nout, dtype=torch.complex128, device=x.device)
    _check(_lib.hm_apply_operator(prob.handle, level, sub, which, _ptr(x), _ptr(out),
                                  _stream(stream)))
    return out


def set_replay(prob, kind, counts):
    arr = (ctypes.c_int * max(1, len(counts)))(*counts)
    _check(_lib.hm_set_replay(prob.handle, kind, arr, len(counts)))


def get_counts(prob, kind):
    n = ctypes.c_int()
    _check(_lib.hm_get_counts(prob.handle, kind, None, 0, ctypes.byref(n)))
    arr = (ctypes.c_int * max(1, n.value))()
    _check(_lib.hm_get_counts(prob.handle, kind, arr, n.value, ctypes.byref(n)))
    return list(arr[: n.value])


def reset_counts(prob):
    _check(_lib.hm_reset_counts(prob.handle))


def set_small_krylov(prob, enable=True):
    """Device-resident (one workgroup) GMRES on small coarse levels, on or off."""
    _check(_lib.hm_set_small_krylov(prob.handle, 1 if enable else 0))


KRYLOV_STEPS_MAX = 3


def set_krylov_steps(prob, steps=KRYLOV_STEPS_MAX):
    """Arnoldi steps per two passes over the basis in the Krylov CSLP of FP64
    levels: 1, 2 or KRYLOV_STEPS_MAX (default)."""
    _check(_lib.hm_set_krylov_steps(prob.handle, int(steps)))


def set_basis_cache(prob, basis_bytes=-1.0, recent_bytes=-1.0):
    """Load hints of the Krylov CSLP's Gram-Schmidt passes (negative: default)."""
    _check(_lib.hm_set_basis_cache(prob.handle, float(basis_bytes), float(recent_bytes)))


def set_timing(prob, mask, every=1):
    """Enables HIP-event timing of every `every`-th launch of the kernel classes in
    `mask` (one bit per class); mask 0 turns it off."""
    _check(_lib.hm_set_timing(prob.handle, ctypes.c_uint(mask), int(every)))


def get_timing(prob):
    """{class name: (milliseconds, algorithmic bytes, launches)} of the timed
    launches since set_timing."""
    out = {}
    for cls, name in TIMING_CLASSES.items():
        ms, by, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_long()
        _check(_lib.hm_get_timing(prob.handle, cls, ctypes.byref(ms), ctypes.byref(by),
                                  ctypes.byref(n)))
        out[name] = (ms.value, by.value, n.value)
    return out


def _f64(x, n, name, device=None):
    if not (x.is_cuda and x.dtype == torch.float64 and x.numel() == n and x.is_contiguous()):
        raise ValueError("%s must be a contiguous float64 GPU tensor with %d entries" % (name, n))
    _same_device(x, device, name)
    return x


def _i32(x, n, name, device=None):
    if not (x.is_cuda and x.dtype == torch.int32 and x.numel() == n and x.is_contiguous()):
        raise ValueError("%s must be a contiguous int32 GPU tensor with %d entries" % (name, n))
    _same_device(x, device, name)
    return x


def matfree_apply(nx, ny, h, k, u, out=None, stream=None):
    """v = A u with the 5-point Sommerfeld Helmholtz stencil, no stored matrix."""
    n = nx * ny
    _f64(k, n, "k")
    _c128(u, n, "u", k.device)
    v = torch.empty_like(u) if out is None else _c128(out, n, "out", k.device)
    _check(_lib.hm_matfree_apply(int(nx), int(ny), float(h), _ptr(k), _ptr(u), _ptr(v),
                                 _stream(stream)))
    return v


def csr_assemble(nx, ny, h, k, stream=None):
    """(row_ptr, col_idx, vals) of the same operator, five entries per row."""
    n = nx * ny
    _f64(k, n, "k")
    row_ptr = torch.empty(n + 1, dtype=torch.int32, device=k.device)
    col_idx = torch.empty(5 * n, dtype=torch.int32, device=k.device)
    vals = torch.empty(5 * n, dtype=torch.complex128, device=k.device)
    _check(_lib.hm_csr_assemble(int(nx), int(ny), float(h), _ptr(k), _ptr(row_ptr),
                                _ptr(col_idx), _ptr(vals), _stream(stream)))
    return row_ptr, col_idx, vals


def csr_spmv(row_ptr, col_idx, vals, x, ncols=None, out=None, stream=None):
    """y = A x for a CSR matrix with int32 indices and complex128 values; x has
    ncols entries (default: square, ncols = the number of rows)."""
    nrows = row_ptr.numel() - 1
    ncols = nrows if ncols is None else int(ncols)
    if x.numel() != ncols:
        # the kernel reads x only at column indices below ncols
        raise ValueError("x has %d entries, the matrix %d columns" % (x.numel(), ncols))
    _i32(row_ptr, nrows + 1, "row_ptr")
    nnz = col_idx.numel()
    _i32(col_idx, nnz, "col_idx", row_ptr.device)
    _c128(vals, nnz, "vals", row_ptr.device)
    _c128(x, ncols, "x", row_ptr.device)
    y = torch.empty(nrows, dtype=torch.complex128, device=x.device) if out is None \
        else _c128(out, nrows, "out", row_ptr.device)
    _check(_lib.hm_csr_spmv(int(nrows), ncols, _ptr(row_ptr), _ptr(col_idx), _ptr(vals),
                            _ptr(x), _ptr(y), _stream(stream)))
    return y


def _residual_args(nx, ny, k, b, u, r, norms):
    n = nx * ny
    _f64(k, n, "k")
    _c128(b, n, "b", k.device)
    _c128(u, n, "u", k.device)
    if r is not None:
        _c128(r, n, "r", k.device)
        if r.data_ptr() == u.data_ptr():
            raise ValueError("r must not alias u")
    if norms is None:
        return torch.empty(2, dtype=torch.float64, device=k.device)
    return _f64(norms, 2, "norms", k.device)


def residual(nx, ny, h, k, b, u, bc=HM_BC_SOMMERFELD, r=None, norms=None, workspace=None,
             stream=None):
    """(||b - A u||_2, ||b||_2) on the device as a float64 tensor of 2 (norms, if
    given, receives them); r, if given, receives b - A u (the 5-point operator
    of the finest level)."""
    norms = _residual_args(nx, ny, k, b, u, r, norms)
    nbytes = _lib.hm_residual_workspace_bytes()
    if workspace is None:
        workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=k.device)
    _same_device(workspace, k.device, "workspace")
    base = workspace.data_ptr()
    off = (-base) % 256
    _check(_lib.hm_residual(int(nx), int(ny), float(h), int(bc), _ptr(k), _ptr(b), _ptr(u),
                            None if r is None else _ptr(r), _ptr(norms),
                            ctypes.c_void_p(base + off), ctypes.c_size_t(workspace.numel() - off),
                            _stream(stream)))
    return norms


def residual_noalloc(nx, ny, h, k, b, u, bc=HM_BC_SOMMERFELD, r=None, norms=None, stream=None):
    """As residual(), through the entry point that allocates nothing (the
    reduction uses the library's static scratch array).  norms: an optional
    float64 GPU tensor of 2 that receives the result (else one is made)."""
    out = _residual_args(nx, ny, k, b, u, r, norms)
    _check(_lib.hm_residual_noalloc(int(nx), int(ny), float(h), int(bc), _ptr(k), _ptr(b),
                                    _ptr(u), None if r is None else _ptr(r), _ptr(out),
                                    _stream(stream)))
    return out


def destroy_problem(prob):
    prob.close()


def batch_workspace_bytes(cfg, nb):
    n = _lib.hm_batch_workspace_bytes(ctypes.byref(cfg), int(nb))
    if n == 0:
        raise HelmDeflError(HM_ERR_ARG, _lib.hm_last_error().decode())
    return n


class BatchProblem:
    """nb problems of one configuration solved in lockstep (hm_create_batch)."""

    def __init__(self, handle, cfg, nb, workspace, device):
        self.handle = handle
        self.cfg = cfg
        self.nb = nb
        self.workspace = workspace
        self.device = device
        self.N = cfg.nx * cfg.ny
        self.members = [Problem(ctypes.c_void_p(_lib.hm_batch_member(handle, i)), cfg, workspace,
                                device, owned=False) for i in range(nb)]

    def close(self):
        if self.handle:
            for m in self.members:
                m.close()
            _lib.hm_destroy_batch(self.handle)
            self.handle = None
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def create_batch(cfg, ks, stream=None, workspace=None):
    """ks: one nodal wavenumber per member (float64 GPU tensors, nx*ny each)."""
    nb = len(ks)
    if nb == 0:
        raise ValueError("a batch needs at least one member")
    n = cfg.nx * cfg.ny
    dev = ks[0].device
    ks = [_ordered(_f64(k.contiguous(), n, "k[%d]" % i, dev), stream) for i, k in enumerate(ks)]
    nbytes = batch_workspace_bytes(cfg, nb)
    if workspace is None:
        workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    _same_device(workspace, dev, "workspace")
    base = workspace.data_ptr()
    off = (-base) % 256
    arr = (ctypes.c_void_p * nb)(*[k.data_ptr() for k in ks])
    handle = ctypes.c_void_p()
    _check(_lib.hm_create_batch(ctypes.byref(cfg), nb, arr, ctypes.c_void_p(base + off),
                                ctypes.c_size_t(workspace.numel() - off), _stream(stream),
                                ctypes.byref(handle)))
    return BatchProblem(handle, cfg, nb, workspace, ks[0].device)


def batch_solve(bt, bs, outs=None, stream=None):
    """Solves member i's system with right-hand side bs[i]; returns (solutions,
    infos), infos[i] as for fgmres_solve with the batch status under "status"."""
    if len(bs) != bt.nb or (outs is not None and len(outs) != bt.nb):
        raise ValueError("need one right-hand side (and output) per member")
    bs = [_c128(b, bt.N, "b[%d]" % i, bt.device) for i, b in enumerate(bs)]
    us = [torch.empty_like(b) for b in bs] if outs is None else \
        [_c128(u, bt.N, "out[%d]" % i, bt.device) for i, u in enumerate(outs)]
    barr = (ctypes.c_void_p * bt.nb)(*[b.data_ptr() for b in bs])
    uarr = (ctypes.c_void_p * bt.nb)(*[u.data_ptr() for u in us])
    infos = (HmSolveInfo * bt.nb)()
    st = _check(_lib.hm_batch_solve(bt.handle, barr, uarr, infos, _stream(stream)))
    out = []
    for i in range(bt.nb):
        d = infos[i].as_dict()
        d["status"] = st
        out.append(d)
    return us, out


def destroy_batch(bt):
    bt.close()


def status_string(status):
    return _lib.hm_status_string(status).decode()
