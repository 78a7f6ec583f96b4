"""Python binding of libdna (ctypes): argument marshalling only.

Every computation runs in the HIP kernels behind the C ABI declared in
include/dna.h; this module checks tensors, allocates the workspace and the
optional outputs with torch, and passes torch's current HIP stream.  Importing
it raises if libdna.so has not been built (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdna.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1301_3389_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

_i64 = ctypes.c_int64
_p = ctypes.c_void_p
_int = ctypes.c_int
_sz = ctypes.c_size_t

GEMM_TYPES = {"fp32": 0, "bf16": 1, "fp16": 2}

STATUS = {0: "DNA_OK", 1: "DNA_EINVAL", 2: "DNA_EWORKSPACE", 3: "DNA_EDOMAIN",
          4: "DNA_ENONFINITE", 5: "DNA_EHIP", 6: "DNA_EUNSUPPORTED"}


class Opts(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_float), ("alpha", ctypes.c_float),
                ("gemm", ctypes.c_int), ("checked", ctypes.c_int),
                ("rho", ctypes.c_float), ("lam", ctypes.c_float),   # dna_opts.rho, dna_opts.lambda
                ("select", ctypes.c_int)]

SELECT_RULES = {"both": 0, "newton_first": 1}


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


def _decl(name, restype, *argtypes):
    f = getattr(_lib, name)
    f.restype = restype
    f.argtypes = list(argtypes)
    return f


_OP = ctypes.POINTER(Opts)
_lib_default_opts = _decl("dna_default_opts", None, _OP)
_lib_ws = _decl("dna_workspace_bytes", _sz, _i64, _i64, _i64, _OP)
_lib_uws = _decl("dna_unrolled_workspace_bytes", _sz, _i64, _i64, _i64, _OP)
_lib_normalize = _decl("dna_normalize", _int, _int, _p, _p, _i64, _i64, _i64, _OP, _p, _sz, _p)
_lib_update_H = _decl("dna_update_H", _int, _p, _p, _p, _i64, _i64, _i64, _OP, _p, _sz, _p, _p, _p, _p)
_lib_update_W = _decl("dna_update_W", _int, _p, _p, _p, _i64, _i64, _i64, _OP, _p, _sz, _p, _p, _p, _p)
_lib_iterate = _decl("dna_iterate", _int, _p, _p, _p, _i64, _i64, _i64, _int, _OP, _p, _sz, _p)
_lib_iterate_noalloc = _decl("dna_iterate_noalloc", _int, _p, _p, _p, _i64, _i64, _i64, _int, _OP, _p)
class SparseVStruct(ctypes.Structure):
    _fields_ = [("nnz", ctypes.c_int64), ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p),
                ("row_of", ctypes.c_void_p), ("csc_row", ctypes.c_void_p), ("csc_col", ctypes.c_void_p),
                ("csc_pos", ctypes.c_void_p), ("nseg_r", ctypes.c_int64), ("nseg_c", ctypes.c_int64),
                ("segr_start", ctypes.c_void_p), ("segr_ptr", ctypes.c_void_p),
                ("segc_start", ctypes.c_void_p), ("segc_ptr", ctypes.c_void_p)]


_SP = ctypes.POINTER(SparseVStruct)
_lib_sp_ws = _decl("dna_sparse_workspace_bytes", _sz, _i64, _i64, _i64, _SP, _OP)
_lib_sp_H = _decl("dna_sparse_update_H", _int, _SP, _p, _p, _i64, _i64, _i64, _OP, _p, _sz, _p, _p, _p, _p)
_lib_sp_W = _decl("dna_sparse_update_W", _int, _SP, _p, _p, _i64, _i64, _i64, _OP, _p, _sz, _p, _p, _p, _p)
_lib_sp_kl = _decl("dna_sparse_kl_cost", _int, _SP, _p, _p, _i64, _i64, _i64, _OP, _p, _sz, _p, _p)
_lib_sp_mu = _decl("dna_sparse_mu_update", _int, _int, _SP, _p, _p, _i64, _i64, _i64, _OP, _p, _sz, _p)
_lib_sp_mu_it = _decl("dna_sparse_mu_iterate", _int, _SP, _p, _p, _i64, _i64, _i64, _int, _OP, _p, _sz, _p)
_lib_sp_it = _decl("dna_sparse_iterate", _int, _SP, _p, _p, _i64, _i64, _i64, _int, _OP, _p, _sz, _p)
_lib_mu_it = _decl("mu_iterate", _int, _p, _p, _p, _i64, _i64, _i64, _int, _int, _OP, _p, _sz, _p)
_lib_mu = _decl("mu_update", _int, _int, _p, _p, _p, _i64, _i64, _i64, _int, _p, _OP, _p, _sz, _p)
_lib_kl = _decl("kl_cost", _int, _p, _p, _p, _i64, _i64, _i64, _OP, _p, _sz, _p, _p)
_lib_gh = _decl("dna_gradient_hessian", _int, _int, _p, _p, _p, _i64, _i64, _i64, _OP, _p, _p, _p, _sz, _p)
_lib_cand = _decl("dna_candidates", _int, _int, _p, _p, _p, _i64, _i64, _i64, _OP, _p, _p, _p, _sz, _p)
_lib_select = _decl("dna_select", _int, _int, _p, _p, _p, _p, _p, _i64, _i64, _i64, _OP, _p, _p, _p,
                    _p, _sz, _p)
_lib_ufwd = _decl("dna_unrolled_H_fwd", _int, _p, _p, _p, _int, _i64, _i64, _i64, _OP, _p, _p, _p, _sz, _p)
_lib_ubwd = _decl("dna_unrolled_H_bwd", _int, _p, _p, _p, _p, _int, _i64, _i64, _i64, _p, _p, _p, _p,
                  _OP, _p, _sz, _p)
_lib_uaux = _decl("dna_unrolled_aux_bytes", _sz, _i64, _i64, _i64, _int, _OP)
_lib_ufwd_aux = _decl("dna_unrolled_H_fwd_aux", _int, _p, _p, _p, _int, _i64, _i64, _i64, _OP, _p, _p, _p, _sz,
                      _p, _sz, _p)
_lib_ubwd_aux = _decl("dna_unrolled_H_bwd_aux", _int, _p, _p, _p, _p, _int, _i64, _i64, _i64, _p, _p, _p, _p,
                      _OP, _p, _sz, _p, _sz, _p)
_lib_status_string = _decl("dna_status_string", ctypes.c_char_p, _int)
_lib_last_error = _decl("dna_last_error", ctypes.c_char_p)
_lib_prof_enable = _decl("dna_profile_enable", None, _int)
_lib_prof_reset = _decl("dna_profile_reset", None)
_lib_prof_read = _decl("dna_profile_read", _int, ctypes.POINTER(KernelStat), _int)
_lib_build_info = _decl("dna_build_info", ctypes.c_char_p)

EXPORTED = [
    "dna_default_opts", "dna_workspace_bytes", "dna_normalize", "dna_update_H", "dna_update_W",
    "dna_iterate", "dna_iterate_noalloc", "dna_sparse_workspace_bytes", "dna_sparse_update_H", "dna_sparse_update_W",
    "dna_sparse_kl_cost", "dna_sparse_mu_update", "dna_sparse_mu_iterate", "dna_sparse_iterate", "mu_update", "mu_iterate", "kl_cost", "dna_gradient_hessian", "dna_candidates", "dna_select",
    "dna_unrolled_workspace_bytes", "dna_unrolled_H_fwd", "dna_unrolled_H_bwd",
    "dna_unrolled_aux_bytes", "dna_unrolled_H_fwd_aux", "dna_unrolled_H_bwd_aux",
    "dna_status_string", "dna_last_error", "dna_profile_enable", "dna_profile_reset",
    "dna_profile_read", "dna_build_info",
]


class DNAError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


def _check(status):
    if status != 0:
        raise DNAError(status, _lib_last_error().decode())


def make_opts(eps=0.01, alpha=4.0, gemm="fp32", checked=False, rho=0.0, lam=0.0, select="both"):
    """dna_opts: eps, alpha (Sec. 2.3), product type, checked mode, the eq. (2)
    weights rho (sum of W) and lam (lambda, sum of H), and the selection rule
    ("both": Algorithm 1; "newton_first": the damped rule)."""
    o = Opts()
    _lib_default_opts(ctypes.byref(o))
    o.eps = float(eps)
    o.alpha = float(alpha)
    o.gemm = GEMM_TYPES[gemm] if isinstance(gemm, str) else int(gemm)
    o.checked = 1 if checked else 0
    o.rho = float(rho)
    o.lam = float(lam)
    o.select = SELECT_RULES[select] if isinstance(select, str) else int(select)
    return o


def build_info():
    return _lib_build_info().decode()


# --------------------------------------------------------------------------- helpers

def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _mat(x, name, shape=None):
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not x.is_cuda or x.dtype != torch.float32 or not x.is_contiguous() or x.dim() != 2:
        raise ValueError(f"{name} must be a contiguous 2-D float32 tensor on the GPU")
    if shape is not None and tuple(x.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(x.shape)}, expected {tuple(shape)}")
    return x


def _dims(V, W, H):
    N, T = V.shape
    R = W.shape[1]
    _mat(V, "V")
    _mat(W, "W", (N, R))
    _mat(H, "H", (R, T))
    return N, T, R


_ws_cache = {}


def _ws_key(kind):
    # one workspace per device and stream: calls enqueued on different streams
    # may run concurrently, so they must not share scratch memory
    dev = torch.cuda.current_device()
    return dev, torch.cuda.current_stream(dev).cuda_stream, kind


def workspace(N, T, R, opts=None, unrolled=False):
    """Device workspace for an N x T x R problem (cached per device and stream,
    grown to the largest size asked for)."""
    o = opts or make_opts()
    nbytes = (_lib_uws if unrolled else _lib_ws)(N, T, R, ctypes.byref(o))
    key = _ws_key("unrolled" if unrolled else "dense")
    dev = key[0]
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < nbytes:
        buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=f"cuda:{dev}")
        _ws_cache[key] = buf
    return buf, nbytes


def release_workspace():
    _ws_cache.clear()


def _opt_out(flag, n, dtype, device):
    if flag is None or flag is False:
        return None
    if isinstance(flag, torch.Tensor):
        return flag
    return torch.empty(n, dtype=dtype, device=device)


# --------------------------------------------------------------------------- entry points

def normalize(side, W, H, **kw):
    """Algorithm 1 steps 1/29 (side 0) or 16 (side 1), in place."""
    _mat(W, "W")
    N, R = W.shape
    _mat(H, "H", (R, H.shape[1]))
    T = H.shape[1]
    o = make_opts(**kw)
    ws, nb = workspace(N, T, R, o)
    _check(_lib_normalize(int(side), _ptr(W), _ptr(H), N, T, R, ctypes.byref(o), _ptr(ws), ws.numel(),
                          _stream()))


def update_H(V, W, H, *, mask=False, d_sel=False, margin=False, **kw):
    """One DNA update of H in place (Algorithm 1 steps 4-15).
    Returns (mask, d_sel, margin); each is None unless requested."""
    N, T, R = _dims(V, W, H)
    o = make_opts(**kw)
    ws, nb = workspace(N, T, R, o)
    m = _opt_out(mask, T, torch.uint8, V.device)
    d = _opt_out(d_sel, T, torch.float64, V.device)
    g = _opt_out(margin, T, torch.float64, V.device)
    _check(_lib_update_H(_ptr(V), _ptr(W), _ptr(H), N, T, R, ctypes.byref(o), _ptr(ws), ws.numel(),
                         _ptr(m), _ptr(d), _ptr(g), _stream()))
    return m, d, g


def update_W(V, W, H, *, mask=False, d_sel=False, margin=False, **kw):
    """One DNA update of W in place (Algorithm 1 steps 17-28)."""
    N, T, R = _dims(V, W, H)
    o = make_opts(**kw)
    ws, nb = workspace(N, T, R, o)
    m = _opt_out(mask, N, torch.uint8, V.device)
    d = _opt_out(d_sel, N, torch.float64, V.device)
    g = _opt_out(margin, N, torch.float64, V.device)
    _check(_lib_update_W(_ptr(V), _ptr(W), _ptr(H), N, T, R, ctypes.byref(o), _ptr(ws), ws.numel(),
                         _ptr(m), _ptr(d), _ptr(g), _stream()))
    return m, d, g


def iterate(V, W, H, iters, **kw):
    """``iters`` full DNA iterations in place (Algorithm 1 steps 4-29), one
    native call; the normalisations hand their factor sums to the next step."""
    N, T, R = _dims(V, W, H)
    o = make_opts(**kw)
    ws, nb = workspace(N, T, R, o)
    _check(_lib_iterate(_ptr(V), _ptr(W), _ptr(H), N, T, R, int(iters), ctypes.byref(o), _ptr(ws), ws.numel(),
                        _stream()))


def iterate_noalloc(V, W, H, iters, **kw):
    """``iterate`` on the library's own scratch array (dna_iterate_noalloc):
    no workspace is allocated, by torch or by the library."""
    N, T, R = _dims(V, W, H)
    o = make_opts(**kw)
    _check(_lib_iterate_noalloc(_ptr(V), _ptr(W), _ptr(H), N, T, R, int(iters), ctypes.byref(o), _stream()))


def mu_update(side, V, W, H, with_cost=False, **kw):
    """Plain MU update (eq. 11) of H (side 0) or W (side 1), in place.  With
    cost: returns the per-column (row) cost of the input state."""
    N, T, R = _dims(V, W, H)
    o = make_opts(**kw)
    ws, nb = workspace(N, T, R, o)
    d = torch.empty(T if side == 0 else N, dtype=torch.float64, device=V.device) if with_cost else None
    _check(_lib_mu(int(side), _ptr(V), _ptr(W), _ptr(H), N, T, R, 1 if with_cost else 0, _ptr(d),
                   ctypes.byref(o), _ptr(ws), ws.numel(), _stream()))
    return d


def kl_cost(V, W, H, out=None, **kw):
    """Eq. (1) at Z = W H; returns a 1-element float64 device tensor."""
    N, T, R = _dims(V, W, H)
    o = make_opts(**kw)
    ws, nb = workspace(N, T, R, o)
    out = torch.empty(1, dtype=torch.float64, device=V.device) if out is None else out
    _check(_lib_kl(_ptr(V), _ptr(W), _ptr(H), N, T, R, ctypes.byref(o), _ptr(ws), ws.numel(), _ptr(out),
                   _stream()))
    return out


def gradient_hessian(side, V, W, H, **kw):
    """A (eq. 7) and B (eq. 14): R x T for side 0, N x R for side 1."""
    N, T, R = _dims(V, W, H)
    o = make_opts(**kw)
    ws, nb = workspace(N, T, R, o)
    shape = (R, T) if side == 0 else (N, R)
    A = torch.empty(shape, dtype=torch.float32, device=V.device)
    B = torch.empty(shape, dtype=torch.float32, device=V.device)
    _check(_lib_gh(int(side), _ptr(V), _ptr(W), _ptr(H), N, T, R, ctypes.byref(o), _ptr(A), _ptr(B),
                   _ptr(ws), ws.numel(), _stream()))
    return A, B


def candidates(side, V, W, H, **kw):
    """MU and renormalised Newton candidates (steps 6 and 11 / 19 and 24)."""
    N, T, R = _dims(V, W, H)
    o = make_opts(**kw)
    ws, nb = workspace(N, T, R, o)
    shape = (R, T) if side == 0 else (N, R)
    Xmu = torch.empty(shape, dtype=torch.float32, device=V.device)
    Xn = torch.empty(shape, dtype=torch.float32, device=V.device)
    _check(_lib_cand(int(side), _ptr(V), _ptr(W), _ptr(H), N, T, R, ctypes.byref(o), _ptr(Xmu), _ptr(Xn),
                     _ptr(ws), ws.numel(), _stream()))
    return Xmu, Xn


def select(side, V, F, X_mu, X_newton, **kw):
    """Costs of both candidates, selection, kept factor (steps 7-9, 12-15 / 20-28).
    F is the fixed factor: W for side 0, H for side 1."""
    _mat(V, "V")
    N, T = V.shape
    if side == 0:
        R = F.shape[1]
        _mat(F, "W", (N, R))
        shape, L = (R, T), T
    else:
        R = F.shape[0]
        _mat(F, "H", (R, T))
        shape, L = (N, R), N
    _mat(X_mu, "X_mu", shape)
    _mat(X_newton, "X_newton", shape)
    o = make_opts(**kw)
    ws, nb = workspace(N, T, R, o)
    out = torch.empty(shape, dtype=torch.float32, device=V.device)
    m = torch.empty(L, dtype=torch.uint8, device=V.device)
    d = torch.empty(L, dtype=torch.float64, device=V.device)
    g = torch.empty(L, dtype=torch.float64, device=V.device)
    _check(_lib_select(int(side), _ptr(V), _ptr(F), _ptr(X_mu), _ptr(X_newton), _ptr(out), N, T, R,
                       ctypes.byref(o), _ptr(m), _ptr(d), _ptr(g), _ptr(ws), ws.numel(), _stream()))
    return out, m, d, g


# --------------------------------------------------------------------------- unrolled H-solve

def unrolled_forward(V, W, H_init, K, keep_sums=False, **kw):
    """K DNA H-updates with W fixed.  Returns (H_ckpt [K+1,R,T], sel [K,T]), and
    with keep_sums=True also the kept-sums buffer (a uint8 tensor, or None where
    the library keeps none) for unrolled_backward(..., aux=...)."""
    N, T, R = _dims(V, W, H_init)
    o = make_opts(**kw)
    ws, nb = workspace(N, T, R, o, unrolled=True)
    H_ckpt = torch.empty((K + 1, R, T), dtype=torch.float32, device=V.device)
    sel = torch.empty((max(K, 1), T), dtype=torch.uint8, device=V.device)
    aux = None
    if keep_sums:
        ab = int(_lib_uaux(N, T, R, int(K), ctypes.byref(o)))
        if ab > 0:
            aux = torch.empty(ab, dtype=torch.uint8, device=V.device)
    if aux is None:
        _check(_lib_ufwd(_ptr(V), _ptr(W), _ptr(H_init), int(K), N, T, R, ctypes.byref(o), _ptr(H_ckpt),
                         _ptr(sel), _ptr(ws), ws.numel(), _stream()))
    else:
        _check(_lib_ufwd_aux(_ptr(V), _ptr(W), _ptr(H_init), int(K), N, T, R, ctypes.byref(o), _ptr(H_ckpt),
                             _ptr(sel), _ptr(ws), ws.numel(), _ptr(aux), aux.numel(), _stream()))
    if keep_sums:
        return H_ckpt, sel[:K], aux
    return H_ckpt, sel[:K]


def unrolled_backward(V, W, H_ckpt, sel, K, dH_K, want_dH_init=True, aux=None, **kw):
    """Vector-Jacobian product of the K updates: returns (dW, dV, dH_init).
    `aux`: the kept sums of unrolled_forward(..., keep_sums=True) for the same
    inputs (the backward then reads them instead of recomputing them)."""
    N, T = V.shape
    R = W.shape[1]
    _mat(V, "V")
    _mat(W, "W", (N, R))
    if tuple(H_ckpt.shape) != (K + 1, R, T) or not H_ckpt.is_contiguous():
        raise ValueError("H_ckpt must be a contiguous (K+1, R, T) tensor")
    _mat(dH_K, "dH_K", (R, T))
    o = make_opts(**kw)
    ws, nb = workspace(N, T, R, o, unrolled=True)
    dW = torch.empty((N, R), dtype=torch.float32, device=V.device)
    dV = torch.empty((N, T), dtype=torch.float32, device=V.device)
    dH0 = torch.empty((R, T), dtype=torch.float32, device=V.device) if want_dH_init else None
    sel = sel.contiguous()
    if aux is None:
        _check(_lib_ubwd(_ptr(V), _ptr(W), _ptr(H_ckpt), _ptr(sel), int(K), N, T, R, _ptr(dH_K), _ptr(dW),
                         _ptr(dV), _ptr(dH0), ctypes.byref(o), _ptr(ws), ws.numel(), _stream()))
    else:
        _check(_lib_ubwd_aux(_ptr(V), _ptr(W), _ptr(H_ckpt), _ptr(sel), int(K), N, T, R, _ptr(dH_K), _ptr(dW),
                             _ptr(dV), _ptr(dH0), ctypes.byref(o), _ptr(ws), ws.numel(), _ptr(aux), aux.numel(),
                             _stream()))
    return dW, dV, dH0


class DNAUnrolledH(torch.autograd.Function):
    """H_K = K DNA H-updates of H_init with W fixed; differentiable in W, V and
    H_init through the hand-written adjoint (selections frozen at their forward
    values, per-iteration checkpoints of H)."""

    @staticmethod
    def forward(ctx, W, V, H_init, K, eps=0.01, alpha=4.0):
        W, V, H_init = W.detach().contiguous(), V.detach().contiguous(), H_init.detach().contiguous()
        H_ckpt, sel, aux = unrolled_forward(V, W, H_init, K, keep_sums=True, eps=eps, alpha=alpha)
        ctx.save_for_backward(W, V, H_ckpt, sel)
        ctx.aux = aux                     # the forward's kept sums (None where none are kept)
        ctx.K, ctx.eps, ctx.alpha = K, eps, alpha
        return H_ckpt[K].clone()

    @staticmethod
    def backward(ctx, gH):
        W, V, H_ckpt, sel = ctx.saved_tensors
        dW, dV, dH0 = unrolled_backward(V, W, H_ckpt, sel, ctx.K, gH.contiguous().float(),
                                        want_dH_init=ctx.needs_input_grad[2], aux=ctx.aux, eps=ctx.eps,
                                        alpha=ctx.alpha)
        ctx.aux = None
        return (dW if ctx.needs_input_grad[0] else None, dV if ctx.needs_input_grad[1] else None,
                dH0, None, None, None)


def unrolled_h(W, V, H_init, K, eps=0.01, alpha=4.0):
    return DNAUnrolledH.apply(W, V, H_init, K, eps, alpha)


# --------------------------------------------------------------------------- profiling

# --------------------------------------------------------------------------- sparse V

SP_SEG = 64     # entries per segment at most (the header's segment tables)


def _segments(keys, ngroups, nnz):
    """Cut positions 0..nnz-1, whose group keys ascend, into segments of at most
    SP_SEG positions of one group: (start[nseg + 1], group_ptr[ngroups + 1])."""
    import numpy as np
    counts = np.bincount(keys, minlength=ngroups).astype(np.int64)
    first = np.concatenate([[0], np.cumsum(counts)])[:-1]
    nseg_g = (counts + SP_SEG - 1) // SP_SEG
    ptr = np.concatenate([[0], np.cumsum(nseg_g)])
    total = int(ptr[-1])
    grp = np.repeat(np.arange(ngroups), nseg_g)
    within = np.arange(total) - np.repeat(ptr[:-1], nseg_g)
    start = np.concatenate([first[grp] + SP_SEG * within, [nnz]])
    return start.astype(np.int32), ptr.astype(np.int32)


class SparseV:
    """A sparse V (N x T, nonzero values > 0) on the GPU in the layout of
    dna_sparse_v: CSR and CSC orders of the nonzeros and their segment tables,
    built on the host from COO triplets (duplicates are added, explicit zeros
    dropped).  Holds the device arrays; ``.c`` is the struct passed to the ABI."""

    def __init__(self, rows, cols, vals, N, T, device=None):
        import numpy as np
        rows = np.asarray(rows, dtype=np.int64)
        cols = np.asarray(cols, dtype=np.int64)
        vals = np.asarray(vals, dtype=np.float32)
        if rows.shape != cols.shape or rows.shape != vals.shape or rows.ndim != 1:
            raise ValueError("rows, cols and vals must be 1-D arrays of one length")
        if rows.size and (rows.min() < 0 or rows.max() >= N or cols.min() < 0 or cols.max() >= T):
            raise ValueError("an index lies outside the N x T matrix")
        key = rows * T + cols
        order = np.argsort(key, kind="stable")
        key, vals = key[order], vals[order]
        uniq, first = np.unique(key, return_index=True)
        vals = np.add.reduceat(vals, first) if key.size else vals
        keep = vals != 0
        uniq, vals = uniq[keep], vals[keep].astype(np.float32)
        r, c = (uniq // T).astype(np.int32), (uniq % T).astype(np.int32)
        nnz = int(uniq.size)
        pos = np.lexsort((r, c)).astype(np.int32)            # CSR positions in CSC order
        segr_start, segr_ptr = _segments(r, N, nnz)
        segc_start, segc_ptr = _segments(c[pos], T, nnz)
        dev = device or torch.device("cuda", torch.cuda.current_device())
        up = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        self.N, self.T, self.nnz = int(N), int(T), nnz
        self.col_idx, self.val, self.row_of = up(c), up(vals), up(r)
        self.csc_row, self.csc_col, self.csc_pos = up(r[pos]), up(c[pos]), up(pos)
        self.segr_start, self.segr_ptr = up(segr_start), up(segr_ptr)
        self.segc_start, self.segc_ptr = up(segc_start), up(segc_ptr)
        self.c = SparseVStruct(nnz, self.col_idx.data_ptr(), self.val.data_ptr(), self.row_of.data_ptr(),
                               self.csc_row.data_ptr(), self.csc_col.data_ptr(), self.csc_pos.data_ptr(),
                               int(segr_start.size - 1), int(segc_start.size - 1), self.segr_start.data_ptr(),
                               self.segr_ptr.data_ptr(), self.segc_start.data_ptr(), self.segc_ptr.data_ptr())

    @classmethod
    def from_dense(cls, V, device=None):
        """From a dense host array (its nonzero entries)."""
        import numpy as np
        V = np.asarray(V)
        rows, cols = np.nonzero(V)
        return cls(rows, cols, V[rows, cols], V.shape[0], V.shape[1], device=device)


def _sp_dims(V, W, H):
    if not isinstance(V, SparseV):
        raise TypeError("V must be a SparseV")
    N, T = V.N, V.T
    R = W.shape[1]
    _mat(W, "W", (N, R))
    _mat(H, "H", (R, T))
    return N, T, R


def sparse_workspace(V, R, opts):
    nbytes = _lib_sp_ws(V.N, V.T, R, ctypes.byref(V.c), ctypes.byref(opts))
    if nbytes == 0:
        raise DNAError(1, "invalid sparse problem size")
    key = _ws_key("sparse")
    dev = key[0]
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < nbytes:
        buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=f"cuda:{dev}")
        _ws_cache[key] = buf
    return buf, nbytes


def sparse_update_H(V, W, H, *, mask=False, d_sel=False, margin=False, **kw):
    """dna_update_H with a sparse V (SparseV), in place; returns (mask, d_sel, margin)."""
    N, T, R = _sp_dims(V, W, H)
    o = make_opts(**kw)
    ws, nb = sparse_workspace(V, R, o)
    m = _opt_out(mask, T, torch.uint8, W.device)
    d = _opt_out(d_sel, T, torch.float64, W.device)
    g = _opt_out(margin, T, torch.float64, W.device)
    _check(_lib_sp_H(ctypes.byref(V.c), _ptr(W), _ptr(H), N, T, R, ctypes.byref(o), _ptr(ws), ws.numel(),
                     _ptr(m), _ptr(d), _ptr(g), _stream()))
    return m, d, g


def sparse_update_W(V, W, H, *, mask=False, d_sel=False, margin=False, **kw):
    """dna_update_W with a sparse V (SparseV), in place; returns (mask, d_sel, margin)."""
    N, T, R = _sp_dims(V, W, H)
    o = make_opts(**kw)
    ws, nb = sparse_workspace(V, R, o)
    m = _opt_out(mask, N, torch.uint8, W.device)
    d = _opt_out(d_sel, N, torch.float64, W.device)
    g = _opt_out(margin, N, torch.float64, W.device)
    _check(_lib_sp_W(ctypes.byref(V.c), _ptr(W), _ptr(H), N, T, R, ctypes.byref(o), _ptr(ws), ws.numel(),
                     _ptr(m), _ptr(d), _ptr(g), _stream()))
    return m, d, g


def sparse_kl_cost(V, W, H, out=None, **kw):
    """eq. 1 with a sparse V; returns a 1-element float64 device tensor."""
    N, T, R = _sp_dims(V, W, H)
    o = make_opts(**kw)
    ws, nb = sparse_workspace(V, R, o)
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=W.device)
    _check(_lib_sp_kl(ctypes.byref(V.c), _ptr(W), _ptr(H), N, T, R, ctypes.byref(o), _ptr(ws), ws.numel(),
                      _ptr(out), _stream()))
    return out


def sparse_mu_update(side, V, W, H, **kw):
    """mu_update with a sparse V (no cost output), in place."""
    N, T, R = _sp_dims(V, W, H)
    o = make_opts(**kw)
    ws, nb = sparse_workspace(V, R, o)
    _check(_lib_sp_mu(int(side), ctypes.byref(V.c), _ptr(W), _ptr(H), N, T, R, ctypes.byref(o), _ptr(ws),
                      ws.numel(), _stream()))


def sparse_mu_iteration(V, W, H, **kw):
    """One MU iteration with a sparse V (H step, step 16, W step, step 29) as
    separate calls; sparse_mu_iterate runs the same in one call."""
    sparse_mu_update(0, V, W, H, **kw)
    normalize(1, W, H, **kw)
    sparse_mu_update(1, V, W, H, **kw)
    normalize(0, W, H, **kw)


def sparse_mu_iterate(V, W, H, iters, **kw):
    """``iters`` MU iterations with a sparse V in place, one native call."""
    N, T, R = _sp_dims(V, W, H)
    o = make_opts(**kw)
    ws, nb = sparse_workspace(V, R, o)
    _check(_lib_sp_mu_it(ctypes.byref(V.c), _ptr(W), _ptr(H), N, T, R, int(iters), ctypes.byref(o), _ptr(ws),
                         ws.numel(), _stream()))


def sparse_iterate(V, W, H, iters, **kw):
    """``iters`` full DNA iterations with a sparse V, in place."""
    N, T, R = _sp_dims(V, W, H)
    o = make_opts(**kw)
    ws, nb = sparse_workspace(V, R, o)
    _check(_lib_sp_it(ctypes.byref(V.c), _ptr(W), _ptr(H), N, T, R, int(iters), ctypes.byref(o), _ptr(ws),
                      ws.numel(), _stream()))


def sparse_fit(V, W, H, iters, record_kl=False, **kw):
    """Algorithm 1 with a sparse V from step 1, in place; the KL after each
    iteration as a float64 device tensor when ``record_kl`` (index 0 = start;
    eq. 2 with ``rho`` / ``lam`` in ``kw``)."""
    normalize(0, W, H, **kw)
    if not record_kl:
        sparse_iterate(V, W, H, iters, **kw)
        return None
    kls = torch.empty(iters + 1, dtype=torch.float64, device=W.device)
    sparse_kl_cost(V, W, H, out=kls[0:1], **kw)
    for k in range(iters):
        sparse_iterate(V, W, H, 1, **kw)
        sparse_kl_cost(V, W, H, out=kls[k + 1:k + 2], **kw)
    return kls


def profile_enable(on=True):
    _lib_prof_enable(1 if on else 0)


def profile_reset():
    _lib_prof_reset()


def profile_read():
    """{kernel name: (launches, total_ms)} since the last reset (synchronises)."""
    n = _lib_prof_read(None, 0)
    arr = (KernelStat * max(n, 1))()
    n = _lib_prof_read(arr, n)
    return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in range(n)}


# --------------------------------------------------------------------------- drivers

def dna_iteration(V, W, H, **kw):
    """One full DNA iteration of Algorithm 1 (H step, step 16, W step, step 29)
    as four separate entry-point calls; ``iterate`` runs the same in one call."""
    update_H(V, W, H, **kw)
    normalize(1, W, H, **kw)
    update_W(V, W, H, **kw)
    normalize(0, W, H, **kw)


def mu_iterate(V, W, H, iters, with_cost=False, **kw):
    """``iters`` MU iterations in place, one native call (mu_iteration's steps)."""
    N, T, R = _dims(V, W, H)
    o = make_opts(**kw)
    ws, nb = workspace(N, T, R, o)
    _check(_lib_mu_it(_ptr(V), _ptr(W), _ptr(H), N, T, R, int(iters), 1 if with_cost else 0, ctypes.byref(o),
                      _ptr(ws), ws.numel(), _stream()))


def mu_iteration(V, W, H, with_cost=False, **kw):
    """One MU iteration (MU-labelled steps of Algorithm 1)."""
    mu_update(0, V, W, H, with_cost=with_cost, **kw)
    normalize(1, W, H, **kw)
    mu_update(1, V, W, H, with_cost=with_cost, **kw)
    normalize(0, W, H, **kw)


def fit(V, W, H, iters, method="dna", record_kl=False, **kw):
    """Algorithm 1 (method='dna') or MU (method='mu') for ``iters`` iterations,
    in place, starting with step 1.  Returns the KL after each iteration as a
    float64 device tensor when ``record_kl`` (index 0 = start); with ``rho`` or
    ``lam`` in ``kw``, the regularised cost of eq. (2) instead."""
    normalize(0, W, H, **kw)
    kls = torch.empty(iters + 1, dtype=torch.float64, device=V.device) if record_kl else None
    if record_kl:
        kl_cost(V, W, H, out=kls[0:1], **kw)
    if method == "dna" and not record_kl:
        iterate(V, W, H, iters, **kw)
        return None
    if method != "dna" and not record_kl:
        mu_iterate(V, W, H, iters, **kw)
        return None
    for k in range(iters):
        if method == "dna":
            iterate(V, W, H, 1, **kw)
        else:
            mu_iterate(V, W, H, 1, **kw)
        if record_kl:
            kl_cost(V, W, H, out=kls[k + 1:k + 2], **kw)
    return kls
