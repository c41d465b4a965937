"""ctypes binding of the C ABI in include/nk.h (marshalling only).

Every function here has the name of the C entry point it calls and does no
arithmetic of its own: all work runs in the HIP library ``libnk.so``.  Device
buffers are torch tensors (complex128, canonical layout, on the GPU); torch
supplies the memory and the stream.  If the library is missing, importing
this module still works but every call raises ``NKLibraryMissing``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnk.so")

NK_OK = 0
NK_EINVAL = -1
NK_ENOGAUGE = -2
NK_ENOMEM = -3
NK_EHIP = -4
NK_WARN_NOTCONV = 1
NK_WARN_BREAKDOWN = 2

NK_PREC_FP64 = 0
NK_PREC_FP32 = 1
NK_PREC_FP32_BF16LINKS = 2

NK_RH_NONE = 0
NK_RH_DET = 1
NK_RH_LEARNED = 2

NK_MLP_IN = 16
NK_MLP_HIDDEN = 64
NK_MLP_STEPS = 4
NK_MLP_NTRAIN = 9668
NK_MLP_NPARAMS = 9700

NK_DEFL_MAX = 1024
NK_NOALLOC_MAX_SITES = 65536

NK_INNER_SAME = 0
NK_INNER_ARNOLDI = 1
NK_TWO_PASS_AUTO = 0
NK_TWO_PASS_ON = 1
NK_TWO_PASS_OFF = 2

# every symbol include/nk.h declares
EXPORTS = (
    "nk_sign_params_default",
    "nk_lattice_create",
    "nk_lattice_destroy",
    "nk_gauge_set",
    "nk_gauge_set_device",
    "nk_apply_dw",
    "nk_apply_dw_device",
    "nk_apply_pair_device",
    "nk_spinor_pack_device",
    "nk_spinor_unpack_device",
    "nk_apply_dw_packed_device",
    "nk_apply_pair_packed_device",
    "nk_krylov_basis_device",
    "nk_small_sign",
    "nk_rh_sign",
    "nk_inner_matrix",
    "nk_rh_model_set",
    "nk_rh_features_device",
    "nk_mlp_forward_device",
    "nk_rh_spectral_loss_device",
    "nk_mlp_backward_device",
    "nk_adam_step_device",
    "nk_sign_apply",
    "nk_sign_apply_device",
    "nk_sign_apply_deflated_device",
    "nk_eig_hermitian_device",
    "nk_eig_critical_device",
    "nk_overlap_apply_device",
    "nk_overlap_solve_device",
    "nk_stencil_groups",
    "nk_block_group",
    "nk_rh_tile_force",
    "nk_rh_tile_choice",
    "nk_rh_newton_schulz",
    "nk_stream_device",
    "nk_apply_dw_noalloc_device",
    "nk_last_error",
    "nk_version",
)


class NKError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"nk error {code}: {msg}")
        self.code = code


class NKLibraryMissing(RuntimeError):
    pass


class nk_sign_params(C.Structure):
    _fields_ = [
        ("m_w", C.c_double),
        ("mu", C.c_double),
        ("k", C.c_int32),
        ("ell", C.c_int32),
        ("tol", C.c_double),
        ("nrhs", C.c_int32),
        ("precision", C.c_int32),
        ("rh_scaling", C.c_int32),
        ("two_pass", C.c_int32),
        ("est_delay", C.c_int32),
        ("check_every", C.c_int32),
        ("rh_maxit", C.c_int32),
        ("rh_tol", C.c_double),
        ("ell_per_rhs", C.POINTER(C.c_int32)),
        ("profile", C.c_int32),
        ("block", C.c_int32),
        ("inner", C.c_int32),
    ]


class nk_sign_info(C.Structure):
    _fields_ = [
        ("k_used", C.c_int32),
        ("ell_used", C.c_int32),
        ("rh_iters", C.c_int32),
        ("breakdown_step", C.c_int32),
        ("two_pass", C.c_int32),
        ("pad", C.c_int32),
        ("est", C.c_double),
        ("rh_residual", C.c_double),
        ("t_basis_ms", C.c_double),
        ("t_small_ms", C.c_double),
        ("t_lift_ms", C.c_double),
        ("t_stencil_ms", C.c_double),
        ("t_update_ms", C.c_double),
        ("n_stencil", C.c_int32),
        ("n_update", C.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad"}


_lib = None


def library():
    """Load libnk.so (once); raise NKLibraryMissing if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise NKLibraryMissing(f"{LIB_PATH} is not built; run python -m paper_0910_2918_amd.build")
    # torch ships its own HIP runtime; load it first so that libnk.so binds to
    # the same libamdhip64 instead of pulling a second runtime into the process
    import torch  # noqa: F401

    lib = C.CDLL(LIB_PATH)
    vp, i32, dbl = C.c_void_p, C.c_int32, C.c_double
    P = C.POINTER
    sig = {
        "nk_sign_params_default": (None, [P(nk_sign_params)]),
        "nk_lattice_create": (C.c_int, [P(i32), P(vp)]),
        "nk_lattice_destroy": (C.c_int, [vp]),
        "nk_gauge_set": (C.c_int, [vp, vp]),
        "nk_gauge_set_device": (C.c_int, [vp, vp, vp]),
        "nk_apply_dw": (C.c_int, [vp, dbl, dbl, i32, vp, vp, i32]),
        "nk_apply_dw_device": (C.c_int, [vp, dbl, dbl, i32, vp, vp, i32, vp]),
        "nk_apply_dw_noalloc_device": (C.c_int, [vp, dbl, dbl, i32, vp, vp, i32, vp]),
        "nk_apply_pair_device": (C.c_int, [vp, dbl, dbl, vp, vp, vp, vp, vp]),
        "nk_spinor_pack_device": (C.c_int, [vp, vp, vp, i32, vp]),
        "nk_spinor_unpack_device": (C.c_int, [vp, vp, vp, i32, vp]),
        "nk_apply_dw_packed_device": (C.c_int, [vp, dbl, dbl, i32, vp, vp, vp]),
        "nk_apply_pair_packed_device": (C.c_int, [vp, dbl, dbl, vp, vp, vp, vp, vp]),
        "nk_krylov_basis_device": (C.c_int, [vp, P(nk_sign_params), vp, vp, vp, vp, P(nk_sign_info), vp]),
        "nk_small_sign": (C.c_int, [i32, i32, i32, vp, vp, vp, P(nk_sign_params), vp, P(nk_sign_info)]),
        "nk_rh_sign": (C.c_int, [i32, i32, P(i32), vp, i32, i32, dbl, P(i32)]),
        "nk_inner_matrix": (C.c_int, [i32, i32, i32, vp, vp, vp, vp, vp, vp, P(i32)]),
        "nk_rh_model_set": (C.c_int, [vp]),
        "nk_rh_features_device": (C.c_int, [i32, i32, P(i32), vp, vp, vp]),
        "nk_mlp_forward_device": (C.c_int, [i32, vp, vp, vp, vp, vp]),
        "nk_rh_spectral_loss_device": (C.c_int, [i32, vp, vp, vp, C.c_float, vp, vp, vp]),
        "nk_mlp_backward_device": (C.c_int, [i32, vp, vp, vp, vp, vp, vp, vp]),
        "nk_adam_step_device": (C.c_int, [i32, vp, vp, vp, vp, i32, C.c_float, C.c_float, C.c_float, C.c_float, vp]),
        "nk_sign_apply": (C.c_int, [vp, P(nk_sign_params), vp, vp, P(nk_sign_info)]),
        "nk_sign_apply_device": (C.c_int, [vp, P(nk_sign_params), vp, vp, P(nk_sign_info), vp]),
        "nk_sign_apply_deflated_device": (C.c_int, [vp, P(nk_sign_params), i32, vp, vp, vp, vp, vp,
                                                    P(nk_sign_info), vp]),
        "nk_eig_hermitian_device": (C.c_int, [vp, C.c_double, i32, i32, i32, C.c_double, i32, vp, vp, vp, P(i32),
                                              P(C.c_double), vp]),
        "nk_eig_critical_device": (C.c_int, [vp, C.c_double, C.c_double, i32, i32, i32, C.c_double, i32, vp, vp, vp,
                                             vp, P(i32), P(C.c_double), vp]),
        "nk_overlap_apply_device": (C.c_int, [vp, P(nk_sign_params), i32, i32, vp, vp, vp, vp, vp,
                                              P(nk_sign_info), vp]),
        "nk_overlap_solve_device": (C.c_int, [vp, P(nk_sign_params), i32, vp, vp, vp, C.c_double, i32, vp, vp,
                                              P(i32), P(C.c_double), vp]),
        "nk_stencil_groups": (C.c_int, [vp, i32, i32]),
        "nk_block_group": (C.c_int, [vp, i32]),
        "nk_rh_tile_force": (C.c_int, [i32, i32, i32]),
        "nk_rh_newton_schulz": (C.c_int, [i32]),
        "nk_stream_device": (C.c_int, [i32, C.c_int64, vp, vp, vp, i32, vp]),
        "nk_rh_tile_choice": (C.c_int, [i32, i32, P(i32)]),
        "nk_last_error": (C.c_char_p, []),
        "nk_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(rc: int) -> int:
    if rc < 0:
        raise NKError(rc, nk_last_error())
    return rc


def _stream(stream):
    if stream is None:
        import torch

        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _dptr(t):
    """Device pointer of a contiguous complex128 CUDA tensor."""
    if not t.is_cuda or not t.is_contiguous() or str(t.dtype) != "torch.complex128":
        raise ValueError("expected a contiguous complex128 CUDA tensor")
    return C.c_void_p(t.data_ptr())


def _hptr(a: np.ndarray):
    if a.dtype != np.complex128 or not a.flags["C_CONTIGUOUS"]:
        raise ValueError("expected a C-contiguous complex128 array")
    return C.c_void_p(a.ctypes.data)


def nk_block_group(h, set: int = 0) -> int:
    """Sources per workgroup of the lockstep stencil kernel: set 1, 2 or 4 to fix it (0: query); returns the previous choice."""
    return _check(library().nk_block_group(h, int(set)))


def nk_stencil_groups(h, precision: int = 0, hermitian: bool = False) -> int:
    """Direction groups the autotuner chose for the stencil kernel (0 = not yet tuned)."""
    return _check(library().nk_stencil_groups(h, int(precision), 1 if hermitian else 0))


def nk_stream_device(kind: int, a, b, c, blocks: int, stream=None) -> None:
    """Streaming measurement kernel over a (complex128 CUDA tensor): 0 read-only, 1 copy c = a, 2 triad c = a + b / 2."""
    _check(library().nk_stream_device(int(kind), int(a.numel()), _dptr(a), None if b is None else _dptr(b), _dptr(c),
                                      int(blocks), _stream(stream)))


def nk_rh_newton_schulz(enable: bool) -> bool:
    """Turn the Newton-Schulz tail of the Roberts-Higham iteration (orders > 128) on or off; returns the previous setting."""
    return bool(library().nk_rh_newton_schulz(1 if enable else 0))


def nk_rh_tile_force(rows_per_thread: int = 0, panel_threads: int = 0, update_tile: int = 0) -> None:
    """Fix the blocked inverse's launch shape for later Roberts-Higham calls (all 0: autotune)."""
    _check(library().nk_rh_tile_force(int(rows_per_thread), int(panel_threads), int(update_tile)))


def nk_rh_tile_choice(n: int, batch: int = 1):
    """(panel width, rows per thread, panel threads, tile) the autotuner chose, or None."""
    shape = (C.c_int32 * 4)()
    have = _check(library().nk_rh_tile_choice(int(n), int(batch), shape))
    return tuple(shape) if have else None


def nk_last_error() -> str:
    return library().nk_last_error().decode()


def nk_version() -> str:
    return library().nk_version().decode()


def nk_sign_params_default(**kw) -> nk_sign_params:
    p = nk_sign_params()
    library().nk_sign_params_default(C.byref(p))
    names = {f[0] for f in nk_sign_params._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"nk_sign_params has no field {k!r}")
        if k == "ell_per_rhs":
            arr = (C.c_int32 * len(v))(*[int(e) for e in v])
            p._ell_keep = arr
            p.ell_per_rhs = C.cast(arr, C.POINTER(C.c_int32))
        else:
            setattr(p, k, v)
    return p


def nk_lattice_create(dims) -> C.c_void_p:
    d = (C.c_int32 * 4)(*[int(x) for x in dims])
    h = C.c_void_p()
    _check(library().nk_lattice_create(d, C.byref(h)))
    return h


def nk_lattice_destroy(h) -> None:
    _check(library().nk_lattice_destroy(h))


def nk_gauge_set(h, U: np.ndarray) -> None:
    U = np.ascontiguousarray(U, dtype=np.complex128)
    _check(library().nk_gauge_set(h, _hptr(U)))


def nk_gauge_set_device(h, dU, stream=None) -> None:
    _check(library().nk_gauge_set_device(h, _dptr(dU), _stream(stream)))


def nk_apply_dw(h, m_w: float, mu: float, gamma5: bool, x: np.ndarray, nrhs: int = 1) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.empty_like(x)
    _check(library().nk_apply_dw(h, m_w, mu, 1 if gamma5 else 0, _hptr(x), _hptr(y), nrhs))
    return y


def nk_apply_dw_device(h, m_w: float, mu: float, gamma5: bool, x, y, nrhs: int = 1, stream=None) -> None:
    _check(library().nk_apply_dw_device(h, m_w, mu, 1 if gamma5 else 0, _dptr(x), _dptr(y), nrhs, _stream(stream)))


def nk_apply_dw_noalloc_device(h, m_w: float, mu: float, gamma5: bool, x, y, nrhs: int = 1, stream=None) -> None:
    """nk_apply_dw_device with its temporaries in the library's fixed device array (no allocation)."""
    _check(library().nk_apply_dw_noalloc_device(h, m_w, mu, 1 if gamma5 else 0, _dptr(x), _dptr(y), nrhs,
                                                _stream(stream)))


def nk_apply_pair_device(h, m_w: float, mu: float, v, w, av, adw, stream=None) -> None:
    _check(library().nk_apply_pair_device(h, m_w, mu, _dptr(v), _dptr(w), _dptr(av), _dptr(adw), _stream(stream)))


def nk_spinor_pack_device(h, x, xp, nrhs: int = 1, stream=None) -> None:
    """canonical -> the library's packed FP64 device layout"""
    _check(library().nk_spinor_pack_device(h, _dptr(x), _dptr(xp), nrhs, _stream(stream)))


def nk_spinor_unpack_device(h, xp, x, nrhs: int = 1, stream=None) -> None:
    _check(library().nk_spinor_unpack_device(h, _dptr(xp), _dptr(x), nrhs, _stream(stream)))


def nk_apply_dw_packed_device(h, m_w: float, mu: float, gamma5: bool, xp, yp, stream=None) -> None:
    _check(library().nk_apply_dw_packed_device(h, m_w, mu, 1 if gamma5 else 0, _dptr(xp), _dptr(yp), _stream(stream)))


def nk_apply_pair_packed_device(h, m_w: float, mu: float, vp, wp, avp, adwp, stream=None) -> None:
    _check(library().nk_apply_pair_packed_device(h, m_w, mu, _dptr(vp), _dptr(wp), _dptr(avp), _dptr(adwp),
                                                 _stream(stream)))


def nk_krylov_basis_device(h, params: nk_sign_params, x, stream=None):
    """Returns (alpha, beta, delta, info, rc); complex arrays of length k."""
    k = params.k
    a = np.zeros(k, np.complex128)
    b = np.zeros(k, np.complex128)
    d = np.zeros(k, np.complex128)
    info = nk_sign_info()
    rc = _check(library().nk_krylov_basis_device(h, C.byref(params), _dptr(x), _hptr(a), _hptr(b), _hptr(d),
                                                 C.byref(info), _stream(stream)))
    return a, b, d, info, rc


def nk_small_sign(k: int, ell: int, hermitian: bool, alpha, beta, delta, params: nk_sign_params | None = None):
    """Returns (z, info, rc) for host tridiagonal coefficients (complex arrays, length k)."""
    al = np.zeros(k, np.complex128)
    be = np.zeros(k, np.complex128)
    de = np.zeros(k, np.complex128)
    al[:k] = np.asarray(alpha)[:k]
    nb = min(len(beta), k)
    be[:nb] = np.asarray(beta)[:nb]
    de[:nb] = np.asarray(delta)[:nb]
    z = np.zeros(k, np.complex128)
    info = nk_sign_info()
    pp = C.byref(params) if params is not None else None
    rc = _check(library().nk_small_sign(k, ell, 1 if hermitian else 0, _hptr(al), _hptr(be), _hptr(de), pp, _hptr(z),
                                        C.byref(info)))
    return z, info, rc


def nk_rh_sign(S: np.ndarray, n=None, scaling: int = NK_RH_NONE, maxit: int = 100, tol: float = 1e-13):
    """S: (batch, ld, ld) complex128; returns (sgn S, iterations, rc)."""
    S = np.ascontiguousarray(S, dtype=np.complex128).copy()
    if S.ndim == 2:
        S = S[None]
    batch, ld, _ = S.shape
    nn = (C.c_int32 * batch)(*([ld] * batch if n is None else [int(e) for e in n]))
    it = (C.c_int32 * batch)()
    rc = _check(library().nk_rh_sign(batch, ld, nn, _hptr(S), scaling, maxit, tol, it))
    return S, np.array(list(it)), rc


def nk_inner_matrix(k: int, ell: int, hermitian: bool, alpha, beta, delta):
    """H_ell of the inner projection (Sec. 3); returns (a, b, d, ell_used, rc)."""
    al = np.zeros(k, np.complex128)
    be = np.zeros(k, np.complex128)
    de = np.zeros(k, np.complex128)
    al[:k] = np.asarray(alpha)[:k]
    nb = min(len(beta), k)
    be[:nb] = np.asarray(beta)[:nb]
    de[:nb] = np.asarray(delta)[:nb]
    a = np.zeros(ell, np.complex128)
    b = np.zeros(ell, np.complex128)
    d = np.zeros(ell, np.complex128)
    lu = C.c_int32()
    rc = _check(library().nk_inner_matrix(k, ell, 1 if hermitian else 0, _hptr(al), _hptr(be), _hptr(de), _hptr(a),
                                          _hptr(b), _hptr(d), C.byref(lu)))
    n = lu.value
    return a[:n], b[:n], d[:n], n, rc


def _fptr(t):
    """Device pointer of a contiguous float32 CUDA tensor."""
    if not t.is_cuda or not t.is_contiguous() or str(t.dtype) != "torch.float32":
        raise ValueError("expected a contiguous float32 CUDA tensor")
    return C.c_void_p(t.data_ptr())


def _iptr(t):
    if not t.is_cuda or not t.is_contiguous() or str(t.dtype) != "torch.int32":
        raise ValueError("expected a contiguous int32 CUDA tensor")
    return C.c_void_p(t.data_ptr())


def nk_rh_model_set(params) -> None:
    """Install (float32 array of NK_MLP_NPARAMS) or remove (None) the NK_RH_LEARNED model."""
    if params is None:
        _check(library().nk_rh_model_set(None))
        return
    a = np.ascontiguousarray(params, dtype=np.float32)
    if a.size != NK_MLP_NPARAMS:
        raise ValueError(f"expected {NK_MLP_NPARAMS} parameters")
    _check(library().nk_rh_model_set(C.c_void_p(a.ctypes.data)))


def nk_rh_features_device(S, n, feat, stream=None) -> None:
    """S: (batch, ld, ld) complex128 CUDA tensor; n: host sizes; feat: (batch, 16) float32 CUDA tensor."""
    batch, ld = S.shape[0], S.shape[1]
    nn = (C.c_int32 * batch)(*[int(e) for e in n])
    _check(library().nk_rh_features_device(batch, ld, nn, _dptr(S), _fptr(feat), _stream(stream)))


def nk_mlp_forward_device(params, feat, y, act=None, stream=None) -> None:
    batch = feat.shape[0]
    _check(library().nk_mlp_forward_device(batch, _fptr(params), _fptr(feat), _fptr(y),
                                           None if act is None else _fptr(act), _stream(stream)))


def nk_rh_spectral_loss_device(off, lam, y, gscale, loss, dy, stream=None) -> None:
    batch = y.shape[0]
    _check(library().nk_rh_spectral_loss_device(batch, _iptr(off), _dptr(lam), _fptr(y), float(gscale), _fptr(loss),
                                                _fptr(dy), _stream(stream)))


def nk_mlp_backward_device(params, feat, act, dy, delta, grad, stream=None) -> None:
    batch = feat.shape[0]
    _check(library().nk_mlp_backward_device(batch, _fptr(params), _fptr(feat), _fptr(act), _fptr(dy), _fptr(delta),
                                            _fptr(grad), _stream(stream)))


def nk_adam_step_device(n, params, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None) -> None:
    _check(library().nk_adam_step_device(int(n), _fptr(params), _fptr(grad), _fptr(m), _fptr(v), int(t), float(lr),
                                         float(beta1), float(beta2), float(eps), _stream(stream)))


def nk_sign_apply(h, params: nk_sign_params, x: np.ndarray):
    """Host arrays; returns (y, info, rc)."""
    x = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.empty_like(x)
    info = nk_sign_info()
    rc = _check(library().nk_sign_apply(h, C.byref(params), _hptr(x), _hptr(y), C.byref(info)))
    return y, info, rc


def nk_sign_apply_device(h, params: nk_sign_params, x, y, stream=None):
    """Device tensors; returns (info, rc)."""
    info = nk_sign_info()
    rc = _check(library().nk_sign_apply_device(h, C.byref(params), _dptr(x), _dptr(y), C.byref(info),
                                               _stream(stream)))
    return info, rc


def nk_sign_apply_deflated_device(h, params: nk_sign_params, lam, R, L, x, y, stream=None):
    """Device tensors x, y, R, L (R and L hold m canonical vectors each) and
    host eigenvalues lam (m complex); returns (info, rc)."""
    lam = np.ascontiguousarray(lam, dtype=np.complex128).reshape(-1)
    m = int(lam.size)
    info = nk_sign_info()
    rc = _check(library().nk_sign_apply_deflated_device(h, C.byref(params), m, _hptr(lam), _dptr(R), _dptr(L),
                                                        _dptr(x), _dptr(y), C.byref(info), _stream(stream)))
    return info, rc


def nk_eig_hermitian_device(h, m_w: float, m: int, p: int, degree: int, tol: float, maxit: int, V0, R, stream=None):
    """The m eigenpairs of gamma5 Dw(0) smallest in modulus; V0 holds p start
    vectors, R receives m.  Returns (lam, passes, resid, rc)."""
    lam = np.zeros(int(m), dtype=np.float64)
    it = C.c_int32(0)
    res = C.c_double(0.0)
    rc = _check(library().nk_eig_hermitian_device(h, float(m_w), int(m), int(p), int(degree), float(tol), int(maxit),
                                                  _dptr(V0), C.c_void_p(lam.ctypes.data), _dptr(R), C.byref(it),
                                                  C.byref(res), _stream(stream)))
    return lam, it.value, res.value, rc


def nk_eig_critical_device(h, m_w: float, mu: float, m: int, p: int, degree: int, tol: float, maxit: int, V0, R, L,
                           stream=None):
    """The m eigenpairs of gamma5 Dw(mu) nearest the imaginary axis (right R,
    left L, L^dag R = I); V0 holds p start vectors.  Returns (lam complex
    array, passes, resid, rc)."""
    lam = np.zeros(2 * int(m), dtype=np.float64)
    it = C.c_int32(0)
    res = C.c_double(0.0)
    rc = _check(library().nk_eig_critical_device(h, float(m_w), float(mu), int(m), int(p), int(degree), float(tol),
                                                 int(maxit), _dptr(V0), C.c_void_p(lam.ctypes.data), _dptr(R),
                                                 _dptr(L), C.byref(it), C.byref(res), _stream(stream)))
    return lam[0::2] + 1j * lam[1::2], it.value, res.value, rc


def _defl_args(lam, R, L):
    """(m, lam pointer, R, L pointers, keep-alive) for the optional deflation arguments."""
    if lam is None:
        return 0, None, None, None, None
    lam = np.ascontiguousarray(lam, dtype=np.complex128).reshape(-1)
    return int(lam.size), _hptr(lam), _dptr(R), _dptr(L), lam


def nk_overlap_apply_device(h, params: nk_sign_params, dagger: bool, x, y, stream=None, lam=None, R=None, L=None):
    """y = Dov x or Dov^dag x on device tensors, optionally with the sign
    deflated by the eigenpairs (lam, R, L) of A; returns (info, rc)."""
    m, lp, rp, lvp, keep = _defl_args(lam, R, L)
    info = nk_sign_info()
    rc = _check(library().nk_overlap_apply_device(h, C.byref(params), 1 if dagger else 0, m, lp, rp, lvp, _dptr(x),
                                                  _dptr(y), C.byref(info), _stream(stream)))
    del keep
    return info, rc


def nk_overlap_solve_device(h, params: nk_sign_params, tol: float, maxit: int, b, y, stream=None, lam=None, R=None,
                            L=None):
    """CGNR for Dov y = b on device tensors, optionally deflated; returns
    (iterations, relative residual, rc)."""
    m, lp, rp, lvp, keep = _defl_args(lam, R, L)
    it = C.c_int32(0)
    res = C.c_double(0.0)
    rc = _check(library().nk_overlap_solve_device(h, C.byref(params), m, lp, rp, lvp, float(tol), int(maxit),
                                                  _dptr(b), _dptr(y), C.byref(it), C.byref(res), _stream(stream)))
    del keep
    return it.value, res.value, rc


def sign_apply(lat, x, mu: float = 0.0, k: int = 100, ell: int = 0, tol: float = 0.0, stream=None, **opts):
    """y ~ sgn(gamma5 Dw(mu)) x for a contiguous complex128 CUDA tensor x holding
    nrhs canonical vectors (nrhs = x.numel() / (12 V) of the Lattice lat);
    other nk_sign_params fields as keywords.  Returns (y, info) with y a new
    tensor shaped like x and the return code (0 or a positive warning) in
    info.rc; a negative code raises NKError."""
    import torch

    V = lat.dims[0] * lat.dims[1] * lat.dims[2] * lat.dims[3]
    if x.numel() % (12 * V) != 0:
        raise ValueError(f"x has {x.numel()} entries, not a multiple of 12 V = {12 * V}")
    p = nk_sign_params_default(mu=mu, k=k, ell=ell, tol=tol, nrhs=x.numel() // (12 * V), **opts)
    y = torch.empty_like(x)
    info, rc = nk_sign_apply_device(lat.h, p, x, y, stream)
    info.rc = rc
    return y, info


def sign_apply_deflated(lat, x, lam, R, L, mu: float = 0.0, k: int = 100, ell: int = 0, tol: float = 0.0,
                        stream=None, **opts):
    """sign_apply with the eigenpairs (lam, R, L) treated exactly: lam host
    complex (m,), R and L contiguous complex128 CUDA tensors of m canonical
    vectors each with L^dag R = I.  Returns (y, info) like sign_apply."""
    import torch

    V = lat.dims[0] * lat.dims[1] * lat.dims[2] * lat.dims[3]
    if x.numel() % (12 * V) != 0:
        raise ValueError(f"x has {x.numel()} entries, not a multiple of 12 V = {12 * V}")
    m = int(np.asarray(lam).size)
    if R.numel() != m * 12 * V or L.numel() != m * 12 * V:
        raise ValueError(f"R and L must hold m = {m} vectors of 12 V = {12 * V} entries")
    p = nk_sign_params_default(mu=mu, k=k, ell=ell, tol=tol, nrhs=x.numel() // (12 * V), **opts)
    y = torch.empty_like(x)
    info, rc = nk_sign_apply_deflated_device(lat.h, p, lam, R, L, x, y, stream)
    info.rc = rc
    return y, info


class Lattice:
    """Owns a lattice handle (context manager)."""

    def __init__(self, dims):
        self.dims = tuple(int(d) for d in dims)
        self.h = nk_lattice_create(self.dims)

    def close(self):
        if self.h is not None:
            nk_lattice_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
