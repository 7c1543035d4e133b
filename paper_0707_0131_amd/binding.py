"""ctypes binding of libeigcg.so: argument marshalling only.

Every function mirrors an ``extern "C"`` entry point of ``include/eigcg.h``
with the same name.  Device buffers are PyTorch tensors (complex128 on a HIP
device, boundary layout ``[nrhs][Lt][Lz][Ly][Lx][4][3]`` for spinors and
``[Lt][Lz][Ly][Lx][4][3][3]`` for links); the binding passes their data
pointers and torch's current stream.  No computation happens here: if the
library is missing the import of the binding fails loudly.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libeigcg.so")

EIGCG_OK, EIGCG_EINVAL, EIGCG_ENOMEM, EIGCG_ENOTCONV = 0, -1, -2, -3
STENCIL_VARIANTS = 15
EIGCG_EBREAKDOWN, EIGCG_EHIP, EIGCG_EBUSY = -4, -5, -6
EIGCG_FP64, EIGCG_MIXED_FP32, EIGCG_MIXED_HALF = 0, 1, 2
EIGCG_MODE_CG, EIGCG_MODE_EIGCG, EIGCG_MODE_INITCG, EIGCG_MODE_AUTO = 0, 1, 2, 3
EIGCG_OP_M, EIGCG_OP_MDAG, EIGCG_OP_A, EIGCG_OP_INNER = 0, 1, 2, 3
EIGCG_PRECOND_NONE, EIGCG_PRECOND_SPECTRAL = 0, 1
EIGCG_RESTART_FIXED, EIGCG_RESTART_DYNAMIC = 0, 1
EIGCG_BICG_GAMMA5, EIGCG_BICG_DEFLATE, EIGCG_BICG_GUESS_ONLY = 1, 2, 4

STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "ENOTCONV", -4: "EBREAKDOWN",
                -5: "EHIP", -6: "EBUSY"}


class Params(ctypes.Structure):
    _fields_ = [
        ("dims", ctypes.c_int32 * 4),
        ("mass", ctypes.c_double),
        ("nev", ctypes.c_int32),
        ("m", ctypes.c_int32),
        ("max_bank", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("max_batch", ctypes.c_int32),
        ("reliable_every", ctypes.c_int32),
        ("max_iter", ctypes.c_int32),
        ("restart_tol", ctypes.c_double),
        ("hbm_budget", ctypes.c_uint64),
        ("compress_links", ctypes.c_int32),
        ("check_every", ctypes.c_int32),
        ("use_graphs", ctypes.c_int32),
        ("stencil_variant", ctypes.c_int32),
        ("plane_pad", ctypes.c_int32),
        ("sample_every", ctypes.c_int32),
        ("schur", ctypes.c_int32),
        ("precond", ctypes.c_int32),
        ("precond_sigma", ctypes.c_double),
        ("restart_rule", ctypes.c_int32),
        ("restart_cost", ctypes.c_double),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32),
        ("restarts", ctypes.c_int32),
        ("outer_steps", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("true_rel_res", ctypes.c_double),
        ("seconds", ctypes.c_double),
        ("bank_added", ctypes.c_int32),
        ("nritz", ctypes.c_int32),
        ("mode_used", ctypes.c_int32),
        ("first_leg_iters", ctypes.c_int32),
        ("restart_tau", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BicgstabStats(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32),
        ("restarts", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("bank_used", ctypes.c_int32),
        ("true_rel_res", ctypes.c_double),
        ("guess_rel_res", ctypes.c_double),
        ("seconds", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_VP = ctypes.c_void_p
_I32 = ctypes.c_int32
_DP = ctypes.POINTER(ctypes.c_double)

# name -> (restype, argtypes), one per declaration of include/eigcg.h
SIGNATURES = {
    "eigcg_default_params": (_I32, [ctypes.POINTER(Params)]),
    "eigcg_create": (_I32, [ctypes.POINTER(Params), _VP, _VP, ctypes.POINTER(_VP)]),
    "eigcg_solve": (_I32, [_VP, _I32, _VP, _VP, ctypes.c_double, _I32, ctypes.POINTER(Stats)]),
    "eigcg_deflate_init": (_I32, [_VP, _I32, _VP, _VP]),
    "eigcg_destroy": (_I32, [_VP]),
    "eigcg_solve_bicgstab": (_I32, [_VP, _I32, _VP, _VP, ctypes.c_double, _I32, _I32,
                                    ctypes.POINTER(BicgstabStats)]),
    "eigcg_apply": (_I32, [_VP, _I32, _I32, _VP, _VP]),
    "eigcg_apply_noalloc": (_I32, [_VP, _I32, _I32, _VP, _VP]),
    "eigcg_noalloc_scratch_bytes": (_I32, [ctypes.POINTER(ctypes.c_uint64)]),
    "eigcg_schur_rhs": (_I32, [_VP, _I32, _VP, _VP]),
    "eigcg_schur_reconstruct": (_I32, [_VP, _I32, _VP, _VP, _VP]),
    "eigcg_bank_info": (_I32, [_VP, ctypes.POINTER(_I32), _DP, _DP]),
    "eigcg_bank_vectors": (_I32, [_VP, _I32, _I32, _VP]),
    "eigcg_bank_load": (_I32, [_VP, _I32, _VP, ctypes.POINTER(_I32)]),
    "eigcg_bank_matrix": (_I32, [_VP, _DP]),
    "eigcg_last_ritz": (_I32, [_VP, _DP, _I32, ctypes.POINTER(_I32)]),
    "eigcg_bank_reset": (_I32, [_VP]),
    "eigcg_bank_truncate": (_I32, [_VP, _I32]),
    "eigcg_bank_lock": (_I32, [_VP, ctypes.c_double, ctypes.POINTER(_I32)]),
    "eigcg_bank_locked": (_I32, [_VP]),
    "eigcg_bank_restore": (_I32, [_VP, _I32, _VP, _DP]),
    "eigcg_memory": (_I32, [_VP, ctypes.POINTER(ctypes.c_uint64)]),
    "eigcg_last_error": (ctypes.c_char_p, [_VP]),
    "eigcg_layout_info": (_I32, [_VP, ctypes.POINTER(_I32)]),
    "eigcg_tune_report": (_I32, [_VP, _DP]),
    "eigcg_tune_cache_reset": (_I32, []),
    "eigcg_time_kernel": (_I32, [_VP, _I32, _I32, _DP]),
    "eigcg_kernel_samples": (_I32, [_VP, _I32, _DP]),
    "eigcg_server_create": (_I32, [ctypes.c_uint64, ctypes.POINTER(_VP)]),
    "eigcg_server_add": (_I32, [_VP, _VP, ctypes.POINTER(_I32)]),
    "eigcg_submit": (_I32, [_VP, _I32, _VP, _VP, ctypes.c_double, ctypes.POINTER(ctypes.c_uint64)]),
    "eigcg_submit_mode": (_I32, [_VP, _I32, _VP, _VP, ctypes.c_double, _I32,
                                 ctypes.POINTER(ctypes.c_uint64)]),
    "eigcg_poll": (_I32, [_VP, ctypes.c_uint64, ctypes.POINTER(Stats)]),
    "eigcg_server_drain": (_I32, [_VP]),
    "eigcg_server_destroy": (_I32, [_VP]),
    "eigcg_debug_mfma_probe": (_I32, [_VP]),
    "eigcg_debug_span": (_I32, [_I32, ctypes.c_uint64, ctypes.c_uint64]),
    "eigcg_debug_gemm": (_I32, [_I32, _I32, ctypes.c_uint64, _I32, _I32, _VP, _VP, _VP, _VP, _VP,
                                ctypes.c_uint64]),
    "eigcg_host_eig_lowest": (_I32, [_I32, _DP, _I32, _DP, _DP]),
    "eigcg_host_qr": (_I32, [_I32, _I32, _DP, _DP, _DP]),
    "eigcg_host_chol_solve": (_I32, [_I32, _DP, _I32, _DP]),
    "eigcg_host_auto_continue": (_I32, [_I32, _I32, _DP, _DP, ctypes.c_double, _I32]),
    "eigcg_restart_model": (_I32, [_I32, _DP, _DP, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, _DP]),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_0707_0131_amd.build`")
    # the device buffers come from PyTorch: load its HIP runtime first so the
    # library binds to the same runtime instance (a second runtime loaded
    # earlier would not see the device PyTorch opened)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


LIB = _load()


class EigcgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(a):
    return a.ctypes.data_as(_DP)


def _check_field(t, what):
    import torch
    if not (t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()):
        raise ValueError(f"{what} must be a contiguous complex128 device tensor")


# Sites of a solver vector and of the lattice, per live context handle (the
# two differ in odd-even contexts, whose vectors hold the even sites only).
# The C ABI takes raw device pointers; sizes are checked here before any call,
# so a mis-sized tensor is refused instead of being read or written past its end.
_GEOM: dict = {}
_SERVERS: dict = {}  # server handle -> {field id: (V, Vfull)}


def _key(h):
    return h.value if isinstance(h, ctypes.c_void_p) else h


def _geom(ctx):
    g = _GEOM.get(_key(ctx))
    if g is None:
        raise ValueError("unknown context: not created by eigcg_create or already destroyed")
    return g


def _check_fields(t, what, sites, count=None):
    """t: a contiguous complex128 device tensor of `count` (default: its
    leading extent) fields of `sites` sites x 12 complex entries."""
    _check_field(t, what)
    if t.dim() < 2:
        raise ValueError(f"{what} needs a leading right-hand-side axis")
    n = t.shape[0] if count is None else count
    if t.numel() != n * 12 * sites:
        raise ValueError(f"{what} holds {t.numel()} complex entries, expected {n} x 12 x {sites}")
    return n


def _same_shape(a, b, what):
    if tuple(a.shape) != tuple(b.shape):
        raise ValueError(f"{what}: shapes {tuple(a.shape)} and {tuple(b.shape)} differ")


_PARAM_NAMES = {name for name, _ in Params._fields_}


def eigcg_default_params(**overrides) -> Params:
    p = Params()
    LIB.eigcg_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        if k == "dims":
            for i in range(4):
                p.dims[i] = int(v[i])
        elif k in _PARAM_NAMES:
            setattr(p, k, v)
        else:
            raise KeyError(f"unknown parameter {k!r}")
    return p


def eigcg_create(params: Params, gauge, stream=None):
    _check_field(gauge, "gauge")
    vfull = 1
    for i in range(4):
        vfull *= max(0, int(params.dims[i]))
    if gauge.numel() != vfull * 4 * 9:
        raise ValueError(f"gauge holds {gauge.numel()} complex entries, expected "
                         f"{vfull} sites x 4 x 3 x 3")
    ctx = ctypes.c_void_p()
    rc = LIB.eigcg_create(ctypes.byref(params), _ptr(gauge), _stream(stream), ctypes.byref(ctx))
    if rc != EIGCG_OK:
        raise EigcgError(rc, "eigcg_create failed: " + eigcg_last_error(None))
    _GEOM[ctx.value] = (vfull // 2 if params.schur else vfull, vfull)
    return ctx


def eigcg_last_error(ctx) -> str:
    msg = LIB.eigcg_last_error(ctx)
    return msg.decode() if msg else ""


def eigcg_destroy(ctx):
    _GEOM.pop(_key(ctx), None)
    return LIB.eigcg_destroy(ctx)


def eigcg_solve(ctx, b, x, tol, mode=EIGCG_MODE_CG):
    """Returns (status, [stats dict per right-hand side])."""
    V, _ = _geom(ctx)
    nrhs = _check_fields(b, "b", V)
    _check_fields(x, "x", V)
    _same_shape(b, x, "b and x")
    st = (Stats * max(1, nrhs))()
    rc = LIB.eigcg_solve(ctx, nrhs, _ptr(b), _ptr(x), float(tol), int(mode), st)
    if rc in (EIGCG_EINVAL, EIGCG_ENOMEM, EIGCG_EHIP):
        raise EigcgError(rc, eigcg_last_error(ctx))
    return rc, [st[i].as_dict() for i in range(nrhs)]


def eigcg_deflate_init(ctx, b, x):
    V, _ = _geom(ctx)
    _check_fields(b, "b", V)
    _check_fields(x, "x", V)
    _same_shape(b, x, "b and x")
    rc = LIB.eigcg_deflate_init(ctx, b.shape[0], _ptr(b), _ptr(x))
    if rc != EIGCG_OK:
        raise EigcgError(rc, eigcg_last_error(ctx))


def eigcg_solve_bicgstab(ctx, b, x, tol, gamma5=True, deflate=True, max_iter=0,
                         guess_only=False):
    """BiCGSTAB on M x = b (gamma5=False) or gamma5 M x = gamma5 b, from the
    guess in x, after the bank's least-squares guess when deflate is set
    (guess_only: stop after it).  Returns (status, [stats dict per right-hand side])."""
    V, _ = _geom(ctx)
    nrhs = _check_fields(b, "b", V)
    _check_fields(x, "x", V)
    _same_shape(b, x, "b and x")
    flags = (EIGCG_BICG_GAMMA5 if gamma5 else 0) | (EIGCG_BICG_DEFLATE if deflate else 0) | \
        (EIGCG_BICG_GUESS_ONLY if guess_only else 0)
    st = (BicgstabStats * max(1, nrhs))()
    rc = LIB.eigcg_solve_bicgstab(ctx, nrhs, _ptr(b), _ptr(x), float(tol), flags,
                                  int(max_iter), st)
    if rc in (EIGCG_EINVAL, EIGCG_ENOMEM, EIGCG_EHIP):
        raise EigcgError(rc, eigcg_last_error(ctx))
    return rc, [st[i].as_dict() for i in range(nrhs)]


def eigcg_apply(ctx, op, inp, out):
    V, _ = _geom(ctx)
    _check_fields(inp, "in", V)
    _check_fields(out, "out", V)
    _same_shape(inp, out, "in and out")
    rc = LIB.eigcg_apply(ctx, int(op), inp.shape[0], _ptr(inp), _ptr(out))
    if rc != EIGCG_OK:
        raise EigcgError(rc, eigcg_last_error(ctx))


def eigcg_apply_noalloc(ctx, op, inp, out):
    """eigcg_apply (FP64 M, M^H or A) without any device allocation: staging
    in the library's fixed scratch array (calls overlapping on one GPU race)."""
    V, _ = _geom(ctx)
    _check_fields(inp, "in", V)
    _check_fields(out, "out", V)
    _same_shape(inp, out, "in and out")
    rc = LIB.eigcg_apply_noalloc(ctx, int(op), inp.shape[0], _ptr(inp), _ptr(out))
    if rc != EIGCG_OK:
        raise EigcgError(rc, eigcg_last_error(ctx))


def eigcg_noalloc_scratch_bytes():
    b = ctypes.c_uint64()
    LIB.eigcg_noalloc_scratch_bytes(ctypes.byref(b))
    return b.value


def eigcg_schur_rhs(ctx, b_full, rhs):
    """rhs (even sites) = Mhat^H (b_e + D_eo b_o / (2 d)) for full-lattice fields b_full."""
    V, Vfull = _geom(ctx)
    if V == Vfull:
        raise EigcgError(EIGCG_EINVAL, "context is not odd-even preconditioned")
    n = _check_fields(b_full, "b_full", Vfull)
    _check_fields(rhs, "rhs", V, n)
    rc = LIB.eigcg_schur_rhs(ctx, b_full.shape[0], _ptr(b_full), _ptr(rhs))
    if rc != EIGCG_OK:
        raise EigcgError(rc, eigcg_last_error(ctx))


def eigcg_schur_reconstruct(ctx, b_full, x_even, x_full):
    """x_full = (x_even, (b_o + D_oe x_even / 2) / d) on the full lattice."""
    V, Vfull = _geom(ctx)
    if V == Vfull:
        raise EigcgError(EIGCG_EINVAL, "context is not odd-even preconditioned")
    n = _check_fields(b_full, "b_full", Vfull)
    _check_fields(x_even, "x_even", V, n)
    _check_fields(x_full, "x_full", Vfull, n)
    rc = LIB.eigcg_schur_reconstruct(ctx, b_full.shape[0], _ptr(b_full), _ptr(x_even),
                                     _ptr(x_full))
    if rc != EIGCG_OK:
        raise EigcgError(rc, eigcg_last_error(ctx))


def eigcg_bank_info(ctx, residuals=False, cap=256):
    l = _I32()
    vals = np.zeros(cap)
    res = np.zeros(cap) if residuals else None
    rc = LIB.eigcg_bank_info(ctx, ctypes.byref(l), _dptr(vals),
                             _dptr(res) if residuals else None)
    if rc != EIGCG_OK:
        raise EigcgError(rc, eigcg_last_error(ctx))
    n = l.value
    return vals[:n].copy(), (res[:n].copy() if residuals else None)


def eigcg_bank_vectors(ctx, first, count, out):
    V, _ = _geom(ctx)
    _check_field(out, "out")
    if out.numel() < int(count) * 12 * V:
        raise ValueError(f"out holds {out.numel()} complex entries, {count} fields need "
                         f"{int(count) * 12 * V}")
    rc = LIB.eigcg_bank_vectors(ctx, int(first), int(count), _ptr(out))
    if rc != EIGCG_OK:
        raise EigcgError(rc, eigcg_last_error(ctx))


def eigcg_bank_load(ctx, vecs):
    V, _ = _geom(ctx)
    _check_fields(vecs, "vectors", V)
    added = _I32()
    rc = LIB.eigcg_bank_load(ctx, vecs.shape[0], _ptr(vecs), ctypes.byref(added))
    if rc != EIGCG_OK:
        raise EigcgError(rc, eigcg_last_error(ctx))
    return added.value


def eigcg_bank_matrix(ctx, l):
    h = np.zeros(2 * l * l)
    rc = LIB.eigcg_bank_matrix(ctx, _dptr(h))
    if rc != EIGCG_OK:
        raise EigcgError(rc, eigcg_last_error(ctx))
    return h.view(np.complex128).reshape(l, l).T.copy()  # column-major -> [row, col]


def eigcg_last_ritz(ctx, cap=4096):
    vals = np.zeros(cap)
    n = _I32()
    LIB.eigcg_last_ritz(ctx, _dptr(vals), cap, ctypes.byref(n))
    return vals[: n.value].copy()


def eigcg_bank_reset(ctx):
    return LIB.eigcg_bank_reset(ctx)


def eigcg_bank_truncate(ctx, k):
    rc = LIB.eigcg_bank_truncate(ctx, int(k))
    if rc != EIGCG_OK:
        raise EigcgError(rc, eigcg_last_error(ctx))


def eigcg_bank_lock(ctx, tol):
    """Lock the bank's Ritz vectors with ||A u - theta u|| <= tol out of
    building H (Section 4); returns the number of locked columns."""
    n = _I32()
    rc = LIB.eigcg_bank_lock(ctx, float(tol), ctypes.byref(n))
    if rc != EIGCG_OK:
        raise EigcgError(rc, eigcg_last_error(ctx))
    return n.value


def eigcg_bank_locked(ctx):
    rc = LIB.eigcg_bank_locked(ctx)
    if rc < 0:
        raise EigcgError(rc, "bad context")
    return rc


def eigcg_bank_restore(ctx, vecs, h):
    """Restore U from l device fields and H (l x l complex, [row, col]) on the host."""
    V, _ = _geom(ctx)
    l = _check_fields(vecs, "vectors", V)
    h = np.asarray(h, dtype=np.complex128)
    if h.shape != (l, l):
        raise ValueError(f"h must be {l} x {l}, got {h.shape}")
    hf = np.ascontiguousarray(h.T)  # column-major
    rc = LIB.eigcg_bank_restore(ctx, l, _ptr(vecs), hf.ctypes.data_as(_DP))
    if rc != EIGCG_OK:
        raise EigcgError(rc, eigcg_last_error(ctx))


def eigcg_memory(ctx):
    b = ctypes.c_uint64()
    LIB.eigcg_memory(ctx, ctypes.byref(b))
    return b.value


def eigcg_layout_info(ctx):
    info = (_I32 * 8)()
    LIB.eigcg_layout_info(ctx, info)
    ms = np.zeros(2 * STENCIL_VARIANTS)
    LIB.eigcg_tune_report(ctx, _dptr(ms))
    return {"sites": info[0], "plane_stride": info[1], "links64_two_rows": bool(info[2]),
            "links32_two_rows": bool(info[3]), "variant64": info[4], "variant32": info[5],
            "cols_per_group64": info[6], "cols_per_group32": info[7],
            "tune_ms64": ms[:STENCIL_VARIANTS].tolist(), "tune_ms32": ms[STENCIL_VARIANTS:].tolist()}


def eigcg_tune_cache_reset():
    return LIB.eigcg_tune_cache_reset()


def eigcg_time_kernel(ctx, what, reps):
    ms = ctypes.c_double()
    rc = LIB.eigcg_time_kernel(ctx, int(what), int(reps), ctypes.byref(ms))
    if rc != EIGCG_OK:
        raise EigcgError(rc, eigcg_last_error(ctx))
    return ms.value


def eigcg_kernel_samples(ctx, reset=False):
    """Sampled stencil pass timings: {"f64": {...}, "f32": {...}} with the
    number of sampled iterations, mean ms of pass 1 and pass 2, mean batch width."""
    out = (ctypes.c_double * 8)()
    rc = LIB.eigcg_kernel_samples(ctx, int(bool(reset)), out)
    if rc != EIGCG_OK:
        raise EigcgError(rc, eigcg_last_error(ctx))
    keys = ("n", "pass1_ms", "pass2_ms", "cols")
    return {"f64": dict(zip(keys, out[0:4])), "f32": dict(zip(keys, out[4:8]))}


# ---- serving ----------------------------------------------------------------

def eigcg_server_create(hbm_budget=0):
    srv = ctypes.c_void_p()
    rc = LIB.eigcg_server_create(ctypes.c_uint64(hbm_budget), ctypes.byref(srv))
    if rc != EIGCG_OK:
        raise EigcgError(rc, "eigcg_server_create failed")
    return srv


def eigcg_server_add(srv, ctx):
    geom = _geom(ctx)
    fid = _I32()
    rc = LIB.eigcg_server_add(srv, ctx, ctypes.byref(fid))
    if rc != EIGCG_OK:
        raise EigcgError(rc, "eigcg_server_add failed")
    _SERVERS.setdefault(_key(srv), {})[fid.value] = geom
    return fid.value


def eigcg_submit(srv, field_id, b, x, tol):
    geom = _SERVERS.get(_key(srv), {}).get(int(field_id))
    if geom is None:
        raise ValueError(f"field {field_id} is not registered with this server")
    _check_fields(b, "b", geom[0], 1)
    _check_fields(x, "x", geom[0], 1)
    t = ctypes.c_uint64()
    rc = LIB.eigcg_submit(srv, int(field_id), _ptr(b), _ptr(x), float(tol), ctypes.byref(t))
    if rc != EIGCG_OK:
        raise EigcgError(rc, "eigcg_submit failed")
    return t.value


def eigcg_submit_mode(srv, field_id, b, x, tol, mode=EIGCG_MODE_INITCG):
    """Enqueue an init-CG (EIGCG_MODE_INITCG) or bank-growing eigCG
    (EIGCG_MODE_EIGCG) request; returns its ticket."""
    geom = _SERVERS.get(_key(srv), {}).get(int(field_id))
    if geom is None:
        raise ValueError(f"field {field_id} is not registered with this server")
    _check_fields(b, "b", geom[0], 1)
    _check_fields(x, "x", geom[0], 1)
    t = ctypes.c_uint64()
    rc = LIB.eigcg_submit_mode(srv, int(field_id), _ptr(b), _ptr(x), float(tol), int(mode),
                               ctypes.byref(t))
    if rc != EIGCG_OK:
        raise EigcgError(rc, "eigcg_submit_mode failed")
    return t.value


def eigcg_poll(srv, ticket):
    st = Stats()
    rc = LIB.eigcg_poll(srv, ctypes.c_uint64(ticket), ctypes.byref(st))
    return rc, st.as_dict()


def eigcg_server_drain(srv):
    return LIB.eigcg_server_drain(srv)


def eigcg_server_destroy(srv):
    _SERVERS.pop(_key(srv), None)
    return LIB.eigcg_server_destroy(srv)


# ---- device probes (test support) ------------------------------------------------

def eigcg_debug_mfma_probe():
    import torch
    out = torch.zeros(1024, dtype=torch.float64, device="cuda:0")
    rc = LIB.eigcg_debug_mfma_probe(_ptr(out))
    if rc != EIGCG_OK:
        raise EigcgError(rc, "probe failed")
    return out.cpu().numpy()


def eigcg_debug_gemm(kind, inp, s=None, r=None, out=None):
    """kind 0: inp (K, n) columns times s (K, N) -> (N, n); kinds 2 / 3: out
    (N, n, device, updated in place and returned) plus / minus that product;
    kind 1: inp^H r -> (K, N).  Tensors are complex128 or complex64 device
    tensors."""
    import torch
    K, n = inp.shape
    prec = 0 if inp.dtype == torch.complex128 else 1
    if kind in (0, 2, 3):
        N = s.shape[1]
        sd = s.to(torch.complex128).t().contiguous()  # column-major (K x N)
        if kind == 0:
            out = torch.zeros((N, n), dtype=inp.dtype, device=inp.device)
        elif (out is None or tuple(out.shape) != (N, n) or out.dtype != inp.dtype
              or not out.is_contiguous() or out.device != inp.device):
            raise ValueError("out must be a contiguous (N, n) tensor like inp")
        rc = LIB.eigcg_debug_gemm(prec, kind, n, K, N, _ptr(inp), None, _ptr(sd), _ptr(out),
                                  None, 0)
    else:
        N = r.shape[0]
        out = torch.zeros((N, K), dtype=torch.complex128, device=inp.device)
        scratch = torch.zeros(1 << 22, dtype=torch.float64, device=inp.device)
        rc = LIB.eigcg_debug_gemm(prec, 1, n, K, N, _ptr(inp), _ptr(r), None, _ptr(out),
                                  _ptr(scratch), scratch.numel())
    if rc != EIGCG_OK:
        raise EigcgError(rc, "debug gemm failed")
    return out.cpu().numpy() if kind != 1 else out.cpu().numpy().T


def eigcg_debug_span(op, addr, nbytes=0):
    """The host-side bounds layer: op 0 registers [addr, addr + nbytes) as an
    allocation, 1 removes it, 2 checks an access (EIGCG_OK or EIGCG_EINVAL)."""
    return LIB.eigcg_debug_span(int(op), ctypes.c_uint64(addr), ctypes.c_uint64(nbytes))


# ---- host linear algebra (no GPU) --------------------------------------------

def eigcg_host_eig_lowest(a: np.ndarray, k: int):
    n = a.shape[0]
    af = np.asfortranarray(a.astype(np.complex128))
    w = np.zeros(n)
    z = np.zeros((n, max(k, 1)), dtype=np.complex128, order="F")
    rc = LIB.eigcg_host_eig_lowest(n, af.ctypes.data_as(_DP), k, _dptr(w),
                                   z.ctypes.data_as(_DP))
    if rc != EIGCG_OK:
        raise EigcgError(rc, "host eigensolver failed")
    return w, z[:, :k]


def eigcg_host_qr(a: np.ndarray):
    m, n = a.shape
    af = np.asfortranarray(a.astype(np.complex128))
    q = np.zeros((m, n), dtype=np.complex128, order="F")
    r = np.zeros((n, n), dtype=np.complex128, order="F")
    rc = LIB.eigcg_host_qr(m, n, af.ctypes.data_as(_DP), q.ctypes.data_as(_DP),
                           r.ctypes.data_as(_DP))
    if rc != EIGCG_OK:
        raise EigcgError(rc, "host QR failed")
    return q, r


def eigcg_host_chol_solve(h: np.ndarray, b: np.ndarray):
    n = h.shape[0]
    hf = np.asfortranarray(h.astype(np.complex128))
    bf = np.asfortranarray(b.astype(np.complex128).reshape(n, -1))
    rc = LIB.eigcg_host_chol_solve(n, hf.ctypes.data_as(_DP), bf.shape[1],
                                   bf.ctypes.data_as(_DP))
    if rc != EIGCG_OK:
        raise EigcgError(rc, "host Cholesky failed")
    return bf.reshape(b.shape)


def eigcg_host_auto_continue(iters, secs, left, iter_ms, bank_room):
    """The automatic mode's rule: True when the next group should run eigCG."""
    it = np.ascontiguousarray(np.asarray(iters, dtype=np.float64))
    sc = np.ascontiguousarray(np.asarray(secs, dtype=np.float64))
    rc = LIB.eigcg_host_auto_continue(len(it), int(left), it.ctypes.data_as(_DP),
                                      sc.ctypes.data_as(_DP), float(iter_ms), int(bank_room))
    if rc < 0:
        raise EigcgError(rc, "bad arguments")
    return rc == 1


def eigcg_restart_model(theta, res, lambda_max, tol, restart_cost):
    """The dynamic init-CG restart threshold on given Ritz values (ascending)
    and residual norms: ``(tau, iterations without, iterations with)``, tau = 0
    for no restart."""
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
    rs = np.ascontiguousarray(np.asarray(res, dtype=np.float64))
    if th.shape != rs.shape or th.ndim != 1:
        raise ValueError("theta and res must be 1-D of one length")
    out = np.zeros(3)
    rc = LIB.eigcg_restart_model(th.size, th.ctypes.data_as(_DP), rs.ctypes.data_as(_DP),
                                 float(lambda_max), float(tol), float(restart_cost),
                                 out.ctypes.data_as(_DP))
    if rc != EIGCG_OK:
        raise EigcgError(rc, "bad restart-model inputs")
    return float(out[0]), float(out[1]), float(out[2])
