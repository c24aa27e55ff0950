"""ctypes binding of include/pf.h (argument marshalling only).

Every function here forwards to the C ABI of ``libpfx.so``; every step of
an extraction runs in the library's HIP kernels.  Tensors are torch device
tensors used only as device memory; matrices are column-major, i.e. a
tensor ``T`` of shape (rows, cols) with ``T.stride(0) == 1`` and leading
dimension ``T.stride(1)`` (``torch.empty(cols, ld).t()[:rows]`` makes one).
Importing this module raises if the library has not been built.
"""
import ctypes
import os

# torch first: its HIP runtime must be the one libpfx.so binds to.  Loading
# the library before torch would bring in a second libamdhip64 (the ROCm
# install's, found through the library's RUNPATH) next to torch's own.
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpfx.so")

PF_OK, PF_ERR_ARG, PF_ERR_NOMEM, PF_ERR_DEVICE, PF_ERR_BREAKDOWN, PF_ERR_NOCONV, PF_ERR_NONFINITE, \
    PF_ERR_BUSY, PF_ERR_UNSUPPORTED = range(9)
PF_F64, PF_F32, PF_BF16, PF_F8E4M3 = range(4)
PF_OP_SYM, PF_OP_GRAM = range(2)
PF_FLAG_NO_PREROTATE = 0x1
PF_FLAG_SCALED = 0x2
PF_FLAG_COLD = 0x4
PF_FLAG_NATIVE_F32 = 0x8
PF_FLAG_OPERATOR_UNCHANGED = 0x10
PF_FLAG_REORTH = 0x20
PF_PROF_FILTER, PF_PROF_FILTER_REDUCE, PF_PROF_RR, PF_PROF_EXTRACT, PF_PROF_FILTER_PRODUCT = range(5)
PF_PROF_MODE_PRODUCT = 2


class PfMat(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int), ("ld", ctypes.c_int64),
                ("tile_scale", ctypes.c_void_p), ("tile", ctypes.c_int32)]


class PfDesc(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("op", ctypes.c_int), ("n", ctypes.c_int64),
                ("m", ctypes.c_int64), ("p", ctypes.c_int32), ("degree", ctypes.c_int32),
                ("q", ctypes.c_int32), ("a", ctypes.c_double), ("b", ctypes.c_double),
                ("spec_ub", ctypes.c_double), ("work", ctypes.c_int), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_int32)]


class PfInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_pos", ctypes.c_int32), ("dense_rr", ctypes.c_int32),
                ("dense_pre", ctypes.c_int32), ("deficient", ctypes.c_int32),
                ("refine_rr", ctypes.c_int32), ("refine_pre", ctypes.c_int32), ("dense_rows", ctypes.c_int32)]


class PfResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_pos", ctypes.c_int32), ("theta", ctypes.c_void_p),
                ("V", ctypes.c_void_p), ("ldv", ctypes.c_int64), ("info", ctypes.c_void_p),
                ("resid", ctypes.c_void_p), ("resid_max", ctypes.c_double)]


class PfExtras(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("reserved", ctypes.c_int32), ("resid", ctypes.c_void_p),
                ("shrink_tau", ctypes.c_double), ("shrink_left", ctypes.c_void_p), ("ld_shrink", ctypes.c_int64)]


class PfSessionState(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("reserved", ctypes.c_int32), ("desc", PfDesc),
                ("steps", ctypes.c_int64)]


APPLY_FN = ctypes.CFUNCTYPE(ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                            ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p)


class PfOperator(ctypes.Structure):
    _fields_ = [("apply", APPLY_FN), ("ctx", ctypes.c_void_p)]


class PfBounds(ctypes.Structure):
    _fields_ = [("theta_min", ctypes.c_double), ("theta_max", ctypes.c_double), ("res_min", ctypes.c_double),
                ("res_max", ctypes.c_double), ("status", ctypes.c_int32), ("replaced", ctypes.c_int32)]


class PfNceOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("degree", ctypes.c_int32), ("guards", ctypes.c_int32),
                ("p_max", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("extrapolation_len", ctypes.c_int32),
                ("lanczos_steps", ctypes.c_int32), ("lanczos_every", ctypes.c_int32), ("tau", ctypes.c_double),
                ("eta", ctypes.c_double), ("tol", ctypes.c_double), ("extrapolation_lambda", ctypes.c_double),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_int32)]


class PfNceResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("n_pos", ctypes.c_int32), ("p", ctypes.c_int32), ("extrapolations", ctypes.c_int32),
                ("F", ctypes.c_double), ("gnorm", ctypes.c_double), ("gnorm0", ctypes.c_double),
                ("a", ctypes.c_double), ("b", ctypes.c_double)]


class PfPfamOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("degree", ctypes.c_int32), ("guards", ctypes.c_int32),
                ("p_max", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("lanczos_steps", ctypes.c_int32),
                ("lanczos_every", ctypes.c_int32), ("flags", ctypes.c_uint32), ("t", ctypes.c_double),
                ("eta", ctypes.c_double), ("tol", ctypes.c_double)]


class PfPfamResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("n_pos", ctypes.c_int32), ("p", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("residual", ctypes.c_double), ("residual0", ctypes.c_double), ("objective", ctypes.c_double),
                ("diag_err", ctypes.c_double), ("a", ctypes.c_double), ("b", ctypes.c_double)]


PF_SERVER_NO_GRAPHS = 0x1
PF_SERVER_NO_GROUPING = 0x2


class PfServerConfig(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("flags", ctypes.c_uint32), ("hbm_budget", ctypes.c_size_t),
                ("max_active", ctypes.c_int32), ("streams", ctypes.c_int32), ("max_batches", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class PfServerEvent(ctypes.Structure):
    _fields_ = [("session", ctypes.c_int32), ("status", ctypes.c_int32), ("n_pos", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("step", ctypes.c_int64), ("tag", ctypes.c_uint64),
                ("submit_ns", ctypes.c_int64), ("launch_ns", ctypes.c_int64), ("done_ns", ctypes.c_int64)]


class PfServerStats(ctypes.Structure):
    _fields_ = [("active", ctypes.c_int32), ("waiting", ctypes.c_int32), ("used_bytes", ctypes.c_size_t),
                ("launched", ctypes.c_int64), ("completed", ctypes.c_int64), ("graph_launches", ctypes.c_int64),
                ("captures", ctypes.c_int64), ("batches", ctypes.c_int64), ("batched_steps", ctypes.c_int64)]


class PfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{status_string(status)}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1904_10585_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    sig = {
        "pf_extract": (i32, [P(PfDesc), P(PfMat), P(PfMat), vp, i64, vp, vp, vp]),
        "pf_extract_ex": (i32, [P(PfDesc), P(PfMat), P(PfMat), vp, i64, vp, vp, P(PfExtras), vp]),
        "pf_workspace_cached": (i32, [P(ctypes.c_size_t), P(i32)]),
        "pf_workspace_release": (i32, [vp]),
        "pf_session_step_ex": (i32, [vp, P(PfMat), P(PfMat), P(PfExtras), P(PfResult), vp]),
        "pf_session_export": (i32, [vp, vp, i64, vp, P(PfSessionState), vp]),
        "pf_session_import": (i32, [P(PfSessionState), vp, i64, vp, P(vp)]),
        "pf_extract_noalloc": (i32, [P(PfDesc), P(PfMat), P(PfMat), vp, i64, vp, vp, vp]),
        "pf_extract_noalloc_max_bytes": (ctypes.c_size_t, []),
        "pf_session_open": (i32, [P(PfDesc), vp, i64, ctypes.c_uint64, P(vp)]),
        "pf_session_step": (i32, [vp, P(PfMat), P(PfMat), P(PfResult), vp]),
        "pf_session_wait": (i32, [vp, P(PfResult)]),
        "pf_session_close": (i32, [vp]),
        "pf_quantize": (i32, [vp, i64, vp, i32, ctypes.c_int, vp, i64, i64, i64, vp]),
        "pf_psd_dense": (i32, [vp, i64, vp, i64, i32, ctypes.c_int, vp, i64, vp]),
        "pf_eigh": (i32, [vp, i64, i32, vp, vp, i64, vp]),
        "pf_workspace_size": (i32, [P(PfDesc), P(ctypes.c_size_t)]),
        "pf_lanczos_bounds": (i32, [P(PfMat), i64, vp, i64, i32, vp, vp]),
        "pf_extract_batch": (i32, [i32, vp, vp, vp, vp, vp, vp, vp, vp]),
        "pf_nce_pfpg": (i32, [P(PfNceOpts), i64, vp, i64, vp, vp, i64, vp, i64, P(PfNceResult), vp, vp]),
        "pf_nce_pfam": (i32, [P(PfPfamOpts), i64, vp, i64, vp, i64, vp, i64, vp, i64, vp, i64, P(PfPfamResult), vp,
                              vp]),
        "pf_extract_op": (i32, [P(PfDesc), P(PfOperator), vp, i64, vp, vp, vp]),
        "pf_session_step_op": (i32, [vp, P(PfOperator), P(PfResult), vp]),
        "pf_interval_policy": (i32, [dbl, dbl, dbl, i32, dbl, P(dbl), P(dbl)]),
        "pf_block_size_policy": (i32, [i32, dbl, i32, i32, P(i32)]),
        "pf_session_set_interval": (i32, [vp, dbl, dbl]),
        "pf_degree_policy": (i32, [dbl, dbl, dbl, i32, dbl, i32, i32, P(i32)]),
        "pf_session_set_filter": (i32, [vp, i32, i32]),
        "pf_profile_set": (i32, [ctypes.c_int]),
        "pf_profile_read": (i32, [ctypes.c_int, P(i64), P(dbl)]),
        "pf_server_create": (i32, [P(PfServerConfig), P(vp)]),
        "pf_server_open": (i32, [vp, P(PfDesc), vp, i64, ctypes.c_uint64, ctypes.c_size_t, P(i32)]),
        "pf_server_submit": (i32, [vp, i32, P(PfMat), P(PfMat), ctypes.c_uint64]),
        "pf_server_poll": (i32, [vp, P(PfServerEvent), i32, P(i32), i64]),
        "pf_server_result": (i32, [vp, i32, P(PfResult)]),
        "pf_server_close": (i32, [vp, i32]),
        "pf_server_stats_get": (i32, [vp, P(PfServerStats)]),
        "pf_server_destroy": (i32, [vp]),
        "pf_status_string": (ctypes.c_char_p, [i32]),
        "pf_last_error": (ctypes.c_char_p, []),
        "pf_abi_version": (ctypes.c_int, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _ = dbl
    return lib


LIB = _load()


def status_string(s):
    return LIB.pf_status_string(int(s)).decode()


def last_error():
    return LIB.pf_last_error().decode()


def _check(s):
    if s != PF_OK:
        raise PfError(s, last_error())


def desc(n, p, degree, a, b, *, q=1, work=PF_F32, op=PF_OP_SYM, m=0, flags=0, spec_ub=0.0):
    d = PfDesc()
    d.struct_size = ctypes.sizeof(PfDesc)
    d.op, d.n, d.m, d.p, d.degree, d.q = op, n, m, p, degree, q
    d.a, d.b, d.spec_ub = float(a), float(b), float(spec_ub)
    d.work, d.flags, d.reserved = work, flags, 0
    return d


_TORCH_DTYPE = {}


def dtype_of(t):
    import torch
    if not _TORCH_DTYPE:
        _TORCH_DTYPE.update({torch.float64: PF_F64, torch.float32: PF_F32, torch.bfloat16: PF_BF16,
                             torch.uint16: PF_BF16, torch.float8_e4m3fn: PF_F8E4M3, torch.uint8: PF_F8E4M3})
    return _TORCH_DTYPE[t.dtype]


def ld_of(t):
    """Leading dimension of a column-major 2-D tensor view."""
    if t.dim() != 2:
        raise ValueError("expected a 2-D tensor")
    if t.stride(0) != 1 and t.shape[1] > 1:
        raise ValueError("expected a column-major view (stride(0) == 1)")
    return max(t.stride(1), t.shape[0]) if t.shape[1] > 1 else t.shape[0]


def mat(t, tile_scale=None, tile=128):
    """pf_mat of a column-major device tensor.  A (tensor, tile_scale, tile)
    tuple or an existing PfMat is accepted too (FP8 operands)."""
    if isinstance(t, PfMat):
        return t
    if isinstance(t, tuple):
        return mat(*t)
    m = PfMat()
    m.data = t.data_ptr()
    m.dtype = dtype_of(t)
    m.ld = ld_of(t)
    m.tile_scale = tile_scale.data_ptr() if tile_scale is not None else None
    m.tile = tile
    return m


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def pf_extract(d, X_filter, X_rr, U, theta, info=None, stream=None):
    """Enqueue one extraction; U (column-major n x p) is overwritten by the Ritz vectors."""
    xf, xr = mat(X_filter), mat(X_rr)
    _check(LIB.pf_extract(ctypes.byref(d), ctypes.byref(xf), ctypes.byref(xr), ctypes.c_void_p(U.data_ptr()),
                          ld_of(U), ctypes.c_void_p(theta.data_ptr()),
                          ctypes.c_void_p(info.data_ptr()) if info is not None else None, _stream(stream)))


def extras(resid=None, shrink_left=None, shrink_tau=0.0):
    """A pf_extras record: resid (device, p doubles) and/or the left factor
    of the Gram form's singular-value shrinkage (device m x p, column-major)."""
    e = PfExtras()
    e.struct_size = ctypes.sizeof(PfExtras)
    e.reserved = 0
    e.resid = resid.data_ptr() if resid is not None else None
    e.shrink_tau = float(shrink_tau)
    e.shrink_left = shrink_left.data_ptr() if shrink_left is not None else None
    e.ld_shrink = ld_of(shrink_left) if shrink_left is not None else 0
    return e


def pf_extract_ex(d, X_filter, X_rr, U, theta, ex, info=None, stream=None):
    """pf_extract with the optional outputs of ``ex`` (see ``extras``)."""
    xf, xr = mat(X_filter), mat(X_rr)
    _check(LIB.pf_extract_ex(ctypes.byref(d), ctypes.byref(xf), ctypes.byref(xr), ctypes.c_void_p(U.data_ptr()),
                             ld_of(U), ctypes.c_void_p(theta.data_ptr()),
                             ctypes.c_void_p(info.data_ptr()) if info is not None else None,
                             ctypes.byref(ex) if ex is not None else None, _stream(stream)))


def pf_extract_noalloc(d, X_filter, X_rr, U, theta, info=None, stream=None):
    """pf_extract with the library's fixed device workspace (no allocation)."""
    xf, xr = mat(X_filter), mat(X_rr)
    _check(LIB.pf_extract_noalloc(ctypes.byref(d), ctypes.byref(xf), ctypes.byref(xr), ctypes.c_void_p(U.data_ptr()),
                                  ld_of(U), ctypes.c_void_p(theta.data_ptr()),
                                  ctypes.c_void_p(info.data_ptr()) if info is not None else None, _stream(stream)))


def pf_extract_noalloc_max_bytes():
    return int(LIB.pf_extract_noalloc_max_bytes())


def pf_session_open(d, U0=None, seed=0):
    h = ctypes.c_void_p()
    _check(LIB.pf_session_open(ctypes.byref(d), ctypes.c_void_p(U0.data_ptr()) if U0 is not None else None,
                               ld_of(U0) if U0 is not None else 0, seed, ctypes.byref(h)))
    return h


def pf_session_step(h, X_filter, X_rr, stream=None):
    r = PfResult()
    xf, xr = mat(X_filter), mat(X_rr)
    _check(LIB.pf_session_step(h, ctypes.byref(xf), ctypes.byref(xr), ctypes.byref(r), _stream(stream)))
    return r


def pf_session_step_ex(h, X_filter, X_rr, ex, stream=None):
    r = PfResult()
    xf, xr = mat(X_filter), mat(X_rr)
    _check(LIB.pf_session_step_ex(h, ctypes.byref(xf), ctypes.byref(xr), ctypes.byref(ex) if ex is not None else None,
                                  ctypes.byref(r), _stream(stream)))
    return r


def pf_session_export(h, U_out, theta_out=None, stream=None):
    """Copy the session's block (and theta) into caller buffers; returns its state."""
    st = PfSessionState()
    _check(LIB.pf_session_export(h, ctypes.c_void_p(U_out.data_ptr()), ld_of(U_out),
                                 ctypes.c_void_p(theta_out.data_ptr()) if theta_out is not None else None,
                                 ctypes.byref(st), _stream(stream)))
    return st


def pf_session_import(state, U, theta=None):
    h = ctypes.c_void_p()
    _check(LIB.pf_session_import(ctypes.byref(state), ctypes.c_void_p(U.data_ptr()), ld_of(U),
                                 ctypes.c_void_p(theta.data_ptr()) if theta is not None else None, ctypes.byref(h)))
    return h


def pf_session_wait(h):
    r = PfResult()
    s = LIB.pf_session_wait(h, ctypes.byref(r))
    return s, r


def pf_session_close(h):
    _check(LIB.pf_session_close(h))


def pf_server_create(hbm_budget, max_active=0, streams=0, flags=0, max_batches=0):
    c = PfServerConfig()
    c.struct_size = ctypes.sizeof(PfServerConfig)
    c.flags, c.hbm_budget, c.max_active, c.streams = flags, int(hbm_budget), max_active, streams
    c.max_batches, c.reserved = max_batches, 0
    h = ctypes.c_void_p()
    _check(LIB.pf_server_create(ctypes.byref(c), ctypes.byref(h)))
    return h


def pf_server_open(h, d, U0=None, seed=0, operator_bytes=0):
    sid = ctypes.c_int32()
    _check(LIB.pf_server_open(h, ctypes.byref(d), ctypes.c_void_p(U0.data_ptr()) if U0 is not None else None,
                              ld_of(U0) if U0 is not None else 0, seed, int(operator_bytes), ctypes.byref(sid)))
    return sid.value


def pf_server_submit(h, session, X_filter, X_rr, tag=0):
    xf, xr = mat(X_filter), mat(X_rr)
    _check(LIB.pf_server_submit(h, session, ctypes.byref(xf), ctypes.byref(xr), tag))


def pf_server_poll(h, max_events=256, timeout_s=0.0):
    """Finished-step events (PfServerEvent), waiting up to timeout_s for the first."""
    buf = (PfServerEvent * max_events)()
    n = ctypes.c_int32()
    _check(LIB.pf_server_poll(h, buf, max_events, ctypes.byref(n), int(timeout_s * 1e9)))
    return [buf[i] for i in range(n.value)]


def pf_server_result(h, session):
    r = PfResult()
    _check(LIB.pf_server_result(h, session, ctypes.byref(r)))
    return r


def pf_server_close(h, session):
    _check(LIB.pf_server_close(h, session))


def pf_server_stats(h):
    st = PfServerStats()
    _check(LIB.pf_server_stats_get(h, ctypes.byref(st)))
    return st


def pf_server_destroy(h):
    _check(LIB.pf_server_destroy(h))


def pf_quantize(dst, tile_scale, tile, dtype, src, stream=None):
    rows, cols = src.shape
    _check(LIB.pf_quantize(ctypes.c_void_p(dst.data_ptr()), ld_of(dst),
                           ctypes.c_void_p(tile_scale.data_ptr()) if tile_scale is not None else None, tile, dtype,
                           ctypes.c_void_p(src.data_ptr()), rows, cols, ld_of(src), _stream(stream)))


def pf_psd_dense(V, theta, n, p, work, out, stream=None):
    _check(LIB.pf_psd_dense(ctypes.c_void_p(V.data_ptr()), ld_of(V), ctypes.c_void_p(theta.data_ptr()), n, p, work,
                            ctypes.c_void_p(out.data_ptr()), ld_of(out), _stream(stream)))


def pf_eigh(H, theta, Z, stream=None):
    """theta (descending), Z = eigenpairs of sym(H); H, Z column-major FP64 p x p."""
    p = H.shape[0]
    _check(LIB.pf_eigh(ctypes.c_void_p(H.data_ptr()), ld_of(H), p, ctypes.c_void_p(theta.data_ptr()),
                       ctypes.c_void_p(Z.data_ptr()), ld_of(Z), _stream(stream)))


def pf_lanczos_bounds(X, V0, steps, stream=None, out=None):
    """Block Lanczos bounds of a symmetric n x n device matrix X (FP32 or
    FP64) from the n x 16 FP64 start block V0.  Without ``out``: waits for
    the stream and returns the PfBounds.  With ``out`` (a device uint8 tensor
    of ctypes.sizeof(PfBounds) bytes): only enqueues; read it with
    ``bounds_of(out)`` once the stream is done."""
    import torch
    n = X.shape[0]
    dst = out if out is not None else torch.zeros(ctypes.sizeof(PfBounds), dtype=torch.uint8, device=X.device)
    m = mat(X)
    _check(LIB.pf_lanczos_bounds(ctypes.byref(m), n, ctypes.c_void_p(V0.data_ptr()), ld_of(V0), steps,
                                 ctypes.c_void_p(dst.data_ptr()), _stream(stream)))
    if out is not None:
        return None
    if stream is not None:
        stream.synchronize()
    else:
        torch.cuda.synchronize(X.device)
    return bounds_of(dst)


def pf_extract_batch(blocks, stream=None):
    """Independent extractions in one call (pf_extract_batch).  blocks: a
    list of (desc, X_filter, X_rr, U, theta, info) as for pf_extract (info
    may be None); U and theta are updated in place, stream-ordered."""
    n = len(blocks)
    D = (PfDesc * n)(*[b[0] for b in blocks])
    XF = (PfMat * n)(*[mat(b[1]) for b in blocks])
    XR = (PfMat * n)(*[mat(b[2]) for b in blocks])
    U = (ctypes.c_void_p * n)(*[b[3].data_ptr() for b in blocks])
    LD = (ctypes.c_int64 * n)(*[ld_of(b[3]) for b in blocks])
    TH = (ctypes.c_void_p * n)(*[b[4].data_ptr() for b in blocks])
    has_info = any(b[5] is not None for b in blocks)
    INF = (ctypes.c_void_p * n)(*[(b[5].data_ptr() if b[5] is not None else None) for b in blocks]) if has_info else None
    _check(LIB.pf_extract_batch(n, D, XF, XR, U, LD, TH, INF, _stream(stream)))


def pf_nce_pfpg(G, x, U0, V0, *, degree=10, guards=8, p_max=128, max_iter=500, extrapolation_len=3,
                lanczos_steps=4, lanczos_every=10, tau=1.6, eta=0.1, tol=1e-7, extrapolation_lambda=1e-8,
                flags=0, stream=None, history=True):
    """Nearest correlation PFPG loop on the device (FP64 column-major G
    n x n, x n (in: start, out: last iterate), U0 n x p_max, V0 n x 16).
    Returns (PfNceResult, history) with history an (iters + 1) x 6 array of
    (F, ||g||, n_pos, p, a, b) rows, or None.  Raises PfError on failure
    (the result is then in the exception's ``result`` attribute)."""
    import numpy as np
    n = G.shape[0]
    o = PfNceOpts()
    o.struct_size = ctypes.sizeof(PfNceOpts)
    o.degree, o.guards, o.p_max, o.max_iter = degree, guards, p_max, max_iter
    o.extrapolation_len, o.lanczos_steps, o.lanczos_every = extrapolation_len, lanczos_steps, lanczos_every
    o.tau, o.eta, o.tol, o.extrapolation_lambda = tau, eta, tol, extrapolation_lambda
    o.flags = flags
    res = PfNceResult()
    hist = np.zeros((max_iter, 6)) if history else None
    hp = ctypes.c_void_p(hist.ctypes.data) if history else ctypes.c_void_p(0)
    s = LIB.pf_nce_pfpg(ctypes.byref(o), n, ctypes.c_void_p(G.data_ptr()), ld_of(G), ctypes.c_void_p(x.data_ptr()),
                        ctypes.c_void_p(U0.data_ptr()), ld_of(U0), ctypes.c_void_p(V0.data_ptr()), ld_of(V0),
                        ctypes.byref(res), hp, _stream(stream))
    if s != PF_OK:
        e = PfError(s, last_error())
        e.result = res
        raise e
    return res, (hist[: res.iters + 1] if history else None)


def pf_nce_pfam(G, Z, X, U0, V0, *, degree=10, guards=8, p_max=128, max_iter=500, lanczos_steps=4,
                lanczos_every=10, t=0.5, eta=0.1, tol=1e-7, flags=0, stream=None, history=True):
    """PFAM on the nearest correlation primal on the device (FP64
    column-major G, Z (in: start, out: last), X (out: primal iterate), all
    n x n; U0 n x p_max, V0 n x 16).  Returns (PfPfamResult, history) with
    history an (iters + 1) x 7 array of (||dZ||, 1/2 ||G - X||^2, n_pos, p,
    a, b, max |diag X - 1|) rows, or None.  Raises PfError on failure (the
    result in the exception's ``result`` attribute)."""
    import numpy as np
    n = G.shape[0]
    o = PfPfamOpts()
    o.struct_size = ctypes.sizeof(PfPfamOpts)
    o.degree, o.guards, o.p_max, o.max_iter = degree, guards, p_max, max_iter
    o.lanczos_steps, o.lanczos_every, o.flags = lanczos_steps, lanczos_every, flags
    o.t, o.eta, o.tol = t, eta, tol
    res = PfPfamResult()
    hist = np.zeros((max_iter, 7)) if history else None
    hp = ctypes.c_void_p(hist.ctypes.data) if history else ctypes.c_void_p(0)
    s = LIB.pf_nce_pfam(ctypes.byref(o), n, ctypes.c_void_p(G.data_ptr()), ld_of(G), ctypes.c_void_p(Z.data_ptr()),
                        ld_of(Z), ctypes.c_void_p(X.data_ptr()), ld_of(X), ctypes.c_void_p(U0.data_ptr()), ld_of(U0),
                        ctypes.c_void_p(V0.data_ptr()), ld_of(V0), ctypes.byref(res), hp, _stream(stream))
    if s != PF_OK:
        e = PfError(s, last_error())
        e.result = res
        raise e
    return res, (hist[: res.iters + 1] if history else None)


def bounds_of(out):
    """PfBounds from the device buffer pf_lanczos_bounds wrote."""
    return PfBounds.from_buffer_copy(bytes(out.cpu().numpy()))


class _DeviceArray:
    """A column-major rows x cols device block at a raw pointer, exposed
    through __cuda_array_interface__ (zero-copy views for operator callbacks)."""

    def __init__(self, ptr, rows, cols, ld, typestr, esz):
        self.__cuda_array_interface__ = {"shape": (rows, cols), "typestr": typestr, "data": (ptr, False),
                                         "strides": (esz, ld * esz), "version": 2}


def device_view(ptr, rows, cols, ld, dtype):
    """torch view of a column-major device block (float32 / float64)."""
    import torch
    typestr, esz = ("<f8", 8) if dtype == torch.float64 else ("<f4", 4)
    return torch.as_tensor(_DeviceArray(ptr, rows, cols, ld, typestr, esz), device="cuda")


def make_operator(fn, n, dtype):
    """PfOperator from fn(Y, AY): torch views of the n x cols blocks (column
    major, dtype the work dtype); fn must write AY = A Y with torch work on
    the current stream (the callback makes the library's stream current).
    The returned object keeps the ctypes callback alive."""
    import torch

    def _apply(ctx, Y, ldy, AY, lday, cols, stream):
        try:
            st = torch.cuda.ExternalStream(stream) if stream else torch.cuda.current_stream()
            with torch.cuda.stream(st):
                fn(device_view(Y, n, cols, ldy, dtype), device_view(AY, n, cols, lday, dtype))
            return PF_OK
        except Exception:                                    # reported as a device error
            return PF_ERR_DEVICE

    cb = APPLY_FN(_apply)
    op = PfOperator(cb, None)
    op._keep = cb
    return op


def pf_extract_op(d, op, U, theta, info=None, stream=None):
    """pf_extract with a PfOperator (make_operator) in place of X."""
    _check(LIB.pf_extract_op(ctypes.byref(d), ctypes.byref(op), ctypes.c_void_p(U.data_ptr()), ld_of(U),
                             ctypes.c_void_p(theta.data_ptr()),
                             ctypes.c_void_p(info.data_ptr()) if info is not None else None, _stream(stream)))


def pf_session_step_op(h, op, stream=None):
    r = PfResult()
    _check(LIB.pf_session_step_op(h, ctypes.byref(op), ctypes.byref(r), _stream(stream)))
    return r


def pf_interval_policy(lam_min, margin, eta, top_r=0, theta_r=0.0):
    """(a, b) of the section 4.1 rule (host arithmetic)."""
    a, b = ctypes.c_double(), ctypes.c_double()
    _check(LIB.pf_interval_policy(lam_min, margin, eta, top_r, theta_r, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def pf_block_size_policy(top_r, q=2.0, n_pos=0, guards=0):
    """p of the section 4.2 rule (host arithmetic)."""
    p = ctypes.c_int32()
    _check(LIB.pf_block_size_policy(top_r, q, n_pos, guards, ctypes.byref(p)))
    return p.value


def pf_session_set_interval(h, a, b):
    _check(LIB.pf_session_set_interval(h, a, b))


def pf_degree_policy(theta_r, a, b, q=1, eps=1e-6, d_min=1, d_max=64):
    """Filter degree of the tolerance rule (host arithmetic)."""
    d = ctypes.c_int32()
    _check(LIB.pf_degree_policy(theta_r, a, b, q, eps, d_min, d_max, ctypes.byref(d)))
    return d.value


def pf_session_set_filter(h, degree, q=1):
    _check(LIB.pf_session_set_filter(h, degree, q))


def pf_workspace_size(d):
    n = ctypes.c_size_t()
    _check(LIB.pf_workspace_size(ctypes.byref(d), ctypes.byref(n)))
    return n.value


def pf_workspace_cached():
    """(device bytes, count) of the workspaces cached by pf_extract."""
    b = ctypes.c_size_t()
    n = ctypes.c_int32()
    _check(LIB.pf_workspace_cached(ctypes.byref(b), ctypes.byref(n)))
    return b.value, n.value


def pf_workspace_release(stream=None):
    """Free the workspaces pf_extract cached for a stream (after waiting for it)."""
    _check(LIB.pf_workspace_release(_stream(stream)))


def pf_profile_set(mode):
    """0: off; 1 (or True): per-kernel classes; PF_PROF_MODE_PRODUCT: the
    filter product (kernel and split-K sum) under one event pair."""
    _check(LIB.pf_profile_set(int(mode)))


def pf_profile_read(which):
    """(launches, total milliseconds) of a kernel class since pf_profile_set(1)."""
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    _check(LIB.pf_profile_read(which, ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


_HIP = None


def device_to_numpy(ptr, shape, dtype):
    """Copy device memory at a raw pointer (e.g. a pf_result field) to a new
    host array of the given shape (C order)."""
    import numpy as np
    global _HIP
    if _HIP is None:
        _HIP = ctypes.CDLL("libamdhip64.so")
        _HIP.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _HIP.hipMemcpy.restype = ctypes.c_int
    out = np.empty(shape, dtype=dtype)
    rc = _HIP.hipMemcpy(out.ctypes.data, ptr, out.nbytes, 2)   # hipMemcpyDeviceToHost
    if rc != 0:
        raise PfError(PF_ERR_DEVICE, f"hipMemcpy failed ({rc})")
    return out


def colmajor(rows, cols, dtype, device, ld=None):
    """A zeroed column-major rows x cols tensor view with leading dimension ld."""
    import torch
    ld = ld or rows
    return torch.zeros((cols, ld), dtype=dtype, device=device).t()[:rows]


def to_colmajor(a, dtype, device):
    """Copy a (rows x cols) array-like into a fresh column-major device tensor."""
    import torch
    t = torch.as_tensor(a)
    out = colmajor(t.shape[0], t.shape[1], dtype, device)
    out.copy_(t.to(dtype))
    return out
