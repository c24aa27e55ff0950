"""C-ABI checks that need no GPU: the library loads, exports every function
include/pf.h declares, and rejects invalid arguments before touching the
device.  Every call below fails validation, so none reaches a kernel."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pf.h")

pf = pytest.importorskip("paper_1904_10585_amd.pf")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"typedef[^;]*;", "", text)                 # function-pointer types are not symbols
    return sorted(set(re.findall(r"\b(pf_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert "pf_extract" in names and "pf_session_step" in names
    lib = ctypes.CDLL(pf.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name


def test_abi_version_and_strings():
    assert pf.LIB.pf_abi_version() == 3
    for s in range(9):
        assert pf.status_string(s).startswith("PF_")
    assert pf.status_string(99) == "unknown pf_status"


def test_binding_constants_match_header():
    """Every #define of pf.h that the binding mirrors has the header's value."""
    text = open(HEADER).read()
    defs = dict(re.findall(r"^#define (PF_[A-Z0-9_]+) (0x[0-9a-fA-F]+|[0-9]+)u?\b", text, re.M))
    assert len(defs) >= 14
    mirrored = 0
    for name, val in defs.items():
        if hasattr(pf, name):
            assert getattr(pf, name) == int(val, 0), name
            mirrored += 1
    assert mirrored >= 12


def test_workspace_cache_query_needs_no_device():
    b, c = pf.pf_workspace_cached()
    assert b >= 0 and c >= 0 and (c > 0 or b == 0)
    assert pf.LIB.pf_workspace_cached(None, None) == pf.PF_ERR_ARG


def test_profile_mode_rejects_unknown():
    assert pf.LIB.pf_profile_set(7) == pf.PF_ERR_ARG
    assert "profiling mode" in pf.LIB.pf_last_error().decode()
    assert pf.LIB.pf_profile_set(0) == 0


def test_struct_layout_matches_c_compiler(tmp_path):
    """ctypes mirrors of the pf.h structs have the C compiler's sizes and offsets."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"pf_desc": pf.PfDesc, "pf_mat": pf.PfMat, "pf_info": pf.PfInfo, "pf_result": pf.PfResult,
               "pf_server_config": pf.PfServerConfig, "pf_server_event": pf.PfServerEvent,
               "pf_server_stats": pf.PfServerStats, "pf_bounds": pf.PfBounds, "pf_operator": pf.PfOperator,
               "pf_nce_opts": pf.PfNceOpts, "pf_nce_result": pf.PfNceResult, "pf_pfam_opts": pf.PfPfamOpts,
               "pf_pfam_result": pf.PfPfamResult, "pf_extras": pf.PfExtras, "pf_session_state": pf.PfSessionState}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pf.h"', "int main(void){"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = dict(l.rsplit(" ", 1) for l in out if l.strip())
    for cname, cls in structs.items():
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(cls, fname).offset, (cname, fname)


def good_desc(**kw):
    args = dict(n=256, p=16, degree=4, a=-1.0, b=0.5)
    args.update(kw)
    return pf.desc(**args)


@pytest.mark.parametrize("field,value", [
    ("n", 0), ("p", 0), ("p", 129), ("p", 300), ("degree", 0), ("q", 0),
    ("a", 1.0), ("b", -2.0), ("work", 7), ("flags", 0x100), ("reserved", 1), ("op", 5),
])
def test_workspace_size_rejects(field, value):
    d = good_desc()
    setattr(d, field, value)
    with pytest.raises(pf.PfError) as e:
        pf.pf_workspace_size(d)
    assert e.value.status == pf.PF_ERR_ARG


def test_struct_size_versioning():
    d = good_desc()
    d.struct_size = 12
    with pytest.raises(pf.PfError) as e:
        pf.pf_workspace_size(d)
    assert e.value.status == pf.PF_ERR_ARG
    assert "struct_size" in pf.last_error()


def test_scaled_needs_upper_bound():
    d = good_desc(flags=pf.PF_FLAG_SCALED, spec_ub=0.2)
    with pytest.raises(pf.PfError) as e:
        pf.pf_workspace_size(d)
    assert e.value.status == pf.PF_ERR_ARG


def test_workspace_size_valid():
    assert pf.pf_workspace_size(good_desc()) > 256 * 16 * 4 * 6
    assert pf.pf_workspace_size(good_desc(work=pf.PF_F64)) > pf.pf_workspace_size(good_desc())


def _extract_raw(d, xf, xr, U, ldu, theta):
    return pf.LIB.pf_extract(ctypes.byref(d), ctypes.byref(xf) if xf else None, ctypes.byref(xr) if xr else None,
                             U, ldu, theta, None, None)


def fake_mat(ptr=0x10000, dtype=pf.PF_F32, ld=256):
    m = pf.PfMat()
    m.data, m.dtype, m.ld, m.tile_scale, m.tile = ptr, dtype, ld, None, 128
    return m


@pytest.mark.parametrize("case", ["null_x", "null_rr", "short_ld", "misaligned", "bad_ld_bytes", "dtype",
                                  "rr_dtype", "null_u", "short_ldu", "null_theta", "f64_rr", "fp8_noscale",
                                  "fp8_tile", "rr_bf16", "native_bf16"])
def test_extract_rejects_before_launch(case):
    d = good_desc()
    xf, xr = fake_mat(), fake_mat()
    U, ldu, theta = 0x20000, 256, 0x30000
    want = pf.PF_ERR_ARG
    if case == "null_x":
        xf = None
    elif case == "null_rr":
        xr = None
    elif case == "short_ld":
        xf.ld = 100
    elif case == "misaligned":
        xf.data = 0x10004
    elif case == "bad_ld_bytes":
        xf.ld = 257
    elif case == "dtype":
        xf.dtype = pf.PF_F64
    elif case == "rr_dtype":
        xr.dtype = 9
    elif case == "null_u":
        U = None
    elif case == "short_ldu":
        ldu = 10
    elif case == "null_theta":
        theta = None
    elif case == "f64_rr":
        xr.dtype = pf.PF_F64
    elif case == "fp8_noscale":
        xf.dtype = pf.PF_F8E4M3
    elif case == "fp8_tile":
        xf.dtype, xf.tile_scale, xf.tile = pf.PF_F8E4M3, 0x40000, 64
    elif case == "rr_bf16":
        xr.dtype = pf.PF_BF16
    elif case == "native_bf16":
        xf.dtype = pf.PF_BF16
        d.flags = pf.PF_FLAG_NATIVE_F32
    assert _extract_raw(d, xf, xr, U, ldu, theta) == want
    assert pf.last_error()


def _extras(**kw):
    e = pf.PfExtras()
    e.struct_size = ctypes.sizeof(pf.PfExtras)
    for k, v in kw.items():
        setattr(e, k, v)
    return e


@pytest.mark.parametrize("case,want", [
    ("size", pf.PF_ERR_ARG), ("reserved", pf.PF_ERR_ARG), ("shrink_sym", pf.PF_ERR_ARG),
    ("tau_neg", pf.PF_ERR_ARG), ("tau_nan", pf.PF_ERR_ARG), ("ld_shrink", pf.PF_ERR_ARG),
])
def test_extract_ex_rejects_before_launch(case, want):
    """Bad optional-output records are refused before anything is enqueued."""
    gram = case in ("tau_neg", "tau_nan", "ld_shrink")
    d = good_desc(op=pf.PF_OP_GRAM, m=300) if gram else good_desc()
    xf = fake_mat(ld=300 if gram else 256)
    e = _extras(shrink_left=0x20000, shrink_tau=0.5, ld_shrink=300)
    if case == "size":
        e.struct_size = 8
    elif case == "reserved":
        e.reserved = 1
    elif case == "tau_neg":
        e.shrink_tau = -1.0
    elif case == "tau_nan":
        e.shrink_tau = float("nan")
    elif case == "ld_shrink":
        e.ld_shrink = 299
    r = pf.LIB.pf_extract_ex(ctypes.byref(d), ctypes.byref(xf), ctypes.byref(xf), ctypes.c_void_p(0x30000), 256,
                             ctypes.c_void_p(0x40000), None, ctypes.byref(e), None)
    assert r == want, pf.last_error()
    assert pf.last_error()


def test_session_import_rejects_bad_state():
    st = pf.PfSessionState()
    st.struct_size = ctypes.sizeof(pf.PfSessionState)
    st.desc = good_desc()
    h = ctypes.c_void_p()
    U = ctypes.c_void_p(0x10000)
    bad = [("struct_size", 4), ("reserved", 1), ("steps", -1)]
    for field, value in bad:
        s2 = pf.PfSessionState.from_buffer_copy(st)
        setattr(s2, field, value)
        assert pf.LIB.pf_session_import(ctypes.byref(s2), U, 256, None, ctypes.byref(h)) == pf.PF_ERR_ARG, field
    s2 = pf.PfSessionState.from_buffer_copy(st)
    s2.desc.p = 0
    assert pf.LIB.pf_session_import(ctypes.byref(s2), U, 256, None, ctypes.byref(h)) == pf.PF_ERR_ARG
    assert pf.LIB.pf_session_import(ctypes.byref(st), U, 100, None, ctypes.byref(h)) == pf.PF_ERR_ARG
    assert pf.LIB.pf_session_import(None, U, 256, None, ctypes.byref(h)) == pf.PF_ERR_ARG
    assert pf.LIB.pf_session_export(None, U, 256, None, ctypes.byref(st), None) == pf.PF_ERR_ARG
    assert pf.LIB.pf_session_step_ex(None, None, None, None, None, None) == pf.PF_ERR_ARG


def test_session_and_helpers_reject_nulls():
    assert pf.LIB.pf_session_close(None) == pf.PF_ERR_ARG
    assert pf.LIB.pf_session_step(None, None, None, None, None) == pf.PF_ERR_ARG
    assert pf.LIB.pf_quantize(None, 1, None, 128, pf.PF_BF16, None, 1, 1, 1, None) == pf.PF_ERR_ARG
    assert pf.LIB.pf_psd_dense(None, 1, None, 1, 1, pf.PF_F32, None, 1, None) == pf.PF_ERR_ARG
    d = good_desc()
    h = ctypes.c_void_p()
    assert pf.LIB.pf_session_open(ctypes.byref(d), ctypes.c_void_p(0x1000), 3, 0, ctypes.byref(h)) == pf.PF_ERR_ARG


def test_server_rejects_bad_config():
    """Configuration errors are found before any HIP call."""
    for kw in (dict(hbm_budget=0), dict(hbm_budget=1 << 30, streams=65), dict(hbm_budget=1 << 30, max_active=-1),
               dict(hbm_budget=1 << 30, flags=0x80)):
        with pytest.raises(pf.PfError) as e:
            pf.pf_server_create(**kw)
        assert e.value.status == pf.PF_ERR_ARG
    c = pf.PfServerConfig()
    c.struct_size = 4
    c.hbm_budget = 1 << 30
    h = ctypes.c_void_p()
    assert pf.LIB.pf_server_create(ctypes.byref(c), ctypes.byref(h)) == pf.PF_ERR_ARG
    for fn, args in (("pf_server_open", (None, None, None, 0, 0, 0, None)), ("pf_server_submit", (None, 1, None, None, 0)),
                     ("pf_server_close", (None, 1)), ("pf_server_destroy", (None,)),
                     ("pf_server_result", (None, 1, None)), ("pf_server_stats_get", (None, None))):
        assert getattr(pf.LIB, fn)(*args) == pf.PF_ERR_ARG, fn


def test_eigh_rejects_before_launch():
    """pf_eigh argument errors are returned before any HIP call (the
    pointers below are never dereferenced)."""
    H, th, Z = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x80000), ctypes.c_void_p(0x100000)
    assert pf.LIB.pf_eigh(None, 4, 4, th, Z, 4, None) == pf.PF_ERR_ARG
    assert pf.LIB.pf_eigh(H, 4, 0, th, Z, 4, None) == pf.PF_ERR_ARG
    assert pf.LIB.pf_eigh(H, 129, 129, th, Z, 129, None) == pf.PF_ERR_ARG
    assert pf.LIB.pf_eigh(H, 3, 4, th, Z, 4, None) == pf.PF_ERR_ARG
    assert pf.LIB.pf_eigh(H, 4, 4, th, Z, 2, None) == pf.PF_ERR_ARG
    assert pf.LIB.pf_eigh(H, 8, 8, th, ctypes.c_void_p(0x10000 + 8 * 8), 8, None) == pf.PF_ERR_ARG
    assert "overlap" in pf.last_error()


def test_interval_and_block_size_policies_match_the_oracle():
    """The host rules of sections 4.1-4.2 in the C ABI agree with the
    oracle's statement of them over a grid of inputs, errors included."""
    import oracle
    for lam in (-7.5, -1.0, 0.3):
        for margin in (0.0, 0.25):
            for eta in (0.1, 0.2):
                for top_r, th in ((0, 0.0), (5, 2.0), (12, -0.2)):
                    try:
                        want = oracle.interval_policy(lam, margin, eta, top_r, th)
                    except ValueError:
                        want = None
                    if want is None:
                        with pytest.raises(pf.PfError) as e:
                            pf.pf_interval_policy(lam, margin, eta, top_r, th)
                        assert e.value.status == pf.PF_ERR_ARG
                    else:
                        got = pf.pf_interval_policy(lam, margin, eta, top_r, th)
                        assert abs(got[0] - want[0]) <= 1e-15 and abs(got[1] - want[1]) <= 1e-14
    for r, q in ((1, 1.5), (3, 2.2), (40, 1.5), (100, 2.0)):
        assert pf.pf_block_size_policy(r, q) == oracle.block_size_policy(r, q)
    for n_pos, guards in ((0, 0), (37, 8), (200, 4)):
        assert pf.pf_block_size_policy(0, 2.0, n_pos, guards) == oracle.block_size_policy(0, 2.0, n_pos, guards)
    for args in ((4, 1.0, 0, 0), (0, 2.0, -1, 0), (3, float("nan"), 0, 0)):
        with pytest.raises(pf.PfError):
            pf.pf_block_size_policy(*args)
    with pytest.raises(pf.PfError):
        pf.pf_interval_policy(-1.0, 0.0, 1.5)


def test_lanczos_rejects_before_launch():
    """pf_lanczos_bounds argument errors are returned before any HIP call."""
    m = fake_mat(ld=256)
    V0, out = ctypes.c_void_p(0x40000), ctypes.c_void_p(0x80000)
    assert pf.LIB.pf_lanczos_bounds(ctypes.byref(m), 256, None, 256, 4, out, None) == pf.PF_ERR_ARG
    assert pf.LIB.pf_lanczos_bounds(ctypes.byref(m), 256, V0, 256, 0, out, None) == pf.PF_ERR_ARG
    assert pf.LIB.pf_lanczos_bounds(ctypes.byref(m), 256, V0, 256, 9, out, None) == pf.PF_ERR_ARG
    assert pf.LIB.pf_lanczos_bounds(ctypes.byref(m), 40, V0, 256, 3, out, None) == pf.PF_ERR_ARG
    assert pf.LIB.pf_lanczos_bounds(ctypes.byref(m), 300, V0, 300, 4, out, None) == pf.PF_ERR_ARG   # ld < n
    bf = fake_mat(dtype=pf.PF_BF16, ld=256)
    assert pf.LIB.pf_lanczos_bounds(ctypes.byref(bf), 256, V0, 256, 4, out, None) == pf.PF_ERR_ARG
    odd = fake_mat(ld=257)
    assert pf.LIB.pf_lanczos_bounds(ctypes.byref(odd), 256, V0, 257, 4, out, None) == pf.PF_ERR_ARG
    assert pf.LIB.pf_session_set_interval(None, -1.0, 1.0) == pf.PF_ERR_ARG


def test_degree_policy_matches_the_oracle():
    import oracle
    for th, a, b in ((1.0, -5.0, 0.8), (1.0, -2.0, 0.8), (5.0, -1.0, 0.5), (20.0, -10.0, 0.8)):
        for q in (1, 2, 3):
            for eps in (1e-2, 1e-6, 1e-10):
                for dmin, dmax in ((1, 64), (8, 12)):
                    assert pf.pf_degree_policy(th, a, b, q, eps, dmin, dmax) == \
                        oracle.degree_policy(th, a, b, q, eps, dmin, dmax)
    for args in ((0.5, -1.0, 0.8, 1, 1e-3, 1, 64), (1.0, -1.0, 0.8, 0, 1e-3, 1, 64),
                 (1.0, -1.0, 0.8, 1, 1.5, 1, 64), (1.0, -1.0, 0.8, 1, 1e-3, 5, 4)):
        with pytest.raises(pf.PfError):
            pf.pf_degree_policy(*args)
    assert pf.LIB.pf_session_set_filter(None, 8, 1) == pf.PF_ERR_ARG


def test_operator_entry_points_reject_before_launch():
    """pf_extract_op / pf_session_step_op argument errors before any HIP
    call: no operator, no callback, a Gram descriptor."""
    d = good_desc()
    U, theta = ctypes.c_void_p(0x20000), ctypes.c_void_p(0x30000)
    assert pf.LIB.pf_extract_op(ctypes.byref(d), None, U, 256, theta, None, None) == pf.PF_ERR_ARG
    op = pf.PfOperator()
    assert pf.LIB.pf_extract_op(ctypes.byref(d), ctypes.byref(op), U, 256, theta, None, None) == pf.PF_ERR_ARG
    good = pf.make_operator(lambda Y, AY: None, 256, None)
    g = good_desc(op=pf.PF_OP_GRAM, m=300)
    assert pf.LIB.pf_extract_op(ctypes.byref(g), ctypes.byref(good), U, 256, theta, None, None) == pf.PF_ERR_ARG
    assert "PF_OP_SYM" in pf.last_error()
    assert pf.LIB.pf_extract_op(ctypes.byref(d), ctypes.byref(good), None, 256, theta, None, None) == pf.PF_ERR_ARG
    assert pf.LIB.pf_session_step_op(None, ctypes.byref(good), None, None) == pf.PF_ERR_ARG


def test_nce_rejects_before_launch():
    """pf_nce_pfpg option and argument errors are returned before any HIP
    call, with the status also in the result record."""
    P = ctypes.c_void_p

    def opts(**kw):
        o = pf.PfNceOpts()
        o.struct_size = ctypes.sizeof(pf.PfNceOpts)
        o.degree, o.guards, o.p_max, o.max_iter = 10, 8, 128, 50
        o.extrapolation_len, o.lanczos_steps, o.lanczos_every = 3, 4, 10
        o.tau, o.eta, o.tol, o.extrapolation_lambda = 1.6, 0.1, 1e-7, 1e-8
        for k, v in kw.items():
            setattr(o, k, v)
        return o

    def call(o, n=512, lds=512, G=P(0x40000)):
        r = pf.PfNceResult()
        s = pf.LIB.pf_nce_pfpg(ctypes.byref(o), n, G, lds, P(0x80000), P(0xC0000), lds, P(0x100000), lds,
                               ctypes.byref(r), None, None)
        assert r.status == s
        return s

    bad = [dict(struct_size=8), dict(p_max=8), dict(p_max=129), dict(degree=0), dict(guards=-1), dict(max_iter=0),
           dict(extrapolation_len=8), dict(extrapolation_len=-1), dict(lanczos_steps=0), dict(lanczos_steps=9),
           dict(lanczos_every=-1), dict(tau=0.0), dict(tau=float("inf")), dict(eta=0.0), dict(eta=1.0),
           dict(tol=0.0), dict(extrapolation_lambda=-1.0), dict(extrapolation_lambda=float("nan")),
           dict(flags=pf.PF_FLAG_SCALED), dict(reserved=1)]
    for kw in bad:
        assert call(opts(**kw)) == pf.PF_ERR_ARG, kw
    assert call(opts(), n=100) == pf.PF_ERR_ARG                      # p_max > n
    assert call(opts(p_max=32, lanczos_steps=8), n=100) == pf.PF_ERR_ARG   # 16 * steps > n
    assert call(opts(), lds=500) == pf.PF_ERR_ARG                    # ld < n
    assert call(opts(), G=None) == pf.PF_ERR_ARG
    r = pf.PfNceResult()
    assert pf.LIB.pf_nce_pfpg(None, 512, P(1), 512, P(1), P(1), 512, P(1), 512, ctypes.byref(r), None, None) == pf.PF_ERR_ARG


def test_pfam_rejects_before_launch():
    """pf_nce_pfam option and argument errors are returned before any HIP
    call, with the status also in the result record."""
    P = ctypes.c_void_p

    def opts(**kw):
        o = pf.PfPfamOpts()
        o.struct_size = ctypes.sizeof(pf.PfPfamOpts)
        o.degree, o.guards, o.p_max, o.max_iter = 10, 8, 128, 50
        o.lanczos_steps, o.lanczos_every, o.flags = 4, 10, 0
        o.t, o.eta, o.tol = 0.5, 0.1, 1e-7
        for k, v in kw.items():
            setattr(o, k, v)
        return o

    def call(o, n=512, ld=512, Z=P(0x80000), X=P(0xC0000)):
        r = pf.PfPfamResult()
        s = pf.LIB.pf_nce_pfam(ctypes.byref(o), n, P(0x40000), ld, Z, ld, X, ld, P(0x100000), ld, P(0x140000), ld,
                               ctypes.byref(r), None, None)
        assert r.status == s
        return s

    bad = [dict(struct_size=8), dict(p_max=8), dict(p_max=129), dict(degree=0), dict(guards=-1), dict(max_iter=0),
           dict(lanczos_steps=0), dict(lanczos_steps=9), dict(lanczos_every=-1), dict(flags=pf.PF_FLAG_SCALED),
           dict(t=0.0), dict(t=float("nan")), dict(eta=0.0), dict(eta=1.0), dict(tol=0.0)]
    for kw in bad:
        assert call(opts(**kw)) == pf.PF_ERR_ARG, kw
    assert call(opts(), n=100) == pf.PF_ERR_ARG                      # p_max > n
    assert call(opts(), ld=500) == pf.PF_ERR_ARG                     # ld < n
    assert call(opts(), Z=P(0x80008)) == pf.PF_ERR_ARG               # Z not 16-byte aligned
    assert call(opts(), X=P(0x80000)) == pf.PF_ERR_ARG               # X aliases Z
    assert call(opts(), Z=None) == pf.PF_ERR_ARG
    assert call(opts(p_max=16), n=70000, ld=70000) == pf.PF_ERR_ARG  # grid extent


def test_extract_batch_rejects_before_launch():
    """pf_extract_batch checks every block before any HIP call; an invalid
    block is named in the message."""
    assert pf.LIB.pf_extract_batch(-1, None, None, None, None, None, None, None, None) == pf.PF_ERR_ARG
    assert pf.LIB.pf_extract_batch(0, None, None, None, None, None, None, None, None) == pf.PF_OK
    assert pf.LIB.pf_extract_batch(2, None, None, None, None, None, None, None, None) == pf.PF_ERR_ARG
    good = pf.desc(256, 16, 6, -1.0, 0.5, work=pf.PF_F32)
    bad = pf.desc(256, 0, 6, -1.0, 0.5, work=pf.PF_F32)
    D = (pf.PfDesc * 2)(good, bad)
    m = fake_mat(dtype=pf.PF_F32, ld=256)
    M = (pf.PfMat * 2)(m, m)
    P = ctypes.c_void_p
    U = (P * 2)(0x40000, 0x80000)
    LD = (ctypes.c_int64 * 2)(256, 256)
    TH = (P * 2)(0xC0000, 0x100000)
    assert pf.LIB.pf_extract_batch(2, D, M, M, U, LD, TH, None, None) == pf.PF_ERR_ARG
    assert "block 1" in pf.last_error()
