"""Optional outputs of an extraction and the checkpoint of a session, through
the C ABI, against the oracle.

  * residual norms ||A v_i - theta_i v_i|| of the returned Ritz pairs
    (eq. RR), SYM and Gram forms, against ``oracle.ritz_residuals`` on the
    GPU's own (V, theta): FP64 work within 1e-10 ||A||, FP32 work within
    1e-6 ||A|| (the library's residual is that of the FP64 vectors Q Z, the
    oracle's that of V rounded to FP32: they differ by ~1e-7 ||A||);
  * the singular-value shrinkage factor of section 5.2.1 against
    ``oracle.svd_shrink_factor`` (1e-10 ||M|| FP64, 1e-6 ||M|| FP32), and
    L V^T against the full-SVD shrinkage ``oracle.svd_shrink`` once the
    chain has converged and tau lies above the noise;
  * pf_session_export / pf_session_import: the imported session's next step
    is bitwise the exported session's.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1904_10585_amd import workloads as wl
from gpu_helpers import device_matrix, pf_module

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pf_module()


def sym_case(n, p, config):
    r = max(1, p // 2)
    X, lam, _ = wl.planted(n, r, (4.0, 10.0), (-1.0, 0.5), config=config, index=n * 100 + p)
    U = wl.start_block(n, p, config=config, index=n + p)
    for _ in range(2):
        U = oracle.extract(X, X, U, 6, -1.0, 0.5)["V"]
    return X, U, float(np.abs(lam).max())


def run_ex(pf, X, U, d, a, b, work, resid=True):
    n, p = U.shape
    tdt = torch.float64 if work == "f64" else torch.float32
    Xd = device_matrix(X, tdt)
    Ud = device_matrix(U, tdt)
    theta = torch.zeros(p, dtype=torch.float64, device="cuda")
    info = torch.zeros(8, dtype=torch.int32, device="cuda")
    res = torch.full((p,), -1.0, dtype=torch.float64, device="cuda")
    dsc = pf.desc(n, p, d, a, b, work=pf.PF_F64 if work == "f64" else pf.PF_F32)
    pf.pf_extract_ex(dsc, Xd, Xd, Ud, theta, pf.extras(resid=res if resid else None), info)
    torch.cuda.synchronize()
    return theta.cpu().numpy(), Ud.cpu().double().numpy(), res.cpu().numpy(), info.cpu().numpy()


@pytest.mark.parametrize("n,p,d", [(300, 16, 4), (777, 33, 3), (1030, 64, 5)])
@pytest.mark.parametrize("work", ["f64", "f32"])
def test_residuals_sym(n, p, d, work):
    pf = pf_module()
    X, U, xnorm = sym_case(n, p, config=120)
    if work == "f32":
        X = X.astype(np.float32).astype(np.float64)
        U = U.astype(np.float32).astype(np.float64)
    th, V, res, info = run_ex(pf, X, U, d, -1.0, 0.5, work)
    assert info[0] == 0, info
    ref = oracle.ritz_residuals(lambda B: X @ B, V, th)
    err = np.abs(res - ref).max() / xnorm
    print(f"residuals sym {work} n={n} p={p}: max |gpu - oracle| / ||X|| = {err:.2e}, "
          f"resid range {res.min():.2e} .. {res.max():.2e}")
    assert np.all(res >= 0.0)
    assert err <= (1e-10 if work == "f64" else 1e-6), err


def gram_case(m, n, r, p, config):
    M = wl.lowrank_plus_noise(m, n, r, 0.01, config=config)
    U = wl.start_block(n, p, config=config)
    b = 4.0 * 0.01 ** 2 * m
    for _ in range(4):
        U = oracle.extract_gram(M, M, U, 4, 0.0, b)["V"]
    return M, U, b


@pytest.mark.parametrize("m,n,r,p,d", [(300, 120, 6, 10, 4), (777, 333, 12, 20, 3), (1030, 513, 20, 48, 5)])
@pytest.mark.parametrize("work", ["f64", "f32"])
def test_gram_residuals_and_shrink(m, n, r, p, d, work):
    pf = pf_module()
    M, U, b = gram_case(m, n, r, p, config=121)
    if work == "f32":
        M = M.astype(np.float32).astype(np.float64)
        U = U.astype(np.float32).astype(np.float64)
    tdt = torch.float64 if work == "f64" else torch.float32
    Md = device_matrix(M, tdt)
    Ud = device_matrix(U, tdt)
    theta = torch.zeros(p, dtype=torch.float64, device="cuda")
    info = torch.zeros(8, dtype=torch.int32, device="cuda")
    res = torch.full((p,), -1.0, dtype=torch.float64, device="cuda")
    L = pf.colmajor(m, p, tdt, "cuda", ld=-(-m // 4) * 4 + 4)
    L.fill_(7.0)
    sv = np.linalg.svd(M, compute_uv=False)
    tau = 0.5 * (sv[r - 1] + sv[r])                 # between the signal and the noise
    dsc = pf.desc(n, p, d, 0.0, b, work=pf.PF_F64 if work == "f64" else pf.PF_F32, op=pf.PF_OP_GRAM, m=m)
    pf.pf_extract_ex(dsc, Md, Md, Ud, theta, pf.extras(resid=res, shrink_left=L, shrink_tau=tau), info)
    torch.cuda.synchronize()
    inf = info.cpu().numpy()
    assert inf[0] == 0, inf
    th, V = theta.cpu().numpy(), Ud.cpu().double().numpy()
    Lg = L.cpu().double().numpy()
    mnorm = sv[0]
    ref_r = oracle.ritz_residuals(lambda B: M.T @ (M @ B), V, th)
    err_r = np.abs(res.cpu().numpy() - ref_r).max() / mnorm ** 2
    ref_L = oracle.svd_shrink_factor(M, V, th, tau)
    err_L = np.abs(Lg - ref_L).max() / mnorm
    full = oracle.svd_shrink(M, tau)
    err_full = np.abs(Lg @ V.T - full).max() / mnorm
    print(f"gram {work} m={m} n={n} p={p} tau={tau:.3e}: resid err {err_r:.2e}, factor err {err_L:.2e}, "
          f"vs full-SVD shrinkage {err_full:.2e}")
    tol = 1e-10 if work == "f64" else 1e-6
    assert err_r <= tol, err_r
    assert err_L <= tol, err_L
    # the chain has converged on the signal subspace and tau is above the
    # noise, so the restricted shrinkage is the full one
    assert err_full <= (1e-8 if work == "f64" else 1e-5), err_full


def test_session_residuals_and_checkpoint():
    pf = pf_module()
    n, p, d = 500, 24, 5
    X, U, xnorm = sym_case(n, p, config=122)
    dsc = pf.desc(n, p, d, -1.0, 0.5, work=pf.PF_F64)
    U0 = device_matrix(U, torch.float64)
    h = pf.pf_session_open(dsc, U0)
    Xs = [X]
    for k in range(1, 6):
        Xs.append(Xs[-1] + wl.perturbation(n, 122, k))
    Xd = [device_matrix(Xk, torch.float64) for Xk in Xs]
    res = torch.zeros(p, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    for k in range(3):
        pf.pf_session_step_ex(h, Xd[k], Xd[k], pf.extras(resid=res), stream=stream)
    s, r = pf.pf_session_wait(h)
    assert s == pf.PF_OK
    rh = res.cpu().numpy()
    assert r.resid == res.data_ptr()
    assert r.resid_max == rh.max()
    V = pf.device_to_numpy(r.V, (p, r.ldv), np.float64).T[:n]
    th = pf.device_to_numpy(r.theta, (p,), np.float64)
    ref = oracle.ritz_residuals(lambda B: Xs[2] @ B, V, th)
    assert np.abs(rh - ref).max() <= 1e-10 * xnorm
    # a plain step reports no residuals
    pf.pf_session_step(h, Xd[3], Xd[3], stream=stream)
    s, r = pf.pf_session_wait(h)
    assert s == pf.PF_OK and not r.resid and np.isnan(r.resid_max)

    # checkpoint after four steps, resume in a new session
    Ue = pf.colmajor(n, p, torch.float64, "cuda", ld=n + 4)
    the = torch.zeros(p, dtype=torch.float64, device="cuda")
    st = pf.pf_session_export(h, Ue, the, stream=stream)
    torch.cuda.synchronize()
    assert st.steps == 4 and st.desc.n == n and st.desc.p == p and st.desc.degree == d
    assert torch.equal(the.cpu(), torch.from_numpy(pf.device_to_numpy(r.theta, (p,), np.float64)))
    h2 = pf.pf_session_import(st, Ue, the)
    for k in (4, 5):
        pf.pf_session_step(h, Xd[k], Xd[k], stream=stream)
        pf.pf_session_step(h2, Xd[k], Xd[k], stream=stream)
    s1, r1 = pf.pf_session_wait(h)
    s2, r2 = pf.pf_session_wait(h2)
    assert s1 == s2 == pf.PF_OK
    V1 = pf.device_to_numpy(r1.V, (p, r1.ldv), np.float64).T[:n]
    V2 = pf.device_to_numpy(r2.V, (p, r2.ldv), np.float64).T[:n]
    t1 = pf.device_to_numpy(r1.theta, (p,), np.float64)
    t2 = pf.device_to_numpy(r2.theta, (p,), np.float64)
    print(f"checkpoint: resumed session max |dV| {np.abs(V1 - V2).max():.1e}, max |dtheta| {np.abs(t1 - t2).max():.1e}")
    assert np.array_equal(V1, V2) and np.array_equal(t1, t2)
    pf.pf_session_close(h)
    pf.pf_session_close(h2)


ROCTX_SCRIPT = r"""
import sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
sys.path.insert(0, sys.argv[1] + "/tests")
from gpu_helpers import run_extract
from paper_1904_10585_amd import workloads as wl
X, _, _ = wl.planted(300, 8, (4.0, 10.0), (-1.0, 0.5), config=123)
U = wl.start_block(300, 16, config=123)
th, V, info = run_extract(X, U, 4, -1.0, 0.5, work="f32")
assert info["status"] == 0
np.save(sys.argv[2], th)
"""


def test_roctx_ranges_leave_results_unchanged(tmp_path):
    """With PF_ROCTX=1 the library marks its phases with roctx ranges; the
    extraction itself is unchanged (bitwise)."""
    import os
    import subprocess
    import sys
    from gpu_helpers import run_extract
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    X, _, _ = wl.planted(300, 8, (4.0, 10.0), (-1.0, 0.5), config=123)
    U = wl.start_block(300, 16, config=123)
    th, V, info = run_extract(X, U, 4, -1.0, 0.5, work="f32")
    out = tmp_path / "theta.npy"
    env = dict(os.environ, PF_ROCTX="1")
    subprocess.run([sys.executable, "-c", ROCTX_SCRIPT, root, str(out)], env=env, check=True, timeout=300)
    assert np.array_equal(np.load(out), th)


def test_workspace_cache_is_keyed_by_shape_and_released():
    """pf_extract caches one workspace per stream and shape: other degrees,
    powers and intervals reuse it; pf_workspace_release frees a stream's."""
    pf = pf_module()
    n, p = 300, 16
    X, U, _ = sym_case(n, p, config=124)
    Xd = device_matrix(X, torch.float32)
    stream = torch.cuda.Stream()
    b0, c0 = pf.pf_workspace_cached()
    theta = torch.zeros(p, dtype=torch.float64, device="cuda")
    for d, q, a in ((3, 1, -1.0), (5, 2, -1.0), (8, 1, -1.5)):
        Ud = device_matrix(U, torch.float32)
        pf.pf_extract(pf.desc(n, p, d, a, 0.5, q=q, work=pf.PF_F32), Xd, Xd, Ud, theta, stream=stream)
    b1, c1 = pf.pf_workspace_cached()
    assert c1 == c0 + 1, (c0, c1)
    Ud = device_matrix(U[:, :8], torch.float32)
    pf.pf_extract(pf.desc(n, 8, 3, -1.0, 0.5, work=pf.PF_F32), Xd, Xd, Ud, theta, stream=stream)
    b2, c2 = pf.pf_workspace_cached()
    assert c2 == c0 + 2 and b2 > b1 > b0
    pf.pf_workspace_release(stream)
    b3, c3 = pf.pf_workspace_cached()
    assert (b3, c3) == (b0, c0)
    # the stream works again afterwards (a new workspace)
    Ud = device_matrix(U, torch.float32)
    pf.pf_extract(pf.desc(n, p, 3, -1.0, 0.5, work=pf.PF_F32), Xd, Xd, Ud, theta, stream=stream)
    stream.synchronize()
    assert pf.pf_workspace_cached()[1] == c0 + 1
    pf.pf_workspace_release(stream)
