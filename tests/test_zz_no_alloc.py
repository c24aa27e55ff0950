"""pf_extract_noalloc (the library's fixed device workspace, no allocation)
against pf_extract on the same inputs, through the C ABI: bitwise equal
results on two calls in a row, the second on a smaller problem, in FP32
and FP64 work; and the size limit."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import device_matrix, pf_module
from paper_1904_10585_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pf_module()


def case(n, p, r, work, cfg):
    X, _, _ = wl.planted(n, r, (1.0, 20.0), (-2.0, 0.8), config=cfg)
    U = wl.start_block(n, p, config=cfg)
    U = oracle.extract(X, X, U, 8, -5.0, 0.8)["V"]            # warm start
    if work == "f32":
        X = X.astype(np.float32).astype(np.float64)
        U = U.astype(np.float32).astype(np.float64)
    return X, U


def run(pf, fn, X, U, work, d=8, a=-5.0, b=0.8):
    n, p = U.shape
    tdt, wk = (torch.float64, pf.PF_F64) if work == "f64" else (torch.float32, pf.PF_F32)
    Xd = device_matrix(X, tdt)
    Ud = device_matrix(U, tdt)
    theta = torch.zeros(p, dtype=torch.float64, device="cuda")
    info = torch.zeros(8, dtype=torch.int32, device="cuda")
    fn(pf.desc(n, p, d, a, b, work=wk), Xd, Xd, Ud, theta, info)
    torch.cuda.synchronize()
    return Ud.cpu().numpy(), theta.cpu().numpy(), info.cpu().numpy()


@pytest.mark.parametrize("work", ["f32", "f64"])
def test_noalloc_equals_extract_two_calls(work):
    pf = pf_module()
    # the second call is smaller: its padding must read as zero although the
    # first call left its own values in the shared array
    for (n, p, r, cfg) in ((2100, 48, 24, 150), (700, 16, 8, 151)):
        X, U = case(n, p, r, work, cfg)
        print(f"noalloc {work} n={n} p={p}", flush=True)
        V_ref, th_ref, info_ref = run(pf, pf.pf_extract, X, U, work)
        V, th, info = run(pf, pf.pf_extract_noalloc, X, U, work)
        assert info_ref[0] == 0 and info[0] == 0, (info_ref, info)
        np.testing.assert_array_equal(info, info_ref)
        np.testing.assert_array_equal(th, th_ref)
        np.testing.assert_array_equal(V, V_ref)


def test_noalloc_rejects_oversized_and_gram():
    pf = pf_module()
    cap = pf.pf_extract_noalloc_max_bytes()
    assert cap == 64 << 20
    big = pf.desc(16384, 128, 8, -5.0, 0.8, work=pf.PF_F32)
    assert pf.pf_workspace_size(big) > cap
    Xm = pf.colmajor(16384, 16384, torch.float32, "cuda")
    U = pf.colmajor(16384, 128, torch.float32, "cuda")
    theta = torch.zeros(128, dtype=torch.float64, device="cuda")
    with pytest.raises(pf.PfError) as e:
        pf.pf_extract_noalloc(big, Xm, Xm, U, theta)
    assert e.value.status == pf.PF_ERR_ARG and "bytes" in pf.last_error()
