"""Extractions on a caller-supplied operator (pf_extract_op,
pf_session_step_op): a sparse symmetric A applied by the caller's SpMM in
the callback, against the oracle on the dense form of the same A."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import compare, device_matrix, pf_module, grade_f64
from paper_1904_10585_amd import workloads as wl

pytestmark = pytest.mark.gpu


def sparse_case(n, r, density, seed):
    """A = S + D: S sparse symmetric with N(0, 0.3^2) entries at a given
    density, D diagonal with r entries in [4, 12] at random positions (the
    wanted part) and the rest in [-1, 0.5].  Returns the dense FP64 A and
    its COO index/value arrays."""
    g = wl.rng(seed, 0)
    nnz = int(density * n * n / 2)
    i = g.integers(0, n, nnz)
    j = g.integers(0, n, nnz)
    v = 0.3 * g.standard_normal(nnz)
    d = g.uniform(-1.0, 0.5, n)
    d[g.choice(n, r, replace=False)] = g.uniform(4.0, 12.0, r)
    A = np.zeros((n, n))
    np.add.at(A, (i, j), v)
    A = A + A.T + np.diag(d)
    ii, jj = np.nonzero(A)
    return A, ii, jj, A[ii, jj]


def spmm_operator(pf, n, ii, jj, vals, dtype):
    S = torch.sparse_coo_tensor(torch.from_numpy(np.vstack([ii, jj])), torch.from_numpy(vals).to(dtype),
                                (n, n), device="cuda").coalesce()

    def apply(Y, AY):
        AY.copy_(torch.sparse.mm(S, Y))

    return pf.make_operator(apply, n, dtype)


def interval(A, r):
    lam = np.linalg.eigvalsh(A)
    return lam[0] - 0.1, lam[-r - 1] + 0.05


@pytest.mark.parametrize("n,p,r,d,work", [(700, 16, 6, 8, "f64"), (2000, 32, 12, 10, "f64"), (2000, 32, 12, 10, "f32"),
                                          (777, 20, 8, 6, "f32")])
def test_sparse_operator_matches_oracle(n, p, r, d, work):
    pf = pf_module()
    A, ii, jj, vals = sparse_case(n, r, 0.004, seed=n + p)
    a, b = interval(A, r)
    f64 = work == "f64"
    tdt, wk = (torch.float64, pf.PF_F64) if f64 else (torch.float32, pf.PF_F32)
    As = A if f64 else A.astype(np.float32).astype(np.float64)
    U = wl.start_block(n, p, config=140, index=n)
    U = oracle.extract(As, As, U, d, a, b)["V"]            # warm start
    Uin = U if f64 else U.astype(np.float32).astype(np.float64)
    ref = oracle.extract(As, As, Uin, d, a, b)
    op = spmm_operator(pf, n, ii, jj, vals, tdt)
    Ud = device_matrix(Uin, tdt)
    theta = torch.zeros(p, dtype=torch.float64, device="cuda")
    info = torch.zeros(8, dtype=torch.int32, device="cuda")
    print(f"operator n={n} p={p} d={d} {work}", flush=True)
    pf.pf_extract_op(pf.desc(n, p, d, a, b, work=wk), op, Ud, theta, info)
    torch.cuda.synchronize()
    assert int(info[0]) == 0
    V = Ud.cpu().numpy().astype(np.float64)
    rel, sin = compare(theta.cpu().numpy(), V, ref, r)
    print(f"  rel {rel:.2e} sin {sin:.2e}")
    if f64:
        assert rel <= 1e-10 and sin <= 1e-10, (rel, sin)
    else:
        assert rel <= 1e-5 and sin <= 1e-4, (rel, sin)


@pytest.mark.parametrize("work", ["f64", "f32"])
def test_sparse_operator_session_chain(work):
    """A session stepped on the operator (the operator's values drift each
    step, as the iterates of an outer method would) matches the oracle
    step by step."""
    pf = pf_module()
    n, p, r, d = 1500, 24, 10, 8
    A, ii, jj, vals = sparse_case(n, r, 0.004, seed=141)
    a, b = interval(A, r)
    f64 = work == "f64"
    tdt, wk = (torch.float64, pf.PF_F64) if f64 else (torch.float32, pf.PF_F32)
    U = wl.start_block(n, p, config=141)
    h = pf.pf_session_open(pf.desc(n, p, d, a, b, work=wk), device_matrix(U, tdt), seed=0)
    g = wl.rng(141, 1)
    try:
        for k in range(4):
            if k:
                vals = vals * (1.0 + 1e-3 * g.standard_normal(vals.shape))
                vals = 0.5 * (vals + pf_sym_partner(ii, jj, vals, n))
            Ak = np.zeros((n, n))
            Ak[ii, jj] = vals
            As = Ak if f64 else Ak.astype(np.float32).astype(np.float64)
            op = spmm_operator(pf, n, ii, jj, vals, tdt)
            pf.pf_session_step_op(h, op)
            s, res = pf.pf_session_wait(h)
            assert s == pf.PF_OK and res.status == 0
            ref = oracle.extract(As, As, U, d, a, b)
            th = pf.device_to_numpy(res.theta, (p,), np.float64)
            V = pf.device_to_numpy(res.V, (p, res.ldv), np.float64 if f64 else np.float32).T[:n].astype(np.float64)
            rel, sin = compare(th, V, ref, r)
            print(f"operator chain {work} step {k}: rel {rel:.2e} sin {sin:.2e}")
            if f64:
                grade_f64(th, V, As, U, d, a, b, r, cold=(k == 0), label=f"operator chain f64 step {k}")
            elif k >= 2:
                assert rel <= 1e-5 and sin <= 1e-4, (k, rel, sin)
            U = V
    finally:
        pf.pf_session_close(h)


def pf_sym_partner(ii, jj, vals, n):
    """Values at the transposed positions (the pattern is symmetric)."""
    pos = {(int(a), int(b)): t for t, (a, b) in enumerate(zip(ii, jj))}
    return np.array([vals[pos[(int(b), int(a))]] for a, b in zip(ii, jj)])


def test_operator_error_propagates():
    """A callback that reports an error aborts the extraction with that
    status (the caller's failure, not the library's)."""
    pf = pf_module()
    n, p = 300, 16
    op = pf.make_operator(lambda Y, AY: (_ for _ in ()).throw(RuntimeError("operator failed")), n, torch.float64)
    Ud = device_matrix(wl.start_block(n, p, config=142), torch.float64)
    theta = torch.zeros(p, dtype=torch.float64, device="cuda")
    with pytest.raises(pf.PfError) as e:
        pf.pf_extract_op(pf.desc(n, p, 4, -2.0, 0.5, work=pf.PF_F64), op, Ud, theta)
    assert e.value.status == pf.PF_ERR_DEVICE
    torch.cuda.synchronize()
