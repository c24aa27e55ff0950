"""Many independent extractions in one call (pf_extract_batch): the blocks
of a block-diagonal operator, run concurrently on the library's streams,
against sequential pf_extract calls (bitwise) and the oracle (per block)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import compare, device_matrix, pf_module
from paper_1904_10585_amd import workloads as wl

pytestmark = pytest.mark.gpu

# (n, p, degree, work): more blocks than the 8 streams, ragged sizes, both
# work precisions
BLOCKS = [(96, 16, 8, "f64"), (200, 24, 6, "f32"), (333, 32, 10, "f64"), (512, 16, 8, "f32"), (64, 16, 6, "f64"),
          (257, 16, 8, "f32"), (128, 32, 8, "f64"), (150, 16, 6, "f32"), (700, 24, 8, "f64"), (80, 16, 6, "f32")]
# (FP32 blocks stay at degree <= 8: at degree 10 the top planted eigenvalue
# grows ~1e8 times faster than the wanted edge, past single precision)


def block_case(i, n, p, d, work):
    r = p // 2
    X, _, _ = wl.planted(n, r, (2.0, 10.0), (-1.0, 0.5), config=180, index=i)
    a, b = -1.2, 0.6
    U = wl.start_block(n, p, config=181, index=i)
    for _ in range(2):                                  # warm start
        U = oracle.extract(X, X, U, d, a, b)["V"]
    if work == "f32":
        X = X.astype(np.float32).astype(np.float64)
        U = U.astype(np.float32).astype(np.float64)
    return X, U, a, b, r


def device_blocks(pf, cases):
    out = []
    for (n, p, d, work), (X, U, a, b, r) in zip(BLOCKS, cases):
        tdt, wk = (torch.float64, pf.PF_F64) if work == "f64" else (torch.float32, pf.PF_F32)
        Xd = device_matrix(X, tdt)
        out.append((pf.desc(n, p, d, a, b, work=wk), Xd, Xd, device_matrix(U, tdt),
                    torch.zeros(p, dtype=torch.float64, device="cuda"),
                    torch.zeros(8, dtype=torch.int32, device="cuda")))
    return out


def test_batch_matches_sequential_and_oracle():
    pf = pf_module()
    cases = [block_case(i, *blk) for i, blk in enumerate(BLOCKS)]
    seq = device_blocks(pf, cases)
    for dsc, Xf, Xr, U, th, info in seq:
        pf.pf_extract(dsc, Xf, Xr, U, th, info)
    torch.cuda.synchronize()
    bat = device_blocks(pf, cases)
    print(f"batch of {len(bat)} blocks", flush=True)
    pf.pf_extract_batch(bat)
    torch.cuda.synchronize()
    for i, ((n, p, d, work), (X, U0, a, b, r)) in enumerate(zip(BLOCKS, cases)):
        s, t = seq[i], bat[i]
        np.testing.assert_array_equal(t[5].cpu().numpy(), s[5].cpu().numpy(), err_msg=f"info block {i}")
        assert int(t[5][0]) == 0, (i, t[5].cpu().numpy())
        np.testing.assert_array_equal(t[4].cpu().numpy(), s[4].cpu().numpy(), err_msg=f"theta block {i}")
        np.testing.assert_array_equal(t[3].cpu().numpy(), s[3].cpu().numpy(), err_msg=f"V block {i}")
        ref = oracle.extract(X, X, U0, d, a, b)
        V = t[3].cpu().double().numpy()
        rel, sin = compare(t[4].cpu().numpy(), V, ref, r)
        print(f"  block {i} n={n} p={p} {work}: rel {rel:.2e} sin {sin:.2e}")
        tol = (1e-10, 1e-10) if work == "f64" else (1e-5, 1e-4)
        assert rel <= tol[0] and sin <= tol[1], (i, rel, sin)


def test_batch_then_caller_stream_work_sees_results():
    """Work enqueued on the caller's stream after the batch runs after every
    block: a copy of each theta taken on that stream equals the final theta."""
    pf = pf_module()
    cases = [block_case(i, *blk) for i, blk in enumerate(BLOCKS[:9])]
    blocks = device_blocks(pf, cases)
    torch.cuda.synchronize()                            # inputs written on the default stream
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        pf.pf_extract_batch(blocks, stream=st)
        copies = [b[4].clone() for b in blocks]
    st.synchronize()
    torch.cuda.synchronize()
    for c, b in zip(copies, blocks):
        np.testing.assert_array_equal(c.cpu().numpy(), b[4].cpu().numpy())
        assert float(c.abs().max()) > 0.0


def test_extract_on_a_nonblocking_stream_first_use():
    """pf_extract on a non-blocking stream with a shape its workspace cache
    has not seen: the new workspace is cleared on that stream before the
    extraction (a null-stream clear is not ordered with it), so the result
    equals the same extraction on the default stream, bitwise."""
    pf = pf_module()
    n, p, d = 389, 24, 8                                 # a shape no other test uses
    X, U, a, b, r = block_case(40, n, p, d, "f64")
    out = []
    for use_stream in (True, False):
        Xd = device_matrix(X, torch.float64)
        Ud = device_matrix(U, torch.float64)
        th = torch.zeros(p, dtype=torch.float64, device="cuda")
        info = torch.zeros(8, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        if use_stream:
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                pf.pf_extract(pf.desc(n, p, d, a, b, work=pf.PF_F64), Xd, Xd, Ud, th, info, stream=st)
            st.synchronize()
        else:
            pf.pf_extract(pf.desc(n, p, d, a, b, work=pf.PF_F64), Xd, Xd, Ud, th, info)
            torch.cuda.synchronize()
        assert int(info[0]) == 0
        out.append((th.cpu().numpy(), Ud.cpu().numpy()))
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])


def test_batch_of_identical_shapes():
    """17 blocks of one shape (different data): blocks i and i + 8 share a
    pool stream and its cached workspace, one after the other; every block
    still equals its own sequential extraction, bitwise."""
    pf = pf_module()
    shape = (160, 16, 8, "f64")
    cases = [block_case(100 + i, *shape) for i in range(17)]

    def blocks():
        out = []
        for X, U, a, b, r in cases:
            Xd = device_matrix(X, torch.float64)
            out.append((pf.desc(shape[0], shape[1], shape[2], a, b, work=pf.PF_F64), Xd, Xd,
                        device_matrix(U, torch.float64), torch.zeros(shape[1], dtype=torch.float64, device="cuda"),
                        torch.zeros(8, dtype=torch.int32, device="cuda")))
        return out

    seq = blocks()
    for dsc, Xf, Xr, U, th, info in seq:
        pf.pf_extract(dsc, Xf, Xr, U, th, info)
    bat = blocks()
    torch.cuda.synchronize()
    pf.pf_extract_batch(bat)
    torch.cuda.synchronize()
    for i, (s, t) in enumerate(zip(seq, bat)):
        np.testing.assert_array_equal(t[5].cpu().numpy(), s[5].cpu().numpy(), err_msg=f"info block {i}")
        np.testing.assert_array_equal(t[4].cpu().numpy(), s[4].cpu().numpy(), err_msg=f"theta block {i}")
        np.testing.assert_array_equal(t[3].cpu().numpy(), s[3].cpu().numpy(), err_msg=f"V block {i}")
