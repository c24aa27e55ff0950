"""Shared helpers of the GPU parity tests: run one extraction through the
C ABI on seeded inputs and compare with the oracle."""
import numpy as np
import torch

import oracle


def pf_module():
    from paper_1904_10585_amd import pf
    return pf


def device_matrix(A, dtype, ld=None):
    pf = pf_module()
    rows, cols = A.shape
    ld = -(-(ld or rows) // 4) * 4            # 16-byte aligned columns
    t = pf.colmajor(rows, cols, dtype, "cuda", ld=ld)
    t.copy_(torch.from_numpy(np.ascontiguousarray(A)).to(dtype))
    return t


def run_extract(X, U, degree, a, b, work="f64", q=1, flags=0, Xrr=None, ld_pad=0):
    """One pf_extract on host arrays; returns (theta, V, info dict)."""
    pf = pf_module()
    n, p = U.shape
    tdt = torch.float64 if work == "f64" else torch.float32
    wk = pf.PF_F64 if work == "f64" else pf.PF_F32
    ldx = n + ld_pad
    Xd = device_matrix(X, tdt, ld=ldx)
    Xr = Xd if Xrr is None else device_matrix(Xrr, tdt, ld=ldx)
    Ud = device_matrix(U, tdt, ld=n + ld_pad)
    theta = torch.zeros(p, dtype=torch.float64, device="cuda")
    info = torch.zeros(8, dtype=torch.int32, device="cuda")
    d = pf.desc(n, p, degree, a, b, q=q, work=wk, flags=flags)
    pf.pf_extract(d, Xd, Xr, Ud, theta, info)
    torch.cuda.synchronize()
    inf = info.cpu().numpy()
    return (theta.cpu().numpy(), Ud.cpu().double().numpy(),
            {"status": int(inf[0]), "n_pos": int(inf[1]), "dense_rr": int(inf[2]),
             "dense_pre": int(inf[3]), "deficient": int(inf[4])})


def compare(theta_g, V_g, ref, r):
    """(Ritz relative error, largest sin-angle) on the leading r Ritz pairs."""
    rel = oracle.ritz_rel_err(theta_g, ref["theta"], r)
    Vg = V_g[:, :r]
    Qg, _ = np.linalg.qr(Vg)
    sin = oracle.sin_theta(Qg, ref["V"][:, :r])
    return rel, sin


def grade_f64(theta_g, V_g, X, U, degree, a, b, r, q=1, cold=False, label=""):
    """FP64 parity of one step, asserted at the FP64 tolerance.

    Warm step: Ritz relative error and sin-angle <= 1e-10 against the oracle
    fed the same U and X.  Cold step (a random start block): the filtered
    block is ill-conditioned (kappa after column equilibration up to ~1e8)
    and the FP64 oracle's own top-r subspace can be off by more than 1e-10
    (its Householder QR and unscaled recurrence are accurate to about
    eps * kappa), so the reference is the extended-precision extraction,
    against which both are asserted at 1e-10.  Returns (rel, sin)."""
    if not cold:
        ref = oracle.extract(X, X, U, degree, a, b, q=q)
        rel, sin = compare(theta_g, V_g, ref, r)
        print(f"{label} rel {rel:.2e} sin {sin:.2e}", flush=True)
        assert rel <= 1e-10 and sin <= 1e-10, (label, rel, sin)
        return rel, sin
    ext = oracle.extract_longdouble(X, U, degree, a, b, q=q)
    Y = ext["Y"].astype(np.float64)
    sv = np.linalg.svd(Y / np.linalg.norm(Y, axis=0), compute_uv=False)
    ekappa = np.finfo(np.float64).eps * sv[0] / sv[-1]
    refL = {"theta": ext["theta"].astype(np.float64), "V": ext["V"].astype(np.float64)}
    rel, sin = compare(theta_g, V_g, refL, r)
    ref = oracle.extract(X, X, U, degree, a, b, q=q)
    rel_o, sin_o = compare(ref["theta"], ref["V"], refL, r)
    print(f"{label} cold, against extended precision: rel {rel:.2e} sin {sin:.2e} (FP64 oracle: rel {rel_o:.2e}"
          f" sin {sin_o:.2e}; eps*kappa(Y_d) {ekappa:.2e})", flush=True)
    assert rel <= 1e-10 and sin <= 1e-10, (label, rel, sin)
    return rel, sin
