"""The serving loop (pf_server_*) on the GPU: graph replays and concurrent
sessions give bitwise the results of eager pf_session stepping on the same
inputs, a session's results do not depend on what runs beside it, and
admission keeps the resident footprint within the HBM budget."""
import math

import numpy as np
import pytest
import torch

from paper_1904_10585_amd import workloads as wl
from gpu_helpers import device_matrix, pf_module

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pf_module()


class Case:
    """One session: planted symmetric X (FP32, device), degree, interval."""

    def __init__(self, n, p, d, idx):
        self.n, self.p, self.d, self.idx = n, p, d, idx
        r = max(1, p // 2)
        X, _, _ = wl.planted(n, r, (4.0, 10.0), (-1.0, 0.5), config=110, index=idx)
        self.X0 = X.astype(np.float32)
        self.a, self.b = -1.0, 0.5

    def fresh_x(self):
        return device_matrix(self.X0, torch.float32)

    def desc(self):
        pf = pf_module()
        return pf.desc(self.n, self.p, self.d, self.a, self.b, work=pf.PF_F32)

    def perturb(self, Xd, k):
        """X_k = X_{k-1} + 1e-3 sym(G)/sqrt(n), seeded by (session, step)."""
        g = torch.Generator(device="cuda")
        g.manual_seed(7919 * self.idx + k)
        G = torch.randn((self.n, self.n), generator=g, device="cuda", dtype=torch.float32)
        Xd.add_((G + G.t()) * (0.5e-3 / math.sqrt(self.n)))


def read_result(pf, r, n, p):
    th = pf.device_to_numpy(r.theta, (p,), np.float64)
    V = pf.device_to_numpy(r.V, (p, r.ldv), np.float32).T[:n].copy()
    return th, V


def run_eager(cases, steps):
    pf = pf_module()
    out = {}
    for c in cases:
        X = c.fresh_x()
        h = pf.pf_session_open(c.desc(), seed=c.idx)
        res = []
        for k in range(steps):
            if k:
                c.perturb(X, k)
            pf.pf_session_step(h, X, X)
            s, r = pf.pf_session_wait(h)
            assert s == pf.PF_OK, s
            res.append(read_result(pf, r, c.n, c.p))
        torch.cuda.synchronize()
        pf.pf_session_close(h)
        out[c.idx] = res
    return out


def run_server(cases, steps, flags=0, streams=0):
    """All sessions advance in lockstep: submit step k of every session,
    wait for their events, read results, perturb every X, repeat."""
    pf = pf_module()
    srv = pf.pf_server_create(64 << 30, streams=streams, flags=flags)
    try:
        Xs = {c.idx: c.fresh_x() for c in cases}
        ids = {c.idx: pf.pf_server_open(srv, c.desc(), seed=c.idx, operator_bytes=c.n * c.n * 4) for c in cases}
        out = {c.idx: [] for c in cases}
        graphs = {c.idx: [] for c in cases}
        for k in range(steps):
            torch.cuda.synchronize()
            for c in cases:
                pf.pf_server_submit(srv, ids[c.idx], Xs[c.idx], Xs[c.idx], tag=k)
            got = {}
            while len(got) < len(cases):
                for ev in pf.pf_server_poll(srv, timeout_s=5.0):
                    got[ev.session] = (ev.status, ev.step, ev.tag, ev.graph)
            for c in cases:
                st, step, tag, graph = got[ids[c.idx]]
                assert st == pf.PF_OK and step == k and tag == k, (st, step, tag)
                graphs[c.idx].append(graph)
                out[c.idx].append(read_result(pf, pf.pf_server_result(srv, ids[c.idx]), c.n, c.p))
            for c in cases:
                if k + 1 < steps:
                    c.perturb(Xs[c.idx], k + 1)
        torch.cuda.synchronize()
        stats = pf.pf_server_stats(srv)
        for c in cases:
            pf.pf_server_close(srv, ids[c.idx])
    finally:
        pf.pf_server_destroy(srv)
    return out, graphs, stats


CASES = [(1000, 16, 6, 1), (777, 32, 8, 2), (2048, 48, 10, 3), (300, 8, 4, 4), (1536, 96, 6, 5)]


def test_server_batches_match_eager_sessions():
    """Sessions of different n, p and degree served together: every pass of
    the worker runs their steps as one batch of grouped launches, and each
    session's steps are bitwise the eager session's."""
    cases = [Case(*c) for c in CASES]
    steps = 4
    eager = run_eager(cases, steps)
    served, graphs, stats = run_server(cases, steps)
    for c in cases:
        assert graphs[c.idx] == [0] * steps, graphs[c.idx]
        for k in range(steps):
            np.testing.assert_array_equal(served[c.idx][k][0], eager[c.idx][k][0], err_msg=f"theta {c.idx} {k}")
            np.testing.assert_array_equal(served[c.idx][k][1], eager[c.idx][k][1], err_msg=f"V {c.idx} {k}")
    # all ready sessions of a pass form one batch (lockstep submission here)
    assert stats.batched_steps == len(cases) * steps and stats.batches < len(cases) * steps, (stats.batches,
                                                                                       stats.batched_steps)


def test_server_graphs_match_eager_sessions():
    """Without batching, warm steps replayed from captured graphs, with
    eager work (the X perturbation, reads of every result) between replays,
    are bitwise the eager session's steps."""
    pf = pf_module()
    cases = [Case(*c) for c in CASES[:3]]
    steps = 5
    eager = run_eager(cases, steps)
    served, graphs, stats = run_server(cases, steps, flags=pf.PF_SERVER_NO_GROUPING)
    for c in cases:
        assert graphs[c.idx] == [0] + [1] * (steps - 1), graphs[c.idx]
        for k in range(steps):
            np.testing.assert_array_equal(served[c.idx][k][0], eager[c.idx][k][0], err_msg=f"theta {c.idx} {k}")
            np.testing.assert_array_equal(served[c.idx][k][1], eager[c.idx][k][1], err_msg=f"V {c.idx} {k}")
    assert stats.captures == len(cases) and stats.graph_launches == len(cases) * (steps - 1)
    assert stats.batches == 0


def test_server_alone_equals_mix():
    """A session's results are the same alone and batched with four others
    of different n, p and degree."""
    steps = 4
    alone, _, _ = run_server([Case(*CASES[0])], steps)
    mix, _, st = run_server([Case(*c) for c in CASES], steps)
    assert st.batches > 0
    idx = CASES[0][3]
    for k in range(steps):
        np.testing.assert_array_equal(alone[idx][k][0], mix[idx][k][0])
        np.testing.assert_array_equal(alone[idx][k][1], mix[idx][k][1])


def test_server_without_graphs_matches():
    pf = pf_module()
    cases = [Case(*CASES[1])]
    a, ga, _ = run_server(cases, 3, flags=pf.PF_SERVER_NO_GROUPING)
    b, gb, _ = run_server([Case(*CASES[1])], 3, flags=pf.PF_SERVER_NO_GRAPHS | pf.PF_SERVER_NO_GROUPING)
    assert gb[CASES[1][3]] == [0, 0, 0]
    for k in range(3):
        np.testing.assert_array_equal(a[CASES[1][3]][k][1], b[CASES[1][3]][k][1])


def test_served_batch_matches_oracle():
    """Served, batched steps against the FP64 oracle fed the same U_in (the
    previous served V) and the same X_k: FP32 tolerance on warm steps."""
    import oracle
    pf = pf_module()
    cases = [Case(*CASES[0]), Case(*CASES[1]), Case(*CASES[3])]
    steps = 4
    srv = pf.pf_server_create(16 << 30)
    try:
        Xs = {c.idx: c.fresh_x() for c in cases}
        ids = {c.idx: pf.pf_server_open(srv, c.desc(), seed=c.idx) for c in cases}
        U_prev = {}
        for k in range(steps):
            torch.cuda.synchronize()
            Xh = {c.idx: Xs[c.idx].cpu().double().numpy() for c in cases}
            for c in cases:
                pf.pf_server_submit(srv, ids[c.idx], Xs[c.idx], Xs[c.idx], tag=k)
            got = 0
            while got < len(cases):
                for ev in pf.pf_server_poll(srv, timeout_s=5.0):
                    assert ev.status == pf.PF_OK
                    got += 1
            for c in cases:
                th, V = read_result(pf, pf.pf_server_result(srv, ids[c.idx]), c.n, c.p)
                V = V.astype(np.float64)
                if k >= 2:
                    ref = oracle.extract(Xh[c.idx], Xh[c.idx], U_prev[c.idx], c.d, c.a, c.b)
                    r = max(1, c.p // 2)
                    rel = oracle.ritz_rel_err(th, ref["theta"], r)
                    Qg, _ = np.linalg.qr(V[:, :r])
                    sin = oracle.sin_theta(Qg, ref["V"][:, :r])
                    print(f"served session {c.idx} step {k}: rel {rel:.2e} sin {sin:.2e}")
                    assert rel <= 1e-5 and sin <= 1e-4, (c.idx, k, rel, sin)
                U_prev[c.idx] = V
            for c in cases:
                if k + 1 < steps:
                    c.perturb(Xs[c.idx], k + 1)
        assert pf.pf_server_stats(srv).batches > 0
    finally:
        pf.pf_server_destroy(srv)


def test_server_admission_within_budget():
    """With room for two sessions, four sessions are served two at a time:
    the others wait, and are admitted as closed sessions free memory."""
    pf = pf_module()
    n, p, steps = 512, 16, 3
    d = pf.desc(n, p, 4, -1.0, 0.5, work=pf.PF_F32)
    declared = 64 << 20                      # operator bytes each session declares
    fp = pf.pf_workspace_size(d) + declared + (1 << 20)
    budget = 2 * fp + fp // 2                 # two sessions fit, three do not
    X = device_matrix(Case(n, p, 4, 9).X0, torch.float32)
    srv = pf.pf_server_create(budget)
    try:
        ids = [pf.pf_server_open(srv, d, seed=i, operator_bytes=declared) for i in range(4)]
        for sid in ids:
            for k in range(steps):
                pf.pf_server_submit(srv, sid, X, X, tag=k)
        done = {sid: 0 for sid in ids}
        max_active, saw_waiting = 0, False
        order = []
        while sum(done.values()) < 4 * steps:
            st = pf.pf_server_stats(srv)
            assert st.used_bytes <= budget
            max_active = max(max_active, st.active)
            saw_waiting = saw_waiting or st.waiting > 0
            for ev in pf.pf_server_poll(srv, timeout_s=5.0):
                assert ev.status == pf.PF_OK
                done[ev.session] += 1
                if done[ev.session] == steps:
                    order.append(ev.session)
                    pf.pf_server_close(srv, ev.session)
        assert max_active == 2 and saw_waiting
        assert sorted(order[:2]) == ids[:2]           # first come, first admitted
    finally:
        pf.pf_server_destroy(srv)


def test_server_reports_step_errors_and_continues():
    """A non-finite operator fails that session's step with its status; the
    other session's steps are unaffected."""
    pf = pf_module()
    good, bad = Case(*CASES[3]), Case(300, 8, 4, 6)
    Xg, Xb = good.fresh_x(), bad.fresh_x()
    Xb[3, 5] = float("nan")
    torch.cuda.synchronize()
    srv = pf.pf_server_create(8 << 30)
    try:
        ig = pf.pf_server_open(srv, good.desc(), seed=1)
        ib = pf.pf_server_open(srv, bad.desc(), seed=2)
        for k in range(2):
            pf.pf_server_submit(srv, ig, Xg, Xg, tag=k)
            pf.pf_server_submit(srv, ib, Xb, Xb, tag=k)
        evs = []
        while len(evs) < 4:
            evs += pf.pf_server_poll(srv, timeout_s=5.0)
        for ev in evs:
            want = pf.PF_OK if ev.session == ig else pf.PF_ERR_NONFINITE
            assert ev.status == want, (ev.session, ev.status)
    finally:
        pf.pf_server_destroy(srv)


def gram_fp8_operands(m, n, config):
    """M = A B^T + 0.01 N(0,1) (rank 10) as FP32 on the device, its FP8-E4M3
    codes with per-128x128 scales from pf_quantize, and ||M||_F^2."""
    pf = pf_module()
    M = wl.lowrank_plus_noise(m, n, 10, 0.01, config=config).astype(np.float32)
    Mr = device_matrix(M, torch.float32)
    codes = pf.colmajor(m, n, torch.uint8, "cuda", ld=-(-m // 16) * 16)
    scales = torch.zeros((-(-n // 128), -(-m // 128)), dtype=torch.float32, device="cuda").t()
    pf.pf_quantize(codes, scales, 128, pf.PF_F8E4M3, Mr)
    torch.cuda.synchronize()
    return (codes, scales, 128), Mr, float((Mr.double() ** 2).sum())


def test_server_gram_fp8_session_matches_eager():
    """A Gram-form session (FP8 M in the filter, FP32 M for Rayleigh-Ritz, M
    fixed over the chain with PF_FLAG_OPERATOR_UNCHANGED, scaled recurrence)
    served next to a planted session: its graph-replayed warm steps are
    bitwise the eager session's steps."""
    pf = pf_module()
    m, n, p, d, steps = 640, 300, 24, 6, 5
    Mf, Mr, fro2 = gram_fp8_operands(m, n, config=111)
    dsc = pf.desc(n, p, d, 0.0, 4.0 * 0.01 ** 2 * m, work=pf.PF_F32, op=pf.PF_OP_GRAM, m=m,
                  flags=pf.PF_FLAG_SCALED | pf.PF_FLAG_OPERATOR_UNCHANGED, spec_ub=fro2)
    h = pf.pf_session_open(dsc, seed=11)
    eager = []
    for _ in range(steps):
        pf.pf_session_step(h, Mf, Mr)
        s, r = pf.pf_session_wait(h)
        assert s == pf.PF_OK and r.status == 0, (s, r.status)
        eager.append(read_result(pf, r, n, p))
    torch.cuda.synchronize()
    pf.pf_session_close(h)

    other = Case(*CASES[0])
    srv = pf.pf_server_create(64 << 30, streams=2)
    try:
        Xo = other.fresh_x()
        gid = pf.pf_server_open(srv, dsc, seed=11, operator_bytes=n * m * 5)
        oid = pf.pf_server_open(srv, other.desc(), seed=other.idx, operator_bytes=other.n * other.n * 4)
        graphs = []
        for k in range(steps):
            torch.cuda.synchronize()
            pf.pf_server_submit(srv, gid, Mf, Mr, tag=k)
            pf.pf_server_submit(srv, oid, Xo, Xo, tag=k)
            got = {}
            while len(got) < 2:
                for ev in pf.pf_server_poll(srv, timeout_s=5.0):
                    got[ev.session] = (ev.status, ev.step, ev.graph)
            assert got[gid][0] == pf.PF_OK and got[gid][1] == k and got[oid][0] == pf.PF_OK
            graphs.append(got[gid][2])
            th, V = read_result(pf, pf.pf_server_result(srv, gid), n, p)
            np.testing.assert_array_equal(th, eager[k][0], err_msg=f"theta step {k}")
            np.testing.assert_array_equal(V, eager[k][1], err_msg=f"V step {k}")
            if k + 1 < steps:
                other.perturb(Xo, k + 1)
        torch.cuda.synchronize()
        assert graphs == [0] + [1] * (steps - 1), graphs
        pf.pf_server_close(srv, gid)
        pf.pf_server_close(srv, oid)
    finally:
        pf.pf_server_destroy(srv)


def test_served_bf16_session_matches_oracle():
    """A precision-form session (the filter on a BF16 copy of X, made by
    pf_quantize each step; Rayleigh-Ritz on the FP32 X) batched with an
    FP32 session: warm steps against the oracle fed the dequantised copy
    for the filter and the FP32 X for Rayleigh-Ritz (same math), at the
    FP32 tolerance."""
    import oracle
    pf = pf_module()
    c, other = Case(*CASES[1]), Case(*CASES[0])
    steps = 4
    srv = pf.pf_server_create(16 << 30)
    try:
        Xf, Xo = c.fresh_x(), other.fresh_x()
        Xq = pf.colmajor(c.n, c.n, torch.bfloat16, "cuda", ld=-(-c.n // 8) * 8)   # 16-byte columns
        sid = pf.pf_server_open(srv, c.desc(), seed=c.idx)
        oid = pf.pf_server_open(srv, other.desc(), seed=other.idx)
        U_prev = None
        for k in range(steps):
            pf.pf_quantize(Xq, None, 0, pf.PF_BF16, Xf)
            torch.cuda.synchronize()
            Xh = Xf.cpu().double().numpy()
            Xqh = Xq.cpu().double().numpy()
            pf.pf_server_submit(srv, sid, Xq, Xf, tag=k)
            pf.pf_server_submit(srv, oid, Xo, Xo, tag=k)
            got = 0
            while got < 2:
                for ev in pf.pf_server_poll(srv, timeout_s=5.0):
                    assert ev.status == pf.PF_OK
                    got += 1
            th, V = read_result(pf, pf.pf_server_result(srv, sid), c.n, c.p)
            V = V.astype(np.float64)
            if k >= 2:
                np.testing.assert_array_equal(Xqh, oracle.bf16_round(Xh))
                ref = oracle.extract(Xqh, Xh, U_prev, c.d, c.a, c.b)
                r = c.p // 2
                rel = oracle.ritz_rel_err(th, ref["theta"], r)
                sin = oracle.sin_theta(np.linalg.qr(V[:, :r])[0], ref["V"][:, :r])
                print(f"served bf16 session step {k}: rel {rel:.2e} sin {sin:.2e}")
                assert rel <= 1e-5 and sin <= 1e-4, (k, rel, sin)
            U_prev = V
            if k + 1 < steps:
                c.perturb(Xf, k + 1)
                other.perturb(Xo, k + 1)
        assert pf.pf_server_stats(srv).batches > 0
    finally:
        pf.pf_server_destroy(srv)
