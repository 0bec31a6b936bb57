"""GPU parity of the batched line: many matrices of uneven order (general and
Hermitian positive definite mixed) inverted by one persistent launch, against
the oracle's complex Gaussian elimination (Algorithm 4) and complex Cholesky
inversion (Algorithm 8), in FP64 and FP32; status words for singular and
indefinite members; replays of a captured HIP graph; the autotuner."""
import numpy as np
import pytest

import oracle
from paper_2208_01239_amd import inputs
from _helpers import relF

pytestmark = pytest.mark.gpu

U64, U32 = 2.0 ** -53, 2.0 ** -24
SIZES = [1, 2, 3, 5, 8, 16, 17, 31, 33, 64, 65, 100, 128, 130, 200, 257, 300, 512]


@pytest.fixture(scope="module")
def h():
    import paper_2208_01239_amd as fi
    hd = fi.Handle(0)
    yield hd
    hd.close()


@pytest.fixture(scope="module")
def mixed():
    mats, kinds, refs = [], [], []
    for i, n in enumerate(SIZES):
        for kind in (0, 1):
            A, B = inputs.general(n, 1000 + i) if kind == 0 else inputs.hpd(n, 2000 + i)
            r = oracle.cinv_lu(A, B) if kind == 0 else oracle.cinv_chol(A, B)
            kC = np.linalg.cond(A + B @ np.linalg.solve(A, B))
            mats.append((A, B)); kinds.append(kind); refs.append((r[0], r[1], kC))
    return mats, kinds, refs


def _run(h, mats, kinds, dtype):
    import torch
    import paper_2208_01239_amd as fi
    As = [torch.from_numpy(A).to(dtype).cuda() for A, _ in mats]
    Bs = [torch.from_numpy(B).to(dtype).cuda() for _, B in mats]
    Xr, Xi, info = fi.frob_inv_batched(h, As, Bs, kinds)
    return [x.double().cpu().numpy() for x in Xr], [x.double().cpu().numpy() for x in Xi], info


def test_batched_fp64_matches_oracle(h, mixed):
    """FP64: every member within max(1e-10, 16 u kappa_2(C)) of the oracle
    (C = A + B A^{-1} B bounds the Frobenius route's forward error)."""
    import torch
    mats, kinds, refs = mixed
    Xr, Xi, info = _run(h, mats, kinds, torch.float64)
    assert np.all(info == 0)
    for i, (A, _) in enumerate(mats):
        e = relF(Xr[i], Xi[i], refs[i][0], refs[i][1])
        assert e <= max(1e-10, 16 * U64 * refs[i][2]), (A.shape[0], kinds[i], e)


def test_batched_fp32_matches_oracle(h, mixed):
    """FP32 storage and arithmetic: within 16 u32 kappa_2(C) of the FP64 oracle
    (inputs rounded to FP32 first; the oracle sees the FP64 values)."""
    import torch
    mats, kinds, refs = mixed
    Xr, Xi, info = _run(h, mats, kinds, torch.float32)
    assert np.all(info == 0)
    for i, (A, _) in enumerate(mats):
        e = relF(Xr[i], Xi[i], refs[i][0], refs[i][1])
        assert e <= 16 * U32 * max(refs[i][2], 1.0), (A.shape[0], kinds[i], e)


def test_batched_status_words(h):
    """Members whose factorizations fail, mixed with good ones: a singular
    real part (diag(0, 1, i): A = diag(0, 1, 0) singular at column 1), an
    indefinite "HPD" member (-I), C singular (A = I, B = [[0, 1], [-1, 0]]:
    C = I + B^2 = 0, Lemma 2.3) and C indefinite (B doubled: C = -3 I, Lemma
    4.5).  Each status word equals the oracle's info code; the good members
    are unaffected.  (The same batch runs on the CPU emulation of the kernel in
    test_batched_emu.py, which checks that every thread passes the same
    barriers.)  An invalid kind is rejected on the host before any launch."""
    import torch
    import paper_2208_01239_amd as fi
    J = np.array([[0.0, 1.0], [-1.0, 0.0]])
    good = inputs.general(40, 5)
    hp = inputs.hpd(30, 6)
    failing = [((np.diag([0.0, 1.0, 0.0]), np.diag([0.0, 0.0, 1.0])), 0), ((-np.eye(4), np.zeros((4, 4))), 1),
               ((np.eye(2), J.copy()), 0), ((np.eye(2), 2.0 * J), 1)]
    mats = [good] + [m for m, _ in failing] + [hp, good]
    kinds = [0] + [k for _, k in failing] + [1, 0]
    expected = [0] + [(oracle.frob_lu(*m) if k == 0 else oracle.frob_chol(*m))[2] for m, k in failing] + [0, 0]
    assert expected[1:5] == [1000001, 1000001, 2000001, 2000001]
    Xr, Xi, info = _run(h, mats, kinds, torch.float64)
    assert list(info) == expected, (list(info), expected)
    r = oracle.cinv_lu(*good)
    assert relF(Xr[0], Xi[0], r[0], r[1]) <= 1e-10 and relF(Xr[6], Xi[6], r[0], r[1]) <= 1e-10
    r = oracle.cinv_chol(*hp)
    assert relF(Xr[5], Xi[5], r[0], r[1]) <= 1e-10
    A = torch.eye(4, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        fi.BatchedPlan([A], [A], [7])


def test_batched_rejects_invalid_entries_before_launch(h):
    import torch
    import paper_2208_01239_amd as fi
    A = torch.eye(4, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        fi.BatchedPlan([A], [A], [7])
    big = torch.eye(513, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        fi.BatchedPlan([big], [big], [0])


def test_batched_graph_replays(h):
    """The launch (queue reset kernel + persistent kernel) captured in a HIP
    graph and replayed three times, with eager work and synchronization
    between replays; every replay reproduces the eager result exactly."""
    import torch
    import paper_2208_01239_amd as fi
    mats = [inputs.general(n, 30 + n) if n % 2 else inputs.hpd(n, 30 + n) for n in (20, 37, 64, 100, 9)]
    kinds = [0 if n % 2 else 1 for n in (20, 37, 64, 100, 9)]
    As = [torch.from_numpy(A).cuda() for A, _ in mats]
    Bs = [torch.from_numpy(B).cuda() for _, B in mats]
    plan = fi.BatchedPlan(As, Bs, kinds)
    plan.launch(h)                       # eager: also grows the workspace to its final size
    torch.cuda.synchronize()
    ref = [(x.clone(), y.clone()) for x, y in zip(plan.Xr, plan.Xi)]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.launch(h)
    for rep in range(3):
        for x, y in zip(plan.Xr, plan.Xi):
            x.fill_(float("nan")); y.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (x, y), (rx, ry) in zip(zip(plan.Xr, plan.Xi), ref):
            assert torch.equal(x, rx) and torch.equal(y, ry), rep
        assert int((plan.info_dev != 0).sum()) == 0


def test_batched_graph_survives_workspace_growth(h):
    """A launch captured into a graph keeps its workspace: a later call on the
    same handle that needs a larger workspace (a general inversion of order
    1500) sets the captured one aside instead of freeing it, so replays still
    reproduce the eager result.  Capturing a launch that would have to grow
    the workspace is refused (FROB_E_CAPTURE) rather than baking in a buffer
    that growth would free."""
    import torch
    import paper_2208_01239_amd as fi
    hd = fi.Handle(0)
    try:
        mats = [inputs.general(n, 60 + n) if n % 2 else inputs.hpd(n, 60 + n) for n in (21, 48, 77)]
        kinds = [0 if n % 2 else 1 for n in (21, 48, 77)]
        plan = fi.BatchedPlan([torch.from_numpy(A).cuda() for A, _ in mats],
                              [torch.from_numpy(B).cuda() for _, B in mats], kinds)
        g0 = torch.cuda.CUDAGraph()
        with pytest.raises(fi.FrobError) as ei:
            with torch.cuda.graph(g0):
                plan.launch(hd)          # fresh handle: the workspace would have to grow inside the capture
        assert ei.value.status == fi._lib.FROB_E_CAPTURE
        del g0
        torch.cuda.synchronize()
        plan.launch(hd)
        torch.cuda.synchronize()
        ref = [(x.clone(), y.clone()) for x, y in zip(plan.Xr, plan.Xi)]
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            plan.launch(hd)
        before = hd.workspace_bytes()
        A, B = inputs.general(1500, 8)
        fi.frob_inv_general(hd, torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda())
        assert hd.workspace_bytes() > before
        for rep in range(2):
            for x, y in zip(plan.Xr, plan.Xi):
                x.fill_(float("nan")); y.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            for (x, y), (rx, ry) in zip(zip(plan.Xr, plan.Xi), ref):
                assert torch.equal(x, rx) and torch.equal(y, ry), rep
        del g
        torch.cuda.synchronize()
    finally:
        hd.close()


def test_batched_autotune(h):
    import torch
    import paper_2208_01239_amd as fi
    table = fi.frob_batched_tune(h, fi.FROB_PREC_F64)
    assert set(table.values()) <= {8, 16, 32} and len(table) == 8
    A, B = inputs.general(150, 9)
    r = oracle.cinv_lu(A, B)
    Xr, Xi, info = _run(h, [(A, B)], [0], torch.float64)
    assert info[0] == 0 and relF(Xr[0], Xi[0], r[0], r[1]) <= 1e-10


def test_batched_full_size_sampled(h):
    """The 2048-matrix workload (orders uniform in [16, 512], half general, half
    HPD, seed 4) in the launch configuration bench.py times; eight seeded
    members checked against the oracle."""
    import torch
    import paper_2208_01239_amd as fi
    ns, kinds, mats = inputs.batch(count=2048, seed=4)
    As = [torch.from_numpy(A).cuda() for A, _ in mats]
    Bs = [torch.from_numpy(B).cuda() for _, B in mats]
    plan = fi.BatchedPlan(As, Bs, kinds)
    plan.launch(h)
    torch.cuda.synchronize()
    assert int((plan.info_dev != 0).sum()) == 0
    pick = np.random.default_rng(2208).choice(len(mats), size=8, replace=False)
    for i in pick:
        A, B = mats[i]
        r = oracle.cinv_lu(A, B) if kinds[i] == 0 else oracle.cinv_chol(A, B)
        kC = np.linalg.cond(A + B @ np.linalg.solve(A, B))
        e = relF(plan.Xr[i].cpu().numpy(), plan.Xi[i].cpu().numpy(), r[0], r[1])
        assert e <= max(1e-10, 16 * U64 * kC), (i, ns[i], kinds[i], e)
