"""The batched kernel's workgroup code run on the CPU under a barrier-checking
emulation (tests/emu/batched_emu.cpp): every thread is a fiber, and a
workgroup barrier is released only when all threads of the workgroup wait at
the same call site with the same barrier count.

These tests show on the CPU that members whose factorizations fail (a singular
real part, an indefinite "HPD" member, C singular, C indefinite) run the same
barrier sequence as good members and leave the persistent loop, that their
status words equal the oracle's, and that a block width of zero -- what an
out-of-range read of the panel-width table can return -- makes the
factorization loop stop advancing (the cause of the batched hangs, which sent a
kind outside {0, 1}).  Numerics of good members are compared with the oracle
(Algorithms 4 and 8)."""
import ctypes
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2208_01239_amd import inputs
from _helpers import relF

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "emu"))

ERR = {0: "ok", 1: "divergent barrier", 2: "deadlock", 3: "watchdog", 4: "exited at barrier", 5: "wave divergence"}
LIMIT = 50_000_000
U64, U32 = 2.0 ** -53, 2.0 ** -24


@pytest.fixture(scope="module")
def emu():
    import build as emu_build
    lib = ctypes.CDLL(emu_build.build())
    vp, ip, i = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.c_int
    lib.emu_batched_run.argtypes = [i, i, i, ip, ip, vp, vp, vp, vp, ip, i, ip, ctypes.c_longlong,
                                    ctypes.POINTER(ctypes.c_longlong)]
    lib.emu_batched_run.restype = i
    lib.emu_potrf.argtypes = [i, ctypes.POINTER(ctypes.c_double), i, ctypes.c_longlong, ip]
    lib.emu_potrf.restype = i
    return lib


def run(lib, mats, kinds, dtype=np.float64, grid=2, nb=16, nmax=None):
    """Run the emulated persistent kernel; returns (err, Xr list, Xi list, info, barriers per block)."""
    count = len(mats)
    ns = np.array([A.shape[0] for A, _ in mats], dtype=np.int32)
    kd = np.array(kinds, dtype=np.int32)
    As = [np.ascontiguousarray(A, dtype=dtype) for A, _ in mats]
    Bs = [np.ascontiguousarray(B, dtype=dtype) for _, B in mats]
    Xr = [np.full_like(A, np.nan) for A in As]
    Xi = [np.full_like(A, np.nan) for A in As]

    def ptrs(arrs):
        return (ctypes.c_void_p * count)(*[a.ctypes.data for a in arrs])

    info = np.full(count, -7, dtype=np.int32)
    table = (ctypes.c_int * 8)(*([nb] * 8))
    bars = (ctypes.c_longlong * grid)()
    ip = ctypes.POINTER(ctypes.c_int)
    err = lib.emu_batched_run(1 if dtype == np.float32 else 0, count, int(nmax or max(max(ns), 1)),
                              ns.ctypes.data_as(ip), kd.ctypes.data_as(ip), ptrs(As), ptrs(Bs), ptrs(Xr), ptrs(Xi),
                              info.ctypes.data_as(ip), grid, table, LIMIT, bars)
    return err, Xr, Xi, info, list(bars)


J = np.array([[0.0, 1.0], [-1.0, 0.0]])
FAILING = [
    # (A, B, kind, expected status word): oracle Algorithm 5 / 7 info codes
    ((np.diag([0.0, 1.0, 0.0]), np.diag([0.0, 0.0, 1.0])), 0),   # diag(0, 1, i): A singular at column 1
    ((-np.eye(4), np.zeros((4, 4))), 1),                       # -I: A not positive definite
    ((np.eye(2), J.copy()), 0),                                # C = I + J^2 = 0: M singular (Lemma 2.3)
    ((np.eye(2), 2.0 * J), 1),                                 # C = I - 4 I: M indefinite (Lemma 4.5)
]


def oracle_info(A, B, kind):
    return oracle.frob_lu(A, B)[2] if kind == 0 else oracle.frob_chol(A, B)[2]


def test_failing_members_keep_barriers_uniform_and_match_oracle_status(emu):
    good_g = inputs.general(40, 5)
    good_h = inputs.hpd(30, 6)
    mats = [good_g] + [m for m, _ in FAILING] + [good_h, good_g]
    kinds = [0] + [k for _, k in FAILING] + [1, 0]
    err, Xr, Xi, info, bars = run(emu, mats, kinds, grid=2)
    assert err == 0, ERR[err]
    expected = [0] + [oracle_info(*m, k) for m, k in FAILING] + [0, 0]
    assert list(info) == expected, (list(info), expected)
    assert expected[1:5] == [1000001, 1000001, 2000001, 2000001]
    for i in (0, 5, 6):
        A, B = mats[i]
        r = oracle.cinv_lu(A, B) if kinds[i] == 0 else oracle.cinv_chol(A, B)
        assert relF(Xr[i], Xi[i], r[0], r[1]) <= 1e-12, i
    assert all(b > 0 for b in bars)


def test_invalid_kind_and_order_are_reported_not_indexed(emu):
    """A kind outside {0, 1} or an order above nmax gets status -1 and is never
    used to index the panel-width table; the batch still completes."""
    good = inputs.general(12, 3)
    big = inputs.general(20, 4)
    mats = [good, good, big, good]
    kinds = [0, 7, 0, -1]
    err, Xr, Xi, info, _ = run(emu, mats, kinds, grid=1, nmax=16)
    assert err == 0, ERR[err]
    assert list(info) == [0, -1, -1, -1]
    r = oracle.cinv_lu(*good)
    assert relF(Xr[0], Xi[0], r[0], r[1]) <= 1e-12


def test_zero_block_width_never_advances(emu):
    """The in-workgroup Cholesky with block width 0 -- a value an out-of-range
    read of the panel-width table could return -- repeats its first block
    forever (caught by the barrier watchdog); widths 1 and 16 finish.  The
    kernel now clamps the width to [1, 32] after validating the kind."""
    A = inputs.hpd(6, 1)[0]
    for nb, expect in ((0, 3), (1, 0), (16, 0)):
        a = np.ascontiguousarray(A.copy())
        ret = ctypes.c_int(-5)
        err = emu.emu_potrf(6, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nb, 200_000, ctypes.byref(ret))
        assert err == expect, (nb, ERR[err])
        if expect == 0:
            assert ret.value == 0
            L = np.tril(a)
            assert np.allclose(L @ L.T, A, rtol=0, atol=1e-12 * np.abs(A).max())


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_emulated_batch_matches_oracle(emu, dtype):
    """Uneven orders (several panels, ragged tails), general and HPD mixed,
    three emulated workgroups sharing the queue, panel widths 8 and 32."""
    sizes = [1, 2, 5, 17, 33, 48, 65]
    mats, kinds = [], []
    for i, n in enumerate(sizes):
        mats.append(inputs.general(n, 100 + i)); kinds.append(0)
        mats.append(inputs.hpd(n, 200 + i)); kinds.append(1)
    for nb in (8, 32):
        err, Xr, Xi, info, bars = run(emu, mats, kinds, dtype=dtype, grid=3, nb=nb)
        assert err == 0, ERR[err]
        assert np.all(info == 0)
        for i, (A, B) in enumerate(mats):
            r = oracle.cinv_lu(A, B) if kinds[i] == 0 else oracle.cinv_chol(A, B)
            kC = np.linalg.cond(A + B @ np.linalg.solve(A, B))
            tol = max(1e-10, 16 * U64 * kC) if dtype == np.float64 else 16 * U32 * max(kC, 1.0)
            e = relF(Xr[i], Xi[i], r[0], r[1])
            assert e <= tol, (A.shape[0], kinds[i], nb, e)


def test_emulated_tall_panels_match_oracle(emu):
    """Orders above the workgroup size: every thread holds two rows of each LU
    panel (one of them padding for the ragged last rows), and panels of the
    default width 16 end in a ragged 12-column panel."""
    mats = [inputs.general(300, 7), inputs.hpd(300, 8), inputs.general(257, 9)]
    kinds = [0, 1, 0]
    err, Xr, Xi, info, bars = run(emu, mats, kinds, dtype=np.float64, grid=2, nb=16)
    assert err == 0, ERR[err]
    assert np.all(info == 0)
    for i, (A, B) in enumerate(mats):
        r = oracle.cinv_lu(A, B) if kinds[i] == 0 else oracle.cinv_chol(A, B)
        kC = np.linalg.cond(A + B @ np.linalg.solve(A, B))
        assert relF(Xr[i], Xi[i], r[0], r[1]) <= max(1e-10, 16 * U64 * kC), i


def test_checker_catches_known_defects(emu):
    """The emulation is not vacuous: a skipped barrier, a half-wave lane
    exchange and a wave that leaves before a barrier are each reported."""
    emu.emu_selftest.argtypes = [ctypes.c_int]
    assert emu.emu_selftest(0) == 0
    assert emu.emu_selftest(1) == 1      # divergent barrier
    assert emu.emu_selftest(2) == 5      # wave divergence
    assert emu.emu_selftest(3) == 4      # exited threads at a barrier
