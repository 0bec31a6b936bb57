"""The no-allocation batched entry point (frob_inv_batched_noalloc): the same
results as frob_inv_batched, bit for bit (every matrix is inverted by one
workgroup running the same code), on two calls in a row -- the second with a
smaller batch -- without the handle allocating any workspace; sizes beyond the
scratch array's limits are rejected before any launch."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2208_01239_amd import inputs
from _helpers import relF

pytestmark = pytest.mark.gpu


def _plan(ns, kinds, seed, dtype):
    import torch
    import paper_2208_01239_amd as fi
    mats = [inputs.general(n, seed + i) if k == 0 else inputs.hpd(n, seed + i) for i, (n, k) in enumerate(zip(ns, kinds))]
    As = [torch.from_numpy(A).to(dtype).cuda() for A, _ in mats]
    Bs = [torch.from_numpy(B).to(dtype).cuda() for _, B in mats]
    return mats, fi.BatchedPlan(As, Bs, kinds)


@pytest.mark.parametrize("dtype_name", ["float64", "float32"])
def test_noalloc_matches_batched_twice(dtype_name):
    import torch
    import paper_2208_01239_amd as fi
    dtype = getattr(torch, dtype_name)
    h_ref = fi.Handle(0)
    h = fi.Handle(0)
    try:
        calls = [([5, 200, 64, 17, 131, 96, 1, 300], [0, 1, 1, 0, 0, 1, 0, 1], 900),
                 ([33, 12, 70], [1, 0, 0], 950)]                           # the second call is smaller
        for ns, kinds, seed in calls:
            mats, p_ref = _plan(ns, kinds, seed, dtype)
            _, p = _plan(ns, kinds, seed, dtype)
            p_ref.launch(h_ref)
            p.launch(h, noalloc=True)
            torch.cuda.synchronize()
            assert torch.equal(p.info_dev, p_ref.info_dev) and int((p.info_dev != 0).sum()) == 0
            for i in range(len(ns)):
                assert torch.equal(p.Xr[i], p_ref.Xr[i]) and torch.equal(p.Xi[i], p_ref.Xi[i]), (ns[i], kinds[i])
            A, B = mats[1]
            r = oracle.cinv_lu(A, B) if kinds[1] == 0 else oracle.cinv_chol(A, B)
            e = relF(p.Xr[1].double().cpu().numpy(), p.Xi[1].double().cpu().numpy(), r[0], r[1])
            assert e <= (1e-10 if dtype == torch.float64 else 1e-4), e
        assert h.workspace_bytes() == 0            # the handle never allocated a workspace
    finally:
        h.close()
        h_ref.close()


def test_noalloc_rejects_sizes_beyond_the_scratch():
    import torch
    import paper_2208_01239_amd as fi
    from paper_2208_01239_amd import _lib
    h = fi.Handle(0)
    try:
        _, p = _plan([8, 9], [0, 1], 3, torch.float64)
        lib = _lib.load()
        vp = ctypes.c_void_p
        args = [vp(p.n_dev.data_ptr()), vp(p.kind_dev.data_ptr()), vp(p.pA.data_ptr()), vp(p.pB.data_ptr()),
                vp(p.pXr.data_ptr()), vp(p.pXi.data_ptr()), vp(p.info_dev.data_ptr()), p.storage]
        assert lib.frob_inv_batched_noalloc(h.ptr, (1 << 20) + 1, 9, *args) == _lib.FROB_E_ARG
        assert lib.frob_inv_batched_noalloc(h.ptr, 2, 513, *args) == _lib.FROB_E_ARG
        assert lib.frob_inv_batched_noalloc(h.ptr, 2, 9, *args) == _lib.FROB_OK
        torch.cuda.synchronize()
        assert int((p.info_dev != 0).sum()) == 0
    finally:
        h.close()
