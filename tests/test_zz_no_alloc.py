"""The cycle entry point that allocates nothing (pod2g_apply_noalloc)
against pod2g_apply with a caller workspace: the same kernels, so the same
bits; two calls in a row on the shared scratch array, the second smaller,
and a too large call refused before any launch."""
import ctypes as C

import numpy as np
import pytest

from gpu_helpers import flush
from oracle import problem as oprob
from paper_2207_02543_amd import inputs as I

pytestmark = pytest.mark.gpu


def _prec(dim, N, batch, mixed):
    import torch
    from paper_2207_02543_amd import capi, pipeline
    w = I.small(dim, N, k=6, n_train=12)
    P, lam, U = oprob.basis(w, I.train_xis(w))
    prob = pipeline.Problem(w)
    sysm = prob.alloc_system(batch, fp32=mixed)
    prob.assemble(sysm, I.query_xis(w, batch))
    pr = prob.setup(sysm, torch.tensor(np.ascontiguousarray(P.T), device="cuda"),
                    precision=capi.MIXED if mixed else capi.FP64)
    return w, prob, pr


def test_apply_noalloc_matches_apply():
    import torch
    from paper_2207_02543_amd import capi
    # the second call is smaller than the first: the scratch array keeps the
    # first call's contents, which must not leak into the second
    for dim, N, batch, mixed in [(2, 40, 6, True), (3, 5, 2, False), (2, 12, 1, True)]:
        flush(f"no-alloc cycle dim={dim} N={N} batch={batch} {'mixed' if mixed else 'fp64'}")
        w, prob, pr = _prec(dim, N, batch, mixed)
        assert capi.pod2g_apply_bytes(pr) <= capi.NOALLOC_SCRATCH_BYTES
        r = torch.tensor(np.random.default_rng(dim * N + batch).standard_normal((batch, w.n)),
                         device="cuda")
        s_ref = torch.empty_like(r)
        prob.apply(pr, r, s_ref)
        for call in range(2):
            s = torch.full_like(r, float("nan"))
            capi.check(capi.pod2g_apply_noalloc(pr, r, s), "pod2g_apply_noalloc")
            torch.cuda.synchronize()
            assert torch.equal(s, s_ref), call


def test_apply_noalloc_refuses_too_large():
    from paper_2207_02543_amd import capi
    w, prob, pr = _prec(2, 12, 1, False)
    big = capi.Prec()
    C.pointer(big)[0] = pr
    big.batch = 4096          # 8 FP64 vectors of 4096 x 312 unknowns: beyond the array
    assert capi.pod2g_apply_bytes(big) > capi.NOALLOC_SCRATCH_BYTES
    assert capi.pod2g_apply_noalloc(big, 1, 1) == capi.ESIZE
