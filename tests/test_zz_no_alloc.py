"""lsop_apply_noalloc (the LS operator of Section 2.2 with its FFT intermediate in the library's fixed device
array) against lsop_apply on the same inputs, through the C ABI: two calls in a row, the second on a smaller
grid with fewer vectors; the library makes no device allocation in either call, and a grid whose intermediate
exceeds the array is refused."""
import numpy as np
import pytest
import torch

from gpu_helpers import announce, dev, host, require_gpu
from paper_2005_01372_amd import lsop, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _op(n, dtype, seed):
    w = synth.model_random_ellipses(n=n, nsrc=1, seed=seed)
    op = lsop.Operator(n, n, dtype, max_vec=16)
    op.set_problem(torch.as_tensor(w.vel).cuda(), w.h, w.freq, w.c0)
    return op


@pytest.mark.parametrize("dtype", [lsop.C64, lsop.C128])
def test_noalloc_apply_matches_lsop_apply(dtype):
    tdt = torch.complex64 if dtype == lsop.C64 else torch.complex128
    # 1024^2: 4 (complex float) or 2 (complex double) vectors per chunk of the 64 MiB array, 9 vectors (ragged
    # last chunk); then 96 x 96 with 3 vectors in one chunk
    for n, nv, mode in ((1024, 9, "A"), (96, 3, "VHG0H")):
        announce(f"noalloc apply {n}^2 x {nv} dtype={dtype} mode={mode}")
        op = _op(n, dtype, 3 + n)
        x = dev(synth.random_vectors((nv, n, n), n), tdt)
        ref = op.apply(x, mode)
        out = torch.full_like(x, float("nan"))
        torch.cuda.synchronize()
        before = lsop.alloc_count()
        op.apply_noalloc(x, mode, out=out)
        torch.cuda.synchronize()
        assert lsop.alloc_count() == before
        assert torch.equal(out, ref)
        del op


def test_noalloc_apply_rejects_oversized_intermediate():
    announce("noalloc apply oversized")
    op = lsop.Operator(2048, 2048, lsop.C128, max_vec=1)   # 2048 x 4096 complex doubles = 128 MiB per vector
    w = synth.model_random_ellipses(n=2048, nsrc=1, seed=1)
    op.set_problem(torch.as_tensor(w.vel).cuda(), w.h, w.freq, w.c0)
    x = torch.zeros((1, 2048, 2048), dtype=torch.complex128, device="cuda")
    out = torch.zeros_like(x)
    with pytest.raises(lsop.LsopError) as e:
        op.apply_noalloc(x, "A", out=out)
    assert e.value.status == lsop.EINVAL
    assert torch.count_nonzero(out) == 0
