"""revo_op_attention_noalloc (the entry point for callers that cannot
allocate) against revo_op_attention on the same inputs: two calls in a row
through the C ABI, the second smaller, each bit-identical to the allocating
entry point's result.  The size limit is checked on the host."""
import math

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

FP32, BF16 = 0, 1


def _lib():
    import paper_2604_27441_amd as pkg
    return pkg.lib


def _swap23(n):
    c = np.arange(n)
    return (c & ~12) | ((c & 4) << 1) | ((c & 8) >> 1)


def _inputs(rng, heads, ntok, prec):
    ld = (ntok + 64 + 15) // 16 * 16
    dt = torch.float32 if prec == FP32 else torch.bfloat16
    q = torch.zeros((heads, ld, 64), dtype=dt)
    k = torch.zeros((heads, ld, 64), dtype=dt)
    vt = torch.zeros((heads, 64, ld), dtype=dt)
    q[:, :ntok] = torch.tensor(rng.standard_normal((heads, ntok, 64)) * 1.5 * math.log2(math.e) / 8,
                               dtype=torch.float32).to(dt)
    k[:, :ntok] = torch.tensor(rng.standard_normal((heads, ntok, 64)) * 1.5, dtype=torch.float32).to(dt)
    vt[:, :, :ntok] = torch.tensor(rng.standard_normal((heads, 64, ntok)), dtype=torch.float32).to(dt)
    if prec == BF16:
        vt = vt[:, :, _swap23(ld)].contiguous()
    return q.cuda(), k.cuda(), vt.cuda(), ld, dt


@pytest.mark.parametrize("prec", [BF16, FP32])
def test_noalloc_attention_matches_the_allocating_entry_point(prec):
    rng = np.random.default_rng(5150 + prec)
    s = torch.cuda.Stream()
    # the second call is smaller: fewer heads and fewer q-tiles than the first
    for heads, ntok in ((3, 1000), (2, 300)):
        q, k, vt, ld, dt = _inputs(rng, heads, ntok, prec)
        ref = torch.full((ntok, heads * 64), float("nan"), dtype=dt, device="cuda")
        got = torch.full((ntok, heads * 64), float("nan"), dtype=dt, device="cuda")
        torch.cuda.synchronize()
        assert _lib().revo_op_attention(prec, q.data_ptr(), k.data_ptr(), vt.data_ptr(), ref.data_ptr(),
                                        heads, ntok, ld, None) == 0
        with torch.cuda.stream(s):
            rc = _lib().revo_op_attention_noalloc(prec, q.data_ptr(), k.data_ptr(), vt.data_ptr(), got.data_ptr(),
                                                  heads, ntok, ld, s.cuda_stream)
        assert rc == 0
        s.synchronize()
        assert torch.equal(got.view(torch.int16 if prec == BF16 else torch.int32),
                           ref.view(torch.int16 if prec == BF16 else torch.int32)), (heads, ntok)


def test_noalloc_attention_rejects_sizes_beyond_its_workspace():
    # checked on the host before any launch; the pointers are never read
    dummy = torch.zeros(16, dtype=torch.bfloat16, device="cuda")
    p = dummy.data_ptr()
    big = 32767 * 128 + 1
    assert _lib().revo_op_attention_noalloc(BF16, p, p, p, p, 1, big, big + 64 + 15 & ~15, None) == -7
    assert _lib().revo_strerror(-7).decode() == "size beyond the fixed workspace"
    assert _lib().revo_op_attention_noalloc(BF16, p, p, p, p, 1, 100, 100, None) == -22
