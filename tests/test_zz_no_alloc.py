"""wcmg_coarse_apply_noalloc, the coarse apply for callers that cannot
allocate device memory, called through the C ABI: the same result as
wcmg_coarse_apply, bit for bit, on two calls in a row (the second with a
smaller input), with its scratch (the five-point scatter buffer) taken from
the library's static per-GPU array instead of an allocation; sizes beyond
that array are refused with an error."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
import synthetic as syn
from tests import brute_force as bf
from tests.test_gpu_parity import dev, host, rel, wc

pytestmark = pytest.mark.gpu


def _noalloc(w, op, x, out):
    nrhs = x.numel() // (op.Vc * op.nb)
    return w.lib().wcmg_coarse_apply_noalloc(op.h, C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()), nrhs)


def _five_point_op(w, Lc, nb, store, seed):
    Vc = int(np.prod(Lc))
    blocks = syn.complex_gaussian((Vc, 9, nb, nb), seed)
    op = w.CoarseOperator(Lc, nb, store)
    op.set_kernel(3)
    op.set(dev(blocks))
    return op, blocks


def test_noalloc_matches_the_allocating_apply_on_consecutive_calls():
    """Five-point owner-computes apply (its scatter buffer is the scratch):
    16,384 coarse sites at Nb = 24 (1 lane per row), two right-hand sides,
    then one (a smaller input into the same scratch), then a smaller operator;
    each against wcmg_coarse_apply on the same inputs (bit-identical: the same
    kernels) and against the oracle applied to the sigma3-mirrored blocks the
    five-point storage represents (FP32, 1e-5)."""
    w = wc()
    nb = 24
    op, blocks = _five_point_op(w, (8, 8, 16, 16), nb, w.F32, 1501)
    small, sblocks = _five_point_op(w, (8, 8, 8, 16), nb, w.F32, 1502)
    cases = [(op, blocks, (8, 8, 16, 16), 2), (op, blocks, (8, 8, 16, 16), 1), (small, sblocks, (8, 8, 8, 16), 2)]
    for k, (o, blk, Lc, nrhs) in enumerate(cases):
        phi = syn.complex_gaussian((nrhs, o.Vc, nb), 1510 + k)
        x = dev(phi.astype(np.complex64))
        out = torch.empty_like(x)
        torch.cuda.synchronize()
        st = _noalloc(w, o, x, out)
        assert st == 0, w.lib().wcmg_coarse_last_error(o.h)
        got = host(out)
        ref_gpu = host(o.apply(x))
        assert np.array_equal(got, ref_gpu), k
        ref = oracle.coarse_apply(Lc, bf.sigma3_mirror(Lc, blk), phi)
        assert rel(got, ref) < 1e-5, k


def test_noalloc_allocates_nothing_and_refuses_oversized_calls():
    """Device free memory is unchanged by the no-allocation calls (the
    allocating entry point grows its scatter buffer on first use: about 25 MB
    here, which the same check sees); six right-hand sides would need 75.5 MB
    of scratch and are refused (WCMG_ERR_ARG) without writing the output."""
    w = wc()
    nb = 24
    op, blocks = _five_point_op(w, (8, 8, 16, 16), nb, w.F32, 1521)
    x = dev(syn.complex_gaussian((2, op.Vc, nb), 1522).astype(np.complex64))
    out = torch.empty_like(x)
    assert _noalloc(w, op, x, out) == 0  # first call on this device looks up the scratch address
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        assert _noalloc(w, op, x, out) == 0
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert abs(free0 - free1) < (2 << 20), (free0, free1)
    op2, _ = _five_point_op(w, (8, 8, 16, 16), nb, w.F32, 1523)
    out2 = torch.empty_like(x)
    torch.cuda.synchronize()
    free2 = torch.cuda.mem_get_info()[0]
    op2.apply(x, out2)  # the allocating form: its first call allocates the scatter buffer
    torch.cuda.synchronize()
    assert free2 - torch.cuda.mem_get_info()[0] >= (20 << 20)
    big = dev(syn.complex_gaussian((6, op.Vc, nb), 1524).astype(np.complex64))
    big_out = torch.zeros_like(big)
    st = _noalloc(w, op, big, big_out)
    assert st == 1
    assert b"scratch" in w.lib().wcmg_coarse_last_error(op.h)
    assert torch.count_nonzero(big_out).item() == 0


@pytest.mark.parametrize("kernel,store,nrhs", [(1, "f32", 1), (2, "bf16", 12), (0, "f32", 5)])
def test_noalloc_other_kernels_need_no_scratch(kernel, store, nrhs):
    """Per-row and matrix-core kernels: the no-allocation entry point gives
    the allocating entry point's result bit for bit."""
    w = wc()
    nb, Lc = 24, (4, 4, 4, 8)
    Vc = int(np.prod(Lc))
    op = w.CoarseOperator(Lc, nb, w.F32 if store == "f32" else w.BF16)
    op.set_kernel(kernel)
    op.set(dev(syn.complex_gaussian((Vc, 9, nb, nb), 1531)))
    x = dev(syn.complex_gaussian((nrhs, Vc, nb), 1532).astype(np.complex64))
    out = torch.empty_like(x)
    assert _noalloc(w, op, x, out) == 0
    assert np.array_equal(host(out), host(op.apply(x)))
