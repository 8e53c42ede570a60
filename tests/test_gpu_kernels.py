"""Kernel-level parity on the GPU, through the C-ABI: the permute against numpy (bit-exact)
and the complex GEMM against numpy complex128 for each precision."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1905_00444_amd import Context
    assert torch.cuda.is_available()
    return Context(0)


def _say(msg):
    print(msg, flush=True)


def _rand_c64(rng, shape):
    return (rng.normal(size=shape) + 1j * rng.normal(size=shape)).astype(np.complex64)


@pytest.mark.parametrize("b", [0, 1, 3, 6, 10, 13, 17, 21])
def test_permute_matches_numpy_transpose(ctx, b):
    import torch
    from paper_1905_00444_amd import permute
    _say(f"permute transpose b={b}")
    rng = np.random.default_rng(b)
    src = _rand_c64(rng, 2 ** b)
    axes = rng.permutation(b)
    # numpy: view as (2,)*b with axis 0 = most significant bit; out = transpose(axes)
    ref = np.transpose(src.reshape((2,) * b), axes).reshape(-1) if b else src.copy()
    # destination bit i (LSB=0) is output axis b-1-i, which is source axis axes[b-1-i],
    # i.e. source bit b-1-axes[b-1-i]
    perm = [b - 1 - int(axes[b - 1 - i]) for i in range(b)]
    s = torch.from_numpy(src).cuda()
    d = torch.empty_like(s)
    permute(ctx, s, d, perm)
    torch.cuda.synchronize()
    assert np.array_equal(d.cpu().numpy(), ref)


@pytest.mark.parametrize("b,extra", [(5, 3), (12, 4), (18, 2)])
def test_permute_gather_with_fixed_bits(ctx, b, extra):
    """Destination takes b of the source's b+extra bits; the rest are fixed via the base."""
    import torch
    from paper_1905_00444_amd import permute
    _say(f"permute gather b={b} extra={extra}")
    rng = np.random.default_rng(100 + b)
    tot = b + extra
    src = _rand_c64(rng, 2 ** tot)
    positions = rng.permutation(tot)
    perm = [int(x) for x in positions[:b]]
    fixed = [int(x) for x in positions[b:]]
    vals = rng.integers(0, 2, size=extra)
    base = int(sum(int(v) << p for v, p in zip(vals, fixed)))
    j = np.arange(2 ** b, dtype=np.int64)
    idx = np.full(2 ** b, base, dtype=np.int64)
    for i, p in enumerate(perm):
        idx |= ((j >> i) & 1) << p
    ref = src[idx] * np.float32(0.5)
    s = torch.from_numpy(src).cuda()
    d = torch.empty(2 ** b, dtype=torch.complex64, device="cuda")
    permute(ctx, s, d, perm, base=base, scale=0.5)
    torch.cuda.synchronize()
    assert np.array_equal(d.cpu().numpy(), ref)


SHAPES = [(1, 1, 1), (3, 5, 7), (16, 8, 4), (32, 32, 32), (64, 32, 64), (128, 64, 32), (256, 128, 512), (256, 128, 16),
          (1024, 64, 256), (512, 512, 2048), (2048, 1024, 128), (1, 1, 65536), (4, 8, 4096), (3, 2, 1000)]
TOL = {"fp32": 2e-6, "bf16x3": 3e-5, "fp16": 3e-3}


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16"])
@pytest.mark.parametrize("M,N,K", SHAPES)
def test_cgemm_matches_numpy(ctx, precision, M, N, K):
    import torch
    from paper_1905_00444_amd import cgemm
    _say(f"cgemm {precision} {M}x{N}x{K}")
    rng = np.random.default_rng(M * 7 + N * 3 + K)
    A = _rand_c64(rng, (M, K))
    B = _rand_c64(rng, (N, K))
    ref = A.astype(np.complex128) @ B.astype(np.complex128).T
    bound = np.abs(A).astype(np.float64) @ np.abs(B).astype(np.float64).T
    C = cgemm(ctx, torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), precision)
    torch.cuda.synchronize()
    got = C.cpu().numpy().astype(np.complex128)
    err = np.max(np.abs(got - ref) / bound)
    assert err <= TOL[precision], err


def test_cgemm_batched(ctx):
    import torch
    from paper_1905_00444_amd import _lib
    import ctypes as Cc
    _say("cgemm batched")
    rng = np.random.default_rng(5)
    Bt, M, N, K = 3, 128, 64, 64
    A = _rand_c64(rng, (Bt, M, K))
    B = _rand_c64(rng, (Bt, N, K))
    ref = np.einsum("bmk,bnk->bmn", A.astype(np.complex128), B.astype(np.complex128))
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    dC = torch.empty((Bt, M, N), dtype=torch.complex64, device="cuda")
    st = ctx.lib.qf_cgemm(ctx.h, 0, M, N, K, Cc.c_void_p(dA.data_ptr()), Cc.c_void_p(dB.data_ptr()),
                          Cc.c_void_p(dC.data_ptr()), Bt, M * K, N * K, M * N)
    _lib.check(st, ctx.h)
    torch.cuda.synchronize()
    assert np.allclose(dC.cpu().numpy(), ref, atol=1e-4)


def test_cgemm_rejects_bad_arguments(ctx):
    import ctypes as Cc
    from paper_1905_00444_amd import _lib
    st = ctx.lib.qf_cgemm(ctx.h, 0, 0, 4, 4, Cc.c_void_p(256), Cc.c_void_p(256), Cc.c_void_p(256), 1, 0, 0, 0)
    assert st == _lib.QF_ERR_ARG
    st = ctx.lib.qf_cgemm(ctx.h, 7, 4, 4, 4, Cc.c_void_p(256), Cc.c_void_p(256), Cc.c_void_p(256), 1, 0, 0, 0)
    assert st == _lib.QF_ERR_ARG
