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


@pytest.mark.parametrize("b", [1, 9, 16])
def test_permute_on_8_byte_aligned_buffers(ctx, b):
    """A source or destination offset by one complex64 (8-byte, not 16-byte, aligned): the
    result still equals numpy's transpose."""
    import torch
    from paper_1905_00444_amd import permute
    _say(f"permute 8-byte aligned b={b}")
    rng = np.random.default_rng(200 + b)
    x = _rand_c64(rng, 2 ** b)
    axes = rng.permutation(b)
    ref = np.transpose(x.reshape((2,) * b), axes).reshape(-1)
    perm = [b - 1 - int(axes[b - 1 - i]) for i in range(b)]
    big_s = torch.zeros(2 ** b + 1, dtype=torch.complex64, device="cuda")
    big_d = torch.zeros(2 ** b + 1, dtype=torch.complex64, device="cuda")
    big_s[1:] = torch.from_numpy(x).cuda()
    for s, d in ((big_s[1:], big_d[1:]), (big_s[1:], big_d[:-1]), (big_s[:-1], big_d[1:])):
        if s.data_ptr() != big_s[1:].data_ptr():
            s.copy_(torch.from_numpy(x).cuda())
        permute(ctx, s, d, perm)
        torch.cuda.synchronize()
        assert np.array_equal(d.cpu().numpy(), ref)


SHAPES = [(1, 1, 1), (3, 5, 7), (16, 8, 4), (32, 32, 32), (64, 32, 64), (128, 64, 32), (256, 128, 512), (256, 128, 16),
          (1024, 64, 256), (512, 512, 2048), (2048, 1024, 128), (1, 1, 65536), (4, 8, 4096), (3, 2, 1000),
          (32768, 64, 8), (4096, 8, 16), (65536, 4, 4), (8192, 16, 64)]
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


SPLIT_SHAPES = [(128, 64, 65536), (64, 32, 131072), (32, 32, 16384), (512, 512, 16384), (256, 128, 32768)]


@pytest.fixture(scope="module")
def split_ctx():
    """A context whose workspace holds split-K partials (qf_cgemm then splits long-K launches
    that have few output tiles)."""
    from paper_1905_00444_amd import Context
    c = Context(0)
    c.ensure_workspace(256 << 20)
    return c


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16"])
@pytest.mark.parametrize("M,N,K", SPLIT_SHAPES)
def test_cgemm_split_k_matches_numpy_and_is_deterministic(split_ctx, precision, M, N, K):
    import torch
    from paper_1905_00444_amd import cgemm
    _say(f"cgemm split-K {precision} {M}x{N}x{K}")
    rng = np.random.default_rng(M + N + K)
    A = _rand_c64(rng, (M, K))
    B = _rand_c64(rng, (N, K))
    ref = A.astype(np.complex128) @ B.astype(np.complex128).T
    bound = np.abs(A).astype(np.float64) @ np.abs(B).astype(np.float64).T
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    C1 = cgemm(split_ctx, dA, dB, precision)
    C2 = cgemm(split_ctx, dA, dB, precision)
    torch.cuda.synchronize()
    got = C1.cpu().numpy().astype(np.complex128)
    err = np.max(np.abs(got - ref) / bound)
    assert err <= TOL[precision], err
    assert np.array_equal(C1.cpu().numpy(), C2.cpu().numpy())


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


def test_split_bf16_matches_torch_rounding(ctx):
    """hi = bf16(x) and lo = bf16(x - hi), round-to-nearest-even, bit-exact vs torch's conversion."""
    import torch
    from paper_1905_00444_amd import split_bf16
    _say("split bf16")
    rng = np.random.default_rng(11)
    x = _rand_c64(rng, 2 ** 14) * np.float32(3.7)
    xt = torch.from_numpy(x).cuda()
    s = split_bf16(ctx, xt)
    torch.cuda.synchronize()
    w = s.cpu().numpy().view(np.uint32)
    n = x.size
    re = torch.from_numpy(x.real.copy()).to(torch.bfloat16)
    im = torch.from_numpy(x.imag.copy()).to(torch.bfloat16)
    hi_re = re.view(torch.int16).numpy().view(np.uint16).astype(np.uint32)
    hi_im = im.view(torch.int16).numpy().view(np.uint16).astype(np.uint32)
    assert np.array_equal(w[:n] & 0xFFFF, hi_re) and np.array_equal(w[:n] >> 16, hi_im)
    lo_re = torch.from_numpy(x.real - re.float().numpy()).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(w[n:] & 0xFFFF, lo_re.astype(np.uint32))
    # hi + lo reconstructs x to about 2^-16 relative
    def f(u):
        return (u.astype(np.uint32) << 16).view(np.float32)
    rec = f(w[:n] & 0xFFFF) + f(w[n:] & 0xFFFF)
    assert np.max(np.abs(rec - x.real) / (np.abs(x.real) + 1e-30)) <= 2.0 ** -15


@pytest.mark.parametrize("M,N,K", [(256, 128, 16), (512, 256, 64), (1024, 512, 2048), (2048, 1024, 512)])
def test_cgemm_presplit_matches_numpy(ctx, M, N, K):
    import torch
    from paper_1905_00444_amd import split_bf16, cgemm_presplit
    _say(f"cgemm presplit {M}x{N}x{K}")
    rng = np.random.default_rng(M + N + K)
    A = _rand_c64(rng, (M, K))
    B = _rand_c64(rng, (N, K))
    ref = A.astype(np.complex128) @ B.astype(np.complex128).T
    bound = np.abs(A).astype(np.float64) @ np.abs(B).astype(np.float64).T
    As = split_bf16(ctx, torch.from_numpy(A).cuda().reshape(-1))
    Bs = split_bf16(ctx, torch.from_numpy(B).cuda().reshape(-1))
    Cg = cgemm_presplit(ctx, As, Bs, M, N, K, precision="bf16x3")
    torch.cuda.synchronize()
    err = np.max(np.abs(Cg.cpu().numpy().astype(np.complex128) - ref) / bound)
    assert err <= TOL["bf16x3"], err


TALL_SHAPES = [(64, 8, 16), (4096, 8, 16), (65536, 32, 32), (1 << 20, 32, 32), (8192, 64, 64), (16384, 16, 64),
               (4096, 64, 16), (2048, 8, 64), (1 << 16, 64, 32), (4096, 64, 8), (2048, 8, 8), (1 << 16, 32, 8)]


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16"])
@pytest.mark.parametrize("M,N,K", TALL_SHAPES)
def test_cgemm_tall_matches_numpy(ctx, precision, M, N, K):
    """The tall-skinny kernel (B in LDS, A streamed into registers), forced by name."""
    import torch
    from paper_1905_00444_amd import cgemm
    _say(f"cgemm tall {precision} {M}x{N}x{K}")
    rng = np.random.default_rng(M + 3 * N + 7 * K)
    A = _rand_c64(rng, (M, K))
    B = _rand_c64(rng, (N, K))
    ref = A.astype(np.complex128) @ B.astype(np.complex128).T
    bound = np.abs(A).astype(np.float64) @ np.abs(B).astype(np.float64).T
    C = cgemm(ctx, torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), precision, variant="tall")
    torch.cuda.synchronize()
    err = np.max(np.abs(C.cpu().numpy().astype(np.complex128) - ref) / bound)
    assert err <= TOL[precision], err


def test_cgemm_tall_batched_and_rejects_other_shapes(ctx):
    import torch
    import ctypes as Cc
    from paper_1905_00444_amd import _lib, cgemm
    _say("cgemm tall batched")
    rng = np.random.default_rng(9)
    Bt, M, N, K = 3, 4096, 32, 32
    A = _rand_c64(rng, (Bt, M, K))
    B = _rand_c64(rng, (Bt, N, K))
    ref = np.einsum("bmk,bnk->bmn", A.astype(np.complex128), B.astype(np.complex128))
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    dC = torch.empty((Bt, M, N), dtype=torch.complex64, device="cuda")
    st = ctx.lib.qf_cgemm_variant(ctx.h, 1, _lib.GEMM_VARIANTS.index("tall"), M, N, K, Cc.c_void_p(dA.data_ptr()),
                                  Cc.c_void_p(dB.data_ptr()), Cc.c_void_p(dC.data_ptr()), Bt, M * K, N * K, M * N)
    _lib.check(st, ctx.h)
    torch.cuda.synchronize()
    bound = np.einsum("bmk,bnk->bmn", np.abs(A).astype(np.float64), np.abs(B).astype(np.float64))
    assert np.max(np.abs(dC.cpu().numpy() - ref) / bound) <= TOL["bf16x3"]
    # K = 4 and N = 4 are below the kernel's operand tiles (K = 8 runs half a K-step)
    with pytest.raises(RuntimeError):
        cgemm(ctx, torch.zeros((4096, 4), dtype=torch.complex64, device="cuda"),
              torch.zeros((32, 4), dtype=torch.complex64, device="cuda"), "bf16x3", variant="tall")
    with pytest.raises(RuntimeError):
        cgemm(ctx, torch.zeros((4096, 32), dtype=torch.complex64, device="cuda"),
              torch.zeros((4, 32), dtype=torch.complex64, device="cuda"), "bf16x3", variant="tall")


def _padded_planes(S, rows, K, ld):
    """Split planes (hi then lo, rows x K words each) copied into rows of ld words; the pad words
    hold a NaN pattern in both bfloat16 halves, so any read of them would poison the result."""
    import torch
    P = torch.full((2, rows, ld), 0x7FC07FC0, dtype=torch.int32, device=S.device)
    P[:, :, :K] = S.view(2, rows, K)
    return P


@pytest.mark.parametrize("M,N,K", [(512, 256, 8192), (512, 256, 32768), (256, 512, 16384)])
def test_cgemm_presplit_padded_rows_match_numpy(ctx, M, N, K):
    """The padded-row form the plan uses for K >= 2^13 (rows K + 64 words apart), on random
    operands, element-wise against numpy complex128."""
    import torch
    from paper_1905_00444_amd import split_bf16, cgemm_presplit
    _say(f"cgemm presplit padded {M}x{N}x{K}")
    rng = np.random.default_rng(M + 2 * N + K)
    A = _rand_c64(rng, (M, K))
    B = _rand_c64(rng, (N, K))
    ref = A.astype(np.complex128) @ B.astype(np.complex128).T
    bound = np.abs(A).astype(np.float64) @ np.abs(B).astype(np.float64).T
    ld = K + 64
    Ap = _padded_planes(split_bf16(ctx, torch.from_numpy(A).cuda().reshape(-1)), M, K, ld)
    Bp = _padded_planes(split_bf16(ctx, torch.from_numpy(B).cuda().reshape(-1)), N, K, ld)
    Cg = cgemm_presplit(ctx, Ap, Bp, M, N, K, lda=ld, ldb=ld)
    torch.cuda.synchronize()
    got = Cg.cpu().numpy().astype(np.complex128)
    assert np.all(np.isfinite(got))
    err = np.max(np.abs(got - ref) / bound)
    assert err <= TOL["bf16x3"], err


def test_cgemm_presplit_full_size_sampled_outputs(ctx):
    """The benchmark's largest contraction shape, 2^15 x 2^15 x 2^15 complex, in the padded-row
    layout, on seeded random normal operands: 512 sampled outputs against numpy complex128 sums
    of the same operands' rows."""
    import torch
    from paper_1905_00444_amd import split_bf16, cgemm_presplit
    M = N = K = 1 << 15
    ld = K + 64
    _say("cgemm presplit full size 2^15 cubed")
    g = torch.Generator(device="cuda")
    g.manual_seed(15)
    A = torch.randn(M * K, dtype=torch.complex64, device="cuda", generator=g)
    B = torch.randn(N * K, dtype=torch.complex64, device="cuda", generator=g)
    Ap = _padded_planes(split_bf16(ctx, A), M, K, ld)
    Bp = _padded_planes(split_bf16(ctx, B), N, K, ld)
    torch.cuda.synchronize()
    Cg = cgemm_presplit(ctx, Ap, Bp, M, N, K, lda=ld, ldb=ld)
    torch.cuda.synchronize()
    del Ap, Bp
    rng = np.random.default_rng(16)
    ms = rng.integers(0, M, 512)
    ns = rng.integers(0, N, 512)
    # every tile corner and edge of the 256 x 128 blocks is among the samples too
    ms[:4] = [0, 255, 256, M - 1]
    ns[:4] = [0, 127, 128, N - 1]
    ar = A.view(M, K)[torch.from_numpy(ms).cuda()].cpu().numpy().astype(np.complex128)
    br = B.view(N, K)[torch.from_numpy(ns).cuda()].cpu().numpy().astype(np.complex128)
    got = Cg[torch.from_numpy(ms).cuda(), torch.from_numpy(ns).cuda()].cpu().numpy().astype(np.complex128)
    ref = np.sum(ar * br, axis=1)
    bound = np.sum(np.abs(ar) * np.abs(br), axis=1)
    err = np.max(np.abs(got - ref) / bound)
    assert err <= TOL["bf16x3"], err


def test_permute_2_30_elements_sampled_bit_exact(ctx):
    """A 2^30-element (8 GiB) bit permutation, byte offsets well past 2^32: 2^16 sampled
    destination elements equal the source elements that numpy's index arithmetic names."""
    import torch
    from paper_1905_00444_amd import permute
    b = 30
    _say("permute 2^30 elements")
    g = torch.Generator(device="cuda")
    g.manual_seed(30)
    src = torch.randn(1 << b, dtype=torch.complex64, device="cuda", generator=g)
    dst = torch.empty_like(src)
    rng = np.random.default_rng(30)
    perm = [int(x) for x in rng.permutation(b)]
    permute(ctx, src, dst, perm)
    torch.cuda.synchronize()
    j = rng.integers(0, 1 << b, 1 << 16, dtype=np.int64)
    j[:2] = [0, (1 << b) - 1]
    idx = np.zeros_like(j)
    for i, p in enumerate(perm):
        idx |= ((j >> i) & 1) << p
    got = dst[torch.from_numpy(j).cuda()].cpu().numpy()
    want = src[torch.from_numpy(idx).cuda()].cpu().numpy()
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


def test_split_f16_matches_torch_rounding(ctx):
    """qf_split_f16: fp16(x * 2^s) for re and im, round-to-nearest-even, bit-exact vs torch."""
    import torch
    from paper_1905_00444_amd import split_f16
    _say("split f16")
    rng = np.random.default_rng(12)
    x = _rand_c64(rng, 2 ** 14) * np.float32(3.7)
    for s in (0, 5, -3):
        w = split_f16(ctx, torch.from_numpy(x).cuda(), s)
        torch.cuda.synchronize()
        w = w.cpu().numpy().view(np.uint32)
        f = np.float32(2.0 ** s)
        re = torch.from_numpy(x.real * f).to(torch.float16).view(torch.int16).numpy().view(np.uint16)
        im = torch.from_numpy(x.imag * f).to(torch.float16).view(torch.int16).numpy().view(np.uint16)
        assert np.array_equal(w & 0xFFFF, re.astype(np.uint32)) and np.array_equal(w >> 16, im.astype(np.uint32))


@pytest.mark.parametrize("M,N,K,pad", [(256, 128, 32, 0), (512, 256, 64, 0), (1024, 512, 2048, 0),
                                       (2048, 1024, 512, 0), (512, 256, 8192, 64), (256, 512, 32768, 64)])
def test_cgemm_presplit_f16_matches_numpy(ctx, M, N, K, pad):
    """The FP16 pre-split kernel (operands converted once by qf_split_f16; K-tiles of 32 complex
    staged as two halves), dense and with padded rows (NaN pads), against numpy complex128."""
    import torch
    from paper_1905_00444_amd import split_f16, cgemm_presplit
    _say(f"cgemm presplit fp16 {M}x{N}x{K} pad {pad}")
    rng = np.random.default_rng(M + 5 * N + K)
    A = _rand_c64(rng, (M, K))
    B = _rand_c64(rng, (N, K))
    ref = A.astype(np.complex128) @ B.astype(np.complex128).T
    bound = np.abs(A).astype(np.float64) @ np.abs(B).astype(np.float64).T
    ld = K + pad
    Af = split_f16(ctx, torch.from_numpy(A).cuda().reshape(-1))
    Bf = split_f16(ctx, torch.from_numpy(B).cuda().reshape(-1))
    if pad:
        Ap = torch.full((M, ld), 0x7E007E00, dtype=torch.int32, device="cuda")
        Bp = torch.full((N, ld), 0x7E007E00, dtype=torch.int32, device="cuda")
        Ap[:, :K] = Af.view(M, K)
        Bp[:, :K] = Bf.view(N, K)
        Af, Bf = Ap, Bp
    Cg = cgemm_presplit(ctx, Af, Bf, M, N, K, lda=ld, ldb=ld, precision="fp16")
    torch.cuda.synchronize()
    got = Cg.cpu().numpy().astype(np.complex128)
    assert np.all(np.isfinite(got))
    err = np.max(np.abs(got - ref) / bound)
    assert err <= TOL["fp16"], err


def test_cgemm_presplit_f16_rejects_short_k(ctx):
    import torch
    from paper_1905_00444_amd import cgemm_presplit
    z = torch.zeros(256 * 16, dtype=torch.int32, device="cuda")
    with pytest.raises(RuntimeError):
        cgemm_presplit(ctx, z, z[:128 * 16], 256, 128, 16, precision="fp16")


def test_ceiling_copy_and_mfma_loops(ctx):
    """qf_time_ceiling: the streaming copy leaves the second half of the buffer equal to the first
    and reports the bytes read plus written; each MFMA loop reports blocks x waves x trips x 32
    MFMAs x the instruction's flops, at a rate below the instruction's nominal peak; sizes the copy
    cannot take are rejected."""
    import torch
    from paper_1905_00444_amd import time_ceiling
    _say("ceilings: copy and MFMA loops")
    n = 1 << 20
    buf = torch.randint(0, 256, (n,), dtype=torch.uint8, device=ctx.device)
    torch.cuda.synchronize()
    ms, work = time_ceiling(ctx, "copy", size=n, buf=buf, reps=2)
    h = buf.cpu().numpy()
    assert work == n and ms > 0
    assert np.array_equal(h[: n // 2], h[n // 2:])
    for prec, per, peak in (("bf16x3", 16384, 2516.6), ("fp16", 16384, 2516.6), ("fp32", 2048, 157.3)):
        ms, fl = time_ceiling(ctx, "mfma", prec, 200, reps=2)
        assert fl == 1024 * 8 * 200 * 32 * per
        assert 0 < fl / ms / 1e9 < 1.05 * peak, prec
    with pytest.raises(Exception):
        time_ceiling(ctx, "copy", size=3 << 10, buf=buf)
