"""GPU tests of the kernel-level entry points against FP64 NumPy references.

complex64 GEMM on FP32 MFMA: rel-L2 <= 1e-5.
Split products: a value is x = hi + lo + d with |d| <= 2^-16 |x| (bf16, 8-bit
significands) or 2^-22 |x| (fp16, 11-bit, inside the scaled range); dropping
lo*lo' adds the same order, so a K-term product has rel-L2 of order 2^-16
(bf16x3) or 2^-21 (fp16x3).  Bars: 1e-4 and 5e-6.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rqc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_15083_amd import rqc as lib
    return lib


def to_dev(z):
    import torch
    z = np.ascontiguousarray(z, dtype=np.complex64)
    return torch.from_numpy(z.view(np.float32).copy()).cuda()


def from_dev(t, shape):
    return t.cpu().numpy().view(np.complex64).reshape(shape).astype(np.complex128)


def rand_c(rng, shape, spread=0):
    z = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    if spread:
        z = z * np.exp2(-rng.uniform(0, spread, size=shape))
    return z


def run_gemm(rqc, A, B, batch, M, N, K, ak, bn, prec):
    import torch
    # A logical [b][m][k]; stored per layout flag
    Ad = A if ak else A.transpose(0, 2, 1)
    Bd = B if bn else B.transpose(0, 2, 1)
    C = torch.empty(batch * M * N * 2, dtype=torch.float32, device="cuda")
    rqc.kernel_cgemm(to_dev(Ad), to_dev(Bd), C, batch, M, N, K, ak, bn, prec)
    torch.cuda.synchronize()
    return from_dev(C, (batch, M, N))


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# every tile size with 8-deep K stages (K = 8) and with 16-deep ones
SHAPES = [(1, 64, 64, 8), (3, 64, 128, 16), (2, 128, 64, 32), (1, 256, 128, 64), (2, 128, 256, 128),
          (2, 128, 64, 8), (1, 128, 128, 8), (2, 64, 128, 8)]


@pytest.mark.parametrize("ak", [0, 1])
@pytest.mark.parametrize("bn", [0, 1])
@pytest.mark.parametrize("shape", SHAPES)
def test_cgemm_fp32_mfma(rqc, ak, bn, shape):
    batch, M, N, K = shape
    rng = np.random.default_rng(hash(shape) & 0xFFFF)
    A, B = rand_c(rng, (batch, M, K)), rand_c(rng, (batch, K, N))
    got = run_gemm(rqc, A, B, batch, M, N, K, ak, bn, rqc.C64)
    ref = np.matmul(A.astype(np.complex64).astype(np.complex128), B.astype(np.complex64).astype(np.complex128))
    assert rel(got, ref) <= 1e-5


@pytest.mark.parametrize("prec,bar", [("BF16X3", 1e-4), ("FP16X3", 5e-6)])
@pytest.mark.parametrize("ak,bn", [(1, 1), (0, 0), (1, 0), (0, 1)])
@pytest.mark.parametrize("shape", [(1, 64, 64, 16), (2, 128, 128, 64), (1, 256, 64, 256)])
def test_cgemm_split(rqc, prec, bar, ak, bn, shape):
    batch, M, N, K = shape
    rng = np.random.default_rng(7 + K)
    A, B = rand_c(rng, (batch, M, K)), rand_c(rng, (batch, K, N))
    got = run_gemm(rqc, A, B, batch, M, N, K, ak, bn, getattr(rqc, prec))
    ref = np.matmul(A.astype(np.complex64).astype(np.complex128), B.astype(np.complex64).astype(np.complex128))
    assert rel(got, ref) <= bar


@pytest.mark.parametrize("scale_exp", [-60, 0, 60])
def test_fp16_split_power_of_two_scaling(rqc, scale_exp):
    """Operands with a 2^-40..2^0 exponent spread, shifted far outside fp16's
    range: the per-operand 2^e scale keeps the rel-L2 at the fp16x3 level."""
    batch, M, N, K = 1, 128, 128, 64
    rng = np.random.default_rng(3)
    A = rand_c(rng, (batch, M, K), spread=40) * 2.0 ** scale_exp
    B = rand_c(rng, (batch, K, N), spread=40) * 2.0 ** (scale_exp // 2)
    got = run_gemm(rqc, A, B, batch, M, N, K, 1, 1, rqc.FP16X3)
    ref = np.matmul(A.astype(np.complex64).astype(np.complex128), B.astype(np.complex64).astype(np.complex128))
    assert rel(got, ref) <= 5e-6


def test_split_falls_back_below_k16(rqc):
    rng = np.random.default_rng(11)
    A, B = rand_c(rng, (1, 64, 8)), rand_c(rng, (1, 8, 64))
    got = run_gemm(rqc, A, B, 1, 64, 64, 8, 1, 1, rqc.BF16X3)
    ref = np.matmul(A.astype(np.complex64).astype(np.complex128), B.astype(np.complex64).astype(np.complex128))
    assert rel(got, ref) <= 1e-5


def test_cgemm_rejects_bad_shapes(rqc):
    import torch
    x = torch.empty(64 * 64 * 2, dtype=torch.float32, device="cuda")
    with pytest.raises(rqc.RqcError):
        rqc.kernel_cgemm(x, x, x, 1, 32, 64, 8)
    with pytest.raises(rqc.RqcError):
        rqc.kernel_cgemm(x, x, x, 1, 64, 64, 12)


@pytest.mark.parametrize("r,seed", [(1, 0), (3, 1), (5, 2), (6, 3), (10, 4), (17, 5), (22, 6)])
def test_permute_matches_numpy(rqc, r, seed):
    import torch
    rng = np.random.default_rng(seed)
    perm = rng.permutation(r).tolist()
    src = rand_c(rng, (1 << r,)).astype(np.complex64)
    dst = torch.empty((1 << r) * 2, dtype=torch.float32, device="cuda")
    rqc.kernel_permute(to_dev(src), dst, perm)
    torch.cuda.synchronize()
    x = np.arange(1 << r)
    pi = np.zeros_like(x)
    for i, p in enumerate(perm):
        pi |= ((x >> i) & 1) << p
    exp = np.empty_like(src)
    exp[pi] = src
    got = dst.cpu().numpy().view(np.complex64)
    assert np.array_equal(got, exp)


def test_permute_rejects_non_permutation(rqc):
    import torch
    x = torch.empty(16, dtype=torch.float32, device="cuda")
    with pytest.raises(rqc.RqcError):
        rqc.kernel_permute(x, x, [0, 0, 1])
