"""Small products, whose launches dominate their time: up to 2^12 points the
two forward transforms interleave level by level and their FFT passes of one
level share a launch, and when the inverse transform is one tile with its
BasisCvt inside and one pointmul tile (up to 2^10 points) pointmul, the
inverse pass, changeRepr back and InterleavedCombine run as one launch
(k_tail): two launches per product.  Every product against the oracle, with the launches the library's
trace records, at ragged and unbalanced sizes on both sides of those bounds."""
import sys

import numpy as np
import pytest

import oracle
import paper_1708_09746_amd as P
from helpers import dev, host
from paper_1708_09746_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


# (na, nb): 2 .. 2^10 points (two launches), 2^11 (paired forward passes, the
# last steps op by op), 2^12 (BasisCvt in passes of its own), 2^13 (two
# streams)
SIZES = [(1, 1), (1, 64), (64, 64), (65, 64), (127, 129), (1000, 999), (64 * 31, 64 * 33), (5000, 70), (70, 5000),
         (4095, 4097), (1 << 16, 1 << 16), (1 << 16, (1 << 16) - 3), (100000, 3), (3, 100000), (64 * 1023, 64 * 1025),
         (1 << 17, 1 << 17), (200000, 61000), (64 * 2047 + 5, 64 * 2049 + 11)]


@pytest.mark.parametrize("na,nb", SIZES)
def test_small_products(ctx, na, nb):
    a = inputs.random_poly(0x5A1 + na % 101, na)
    b = inputs.random_poly(0x5A2 + nb % 103, nb)
    m = P.fft_log2(na, nb)
    say(f"case small product {na}x{nb} (2^{m} points)")
    c = torch.full((P.out_words(na, nb),), -1, dtype=torch.int64, device="cuda")
    ctx.trace_begin(0x3FF)
    ctx.mul_into(dev(a), na, dev(b), nb, c)
    recs = ctx.trace_end()
    assert np.array_equal(host(c), oracle.mul(a, na, b, nb, threads=8)), (na, nb)
    kernels = [r["kernel"] for r in recs]
    if m <= 10:
        # the forward passes share a launch when their tiles fit one round of
        # the grid (an operand far shorter than the other has many cosets)
        assert kernels[-1] == "k_tail" and recs[-1]["elements"] == 1 << m, kernels
        assert kernels[:-1] in (["k_fft"], ["k_fft", "k_fft"]), kernels
        if max(na, nb) <= 2 * min(na, nb):
            assert len(kernels) == 2, kernels
    elif m <= 12:
        assert "k_tail" not in kernels, kernels
        if na == nb:
            # same plans for both operands: one launch for both forward
            # passes, one for the inverse pass
            assert kernels.count("k_fft") == 2, kernels
        if m == 11 and max(na, nb) <= 2 * min(na, nb):
            assert kernels == ["k_fft", "k_pmul", "k_fft", "k_psi"], kernels
    else:
        assert "k_tail" not in kernels, kernels


def test_small_products_repeat_and_squares(ctx):
    """The same buffers reused call after call, and squares with aliased
    operands, stay exact."""
    for na in [1, 64, 777, 1 << 15, 100000]:
        a = inputs.random_poly(0x5A3 + na, na)
        da = dev(a)
        want = oracle.mul(a, na, a, na, threads=8)
        c = torch.full((P.out_words(na, na),), -1, dtype=torch.int64, device="cuda")
        for _ in range(3):
            ctx.mul_into(da, na, da, na, c)
            assert np.array_equal(host(c), want), na
