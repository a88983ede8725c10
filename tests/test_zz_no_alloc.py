"""The no-allocation product entry point (gf2x_mul_dev_static) against the
ordinary one (gf2x_mul_dev), through the C ABI: the same words bit for bit,
on two calls in a row with the second smaller (the fixed buffer keeps the
first call's contents), at w = 64 and w = 128; products too large for the
buffer are refused with ENOMEM and nothing written."""
import ctypes
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


def _operands(seed, na, nb):
    a = inputs.random_poly(seed, na)
    b = inputs.random_poly(seed + 1, nb)
    return a, b, dev(a), dev(b)


def _both(ctx, da, na, db, nb):
    """The product by gf2x_mul_dev_static and by gf2x_mul_dev, each into an
    output filled with a sentinel first, both on the current stream."""
    L = P.lib()
    ow = P.out_words(na, nb)
    c_static = torch.full((ow,), -1, dtype=torch.int64, device="cuda")
    c_plain = torch.full((ow,), -1, dtype=torch.int64, device="cuda")
    st = P._stream_handle(None)
    rc = L.gf2x_mul_dev_static(ctx.handle, P._ptr(da), na, P._ptr(db), nb, P._ptr(c_static), st)
    assert rc == P.GF2X_OK, L.gf2x_last_error(ctx.handle).decode()
    rc = L.gf2x_mul_dev(ctx.handle, P._ptr(da), na, P._ptr(db), nb, P._ptr(c_plain), st)
    assert rc == P.GF2X_OK, L.gf2x_last_error(ctx.handle).decode()
    torch.cuda.synchronize()
    return host(c_static), host(c_plain)


# (first, second): the second call is smaller than the first
PAIRS = [
    ((1 << 25, 1 << 25), ((1 << 16) + 5, 3000)),          # the largest product the buffer holds, then a small one
    (((1 << 20) + 77, (1 << 19) - 1), (1 << 16, 1 << 16)),
    ((64 * 2049 + 11, 64 * 2047 + 5), (65, 63)),
]


@pytest.mark.parametrize("w", [64, 128])
@pytest.mark.parametrize("first,second", PAIRS)
def test_static_equals_plain_two_calls(first, second, w):
    ctx = P.Context(0)
    try:
        ctx.set_word_bits(w)
        for k, (na, nb) in enumerate((first, second)):
            if P.workspace_bytes(na, nb, w) > P.STATIC_SCRATCH_BYTES:
                continue  # w = 128 needs more workspace than the buffer holds at the largest size
            say(f"case static vs plain w={w} call {k}: {na}x{nb}")
            a, b, da, db = _operands(0x7A00 + 16 * k, na, nb)
            got, want = _both(ctx, da, na, db, nb)
            assert np.array_equal(got, want), (w, k, na, nb)
            if na + nb <= (1 << 21):
                assert np.array_equal(got, oracle.mul(a, na, b, nb, threads=8)), (w, k, na, nb)
    finally:
        torch.cuda.synchronize()
        ctx.close()


def test_static_refuses_products_beyond_the_buffer():
    ctx = P.Context(0)
    try:
        L = P.lib()
        na = nb = (1 << 25) + 64  # 2^21 points: more workspace than the buffer holds
        assert P.workspace_bytes(na, nb) > P.STATIC_SCRATCH_BYTES
        a = torch.zeros((na + 63) // 64, dtype=torch.int64, device="cuda")
        c = torch.full((P.out_words(na, nb),), -1, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        rc = L.gf2x_mul_dev_static(ctx.handle, P._ptr(a), na, P._ptr(a), nb, P._ptr(c), P._stream_handle(None))
        assert rc == P.GF2X_ENOMEM
        assert "static buffer" in L.gf2x_last_error(ctx.handle).decode()
        torch.cuda.synchronize()
        assert bool((c == -1).all())
        # empty operands: nothing written, OK
        assert L.gf2x_mul_dev_static(ctx.handle, None, 0, P._ptr(a), 64, P._ptr(c), P._stream_handle(None)) == P.GF2X_OK
        # overlap of the product with an operand is refused as in gf2x_mul_dev
        assert L.gf2x_mul_dev_static(ctx.handle, P._ptr(a), 640, P._ptr(a), 640, P._ptr(a),
                                     P._stream_handle(None)) == P.GF2X_EINVAL
    finally:
        torch.cuda.synchronize()
        ctx.close()
