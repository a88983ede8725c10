"""The C-ABI library loads on the CPU and exports every function declared in
include/gf2x_afft.h; the size helpers follow the documented conventions.  No
GPU work is launched here."""
import ctypes

import pytest

import paper_1708_09746_amd as P


def test_library_exports_every_declared_function():
    L = ctypes.CDLL(P.LIB_PATH)
    names = P.header_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n


def test_binding_names_match_header():
    P.lib()  # binds signatures for all of them
    for n in P.header_functions():
        assert getattr(P.lib(), n).argtypes is not None, n


@pytest.mark.parametrize("na,nb,ow", [(0, 5, 0), (5, 0, 0), (1, 1, 1), (64, 1, 1), (64, 2, 2), (65, 64, 2),
                                      (64, 64, 2), (1 << 16, 1 << 16, 2048), (1 << 28, 1 << 28, 1 << 23)])
def test_out_words(na, nb, ow):
    assert P.out_words(na, nb) == ow


@pytest.mark.parametrize("na,nb,m", [(1, 1, 1), (64, 64, 1), (65, 64, 1), (65, 65, 2), (64 * 3, 64 * 2, 2), (64 * 3, 64 * 3, 3),
                                     (1 << 16, 1 << 16, 11), (1 << 20, 1 << 20, 15), (1 << 28, 1 << 28, 23),
                                     (1 << 29, 1 << 29, 24), (0, 7, -1)])
def test_fft_size(na, nb, m):
    assert P.fft_log2(na, nb) == m


def test_workspace_grows_with_size():
    small = P.workspace_bytes(1 << 16, 1 << 16)
    big = P.workspace_bytes(1 << 28, 1 << 28)
    # two spectra of N = 2^23 elements (16 B) plus two 2^22-word operands
    assert big >= 2 * 16 * (1 << 23) + 2 * 8 * (1 << 22)
    assert 0 < small < big


def test_workspace_by_word_width():
    """Workspace = converted words + two spectra, each 256-byte aligned; for
    w = 128 the words are 16 bytes and a spectrum is two planes of 16-byte
    halves (the same bytes as w = 64 for large balanced products)."""
    def al(x):
        return (x + 255) // 256 * 256

    def expect(na, nb, w):
        ka, kb = (na + w - 1) // w, (nb + w - 1) // w
        ma, mb = (ka - 1).bit_length(), (kb - 1).bit_length()
        m = max(1, (ka + kb - 2).bit_length())
        return al((w // 8) << ma) + al((w // 8) << mb) + 2 * al((16 * w // 64) << m)

    for na, nb in [(1, 1), (64, 64), (65, 64), (128, 129), (1000, 7), (1 << 20, 1 << 19), (1 << 28, 1 << 28)]:
        assert P.workspace_bytes(na, nb) == expect(na, nb, 64), (na, nb)
        assert P.workspace_bytes(na, nb, 128) == expect(na, nb, 128), (na, nb)
    assert P.workspace_bytes(1 << 28, 1 << 28, 128) == P.workspace_bytes(1 << 28, 1 << 28)
    assert P.lib().gf2x_workspace_bytes_w(100, 100, 96) == 0
    assert P.lib().gf2x_workspace_bytes_w(0, 100, 128) == 0


def test_status_names():
    for code in (0, -1, -2, -3, -4):
        assert P.strerror(code)
    assert P.strerror(-99) == "unknown status"


def test_static_buffer_size_matches_header():
    """The binding's size of gf2x_mul_dev_static's fixed buffer is the
    header's GF2X_STATIC_SCRATCH_BYTES, and that buffer holds the workspace of
    every product of up to 2^20 points (operands of 2^25 bits each) and none
    beyond."""
    import re

    with open(P.HEADER_PATH) as f:
        m = re.search(r"#define\s+GF2X_STATIC_SCRATCH_BYTES\s+\((\d+)u\s*<<\s*(\d+)\)", f.read())
    assert m and int(m.group(1)) << int(m.group(2)) == P.STATIC_SCRATCH_BYTES
    assert P.workspace_bytes(1 << 25, 1 << 25) <= P.STATIC_SCRATCH_BYTES
    assert P.workspace_bytes(64 << 20, 64) <= P.STATIC_SCRATCH_BYTES  # 2^20 words: 2^20 points
    assert P.fft_log2((1 << 25) + 65, 1 << 25) == 21
    assert P.workspace_bytes((1 << 25) + 65, 1 << 25) > P.STATIC_SCRATCH_BYTES
