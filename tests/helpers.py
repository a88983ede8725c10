"""Shared test helpers: conversions between numpy words, Python ints and
device tensors.  No arithmetic of the method lives here."""
import numpy as np


def to_int(words) -> int:
    return int.from_bytes(np.ascontiguousarray(words, dtype=np.uint64).tobytes(), "little")


def to_words(x: int, nbits: int) -> np.ndarray:
    nw = (nbits + 63) // 64
    return np.frombuffer(x.to_bytes(8 * nw, "little"), dtype=np.uint64).copy()


def dev(words):
    """numpy uint64 words -> int64 CUDA tensor (same bits)."""
    import torch

    w = np.ascontiguousarray(words, dtype=np.uint64)
    if w.size == 0:
        w = np.zeros(1, dtype=np.uint64)
    return torch.from_numpy(w.view(np.int64).copy()).cuda()


def host(t) -> np.ndarray:
    """CUDA int64 tensor -> numpy uint64 words."""
    return t.detach().cpu().numpy().view(np.uint64).reshape(-1).copy()


def spectrum_ints(spec_tensor) -> list:
    """(N, 2) int64 spectrum tensor -> list of 128-bit Python ints."""
    raw = host(spec_tensor)
    return [int(raw[2 * j]) | (int(raw[2 * j + 1]) << 64) for j in range(raw.size // 2)]


def spread_words(a: np.ndarray, nbits: int) -> np.ndarray:
    """a(x)^2 as words: bit i of a moves to bit 2i (closed form of squaring in
    GF(2)[x]); returns ceil((2 nbits - 1) / 64) words."""
    a = np.ascontiguousarray(a, dtype=np.uint64)
    tab = np.zeros(1 << 16, dtype=np.uint64)
    x = np.arange(1 << 16, dtype=np.uint64)
    for i in range(16):
        tab |= ((x >> np.uint64(i)) & np.uint64(1)) << np.uint64(2 * i)
    out = np.empty(2 * a.size, dtype=np.uint64)
    m = np.uint64(0xFFFF)
    lo = tab[a & m] | (tab[(a >> np.uint64(16)) & m] << np.uint64(32))
    hi = tab[(a >> np.uint64(32)) & m] | (tab[(a >> np.uint64(48)) & m] << np.uint64(32))
    out[0::2] = lo
    out[1::2] = hi
    nw = (2 * nbits - 1 + 63) // 64
    return out[:nw]
