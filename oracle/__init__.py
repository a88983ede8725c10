"""Oracle for the GF(2)[x] multiplier -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It holds:

* ``gf2x_oracle.c`` (built to ``liboracle.so``): the product by its definition,
  c_k = XOR_{i+j=k} a_i b_j, on 64-bit words with a software carry-less
  multiply, schoolbook + Karatsuba, optional POSIX threads; plus single output
  words and residues mod x^64 + q(x) for sampled checks at large sizes.
* ``tower.py``: the paper's stage definitions (tower field, s_i, novel basis,
  Alg. 1/2/3/5, changeRepr) for small inputs.
* ``simple.py``: the simple variant (Alg. 4): GF(2^128) in the polynomial
  basis of Sec. 3.1, Cantor-basis points, for small inputs.
* ``frobenius.py``: the Frobenius-partition variant (App. C): values at
  beta_{m+64} + V_m, the seven-layer encoding, for small inputs.

Nothing here is shared with, or imported by, the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "gf2x_oracle.c")

_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C, no GPU code)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared", "-pthread", "-o", tmp, SRC_PATH]
        )
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(LIB_PATH)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        L.oracle_clmul64_bitloop.argtypes = [ctypes.c_uint64, ctypes.c_uint64, u64p]
        L.oracle_clmul64_window.argtypes = [ctypes.c_uint64, ctypes.c_uint64, u64p]
        L.oracle_mul_schoolbook.argtypes = [u64p, ctypes.c_size_t, u64p, ctypes.c_size_t, u64p]
        L.oracle_out_words.argtypes = [ctypes.c_size_t, ctypes.c_size_t]
        L.oracle_out_words.restype = ctypes.c_size_t
        L.oracle_mul.argtypes = [u64p, ctypes.c_size_t, u64p, ctypes.c_size_t, u64p, ctypes.c_int]
        L.oracle_mul.restype = ctypes.c_int
        L.oracle_word.argtypes = [u64p, ctypes.c_size_t, u64p, ctypes.c_size_t, ctypes.c_size_t]
        L.oracle_word.restype = ctypes.c_uint64
        L.oracle_mod.argtypes = [u64p, ctypes.c_size_t, ctypes.c_uint64]
        L.oracle_mod.restype = ctypes.c_uint64
        L.oracle_mulmod.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        L.oracle_mulmod.restype = ctypes.c_uint64
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _as_words(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    if a.size == 0:
        a = np.zeros(1, dtype=np.uint64)
    return a


def clmul64(x: int, y: int, method: str = "window") -> int:
    out = (ctypes.c_uint64 * 2)()
    fn = lib().oracle_clmul64_window if method == "window" else lib().oracle_clmul64_bitloop
    fn(x, y, out)
    return int(out[0]) | (int(out[1]) << 64)


def out_words(na_bits: int, nb_bits: int) -> int:
    return int(lib().oracle_out_words(na_bits, nb_bits))


def mul(a, na_bits: int, b, nb_bits: int, threads: int = 1) -> np.ndarray:
    """The product a*b as ceil((na+nb-1)/64) words (empty if an operand is empty)."""
    ow = out_words(na_bits, nb_bits)
    c = np.zeros(max(ow, 1), dtype=np.uint64)
    if ow == 0:
        return c[:0]
    a = _as_words(a)
    b = _as_words(b)
    rc = lib().oracle_mul(_ptr(a), na_bits, _ptr(b), nb_bits, _ptr(c), int(threads))
    if rc != 0:
        raise RuntimeError(f"oracle_mul failed: {rc}")
    return c


def mul_schoolbook(a, b) -> np.ndarray:
    a = _as_words(a)
    b = _as_words(b)
    c = np.zeros(a.size + b.size, dtype=np.uint64)
    lib().oracle_mul_schoolbook(_ptr(a), a.size, _ptr(b), b.size, _ptr(c))
    return c


def word(a, na_bits: int, b, nb_bits: int, k: int) -> int:
    """Output word k of a*b straight from the convolution sum."""
    a = _as_words(a)
    b = _as_words(b)
    return int(lib().oracle_word(_ptr(a), na_bits, _ptr(b), nb_bits, k))


def mod(p, nbits: int, q: int) -> int:
    """p(x) mod (x^64 + q(x))."""
    p = _as_words(p)
    return int(lib().oracle_mod(_ptr(p), nbits, q))


def mulmod(x: int, y: int, q: int) -> int:
    return int(lib().oracle_mulmod(x, y, q))
