"""MI355X (gfx950) multiplier for long binary polynomials: the additive FFT over
a tower field (Chen, Cheng, Kuo, Li, Yang, arXiv:1708.09746, Alg. 5).

This module only marshals arguments to the C ABI of ``libgf2x_afft.so``
(declared in ``include/gf2x_afft.h``); every step of the product runs in the
library's HIP kernels.  PyTorch supplies device memory and streams.  Polynomials
are 1-D int64/uint64 tensors of little-endian 64-bit words; spectra are int64
tensors of shape (N, 2) (16-byte TGF(2^128) elements).

If the library is missing, every call raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgf2x_afft.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "gf2x_afft.h")

GF2X_OK, GF2X_EINVAL, GF2X_ERANGE, GF2X_ENOMEM, GF2X_EDEVICE = 0, -1, -2, -3, -4
STATIC_SCRATCH_BYTES = 64 << 20  # GF2X_STATIC_SCRATCH_BYTES: the fixed buffer of gf2x_mul_dev_static

_lib = None


class Gf2xError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class TraceRec(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("elements", ctypes.c_uint64), ("bytes_read", ctypes.c_uint64),
                ("bytes_written", ctypes.c_uint64), ("lookups", ctypes.c_uint64), ("ms", ctypes.c_float)]


KIND_NAMES = ["pack", "basiscvt_tile", "basiscvt_layer", "fft_pass", "pointmul", "psi_combine", "basiscvt_class",
              "spine", "whole_product", "product_tail"]
KERNEL_OF_KIND = ["k_pack", "k_bc_tile", "k_bc_layer", "k_fft", "k_pmul", "k_psi", "k_bc_class", "k_spine",
                  "k_single", "k_tail"]


class BatchStats(ctypes.Structure):
    _fields_ = [("ops", ctypes.c_uint64), ("ranks", ctypes.c_uint64), ("launches", ctypes.c_uint64),
                ("tiles", ctypes.c_uint64), ("workspace_bytes", ctypes.c_uint64)]


class TuneRec(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("bottom_log", ctypes.c_int32), ("col_rows_log", ctypes.c_int32),
                ("copies", ctypes.c_int32), ("candidates", ctypes.c_int32), ("us_default", ctypes.c_float),
                ("us_best", ctypes.c_float)]


class ServerCfg(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_uint64), ("max_active", ctypes.c_uint32),
                ("levels_per_iter", ctypes.c_uint32), ("inflight", ctypes.c_uint32), ("mode", ctypes.c_int32),
                ("iter_tiles", ctypes.c_uint64)]


class Done(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("iterations", ctypes.c_uint32),
                ("t_submit_ns", ctypes.c_uint64), ("t_admit_ns", ctypes.c_uint64), ("t_done_ns", ctypes.c_uint64)]


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in ("submitted", "admitted", "completed", "iterations", "launches",
                                              "queued", "active", "arena_used", "arena_peak", "active_peak")]


class Job(ctypes.Structure):
    _fields_ = [("a", ctypes.c_void_p), ("na_bits", ctypes.c_uint64), ("b", ctypes.c_void_p),
                ("nb_bits", ctypes.c_uint64), ("c", ctypes.c_void_p)]


def lib():
    """The loaded C library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, u64, i32, sz = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_size_t
        sig = {
            "gf2x_ctx_create": (i32, [ctypes.POINTER(vp), i32]),
            "gf2x_ctx_destroy": (None, [vp]),
            "gf2x_out_words": (sz, [u64, u64]),
            "gf2x_fft_log2": (i32, [u64, u64]),
            "gf2x_workspace_bytes": (sz, [u64, u64]),
            "gf2x_workspace_bytes_w": (sz, [u64, u64, i32]),
            "gf2x_mul": (i32, [vp, u64, vp, u64, vp]),
            "gf2x_mul_dev": (i32, [vp, vp, u64, vp, u64, vp, vp]),
            "gf2x_mul_dev_static": (i32, [vp, vp, u64, vp, u64, vp, vp]),
            "gf2x_set_single_launch": (i32, [vp, i32]),
            "gf2x_set_fusion": (i32, [vp, i32, i32, i32]),
            "gf2x_forward_dev": (i32, [vp, vp, u64, i32, vp, vp]),
            "gf2x_pointmul_dev": (i32, [vp, vp, vp, vp, u64, vp]),
            "gf2x_inverse_dev": (i32, [vp, vp, i32, vp, u64, vp]),
            "gf2x_basiscvt_dev": (i32, [vp, vp, i32, i32, vp]),
            "gf2x_simple_mul_dev": (i32, [vp, vp, u64, vp, u64, vp, vp]),
            "gf2x_simple_forward_dev": (i32, [vp, vp, u64, i32, vp, vp]),
            "gf2x_frobenius_log2n": (i32, [u64, u64]),
            "gf2x_frobenius_workspace_bytes": (sz, [u64, u64]),
            "gf2x_frobenius_mul_dev": (i32, [vp, vp, u64, vp, u64, vp, vp]),
            "gf2x_frobenius_forward_dev": (i32, [vp, vp, u64, i32, vp, vp]),
            "gf2x_frobenius_inverse_dev": (i32, [vp, vp, i32, vp, u64, vp]),
            "gf2x_mul_batch": (i32, [vp, ctypes.POINTER(Job), sz, vp]),
            "gf2x_batch_create": (i32, [vp, ctypes.POINTER(Job), sz, i32, ctypes.POINTER(vp)]),
            "gf2x_batch_check": (i32, [vp]),
            "gf2x_batch_set_spin_limit": (i32, [vp, ctypes.c_uint32]),
            "gf2x_batch_run": (i32, [vp, vp]),
            "gf2x_batch_info": (i32, [vp, ctypes.POINTER(BatchStats)]),
            "gf2x_batch_destroy": (None, [vp]),
            "gf2x_set_schedule": (i32, [vp, i32, i32, i32]),
            "gf2x_get_schedule": (i32, [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
            "gf2x_autotune": (i32, [vp, i32, i32, i32, ctypes.POINTER(TuneRec)]),
            "gf2x_set_truncation": (i32, [vp, i32, i32, i32]),
            "gf2x_eval_points": (u64, [vp, u64, u64]),
            "gf2x_set_word_bits": (i32, [vp, i32]),
            "gf2x_get_word_bits": (i32, [vp]),
            "gf2x_lookup_rate": (i32, [vp, ctypes.POINTER(ctypes.c_double)]),
            "gf2x_now_ns": (u64, []),
            "gf2x_server_create": (i32, [vp, ctypes.POINTER(ServerCfg), ctypes.POINTER(vp)]),
            "gf2x_server_submit": (i32, [vp, vp, u64, vp, u64, vp, u64, vp]),
            "gf2x_server_step": (i32, [vp, u64]),
            "gf2x_server_poll": (sz, [vp, ctypes.POINTER(Done), sz]),
            "gf2x_server_info": (i32, [vp, ctypes.POINTER(ServerStats)]),
            "gf2x_server_destroy": (None, [vp]),
            "gf2x_trace_begin": (i32, [vp, ctypes.c_uint32]),
            "gf2x_trace_read": (ctypes.c_int64, [vp, ctypes.POINTER(TraceRec), sz]),
            "gf2x_strerror": (ctypes.c_char_p, [i32]),
            "gf2x_last_error": (ctypes.c_char_p, [vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def header_functions() -> list[str]:
    """Names of the functions declared in include/gf2x_afft.h."""
    with open(HEADER_PATH) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gf2x_[a-z0-9_]+)\s*\(", text)))


def out_words(na_bits: int, nb_bits: int) -> int:
    return int(lib().gf2x_out_words(na_bits, nb_bits))


def fft_log2(na_bits: int, nb_bits: int) -> int:
    return int(lib().gf2x_fft_log2(na_bits, nb_bits))


def frobenius_log2n(na_bits: int, nb_bits: int) -> int:
    return int(lib().gf2x_frobenius_log2n(na_bits, nb_bits))


def workspace_bytes(na_bits: int, nb_bits: int, w: int = 64) -> int:
    """Device workspace of one product with Split into w-bit words (64 or 128)."""
    if w == 64:
        return int(lib().gf2x_workspace_bytes(na_bits, nb_bits))
    return int(lib().gf2x_workspace_bytes_w(na_bits, nb_bits, w))


def strerror(code: int) -> str:
    return lib().gf2x_strerror(code).decode()


def _stream_handle(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _ptr(t):
    return ctypes.c_void_p(int(t.data_ptr())) if t is not None else ctypes.c_void_p(0)


class Context:
    """A library context on one HIP device (tables and workspace)."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        rc = lib().gf2x_ctx_create(ctypes.byref(h), int(device))
        if rc != GF2X_OK:
            raise Gf2xError(rc, f"gf2x_ctx_create({device}): {strerror(rc)}")
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            lib().gf2x_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int, what: str):
        if rc != GF2X_OK:
            msg = lib().gf2x_last_error(self._h).decode()
            raise Gf2xError(rc, f"{what}: {strerror(rc)}: {msg}")

    @property
    def handle(self):
        return self._h

    # ---- products
    def mul_into(self, a, na_bits: int, b, nb_bits: int, c, stream=None):
        rc = lib().gf2x_mul_dev(self._h, _ptr(a), na_bits, _ptr(b), nb_bits, _ptr(c), _stream_handle(stream))
        self._check(rc, "gf2x_mul_dev")
        return c

    def set_single_launch(self, max_log2n: int):
        """Products of at most 2^max_log2n points in one launch (-1: never)."""
        self._check(lib().gf2x_set_single_launch(self._h, int(max_log2n)), "gf2x_set_single_launch")

    def set_fusion(self, mask: int, single_max_log2n: int = 13, batch_max_log2n: int = 11):
        """Which BasisCvt sub-conversions run inside FFT passes (bits: 1
        forward transforms, 2 inverse transforms, 4 pass split aligned to
        BasisCvt's top level), for transforms of at most 2^single_max_log2n
        points in single products and 2^batch_max_log2n in batches and
        serving iterations."""
        self._check(lib().gf2x_set_fusion(self._h, int(mask), int(single_max_log2n), int(batch_max_log2n)),
                    "gf2x_set_fusion")

    def mul_static_into(self, a, na_bits: int, b, nb_bits: int, c, stream=None):
        """The same product with the workspace in the library's fixed device
        buffer (gf2x_mul_dev_static: no device allocation in the call)."""
        rc = lib().gf2x_mul_dev_static(self._h, _ptr(a), na_bits, _ptr(b), nb_bits, _ptr(c), _stream_handle(stream))
        self._check(rc, "gf2x_mul_dev_static")
        return c

    def mul(self, a, na_bits: int, b, nb_bits: int, stream=None):
        import torch

        ow = out_words(na_bits, nb_bits)
        c = torch.empty(max(ow, 1), dtype=torch.int64, device=a.device)[:ow]
        return self.mul_into(a, na_bits, b, nb_bits, c, stream)

    def simple_mul_into(self, a, na_bits: int, b, nb_bits: int, c, stream=None):
        """The same product by the simple variant (Alg. 4)."""
        rc = lib().gf2x_simple_mul_dev(self._h, _ptr(a), na_bits, _ptr(b), nb_bits, _ptr(c), _stream_handle(stream))
        self._check(rc, "gf2x_simple_mul_dev")
        return c

    def simple_mul(self, a, na_bits: int, b, nb_bits: int, stream=None):
        import torch

        ow = out_words(na_bits, nb_bits)
        c = torch.empty(max(ow, 1), dtype=torch.int64, device=a.device)[:ow]
        return self.simple_mul_into(a, na_bits, b, nb_bits, c, stream)

    def simple_forward(self, a, na_bits: int, log2n: int, spec=None, stream=None):
        """Values of the operand's word polynomial at the Cantor points phi(j),
        j < 2^log2n, in the polynomial-basis GF(2^128) (Alg. 4)."""
        import torch

        if spec is None:
            spec = torch.empty((1 << log2n, 2), dtype=torch.int64, device=a.device)
        rc = lib().gf2x_simple_forward_dev(self._h, _ptr(a), na_bits, log2n, _ptr(spec), _stream_handle(stream))
        self._check(rc, "gf2x_simple_forward_dev")
        return spec

    def frobenius_mul_into(self, a, na_bits: int, b, nb_bits: int, c, stream=None):
        """The same product by the Frobenius partition (App. C)."""
        rc = lib().gf2x_frobenius_mul_dev(self._h, _ptr(a), na_bits, _ptr(b), nb_bits, _ptr(c),
                                          _stream_handle(stream))
        self._check(rc, "gf2x_frobenius_mul_dev")
        return c

    def frobenius_mul(self, a, na_bits: int, b, nb_bits: int, stream=None):
        import torch

        ow = out_words(na_bits, nb_bits)
        c = torch.empty(max(ow, 1), dtype=torch.int64, device=a.device)[:ow]
        return self.frobenius_mul_into(a, na_bits, b, nb_bits, c, stream)

    def frobenius_forward(self, a, na_bits: int, log2n: int, spec=None, stream=None):
        """Values of the operand at the 2^log2n points beta_{m+64} + phi(j)
        (App. C), elements of the polynomial-basis GF(2^128)."""
        import torch

        if spec is None:
            spec = torch.empty((1 << log2n, 2), dtype=torch.int64, device=a.device)
        rc = lib().gf2x_frobenius_forward_dev(self._h, _ptr(a), na_bits, log2n, _ptr(spec), _stream_handle(stream))
        self._check(rc, "gf2x_frobenius_forward_dev")
        return spec

    def frobenius_inverse(self, spec, log2n: int, nc_bits: int, c=None, stream=None):
        """The polynomial (first nc_bits bits) with these values; spec is overwritten."""
        import torch

        if c is None:
            ow = (nc_bits + 63) // 64
            c = torch.empty(max(ow, 1), dtype=torch.int64, device=spec.device)[:ow]
        rc = lib().gf2x_frobenius_inverse_dev(self._h, _ptr(spec), log2n, _ptr(c), nc_bits, _stream_handle(stream))
        self._check(rc, "gf2x_frobenius_inverse_dev")
        return c

    def mul_batch(self, jobs, stream=None):
        """jobs: list of (a, na_bits, b, nb_bits, c) with device tensors."""
        rc = lib().gf2x_mul_batch(self._h, _job_array(jobs), len(jobs), _stream_handle(stream))
        self._check(rc, "gf2x_mul_batch")

    def batch(self, jobs, persistent: bool = False):
        """A reusable Batch of (a, na_bits, b, nb_bits, c) device-tensor jobs."""
        return Batch(self, jobs, persistent)

    def server(self, arena_bytes: int, max_active: int = 4096, levels_per_iter: int = 4, inflight: int = 2,
               persistent=False, iter_tiles: int = 0):
        """A continuous-batching request loop (Server) on this context;
        persistent: False (staged), True, or "adaptive"."""
        return Server(self, arena_bytes, max_active, levels_per_iter, inflight, persistent, iter_tiles)

    def lookup_rate(self) -> float:
        """Measured rate of random byte lookups into an LDS table (per second, whole device)."""
        v = ctypes.c_double()
        self._check(lib().gf2x_lookup_rate(self._h, ctypes.byref(v)), "gf2x_lookup_rate")
        return v.value

    # ---- truncated transforms
    def set_truncation(self, levels: int, min_log2n: int = 23, max_terms: int = 2):
        """Evaluate products of at least 2^min_log2n points at n_c rounded up
        to a multiple of 2^(m - levels) points, and further to at most
        max_terms set bits in blocks (0: any; levels 0: all N)."""
        self._check(lib().gf2x_set_truncation(self._h, levels, min_log2n, max_terms), "gf2x_set_truncation")

    def eval_points(self, na_bits: int, nb_bits: int) -> int:
        return int(lib().gf2x_eval_points(self._h, na_bits, nb_bits))

    # ---- word width of Split: 64 (TGF(2^128)) or 128 (TGF(2^256))
    def set_word_bits(self, w: int):
        self._check(lib().gf2x_set_word_bits(self._h, w), "gf2x_set_word_bits")

    def word_bits(self) -> int:
        return int(lib().gf2x_get_word_bits(self._h))

    # ---- FFT pass schedules
    def set_schedule(self, m: int, bottom_log: int, col_rows_log: int):
        self._check(lib().gf2x_set_schedule(self._h, m, bottom_log, col_rows_log), "gf2x_set_schedule")

    def get_schedule(self, m: int):
        b, r = ctypes.c_int(), ctypes.c_int()
        self._check(lib().gf2x_get_schedule(self._h, m, ctypes.byref(b), ctypes.byref(r)), "gf2x_get_schedule")
        return b.value, r.value

    def autotune(self, m_lo: int, m_hi: int, reps: int = 5):
        """Pick the fastest FFT pass schedule for each size 2^m, m in [m_lo, m_hi]."""
        out = (TuneRec * (m_hi - m_lo + 1))()
        self._check(lib().gf2x_autotune(self._h, m_lo, m_hi, reps, out), "gf2x_autotune")
        return [{k: (round(getattr(r, k), 2) if k.startswith("us") else int(getattr(r, k)))
                 for k, _ in TuneRec._fields_} for r in out]

    # ---- tracing
    def trace_begin(self, kind_mask: int = 0x3FF):
        self._check(lib().gf2x_trace_begin(self._h, kind_mask), "gf2x_trace_begin")

    def trace_end(self):
        """Stop tracing and return the traced launches (see trace_collect)."""
        recs = self.trace_collect()
        lib().gf2x_trace_begin(self._h, 0)
        return recs

    def trace_collect(self):
        """Wait for and return the traced launches so far (tracing continues)."""
        n = 1 << 16
        buf = (TraceRec * n)()
        got = lib().gf2x_trace_read(self._h, buf, n)
        if got < 0:
            self._check(int(got), "gf2x_trace_read")
        return [dict(kind=KIND_NAMES[r.kind], kernel=KERNEL_OF_KIND[r.kind], elements=r.elements,
                     bytes_read=r.bytes_read, bytes_written=r.bytes_written, lookups=r.lookups, ms=r.ms)
                for r in buf[:min(got, n)]]

    # ---- stages
    def forward(self, a, na_bits: int, log2n: int, spec=None, stream=None):
        import torch

        if spec is None:
            spec = torch.empty((1 << log2n, 2), dtype=torch.int64, device=a.device)
        rc = lib().gf2x_forward_dev(self._h, _ptr(a), na_bits, log2n, _ptr(spec), _stream_handle(stream))
        self._check(rc, "gf2x_forward_dev")
        return spec

    def pointmul(self, sa, sb, sc=None, stream=None):
        import torch

        if sc is None:
            sc = torch.empty_like(sa)
        rc = lib().gf2x_pointmul_dev(self._h, _ptr(sa), _ptr(sb), _ptr(sc), sa.shape[0], _stream_handle(stream))
        self._check(rc, "gf2x_pointmul_dev")
        return sc

    def inverse(self, spec, log2n: int, nc_bits: int, c=None, stream=None):
        import torch

        if c is None:
            nw = (nc_bits + 63) // 64
            c = torch.empty(max(nw, 1), dtype=torch.int64, device=spec.device)[:nw]
        rc = lib().gf2x_inverse_dev(self._h, _ptr(spec), log2n, _ptr(c), nc_bits, _stream_handle(stream))
        self._check(rc, "gf2x_inverse_dev")
        return c

    def basiscvt(self, words, log2n: int, inverse: bool = False, stream=None):
        rc = lib().gf2x_basiscvt_dev(self._h, _ptr(words), log2n, 1 if inverse else 0, _stream_handle(stream))
        self._check(rc, "gf2x_basiscvt_dev")
        return words


def _job_array(jobs):
    arr = (Job * max(len(jobs), 1))()
    for i, (a, na, b, nb, c) in enumerate(jobs):
        arr[i] = Job(int(a.data_ptr()), na, int(b.data_ptr()), nb, int(c.data_ptr()))
    return arr


class Batch:
    """Products planned once (gf2x_batch_create) and run many times; the first
    run records a hipGraph that later runs replay."""

    STAGED, PERSISTENT = 0, 1

    def __init__(self, ctx: "Context", jobs, persistent: bool = False):
        self.ctx = ctx
        self.jobs = list(jobs)  # keeps the tensors alive
        self.mode = self.PERSISTENT if persistent else self.STAGED
        h = ctypes.c_void_p()
        rc = lib().gf2x_batch_create(ctx.handle, _job_array(self.jobs), len(self.jobs), self.mode, ctypes.byref(h))
        ctx._check(rc, "gf2x_batch_create")
        self._h = h

    def run(self, stream=None):
        rc = lib().gf2x_batch_run(self._h, _stream_handle(stream))
        self.ctx._check(rc, "gf2x_batch_run")

    def set_spin_limit(self, polls: int):
        self.ctx._check(lib().gf2x_batch_set_spin_limit(self._h, polls), "gf2x_batch_set_spin_limit")

    def check(self):
        """Wait for the device; raise if the last persistent run stopped early."""
        self.ctx._check(lib().gf2x_batch_check(self._h), "gf2x_batch_check")

    def stats(self) -> dict:
        st = BatchStats()
        lib().gf2x_batch_info(self._h, ctypes.byref(st))
        return {k: int(getattr(st, k)) for k, _ in BatchStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib().gf2x_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def now_ns() -> int:
    """The library's clock (CLOCK_MONOTONIC, ns), the one completion times use."""
    return int(lib().gf2x_now_ns())


class Server:
    """Continuous batching of products (gf2x_server_*): submit requests whose
    device tensors stay alive until they complete, drive the engine with
    step(), collect completion records with poll()."""

    def __init__(self, ctx: "Context", arena_bytes: int, max_active: int, levels_per_iter: int, inflight: int,
                 persistent: bool, iter_tiles: int = 0):
        self.ctx = ctx
        mode = 2 if persistent == "adaptive" else (1 if persistent else 0)
        cfg = ServerCfg(arena_bytes, max_active, levels_per_iter, inflight, mode, iter_tiles)
        h = ctypes.c_void_p()
        ctx._check(lib().gf2x_server_create(ctx.handle, ctypes.byref(cfg), ctypes.byref(h)), "gf2x_server_create")
        self._h = h
        self._buf = (Done * 4096)()

    def submit(self, a, na_bits: int, b, nb_bits: int, c, tag: int, stream=None):
        """Queue c = a * b; the request starts after the work already enqueued
        on `stream` (default: the current stream), which produced a and b."""
        rc = lib().gf2x_server_submit(self._h, _ptr(a), na_bits, _ptr(b), nb_bits, _ptr(c), tag,
                                      _stream_handle(stream))
        self.ctx._check(rc, "gf2x_server_submit")

    def step(self, until_ns: int = 0):
        """Run the engine until now_ns() >= until_ns or nothing is left to do."""
        self.ctx._check(lib().gf2x_server_step(self._h, until_ns), "gf2x_server_step")

    def poll(self):
        """Completion records since the last poll: dicts with tag, status,
        iterations and the submit/admit/done times in ns."""
        out = []
        while True:
            n = lib().gf2x_server_poll(self._h, self._buf, len(self._buf))
            out.extend(dict(tag=d.tag, status=d.status, iterations=d.iterations, t_submit_ns=d.t_submit_ns,
                            t_admit_ns=d.t_admit_ns, t_done_ns=d.t_done_ns) for d in self._buf[:n])
            if n < len(self._buf):
                return out

    def drain(self):
        """Step until every submitted request has completed; return their records."""
        done = []
        while True:
            self.step(now_ns() + 10_000_000)
            done.extend(self.poll())
            st = self.stats()
            if st["queued"] == 0 and st["active"] == 0 and st["completed"] == st["submitted"]:
                return done

    def stats(self) -> dict:
        st = ServerStats()
        lib().gf2x_server_info(self._h, ctypes.byref(st))
        return {k: int(getattr(st, k)) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib().gf2x_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mul_host(a, na_bits: int, b, nb_bits: int):
    """c = a * b for numpy uint64 word arrays through the blocking host-pointer call."""
    import numpy as np

    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    ow = out_words(na_bits, nb_bits)
    c = np.zeros(max(ow, 1), dtype=np.uint64)
    rc = lib().gf2x_mul(a.ctypes.data_as(ctypes.c_void_p), na_bits, b.ctypes.data_as(ctypes.c_void_p), nb_bits,
                        c.ctypes.data_as(ctypes.c_void_p))
    if rc != GF2X_OK:
        raise Gf2xError(rc, f"gf2x_mul: {strerror(rc)}")
    return c[:ow]
