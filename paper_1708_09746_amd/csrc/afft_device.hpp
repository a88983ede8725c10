// Device arithmetic and per-tile kernel bodies of the additive-FFT multiplier.
//
// Every kernel body is written as phases separated by AFFT_SYNC(); inside a
// phase, work items are visited by a strided loop (tid, tid + nt, ...).  On the
// GPU tid/nt are the thread index and block size; the same body also runs on
// the host with tid = 0, nt = 1 (a sequential emulation used for debugging).
//
// Field elements: TGF(2^128) elements are uint4 (x = bits 0..31, ..., w = bits
// 96..127).  Word c of an element is its component in TGF(2^32) along the basis
// element {1, x6, x7, x6 x7}[c]; multiplying by a subfield element acts on each
// word independently (Prop. 2).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#if defined(__HIP_DEVICE_COMPILE__)
#define AFFT_SYNC() __syncthreads()
#else
#define AFFT_SYNC() \
    do {            \
    } while (0)
#endif
#define AFFT_HD __host__ __device__ __forceinline__

// Ordering among the lanes of one wave only: the LDS writes of this wave are
// complete and visible to its own later LDS reads (a wave's LDS operations are
// executed in order; the fence keeps the compiler from moving accesses across
// it).  For phases whose LDS data each wave owns alone.
#if defined(__HIP_DEVICE_COMPILE__)
#define AFFT_WAVE_SYNC()                                     \
    do {                                                     \
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront"); \
        __builtin_amdgcn_wave_barrier();                     \
    } while (0)
#else
#define AFFT_WAVE_SYNC() \
    do {                 \
    } while (0)
#endif

namespace gf2x {

struct BcLayer {
    uint32_t log_d;  // D = 2^log_d units
    uint32_t log_k;  // k = 2^log_k units
    uint32_t log_u;  // unit = 2^log_u elements
    uint32_t pad;
};

// ------------------------------------------------------------ GF(256) table
// mt[(x << 8) | y] = x * y in GF(256) = TGF(2^8), tower basis.

AFFT_HD uint32_t m8(const uint8_t* mt, uint32_t x, uint32_t y) { return mt[(x << 8) | y]; }

// ----------------------------------------- multiplication by a subfield scalar
// e * x4 for e in TGF(2^16) = GF(256)[x4]: e0 + e1 x4 -> e1 c16 + (e0 + e1) x4,
// with c16 = x1 x2 x3 = 0x80.
AFFT_HD uint32_t mulx4_16(const uint8_t* mt, uint32_t e) {
    uint32_t e0 = e & 255u, e1 = (e >> 8) & 255u;
    return m8(mt, 0x80u, e1) | ((e0 ^ e1) << 8);
}
// e * c32 for e in TGF(2^16), c32 = x1 x2 x3 x4 = 0x8000 = c16 * x4
AFFT_HD uint32_t mulc32(const uint8_t* mt, uint32_t e) {
    uint32_t t = mulx4_16(mt, e);
    return m8(mt, 0x80u, t & 255u) | (m8(mt, 0x80u, t >> 8) << 8);
}

// ---------------------------------------------- Karatsuba form of the product
// A TGF(2^16) scalar s = s0 + s1 x4 times e = e0 + e1 x4 needs three GF(256)
// products: t1 = e0 s0, t2 = e1 (c16 s1), t3 = (e0 + e1)(s0 + s1), and then
// e s = (t1 + t2) + (t3 + t1) x4.  The scalar enters only through the three
// bytes k3(s) = (s0, c16 s1, s0 + s1).  A TGF(2^32) scalar l = l0 + l1 x5
// times a = a0 + a1 x5 splits the same way over TGF(2^16):
//   a l = (a0 l0 + a1 (c32 l1)) + ((a0 + a1)(l0 + l1) + a0 l0) x5,
// so its "mu-set" is k3(l0), k3(c32 l1), k3(l0 + l1) (9 bytes, 9 lookups per
// word instead of 16; 3 per 16-bit half instead of 4 when l1 = 0).

AFFT_HD uint32_t k3_of(const uint8_t* mt, uint32_t s) {
    uint32_t s0 = s & 255u, s1 = (s >> 8) & 255u;
    return s0 | (m8(mt, 0x80u, s1) << 8) | ((s0 ^ s1) << 16);
}

AFFT_HD uint4 make_mu_k(const uint8_t* mt, uint32_t lam) {
    uint32_t l0 = lam & 0xffffu, l1 = lam >> 16;
    uint4 m;
    m.x = k3_of(mt, l0);
    m.y = k3_of(mt, mulc32(mt, l1));
    m.z = k3_of(mt, l0 ^ l1);
    m.w = lam;
    return m;
}

// Byte permute of the pair (hi, lo): byte i of the result is selected by
// byte i of sel: 0..3 take bytes 0..3 of lo, 4..7 bytes 0..3 of hi, 0x0c
// gives 0 (the other selector values are not used here).  One v_perm_b32.
AFFT_HD uint32_t perm32(uint32_t hi, uint32_t lo, uint32_t sel) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_perm(hi, lo, sel);
#else
    uint32_t r = 0;
    for (int i = 0; i < 4; ++i) {
        uint32_t v = (sel >> (8 * i)) & 255u, b = 0;
        if (v < 4)
            b = (lo >> (8 * v)) & 255u;
        else if (v < 8)
            b = (hi >> (8 * (v - 4))) & 255u;
        r |= b << (8 * i);
    }
    return r;
#endif
}

// Table index (k << 8) | e with k = byte kb of kw and e = byte eb of ew.
// a ^ b ^ c in one instruction (gfx950's three-input bit operation, truth
// table 0x96: the parity of the three inputs)
AFFT_HD uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
#else
    return a ^ b ^ c;
#endif
}

#define AFFT_IX(kw, kb, ew, eb) perm32((kw), (ew), 0x0c0c0000u | ((4u + (kb)) << 8) | (eb))

// word times lambda; mode 0: lambda in GF(256), 1: TGF(2^16), 2: TGF(2^32),
// 3: TGF(2^32) with l1 in GF(256).
// The Karatsuba products above, arranged so that every lookup index is one
// byte permute of a mu-set word and a data word, and the byte results are
// placed and summed with permutes and XORs (no shifts or masks):
//   mode 2, with a = (a.b0..a.b3), p1 = a0 k3(l0), p2 = a1 k3(c32 l1),
//   p3 = (a0 + a1) k3(l0 + l1), each p = (t1 + t2) + (t3 + t1) x4:
//   out = [t1a t1a t1a t1a] + [t2a t3a t2a t3a] + [t1b t1b t1c t1c]
//       + [t2b t3b 0 0] + [0 0 t2c t3c]     (bytes 0..3)
// Mode 3: with l1 in GF(256), c32 l1 = (c16 l1) x4 has a zero low byte, so
// the first byte of k3(c32 l1) is 0 and t1b = 0 (8 lookups instead of 9).
AFFT_HD uint32_t mul_word_k(const uint8_t* mt, const uint4& m, uint32_t a, int mode) {
    if (mode == 0) {
        const uint32_t t0 = mt[AFFT_IX(m.x, 0, a, 0)], t1 = mt[AFFT_IX(m.x, 0, a, 1)];
        const uint32_t t2 = mt[AFFT_IX(m.x, 0, a, 2)], t3 = mt[AFFT_IX(m.x, 0, a, 3)];
        return perm32(t1, t0, 0x0c0c0400u) | perm32(t3, t2, 0x04000c0cu);
    }
    const uint32_t dd = a ^ (a >> 8);  // byte 0: a.b0 + a.b1, byte 2: a.b2 + a.b3
    const uint32_t t1a = mt[AFFT_IX(m.x, 0, a, 0)], t2a = mt[AFFT_IX(m.x, 1, a, 1)];
    const uint32_t t3a = mt[AFFT_IX(m.x, 2, dd, 0)];
    if (mode == 1) {
        const uint32_t t1b = mt[AFFT_IX(m.x, 0, a, 2)], t2b = mt[AFFT_IX(m.x, 1, a, 3)];
        const uint32_t t3b = mt[AFFT_IX(m.x, 2, dd, 2)];
        return xor3(perm32(t1b, t1a, 0x04040000u), perm32(t2b, t2a, 0x0c040c00u), perm32(t3b, t3a, 0x040c000cu));
    }
    const uint32_t sw = a ^ (a >> 16);   // low half: a0 + a1
    const uint32_t sd = sw ^ (sw >> 8);  // byte 0: its two bytes summed
    const uint32_t t1b = mode == 3 ? 0u : (uint32_t)mt[AFFT_IX(m.y, 0, a, 2)];
    const uint32_t t2b = mt[AFFT_IX(m.y, 1, a, 3)];
    const uint32_t t3b = mt[AFFT_IX(m.y, 2, dd, 2)];
    const uint32_t t1c = mt[AFFT_IX(m.z, 0, sw, 0)], t2c = mt[AFFT_IX(m.z, 1, sw, 1)];
    const uint32_t t3c = mt[AFFT_IX(m.z, 2, sd, 0)];
    return xor3(xor3(perm32(t1a, t1a, 0x00000000u), perm32(t3a, t2a, 0x04000400u), perm32(t1c, t1b, 0x04040000u)),
                perm32(t3b, t2b, 0x0c0c0400u), perm32(t3c, t2c, 0x04000c0cu));
}

AFFT_HD uint4 mul_sub_k(const uint8_t* mt, const uint4& m, const uint4& v, int mode) {
    uint4 r;
    r.x = mul_word_k(mt, m, v.x, mode);
    r.y = mul_word_k(mt, m, v.y, mode);
    r.z = mul_word_k(mt, m, v.z, mode);
    r.w = mul_word_k(mt, m, v.w, mode);
    return r;
}

AFFT_HD uint4 xor4(const uint4& a, const uint4& b) {
    uint4 r;
    r.x = a.x ^ b.x;
    r.y = a.y ^ b.y;
    r.z = a.z ^ b.z;
    r.w = a.w ^ b.w;
    return r;
}

// ------------------------------------------------- generic tower product
// Karatsuba form of the defining relation, down to GF(256):
//   t = a1 b1, lo = a0 b0 + c_W t, hi = (a0 + a1)(b0 + b1) + a0 b0.
// c_W (the product of the generators below the top one) satisfies
// c_{2W} = x_{log2 W} c_W, so e * c_{2W} = (e * x) * c_W with
// (e0 + e1 x) x = e1 c_W + (e0 + e1) x:  mulc_{2W}(e) = (c_W c_W e1, c_W (e0 + e1)).

AFFT_HD uint32_t gm16(const uint8_t* mt, uint32_t a, uint32_t b) {
    uint32_t a0 = a & 255u, a1 = a >> 8, b0 = b & 255u, b1 = b >> 8;
    uint32_t t = m8(mt, a1, b1), p0 = m8(mt, a0, b0), p1 = m8(mt, a0 ^ a1, b0 ^ b1);
    return (p0 ^ m8(mt, 0x80u, t)) | ((p1 ^ p0) << 8);
}
// The generic product with its constant multiples by word tables (the
// pointwise products): the multiples by c32 and c64 are GF(2)-linear, so
// c32 e = T32[0][e0] + T32[1][e1] over the bytes of e in TGF(2^16) and
// c64 e = sum_k T64[k][byte k of e] for e in TGF(2^32).  ctab holds T64 (4 x
// 256 words), T32 (2 x 256 halfwords), both built on the host (2 + 4 lookups
// where the byte-level recursion takes 3 + 9), then at kC16Tab the three
// 3-bit-group tables of multiplication by c16 in GF(256) (5 words, as for an
// 8-bit FFT multiplier).  The c16 multiple of the innermost level,
// c16 (a1 b1) = (c16 a1) b1, is taken on the operand: c16 acts byte-wise and
// linearly, so the scaled bytes of every leaf operand are the same
// combinations of the bytes of ca = c16 a (one register-table multiply per
// word of a) as the leaf operands are of a.
constexpr int kC16Tab = 4 * 256 + 256;
constexpr int kConstTabWords = kC16Tab + 8;
AFFT_HD uint32_t mulc32_t(const uint32_t* ctab, uint32_t e) {  // e in TGF(2^16), times c32 (bit 15)
    const uint16_t* t = (const uint16_t*)(ctab + 1024);
    return (uint32_t)t[e & 255u] ^ (uint32_t)t[256 + ((e >> 8) & 255u)];
}
AFFT_HD uint32_t mulc64_t(const uint32_t* ctab, uint32_t e) {  // e in TGF(2^32), times c64 (bit 31)
    return ctab[e & 255u] ^ ctab[256 + ((e >> 8) & 255u)] ^ ctab[512 + ((e >> 16) & 255u)] ^ ctab[768 + (e >> 24)];
}
AFFT_HD uint64_t mulc128_t(const uint32_t* ctab, uint64_t e) {  // e in TGF(2^64), times c128 (bit 63)
    const uint32_t e0 = (uint32_t)e, e1 = (uint32_t)(e >> 32);
    return (uint64_t)mulc64_t(ctab, mulc64_t(ctab, e1)) | ((uint64_t)mulc64_t(ctab, e0 ^ e1) << 32);
}
// a, b in TGF(2^16); ca = c16 a byte-wise
AFFT_HD uint32_t gm16c(const uint8_t* mt, uint32_t a, uint32_t ca, uint32_t b) {
    const uint32_t a0 = a & 255u, a1 = a >> 8, b0 = b & 255u, b1 = b >> 8;
    const uint32_t t = m8(mt, ca >> 8, b1), p0 = m8(mt, a0, b0), p1 = m8(mt, a0 ^ a1, b0 ^ b1);
    return (p0 ^ t) | ((p1 ^ p0) << 8);
}
AFFT_HD uint32_t gm32_t(const uint8_t* mt, const uint32_t* ctab, uint32_t a, uint32_t ca, uint32_t b) {
    const uint32_t a0 = a & 0xffffu, a1 = a >> 16, c0 = ca & 0xffffu, c1 = ca >> 16, b0 = b & 0xffffu, b1 = b >> 16;
    const uint32_t t = gm16c(mt, a1, c1, b1), p0 = gm16c(mt, a0, c0, b0), p1 = gm16c(mt, a0 ^ a1, c0 ^ c1, b0 ^ b1);
    return (p0 ^ mulc32_t(ctab, t)) | ((p1 ^ p0) << 16);
}
AFFT_HD uint64_t gm64_t(const uint8_t* mt, const uint32_t* ctab, uint64_t a, uint64_t ca, uint64_t b) {
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32), c0 = (uint32_t)ca, c1 = (uint32_t)(ca >> 32);
    const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
    const uint32_t t = gm32_t(mt, ctab, a1, c1, b1), p0 = gm32_t(mt, ctab, a0, c0, b0);
    const uint32_t p1 = gm32_t(mt, ctab, a0 ^ a1, c0 ^ c1, b0 ^ b1);
    return (uint64_t)(p0 ^ mulc64_t(ctab, t)) | ((uint64_t)(p1 ^ p0) << 32);
}
AFFT_HD uint4 gm128_t(const uint8_t* mt, const uint32_t* ctab, const uint4& a, const uint4& ca, const uint4& b) {
    const uint64_t a0 = a.x | ((uint64_t)a.y << 32), a1 = a.z | ((uint64_t)a.w << 32);
    const uint64_t c0 = ca.x | ((uint64_t)ca.y << 32), c1 = ca.z | ((uint64_t)ca.w << 32);
    const uint64_t b0 = b.x | ((uint64_t)b.y << 32), b1 = b.z | ((uint64_t)b.w << 32);
    const uint64_t t = gm64_t(mt, ctab, a1, c1, b1), p0 = gm64_t(mt, ctab, a0, c0, b0);
    const uint64_t p1 = gm64_t(mt, ctab, a0 ^ a1, c0 ^ c1, b0 ^ b1);
    const uint64_t lo = p0 ^ mulc128_t(ctab, t), hi = p1 ^ p0;
    return make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
}

// TGF(2^256) = TGF(2^128)[x_8]/(x_8^2 + x_8 + c256), elements as two uint4
// halves (lo, hi); c256 = x_1 ... x_7 = c128 x_7, so for e = e0 + e1 x_7 in
// TGF(2^128):  e c256 = (e x_7) c128 = c128 c128 e1 + c128 (e0 + e1) x_7.
AFFT_HD uint4 mulc256_t(const uint32_t* ctab, const uint4& e) {  // e in TGF(2^128), times c256 (bit 127)
    const uint64_t e0 = e.x | ((uint64_t)e.y << 32), e1 = e.z | ((uint64_t)e.w << 32);
    const uint64_t lo = mulc128_t(ctab, mulc128_t(ctab, e1)), hi = mulc128_t(ctab, e0 ^ e1);
    return make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
}
// (a0, a1), (b0, b1) in TGF(2^256); (ca0, ca1) = c16 (a0, a1) byte-wise
AFFT_HD void gm256_t(const uint8_t* mt, const uint32_t* ctab, const uint4& a0, const uint4& a1, const uint4& ca0,
                     const uint4& ca1, const uint4& b0, const uint4& b1, uint4& c0, uint4& c1) {
    const uint4 t = gm128_t(mt, ctab, a1, ca1, b1), p0 = gm128_t(mt, ctab, a0, ca0, b0);
    const uint4 p1 = gm128_t(mt, ctab, xor4(a0, a1), xor4(ca0, ca1), xor4(b0, b1));
    c0 = xor4(p0, mulc256_t(ctab, t));
    c1 = xor4(p1, p0);
}

// ------------------------------------------------------- table loaders

template <typename W>
AFFT_HD void copy_words(int tid, int nt, W* dst, const W* src, int n) {
    for (int i = tid; i < n; i += nt) dst[i] = src[i];
}

}  // namespace gf2x
