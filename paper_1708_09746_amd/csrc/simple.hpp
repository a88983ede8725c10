// The simple variant of the multiplier (Alg. 4): the working field stays
// GF(2^128) = GF(2)[x]/(x^128 + x^7 + x^2 + x + 1) in its polynomial basis
// (Sec. 3.1), the LCH FFT (Alg. 1) evaluates at the points phi(j) of a Cantor
// basis (Sec. 3.3), and every butterfly product is a full GF(2^128) product.
//
// The multipliers of a layer-k butterfly block at offset o are
// s_k(phi(o)) = phi(o >> k) (Sec. 3.3: s_k shifts Cantor coordinates), mapped
// into the field through a table of the basis.  BasisCvt is shared with the
// tower variant (the s_i are the same GF(2) polynomials for both bases), and
// InterleavedCombine needs no change of representation: a 64-bit word is the
// field element of degree < 64 with the same bits, and a product of two of
// them has degree < 127, so it is never reduced.
//
// Products by a field element v use a table of the 16 multiples v * n(x),
// deg n < 4: v * w is the sum over the 32 nibbles of w of table entries times
// x^(4p), accumulated unreduced in 256 bits and reduced once.  A strided FFT
// pass builds one table per distinct multiplier of its group (shared by all
// butterflies of that block); in the contiguous bottom pass each thread holds
// a group of 8 points and builds the table of each block's multiplier once.
#pragma once

#include <stdint.h>

#include <vector>

#include "afft_device.hpp"

namespace gf2x {

constexpr int kSfThreads = 256;       // strided-pass workgroup
constexpr int kSfLaneThreads = 128;   // pointmul workgroups
constexpr int kSfTabL = 7;            // layers of one strided pass, at most
constexpr int kSfTabPtsLog = 10;      // points of one strided-pass workgroup, at most 2^10
constexpr int kSfTabStride = 17;      // uint4 per table: 16 entries and one pad (spreads LDS banks)
constexpr int kSfGroupMaxLog = 3;     // bottom pass: layers 0..G-1 on groups of 2^G points (G = 2 or 3), one per thread
constexpr int kSfGroupSmallLog = 18;  // G = 2 up to N = 2^18 points when that adds no strided pass
constexpr int kCantorBeta = 128;      // beta_0 .. beta_127 in the device table (the whole Cantor basis)
constexpr int kCantorTotal = kCantorBeta + (1 << kSfGroupMaxLog);  // then phi(u) for u < 2^kSfGroupMaxLog

struct SfftPass {
    uint4* x;               // N points, 16 bytes each, read and written in place
    const uint64_t* words;  // non-null: the pass reads word j & wmask as the point j instead of x
    uint64_t wmask;
    uint64_t n;             // N
    int lo, L, c, inverse;  // layers [lo, lo + L); 2^c consecutive low indices per group
    int alpha;              // >= 0: the transform is at alpha = beta_alpha (its points alpha + phi(j)); -1: at 0
};

// ------------------------------------------ bodies (kernels and host checks)


// v * x mod x^128 + x^7 + x^2 + x + 1
AFFT_HD uint4 gcm_mulx(uint4 v) {
    const uint32_t top = v.w >> 31;
    uint4 r;
    r.w = (v.w << 1) | (v.z >> 31);
    r.z = (v.z << 1) | (v.y >> 31);
    r.y = (v.y << 1) | (v.x >> 31);
    r.x = (v.x << 1) ^ (0x87u & (0u - top));
    return r;
}

// T[n S] = v * n(x) for the 16 polynomials n of degree < 4 (bit i of n is the
// coefficient of x^i), walked in Gray-code order so that each entry is the
// previous one plus a single v * x^i.  S = 1: a contiguous table; S =
// kSfLaneTabStride: a per-thread table in the lane-interleaved layout.
template <int S = 1>
AFFT_HD void gcm_build_tab(uint4 v, uint4* T) {
    uint4 b[4];
    b[0] = v;
    b[1] = gcm_mulx(b[0]);
    b[2] = gcm_mulx(b[1]);
    b[3] = gcm_mulx(b[2]);
    uint4 cur = make_uint4(0, 0, 0, 0);
    T[0] = cur;
#pragma unroll
    for (int i = 1; i < 16; ++i) {
        const int flip = __builtin_ctz(i);  // Gray code i ^ (i >> 1) changes this bit
        cur = xor4(cur, b[flip]);
        T[(i ^ (i >> 1)) * S] = cur;
    }
}

// The 256-bit polynomial a[0..7] modulo x^128 + x^7 + x^2 + x + 1: the high
// half H enters as H (x^7 + x^2 + x + 1); the up to 7 bits that this pushes
// past x^127 are folded in the same way once more.
AFFT_HD uint4 gcm_reduce(const uint32_t (&a)[8]) {
    const uint32_t h0 = a[4], h1 = a[5], h2 = a[6], h3 = a[7];
    uint4 r;
    r.x = xor3(xor3(a[0], h0, h0 << 1), h0 << 2, h0 << 7);
    r.y = xor3(xor3(a[1], h1, (h1 << 1) | (h0 >> 31)), (h1 << 2) | (h0 >> 30), (h1 << 7) | (h0 >> 25));
    r.z = xor3(xor3(a[2], h2, (h2 << 1) | (h1 >> 31)), (h2 << 2) | (h1 >> 30), (h2 << 7) | (h1 >> 25));
    r.w = xor3(xor3(a[3], h3, (h3 << 1) | (h2 >> 31)), (h3 << 2) | (h2 >> 30), (h3 << 7) | (h2 >> 25));
    const uint32_t ov = xor3(h3 >> 31, h3 >> 30, h3 >> 25);
    r.x = xor3(xor3(r.x, ov, ov << 1), ov << 2, ov << 7);
    return r;
}

// base + (selected part of v) in one VOP2 add that reads a byte or a 16-bit
// half of its second operand (SDWA): the LDS address of a table entry whose
// byte offset was placed in that part of v beforehand.
#if defined(__HIP_DEVICE_COMPILE__)
typedef const __attribute__((address_space(3))) uint4* gcm_lds_ptr;
#define GCM_ADD_SEL(SEL, r, base, v)                                                                      \
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:" SEL \
        : "=v"(r)                                                                                        \
        : "v"(base), "v"(v))
#endif

// The entry of the contiguous LDS table T at byte offset (byte k of v).
AFFT_HD uint4 gcm_entry(const uint4* T, uint32_t v, int k) {
#if defined(__HIP_DEVICE_COMPILE__)
    const uint32_t base = (uint32_t)(uintptr_t)(gcm_lds_ptr)T;
    uint32_t a;
    switch (k) {
        case 0: GCM_ADD_SEL("BYTE_0", a, base, v); break;
        case 1: GCM_ADD_SEL("BYTE_1", a, base, v); break;
        case 2: GCM_ADD_SEL("BYTE_2", a, base, v); break;
        default: GCM_ADD_SEL("BYTE_3", a, base, v); break;
    }
    return *(gcm_lds_ptr)(uintptr_t)a;
#else
    return T[((v >> (8 * k)) & 255u) >> 4];
#endif
}

// The entry of the lane-interleaved LDS table at T0 at byte offset (16-bit
// half h of v).
AFFT_HD uint4 gcm_entry_lane(const uint4* T0, uint32_t v, int h) {
#if defined(__HIP_DEVICE_COMPILE__)
    const uint32_t base = (uint32_t)(uintptr_t)(gcm_lds_ptr)T0;
    uint32_t a;
    if (h == 0)
        GCM_ADD_SEL("WORD_0", a, base, v);
    else
        GCM_ADD_SEL("WORD_1", a, base, v);
    return *(gcm_lds_ptr)(uintptr_t)a;
#else
    return T0[((v >> (16 * h)) & 0xFFFFu) >> 4];
#endif
}

// v * w from entry(q, r) = T[nibble r of word q of w], T the table of v: sum
// over nibble positions p = 8q + r of T[nibble] x^(32q) x^(4r), by Horner's
// rule in x^4 over r.  The four lookups of one r land on words q .. q + 3 of
// the accumulator; each word takes its (up to four) terms through
// three-input XORs.
template <class E>
AFFT_HD uint4 gcm_horner(const E& entry) {
    uint32_t a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int r = 7; r >= 0; --r) {
        if (r != 7) {
#pragma unroll
            for (int i = 7; i > 0; --i) a[i] = (a[i] << 4) | (a[i - 1] >> 28);
            a[0] <<= 4;
        }
        const uint4 t0 = entry(0, r), t1 = entry(1, r), t2 = entry(2, r), t3 = entry(3, r);
        a[0] ^= t0.x;
        a[1] = xor3(a[1], t0.y, t1.x);
        a[2] = xor3(a[2], t0.z, t1.y) ^ t2.x;
        a[3] = xor3(xor3(a[3], t0.w, t1.z), t2.y, t3.x);
        a[4] = xor3(a[4], t1.w, t2.z) ^ t3.y;
        a[5] = xor3(a[5], t2.w, t3.z);
        a[6] ^= t3.w;
    }
    return gcm_reduce(a);
}

// v * w with T the contiguous table of v (16 entries, 16 B apart).  The
// nibbles of word q are spread once into the bytes of ev[q] (even r) and
// od[q] (odd r), times 16: the byte offsets of the entries.
AFFT_HD uint4 gcm_mul_tab(const uint4* T, uint4 w) {
    const uint32_t ev[4] = {(w.x << 4) & 0xF0F0F0F0u, (w.y << 4) & 0xF0F0F0F0u, (w.z << 4) & 0xF0F0F0F0u,
                            (w.w << 4) & 0xF0F0F0F0u};
    const uint32_t od[4] = {w.x & 0xF0F0F0F0u, w.y & 0xF0F0F0F0u, w.z & 0xF0F0F0F0u, w.w & 0xF0F0F0F0u};
    return gcm_horner([&](int q, int r) __attribute__((always_inline)) {
        return gcm_entry(T, (r & 1) ? od[q] : ev[q], r >> 1);
    });
}

// Per-thread tables in the lane-interleaved layout: the 64 tables of a wave
// take 16 KiB, and entry n of lane t is uint4 (t >> 4) 256 + 16 n + (t mod 16)
// of the region.  A b128 read is served 16 lanes at a time, and entry n of any
// lane t sits in bank group t mod 16 whatever n is, so the random lookups of a
// product never meet in a bank.  T0 is the lane's entry 0.
constexpr int kSfLaneTabStride = 16;  // uint4 from one entry of a lane's table to the next
constexpr int kSfLaneTabWave = 64 * 16;  // uint4 per wave
AFFT_HD uint32_t sf_lane_tab(uint32_t lane) { return (lane >> 4) * 256 + (lane & 15); }

// v * w with T0 the lane-interleaved table of v.  Nibbles r and r + 4 of word
// q sit in the low and high halves of P[r mod 4][q], times 256: the byte
// offsets of the entries.
AFFT_HD uint4 gcm_mul_tab_lane(const uint4* T0, uint4 w) {
    const uint32_t W[4] = {w.x, w.y, w.z, w.w};
    uint32_t P[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        P[0][q] = (W[q] << 8) & 0x0F000F00u;
        P[1][q] = (W[q] << 4) & 0x0F000F00u;
        P[2][q] = W[q] & 0x0F000F00u;
        P[3][q] = (W[q] >> 4) & 0x0F000F00u;
    }
    return gcm_horner([&](int q, int r) __attribute__((always_inline)) {
        return gcm_entry_lane(T0, P[r & 3][q], r >> 2);
    });
}

// phi(v) = sum of beta_t over the set bits t of v (v < 2^64)
AFFT_HD uint4 phi_cantor(uint64_t v, const uint4* beta) {
    uint4 r = make_uint4(0, 0, 0, 0);
    while (v) {
        r = xor4(r, beta[__builtin_ctzll(v)]);
        v &= v - 1;
    }
    return r;
}

// The constant part of a layer-k multiplier of a transform at
// alpha = beta_A: s_k(alpha) = beta_{A-k} (Sec. 3.3: s_k shifts Cantor
// coordinates down by k); zero for a transform at 0.
AFFT_HD uint4 sf_alpha_term(const SfftPass& P, int k, const uint4* beta) {
    return P.alpha >= 0 ? beta[P.alpha - k] : make_uint4(0u, 0u, 0u, 0u);
}

AFFT_HD uint4 sfft_load(const SfftPass& P, uint64_t j) {
    if (P.words) {
        const uint64_t w = P.words[j & P.wmask];
        return make_uint4((uint32_t)w, (uint32_t)(w >> 32), 0u, 0u);
    }
    return P.x[j];
}

// A strided pass: layers [lo, lo + L) on groups of 2^L points 2^lo apart,
// 2^c neighbouring groups per workgroup (c <= lo) so that loads and stores
// run over 2^c consecutive points.  Group g = (hi, lowblk) holds the points
// j = (hi << (lo + L)) | ((e >> c) << lo) | (lowblk << c) | (e mod 2^c),
// e < 2^(L + c).  At relative layer r (layer k = lo + r) the block of e holds
// the rho = L - 1 - r group bits above r, b = e >> (c + r + 1), and its
// multiplier is phi(o >> k) = phi((hi << (rho + 1)) | (b << 1)), kept in
// table 2^rho - 1 + b.
AFFT_HD uint64_t sf_tab_groups(const SfftPass& P) { return P.n >> (P.L + P.c); }

AFFT_HD uint64_t sf_tab_point(const SfftPass& P, uint64_t g, uint32_t e) {
    const uint64_t hi = g >> (P.lo - P.c), lowblk = g & ((1ull << (P.lo - P.c)) - 1);
    return (hi << (P.lo + P.L)) | ((uint64_t)(e >> P.c) << P.lo) | (lowblk << P.c) | (e & ((1u << P.c) - 1));
}

AFFT_HD void sf_tab_table(const SfftPass& P, uint64_t g, uint32_t t, const uint4* beta, uint4* tab) {
    const uint64_t hi = g >> (P.lo - P.c);
    const int rho = 31 - __builtin_clz(t + 1);
    const uint64_t b = t + 1 - (1u << rho);
    const int k = P.lo + P.L - 1 - rho;
    gcm_build_tab(xor4(phi_cantor((hi << (rho + 1)) | (b << 1), beta), sf_alpha_term(P, k, beta)),
                  tab + t * kSfTabStride);
}

// Butterfly q of step s (forward: layers top-down; inverse: bottom-up).
AFFT_HD void sf_tab_bfly(const SfftPass& P, int s, uint32_t q, uint4* dat, const uint4* tab) {
    const int r = P.inverse ? s : P.L - 1 - s;
    const int sh = P.c + r;
    const uint32_t e0 = ((q >> sh) << (sh + 1)) | (q & ((1u << sh) - 1));
    const uint32_t e1 = e0 | (1u << sh);
    const uint4* T = tab + (((1u << (P.L - 1 - r)) - 1) + (e0 >> (sh + 1))) * kSfTabStride;
    uint4 u = dat[e0], w = dat[e1];
    if (!P.inverse) {
        u = xor4(u, gcm_mul_tab(T, w));
        w = xor4(w, u);
    } else {
        w = xor4(w, u);
        u = xor4(u, gcm_mul_tab(T, w));
    }
    dat[e0] = u;
    dat[e1] = w;
}

// Steps s and s + 1 on quad q (two layers per LDS round trip): the points
// whose index bits c + lo and c + hi take all four values, lo < hi the two
// relative layers.  Layer hi pairs (p0, p2) and (p1, p3) within one block
// (one table), layer lo pairs (p0, p1) and (p2, p3) in two blocks; forward
// runs hi then lo, inverse lo then hi, as the single steps do.
// Steps s, s + 1 run as quads when a workgroup of kSfThreads has a quad for
// every thread (groups of at least 1024 points); smaller groups keep single
// steps, which give every thread a butterfly.
AFFT_HD bool sf_tab_quads(const SfftPass& P, int s) {
    return P.L - s >= 2 && (1u << (P.L + P.c)) >= 4u * kSfThreads;
}

AFFT_HD const uint4* sf_tab_of(const SfftPass& P, int r, uint32_t e0, const uint4* tab) {
    return tab + (((1u << (P.L - 1 - r)) - 1) + (e0 >> (P.c + r + 1))) * kSfTabStride;
}

AFFT_HD void sf_tab_quad(const SfftPass& P, int s, uint32_t q, uint4* dat, const uint4* tab) {
    const int lo = P.inverse ? s : P.L - 2 - s, hi = lo + 1;
    const int sl = P.c + lo, sh = P.c + hi;
    const uint32_t q1 = ((q >> sl) << (sl + 1)) | (q & ((1u << sl) - 1));
    const uint32_t p0 = ((q1 >> sh) << (sh + 1)) | (q1 & ((1u << sh) - 1));
    const uint32_t p1 = p0 | (1u << sl), p2 = p0 | (1u << sh), p3 = p1 | (1u << sh);
    const uint4* Th = sf_tab_of(P, hi, p0, tab);
    const uint4* Tl0 = sf_tab_of(P, lo, p0, tab);
    const uint4* Tl1 = sf_tab_of(P, lo, p2, tab);
    uint4 x0 = dat[p0], x1 = dat[p1], x2 = dat[p2], x3 = dat[p3];
    if (!P.inverse) {
        x0 = xor4(x0, gcm_mul_tab(Th, x2));
        x2 = xor4(x2, x0);
        x1 = xor4(x1, gcm_mul_tab(Th, x3));
        x3 = xor4(x3, x1);
        x0 = xor4(x0, gcm_mul_tab(Tl0, x1));
        x1 = xor4(x1, x0);
        x2 = xor4(x2, gcm_mul_tab(Tl1, x3));
        x3 = xor4(x3, x2);
    } else {
        x1 = xor4(x1, x0);
        x0 = xor4(x0, gcm_mul_tab(Tl0, x1));
        x3 = xor4(x3, x2);
        x2 = xor4(x2, gcm_mul_tab(Tl1, x3));
        x2 = xor4(x2, x0);
        x0 = xor4(x0, gcm_mul_tab(Th, x2));
        x3 = xor4(x3, x1);
        x1 = xor4(x1, gcm_mul_tab(Th, x3));
    }
    dat[p0] = x0;
    dat[p1] = x1;
    dat[p2] = x2;
    dat[p3] = x3;
}

// The contiguous bottom pass: layers [0, L) (L <= G, G = 2 or 3) on groups
// of 2^G consecutive points, one group per thread, held in registers.  A wave
// takes a chunk of 64 groups at J0 (a multiple of 2^(G+6)); the layer-k
// multiplier of the block of group g that starts at local point e 2^(k+1) is
// s_k(alpha + phi(J0 + g 2^G + e 2^(k+1)))
//     = beta_{A-k} + phi(J0 >> k) + phi(g << (G - k)) + phi(2e)
// (Sec. 3.3; the index bits of the three phi terms are disjoint).
//
// At the step of layer k register p holds point rotl(p, k + 1) of the group
// (a rotation of G-bit indices), so every layer pairs registers i and i + H
// (H = 2^(G-1), i < H); between steps the points move to register rotl(p, 1)
// (forward, layers top-down) or rotr(p, 1) (inverse, bottom-up).  Pair i lies
// in block e = i mod 2^(G-1-k); visiting the pairs as i = rev(s), the reversal
// of the G - 1 bits of s < H, takes the blocks one after another, so the
// table of each block's multiplier is built once (lane-interleaved) and
// serves its 2^k butterflies.
template <int G>
AFFT_HD constexpr int sf_rev(int s) {
    int r = 0;
    for (int b = 0; b < G - 1; ++b) r |= ((s >> b) & 1) << (G - 2 - b);
    return r;
}

// Keeps a butterfly's results computed where it stands: without it the
// compiler sinks the arithmetic of all products of a step below the last
// table build (the loads stay put), and their table entries spill.
AFFT_HD void sf_pin(uint4& v) {
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" : "+v"(v.x), "+v"(v.y), "+v"(v.z), "+v"(v.w));
#else
    (void)v;
#endif
}

// x[p] -> x[rotl(p, 1)] (forward) or x[rotr(p, 1)] (inverse)
template <int G, bool INV>
AFFT_HD void sf_group_rotate(uint4 (&x)[1 << G]) {
    uint4 y[1 << G];
#pragma unroll
    for (int p = 0; p < (1 << G); ++p) y[INV ? ((p >> 1) | ((p & 1) << (G - 1))) : (((p << 1) | (p >> (G - 1))) & ((1 << G) - 1))] = x[p];
#pragma unroll
    for (int p = 0; p < (1 << G); ++p) x[p] = y[p];
}

// T0: the thread's lane-interleaved table
template <int G, bool INV>
AFFT_HD void sf_group_layers(const SfftPass& P, uint64_t J0, uint32_t g, uint4 (&x)[1 << G], uint4* T0,
                             const uint4* beta) {
    constexpr int H = 1 << (G - 1);
    const uint4* phit = beta + kCantorBeta;  // phi(u), u < 2^G
#pragma unroll
    for (int st = 0; st < G; ++st) {
        const int k = INV ? st : G - 1 - st;
        if (INV) sf_group_rotate<G, true>(x);
        if (k < P.L) {
            uint4 mb = xor4(phi_cantor(J0 >> k, beta), sf_alpha_term(P, k, beta));
#pragma unroll
            for (int b = 0; b < 6; ++b)
                if ((g >> b) & 1) mb = xor4(mb, beta[b + G - k]);
#pragma unroll
            for (int s = 0; s < H; ++s) {
                const int i = sf_rev<G>(s);
                if ((s & ((1 << k) - 1)) == 0)
                    gcm_build_tab<kSfLaneTabStride>(xor4(mb, phit[(i & ((H >> k) - 1)) << 1]), T0);
                uint4 u = x[i], w = x[i + H];
                if (!INV) {
                    u = xor4(u, gcm_mul_tab_lane(T0, w));
                    w = xor4(w, u);
                } else {
                    w = xor4(w, u);
                    u = xor4(u, gcm_mul_tab_lane(T0, w));
                }
                sf_pin(u);
                sf_pin(w);
                x[i] = u;
                x[i + H] = w;
            }
        }
        if (!INV) sf_group_rotate<G, false>(x);
    }
}

// InterleavedCombine, word k: the low half of coefficient k plus the high
// half of coefficient k - 1 (coefficients have degree < 127); the last word
// keeps nc_bits mod 64 bits.
AFFT_HD uint64_t sf_combine_word(const uint4* F, uint64_t n, uint64_t k, uint64_t nwords, uint64_t nc_bits) {
    uint64_t v = 0;
    if (k < n) v = (uint64_t)F[k].x | ((uint64_t)F[k].y << 32);
    if (k >= 1 && k - 1 < n) v ^= (uint64_t)F[k - 1].z | ((uint64_t)F[k - 1].w << 32);
    if (k == nwords - 1 && (nc_bits & 63)) v &= (1ull << (nc_bits & 63)) - 1;
    return v;
}

// ------------------------------------------------------------------- host

using gcm_u128 = unsigned __int128;

inline gcm_u128 gcm_mul_host(gcm_u128 a, gcm_u128 b) {
    gcm_u128 r = 0;
    for (int i = 127; i >= 0; --i) {
        const bool top = (r >> 127) & 1;
        r <<= 1;
        if (top) r ^= 0x87;
        if ((b >> i) & 1) r ^= a;
    }
    return r;
}

// The Cantor basis beta_0 = 1, beta_i^2 + beta_i = beta_{i-1}, each beta_i the
// root without an x^0 term.  y -> y^2 + y is GF(2)-linear with kernel {0, 1};
// its images of x^1 .. x^127 are row-reduced once, then each equation is
// solved by eliminating along the pivots.  False if some equation has no root.
inline bool build_cantor(gcm_u128* beta, int count) {
    struct Row {
        int piv;
        gcm_u128 img, pre;
    };
    std::vector<Row> rows;
    for (int i = 1; i < 128; ++i) {
        const gcm_u128 xi = (gcm_u128)1 << i;
        gcm_u128 img = gcm_mul_host(xi, xi) ^ xi, pre = xi;
        for (const Row& R : rows)
            if ((img >> R.piv) & 1) {
                img ^= R.img;
                pre ^= R.pre;
            }
        if (!img) return false;
        int piv = 127;
        while (!((img >> piv) & 1)) --piv;
        for (Row& R : rows)
            if ((R.img >> piv) & 1) {
                R.img ^= img;
                R.pre ^= pre;
            }
        rows.push_back(Row{piv, img, pre});
    }
    beta[0] = 1;
    for (int i = 1; i < count; ++i) {
        gcm_u128 c = beta[i - 1], y = 0;
        for (const Row& R : rows)
            if ((c >> R.piv) & 1) {
                c ^= R.img;
                y ^= R.pre;
            }
        if (c) return false;
        beta[i] = y;
    }
    return true;
}

// The device table: beta_0 .. beta_127, then phi(u) for u < 2^kSfGroupMaxLog.
inline bool build_cantor_table(std::vector<gcm_u128>& out) {
    out.assign(kCantorTotal, 0);
    if (!build_cantor(out.data(), kCantorBeta)) return false;
    for (uint32_t u = 0; u < (1u << kSfGroupMaxLog); ++u) {
        gcm_u128 r = 0;
        for (int t = 0; t < kSfGroupMaxLog; ++t)
            if ((u >> t) & 1) r ^= out[t];
        out[kCantorBeta + u] = r;
    }
    return true;
}

// The passes of one transform over N = 2^m points: layers [0, M) with
// M = m_op forward (the layers above the operand's converted length 2^m_op
// only copy it: its top half is zero) and M = m inverse.  Bottom pass first
// (groups of 2^G consecutive points, G = 2 or 3 in c, layers
// [0, min(M, G))), then strided passes of at most 7 layers; the forward
// transform runs them in the reverse order, its first pass reading the
// converted words.
inline std::vector<SfftPass> sfft_passes(uint4* x, const uint64_t* words, int m_op, int m, bool inverse,
                                         int alpha = -1) {
    std::vector<SfftPass> v;
    const int M = inverse ? m : m_op;
    // the bottom pass's group size 2^G (in c): groups of 4 for small
    // transforms (twice the threads) unless that adds a strided pass
    const int L2 = M < 2 ? M : 2, L3 = M < 3 ? M : 3;
    const int C = m <= kSfGroupSmallLog && (M - L2 + kSfTabL - 1) / kSfTabL == (M - L3 + kSfTabL - 1) / kSfTabL ? 2 : 3;
    const int Lb = C == 2 ? L2 : L3;
    v.push_back(SfftPass{x, nullptr, 0, 1ull << m, 0, Lb, C, inverse ? 1 : 0, alpha});
    const int up = M - Lb;
    if (up > 0) {
        const int np = (up + kSfTabL - 1) / kSfTabL;
        int lo = Lb;
        for (int p = 0; p < np; ++p) {
            const int L = up / np + (p < up % np ? 1 : 0);
            int c = kSfTabPtsLog - L;
            if (c > lo) c = lo;
            v.push_back(SfftPass{x, nullptr, 0, 1ull << m, lo, L, c, inverse ? 1 : 0, alpha});
            lo += L;
        }
    }
    if (!inverse) {
        std::vector<SfftPass> r(v.rbegin(), v.rend());
        r[0].words = words;
        r[0].wmask = (1ull << m_op) - 1;
        return r;
    }
    return v;
}

}  // namespace gf2x
