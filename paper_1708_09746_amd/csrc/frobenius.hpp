// The Frobenius-partition variant of the multiplier (App. C): no Kronecker
// segmentation.  A polynomial of GF(2)[x] with fewer than 128 n coefficients
// (n = 2^m points) is represented by its values at the n points
// beta_{m+64} + V_m of GF(2^128), in the field and Cantor basis of the simple
// variant (simple.hpp).  The Frobenius orbits of these points are disjoint and
// hold 128 points each, so the map is a bijection (App. C, the partition of
// the evaluation points), and a product c = a b with deg c < 128 n is
// recovered from the n pointwise products of the two value vectors.
//
// Forward, per operand (App. C, the truncated FFT and its encoding):
//   1. Split into 64-bit words, zero-padded to 2^W words;
//   2. BasisCvt (Alg. 3) over the bits, factored through the words: with
//      z = s_6(x) = x^64 + x^16 + x^4 + x, the novel basis satisfies
//      X_{64q+r}(x) = X_r(x) X_q(z) (because s_{6+j} = s_j o s_6), so the
//      conversion is (a) the z-adic expansion a = sum_q H_q(x) z^q with
//      deg H_q < 64, (b) BasisCvt of the word sequence (H_q) (the word-level
//      kernels of the tower variant), (c) inside each word, h -> g with
//      sum_r g_r X_r(x) = h(x), a fixed 64 x 64 GF(2) map;
//   3. the encoding: the first seven layers of FFT_LCH at alpha = beta_{m+64}
//      over 2^(m+7) points, keeping the first 2^m outputs.  Coefficient j n + i
//      enters element i with weight P_j = product over the set bits t of j of
//      s_{m+t}(alpha) = beta_{64-t} (Sec. 3.3's shift rule), so element
//      i = sum_{j<128} g_{jn+i} P_j: a 128 x n bit transpose and a 128 x 128
//      GF(2) map per element;
//   4. FFT_LCH (Alg. 1) at alpha over the n elements: the simple variant's
//      passes with every block multiplier s_k(alpha + phi(o)) =
//      beta_{m+64-k} + phi(o >> k).
// The product takes pointmul in GF(2^128), iFFT_LCH at alpha, the inverse of
// the encoding, the inverse per-word map, iBasisCvt of the word sequence and
// the z-adic recomposition c = sum_q H_q z^q.
#pragma once

#include <stdint.h>

#include <vector>

#include "afft_device.hpp"
#include "afft_ops.hpp"
#include "simple.hpp"

namespace gf2x {

// ------------------------------------------------------------ z-adic levels
// A polynomial of 128 d bits (d = 2^j) is q z^(2^j) + r with q and r of 64 d
// bits each.  Squaring is additive, so z^(2^j) = x^(64d) + x^(16d) + x^(4d) +
// x^d, and therefore
//   high half h = q + (q >> 48d) + (q >> 60d) + (q >> 63d),
//   low half  l = r + (q << 16d) + (q << 4d) + (q << d)  (mod x^(64d)),
// where >> drops the bits moved below 0.  The map q -> h is an involution
// (two of its shifts add up to more than 64 d), so one level sets, in place,
// q = h + (h >> 48d) + (h >> 60d) + (h >> 63d) and then
// r = l + (q << 16d) + (q << 4d) + (q << d).  The expansion runs the levels
// from the top (j = W - 1: the halves of the whole 2^W-word array) down to
// j = 0 (one word per half); digit H_q is then word q.  The recomposition runs
// them bottom up, each inverted: the low half first, then the involution.
//
// At a level j >= 6 every shift is a multiple of U = 2^(j-6) words, and the
// level only mixes words of one residue class modulo U: a class of one
// 2^(j+1)-word block is 128 rows (words U apart), with high-half row moves by
// 48, 60, 63 and low-half moves by 16, 4, 1.  A pass runs the levels
// [j_lo, j_hi] of tiles of 2^log_rows rows (2^log_stride words apart, with
// 2^log_stride = 2^(j_lo-6) the class modulus of the lowest level) by 2^log_tc
// adjacent classes; level j then moves rows by multiples of 2^(j - j_lo).
// The contiguous pass (log_stride = 0, rows are words) also runs the levels
// below 6, where the shifts are bit shifts inside blocks of at most 64 words.
constexpr int kZTileLog = 12;        // words per tile: 4096 (32 KiB)
constexpr int kZThreads = 512;       // threads per block
constexpr int kZLevelsPerPass = 3;   // levels of one strided pass, at most

struct ZadicPass {
    uint64_t* data;         // 2^log_words words, in place
    uint64_t* out;          // non-null: the pass stores word k < out_words to out[k] instead of data[k]
    uint64_t out_words;
    uint32_t log_words;     // W
    int32_t j_lo, j_hi;     // levels run (none if j_hi < j_lo)
    uint32_t log_rows, log_stride, log_tc;
    uint32_t inverse;       // 0: expansion (levels top down), 1: recomposition (bottom up)
};

AFFT_HD uint64_t zadic_tiles(const ZadicPass& Z) { return 1ull << (Z.log_words - Z.log_rows - Z.log_tc); }

// word index of tile element e (row e >> log_tc, column e mod 2^log_tc)
AFFT_HD uint64_t zadic_word(const ZadicPass& Z, uint64_t tile, uint32_t e) {
    const uint32_t cgl = Z.log_stride - Z.log_tc;
    const uint64_t base = ((tile >> cgl) << (Z.log_rows + Z.log_stride)) | ((tile & ((1ull << cgl) - 1)) << Z.log_tc);
    return base + ((uint64_t)(e >> Z.log_tc) << Z.log_stride) + (e & ((1u << Z.log_tc) - 1));
}

// the 64 bits of the hw-word array h starting at bit p (zero outside it)
AFFT_HD uint64_t zbits(const uint64_t* h, int64_t hw, int64_t p) {
    const int64_t w = p >> 6;  // floor, also for p < 0
    const uint32_t s = (uint32_t)(p & 63);
    const uint64_t a = (w >= 0 && w < hw) ? h[w] : 0;
    if (!s) return a;
    const uint64_t b = (w + 1 >= 0 && w + 1 < hw) ? h[w + 1] : 0;
    return (a >> s) | (b << (64 - s));
}

// Level j >= 6 on the tile: rows move by multiples of U = 2^lu rows.  The
// high step writes only rows t < 16U of a high half and reads rows >= 48U, and
// the low step writes the low half and reads the high half, so each step is
// free of races without a barrier inside it.
AFFT_HD void zadic_word_level(uint32_t tid, uint32_t nt, const ZadicPass& Z, int j, uint64_t* lds, bool inv) {
    const uint32_t lu = (uint32_t)j - 6 - Z.log_stride, ltc = Z.log_tc;
    const uint32_t U = 1u << lu, cm = (1u << ltc) - 1;
    const uint32_t nblk = 1u << (Z.log_rows - lu - 7);
    for (int step = 0; step < 2; ++step) {
        const bool high = (step == 0) != inv;
        if (high) {
            const uint32_t items = (nblk << (lu + 4)) << ltc;  // rows t < 16U of each high half
            for (uint32_t it = tid; it < items; it += nt) {
                const uint32_t c = it & cm, r = it >> ltc;
                const uint32_t t = r & ((16u << lu) - 1);
                const uint32_t h0 = ((r >> (lu + 4)) << (lu + 7)) + (64u << lu);
                uint64_t v = lds[((h0 + t + 48 * U) << ltc) | c];
                if (t < 4 * U) v ^= lds[((h0 + t + 60 * U) << ltc) | c];
                if (t < U) v ^= lds[((h0 + t + 63 * U) << ltc) | c];
                lds[((h0 + t) << ltc) | c] ^= v;
            }
        } else {
            const uint32_t items = (nblk << (lu + 6)) << ltc;  // every row of each low half
            for (uint32_t it = tid; it < items; it += nt) {
                const uint32_t c = it & cm, r = it >> ltc;
                const uint32_t t = r & ((64u << lu) - 1);
                const uint32_t l0 = (r >> (lu + 6)) << (lu + 7), h0 = l0 + (64u << lu);
                uint64_t v = 0;
                if (t >= 16 * U) v ^= lds[((h0 + t - 16 * U) << ltc) | c];
                if (t >= 4 * U) v ^= lds[((h0 + t - 4 * U) << ltc) | c];
                if (t >= U) v ^= lds[((h0 + t - U) << ltc) | c];
                lds[((l0 + t) << ltc) | c] ^= v;
            }
        }
        AFFT_SYNC();
    }
}

// Level j < 6 of the contiguous pass (rows are words): halves of hw = 2^j
// words, shifts of d = 2^j bits, inside blocks of at most 64 words.  The high
// step changes only the words that hold bits below 16d (the first
// max(1, hw/4)) and reads words holding bits at or above 48d, which it never
// changes; the low step writes the low half and reads the high half.
AFFT_HD void zadic_bit_level(uint32_t tid, uint32_t nt, const ZadicPass& Z, int j, uint64_t* lds, bool inv) {
    const int64_t hw = 1ll << j, d = 1ll << j;
    const uint32_t nblk = 1u << (Z.log_rows - j - 1);
    const uint32_t nchg = hw >= 4 ? (uint32_t)(hw / 4) : 1u;
    for (int step = 0; step < 2; ++step) {
        const bool high = (step == 0) != inv;
        if (high) {
            for (uint32_t it = tid; it < nblk * nchg; it += nt) {
                const uint32_t b = it / nchg, t = it % nchg;
                uint64_t* h = lds + ((uint64_t)b << (j + 1)) + hw;
                const int64_t p = 64 * (int64_t)t;
                h[t] ^= zbits(h, hw, p + 48 * d) ^ zbits(h, hw, p + 60 * d) ^ zbits(h, hw, p + 63 * d);
            }
        } else {
            for (uint32_t it = tid; it < (nblk << j); it += nt) {
                const uint32_t b = it >> j, t = it & ((1u << j) - 1);
                uint64_t* l = lds + ((uint64_t)b << (j + 1));
                const uint64_t* h = l + hw;
                const int64_t p = 64 * (int64_t)t;
                l[t] ^= zbits(h, hw, p - 16 * d) ^ zbits(h, hw, p - 4 * d) ^ zbits(h, hw, p - d);
            }
        }
        AFFT_SYNC();
    }
}

AFFT_HD void zadic_tile(uint32_t tid, uint32_t nt, uint64_t tile, const ZadicPass& Z, uint64_t* lds) {
    const uint32_t ne = 1u << (Z.log_rows + Z.log_tc);
    for (uint32_t e = tid; e < ne; e += nt) lds[e] = Z.data[zadic_word(Z, tile, e)];
    AFFT_SYNC();
    if (!Z.inverse) {
        for (int j = Z.j_hi; j >= Z.j_lo; --j) {
            if (j >= 6)
                zadic_word_level(tid, nt, Z, j, lds, false);
            else
                zadic_bit_level(tid, nt, Z, j, lds, false);
        }
    } else {
        for (int j = Z.j_lo; j <= Z.j_hi; ++j) {
            if (j >= 6)
                zadic_word_level(tid, nt, Z, j, lds, true);
            else
                zadic_bit_level(tid, nt, Z, j, lds, true);
        }
    }
    for (uint32_t e = tid; e < ne; e += nt) {
        const uint64_t k = zadic_word(Z, tile, e);
        if (Z.out) {
            if (k < Z.out_words) Z.out[k] = lds[e];
        } else {
            Z.data[k] = lds[e];
        }
    }
    AFFT_SYNC();
}

// The passes of the expansion (inverse = 0) or the recomposition of 2^W
// words: one contiguous pass for the levels below min(W, kZTileLog), and
// strided passes of at most kZLevelsPerPass levels above it (top down for the
// expansion, bottom up for the recomposition).  `out`: the recomposition's
// last pass stores its first out_words words there.
inline std::vector<ZadicPass> zadic_passes(uint64_t* data, int W, bool inverse, uint64_t* out = nullptr,
                                           uint64_t out_words = 0) {
    std::vector<ZadicPass> v;
    const int T = W < kZTileLog ? W : kZTileLog;
    ZadicPass c{};
    c.data = data;
    c.log_words = (uint32_t)W;
    c.j_lo = 0;
    c.j_hi = T - 1;
    c.log_rows = (uint32_t)T;
    c.log_stride = 0;
    c.log_tc = 0;
    c.inverse = inverse ? 1 : 0;
    v.push_back(c);
    const int up = W - T;  // levels T .. W - 1
    if (up > 0) {
        const int np = (up + kZLevelsPerPass - 1) / kZLevelsPerPass;
        int lo = T;
        for (int p = 0; p < np; ++p) {
            const int L = up / np + (p < up % np ? 1 : 0);
            ZadicPass s{};
            s.data = data;
            s.log_words = (uint32_t)W;
            s.j_lo = lo;
            s.j_hi = lo + L - 1;
            s.log_rows = (uint32_t)(L + 6);
            s.log_stride = (uint32_t)(lo - 6);
            s.log_tc = (uint32_t)(kZTileLog - (L + 6));
            s.inverse = inverse ? 1 : 0;
            v.push_back(s);
            lo += L;
        }
    }
    if (!inverse) {
        std::vector<ZadicPass> r(v.rbegin(), v.rend());
        return r;
    }
    v.back().out = out;
    v.back().out_words = out_words;
    return v;
}

// ----------------------------------------------------- per-word conversion
// Inside a 64-bit word h (a polynomial of degree < 64) the conversion is
// g with sum_r g_r X_r(x) = h(x); both directions are GF(2)-linear maps of the
// word, applied through 16 tables of 16 words (one per nibble of the input).
constexpr int kWordTab = 16 * 16;

AFFT_HD uint64_t word_map(const uint64_t* tab, uint64_t v) {
    uint64_t r = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) r ^= tab[(q << 4) | ((v >> (4 * q)) & 15u)];
    return r;
}

// ------------------------------------------------------ encoding, decoding
// Element i of the encoding takes bit j n + i of the converted bits for every
// j < 128: the 128 x n bit matrix (row j = bits j n .. j n + n - 1) read by
// columns.  For n >= 64 a row is 2^(m-6) words; a tile covers G consecutive
// groups of 64 columns (G words of every row, staged through LDS so that
// global loads and stores run along rows), and one wave turns the 128 words
// of a group into the 64 columns by two 64 x 64 bit transposes done with
// lane exchanges (six stages each).  The 128 bits of a column enter the
// 128 x 128 map E(b) = sum_j b_j P_j through 32 tables of 16 elements (one per
// nibble of the column); decoding applies the inverse map the same way, then
// the transposes back.  For n < 64 one tile holds the whole array (at most 64
// words) and each column is gathered bit by bit.
constexpr int kFeGroupsLog = 4;  // groups of 64 elements per tile: 16 (1024 elements)
constexpr int kFeThreads = 1024;
constexpr int kFeRowPad = (1 << kFeGroupsLog) + 1;  // words per staged row
constexpr int kElemTab = 32 * 16;                    // entries of an element-map table (uint4)
// device table image of the variant, in uint4 units: the encoding map, its
// inverse, then the per-word forward and inverse conversions (64-bit entries)
constexpr int kFrobEncOff = 0, kFrobDecOff = kElemTab, kFrobWordOff = 2 * kElemTab;
constexpr int kFrobTabU4 = 2 * kElemTab + kWordTab;  // two word tables = kWordTab uint4
constexpr int kFeStage = 128 * kFeRowPad;            // staged words of a tile

struct FrobEncode {
    const uint64_t* words;  // 2^log_words words of the word-level conversion (before the per-word map)
    uint4* spec;            // n = 2^m elements
    uint32_t log_words, m;
};

struct FrobDecode {
    const uint4* spec;  // n = 2^m elements
    uint64_t* words;    // 2^(m+1) words out (after the inverse per-word map)
    uint32_t m;
};

AFFT_HD uint64_t frob_tiles(uint32_t m) { return m >= 6 + kFeGroupsLog ? 1ull << (m - 6 - kFeGroupsLog) : 1ull; }
AFFT_HD uint32_t frob_groups(uint32_t m) { return m >= 6 + kFeGroupsLog ? 1u << kFeGroupsLog : 1u << (m - 6); }

AFFT_HD uint4 elem_map(const uint4* tab, uint64_t lo, uint64_t hi) {
    uint4 r = make_uint4(0, 0, 0, 0);
#pragma unroll
    for (int q = 0; q < 16; q += 2)
        r = xor3_4(r, tab[(q << 4) | ((lo >> (4 * q)) & 15u)], tab[((q + 1) << 4) | ((lo >> (4 * q + 4)) & 15u)]);
#pragma unroll
    for (int q = 0; q < 16; q += 2)
        r = xor3_4(r, tab[((16 + q) << 4) | ((hi >> (4 * q)) & 15u)],
                   tab[((17 + q) << 4) | ((hi >> (4 * q + 4)) & 15u)]);
    return r;
}

// The 64 x 64 bit transpose of a matrix whose row r is the word v[r]: on
// return v[c] holds column c (bit r of v[c] = bit c of the old v[r]).  Stage
// s pairs rows r and r + s (bit s of r clear) and swaps the s x s blocks off
// the diagonal: row r keeps its bits i with bit s of i clear and takes those
// of row r + s, moved up by s; row r + s keeps the others and takes row r's,
// moved down by s.
AFFT_HD uint64_t tr_mask(int s) {
    return s == 32 ? 0x00000000FFFFFFFFull
         : s == 16 ? 0x0000FFFF0000FFFFull
         : s == 8  ? 0x00FF00FF00FF00FFull
         : s == 4  ? 0x0F0F0F0F0F0F0F0Full
         : s == 2  ? 0x3333333333333333ull
                   : 0x5555555555555555ull;
}

AFFT_HD void transpose64_host(uint64_t* v) {
    for (int s = 32; s >= 1; s >>= 1) {
        const uint64_t M = tr_mask(s);
        for (int r = 0; r < 64; ++r) {
            if (r & s) continue;
            const uint64_t a = v[r], b = v[r + s];
            v[r] = (a & M) | ((b & M) << s);
            v[r + s] = (b & ~M) | ((a >> s) & M);
        }
    }
}

#if defined(__HIP_DEVICE_COMPILE__)
// The same transpose across the lanes of a wave: lane r holds row r on
// entry and column r on return.  A lane needs half of its partner's bits per
// stage; for s = 32 that half is one 32-bit word, otherwise two.
__device__ __forceinline__ uint64_t transpose64_wave(uint64_t v) {
    const uint32_t lane = threadIdx.x & 63u;
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
        const uint64_t M = tr_mask(s);
        const bool up = (lane & (uint32_t)s) != 0;
        // what the partner needs from this lane, in the place it goes
        const uint64_t send = up ? (v & M) : ((v >> s) & M);
        uint64_t got;
        if (s == 32) {
            got = (uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)send, 32);
        } else {
            const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)send, s);
            const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(send >> 32), s);
            got = ((uint64_t)hi << 32) | lo;
        }
        v = up ? ((v & ~M) | got) : ((v & M) | (got << s));
    }
    return v;
}
#endif

// the encoding of one tile; lds holds the staged rows (128 rows of
// kFeRowPad words, or the whole array of at most 64 words when n < 64)
AFFT_HD void frob_encode_tile(uint32_t tid, uint32_t nt, uint64_t tile, const FrobEncode& F, const uint4* etab,
                              const uint64_t* wtab, uint64_t* lds) {
    const uint64_t nw = 1ull << F.log_words;
    if (F.m < 6) {
        const uint32_t n = 1u << F.m, tw = 2u << F.m;  // the 128 n bits are 2n words
        for (uint32_t k = tid; k < tw; k += nt) lds[k] = k < nw ? word_map(wtab, F.words[k]) : 0;
        AFFT_SYNC();
        for (uint32_t i = tid; i < n; i += nt) {
            uint64_t lo = 0, hi = 0;
            for (uint32_t j = 0; j < 128; ++j) {
                const uint32_t p = j * n + i;
                const uint64_t bit = (lds[p >> 6] >> (p & 63)) & 1;
                if (j < 64)
                    lo |= bit << j;
                else
                    hi |= bit << (j - 64);
            }
            F.spec[i] = elem_map(etab, lo, hi);
        }
        AFFT_SYNC();
        return;
    }
    const uint32_t G = frob_groups(F.m);
    const uint64_t rw = 1ull << (F.m - 6);  // words per row
    const uint64_t w0 = tile * G;
    // rows in, along the rows: the per-word map on the way
    for (uint32_t it = tid; it < 128 * G; it += nt) {
        const uint32_t j = it / G, c = it % G;
        const uint64_t k = j * rw + w0 + c;
        lds[j * kFeRowPad + c] = k < nw ? word_map(wtab, F.words[k]) : 0;
    }
    AFFT_SYNC();
#if defined(__HIP_DEVICE_COMPILE__)
    {
        const uint32_t lane = tid & 63u, wave = tid >> 6, nwaves = nt >> 6;
        for (uint32_t c = wave; c < G; c += nwaves) {
            const uint64_t lo = transpose64_wave(lds[lane * kFeRowPad + c]);
            const uint64_t hi = transpose64_wave(lds[(64 + lane) * kFeRowPad + c]);
            F.spec[((w0 + c) << 6) + lane] = elem_map(etab, lo, hi);
        }
    }
#else
    for (uint32_t c = 0; c < G; ++c) {
        uint64_t lo[64], hi[64];
        for (int r = 0; r < 64; ++r) {
            lo[r] = lds[r * kFeRowPad + c];
            hi[r] = lds[(64 + r) * kFeRowPad + c];
        }
        transpose64_host(lo);
        transpose64_host(hi);
        for (int l = 0; l < 64; ++l) F.spec[((w0 + c) << 6) + l] = elem_map(etab, lo[l], hi[l]);
    }
#endif
    AFFT_SYNC();
}

// the decoding of one tile; lds stages the tile's rows (as the encoding)
AFFT_HD void frob_decode_tile(uint32_t tid, uint32_t nt, uint64_t tile, const FrobDecode& F, const uint4* dtab,
                              const uint64_t* wtab, uint64_t* lds) {
    if (F.m < 6) {
        const uint32_t n = 1u << F.m, tw = 2u << F.m;
        for (uint32_t i = tid; i < n; i += nt) {
            const uint4 e = F.spec[i];
            const uint4 b = elem_map(dtab, (uint64_t)e.x | ((uint64_t)e.y << 32), (uint64_t)e.z | ((uint64_t)e.w << 32));
            lds[2 * i] = (uint64_t)b.x | ((uint64_t)b.y << 32);
            lds[2 * i + 1] = (uint64_t)b.z | ((uint64_t)b.w << 32);
        }
        AFFT_SYNC();
        for (uint32_t k = tid; k < tw; k += nt) {
            uint64_t v = 0;
            for (uint32_t b = 0; b < 64; ++b) {
                const uint32_t p = 64 * k + b, j = p >> F.m, i = p & (n - 1);
                v |= ((lds[2 * i + (j >> 6)] >> (j & 63)) & 1) << b;
            }
            F.words[k] = word_map(wtab, v);
        }
        AFFT_SYNC();
        return;
    }
    const uint32_t G = frob_groups(F.m);
    const uint64_t rw = 1ull << (F.m - 6);
    const uint64_t w0 = tile * G;
#if defined(__HIP_DEVICE_COMPILE__)
    {
        const uint32_t lane = tid & 63u, wave = tid >> 6, nwaves = nt >> 6;
        for (uint32_t c = wave; c < G; c += nwaves) {
            const uint4 x = F.spec[((w0 + c) << 6) + lane];
            const uint4 b =
                elem_map(dtab, (uint64_t)x.x | ((uint64_t)x.y << 32), (uint64_t)x.z | ((uint64_t)x.w << 32));
            const uint64_t lo = transpose64_wave((uint64_t)b.x | ((uint64_t)b.y << 32));
            const uint64_t hi = transpose64_wave((uint64_t)b.z | ((uint64_t)b.w << 32));
            lds[lane * kFeRowPad + c] = word_map(wtab, lo);
            lds[(64 + lane) * kFeRowPad + c] = word_map(wtab, hi);
        }
    }
#else
    for (uint32_t c = 0; c < G; ++c) {
        uint64_t lo[64], hi[64];
        for (int l = 0; l < 64; ++l) {
            const uint4 x = F.spec[((w0 + c) << 6) + l];
            const uint4 b =
                elem_map(dtab, (uint64_t)x.x | ((uint64_t)x.y << 32), (uint64_t)x.z | ((uint64_t)x.w << 32));
            lo[l] = (uint64_t)b.x | ((uint64_t)b.y << 32);
            hi[l] = (uint64_t)b.z | ((uint64_t)b.w << 32);
        }
        transpose64_host(lo);
        transpose64_host(hi);
        for (int r = 0; r < 64; ++r) {
            lds[r * kFeRowPad + c] = word_map(wtab, lo[r]);
            lds[(64 + r) * kFeRowPad + c] = word_map(wtab, hi[r]);
        }
    }
#endif
    AFFT_SYNC();
    for (uint32_t it = tid; it < 128 * G; it += nt) {
        const uint32_t j = it / G, c = it % G;
        F.words[j * rw + w0 + c] = lds[j * kFeRowPad + c];
    }
    AFFT_SYNC();
}

// ------------------------------------------------------------------- host

struct FrobSizes {
    uint64_t na_bits, nb_bits, nc_bits, out_words;
    int m;          // n = 2^m points: the least with 128 n >= na + nb - 1
    int w_a, w_b;   // operand words, padded: 2^w_a, 2^w_b
};

inline int frob_ceil_log2(uint64_t v) {
    int r = 0;
    while ((1ull << r) < v) ++r;
    return r;
}

inline FrobSizes frob_sizes(uint64_t na, uint64_t nb) {
    FrobSizes s{};
    s.na_bits = na;
    s.nb_bits = nb;
    if (!na || !nb) return s;
    s.nc_bits = na + nb - 1;
    s.out_words = (s.nc_bits + 63) / 64;
    s.m = frob_ceil_log2((s.nc_bits + 127) / 128);
    s.w_a = frob_ceil_log2((na + 63) / 64);
    s.w_b = frob_ceil_log2((nb + 63) / 64);
    return s;
}

struct FrobWorkspace {
    size_t off_wa, off_wb, off_sa, off_sb, bytes;
};

inline FrobWorkspace frob_workspace(const FrobSizes& s) {
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    FrobWorkspace w{};
    size_t o = 0;
    w.off_wa = o;
    o = al(o + (8ull << s.w_a));
    w.off_wb = o;
    o = al(o + (8ull << s.w_b));
    w.off_sa = o;  // after the pointwise product: the decoded 2^(m+1) words
    o = al(o + (16ull << s.m));
    w.off_sb = o;
    o = al(o + (16ull << s.m));
    w.bytes = o;
    return w;
}

// X_r(x) for r < 64 as 64-bit polynomials: the product of s_i(x) over the set
// bits i of r, with s_0 = x and s_{i+1} = s_i^2 + s_i.
inline void frob_novel_words(uint64_t X[64]) {
    auto clmul_lo = [](uint64_t a, uint64_t b) {
        uint64_t r = 0;
        for (int i = 0; i < 64; ++i)
            if ((b >> i) & 1) r ^= a << i;
        return r;
    };
    uint64_t s[6];
    s[0] = 2;  // x
    for (int i = 1; i < 6; ++i) s[i] = clmul_lo(s[i - 1], s[i - 1]) ^ s[i - 1];
    for (int r = 0; r < 64; ++r) {
        uint64_t p = 1;
        for (int i = 0; i < 6; ++i)
            if ((r >> i) & 1) p = clmul_lo(p, s[i]);
        X[r] = p;
    }
}

// The device tables: encoding map, decoding map (each 32 x 16 elements), the
// per-word conversion and its inverse (each 16 x 16 words).  False if the
// encoding products are dependent (they are not; checked here).
inline bool build_frob_tables(const gcm_u128* beta, std::vector<gcm_u128>& enc, std::vector<gcm_u128>& dec,
                              std::vector<uint64_t>& wfwd, std::vector<uint64_t>& winv) {
    // P_j = product of beta_{64-t} over the set bits t of j
    gcm_u128 P[128];
    for (int j = 0; j < 128; ++j) {
        gcm_u128 p = 1;
        for (int t = 0; t < 7; ++t)
            if ((j >> t) & 1) p = gcm_mul_host(p, beta[64 - t]);
        P[j] = p;
    }
    // invert E(b) = sum_j b_j P_j: Gauss-Jordan on the rows (P_j | e_j)
    gcm_u128 rowv[128], rowc[128];
    for (int j = 0; j < 128; ++j) {
        rowv[j] = P[j];
        rowc[j] = (gcm_u128)1 << j;
    }
    gcm_u128 inv[128];  // inv[bit] = the b with E(b) = x^bit
    for (int bit = 127, r = 0; bit >= 0; --bit, ++r) {
        int piv = -1;
        for (int k = r; k < 128; ++k)
            if ((rowv[k] >> bit) & 1) {
                piv = k;
                break;
            }
        if (piv < 0) return false;
        std::swap(rowv[r], rowv[piv]);
        std::swap(rowc[r], rowc[piv]);
        for (int k = 0; k < 128; ++k)
            if (k != r && ((rowv[k] >> bit) & 1)) {
                rowv[k] ^= rowv[r];
                rowc[k] ^= rowc[r];
            }
    }
    for (int r = 0; r < 128; ++r) {
        int bit = 127;
        while (!((rowv[r] >> bit) & 1)) --bit;
        inv[bit] = rowc[r];
    }
    enc.assign(kElemTab, 0);
    dec.assign(kElemTab, 0);
    for (int q = 0; q < 32; ++q)
        for (int v = 0; v < 16; ++v) {
            gcm_u128 e = 0, d = 0;
            for (int t = 0; t < 4; ++t)
                if ((v >> t) & 1) {
                    e ^= P[4 * q + t];
                    d ^= inv[4 * q + t];
                }
            enc[(q << 4) | v] = e;
            dec[(q << 4) | v] = d;
        }
    // per-word conversion: column e (the image of x^e) by the triangular solve
    // with the X_r, whose leading term is x^r
    uint64_t X[64], col[64];
    frob_novel_words(X);
    for (int e = 0; e < 64; ++e) {
        uint64_t h = 1ull << e, g = 0;
        for (int r = 63; r >= 0; --r)
            if ((h >> r) & 1) {
                g |= 1ull << r;
                h ^= X[r];
            }
        col[e] = g;
    }
    wfwd.assign(kWordTab, 0);
    winv.assign(kWordTab, 0);
    for (int q = 0; q < 16; ++q)
        for (int v = 0; v < 16; ++v) {
            uint64_t f = 0, i = 0;
            for (int t = 0; t < 4; ++t)
                if ((v >> t) & 1) {
                    f ^= col[4 * q + t];
                    i ^= X[4 * q + t];
                }
            wfwd[(q << 4) | v] = f;
            winv[(q << 4) | v] = i;
        }
    return true;
}

}  // namespace gf2x
