// Work descriptors ("ops") of the multiplier and their per-tile bodies.
//
// A product is a short list of ops; each op is a set of independent tiles.  A
// GPU kernel runs the tiles of one op with a block-strided loop (tables are
// loaded into LDS once per block); the bodies are __host__ __device__ so the
// same code also runs sequentially on the host.
#pragma once
#include "afft_device.hpp"

namespace gf2x {

constexpr int kThreads = 1024;    // threads per block in every kernel
constexpr int kFftTileLog = 12;   // FFT tile: up to 2^12 elements (64 KiB)
constexpr int kFftRL = 2;         // FFT layers per LDS round trip (4 elements per thread)
// Local mu-set tables of an FFT pass (see fft_local_mu): local layer li has
// nb <= kFftTileLog - 1 - li block bits, a table over the low min(nb, 6) of
// them (mu_lo_off) and one over the rest (mu_hi_off), the latter kept twice
// (pass part, pass + tile part); tables packed back to back, sized for 4096-
// point tiles.
static_assert(kFftTileLog == 12, "mu-set table offsets are written for 4096-point tiles");
AFFT_HD int mu_lo_off(int li) { return li <= 5 ? 64 * li : 448 - (1 << (12 - li)); }
AFFT_HD int mu_hi_off(int li) { return li <= 5 ? 64 - (64 >> li) : 57 + li; }
constexpr int kMuLoN = 447, kMuHiN = 69;
constexpr int kMuHiBase = kMuLoN;
constexpr int kMuHiCur = kMuHiBase + kMuHiN;
constexpr int kMuEntries = kMuHiCur + kMuHiN;
// BasisCvt tiles: 64 KiB, or 32 KiB for single products (PlanParams::bc_small),
// whose tile and class passes run on blocks of 512 threads: the layer sweeps
// are bound by their barriers, and four blocks of 512 threads per CU
// interleave them better than two of 1024.  Batches and the serving engine
// keep the 64 KiB tiles: their multi-op and persistent kernels run 1024-thread
// blocks, for which a halved tile only doubles the barriers per element.
constexpr int kBcTileLog64 = 13;  // BasisCvt tile on 64-bit words: 64 KiB
constexpr int kBcTileLog128 = 12; // BasisCvt tile on 128-bit elements: 64 KiB
constexpr int kBcSmallShift = 1;  // a small tile holds half the elements
// single products of at most 2^kBcTinyMaxLog elements: tiles of 1/2^kBcTinyShift
// (more blocks for arrays that fill only a few 32 KiB tiles)
constexpr int kBcTinyShift = 3, kBcTinyMaxLog = 17;
constexpr int kBcThreadsSmall = 512;
constexpr int kPmulTile = 1024;
constexpr int kPsiTile = 1024;
constexpr int kPackTile = 4096;

// ------------------------------------------------------------------ pack
// Split (Alg. 5 first step, w = 64): the operand's words, bits at and above
// nbits cleared, zero-padded to ndst words.
struct PackOp {
    const uint64_t* src;
    uint64_t nbits;
    uint64_t* dst;
    uint64_t ndst;
};

AFFT_HD uint64_t pack_tiles(const PackOp& P) { return (P.ndst + kPackTile - 1) / kPackTile; }

// Word k of an operand of nbits bits: its bits at and above nbits cleared,
// zero past its last word.
AFFT_HD uint64_t operand_word(const uint64_t* src, uint64_t nbits, uint64_t k) {
    const uint64_t nw = (nbits + 63) / 64;
    if (k >= nw) return 0;
    uint64_t w = src[k];
    if (k == nw - 1 && (nbits % 64)) w &= ~0ull >> (64 - nbits % 64);
    return w;
}

AFFT_HD void pack_tile(int tid, int nt, uint64_t tile, const PackOp& P) {
    for (int e = tid; e < kPackTile; e += nt) {
        uint64_t k = tile * kPackTile + e;
        if (k >= P.ndst) break;
        P.dst[k] = operand_word(P.src, P.nbits, k);
    }
}

// Element e of a split operand read in place of its packed copy: the word
// (w = 64) or the two words 2e, 2e + 1 (w = 128).
template <typename T>
AFFT_HD T operand_elem(const void* src, uint64_t nbits, uint64_t e);
template <>
AFFT_HD uint64_t operand_elem<uint64_t>(const void* src, uint64_t nbits, uint64_t e) {
    return operand_word((const uint64_t*)src, nbits, e);
}
template <>
AFFT_HD uint4 operand_elem<uint4>(const void* src, uint64_t nbits, uint64_t e) {
    const uint64_t lo = operand_word((const uint64_t*)src, nbits, 2 * e);
    const uint64_t hi = operand_word((const uint64_t*)src, nbits, 2 * e + 1);
    return make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
}

// --------------------------------------------------------------- BasisCvt
// BasisCvt runs as tile passes: layers whose blocks fit a tile run together
// in LDS (BcTileOp, contiguous or strided "column" tiles), the VarSubs layers
// of a large block run as one class pass (BcClassOp).  A layer that fits
// neither runs as two global passes (BcLayerOp, which = 0 then 1; reversed for
// the inverse).  The first tile op of a forward conversion may read the
// operand itself (src, src_bits; see operand_elem) in place of its packed
// copy, and writes the converted elements to data.

template <typename T>
AFFT_HD T zero_elem();
template <>
AFFT_HD uint64_t zero_elem<uint64_t>() { return 0; }
template <>
AFFT_HD uint4 zero_elem<uint4>() { return make_uint4(0, 0, 0, 0); }

template <typename T>
AFFT_HD void bc_part(int tid, int nt, T* a, uint64_t nelem, const BcLayer& L, int which) {
    // Enumerates (block, t, column) with a power-of-two count; see bc_layer_part.
    uint64_t D = 1ull << L.log_d, k = 1ull << L.log_k;
    uint32_t lu = L.log_u;
    uint32_t log_cnt = which == 0 ? L.log_k : L.log_d;
    uint64_t t0 = which == 0 ? 2 * D - k : D;
    uint64_t tend = which == 0 ? 2 * D : 2 * D - k;
    uint64_t shift = (D - k) << lu;
    uint64_t nblk = nelem >> (L.log_d + 1 + lu);
    uint64_t items = nblk << (log_cnt + lu);
    for (uint64_t w = tid; w < items; w += nt) {
        uint64_t c = w & ((1ull << lu) - 1);
        uint64_t rest = w >> lu;
        uint64_t t = t0 + (rest & ((1ull << log_cnt) - 1));
        if (t >= tend) continue;
        uint64_t b = rest >> log_cnt;
        uint64_t e = (((b << (L.log_d + 1)) + t) << lu) + c;
        a[e - shift] = a[e - shift] ^ a[e];
    }
}

// The same layer part on an LDS tile (32-bit indices).
template <typename T>
AFFT_HD void bc_part_lds(int tid, int nt, T* a, uint32_t nelem, const BcLayer& L, int which) {
    const uint32_t ld = L.log_d, lk = L.log_k, lu = L.log_u;
    const uint32_t D = 1u << ld, k = 1u << lk;
    const uint32_t log_cnt = which == 0 ? lk : ld;
    const uint32_t t0 = which == 0 ? 2 * D - k : D;
    const uint32_t tend = which == 0 ? 2 * D : 2 * D - k;
    const uint32_t shift = (D - k) << lu;
    const uint32_t items = (nelem >> (ld + 1 + lu)) << (log_cnt + lu);
    const uint32_t cm = (1u << lu) - 1, tm = (1u << log_cnt) - 1;
    for (uint32_t w = tid; w < items; w += nt) {
        uint32_t rest = w >> lu;
        uint32_t t = t0 + (rest & tm);
        if (t >= tend) continue;
        uint32_t e = ((((rest >> log_cnt) << (ld + 1)) + t) << lu) + (w & cm);
        a[e - shift] = a[e - shift] ^ a[e];
    }
}

// A tile of 2^log_rows rows, 2^log_stride elements apart, each holding
// 2^log_tc consecutive elements; LDS keeps it row-major ([row][col]).  The
// layer list is in LDS-element units, so a layer on whole rows of a strided
// view ("columns") has its unit scaled by 2^log_tc.  A contiguous tile is
// log_stride = log_tc = 0.
struct BcTileOp {
    void* data;
    uint64_t nelem;
    uint32_t log_rows, log_stride, log_tc;
    uint32_t wide;     // 0: 64-bit words, 1: 128-bit elements
    uint32_t inverse;  // run the layers (and their two parts) in reverse
    uint32_t nlayers;
    const BcLayer* layers;  // nlayers entries (device memory shared by all ops)
    const void* src;        // non-null: gather from the operand (src_bits bits)
    uint64_t src_bits;
};

struct BcLayerOp {
    void* data;
    uint64_t nelem;
    uint32_t wide;
    uint32_t which;
    BcLayer layer;
};

AFFT_HD uint64_t bc_tiles(const BcTileOp& B) { return B.nelem >> (B.log_rows + B.log_tc); }

// Tile geometry: element e of a tile sits at base + off(e).
struct BcTileGeom {
    uint64_t base;  // element index of the tile's first element
    uint32_t ne;    // elements in the tile
};

AFFT_HD BcTileGeom bc_tile_geom(const BcTileOp& B, uint64_t tile) {
    const uint32_t ncb_log = B.log_stride - B.log_tc;
    const uint64_t cb = tile & ((1ull << ncb_log) - 1);
    const uint64_t o = tile >> ncb_log;
    return BcTileGeom{(o << (B.log_rows + B.log_stride)) + (cb << B.log_tc), 1u << (B.log_rows + B.log_tc)};
}

AFFT_HD uint64_t bc_tile_off(const BcTileOp& B, uint32_t e) {
    return ((uint64_t)(e >> B.log_tc) << B.log_stride) + (e & ((1u << B.log_tc) - 1));
}

// The tile's layers on its LDS copy.
template <typename T>
AFFT_HD void bc_tile_layers(int tid, int nt, const BcTileOp& B, uint32_t ne, T* lds) {
    const int n = (int)B.nlayers;
    for (int li = 0; li < n; ++li) {
        const BcLayer L = B.layers[B.inverse ? n - 1 - li : li];
        for (int part = 0; part < 2; ++part) {
            bc_part_lds<T>(tid, nt, lds, ne, L, B.inverse ? 1 - part : part);
            AFFT_SYNC();
        }
    }
}

// One whole tile: gather, layers, scatter (the GPU kernel overlaps the next
// tile's gather with these layers).
template <typename T>
AFFT_HD void bc_tile(int tid, int nt, uint64_t tile, const BcTileOp& B, T* lds) {
    const BcTileGeom G = bc_tile_geom(B, tile);
    T* g = (T*)B.data + G.base;
    if (B.src)
        for (uint32_t e = tid; e < G.ne; e += nt) lds[e] = operand_elem<T>(B.src, B.src_bits, G.base + bc_tile_off(B, e));
    else
        for (uint32_t e = tid; e < G.ne; e += nt) lds[e] = g[bc_tile_off(B, e)];
    AFFT_SYNC();
    bc_tile_layers<T>(tid, nt, B, G.ne, lds);
    for (uint32_t e = tid; e < G.ne; e += nt) g[bc_tile_off(B, e)] = lds[e];
    AFFT_SYNC();
}

// VarSubs (Alg. 2) with y = x^(2^K) + x on blocks of 2^m units of 2^log_u
// elements, all m-K division layers in one pass.  Layer j moves unit t to
// t - 2^j (2^K - 1), so it only combines units in the same residue class
// mod P = 2^K - 1.  Writing t = q P + r, a tile holds the positions
// x = r 2^log_u + c in [x0, x0 + W) of every row q (Q rows cover the block);
// the layer becomes  row[q - 2^j] ^= row[q]  for the rows whose t has
// t mod 2D in the layer's source range.  Q is always just above a power of
// two (2^m / P = 2^(m-K) (1 + 2^-K + ...)), so W is not restricted to powers
// of two: the tile holds Q W elements, close to its capacity; element e of
// the tile is row e / W (exact as (e ceil(2^32 / W)) >> 32 for e < 2^14).
struct BcClassOp {
    void* data;
    uint64_t nelem;
    uint32_t m, K, log_u;
    uint32_t w;       // W positions per tile
    uint32_t q_rows;  // Q = ceil(2^m / P)
    uint32_t wide, inverse, pad;
    uint64_t w_magic;  // ceil(2^32 / W)
};

static_assert(kBcTileLog64 < 14, "class tile rows come from a multiply-shift that is exact below 2^14 elements");
AFFT_HD uint32_t bc_class_row(const BcClassOp& C, uint32_t e) { return (uint32_t)((e * C.w_magic) >> 32); }

AFFT_HD uint64_t bc_class_tiles_per_block(const BcClassOp& C) {
    uint64_t X = ((1ull << C.K) - 1) << C.log_u;
    return (X + C.w - 1) / C.w;
}
AFFT_HD uint64_t bc_class_tiles(const BcClassOp& C) {
    return (C.nelem >> (C.m + C.log_u)) * bc_class_tiles_per_block(C);
}

// Class tile geometry: position (q, xw) of the tile (e = q W + xw) holds
// unit t = q P + ((x0 + xw) >> log_u) of block blk; it is absent (zero in the
// tile, never stored) if x0 + xw >= X or t >= 2^m.
struct BcClassGeom {
    uint64_t base;  // element index of the block's first element
    uint64_t x0;    // first position of the tile
    uint32_t ne;    // Q W
};

AFFT_HD BcClassGeom bc_class_geom(const BcClassOp& C, uint64_t tile) {
    const uint64_t tpb = bc_class_tiles_per_block(C);
    const uint64_t blk = tile / tpb;
    return BcClassGeom{blk << (C.m + C.log_u), (tile - blk * tpb) * C.w, C.q_rows * C.w};
}

// Offset of element e in its block, or ~0 if it is absent.
AFFT_HD uint64_t bc_class_off(const BcClassOp& C, const BcClassGeom& G, uint32_t e) {
    const uint64_t P = (1ull << C.K) - 1, X = P << C.log_u;
    const uint32_t qe = bc_class_row(C, e);
    const uint64_t q = qe, x = G.x0 + (e - qe * C.w);
    if (x >= X || q * P + (x >> C.log_u) >= (1ull << C.m)) return ~0ull;
    return q * X + x;
}

template <typename T>
AFFT_HD void bc_class_layers(int tid, int nt, const BcClassOp& C, const BcClassGeom& G, T* lds) {
    const uint64_t P = (1ull << C.K) - 1;
    const uint64_t X = P << C.log_u;
    const uint64_t nunits = 1ull << C.m;
    const uint32_t ne = G.ne;
    const int nl = (int)(C.m - C.K);
    // Layer j moves unit t to t - (D - k) = t - k P (the same position x of
    // row q - k) for t = 2D-1 down to D in every 2D-unit block.  A target is
    // itself a source only for t in [2D-k, 2D), and its own target then lies
    // below D, so the layer is a set of independent chains t -> t' -> t''
    // and single moves (t in [D+k, 2D-k)): one sweep, each element starting a
    // chain, a single move or nothing, a chain run by one thread in the
    // layer's order (reversed for the inverse).
    for (int li = 0; li < nl; ++li) {
        const int j = C.inverse ? li : nl - 1 - li;
        const uint64_t D = 1ull << (C.K + j), k = 1ull << j;
        const uint32_t rs = (uint32_t)k * C.w;  // k rows
        for (uint32_t e = tid; e < ne; e += nt) {
            const uint32_t qe = bc_class_row(C, e);
            const uint64_t x = G.x0 + (e - qe * C.w);
            if (x >= X) continue;
            const uint64_t t = (uint64_t)qe * P + (x >> C.log_u);
            if (t >= nunits) continue;
            const uint64_t pos = t & (2 * D - 1);
            if (pos >= 2 * D - k) {
                const uint32_t e1 = e - rs, e2 = e1 - rs;
                if (!C.inverse) {
                    const T v = lds[e1] ^ lds[e];
                    lds[e1] = v;
                    lds[e2] = lds[e2] ^ v;
                } else {
                    const T v = lds[e1];
                    lds[e2] = lds[e2] ^ v;
                    lds[e1] = v ^ lds[e];
                }
            } else if (pos >= D + k) {
                lds[e - rs] = lds[e - rs] ^ lds[e];
            }
        }
        AFFT_SYNC();
    }
}

template <typename T>
AFFT_HD void bc_class_tile(int tid, int nt, uint64_t tile, const BcClassOp& C, T* lds) {
    const BcClassGeom G = bc_class_geom(C, tile);
    T* g = (T*)C.data + G.base;
    for (uint32_t e = tid; e < G.ne; e += nt) {
        const uint64_t o = bc_class_off(C, G, e);
        lds[e] = o != ~0ull ? g[o] : zero_elem<T>();
    }
    AFFT_SYNC();
    bc_class_layers<T>(tid, nt, C, G, lds);
    for (uint32_t e = tid; e < G.ne; e += nt) {
        const uint64_t o = bc_class_off(C, G, e);
        if (o != ~0ull) g[o] = lds[e];
    }
    AFFT_SYNC();
}

// -------------------------------------------------------------- FFT pass
// One pass runs layers [lo, hi) of an in-place LCH FFT (or its inverse) of
// length 2^log_m.  Element index p = (outer << hi) | (row << lo) | col, with
// row in [0, 2^(hi-lo)) and col in [0, 2^lo); a tile holds all rows of
// 2^log_tc consecutive columns.  The pass covers the aligned blocks (cosets)
// coset0 .. coset0 + ncosets - 1 of length 2^log_m of the whole transform:
// the forward FFT of an operand converted at length 2^log_m evaluates at the
// cosets S + V_log_m (S = c << log_m), because the top layers of the full
// transform are fan-outs, and a sub-block of a truncated transform is one
// such block.  Each block is an independent FFT whose multipliers use the
// global block index S | s: the block of layer i starting at global index s
// uses lambda = s_i(s̄) = XOR of lam[i][t] over the set bits t of s.
// Butterfly (Alg. 1):
//   forward: u += lambda v; v += u        inverse: v += u; u += lambda v.
// phi_in: 0 the pass reads the spectrum; 1 it reads 64-bit words and applies
// changeRepr into TGF(2^128); 2 / 3 it reads 128-bit words and keeps the low /
// high TGF(2^128) half of their changeRepr into TGF(2^256) (w = 128: the
// spectrum is two planes of halves, each transformed alone, Prop. 2).
//
// A pass may also run a BasisCvt sub-conversion on its tile (bc_n layers in
// tile-element units): the conversion of 2^mb units of 2^q elements (Alg. 3
// on index bits [q, q + mb), the same map for every value of the other
// bits) commutes with every FFT layer at or above q + mb (such a layer acts
// on a higher bit, with a multiplier that depends only on still higher bits),
// with changeRepr (GF(2)-linear on each element), and with the BasisCvt ops
// on disjoint bits that follow it in Alg. 3's recursion.  A forward pass whose
// rows hold those bits runs it on its tile before its layers, an inverse pass
// (its inverse) after them.
enum : uint32_t { kPhiNone = 0, kPhi64 = 1, kPhi128Lo = 2, kPhi128Hi = 3 };
struct FftPass {
    const void* src;  // phi_in: the words (2^log_m of them); else == dst
    uint4* dst;       // the whole transform; blocks are at (coset0 + c) << log_m
    uint32_t log_m, lo, hi, log_tc;
    uint32_t ncosets, coset0, inverse, phi_in;
    uint32_t log_total;  // log2 of the whole transform's length
    uint32_t pack;       // a one-pass transform (lo = 0, hi = log_m): 2^pack cosets per tile
    uint32_t bc_n, pad;
    const BcLayer* bc_layers;
    uint64_t src_bits;   // phi_in with src_bits > 0: src is the operand itself (operand_elem)
};

AFFT_HD uint64_t fft_tiles(const FftPass& A) {
    return (uint64_t)(A.ncosets >> A.pack) << ((A.log_m - A.hi) + (A.lo - A.log_tc));
}

// Row bits of a tile: the layer range, and for a one-pass transform of
// cosets packed 2^pack to a tile, the coset bits above it (the multipliers
// of those rows differ only by their global index, which the row bits carry).
AFFT_HD int fft_row_bits(const FftPass& A) { return (int)(A.hi - A.lo + A.pack); }

// Multiplication mode of a multiplier of at most w bits: 0 GF(256), 1
// TGF(2^16), 3 TGF(2^32) with a high TGF(2^16) half in GF(256) (w <= 24), 2
// the rest of TGF(2^32).
AFFT_HD int width_mode(int w) { return w <= 8 ? 0 : (w <= 16 ? 1 : (w <= 24 ? 3 : 2)); }

// changeRepr into the tower (Sec. 4.3) by M4R over the nibbles of a word:
// the table of a mode holds Phi(v << 4k) (or its half) at 16 k + v.  The
// device table (host-built) is the w = 64 table (16 nibbles, 256 entries)
// followed by the low and high halves of the w = 128 table (32 nibbles, 512
// entries each); a kernel keeps the one slice its pass needs in LDS (at most
// kPhiNib entries, 8 KiB).
constexpr int kPhiNib = 512;
constexpr int kPhinTotal = 256 + 2 * 512;
AFFT_HD int phin_off(uint32_t mode) { return mode <= kPhi64 ? 0 : 256 + 512 * (int)(mode - kPhi128Lo); }
AFFT_HD int phin_len(uint32_t mode) { return mode <= kPhi64 ? 256 : 512; }
// r + a + b componentwise, by three-input XORs
AFFT_HD uint4 xor3_4(const uint4& r, const uint4& a, const uint4& b) {
    return make_uint4(xor3(r.x, a.x, b.x), xor3(r.y, a.y, b.y), xor3(r.z, a.z, b.z), xor3(r.w, a.w, b.w));
}

AFFT_HD uint4 phi_word(const uint4* phin, uint64_t w) {
    uint4 r = make_uint4(0, 0, 0, 0);
#pragma unroll
    for (int k = 0; k < 16; k += 2)
        r = xor3_4(r, phin[k * 16 + ((w >> (4 * k)) & 15u)], phin[(k + 1) * 16 + ((w >> (4 * k + 4)) & 15u)]);
    return r;
}
AFFT_HD uint4 phi_word128(const uint4* phin, const uint4& w) {
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
    uint4 r = make_uint4(0, 0, 0, 0);
#pragma unroll
    for (int k = 0; k < 32; k += 2)
        r = xor3_4(r, phin[k * 16 + ((ws[k >> 3] >> (4 * (k & 7))) & 15u)],
                   phin[(k + 1) * 16 + ((ws[(k + 1) >> 3] >> (4 * ((k + 1) & 7))) & 15u)]);
    return r;
}

// Products by an 8-bit multiplier without table lookups per byte: for each
// lambda in GF(256) three small tables of lambda times the 3-bit groups of a
// byte, T0[y] = lambda y, T1[y] = lambda (y << 3) (y < 8), T2[y] = lambda (y << 6)
// (y < 4), so lambda e = T0[e & 7] + T1[(e >> 3) & 7] + T2[e >> 6]; one
// v_perm_b32 looks up a group of all four bytes of a word at once.  mt3 holds
// the three tables of every lambda (3 uint2 per lambda, 6 KiB).
AFFT_HD void build_mt3(int tid, int nt, const uint8_t* mt, uint2* mt3) {
    for (int l = tid; l < 256; l += nt) {
        const uint8_t* row = mt + (l << 8);
        uint32_t t[5] = {0, 0, 0, 0, 0};
        for (int y = 0; y < 8; ++y) {
            t[y >> 2] |= (uint32_t)row[y] << (8 * (y & 3));
            t[2 + (y >> 2)] |= (uint32_t)row[y << 3] << (8 * (y & 3));
        }
        for (int y = 0; y < 4; ++y) t[4] |= (uint32_t)row[y << 6] << (8 * y);
        mt3[3 * l] = make_uint2(t[0], t[1]);
        mt3[3 * l + 1] = make_uint2(t[2], t[3]);
        mt3[3 * l + 2] = make_uint2(t[4], 0);
    }
}

AFFT_HD uint32_t mul_word8_t(const uint2& t0, const uint2& t1, uint32_t t2, uint32_t a) {
    return xor3(perm32(t0.y, t0.x, a & 0x07070707u), perm32(t1.y, t1.x, (a >> 3) & 0x07070707u),
                perm32(0u, t2, (a >> 6) & 0x03030303u));
}

AFFT_HD uint4 mul_sub8_t(const uint2* mt3, uint32_t lam8, const uint4& v) {
    const uint2 t0 = mt3[3 * lam8], t1 = mt3[3 * lam8 + 1];
    const uint32_t t2 = mt3[3 * lam8 + 2].x;
    return make_uint4(mul_word8_t(t0, t1, t2, v.x), mul_word8_t(t0, t1, t2, v.y), mul_word8_t(t0, t1, t2, v.z),
                      mul_word8_t(t0, t1, t2, v.w));
}

// mu-set of local layer li for block row bits b (b < 2^(rlog - li - 1))
AFFT_HD uint4 fft_mu(const uint4* mu, int li, uint32_t b) {
    return xor4(mu[mu_lo_off(li) + (int)(b & 63u)], mu[kMuHiCur + mu_hi_off(li) + (int)(b >> 6)]);
}

// One step of RL consecutive layers [i0, i0 + RL) held in registers: a thread
// owns the 2^RL elements whose rows differ only in the bits (i0 - lo) ..
// (i0 - lo + RL - 1) (same column) and runs all their butterflies.
template <int RL, bool INV>
AFFT_HD void fft_step(int tid, int nt, const FftPass& A, int i0, const uint8_t* mt, const uint2* mt3, uint4* tl,
                      const uint4* mu) {
    const uint32_t nel = 1u << (A.hi - A.lo + A.pack + A.log_tc);
    const uint32_t groups = nel >> RL;
    const uint32_t tcm = (1u << A.log_tc) - 1;
    const int h0 = i0 - (int)A.lo;
    for (uint32_t g = tid; g < groups; g += nt) {
        uint32_t c = g & tcm;
        uint32_t rr = g >> A.log_tc;
        uint32_t base_r = ((rr >> h0) << (h0 + RL)) | (rr & ((1u << h0) - 1));
        uint4 x[1 << RL];
#pragma unroll
        for (int j = 0; j < (1 << RL); ++j) x[j] = tl[((base_r | ((uint32_t)j << h0)) << A.log_tc) | c];
#pragma unroll
        for (int s = 0; s < RL; ++s) {
            const int l = INV ? s : RL - 1 - s;  // layer i0 + l
            const int i = i0 + l;
            const int li = i - (int)A.lo;
            const int mode = width_mode((int)A.log_total - i);
#pragma unroll
            for (int j = 0; j < (1 << RL); ++j) {
                if (j & (1 << l)) continue;
                uint32_t r0 = base_r | ((uint32_t)j << h0);
                uint4 m = fft_mu(mu, li, r0 >> (li + 1));
                uint4 u = x[j], v = x[j | (1 << l)];
                if (!INV) {
                    u = u ^ (mode == 0 ? mul_sub8_t(mt3, m.w & 255u, v) : mul_sub_k(mt, m, v, mode));
                    v = v ^ u;
                } else {
                    v = v ^ u;
                    u = u ^ (mode == 0 ? mul_sub8_t(mt3, m.w & 255u, v) : mul_sub_k(mt, m, v, mode));
                }
                x[j] = u;
                x[j | (1 << l)] = v;
            }
        }
#pragma unroll
        for (int j = 0; j < (1 << RL); ++j) tl[((base_r | ((uint32_t)j << h0)) << A.log_tc) | c] = x[j];
    }
}

// The multiplier of layer i for the block starting at global index s is
// lambda = s_i(s̄) = XOR of lam[i][t] over the set bits t of s.  Inside a tile,
// s = S | (b << (i + 1)) with S the tile's bits at and above `hi` and b the
// block's row bits (nb = hi - i - 1 of them), and the mu-set of lambda is
// GF(2)-linear in lambda, so
//   mu(lambda) = mu(s_i(S̄)) + mu(s_i(low 6 bits of b)) + mu(s_i(high bits of b))
// (each s_i of its bits of b placed at their positions in s).  The middle term
// is table lo[li][b & 63], the others table hi[li][b >> 6]: its pass part is
// the same for every tile of the pass (written here), and each tile adds its
// own tile part (fft_tile_layers).  li = i - lo is the local layer.
AFFT_HD void fft_local_mu(int tid, int nt, const FftPass& A, const uint8_t* mt, const uint32_t* lam, uint4* mu) {
    const int nlay = (int)(A.hi - A.lo), rlog = fft_row_bits(A);
    for (int E = tid; E < kMuLoN + kMuHiN; E += nt) {
        const bool hi = E >= kMuLoN;
        const int F = hi ? E - kMuLoN : E;
        int li = 0;
        while (li + 1 < kFftTileLog && (hi ? mu_hi_off(li + 1) : mu_lo_off(li + 1)) <= F) ++li;
        const uint32_t x = (uint32_t)(F - (hi ? mu_hi_off(li) : mu_lo_off(li)));
        if (li >= nlay) continue;
        const int nb = rlog - li - 1;
        const int lob = nb < 6 ? nb : 6;
        if (x >= (1u << (hi ? nb - lob : lob))) continue;
        const int i = (int)A.lo + li;
        const int t0 = i + 1 + (hi ? 6 : 0);
        uint32_t lv = 0;
        for (uint32_t q = x; q; q &= q - 1) lv ^= lam[i * 32 + t0 + __builtin_ctz(q)];
        mu[hi ? kMuHiBase + F : F] = make_mu_k(mt, lv);
    }
}

struct FftTileGeom {
    uint64_t base_p, gbase, s_hi;
    uint32_t nel;
};

AFFT_HD FftTileGeom fft_geom(const FftPass& A, uint64_t tile) {
    const uint64_t ncb = 1ull << (A.lo - A.log_tc), nouter = 1ull << (A.log_m - A.hi);
    const uint64_t cb = tile & (ncb - 1);
    const uint64_t rest = tile >> (A.lo - A.log_tc);
    const uint64_t outer = rest & (nouter - 1);
    const uint64_t coset = (rest >> (A.log_m - A.hi)) << A.pack;
    FftTileGeom G;
    G.base_p = (outer << A.hi) | (cb << A.log_tc);
    G.gbase = ((uint64_t)A.coset0 + coset) << A.log_m;
    G.s_hi = G.gbase | (outer << A.hi);
    G.nel = 1u << (A.hi - A.lo + A.pack + A.log_tc);
    return G;
}

AFFT_HD uint64_t fft_elem_index(const FftPass& A, const FftTileGeom& G, uint32_t e) {
    return G.base_p | ((uint64_t)(e >> A.log_tc) << A.lo) | (e & ((1u << A.log_tc) - 1));
}

// Tile element e: in a pass that applies changeRepr, (the kept half of) Phi
// of its converted word (fft_word, fft_word128), else the element of the
// spectrum (fft_spec).  phin is the table of the pass's mode.
AFFT_HD uint64_t fft_word(const FftPass& A, const FftTileGeom& G, uint32_t e) {
    const uint64_t k = fft_elem_index(A, G, e) & ((1ull << A.log_m) - 1);
    return A.src_bits ? operand_elem<uint64_t>(A.src, A.src_bits, k) : ((const uint64_t*)A.src)[k];
}
AFFT_HD uint4 fft_word128(const FftPass& A, const FftTileGeom& G, uint32_t e) {
    const uint64_t k = fft_elem_index(A, G, e) & ((1ull << A.log_m) - 1);
    return A.src_bits ? operand_elem<uint4>(A.src, A.src_bits, k) : ((const uint4*)A.src)[k];
}
AFFT_HD uint4 fft_spec(const FftPass& A, const FftTileGeom& G, uint32_t e) {
    return A.dst[G.gbase | fft_elem_index(A, G, e)];
}
AFFT_HD uint4 fft_load(const FftPass& A, const uint4* phin, const FftTileGeom& G, uint32_t e) {
    if (A.phi_in == kPhi64) return phi_word(phin, fft_word(A, G, e));
    if (A.phi_in >= kPhi128Lo) return phi_word128(phin, fft_word128(A, G, e));
    return fft_spec(A, G, e);
}

// The BasisCvt layers fused into a pass, on its tile (nel elements), in the
// direction of the pass; every thread's tile writes are visible at the end.
AFFT_HD void fft_tile_bc(int tid, int nt, const FftPass& A, uint32_t nel, uint4* tl) {
    const int n = (int)A.bc_n;
    for (int li = 0; li < n; ++li) {
        const BcLayer L = A.bc_layers[A.inverse ? n - 1 - li : li];
        for (int part = 0; part < 2; ++part) {
            bc_part_lds<uint4>(tid, nt, tl, nel, L, A.inverse ? 1 - part : part);
            AFFT_SYNC();
        }
    }
}

// Layers [lo, hi) of one tile already in LDS (tl); mu holds the pass's local
// mu-set tables (fft_local_mu), completed here with the tile part of every
// layer (mu_tile, up to 32 entries).  RL: layers kept in registers per LDS
// round trip.  A fused BasisCvt (bc_n > 0) runs first (forward) or last
// (inverse).
template <int RL>
AFFT_HD void fft_tile_layers(int tid, int nt, const FftPass& A, const FftTileGeom& G, const uint8_t* mt,
                             const uint2* mt3, const uint32_t* lam, uint4* tl, uint4* mu, uint4* mu_tile) {
    const int rlog = (int)(A.hi - A.lo), rbits = fft_row_bits(A);
    for (int li = tid; li < rlog; li += nt) {
        int i = (int)A.lo + li;
        uint32_t lv = 0;
        for (uint64_t sb = G.s_hi >> A.hi; sb; sb &= sb - 1) lv ^= lam[i * 32 + (int)A.hi + __builtin_ctzll(sb)];
        mu_tile[li] = make_mu_k(mt, lv);
    }
    AFFT_SYNC();
    // high tables of this tile: pass part + tile part
    for (int E = tid; E < kMuHiN; E += nt) {
        int li = 0;
        while (li + 1 < kFftTileLog && mu_hi_off(li + 1) <= E) ++li;
        const int y = E - mu_hi_off(li), nb = rbits - li - 1;
        if (li < rlog && y < (1 << (nb > 6 ? nb - 6 : 0))) mu[kMuHiCur + E] = xor4(mu[kMuHiBase + E], mu_tile[li]);
    }
    AFFT_SYNC();
    const uint32_t nel = 1u << (A.hi - A.lo + A.pack + A.log_tc);
    if (A.bc_n && !A.inverse) fft_tile_bc(tid, nt, A, nel, tl);
    // A step of R layers from local layer h0 gives thread g the rows of group
    // g; with contiguous rows (log_tc = 0), one group per thread and
    // h0 <= 6, the 64 threads of a wave then own exactly the 64 2^R rows from
    // 64 2^R w on, so between two such steps of equal R the exchange stays
    // inside each wave: a wave-level sync replaces the workgroup barrier.
    auto wave_owned = [&](int d, int& Rd) {
        const int r = rlog - d;
        Rd = r >= RL ? RL : r;
        const int i0 = A.inverse ? (int)A.lo + d : (int)A.hi - d - Rd;
        return A.log_tc == 0 && (nel >> Rd) <= (uint32_t)nt && i0 - (int)A.lo <= 6;
    };
    int done = 0;
    while (done < rlog) {
        int r = rlog - done;
        int R = r >= RL ? RL : r;
        int i0 = A.inverse ? (int)A.lo + done : (int)A.hi - done - R;
        if (A.inverse) {
            if (R == 3)
                fft_step<3, true>(tid, nt, A, i0, mt, mt3, tl, mu);
            else if (R == 2)
                fft_step<2, true>(tid, nt, A, i0, mt, mt3, tl, mu);
            else
                fft_step<1, true>(tid, nt, A, i0, mt, mt3, tl, mu);
        } else {
            if (R == 3)
                fft_step<3, false>(tid, nt, A, i0, mt, mt3, tl, mu);
            else if (R == 2)
                fft_step<2, false>(tid, nt, A, i0, mt, mt3, tl, mu);
            else
                fft_step<1, false>(tid, nt, A, i0, mt, mt3, tl, mu);
        }
        int Rc = 0, Rn = 0;
        const bool here = wave_owned(done, Rc);
        done += R;
        if (done < rlog && here && wave_owned(done, Rn) && Rn == Rc)
            AFFT_WAVE_SYNC();
        else
            AFFT_SYNC();
    }
    if (A.bc_n && A.inverse) fft_tile_bc(tid, nt, A, nel, tl);
}

// One whole tile: load, layers, store (the sequential form; the GPU kernel
// overlaps the next tile's loads with these layers).
template <int RL>
AFFT_HD void fft_tile(int tid, int nt, uint64_t tile, const FftPass& A, const uint8_t* mt, const uint2* mt3,
                      const uint32_t* lam, const uint4* phin, uint4* tl, uint4* mu, uint4* mu_tile) {
    FftTileGeom G = fft_geom(A, tile);
    for (uint32_t e = tid; e < G.nel; e += nt) tl[e] = fft_load(A, phin, G, e);
    fft_tile_layers<RL>(tid, nt, A, G, mt, mt3, lam, tl, mu, mu_tile);
    for (uint32_t e = tid; e < G.nel; e += nt) A.dst[G.gbase | fft_elem_index(A, G, e)] = tl[e];
    AFFT_SYNC();
}

// ------------------------------------------------------- truncated transforms
// Element-wise steps of a truncated transform (evaluation at the first M
// points only, and its inverse), all with one multiplier lambda per op:
//   kSpineHalf:  x += lambda y            (half butterfly)
//   kSpineAdd:   y += x
//   kSpineFwd:   x += lambda y; y += x    (forward butterfly)
//   kSpineInv:   y += x; x += lambda y    (inverse butterfly)
//   kSpineZero:  x = 0
//   kSpinePhi:   x = changeRepr(words)    (the coefficients of one coset)
// over x[p], y[p] for p < n.
enum : uint32_t { kSpineHalf = 0, kSpineAdd = 1, kSpineFwd = 2, kSpineInv = 3, kSpineZero = 4, kSpinePhi = 5 };
constexpr int kSpineTile = 4096;

struct SpineOp {
    uint4* x;
    uint4* y;
    const uint64_t* words;  // kSpinePhi
    uint64_t n;
    uint4 mu;               // mu-set of lambda (make_mu_k)
    uint32_t mode, width;   // width: width_mode of lambda
    uint32_t pad0, pad1;
};

AFFT_HD uint64_t spine_tiles(const SpineOp& S) { return (S.n + kSpineTile - 1) / kSpineTile; }

AFFT_HD void spine_tile(int tid, int nt, uint64_t tile, const SpineOp& S, const uint8_t* mt, const uint4* phin) {
    for (int e = tid; e < kSpineTile; e += nt) {
        const uint64_t p = tile * kSpineTile + e;
        if (p >= S.n) break;
        switch (S.mode) {
            case kSpineHalf: S.x[p] = xor4(S.x[p], mul_sub_k(mt, S.mu, S.y[p], (int)S.width)); break;
            case kSpineAdd: S.y[p] = xor4(S.y[p], S.x[p]); break;
            case kSpineFwd: {
                const uint4 u = xor4(S.x[p], mul_sub_k(mt, S.mu, S.y[p], (int)S.width));
                S.x[p] = u;
                S.y[p] = xor4(S.y[p], u);
                break;
            }
            case kSpineInv: {
                const uint4 v = xor4(S.y[p], S.x[p]);
                S.y[p] = v;
                S.x[p] = xor4(S.x[p], mul_sub_k(mt, S.mu, v, (int)S.width));
                break;
            }
            case kSpineZero: S.x[p] = make_uint4(0, 0, 0, 0); break;
            default: S.x[p] = phi_word(phin, S.words[p]); break;
        }
    }
}

// ------------------------------------------------------------- pointmul
// c_j = a_j b_j for j < n; c_j = 0 for n <= j < n_out (the coefficients a
// truncated inverse starts from).
// w = 128 (ah != nullptr): the points are TGF(2^256) elements held as two
// planes (a, ah), (b, bh) -> (c, ch) of low and high halves.
struct PmulOp {
    const uint4* a;
    const uint4* b;
    uint4* c;
    uint64_t n;
    uint64_t n_out;
    const uint4* ah;
    const uint4* bh;
    uint4* ch;
};

AFFT_HD uint64_t pmul_tiles(const PmulOp& P) { return (P.n_out + kPmulTile - 1) / kPmulTile; }

// ctab: the constant-multiple tables (kConstTabWords words)
AFFT_HD void pmul_tile(int tid, int nt, uint64_t tile, const PmulOp& P, const uint8_t* mt, const uint32_t* ctab) {
    // multiplication by c16 of every byte of a word (register tables)
    const uint2 t0 = make_uint2(ctab[kC16Tab], ctab[kC16Tab + 1]), t1 = make_uint2(ctab[kC16Tab + 2], ctab[kC16Tab + 3]);
    const uint32_t t2 = ctab[kC16Tab + 4];
    auto c16x = [&](const uint4& v) {
        return make_uint4(mul_word8_t(t0, t1, t2, v.x), mul_word8_t(t0, t1, t2, v.y), mul_word8_t(t0, t1, t2, v.z),
                          mul_word8_t(t0, t1, t2, v.w));
    };
    for (int e = tid; e < kPmulTile; e += nt) {
        uint64_t j = tile * kPmulTile + e;
        if (j >= P.n_out) break;
        if (P.ah) {
            uint4 c0 = make_uint4(0, 0, 0, 0), c1 = c0;
            if (j < P.n) {
                const uint4 a0 = P.a[j], a1 = P.ah[j];
                gm256_t(mt, ctab, a0, a1, c16x(a0), c16x(a1), P.b[j], P.bh[j], c0, c1);
            }
            P.c[j] = c0;
            P.ch[j] = c1;
        } else if (j < P.n) {
            const uint4 a = P.a[j];
            P.c[j] = gm128_t(mt, ctab, a, c16x(a), P.b[j]);
        } else {
            P.c[j] = make_uint4(0, 0, 0, 0);
        }
    }
}

// --------------------------------------- changeRepr back + InterleavedCombine
// w = 64:  out[k] = lo64(Psi c_k) + hi64(Psi c_{k-1}); c_k = 0 for k >= nspec.
// w = 128 (spech != nullptr, c_k = (spec[k], spech[k]) in TGF(2^256)): the
// 128-bit output word K (64-bit words 2K, 2K + 1) is
// lo128(Psi c_K) + hi128(Psi c_{K-1}).
// The device table of Psi: the w = 64 byte-indexed table (16 x 256 entries)
// followed by the w = 128 nibble-indexed one, low half then high half (each
// 64 nibbles x 16 entries).
struct PsiOp {
    const uint4* spec;
    uint64_t nspec;
    uint64_t* out;
    uint64_t nwords;
    uint64_t nbits;
    const uint4* spech;
};
constexpr int kPsiTab64 = 16 * 256, kPsiTab128 = 2 * 64 * 16;
AFFT_HD int psi_tab_off(const PsiOp& P) { return P.spech ? kPsiTab64 : 0; }
AFFT_HD int psi_tab_len(const PsiOp& P) { return P.spech ? kPsiTab128 : kPsiTab64; }

// 64-bit output words per tile: one per thread (w = 64) or two (w = 128)
AFFT_HD uint64_t psi_tile_words(const PsiOp& P) { return P.spech ? 2 * kPsiTile : kPsiTile; }
AFFT_HD uint64_t psi_tiles(const PsiOp& P) { return (P.nwords + psi_tile_words(P) - 1) / psi_tile_words(P); }

// One half of Psi of a TGF(2^256) element (c0, c1) by M4R over its 64
// nibbles; tab: that half's table.
AFFT_HD uint4 psi_half(const uint4* tab, const uint4& c0, const uint4& c1) {
    const uint32_t w[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
    uint4 r = make_uint4(0, 0, 0, 0);
#pragma unroll
    for (int k = 0; k < 64; k += 2)
        r = xor3_4(r, tab[k * 16 + ((w[k >> 3] >> (4 * (k & 7))) & 15u)],
                   tab[(k + 1) * 16 + ((w[(k + 1) >> 3] >> (4 * ((k + 1) & 7))) & 15u)]);
    return r;
}

// One 64-bit half (half 0: bits 0..63, half 1: bits 64..127) of Psi of a
// TGF(2^128) element: only that half of every table entry is read.
AFFT_HD uint64_t psi_half64(const uint4* psi_tab, const uint4& e, int half) {
    const uint2* t2 = (const uint2*)psi_tab;
    uint32_t lo = 0, hi = 0;
    const uint32_t w[4] = {e.x, e.y, e.z, e.w};
#pragma unroll
    for (int k = 0; k < 16; k += 2) {
        const uint2 v = t2[2 * (k * 256 + ((w[k >> 2] >> (8 * (k & 3))) & 255u)) + half];
        const uint2 u = t2[2 * ((k + 1) * 256 + ((w[(k + 1) >> 2] >> (8 * ((k + 1) & 3))) & 255u)) + half];
        lo = xor3(lo, v.x, u.x);
        hi = xor3(hi, v.y, u.y);
    }
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// psi_tab: the table of the op's width (psi_tab_off into the device table)
AFFT_HD void psi_tile(int tid, int nt, uint64_t tile, const PsiOp& P, const uint4* psi_tab) {
    if (P.spech) {
        for (int e = tid; e < kPsiTile; e += nt) {
            const uint64_t K = tile * kPsiTile + e, k0 = 2 * K;
            if (k0 >= P.nwords) break;
            uint4 r = make_uint4(0, 0, 0, 0);
            if (K < P.nspec) r = r ^ psi_half(psi_tab, P.spec[K], P.spech[K]);
            if (K >= 1 && K - 1 < P.nspec) r = r ^ psi_half(psi_tab + 64 * 16, P.spec[K - 1], P.spech[K - 1]);
            uint64_t w0 = (uint64_t)r.x | ((uint64_t)r.y << 32), w1 = (uint64_t)r.z | ((uint64_t)r.w << 32);
            const uint64_t tail = P.nbits % 64 ? ~0ull >> (64 - P.nbits % 64) : ~0ull;
            if (k0 == P.nwords - 1) w0 &= tail;
            P.out[k0] = w0;
            if (k0 + 1 < P.nwords) {
                if (k0 + 1 == P.nwords - 1) w1 &= tail;
                P.out[k0 + 1] = w1;
            }
        }
        return;
    }
    for (int e = tid; e < kPsiTile; e += nt) {
        uint64_t k = tile * kPsiTile + e;
        if (k >= P.nwords) break;
        uint64_t w = 0;
        if (k < P.nspec) w ^= psi_half64(psi_tab, P.spec[k], 0);
        if (k >= 1 && k - 1 < P.nspec) w ^= psi_half64(psi_tab, P.spec[k - 1], 1);
        if (k == P.nwords - 1 && (P.nbits % 64)) w &= ~0ull >> (64 - P.nbits % 64);
        P.out[k] = w;
    }
}

// ------------------------------------------------ block to tile (XCD aware)
// The chip dispatches the blocks of a launch to its eight XCDs round robin
// (block b to XCD b mod 8), and each XCD has an L2 of its own.  Neighbouring
// tiles of a strided pass share cache lines, so a block-strided loop (tile
// b, b + grid, ...) would fetch every such line into several L2s.  Within
// each full round of `grid` tiles, xcd_tile hands the blocks of one XCD a
// contiguous run of grid/8 tiles; a partial last round, or a grid that is
// not a multiple of 8, keeps the identity.  A bijection on [0, ntiles).
constexpr uint32_t kXcds = 8;
AFFT_HD uint64_t xcd_tile(uint64_t t, uint64_t grid, uint64_t ntiles) {
    if (grid % kXcds) return t;
    const uint64_t round = t / grid, r = t - round * grid;
    if ((round + 1) * grid > ntiles) return t;
    return round * grid + (r % kXcds) * (grid / kXcds) + r / kXcds;
}

// ------------------------------------------------------- op arrays (batches)
// prefix[o] is the first tile of op o and prefix[nops] the total; op_of_tile
// returns the op holding tile g, walking forward from `hint` (tiles are
// visited in increasing order) or searching when hint < 0.
AFFT_HD int op_of_tile(const uint64_t* prefix, int nops, uint64_t g, int hint) {
    if (hint < 0) {
        int lo = 0, hi = nops - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= g)
                lo = mid;
            else
                hi = mid - 1;
        }
        return lo;
    }
    while (hint + 1 < nops && prefix[hint + 1] <= g) ++hint;
    return hint;
}

}  // namespace gf2x
