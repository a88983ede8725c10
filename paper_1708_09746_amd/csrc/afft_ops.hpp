// Work descriptors ("ops") of the multiplier and their per-tile bodies.
//
// A product is a short list of ops; each op is a set of independent tiles.  A
// GPU kernel runs the tiles of one op with a block-strided loop (tables are
// loaded into LDS once per block); the bodies are __host__ __device__ so the
// same code also runs sequentially on the host.
#pragma once
#include "afft_device.hpp"

namespace gf2x {

constexpr int kThreads = 512;     // threads per block in every kernel
constexpr int kFftTileLog = 11;   // FFT tile: up to 2^11 elements (32 KiB)
constexpr int kFftColRowsLog = 8; // strided passes: up to 2^8 rows per tile
constexpr int kBcTileLog64 = 13;  // BasisCvt tile on 64-bit words: 64 KiB
constexpr int kBcTileLog128 = 12; // BasisCvt tile on 128-bit elements: 64 KiB
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

AFFT_HD void pack_tile(int tid, int nt, uint64_t tile, const PackOp& P) {
    uint64_t nw = (P.nbits + 63) / 64;
    uint64_t mask = (P.nbits % 64) ? (~0ull >> (64 - P.nbits % 64)) : ~0ull;
    for (int e = tid; e < kPackTile; e += nt) {
        uint64_t k = tile * kPackTile + e;
        if (k >= P.ndst) break;
        uint64_t w = 0;
        if (k < nw) {
            w = P.src[k];
            if (k == nw - 1) w &= mask;
        }
        P.dst[k] = w;
    }
}

// --------------------------------------------------------------- BasisCvt
// Layers whose blocks fit in a tile run together in LDS (BcTileOp); a layer
// with larger blocks runs as two global passes (BcLayerOp, which = 0 then 1;
// reversed for the inverse).

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

struct BcTileOp {
    void* data;
    uint64_t nelem;
    uint32_t log_tile;
    uint32_t wide;     // 0: 64-bit words, 1: 128-bit elements
    uint32_t inverse;  // run the layers (and their two parts) in reverse
    uint32_t pad;
    BcLayerList layers;
};

struct BcLayerOp {
    void* data;
    uint64_t nelem;
    uint32_t wide;
    uint32_t which;
    BcLayer layer;
};

AFFT_HD uint64_t bc_tiles(const BcTileOp& B) { return B.nelem >> B.log_tile; }

template <typename T>
AFFT_HD void bc_tile(int tid, int nt, uint64_t tile, const BcTileOp& B, T* lds) {
    T* g = (T*)B.data + (tile << B.log_tile);
    uint32_t ne = 1u << B.log_tile;
    for (uint32_t e = tid; e < ne; e += nt) lds[e] = g[e];
    AFFT_SYNC();
    int n = B.layers.n;
    for (int li = 0; li < n; ++li) {
        const BcLayer& L = B.layers.l[B.inverse ? n - 1 - li : li];
        for (int part = 0; part < 2; ++part) {
            bc_part<T>(tid, nt, lds, ne, L, B.inverse ? 1 - part : part);
            AFFT_SYNC();
        }
    }
    for (uint32_t e = tid; e < ne; e += nt) g[e] = lds[e];
    AFFT_SYNC();
}

// -------------------------------------------------------------- FFT pass
// One pass runs layers [lo, hi) of an in-place LCH FFT (or its inverse) of
// length 2^log_m.  Element index p = (outer << hi) | (row << lo) | col, with
// row in [0, 2^(hi-lo)) and col in [0, 2^lo); a tile holds all rows of
// 2^log_tc consecutive columns.  The forward FFT of an operand converted at
// length 2^log_m evaluates at 2^log_cosets cosets S + V_log_m (S = c << log_m):
// the top layers of the full transform are fan-outs, so each coset is an
// independent FFT whose multipliers use the global block index S | s.
// The block of layer i starting at global index s uses lambda = s_i(s̄) =
// XOR of lam[i][t] over the set bits t of s.  Butterfly (Alg. 1):
//   forward: u += lambda v; v += u        inverse: v += u; u += lambda v.
struct FftPass {
    const void* src;  // phi_in: 64-bit words (2^log_m of them); else == dst
    uint4* dst;       // 2^(log_m + log_cosets) elements
    uint32_t log_m, lo, hi, log_tc;
    uint32_t log_cosets, inverse, phi_in, log_total;
};

AFFT_HD uint64_t fft_tiles(const FftPass& A) {
    return 1ull << (A.log_cosets + (A.log_m - A.hi) + (A.lo - A.log_tc));
}

AFFT_HD int width_mode(int w) { return w <= 8 ? 0 : (w <= 16 ? 1 : 2); }

// changeRepr into the tower (Sec. 4.3): M4R over the 8 bytes of the word
AFFT_HD uint4 phi_word(const uint4* phi_tab, uint64_t w) {
    uint4 r = make_uint4(0, 0, 0, 0);
#pragma unroll
    for (int k = 0; k < 8; ++k) r = r ^ phi_tab[k * 256 + ((w >> (8 * k)) & 255u)];
    return r;
}

AFFT_HD void fft_tile(int tid, int nt, uint64_t tile, const FftPass& A, const uint8_t* mt, const uint32_t* lam,
                      const uint4* phi_tab, uint4* tl, uint4* mu) {
    const uint32_t rlog = A.hi - A.lo, tc = 1u << A.log_tc;
    const uint64_t ncb = 1ull << (A.lo - A.log_tc), nouter = 1ull << (A.log_m - A.hi);
    const uint64_t cb = tile & (ncb - 1);
    const uint64_t rest = tile >> (A.lo - A.log_tc);
    const uint64_t outer = rest & (nouter - 1);
    const uint64_t coset = rest >> (A.log_m - A.hi);
    const uint64_t base_p = (outer << A.hi) | (cb << A.log_tc);
    const uint64_t gbase = coset << A.log_m;
    const uint32_t nel = 1u << (rlog + A.log_tc);

    for (uint32_t e = tid; e < nel; e += nt) {
        uint64_t p = base_p | ((uint64_t)(e >> A.log_tc) << A.lo) | (e & (tc - 1));
        uint4 v;
        if (A.phi_in)
            v = phi_word(phi_tab, ((const uint64_t*)A.src)[p]);
        else
            v = A.dst[gbase | p];
        tl[e] = v;
    }
    // multipliers of every (layer, block) of the tile: entry E <-> layer
    // i = hi - 1 - floor(log2(E + 1)), block b = E + 1 - 2^floor(log2(E + 1))
    const uint32_t nmu = (1u << rlog) - 1;
    const uint64_t s_hi = gbase | (outer << A.hi);
    for (uint32_t E = tid; E < nmu; E += nt) {
        uint32_t q = E + 1;
        int lg = 31 - __builtin_clz(q);
        int i = (int)A.hi - 1 - lg;
        uint64_t s = s_hi | ((uint64_t)(q - (1u << lg)) << (i + 1));
        uint32_t lv = 0;
        for (int t = i + 1; t < 32; ++t)
            if ((s >> t) & 1) lv ^= lam[i * 32 + t];
        mu[E] = make_mu(mt, lv);
    }
    AFFT_SYNC();
    for (uint32_t li = 0; li < rlog; ++li) {
        int i = A.inverse ? (int)(A.lo + li) : (int)(A.hi - 1 - li);
        int h = i - (int)A.lo;
        int mode = width_mode((int)A.log_total - i);
        uint32_t off = (1u << (A.hi - 1 - i)) - 1;
        for (uint32_t w = tid; w < nel / 2; w += nt) {
            uint32_t c = w & (tc - 1);
            uint32_t q = w >> A.log_tc;
            uint32_t blk = q >> h;
            uint32_t r0 = (blk << (h + 1)) | (q & ((1u << h) - 1));
            uint32_t r1 = r0 | (1u << h);
            uint32_t i0 = (r0 << A.log_tc) | c, i1 = (r1 << A.log_tc) | c;
            uint4 u = tl[i0], v = tl[i1];
            uint4 m = mu[off + blk];
            if (!A.inverse) {
                u = u ^ mul_sub(mt, m, v, mode);
                v = v ^ u;
            } else {
                v = v ^ u;
                u = u ^ mul_sub(mt, m, v, mode);
            }
            tl[i0] = u;
            tl[i1] = v;
        }
        AFFT_SYNC();
    }
    for (uint32_t e = tid; e < nel; e += nt) {
        uint64_t p = base_p | ((uint64_t)(e >> A.log_tc) << A.lo) | (e & (tc - 1));
        A.dst[gbase | p] = tl[e];
    }
    AFFT_SYNC();
}

// ------------------------------------------------------------- pointmul
struct PmulOp {
    const uint4* a;
    const uint4* b;
    uint4* c;
    uint64_t n;
};

AFFT_HD uint64_t pmul_tiles(const PmulOp& P) { return (P.n + kPmulTile - 1) / kPmulTile; }

AFFT_HD void pmul_tile(int tid, int nt, uint64_t tile, const PmulOp& P, const uint8_t* mt) {
    for (int e = tid; e < kPmulTile; e += nt) {
        uint64_t j = tile * kPmulTile + e;
        if (j >= P.n) break;
        P.c[j] = gm128(mt, P.a[j], P.b[j]);
    }
}

// --------------------------------------- changeRepr back + InterleavedCombine
// out[k] = lo64(Psi c_k) + hi64(Psi c_{k-1}); c_k = 0 for k >= nspec.
struct PsiOp {
    const uint4* spec;
    uint64_t nspec;
    uint64_t* out;
    uint64_t nwords;
    uint64_t nbits;
};

AFFT_HD uint64_t psi_tiles(const PsiOp& P) { return (P.nwords + kPsiTile - 1) / kPsiTile; }

AFFT_HD uint4 psi_elem(const uint4* psi_tab, const uint4& e) {
    uint4 r = make_uint4(0, 0, 0, 0);
    const uint32_t w[4] = {e.x, e.y, e.z, e.w};
#pragma unroll
    for (int k = 0; k < 16; ++k) r = r ^ psi_tab[k * 256 + ((w[k >> 2] >> (8 * (k & 3))) & 255u)];
    return r;
}

AFFT_HD void psi_tile(int tid, int nt, uint64_t tile, const PsiOp& P, const uint4* psi_tab) {
    for (int e = tid; e < kPsiTile; e += nt) {
        uint64_t k = tile * kPsiTile + e;
        if (k >= P.nwords) break;
        uint64_t w = 0;
        if (k < P.nspec) {
            uint4 r = psi_elem(psi_tab, P.spec[k]);
            w ^= (uint64_t)r.x | ((uint64_t)r.y << 32);
        }
        if (k >= 1 && k - 1 < P.nspec) {
            uint4 r = psi_elem(psi_tab, P.spec[k - 1]);
            w ^= (uint64_t)r.z | ((uint64_t)r.w << 32);
        }
        if (k == P.nwords - 1 && (P.nbits % 64)) w &= ~0ull >> (64 - P.nbits % 64);
        P.out[k] = w;
    }
}

}  // namespace gf2x
