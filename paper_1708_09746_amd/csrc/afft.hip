// GPU executor and C ABI of the additive-FFT GF(2)[x] multiplier (gfx950).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <ctime>
#include <deque>
#include <mutex>
#include <thread>
#include <type_traits>
#include <string>
#include <vector>

#include "../../include/gf2x_afft.h"
#include "afft_plan.hpp"
#include "arena.hpp"
#include "frobenius.hpp"
#include "simple.hpp"
#include "tower_host.hpp"

using namespace gf2x;

// ------------------------------------------------------------------ kernels

__global__ __launch_bounds__(kThreads) void k_pack(PackOp P) {
    const uint64_t nt = pack_tiles(P);
    for (uint64_t t = blockIdx.x; t < nt; t += gridDim.x) pack_tile(threadIdx.x, blockDim.x, t, P);
}

// SMALL: a 32 KiB tile (single products) on a 512-thread block, else a 64 KiB
// tile on a 1024-thread block
template <int WIDE, int SMALL>
__global__ __launch_bounds__(SMALL ? kBcThreadsSmall : kThreads) void k_bc_tile(BcTileOp B) {
    __shared__ uint4 lds[(1 << kBcTileLog128) >> (SMALL ? kBcSmallShift : 0)];
    const uint64_t nt = bc_tiles(B);
    for (uint64_t t = blockIdx.x; t < nt; t += gridDim.x) {
        const uint64_t tile = xcd_tile(t, gridDim.x, nt);
        if (WIDE)
            bc_tile<uint4>(threadIdx.x, blockDim.x, tile, B, lds);
        else
            bc_tile<uint64_t>(threadIdx.x, blockDim.x, tile, B, (uint64_t*)lds);
    }
}

template <int WIDE, int SMALL>
__global__ __launch_bounds__(SMALL ? kBcThreadsSmall : kThreads) void k_bc_class(BcClassOp C) {
    __shared__ uint4 lds[(1 << kBcTileLog128) >> (SMALL ? kBcSmallShift : 0)];
    const uint64_t nt = bc_class_tiles(C);
    for (uint64_t t = blockIdx.x; t < nt; t += gridDim.x) {
        const uint64_t tile = xcd_tile(t, gridDim.x, nt);
        if (WIDE)
            bc_class_tile<uint4>(threadIdx.x, blockDim.x, tile, C, lds);
        else
            bc_class_tile<uint64_t>(threadIdx.x, blockDim.x, tile, C, (uint64_t*)lds);
    }
}

template <int WIDE>
__global__ __launch_bounds__(kThreads) void k_bc_layer(BcLayerOp L) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nt = gridDim.x * blockDim.x;
    if (WIDE)
        bc_part<uint4>(tid, nt, (uint4*)L.data, L.nelem, L.layer, (int)L.which);
    else
        bc_part<uint64_t>(tid, nt, (uint64_t*)L.data, L.nelem, L.layer, (int)L.which);
}

// Tiles of one FFT pass, block-strided (XCD-aware order); each block loads the
// tables and the pass's local mu-sets once, and prefetches the next tile's
// input (elements, or words for a changeRepr pass) into registers while the
// current tile's layers run.  Every slot of a full tile is loaded, written to
// LDS and stored, also in a smaller tile (slots past its end repeat its last
// element: same address, same value), so each tile issues a fixed number of
// loads and stores, and the wait for the next tile's loads (issued before
// this tile's stores) does not wait for the stores.
constexpr int kFftPrefetch = (1 << kFftTileLog) / kThreads;
static_assert(kFftPrefetch * kThreads == (1 << kFftTileLog), "every tile element has a prefetch slot");
static_assert(((1 << kFftTileLog) >> kFftRL) <= kThreads, "one group of kFftRL layers per thread");
static_assert(16 * ((1 << kFftTileLog) + kMuEntries) + 65536 + 4096 + 16 * 32 + 8 * 768 + 16 * kPhiNib + 64 <= 163840,
              "FFT kernels fit in LDS");

// PHI: 0 the pass reads the spectrum, 1 64-bit words (kPhi64), 2 128-bit
// words (kPhi128Lo / kPhi128Hi).  The body of one block of a pass launched
// over nblk blocks (block bid of them); inlined into each kernel, so that the
// LDS pointers keep their address space.
template <int PHI>
__device__ __forceinline__ void fft_pass_block(const FftPass& A, uint32_t bid, uint32_t nblk, const uint8_t* g_mt,
                                               const uint32_t* g_lam, const uint4* g_phi, uint8_t* mt, uint32_t* lam,
                                               uint4* tl, uint4* mu, uint4* mu_tile, uint2* mt3, uint4* phin) {
    const uint32_t tid = threadIdx.x;
    const int nt = kThreads;  // the launch uses kThreads threads per block
    copy_words(tid, nt, (uint32_t*)mt, (const uint32_t*)g_mt, 16384);
    copy_words(tid, nt, lam, g_lam, 1024);
    if (PHI) copy_words(tid, nt, (uint32_t*)phin, (const uint32_t*)(g_phi + phin_off(A.phi_in)), 4 * phin_len(A.phi_in));
    __syncthreads();
    build_mt3(tid, nt, mt, mt3);
    fft_local_mu(tid, nt, A, mt, lam, mu);
    const uint64_t ntiles = fft_tiles(A);
    uint64_t t = bid;
    if (t >= ntiles) return;
    FftTileGeom G = fft_geom(A, xcd_tile(t, nblk, ntiles));
    // prefetch registers: the words of a changeRepr pass (PHI), else elements
    std::conditional_t<PHI == 1, uint64_t, uint4> pre[kFftPrefetch];
    // (both lambdas inlined: called out of line, the prefetch registers go
    // through scratch and the LDS tables through generic addresses)
    auto fetch = [&](const FftTileGeom& Gx) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < kFftPrefetch; ++j) {
            const uint32_t e = min(tid + j * kThreads, Gx.nel - 1);
            if constexpr (PHI == 1)
                pre[j] = fft_word(A, Gx, e);
            else if constexpr (PHI == 2)
                pre[j] = fft_word128(A, Gx, e);
            else
                pre[j] = fft_spec(A, Gx, e);
        }
    };
    auto fill = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < kFftPrefetch; ++j) {
            if constexpr (PHI == 1)
                tl[tid + j * kThreads] = phi_word(phin, pre[j]);
            else if constexpr (PHI == 2)
                tl[tid + j * kThreads] = phi_word128(phin, pre[j]);
            else
                tl[tid + j * kThreads] = pre[j];
        }
    };
    fetch(G);
    fill();
    while (true) {
        __syncthreads();
        // the next tile; the last one fetches its own tile again, unused, so
        // that every iteration issues the same loads
        const uint64_t tn = t + nblk;
        const bool more = tn < ntiles;
        const FftTileGeom Gn = fft_geom(A, xcd_tile(more ? tn : t, nblk, ntiles));
        fetch(Gn);
        fft_tile_layers<kFftRL>(tid, nt, A, G, mt, mt3, lam, tl, mu, mu_tile);
#pragma unroll
        for (int j = 0; j < kFftPrefetch; ++j) {
            const uint32_t e = min(tid + j * kThreads, G.nel - 1);
            A.dst[G.gbase | fft_elem_index(A, G, e)] = tl[e];
        }
        if (!more) break;
        __syncthreads();
        fill();
        t = tn;
        G = Gn;
    }
}

#define AFFT_FFT_LDS                          \
    __shared__ __align__(16) uint8_t mt[65536]; \
    __shared__ uint32_t lam[1024];            \
    __shared__ uint4 tl[1 << kFftTileLog];    \
    __shared__ uint4 mu[kMuEntries];          \
    __shared__ uint4 mu_tile[32];             \
    __shared__ uint2 mt3[768];                \
    __shared__ uint4 phin[kPhiNib]

template <int PHI>
__global__ __launch_bounds__(kThreads) void k_fft(FftPass A, const uint8_t* g_mt, const uint32_t* g_lam,
                                                  const uint4* g_phi) {
    AFFT_FFT_LDS;
    fft_pass_block<PHI>(A, blockIdx.x, gridDim.x, g_mt, g_lam, g_phi, mt, lam, tl, mu, mu_tile, mt3, phin);
}

// Two independent passes of the same kind in one launch (the two operands'
// forward transforms of a small product, whose passes hold few tiles each):
// blocks [0, nA) run A, the rest B.
template <int PHI>
__global__ __launch_bounds__(kThreads) void k_fft_pair(FftPass A, FftPass B, uint32_t nA, const uint8_t* g_mt,
                                                       const uint32_t* g_lam, const uint4* g_phi) {
    AFFT_FFT_LDS;
    if (blockIdx.x < nA)
        fft_pass_block<PHI>(A, blockIdx.x, nA, g_mt, g_lam, g_phi, mt, lam, tl, mu, mu_tile, mt3, phin);
    else
        fft_pass_block<PHI>(B, blockIdx.x - nA, gridDim.x - nA, g_mt, g_lam, g_phi, mt, lam, tl, mu, mu_tile, mt3,
                            phin);
}

// The last three steps of a small product in one block, when its inverse
// transform is one tile whose BasisCvt runs inside the pass: pointmul into
// the tile (untruncated, w = 64), the inverse pass, then changeRepr back and
// InterleavedCombine straight from the tile (the Psi table takes the place
// of the product table, which the pass no longer needs).  The spectrum never
// goes back to memory.
struct TailOp {
    PmulOp pm;
    FftPass fft;
    PsiOp psi;
};
static_assert(kPsiTab64 * 16 == 65536, "the Psi table takes the product table's place");

__global__ __launch_bounds__(kThreads) void k_tail(TailOp T, const uint8_t* g_mt, const uint32_t* g_lam,
                                                   const uint32_t* g_ctab, const uint4* g_psi) {
    __shared__ __align__(16) uint8_t mt[65536];
    __shared__ uint32_t lam[1024];
    __shared__ uint4 tl[1 << kFftTileLog];
    __shared__ uint4 mu[kMuEntries];
    __shared__ uint4 mu_tile[32];
    __shared__ uint2 mt3[768];
    __shared__ uint32_t ctab[kConstTabWords];
    const uint32_t tid = threadIdx.x;
    const int nt = kThreads;
    copy_words(tid, nt, (uint32_t*)mt, (const uint32_t*)g_mt, 16384);
    copy_words(tid, nt, lam, g_lam, 1024);
    copy_words(tid, nt, ctab, g_ctab, kConstTabWords);
    __syncthreads();
    build_mt3(tid, nt, mt, mt3);
    fft_local_mu(tid, nt, T.fft, mt, lam, mu);
    // pointmul into the tile (element e is point e: one coset, no column bits)
    const FftTileGeom G = fft_geom(T.fft, 0);
    const uint2 c0 = make_uint2(ctab[kC16Tab], ctab[kC16Tab + 1]), c1 = make_uint2(ctab[kC16Tab + 2], ctab[kC16Tab + 3]);
    const uint32_t c2 = ctab[kC16Tab + 4];
    for (uint32_t e = tid; e < G.nel; e += nt) {
        const uint4 a = T.pm.a[e];
        const uint4 ca = make_uint4(mul_word8_t(c0, c1, c2, a.x), mul_word8_t(c0, c1, c2, a.y),
                                    mul_word8_t(c0, c1, c2, a.z), mul_word8_t(c0, c1, c2, a.w));
        tl[e] = gm128_t(mt, ctab, a, ca, T.pm.b[e]);
    }
    // (fft_tile_layers starts with a barrier and ends with one)
    fft_tile_layers<kFftRL>(tid, nt, T.fft, G, mt, mt3, lam, tl, mu, mu_tile);
    copy_words(tid, nt, (uint32_t*)mt, (const uint32_t*)g_psi, 4 * kPsiTab64);
    __syncthreads();
    const uint4* ptab = (const uint4*)mt;
    const PsiOp& P = T.psi;
    for (uint64_t k = tid; k < P.nwords; k += nt) {
        uint64_t w = 0;
        if (k < P.nspec) w ^= psi_half64(ptab, tl[k], 0);
        if (k >= 1 && k - 1 < P.nspec) w ^= psi_half64(ptab, tl[k - 1], 1);
        if (k == P.nwords - 1 && (P.nbits % 64)) w &= ~0ull >> (64 - P.nbits % 64);
        P.out[k] = w;
    }
}

__global__ __launch_bounds__(kThreads) void k_pmul(PmulOp P, const uint8_t* g_mt, const uint32_t* g_ctab) {
    __shared__ __align__(16) uint8_t mt[65536];
    __shared__ uint32_t ctab[kConstTabWords];
    copy_words(threadIdx.x, blockDim.x, (uint32_t*)mt, (const uint32_t*)g_mt, 16384);
    copy_words(threadIdx.x, blockDim.x, ctab, g_ctab, kConstTabWords);
    __syncthreads();
    const uint64_t nt = pmul_tiles(P);
    for (uint64_t t = blockIdx.x; t < nt; t += gridDim.x) pmul_tile(threadIdx.x, blockDim.x, t, P, mt, ctab);
}

__global__ __launch_bounds__(kThreads) void k_psi(PsiOp P, const uint4* g_psi) {
    __shared__ uint4 tab[kPsiTab64];  // 64 KiB
    static_assert(kPsiTab128 <= kPsiTab64, "both Psi tables fit");
    copy_words(threadIdx.x, blockDim.x, tab, g_psi + psi_tab_off(P), psi_tab_len(P));
    __syncthreads();
    const uint64_t nt = psi_tiles(P);
    for (uint64_t t = blockIdx.x; t < nt; t += gridDim.x) psi_tile(threadIdx.x, blockDim.x, t, P, tab);
}

// Random byte lookups into a 64 KiB LDS table: 8 independent address streams
// per thread (a linear congruential sequence each), every address masked to
// the table.
constexpr int kLookupIters = 2000;
// ---- the simple variant (Alg. 4): polynomial-basis GF(2^128), Cantor points

// The Cantor basis is staged in LDS once per block: the multipliers of a
// group's tables are sums of up to m basis elements, taken one after another.
__global__ __launch_bounds__(kSfThreads) void k_sfft_tab(SfftPass P, const uint4* g_cantor) {
    __shared__ uint4 tab[((1 << kSfTabL) - 1) * kSfTabStride];
    __shared__ uint4 dat[1 << kSfTabPtsLog];
    __shared__ uint4 beta[kCantorBeta];
    const uint32_t npts = 1u << (P.L + P.c), ntab = (1u << P.L) - 1;
    const uint64_t ngroups = sf_tab_groups(P);
    for (uint32_t i = threadIdx.x; i < kCantorBeta; i += blockDim.x) beta[i] = g_cantor[i];
    __syncthreads();
    for (uint64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
        for (uint32_t e = threadIdx.x; e < npts; e += blockDim.x) dat[e] = sfft_load(P, sf_tab_point(P, g, e));
        for (uint32_t t = threadIdx.x; t < ntab; t += blockDim.x) sf_tab_table(P, g, t, beta, tab);
        __syncthreads();
        for (int s = 0; s < P.L;) {
            if (sf_tab_quads(P, s)) {  // two layers per LDS round trip
                for (uint32_t q = threadIdx.x; q < npts / 4; q += blockDim.x) sf_tab_quad(P, s, q, dat, tab);
                s += 2;
            } else {
                for (uint32_t q = threadIdx.x; q < npts / 2; q += blockDim.x) sf_tab_bfly(P, s, q, dat, tab);
                s += 1;
            }
            __syncthreads();
        }
        for (uint32_t e = threadIdx.x; e < npts; e += blockDim.x) P.x[sf_tab_point(P, g, e)] = dat[e];
        __syncthreads();
    }
}

// The bottom pass: one wave per chunk of 64 groups of 2^G consecutive
// points, one group per thread.  The wave's table region (the 64
// lane-interleaved tables) also carries the groups in and out: lane l loads
// points 64 i + l of the chunk (coalesced) into slot (2^G + 1) g + p for point
// p of group g (the pad keeps both the writes and the reads of a group's
// points apart in the banks), and every thread then reads its own.  Each wave
// touches only its own region, so wave-level ordering replaces workgroup
// barriers.
constexpr int kSfGroupThreads = 64;

template <int G, bool INV>
__global__ __launch_bounds__(kSfGroupThreads) void k_sfft_lane(SfftPass P, const uint4* g_cantor) {
    constexpr int CL = G + 6;            // log2 of the chunk's points
    constexpr int GS = (1 << G) + 1;     // staging slots per group
    __shared__ uint4 ltab[kSfLaneTabWave];
    const uint32_t g = threadIdx.x;
    uint4* T0 = ltab + sf_lane_tab(g);
    uint4* X = ltab + g * GS;
    const uint64_t nchunks = (P.n + (1u << CL) - 1) >> CL;
    for (uint64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const uint64_t J0 = c << CL;
#pragma unroll
        for (int i = 0; i < (1 << G); ++i) {
            const uint32_t p = 64 * i + g;
            const uint64_t j = J0 + p;
            ltab[(p >> G) * GS + (p & ((1 << G) - 1))] = j < P.n ? sfft_load(P, j) : make_uint4(0u, 0u, 0u, 0u);
        }
        AFFT_WAVE_SYNC();
        uint4 x[1 << G];
#pragma unroll
        for (int p = 0; p < (1 << G); ++p) x[p] = X[p];
        AFFT_WAVE_SYNC();
        sf_group_layers<G, INV>(P, J0, g, x, T0, g_cantor);
        AFFT_WAVE_SYNC();
#pragma unroll
        for (int p = 0; p < (1 << G); ++p) X[p] = x[p];
        AFFT_WAVE_SYNC();
#pragma unroll
        for (int i = 0; i < (1 << G); ++i) {
            const uint32_t p = 64 * i + g;
            const uint64_t j = J0 + p;
            if (j < P.n) P.x[j] = ltab[(p >> G) * GS + (p & ((1 << G) - 1))];
        }
        AFFT_WAVE_SYNC();
    }
}

// pointmul of Alg. 4: sc[j] = sa[j] * sb[j] in GF(2^128)
__global__ __launch_bounds__(kSfLaneThreads) void k_spmul(const uint4* sa, const uint4* sb, uint4* sc, uint64_t n) {
    __shared__ uint4 ltab[kSfLaneThreads / 64 * kSfLaneTabWave];
    uint4* T0 = ltab + (threadIdx.x >> 6) * kSfLaneTabWave + sf_lane_tab(threadIdx.x & 63);
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (uint64_t)gridDim.x * blockDim.x) {
        const uint4 a = sa[j], b = sb[j];
        gcm_build_tab<kSfLaneTabStride>(a, T0);
        sc[j] = gcm_mul_tab_lane(T0, b);
    }
}

__global__ __launch_bounds__(kSfThreads) void k_scombine(const uint4* F, uint64_t n, uint64_t* c, uint64_t nwords,
                                                         uint64_t nc_bits) {
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nwords;
         k += (uint64_t)gridDim.x * blockDim.x)
        c[k] = sf_combine_word(F, n, k, nwords, nc_bits);
}

// ---- the Frobenius-partition variant (App. C)

// z-adic expansion or recomposition: the levels of one pass, tile by tile
__global__ __launch_bounds__(kZThreads) void k_zadic(ZadicPass Z) {
    __shared__ uint64_t lds[1 << kZTileLog];
    const uint64_t nt = zadic_tiles(Z);
    for (uint64_t t = blockIdx.x; t < nt; t += gridDim.x)
        zadic_tile(threadIdx.x, blockDim.x, xcd_tile(t, gridDim.x, nt), Z, lds);
}

// per-word conversion, bit transpose and encoding map: the n elements
__global__ __launch_bounds__(kFeThreads) void k_fencode(FrobEncode F, const uint4* g_tab) {
    __shared__ uint4 etab[kElemTab];
    __shared__ uint64_t wtab[kWordTab];
    __shared__ uint64_t lds[kFeStage];
    const uint64_t* gw = (const uint64_t*)(g_tab + kFrobWordOff);
    for (uint32_t i = threadIdx.x; i < kElemTab; i += blockDim.x) etab[i] = g_tab[kFrobEncOff + i];
    for (uint32_t i = threadIdx.x; i < kWordTab; i += blockDim.x) wtab[i] = gw[i];
    __syncthreads();
    const uint64_t nt = frob_tiles(F.m);
    for (uint64_t t = blockIdx.x; t < nt; t += gridDim.x) frob_encode_tile(threadIdx.x, blockDim.x, t, F, etab, wtab, lds);
}

// inverse encoding map, bit transpose back, inverse per-word conversion
// (512-thread blocks: the decoding body needs more than the 128 registers a
// 1024-thread block leaves each lane, and spilled with them)
constexpr int kFdThreads = 512;
__global__ __launch_bounds__(kFdThreads) void k_fdecode(FrobDecode F, const uint4* g_tab) {
    __shared__ uint4 dtab[kElemTab];
    __shared__ uint64_t wtab[kWordTab];
    __shared__ uint64_t lds[kFeStage];
    const uint64_t* gw = (const uint64_t*)(g_tab + kFrobWordOff) + kWordTab;
    for (uint32_t i = threadIdx.x; i < kElemTab; i += blockDim.x) dtab[i] = g_tab[kFrobDecOff + i];
    for (uint32_t i = threadIdx.x; i < kWordTab; i += blockDim.x) wtab[i] = gw[i];
    __syncthreads();
    const uint64_t nt = frob_tiles(F.m);
    for (uint64_t t = blockIdx.x; t < nt; t += gridDim.x) frob_decode_tile(threadIdx.x, blockDim.x, t, F, dtab, wtab, lds);
}

__global__ __launch_bounds__(kThreads) void k_lookup_rate(const uint8_t* g_mt, uint32_t* out) {
    __shared__ __align__(16) uint8_t mt[65536];
    copy_words(threadIdx.x, blockDim.x, (uint32_t*)mt, (const uint32_t*)g_mt, 16384);
    __syncthreads();
    const uint32_t id = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t st[8], acc = 0;
    for (int j = 0; j < 8; ++j) st[j] = id * 2654435761u + 40503u * (uint32_t)j + 1u;
    for (int it = 0; it < kLookupIters; ++it) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            st[j] = st[j] * 1664525u + 1013904223u;
            acc += mt[st[j] >> 16];
        }
    }
    out[id] = acc;
}

__global__ __launch_bounds__(kThreads) void k_spine(SpineOp S, const uint8_t* g_mt, const uint4* g_phi) {
    __shared__ __align__(16) uint8_t mt[65536];
    __shared__ uint4 phin[kPhiNib];
    copy_words(threadIdx.x, blockDim.x, (uint32_t*)mt, (const uint32_t*)g_mt, 16384);
    copy_words(threadIdx.x, blockDim.x, (uint32_t*)phin, (const uint32_t*)g_phi, 4 * phin_len(kPhi64));
    __syncthreads();
    const uint64_t nt = spine_tiles(S);
    for (uint64_t t = blockIdx.x; t < nt; t += gridDim.x) spine_tile(threadIdx.x, blockDim.x, t, S, mt, phin);
}

// ------------------------------------------------------- multi-op kernels
// One launch runs the tiles of an array of ops of one kind (a batch group).
// Block b takes a contiguous chunk of the tiles, so consecutive tiles mostly
// belong to the same op.

__device__ inline void block_chunk(uint64_t total, uint64_t& g0, uint64_t& g1) {
    uint64_t per = (total + gridDim.x - 1) / gridDim.x;
    g0 = (uint64_t)blockIdx.x * per;
    g1 = g0 + per < total ? g0 + per : total;
}

__global__ __launch_bounds__(kThreads) void k_pack_multi(const PackOp* ops, const uint64_t* prefix, int nops,
                                                         uint64_t total) {
    uint64_t g0, g1;
    block_chunk(total, g0, g1);
    int o = -1;
    for (uint64_t g = g0; g < g1; ++g) {
        o = op_of_tile(prefix, nops, g, o);
        pack_tile(threadIdx.x, blockDim.x, g - prefix[o], ops[o]);
    }
}

template <int WIDE>
__global__ __launch_bounds__(kThreads) void k_bc_tile_multi(const BcTileOp* ops, const uint64_t* prefix, int nops,
                                                            uint64_t total) {
    __shared__ uint4 lds[1 << kBcTileLog128];  // 64 KiB
    uint64_t g0, g1;
    block_chunk(total, g0, g1);
    int o = -1;
    for (uint64_t g = g0; g < g1; ++g) {
        o = op_of_tile(prefix, nops, g, o);
        const BcTileOp B = ops[o];
        if (WIDE)
            bc_tile<uint4>(threadIdx.x, blockDim.x, g - prefix[o], B, lds);
        else
            bc_tile<uint64_t>(threadIdx.x, blockDim.x, g - prefix[o], B, (uint64_t*)lds);
    }
}

template <int WIDE>
__global__ __launch_bounds__(kThreads) void k_bc_class_multi(const BcClassOp* ops, const uint64_t* prefix, int nops,
                                                             uint64_t total) {
    __shared__ uint4 lds[1 << kBcTileLog128];  // 64 KiB
    uint64_t g0, g1;
    block_chunk(total, g0, g1);
    int o = -1;
    for (uint64_t g = g0; g < g1; ++g) {
        o = op_of_tile(prefix, nops, g, o);
        const BcClassOp C = ops[o];
        if (WIDE)
            bc_class_tile<uint4>(threadIdx.x, blockDim.x, g - prefix[o], C, lds);
        else
            bc_class_tile<uint64_t>(threadIdx.x, blockDim.x, g - prefix[o], C, (uint64_t*)lds);
    }
}

__global__ __launch_bounds__(kThreads) void k_fft_multi(const FftPass* ops, const uint64_t* prefix, int nops,
                                                        uint64_t total, const uint8_t* g_mt, const uint32_t* g_lam,
                                                        const uint4* g_phi) {
    __shared__ __align__(16) uint8_t mt[65536];
    __shared__ uint32_t lam[1024];
    __shared__ uint4 tl[1 << kFftTileLog];
    __shared__ uint4 mu[kMuEntries];
    __shared__ uint4 mu_tile[32];
    __shared__ uint2 mt3[768];
    __shared__ uint4 phin[kPhiNib];
    const int tid = threadIdx.x, nt = blockDim.x;
    copy_words(tid, nt, (uint32_t*)mt, (const uint32_t*)g_mt, 16384);
    copy_words(tid, nt, lam, g_lam, 1024);
    __syncthreads();
    build_mt3(tid, nt, mt, mt3);
    __syncthreads();
    uint64_t g0, g1;
    block_chunk(total, g0, g1);
    int o = -1;
    uint32_t cur_lo = ~0u, cur_hi = ~0u, cur_pack = ~0u, cur_phi = kPhiNone;
    for (uint64_t g = g0; g < g1; ++g) {
        o = op_of_tile(prefix, nops, g, o);
        const FftPass A = ops[o];
        if (A.phi_in != kPhiNone && A.phi_in != cur_phi) {
            // the changeRepr table of this pass (every thread is past the last tile)
            copy_words(tid, nt, (uint32_t*)phin, (const uint32_t*)(g_phi + phin_off(A.phi_in)), 4 * phin_len(A.phi_in));
            __syncthreads();
            cur_phi = A.phi_in;
        }
        if (A.lo != cur_lo || A.hi != cur_hi || A.pack != cur_pack) {
            // the local mu-sets depend only on the layer range and row bits of the pass
            fft_local_mu(tid, nt, A, mt, lam, mu);
            cur_lo = A.lo;
            cur_hi = A.hi;
            cur_pack = A.pack;
        }
        fft_tile<kFftRL>(tid, nt, g - prefix[o], A, mt, mt3, lam, phin, tl, mu, mu_tile);
    }
}

__global__ __launch_bounds__(kThreads) void k_pmul_multi(const PmulOp* ops, const uint64_t* prefix, int nops,
                                                         uint64_t total, const uint8_t* g_mt, const uint32_t* g_ctab) {
    __shared__ __align__(16) uint8_t mt[65536];
    __shared__ uint32_t ctab[kConstTabWords];
    copy_words(threadIdx.x, blockDim.x, (uint32_t*)mt, (const uint32_t*)g_mt, 16384);
    copy_words(threadIdx.x, blockDim.x, ctab, g_ctab, kConstTabWords);
    __syncthreads();
    uint64_t g0, g1;
    block_chunk(total, g0, g1);
    int o = -1;
    for (uint64_t g = g0; g < g1; ++g) {
        o = op_of_tile(prefix, nops, g, o);
        pmul_tile(threadIdx.x, blockDim.x, g - prefix[o], ops[o], mt, ctab);
    }
}

__global__ __launch_bounds__(kThreads) void k_spine_multi(const SpineOp* ops, const uint64_t* prefix, int nops,
                                                          uint64_t total, const uint8_t* g_mt, const uint4* g_phi) {
    __shared__ __align__(16) uint8_t mt[65536];
    __shared__ uint4 phin[kPhiNib];
    copy_words(threadIdx.x, blockDim.x, (uint32_t*)mt, (const uint32_t*)g_mt, 16384);
    copy_words(threadIdx.x, blockDim.x, (uint32_t*)phin, (const uint32_t*)g_phi, 4 * phin_len(kPhi64));
    __syncthreads();
    uint64_t g0, g1;
    block_chunk(total, g0, g1);
    int o = -1;
    for (uint64_t g = g0; g < g1; ++g) {
        o = op_of_tile(prefix, nops, g, o);
        spine_tile(threadIdx.x, blockDim.x, g - prefix[o], ops[o], mt, phin);
    }
}

__global__ __launch_bounds__(kThreads) void k_psi_multi(const PsiOp* ops, const uint64_t* prefix, int nops,
                                                        uint64_t total, const uint4* g_psi) {
    __shared__ uint4 tab[kPsiTab64];
    uint64_t g0, g1;
    block_chunk(total, g0, g1);
    int o = -1, cur = -1;  // cur: the table in LDS (psi_tab_off), -1 none
    for (uint64_t g = g0; g < g1; ++g) {
        o = op_of_tile(prefix, nops, g, o);
        if (psi_tab_off(ops[o]) != cur) {
            __syncthreads();
            cur = psi_tab_off(ops[o]);
            copy_words(threadIdx.x, blockDim.x, tab, g_psi + cur, psi_tab_len(ops[o]));
            __syncthreads();
        }
        psi_tile(threadIdx.x, blockDim.x, g - prefix[o], ops[o], tab);
    }
}

// ------------------------------------------------ persistent batch kernel
// All tiles of a batch in one launch.  Items (op, tile) are numbered rank by
// rank; inside a rank, blocks take items from the rank's counter, and the
// grid meets at a barrier between ranks (op r of a job needs op r - 1 done).
// Every block is resident (one per CU), and every wait is bounded: a timeout
// raises the abort flag, after which all blocks leave.
struct DevOp {
    int kind;
    int wide;
    int pad0;
    uint32_t tiles;  // tiles of this op
    union {
        PackOp pack;
        BcTileOp bct;
        BcLayerOp bcl;
        FftPass fft;
        PmulOp pmul;
        PsiOp psi;
        BcClassOp bcc;
        SpineOp spn;
    };
};

struct PersistArgs {
    const DevOp* ops;
    const uint64_t* prefix;      // first item of each op (ops in item order), prefix[nops] = items
    const uint64_t* rank_first;  // first item of each rank, rank_first[nranks] = items
    int nops;
    int nranks;
    uint64_t items;
    unsigned long long* next;    // per rank: item counter
    uint32_t* arrive;            // per rank: blocks past the rank
    uint32_t* abort;             // set when a wait times out
    uint32_t spin_limit;
};

// Where the parts of a persistent launch's descriptor image sit.
struct PersistLayout {
    size_t ops_off = 0, prefix_off = 0, rank_off = 0, state_off = 0, state_words = 0, bytes = 0;
    int nops = 0, nranks = 0;
    uint64_t items = 0;
};

__global__ __launch_bounds__(kThreads) void k_zero_u32(uint32_t* p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) p[i] = 0;
}

static_assert(kConstTabWords <= 4 * ((1 << kFftTileLog) + kMuEntries), "the pointmul tables fit the work area");

// One block's state for running items (op, tile) of any kind: the LDS tables
// of the kernels above and what the shared work area currently holds (0
// nothing reusable, 1 the FFT local mu-sets of (cur_lo, cur_hi), 2 the w = 64
// Psi table, 3 the w = 128 one, 4 the constant-multiple tables of pointmul);
// phin holds the changeRepr table of mode cur_phi.  Used by the persistent
// kernel and the single-block product kernel.
struct ItemBlock {
    uint8_t* mt;
    uint32_t* lam;
    uint4* work;  // FFT tile + mu-set tables, a BasisCvt tile, or the Psi table
    uint4* mu_tile;
    uint2* mt3;
    uint4* phin;
    const uint4* g_phi;
    const uint4* g_psi;
    const uint32_t* g_ctab;
    int held;
    uint32_t cur_lo, cur_hi, cur_phi, cur_pack;
};

__device__ __forceinline__ void block_need_phin(int tid, int nt, ItemBlock& S, uint32_t mode) {
    if (mode == kPhiNone || mode == S.cur_phi) return;
    copy_words(tid, nt, (uint32_t*)S.phin, (const uint32_t*)(S.g_phi + phin_off(mode)), 4 * phin_len(mode));
    __syncthreads();
    S.cur_phi = mode;
}

// Tile t of op D, by the whole block (inlined into each kernel, so that the
// LDS pointers keep their address space).  The tile bodies that use the LDS
// as a work area end with a barrier; the others only read their tables.
__device__ __forceinline__ void run_item(int tid, int nt, ItemBlock& S, const DevOp& D, uint64_t t) {
    uint4* tl = S.work;
    uint4* mu = S.work + (1 << kFftTileLog);
    switch ((OpKind)D.kind) {
        case OpKind::Pack: pack_tile(tid, nt, t, D.pack); break;
        case OpKind::BcTile:
            if (D.wide)
                bc_tile<uint4>(tid, nt, t, D.bct, S.work);
            else
                bc_tile<uint64_t>(tid, nt, t, D.bct, (uint64_t*)S.work);
            S.held = 0;
            break;
        case OpKind::BcClass:
            if (D.wide)
                bc_class_tile<uint4>(tid, nt, t, D.bcc, S.work);
            else
                bc_class_tile<uint64_t>(tid, nt, t, D.bcc, (uint64_t*)S.work);
            S.held = 0;
            break;
        case OpKind::BcLayer: {
            // one item covers one global layer part (only very long jobs)
            const BcLayerOp L = D.bcl;
            if (L.wide)
                bc_part<uint4>(tid, nt, (uint4*)L.data, L.nelem, L.layer, (int)L.which);
            else
                bc_part<uint64_t>(tid, nt, (uint64_t*)L.data, L.nelem, L.layer, (int)L.which);
            break;
        }
        case OpKind::Fft: {
            const FftPass A = D.fft;
            block_need_phin(tid, nt, S, A.phi_in);
            if (S.held != 1 || A.lo != S.cur_lo || A.hi != S.cur_hi || A.pack != S.cur_pack) {
                fft_local_mu(tid, nt, A, S.mt, S.lam, mu);
                S.held = 1;
                S.cur_lo = A.lo;
                S.cur_hi = A.hi;
                S.cur_pack = A.pack;
            }
            fft_tile<kFftRL>(tid, nt, t, A, S.mt, S.mt3, S.lam, S.phin, tl, mu, S.mu_tile);
            break;
        }
        case OpKind::Pmul:
            if (S.held != 4) {
                copy_words(tid, nt, (uint32_t*)S.work, S.g_ctab, kConstTabWords);
                __syncthreads();
                S.held = 4;
            }
            pmul_tile(tid, nt, t, D.pmul, S.mt, (const uint32_t*)S.work);
            break;
        case OpKind::Psi: {
            const int want = D.psi.spech ? 3 : 2;
            if (S.held != want) {
                copy_words(tid, nt, S.work, S.g_psi + psi_tab_off(D.psi), psi_tab_len(D.psi));
                __syncthreads();
                S.held = want;
            }
            psi_tile(tid, nt, t, D.psi, S.work);
            break;
        }
        case OpKind::Spine:
            block_need_phin(tid, nt, S, kPhi64);
            spine_tile(tid, nt, t, D.spn, S.mt, S.phin);
            break;
    }
}

__global__ __launch_bounds__(kThreads) void k_persistent(PersistArgs P, const uint8_t* g_mt, const uint32_t* g_lam,
                                                         const uint4* g_phi, const uint4* g_psi,
                                                         const uint32_t* g_ctab) {
    __shared__ __align__(16) uint8_t mt[65536];
    __shared__ uint32_t lam[1024];
    __shared__ uint4 work[(1 << kFftTileLog) + kMuEntries];
    __shared__ uint4 mu_tile[32];
    __shared__ uint2 mt3[768];
    __shared__ uint4 phin[kPhiNib];
    __shared__ uint64_t s_item;
    __shared__ int s_stop;
    const int tid = threadIdx.x, nt = blockDim.x;
    copy_words(tid, nt, (uint32_t*)mt, (const uint32_t*)g_mt, 16384);
    copy_words(tid, nt, lam, g_lam, 1024);
    __syncthreads();
    build_mt3(tid, nt, mt, mt3);  // visible after the item loop's first barrier
    ItemBlock S{mt, lam, work, mu_tile, mt3, phin, g_phi, g_psi, g_ctab, 0, ~0u, ~0u, kPhiNone, ~0u};
    int o = -1;
    for (int r = 0; r < P.nranks; ++r) {
        const uint64_t end = P.rank_first[r + 1];
        while (true) {
            __syncthreads();
            if (tid == 0) {
                uint64_t it = end;
                if (!__hip_atomic_load(P.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                    it = P.rank_first[r] + __hip_atomic_fetch_add(&P.next[r], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_item = it;
            }
            __syncthreads();
            const uint64_t item = s_item;
            if (item >= end) break;
            o = op_of_tile(P.prefix, P.nops, item, -1);
            run_item(tid, nt, S, P.ops[o], item - P.prefix[o]);
        }
        // grid barrier between ranks.  After the workgroup barrier every store
        // of this block has completed; one thread releases them at agent
        // scope with its arrival (an agent-scope fence writes back the whole
        // L2 of this XCD, so one per block suffices, and one per wave would
        // repeat it 16 times), polls with relaxed loads (an acquiring poll
        // would invalidate the L2 on every iteration), and acquires once; the
        // second workgroup barrier orders the block's later loads after it.
        __syncthreads();
        if (tid == 0) {
            int stop = 0;
            __hip_atomic_fetch_add(&P.arrive[r], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            uint32_t spins = 0;
            while (__hip_atomic_load(&P.arrive[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gridDim.x) {
                if (__hip_atomic_load(P.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    stop = 1;
                    break;
                }
                if (++spins > P.spin_limit) {
                    __hip_atomic_store(P.abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    stop = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            s_stop = stop;
        }
        __syncthreads();
        if (s_stop) break;
    }
}

// ------------------------------------------------ whole product in one launch
// A small product's ops, carried in the kernel arguments, run one after the
// other by a single block: every tile of an op, then a barrier (op k + 1
// reads what op k wrote, through the block's own cache), then the next op.
// One dispatch per product; the spectra stay in that CU's cache hierarchy.
constexpr int kSingleMaxOps = 32;
constexpr int kSingleMaxLog = 12;  // transforms of at most 2^12 points take this path
struct SingleArgs {
    DevOp ops[kSingleMaxOps];
    int nops;
};
static_assert(sizeof(SingleArgs) <= 4096, "the op list fits the kernel arguments");

__global__ __launch_bounds__(kThreads) void k_single(SingleArgs P, const uint8_t* g_mt, const uint32_t* g_lam,
                                                     const uint4* g_phi, const uint4* g_psi, const uint32_t* g_ctab) {
    __shared__ __align__(16) uint8_t mt[65536];
    __shared__ uint32_t lam[1024];
    __shared__ uint4 work[(1 << kFftTileLog) + kMuEntries];
    __shared__ uint4 mu_tile[32];
    __shared__ uint2 mt3[768];
    __shared__ uint4 phin[kPhiNib];
    const int tid = threadIdx.x, nt = blockDim.x;
    copy_words(tid, nt, (uint32_t*)mt, (const uint32_t*)g_mt, 16384);
    copy_words(tid, nt, lam, g_lam, 1024);
    __syncthreads();
    build_mt3(tid, nt, mt, mt3);
    __syncthreads();
    ItemBlock S{mt, lam, work, mu_tile, mt3, phin, g_phi, g_psi, g_ctab, 0, ~0u, ~0u, kPhiNone, ~0u};
    for (int o = 0; o < P.nops; ++o) {
        const DevOp D = P.ops[o];
        for (uint64_t t = 0; t < D.tiles; ++t) run_item(tid, nt, S, D, t);
        __syncthreads();
    }
}

// ------------------------------------------------------- the static buffer

// Workspace of gf2x_mul_dev_static: a fixed array in device memory, one copy
// per GPU, held until the process ends.  In host code `scratch` names a host
// stand-in, not the device copy: host code only ever uses the address that
// hipGetSymbolAddress returns for the current device (scratch_address).
static __device__ __align__(256) char scratch[GF2X_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// This device's copy of `scratch`, looked up once per device with that
// device current (gf2x_ctx_create makes it current).
hipError_t scratch_address(int device, char** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = (char*)p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}
}  // namespace

// ------------------------------------------------------------------ context

struct gf2x_ctx {
    int device = 0;
    int ncu = 256;
    uint8_t* d_mt = nullptr;
    uint32_t* d_lam = nullptr;
    uint4* d_phi = nullptr;
    uint4* d_psi = nullptr;
    uint32_t* d_ctab = nullptr;  // constant-multiple tables of the generic product
    uint4* d_cantor = nullptr;   // simple variant: Cantor basis and phi table
    uint4* d_frob = nullptr;     // Frobenius variant: encoding maps and per-word conversions
    char* ws = nullptr;
    size_t ws_bytes = 0;
    char* io = nullptr;  // operand/product staging for the host-pointer entry point
    size_t io_bytes = 0;
    hipStream_t own_stream = nullptr;
    // second stream for the forward transform of b in single products small
    // enough to leave most CUs idle; fork and join events
    hipStream_t aux_stream = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // calls that use the workspace on a stream other than the previous such
    // call's wait for ev_last, recorded at the end of that call
    hipEvent_t ev_last = nullptr;
    hipStream_t last_st = nullptr;
    bool has_last = false;
    // this device's copy of the static product buffer (gf2x_mul_dev_static)
    char* scratch = nullptr;
    // blocks of the persistent kernel one CU holds at once (its launch needs
    // at least one: the grid is one block per CU and its blocks wait for
    // each other)
    int persist_per_cu = 0;
    // products of at most 2^single_max_log points run in one dispatch (-1:
    // never, the default: one block running every stage measured slower than
    // the op-by-op launches, which spread each stage's tiles over the device)
    int single_max_log = -1;
    // BasisCvt inside FFT passes for single products (gf2x_mul_dev, the
    // no-allocation entry, served requests on an idle engine) up to 2^13
    // points; batches and serving iterations use params.fuse_max_log (2^11)
    int fuse_single_max_log = 13;
    std::string err;
    gf2x_batch* transient = nullptr;  // the last gf2x_mul_batch call's plan
    hipStream_t transient_stream = nullptr;
    LayerPool pool;  // BasisCvt layer lists; pool.base points at d_layers
    BcLayer* d_layers = nullptr;
    PlanParams params;  // params.lam / params.mt point at the host tables below
    uint32_t h_lam[32 * 32];
    std::vector<uint8_t> h_mt;
    // tracing
    uint32_t trace_mask = 0;
    struct Pending {
        gf2x_trace_rec rec;
        hipEvent_t start, stop;
    };
    std::vector<Pending> trace;
};

struct gf2x_batch {
    gf2x_ctx* ctx = nullptr;
    int mode = 0;
    BatchPlan plan;
    char* ws = nullptr;
    char* desc = nullptr;
    size_t desc_bytes = 0;
    std::vector<gf2x::LaunchGroup> groups;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool use_graph = true;
    // persistent mode: ops in item order, their item prefix, scheduler state
    char* pdesc = nullptr;
    PersistLayout play;
    uint32_t spin_limit = 1u << 26;
};

// Serving engine state (host side); see gf2x_server_* in the header.
struct gf2x_server {
    gf2x_ctx* ctx = nullptr;
    gf2x_server_cfg cfg{};
    hipStream_t st = nullptr;
    char* arena = nullptr;
    gf2x::Arena alloc;
    struct Req {
        const uint64_t* a = nullptr;
        const uint64_t* b = nullptr;
        uint64_t* c = nullptr;
        uint64_t na = 0, nb = 0, tag = 0, t_submit = 0, t_admit = 0;
        int w = 64;  // word width when submitted (its footprint is for that width)
        hipStream_t src = nullptr;  // the caller's stream at submit, and an event recorded on it then
        hipEvent_t ready = nullptr;
        size_t off = 0, bytes = 0;
        std::vector<gf2x::Op> ops;
        std::vector<uint64_t> level_tiles;  // tiles of each dependency level
        uint32_t levels = 0, next = 0, iters = 0;
    };
    std::deque<Req> queue;
    std::vector<Req> active;
    // one descriptor buffer pair per iteration that can be queued at once
    struct Slot {
        char* host = nullptr;  // pinned
        char* dev = nullptr;
        size_t cap = 0;
        hipEvent_t ev = nullptr;
        std::vector<gf2x_done> fin;  // requests whose last op is in this iteration
        size_t abort_off = 0;        // persistent mode: the abort word is copied back here
        bool persistent = false;
    };
    std::vector<Slot> slots;
    std::deque<int> inflight;  // slots in launch order
    std::vector<int> free_slots;
    std::deque<gf2x_done> done;
    gf2x_server_stats stats{};
    int sticky = GF2X_OK;
    uint32_t spin_limit = 1u << 26;
    // per-iteration scratch, reused
    std::vector<gf2x::Op> it_ops;
    std::vector<uint32_t> it_rank;
    std::vector<gf2x::BatchGroup> it_groups;
    std::vector<gf2x::LaunchGroup> it_launch;
    std::vector<char> it_host;
    // events recorded on callers' streams at submit, reused
    std::vector<hipEvent_t> free_events, all_events;
};


// (defined below, with the single-product launchers; the serving engine's
// light-load path uses it too)
int run_product(gf2x_ctx* ctx, const std::vector<Op>& ops, const size_t* split, int m, hipStream_t st,
                bool may_trace);
PlanParams single_params(const gf2x_ctx* ctx);

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

int fail(gf2x_ctx* ctx, int code, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return code;
}

int hip_fail(gf2x_ctx* ctx, hipError_t e, const char* where) {
    return fail(ctx, GF2X_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

uint4 to_u4(u128 v) {
    uint4 r;
    r.x = (uint32_t)v;
    r.y = (uint32_t)(v >> 32);
    r.z = (uint32_t)(v >> 64);
    r.w = (uint32_t)(v >> 96);
    return r;
}

bool ranges_overlap(const void* p, size_t pn, const void* q, size_t qn) {
    if (!p || !q || !pn || !qn) return false;
    auto a = (uintptr_t)p, b = (uintptr_t)q;
    return a < b + qn && b < a + pn;
}

// Calls on one context share its workspace.  A call on a stream other than
// the previous workspace call's waits for everything that call enqueued (an
// event recorded at its end), so calls on mixed streams run one after the
// other instead of racing.  Calls under stream capture take no part (an event
// recorded outside a capture cannot be waited on inside it).
bool stream_capturing(hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return cs != hipStreamCaptureStatusNone;
}

int ws_enter(gf2x_ctx* ctx, hipStream_t st, bool capturing) {
    if (capturing || !ctx->has_last || st == ctx->last_st) return GF2X_OK;
    hipError_t e = hipStreamWaitEvent(st, ctx->ev_last, 0);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamWaitEvent (stream order)");
    return GF2X_OK;
}

int ws_leave(gf2x_ctx* ctx, hipStream_t st, bool capturing, int rc) {
    if (rc) return rc;
    if (capturing) {
        ctx->has_last = false;
        return GF2X_OK;
    }
    hipError_t e = hipEventRecord(ctx->ev_last, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipEventRecord (stream order)");
    ctx->last_st = st;
    ctx->has_last = true;
    return GF2X_OK;
}

int ensure_ws(gf2x_ctx* ctx, size_t bytes, hipStream_t st) {
    if (bytes <= ctx->ws_bytes) return GF2X_OK;
    // work already enqueued may still use the old buffer
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess && ctx->aux_stream) e = hipStreamSynchronize(ctx->aux_stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
    if (ctx->ws) (void)hipFree(ctx->ws);
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
    size_t want = std::max(bytes, (size_t)1 << 20);
    e = hipMalloc((void**)&ctx->ws, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, GF2X_ENOMEM, "workspace of " + std::to_string(want) + " bytes: " + hipGetErrorString(e));
    }
    ctx->ws_bytes = want;
    return GF2X_OK;
}

unsigned grid_for(uint64_t tiles, uint64_t cap) {
    uint64_t g = std::min<uint64_t>(tiles, cap);
    return (unsigned)std::max<uint64_t>(g, 1);
}

// Bytes a launch must move through memory, by its definition (each element it
// covers is read once and written once), and the elements it covers.
void op_traffic(const Op& op, gf2x_trace_rec& r) {
    r.kind = (int)op.kind;
    r.lookups = 0;
    switch (op.kind) {
        case OpKind::Pack:
            r.elements = op.pack.ndst;
            r.bytes_read = 8 * std::min<uint64_t>(op.pack.ndst, (op.pack.nbits + 63) / 64);
            r.bytes_written = 8 * op.pack.ndst;
            break;
        case OpKind::BcTile:
            r.elements = op.bct.nelem;
            r.bytes_read = r.bytes_written = op.bct.nelem * (op.bct.wide ? 16 : 8);
            break;
        case OpKind::BcLayer: {
            uint64_t half = op.bcl.nelem / 2, es = op.bcl.wide ? 16 : 8;
            uint64_t D = 1ull << op.bcl.layer.log_d, k = 1ull << op.bcl.layer.log_k;
            uint64_t part = op.bcl.which == 0 ? half / D * k : half / D * (D - k);
            r.elements = part;
            r.bytes_read = 2 * part * es;  // source and target
            r.bytes_written = part * es;
            break;
        }
        case OpKind::Fft: {
            uint64_t n = (uint64_t)op.fft.ncosets << op.fft.log_m;
            r.elements = n;
            r.bytes_read = op.fft.phi_in == kPhi64 ? 8 * n : 16 * n;  // words, 128-bit words or elements
            r.bytes_written = 16 * n;
            // LDS table reads per butterfly (index: width_mode): 6, 9 or 8 byte
            // lookups per word (4 words) for 16-bit, 32-bit and 17..24-bit
            // multipliers; 3 table reads for 8-bit ones (their bytes are looked
            // up in registers)
            static const uint64_t per_bfly[4] = {3, 24, 36, 32};
            for (uint32_t i = op.fft.lo; i < op.fft.hi; ++i)
                r.lookups += (n / 2) * per_bfly[width_mode((int)op.fft.log_total - (int)i)];
            break;
        }
        case OpKind::Pmul: {
            const uint64_t eb = op.pmul.ah ? 32 : 16;  // bytes of a TGF(2^256) / TGF(2^128) point
            r.elements = op.pmul.n;
            r.bytes_read = 2 * eb * op.pmul.n;
            r.bytes_written = eb * op.pmul.n;
            break;
        }
        case OpKind::BcClass:
            r.elements = op.bcc.nelem;
            r.bytes_read = r.bytes_written = op.bcc.nelem * (op.bcc.wide ? 16 : 8);
            break;
        case OpKind::Psi:
            r.elements = op.psi.nwords;
            if (op.psi.spech)
                r.bytes_read = 32 * std::min((op.psi.nwords + 1) / 2, op.psi.nspec);
            else
                r.bytes_read = 16 * std::min(op.psi.nwords, op.psi.nspec);
            r.bytes_written = 8 * op.psi.nwords;
            break;
        case OpKind::Spine: {
            const uint64_t n = op.spn.n;
            const uint32_t md = op.spn.mode;
            r.elements = n;
            r.bytes_read = md == kSpineZero ? 0 : md == kSpinePhi ? 8 * n : md == kSpineHalf || md == kSpineAdd ? 32 * n : 32 * n;
            r.bytes_written = md == kSpineFwd || md == kSpineInv ? 32 * n : 16 * n;
            break;
        }
    }
}

// A launch of the executor: with tracing on, the start and stop events ride
// in the dispatch itself (hipExtLaunchKernelGGL), so the recorded time is the
// kernel's own, as a profiler measures it.
#define GF2X_LAUNCH_N(K, GRID, NT, ...)                                                               \
    do {                                                                                              \
        if (traced)                                                                                   \
            hipExtLaunchKernelGGL(K, GRID, dim3(NT), 0, st, pend.start, pend.stop, 0, __VA_ARGS__); \
        else                                                                                          \
            hipLaunchKernelGGL(K, GRID, dim3(NT), 0, st, __VA_ARGS__);                               \
    } while (0)
#define GF2X_LAUNCH(K, GRID, ...) GF2X_LAUNCH_N(K, GRID, kThreads, __VA_ARGS__)

// `may_trace` false: no launch is traced whatever the trace mask says (tracing
// creates events, and some callers must not have anything created for them).
// `pair_levels`: the list's levels are dependency levels (plan_mul), and two
// consecutive FFT passes of one level whose tiles fit one round of the grid
// run in one launch (one trace record covers both).
int run_ops(gf2x_ctx* ctx, const std::vector<Op>& ops, hipStream_t st, bool may_trace = true,
            bool pair_levels = false) {
    const uint64_t ncu = (uint64_t)ctx->ncu;
    for (size_t oi = 0; oi < ops.size(); ++oi) {
        const Op& op = ops[oi];
        const Op* mate = nullptr;
        if (pair_levels && op.kind == OpKind::Fft && oi + 1 < ops.size()) {
            const Op& nx = ops[oi + 1];
            if (nx.kind == OpKind::Fft && nx.level == op.level && nx.fft.phi_in == op.fft.phi_in &&
                fft_tiles(op.fft) + fft_tiles(nx.fft) <= ncu)
                mate = &nx;
        }
        gf2x_ctx::Pending pend{};
        const bool traced = may_trace && ((ctx->trace_mask >> (int)op.kind) & 1u);
        if (traced) {
            op_traffic(op, pend.rec);
            if (mate) {
                gf2x_trace_rec r2{};
                op_traffic(*mate, r2);
                pend.rec.elements += r2.elements;
                pend.rec.bytes_read += r2.bytes_read;
                pend.rec.bytes_written += r2.bytes_written;
                pend.rec.lookups += r2.lookups;
            }
            hipError_t e = hipEventCreate(&pend.start);
            if (e == hipSuccess) e = hipEventCreate(&pend.stop);
            if (e != hipSuccess) return hip_fail(ctx, e, "trace event");
        }
        switch (op.kind) {
            case OpKind::Pack:
                GF2X_LAUNCH(k_pack, dim3(grid_for(pack_tiles(op.pack), 8 * ncu)), op.pack);
                break;
            case OpKind::BcTile: {
                const bool small = (int)(op.bct.log_rows + op.bct.log_tc) <=
                                   (op.bct.wide ? kBcTileLog128 : kBcTileLog64) - kBcSmallShift;
                const dim3 g(grid_for(bc_tiles(op.bct), (small ? 4 : 2) * ncu));
                if (small && op.bct.wide)
                    GF2X_LAUNCH_N((k_bc_tile<1, 1>), g, kBcThreadsSmall, op.bct);
                else if (small)
                    GF2X_LAUNCH_N((k_bc_tile<0, 1>), g, kBcThreadsSmall, op.bct);
                else if (op.bct.wide)
                    GF2X_LAUNCH_N((k_bc_tile<1, 0>), g, kThreads, op.bct);
                else
                    GF2X_LAUNCH_N((k_bc_tile<0, 0>), g, kThreads, op.bct);
                break;
            }
            case OpKind::BcLayer: {
                uint64_t items = op.bcl.nelem / 2;
                uint64_t blocks = (items + kThreads - 1) / kThreads;
                if (op.bcl.wide)
                    GF2X_LAUNCH(k_bc_layer<1>, dim3(grid_for(blocks, 16 * ncu)), op.bcl);
                else
                    GF2X_LAUNCH(k_bc_layer<0>, dim3(grid_for(blocks, 16 * ncu)), op.bcl);
                break;
            }
            case OpKind::Fft:
                if (mate) {
                    const uint32_t nA = (uint32_t)fft_tiles(op.fft);
                    const dim3 g((unsigned)(nA + fft_tiles(mate->fft)));
                    if (op.fft.phi_in == kPhi64)
                        GF2X_LAUNCH(k_fft_pair<1>, g, op.fft, mate->fft, nA, (const uint8_t*)ctx->d_mt,
                                    (const uint32_t*)ctx->d_lam, (const uint4*)ctx->d_phi);
                    else if (op.fft.phi_in != kPhiNone)
                        GF2X_LAUNCH(k_fft_pair<2>, g, op.fft, mate->fft, nA, (const uint8_t*)ctx->d_mt,
                                    (const uint32_t*)ctx->d_lam, (const uint4*)ctx->d_phi);
                    else
                        GF2X_LAUNCH(k_fft_pair<0>, g, op.fft, mate->fft, nA, (const uint8_t*)ctx->d_mt,
                                    (const uint32_t*)ctx->d_lam, (const uint4*)ctx->d_phi);
                } else if (op.fft.phi_in == kPhi64)
                    GF2X_LAUNCH(k_fft<1>, dim3(grid_for(fft_tiles(op.fft), ncu)), op.fft,
                                (const uint8_t*)ctx->d_mt, (const uint32_t*)ctx->d_lam, (const uint4*)ctx->d_phi);
                else if (op.fft.phi_in != kPhiNone)
                    GF2X_LAUNCH(k_fft<2>, dim3(grid_for(fft_tiles(op.fft), ncu)), op.fft,
                                (const uint8_t*)ctx->d_mt, (const uint32_t*)ctx->d_lam, (const uint4*)ctx->d_phi);
                else
                    GF2X_LAUNCH(k_fft<0>, dim3(grid_for(fft_tiles(op.fft), ncu)), op.fft,
                                (const uint8_t*)ctx->d_mt, (const uint32_t*)ctx->d_lam, (const uint4*)ctx->d_phi);
                break;
            case OpKind::Pmul:
                GF2X_LAUNCH(k_pmul, dim3(grid_for(pmul_tiles(op.pmul), 2 * ncu)), op.pmul,
                                   (const uint8_t*)ctx->d_mt, (const uint32_t*)ctx->d_ctab);
                break;
            case OpKind::BcClass: {
                const bool small = (uint64_t)op.bcc.q_rows * op.bcc.w <=
                                   (1ull << ((op.bcc.wide ? kBcTileLog128 : kBcTileLog64) - kBcSmallShift));
                const dim3 g(grid_for(bc_class_tiles(op.bcc), (small ? 4 : 2) * ncu));
                if (small && op.bcc.wide)
                    GF2X_LAUNCH_N((k_bc_class<1, 1>), g, kBcThreadsSmall, op.bcc);
                else if (small)
                    GF2X_LAUNCH_N((k_bc_class<0, 1>), g, kBcThreadsSmall, op.bcc);
                else if (op.bcc.wide)
                    GF2X_LAUNCH_N((k_bc_class<1, 0>), g, kThreads, op.bcc);
                else
                    GF2X_LAUNCH_N((k_bc_class<0, 0>), g, kThreads, op.bcc);
                break;
            }
            case OpKind::Psi:
                GF2X_LAUNCH(k_psi, dim3(grid_for(psi_tiles(op.psi), 2 * ncu)), op.psi,
                                   (const uint4*)ctx->d_psi);
                break;
            case OpKind::Spine:
                GF2X_LAUNCH(k_spine, dim3(grid_for(spine_tiles(op.spn), 2 * ncu)), op.spn,
                                   (const uint8_t*)ctx->d_mt, (const uint4*)ctx->d_phi);
                break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(ctx, e, "kernel launch");
        if (traced) ctx->trace.push_back(pend);
        if (mate) ++oi;
    }
    return GF2X_OK;
}

// Upload every group's op array and tile prefix sums in one copy.
// Descriptor image of a list of groups: per group the op records of its kind
// and their tile prefix sums, at 256-byte aligned offsets of `host`.
void pack_groups(const std::vector<Op>& ops, const std::vector<BatchGroup>& groups, std::vector<char>& host,
                 std::vector<LaunchGroup>& out) {
    auto put = [&](const void* p, size_t n) {
        size_t off = (host.size() + 255) & ~(size_t)255;
        host.resize(off + n);
        memcpy(host.data() + off, p, n);
        return off;
    };
    std::vector<uint64_t> prefix;
    for (const BatchGroup& G : groups) {
        LaunchGroup d{};
        d.kind = G.kind;
        d.wide = G.wide;
        d.nops = (int)G.ops.size();
        prefix.assign(G.ops.size() + 1, 0);
        for (size_t i = 0; i < G.ops.size(); ++i) prefix[i + 1] = prefix[i] + op_tiles(ops[G.ops[i]]);
        d.total = prefix.back();
        auto gather = [&](auto member) {
            using T = std::decay_t<decltype(ops[0].*member)>;
            std::vector<T> v;
            v.reserve(G.ops.size());
            for (uint32_t i : G.ops) v.push_back(ops[i].*member);
            return put(v.data(), v.size() * sizeof(T));
        };
        switch (G.kind) {
            case OpKind::Pack: d.ops_off = gather(&Op::pack); break;
            case OpKind::BcTile: d.ops_off = gather(&Op::bct); break;
            case OpKind::BcLayer:
                for (uint32_t i : G.ops) d.layers.push_back(ops[i].bcl);
                break;
            case OpKind::Fft: d.ops_off = gather(&Op::fft); break;
            case OpKind::Pmul: d.ops_off = gather(&Op::pmul); break;
            case OpKind::Psi: d.ops_off = gather(&Op::psi); break;
            case OpKind::BcClass: d.ops_off = gather(&Op::bcc); break;
            case OpKind::Spine: d.ops_off = gather(&Op::spn); break;
        }
        d.prefix_off = put(prefix.data(), prefix.size() * sizeof(uint64_t));
        out.push_back(std::move(d));
    }
}

// One multi-op launch per group, in order, reading the descriptor image at `desc`.
int launch_groups(gf2x_ctx* ctx, const std::vector<LaunchGroup>& groups, const char* desc, hipStream_t st) {
    const uint64_t ncu = (uint64_t)ctx->ncu;
    for (const auto& G : groups) {
        const uint64_t* prefix = (const uint64_t*)(desc + G.prefix_off);
        const void* ops = desc + G.ops_off;
        switch (G.kind) {
            case OpKind::Pack:
                hipLaunchKernelGGL(k_pack_multi, dim3(grid_for(G.total, 8 * ncu)), dim3(kThreads), 0, st,
                                   (const PackOp*)ops, prefix, G.nops, G.total);
                break;
            case OpKind::BcTile:
                if (G.wide)
                    hipLaunchKernelGGL(k_bc_tile_multi<1>, dim3(grid_for(G.total, 2 * ncu)), dim3(kThreads), 0, st,
                                       (const BcTileOp*)ops, prefix, G.nops, G.total);
                else
                    hipLaunchKernelGGL(k_bc_tile_multi<0>, dim3(grid_for(G.total, 2 * ncu)), dim3(kThreads), 0, st,
                                       (const BcTileOp*)ops, prefix, G.nops, G.total);
                break;
            case OpKind::BcClass:
                if (G.wide)
                    hipLaunchKernelGGL(k_bc_class_multi<1>, dim3(grid_for(G.total, 2 * ncu)), dim3(kThreads), 0, st,
                                       (const BcClassOp*)ops, prefix, G.nops, G.total);
                else
                    hipLaunchKernelGGL(k_bc_class_multi<0>, dim3(grid_for(G.total, 2 * ncu)), dim3(kThreads), 0, st,
                                       (const BcClassOp*)ops, prefix, G.nops, G.total);
                break;
            case OpKind::BcLayer:
                // global layers (only for very long jobs): one launch per op
                for (const BcLayerOp& L : G.layers) {
                    uint64_t blocks = (L.nelem / 2 + kThreads - 1) / kThreads;
                    if (L.wide)
                        hipLaunchKernelGGL(k_bc_layer<1>, dim3(grid_for(blocks, 16 * ncu)), dim3(kThreads), 0, st, L);
                    else
                        hipLaunchKernelGGL(k_bc_layer<0>, dim3(grid_for(blocks, 16 * ncu)), dim3(kThreads), 0, st, L);
                }
                break;
            case OpKind::Fft:
                hipLaunchKernelGGL(k_fft_multi, dim3(grid_for(G.total, ncu)), dim3(kThreads), 0, st, (const FftPass*)ops,
                                   prefix, G.nops, G.total, (const uint8_t*)ctx->d_mt, (const uint32_t*)ctx->d_lam,
                                   (const uint4*)ctx->d_phi);
                break;
            case OpKind::Pmul:
                hipLaunchKernelGGL(k_pmul_multi, dim3(grid_for(G.total, 2 * ncu)), dim3(kThreads), 0, st,
                                   (const PmulOp*)ops, prefix, G.nops, G.total, (const uint8_t*)ctx->d_mt,
                                   (const uint32_t*)ctx->d_ctab);
                break;
            case OpKind::Psi:
                hipLaunchKernelGGL(k_psi_multi, dim3(grid_for(G.total, 2 * ncu)), dim3(kThreads), 0, st,
                                   (const PsiOp*)ops, prefix, G.nops, G.total, (const uint4*)ctx->d_psi);
                break;
            case OpKind::Spine:
                hipLaunchKernelGGL(k_spine_multi, dim3(grid_for(G.total, 2 * ncu)), dim3(kThreads), 0, st,
                                   (const SpineOp*)ops, prefix, G.nops, G.total, (const uint8_t*)ctx->d_mt,
                                   (const uint4*)ctx->d_phi);
                break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(ctx, e, "batch launch");
    }
    return GF2X_OK;
}

int batch_upload(gf2x_batch* B) {
    gf2x_ctx* ctx = B->ctx;
    std::vector<char> host;
    B->groups.clear();
    pack_groups(B->plan.ops, B->plan.groups, host, B->groups);
    B->desc_bytes = host.size();
    hipError_t e = hipMalloc((void**)&B->desc, std::max<size_t>(host.size(), 256));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, GF2X_ENOMEM, "batch descriptors");
    }
    if (!host.empty()) {
        e = hipMemcpy(B->desc, host.data(), host.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(ctx, e, "batch descriptor upload");
    }
    return GF2X_OK;
}

int batch_launch_groups(gf2x_batch* B, hipStream_t st) { return launch_groups(B->ctx, B->groups, B->desc, st); }

// The device form of an op (its record and tile count).
DevOp make_devop(const Op& op) {
    DevOp d;
    memset(&d, 0, sizeof(d));
    d.kind = (int)op.kind;
    d.wide = op_wide(op);
    d.tiles = (uint32_t)(op.kind == OpKind::BcLayer ? 1 : op_tiles(op));
    switch (op.kind) {
        case OpKind::Pack: d.pack = op.pack; break;
        case OpKind::BcTile: d.bct = op.bct; break;
        case OpKind::BcLayer: d.bcl = op.bcl; break;
        case OpKind::Fft: d.fft = op.fft; break;
        case OpKind::Pmul: d.pmul = op.pmul; break;
        case OpKind::Psi: d.psi = op.psi; break;
        case OpKind::BcClass: d.bcc = op.bcc; break;
        case OpKind::Spine: d.spn = op.spn; break;
    }
    return d;
}

// Persistent descriptor image: one array of DevOp in item order (group after
// group, so rank by rank), the op and rank item prefixes, then the scheduler
// words (abort flag, per-rank arrive counters, per-rank 64-bit item counters).
// The image is appended to `host` at a 256-byte aligned offset `base`.
void pack_persistent(const std::vector<Op>& ops, const std::vector<uint32_t>& rank_of,
                     const std::vector<BatchGroup>& groups, std::vector<char>& host, size_t& base, PersistLayout& L) {
    std::vector<DevOp> dops;
    std::vector<uint64_t> prefix(1, 0);
    std::vector<uint64_t> rank_first;
    uint32_t cur_rank = ~0u;
    for (const BatchGroup& G : groups)
        for (uint32_t i : G.ops) {
            const Op& op = ops[i];
            if (rank_of[i] != cur_rank) {
                cur_rank = rank_of[i];
                rank_first.push_back(prefix.back());
            }
            const DevOp d = make_devop(op);
            dops.push_back(d);
            prefix.push_back(prefix.back() + d.tiles);
        }
    rank_first.push_back(prefix.back());
    L = PersistLayout();
    L.nranks = (int)rank_first.size() - 1;
    L.nops = (int)dops.size();
    L.items = prefix.back();
    size_t off = 0;
    L.ops_off = off;
    off = align256(off + dops.size() * sizeof(DevOp));
    L.prefix_off = off;
    off = align256(off + prefix.size() * sizeof(uint64_t));
    L.rank_off = off;
    off = align256(off + rank_first.size() * sizeof(uint64_t));
    L.state_off = off;
    L.state_words = 2 + 3 * (size_t)L.nranks;  // abort, pad, arrive[nranks], next[nranks] (64-bit)
    if (L.state_words & 1) ++L.state_words;
    off = align256(off + L.state_words * sizeof(uint32_t));
    L.bytes = off;
    base = align256(host.size());
    host.resize(base + off, 0);
    char* h = host.data() + base;
    memcpy(h + L.ops_off, dops.data(), dops.size() * sizeof(DevOp));
    memcpy(h + L.prefix_off, prefix.data(), prefix.size() * sizeof(uint64_t));
    memcpy(h + L.rank_off, rank_first.data(), rank_first.size() * sizeof(uint64_t));
}

PersistArgs persist_args(const char* dev, const PersistLayout& L, uint32_t spin_limit) {
    PersistArgs a;
    a.ops = (const DevOp*)(dev + L.ops_off);
    a.prefix = (const uint64_t*)(dev + L.prefix_off);
    a.rank_first = (const uint64_t*)(dev + L.rank_off);
    a.nops = L.nops;
    a.nranks = L.nranks;
    a.items = L.items;
    uint32_t* st = (uint32_t*)(dev + L.state_off);
    a.abort = st;
    a.arrive = st + 2;
    size_t nxt = 2 + (size_t)L.nranks;
    if (nxt & 1) ++nxt;
    a.next = (unsigned long long*)(st + nxt);
    a.spin_limit = spin_limit;
    return a;
}

// Clears the scheduler words with a kernel (so the sequence can sit inside a
// graph), then launches one persistent block per CU.
int launch_persistent(gf2x_ctx* ctx, char* dev, const PersistLayout& L, uint32_t spin_limit, hipStream_t st) {
    if (!L.items) return GF2X_OK;
    if (ctx->persist_per_cu < 1)
        return fail(ctx, GF2X_EDEVICE, "the persistent kernel does not fit a compute unit (occupancy 0)");
    PersistArgs a = persist_args(dev, L, spin_limit);
    hipLaunchKernelGGL(k_zero_u32, dim3(grid_for((L.state_words + kThreads - 1) / kThreads, 64)), dim3(kThreads), 0, st,
                       (uint32_t*)(dev + L.state_off), (uint64_t)L.state_words);
    hipLaunchKernelGGL(k_persistent, dim3((unsigned)std::max(1, ctx->ncu)), dim3(kThreads), 0, st, a,
                       (const uint8_t*)ctx->d_mt, (const uint32_t*)ctx->d_lam, (const uint4*)ctx->d_phi,
                       (const uint4*)ctx->d_psi, (const uint32_t*)ctx->d_ctab);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "persistent launch");
    return GF2X_OK;
}

int batch_upload_persistent(gf2x_batch* B) {
    gf2x_ctx* ctx = B->ctx;
    std::vector<char> host;
    size_t base = 0;
    pack_persistent(B->plan.ops, B->plan.rank_of, B->plan.groups, host, base, B->play);
    hipError_t e = hipMalloc((void**)&B->pdesc, std::max<size_t>(host.size(), 256));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, GF2X_ENOMEM, "persistent batch descriptors");
    }
    e = hipMemcpy(B->pdesc, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(ctx, e, "persistent descriptor upload");
    return GF2X_OK;
}

int batch_launch_persistent(gf2x_batch* B, hipStream_t st) {
    return launch_persistent(B->ctx, B->pdesc, B->play, B->spin_limit, st);
}

void batch_free(gf2x_batch* B) {
    if (!B) return;
    if (B->pdesc) (void)hipFree(B->pdesc);
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    if (B->ws) (void)hipFree(B->ws);
    if (B->desc) (void)hipFree(B->desc);
    delete B;
}

int check_jobs(gf2x_ctx* ctx, const gf2x_job* jobs, size_t njobs) {
    for (size_t j = 0; j < njobs; ++j) {
        const gf2x_job& J = jobs[j];
        Sizes s = make_sizes(J.na_bits, J.nb_bits, ctx->params.word_bits);
        if (!s.out_words) continue;
        if (!J.a || !J.b || !J.c) return fail(ctx, GF2X_EINVAL, "NULL pointer in job " + std::to_string(j));
        if (s.m > 32) return fail(ctx, GF2X_ERANGE, "job " + std::to_string(j) + " too long");
        if (ranges_overlap(J.c, 8 * s.out_words, J.a, 8 * s.n_a) || ranges_overlap(J.c, 8 * s.out_words, J.b, 8 * s.n_b))
            return fail(ctx, GF2X_EINVAL, "job " + std::to_string(j) + ": product overlaps an operand");
    }
    return GF2X_OK;
}

int batch_build(gf2x_ctx* ctx, const gf2x_job* jobs, size_t njobs, int mode, gf2x_batch** out) {
    std::vector<BatchJob> bj(njobs);
    for (size_t j = 0; j < njobs; ++j) bj[j] = BatchJob{jobs[j].a, jobs[j].na_bits, jobs[j].b, jobs[j].nb_bits, jobs[j].c};
    gf2x_batch* B = new gf2x_batch();
    B->ctx = ctx;
    plan_batch(B->plan, ctx->pool, ctx->params, bj.data(), njobs, nullptr);
    if (B->plan.ws_bytes) {
        hipError_t e = hipMalloc((void**)&B->ws, B->plan.ws_bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            batch_free(B);
            return fail(ctx, GF2X_ENOMEM, "batch workspace of " + std::to_string(B->plan.ws_bytes) + " bytes");
        }
    }
    plan_batch(B->plan, ctx->pool, ctx->params, bj.data(), njobs, B->ws);
    B->mode = mode;
    int rc = batch_upload(B);
    if (!rc && mode == GF2X_BATCH_PERSISTENT) rc = batch_upload_persistent(B);
    if (rc) {
        batch_free(B);
        return rc;
    }
    *out = B;
    return GF2X_OK;
}

constexpr int kMaxLog2N = 32;  // multipliers s_i(v_t) are tabulated for t < 32
// Single products of 2^15 to 2^19 points overlap their two forward
// transforms on two streams: below that the two transforms run interleaved on
// one stream with their FFT passes paired (run_product), which beats the
// fork and join (2^18-bit products 0.148 -> 0.131 ms, 2^19-bit 0.177 ->
// 0.171); above it each transform fills the device on its own (the overlap
// still saves about 2 % at 2^23 points, but then no kernel's time can be read
// on its own).
constexpr int kForkMinLog = 15, kForkMaxLog = 19;

int check_ctx(gf2x_ctx* ctx) { return ctx ? GF2X_OK : GF2X_EINVAL; }

std::mutex g_default_mu;
gf2x_ctx* g_default = nullptr;

// ------------------------------------------------------------------ serving
uint64_t now_ns() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

void server_free(gf2x_server* S) {
    if (!S) return;
    for (auto& sl : S->slots) {
        if (sl.host) (void)hipHostFree(sl.host);
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.ev) (void)hipEventDestroy(sl.ev);
    }
    if (S->arena) (void)hipFree(S->arena);
    if (S->st) (void)hipStreamDestroy(S->st);
    for (hipEvent_t ev : S->all_events) (void)hipEventDestroy(ev);
    delete S;
}

// After a device failure every request still held completes with `status`
// and the server accepts no more work.
void server_fail_all(gf2x_server* S, int status) {
    S->sticky = status;
    const uint64_t t = now_ns();
    for (int i : S->inflight) {
        for (auto d : S->slots[i].fin) {
            d.status = status;
            d.t_done_ns = t;
            S->done.push_back(d);
            ++S->stats.completed;
        }
        S->slots[i].fin.clear();
    }
    auto finish = [&](gf2x_server::Req& r) {
        if (r.ready) S->free_events.push_back(r.ready);
        r.ready = nullptr;
        S->done.push_back(gf2x_done{r.tag, status, r.iters, r.t_submit, r.t_admit, t});
        ++S->stats.completed;
    };
    for (auto& r : S->active) finish(r);
    for (auto& r : S->queue) finish(r);
    S->active.clear();
    S->queue.clear();
}

// Completes every finished iteration, oldest first.
int server_retire(gf2x_server* S) {
    while (!S->inflight.empty()) {
        const int i = S->inflight.front();
        gf2x_server::Slot& sl = S->slots[i];
        hipError_t e = hipEventQuery(sl.ev);
        if (e == hipErrorNotReady) break;
        int status = GF2X_OK;
        if (e != hipSuccess)
            status = hip_fail(S->ctx, e, "serving iteration");
        else if (sl.persistent && *(volatile uint32_t*)(sl.host + sl.abort_off))
            status = fail(S->ctx, GF2X_EDEVICE, "serving iteration: a persistent barrier wait timed out");
        const uint64_t t = now_ns();
        for (auto d : sl.fin) {
            d.status = status;
            d.t_done_ns = t;
            S->done.push_back(d);
            ++S->stats.completed;
        }
        sl.fin.clear();
        S->inflight.pop_front();
        S->free_slots.push_back(i);
        if (status) {
            server_fail_all(S, status);
            return status;
        }
    }
    return GF2X_OK;
}

// First come, first served: admits the head of the queue while a slot is free
// and its footprint fits in the arena.
void server_admit(gf2x_server* S) {
    gf2x_ctx* ctx = S->ctx;
    while (!S->queue.empty() && S->active.size() < S->cfg.max_active) {
        gf2x_server::Req& q = S->queue.front();
        const size_t off = S->alloc.alloc(q.bytes);
        if (off == Arena::npos) break;
        q.off = off;
        q.t_admit = now_ns();
        const Sizes s = make_sizes(q.na, q.nb, q.w);
        q.ops.clear();
        plan_mul(q.ops, ctx->pool, ctx->params, s, q.a, q.b, q.c, S->arena + off);
        q.levels = plan_levels(q.ops);
        q.level_tiles.assign(q.levels, 0);
        for (const Op& op : q.ops) q.level_tiles[op.level] += op_tiles(op);
        S->active.push_back(std::move(q));
        S->queue.pop_front();
        ++S->stats.admitted;
    }
    S->stats.active_peak = std::max<uint64_t>(S->stats.active_peak, S->active.size());
    S->stats.arena_peak = std::max<uint64_t>(S->stats.arena_peak, S->alloc.used());
}

int server_ensure_slot(gf2x_server* S, gf2x_server::Slot& sl, size_t need) {
    if (need <= sl.cap) return GF2X_OK;
    const size_t cap = std::max<size_t>(need, 2 * sl.cap);
    if (sl.host) (void)hipHostFree(sl.host);
    if (sl.dev) (void)hipFree(sl.dev);
    sl.host = nullptr;
    sl.dev = nullptr;
    sl.cap = 0;
    hipError_t e = hipHostMalloc((void**)&sl.host, cap, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&sl.dev, cap);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(S->ctx, GF2X_ENOMEM, "serving descriptor buffers");
    }
    sl.cap = cap;
    return GF2X_OK;
}

// Admits, then advances every admitted request by up to levels_per_iter
// levels in one iteration queued on the server's stream.  Arena space of a
// request that finishes here is reused at once: later iterations run after
// this one on the same stream.
int server_iterate(gf2x_server* S, bool& launched) {
    launched = false;
    server_admit(S);
    if (S->active.empty()) return GF2X_OK;
    launched = true;
    const int si = S->free_slots.back();
    gf2x_server::Slot& sl = S->slots[si];
    uint32_t L = S->cfg.levels_per_iter;
    // adaptive mode, light load (nothing queued, at most kLightActive
    // requests admitted): they run all their remaining levels in this
    // iteration, as plain calls would (too few to gain from sharing launches)
    constexpr size_t kLightActive = 2;
    const bool idle = S->cfg.mode == GF2X_SERVER_ADAPTIVE && S->queue.empty() && S->active.size() <= kLightActive;
    if (idle) {
        for (const auto& r : S->active) L = std::max<uint32_t>(L, r.levels - r.next);
    } else if (S->cfg.iter_tiles) {
        // as many levels as fit the work bound (at least one)
        uint64_t acc = 0;
        uint32_t l = 0;
        while (l < L) {
            uint64_t add = 0;
            for (const auto& r : S->active)
                if (r.next + l < r.levels) add += r.level_tiles[r.next + l];
            if (add == 0 || (l > 0 && acc + add > S->cfg.iter_tiles)) break;
            acc += add;
            ++l;
        }
        L = std::max<uint32_t>(l, 1);
    }
    // a lone request starting on a lightly loaded engine runs as a plain call
    // does: replanned with the single-product tiles, one launch per op, no
    // descriptor upload (its arena region fits either plan)
    const bool direct = idle && S->active.size() == 1 && S->active[0].next == 0;
    std::vector<Op> direct_ops;
    size_t direct_split[2] = {0, 0};
    int direct_m = 0;
    if (direct) {
        const gf2x_server::Req& r = S->active[0];
        const PlanParams pp = single_params(S->ctx);
        const Sizes sz = make_sizes(r.na, r.nb, r.w);
        direct_m = sz.m;
        plan_mul(direct_ops, S->ctx->pool, pp, sz, r.a, r.b, r.c, S->arena + r.off, direct_split);
    }
    S->it_ops.clear();
    S->it_rank.clear();
    // requests starting in this iteration: their operands are ready once the
    // work enqueued on the submitter's stream before the submit is done (one
    // wait per distinct stream, on its newest event: submits are admitted in
    // order)
    std::vector<std::pair<hipStream_t, hipEvent_t>> waits;
    for (auto& r : S->active) {
        if (r.next != 0 || !r.ready) continue;
        if (hipEventQuery(r.ready) == hipSuccess) {
            // the submitter's work is already done: nothing to wait for
            S->free_events.push_back(r.ready);
            r.ready = nullptr;
            continue;
        }
        (void)hipGetLastError();
        bool found = false;
        for (auto& w : waits)
            if (w.first == r.src) {
                S->free_events.push_back(w.second);
                w.second = r.ready;
                found = true;
            }
        if (!found) waits.push_back({r.src, r.ready});
        r.ready = nullptr;
    }
    std::vector<gf2x_server::Req> keep;
    keep.reserve(S->active.size());
    for (auto& r : S->active) {
        for (const Op& op : r.ops)
            if (op.level >= r.next && op.level - r.next < L) {
                S->it_ops.push_back(op);
                S->it_rank.push_back(op.level - r.next);
            }
        r.next += L;
        ++r.iters;
        if (r.next >= r.levels) {
            sl.fin.push_back(gf2x_done{r.tag, GF2X_OK, r.iters, r.t_submit, r.t_admit, 0});
            S->alloc.release(r.off, r.bytes);
        } else {
            keep.push_back(std::move(r));
        }
    }
    S->active.swap(keep);
    if (direct) {
        S->free_slots.pop_back();
        S->inflight.push_back(si);
        sl.persistent = false;
        hipStream_t st = S->st;
        hipError_t e = hipSuccess;
        for (auto& w : waits) {
            if (e == hipSuccess) e = hipStreamWaitEvent(st, w.second, 0);
            S->free_events.push_back(w.second);
        }
        if (e != hipSuccess) return hip_fail(S->ctx, e, "serving: wait for the submitters' streams");
        int rc = run_product(S->ctx, direct_ops, direct_split, direct_m, st, true);
        if (rc) return rc;
        S->stats.launches += direct_ops.size();  // ops (paired passes and a merged tail launch fewer)
        e = hipEventRecord(sl.ev, st);
        if (e != hipSuccess) return hip_fail(S->ctx, e, "serving event");
        ++S->stats.iterations;
        return GF2X_OK;
    }
    S->it_groups.clear();
    group_by_rank(S->it_ops, S->it_rank, 0, L, S->it_groups);
    S->it_host.clear();
    S->it_launch.clear();
    PersistLayout PL;
    size_t base = 0;
    const size_t admitted = S->active.size() + sl.fin.size();
    const bool pers = S->cfg.mode == GF2X_BATCH_PERSISTENT ||
                      (S->cfg.mode == GF2X_SERVER_ADAPTIVE && admitted >= GF2X_SERVER_ADAPTIVE_ACTIVE &&
                       S->queue.size() < GF2X_SERVER_ADAPTIVE_BACKLOG);
    if (pers)
        pack_persistent(S->it_ops, S->it_rank, S->it_groups, S->it_host, base, PL);
    else
        pack_groups(S->it_ops, S->it_groups, S->it_host, S->it_launch);
    const size_t image = S->it_host.size();
    sl.abort_off = align256(image);
    // queued from here on: a failure below reports this iteration's requests
    S->free_slots.pop_back();
    S->inflight.push_back(si);
    int rc = server_ensure_slot(S, sl, sl.abort_off + 256);
    if (rc) return rc;
    sl.persistent = pers;
    memcpy(sl.host, S->it_host.data(), image);
    *(uint32_t*)(sl.host + sl.abort_off) = 0;
    hipStream_t st = S->st;
    hipError_t e = hipSuccess;
    for (auto& w : waits) {
        if (e == hipSuccess) e = hipStreamWaitEvent(st, w.second, 0);
        S->free_events.push_back(w.second);
    }
    if (e != hipSuccess) return hip_fail(S->ctx, e, "serving: wait for the submitters' streams");
    if (image) e = hipMemcpyAsync(sl.dev, sl.host, image, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(S->ctx, e, "serving descriptor upload");
    if (pers) {
        rc = launch_persistent(S->ctx, sl.dev, PL, S->spin_limit, st);
        if (rc) return rc;
        if (PL.items) {
            e = hipMemcpyAsync(sl.host + sl.abort_off, sl.dev + PL.state_off, 4, hipMemcpyDeviceToHost, st);
            if (e != hipSuccess) return hip_fail(S->ctx, e, "serving abort flag copy");
            S->stats.launches += 2;
        }
    } else {
        rc = launch_groups(S->ctx, S->it_launch, sl.dev, st);
        if (rc) return rc;
        for (const auto& G : S->it_launch) S->stats.launches += G.kind == OpKind::BcLayer ? G.layers.size() : 1;
    }
    e = hipEventRecord(sl.ev, st);
    if (e != hipSuccess) return hip_fail(S->ctx, e, "serving event");
    ++S->stats.iterations;
    return GF2X_OK;
}

// ------------------------------------------------------------------ autotuner
// Forward + inverse FFT passes of `copies` independent 2^M-point transforms
// laid out in `scratch`, grouped by pass as a batch would run them.
void tune_ops(const PlanParams& pp, int M, int copies, char* scratch, std::vector<Op>& ops,
              std::vector<BatchGroup>& groups) {
    const size_t wbytes = align256(8ull << M), per = wbytes + align256(16ull << M);
    std::vector<uint32_t> rank;
    ops.clear();
    groups.clear();
    uint32_t nr = 0;
    for (int c = 0; c < copies; ++c) {
        uint64_t* words = (uint64_t*)(scratch + (size_t)c * per);
        uint4* spec = (uint4*)(scratch + (size_t)c * per + wbytes);
        const size_t f = ops.size();
        emit_fft_forward(ops, pp, words, spec, M, 0);
        emit_fft_inverse(ops, pp, spec, M);
        for (size_t i = f; i < ops.size(); ++i) rank.push_back((uint32_t)(i - f));
        nr = std::max<uint32_t>(nr, (uint32_t)(ops.size() - f));
    }
    group_by_rank(ops, rank, 0, nr, groups);
}

struct TuneBuffers {
    char* scratch = nullptr;
    char* desc = nullptr;
    size_t desc_cap = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~TuneBuffers() {
        if (scratch) (void)hipFree(scratch);
        if (desc) (void)hipFree(desc);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

// Average time (us) of one run of the candidate's launches, or < 0 on error.
int tune_time(gf2x_ctx* ctx, TuneBuffers& T, const PlanParams& pp, int M, int copies, int reps, float& us) {
    std::vector<Op> ops;
    std::vector<BatchGroup> groups;
    tune_ops(pp, M, copies, T.scratch, ops, groups);
    std::vector<char> host;
    std::vector<LaunchGroup> launch;
    pack_groups(ops, groups, host, launch);
    if (host.size() > T.desc_cap) {
        if (T.desc) (void)hipFree(T.desc);
        T.desc = nullptr;
        T.desc_cap = 0;
        if (hipMalloc((void**)&T.desc, host.size()) != hipSuccess) {
            (void)hipGetLastError();
            return fail(ctx, GF2X_ENOMEM, "autotune descriptors");
        }
        T.desc_cap = host.size();
    }
    hipStream_t st = ctx->own_stream;
    hipError_t e = hipMemcpy(T.desc, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(ctx, e, "autotune upload");
    int rc = launch_groups(ctx, launch, T.desc, st);  // warm-up
    if (rc) return rc;
    e = hipEventRecord(T.e0, st);
    for (int r = 0; r < reps && e == hipSuccess && !rc; ++r) rc = launch_groups(ctx, launch, T.desc, st);
    if (rc) return rc;
    if (e == hipSuccess) e = hipEventRecord(T.e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(T.e1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, T.e0, T.e1);
    if (e != hipSuccess) return hip_fail(ctx, e, "autotune timing");
    us = 1000.0f * ms / (float)reps;
    return GF2X_OK;
}

}  // namespace

// ------------------------------------------------------------------ C ABI

// Plans of single products (run op by op on their own kernels) take the small
// BasisCvt tiles; batches and the server plan with ctx->params.
PlanParams single_params(const gf2x_ctx* ctx) {
    PlanParams pp = ctx->params;
    pp.bc_small = 1;
    pp.fft_pack_min_tiles = (uint32_t)ctx->ncu;
    pp.fuse_max_log = ctx->fuse_single_max_log;
    return pp;
}

// ------------------------------------------------ the simple variant (Alg. 4)

int launch_sfft(gf2x_ctx* ctx, const std::vector<SfftPass>& passes, hipStream_t st) {
    for (const SfftPass& p : passes) {
        if (p.lo == 0) {
            if (p.c != 2 && p.c != 3) return fail(ctx, GF2X_EINVAL, "simple-variant bottom pass: group size 2^c with c not 2 or 3");
            const uint64_t chunks = (p.n + (1ull << (p.c + 6)) - 1) >> (p.c + 6);
            const dim3 grid(grid_for(chunks, 18ull * ctx->ncu)), block(kSfGroupThreads);
            const uint4* cantor = (const uint4*)ctx->d_cantor;
            if (p.c == 2)
                if (p.inverse)
                    hipLaunchKernelGGL((k_sfft_lane<2, true>), grid, block, 0, st, p, cantor);
                else
                    hipLaunchKernelGGL((k_sfft_lane<2, false>), grid, block, 0, st, p, cantor);
            else if (p.inverse)
                hipLaunchKernelGGL((k_sfft_lane<3, true>), grid, block, 0, st, p, cantor);
            else
                hipLaunchKernelGGL((k_sfft_lane<3, false>), grid, block, 0, st, p, cantor);
        } else {
            const uint64_t groups = p.n >> (p.L + p.c);
            hipLaunchKernelGGL(k_sfft_tab, dim3(grid_for(groups, 12ull * ctx->ncu)), dim3(kSfThreads), 0, st, p,
                               (const uint4*)ctx->d_cantor);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(ctx, e, "simple-variant FFT launch");
    }
    return GF2X_OK;
}

// Split, BasisCvt on 64-bit words, FFT_LCH at the Cantor points (Alg. 4).
int simple_forward(gf2x_ctx* ctx, const uint64_t* src, uint64_t nbits, uint64_t* words, int m_op, uint4* spec, int m,
                   hipStream_t st) {
    std::vector<Op> ops;
    emit_pack(ops, src, nbits, words, 1ull << m_op);
    emit_bc(ops, ctx->pool, words, 0, m_op, 0, single_params(ctx).bc_small);
    int rc = run_ops(ctx, ops, st);
    if (rc) return rc;
    return launch_sfft(ctx, sfft_passes(spec, words, m_op, m, false), st);
}

int simple_mul(gf2x_ctx* ctx, const uint64_t* a, uint64_t na_bits, const uint64_t* b, uint64_t nb_bits, uint64_t* c,
               hipStream_t st) {
    const Sizes s = make_sizes(na_bits, nb_bits, 64);
    const Workspace w = workspace_for(s);
    int rc = ensure_ws(ctx, w.bytes, st);
    if (rc) return rc;
    uint64_t* wa = (uint64_t*)(ctx->ws + w.off_wa);
    uint64_t* wb = (uint64_t*)(ctx->ws + w.off_wb);
    uint4* sa = (uint4*)(ctx->ws + w.off_sa);
    uint4* sb = (uint4*)(ctx->ws + w.off_sb);
    const uint64_t N = 1ull << s.m;
    if ((rc = simple_forward(ctx, a, na_bits, wa, s.m_a, sa, s.m, st))) return rc;
    if ((rc = simple_forward(ctx, b, nb_bits, wb, s.m_b, sb, s.m, st))) return rc;
    hipLaunchKernelGGL(k_spmul, dim3(grid_for((N + kSfLaneThreads - 1) / kSfLaneThreads, 16ull * ctx->ncu)),
                       dim3(kSfLaneThreads), 0, st, (const uint4*)sa, (const uint4*)sb, sb, N);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "simple-variant pointmul launch");
    if ((rc = launch_sfft(ctx, sfft_passes(sb, nullptr, s.m, s.m, true), st))) return rc;
    std::vector<Op> ops;
    emit_bc(ops, ctx->pool, sb, 1, s.m, 1, single_params(ctx).bc_small);
    if ((rc = run_ops(ctx, ops, st))) return rc;
    hipLaunchKernelGGL(k_scombine, dim3(grid_for((s.out_words + kSfThreads - 1) / kSfThreads, 8ull * ctx->ncu)),
                       dim3(kSfThreads), 0, st, (const uint4*)sb, N, c, s.out_words, s.nc_bits);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "simple-variant combine launch");
    return GF2X_OK;
}

// ------------------------------ the Frobenius-partition variant (App. C)

int launch_zadic(gf2x_ctx* ctx, const std::vector<ZadicPass>& passes, hipStream_t st) {
    for (const ZadicPass& z : passes) {
        hipLaunchKernelGGL(k_zadic, dim3(grid_for(zadic_tiles(z), 4ull * ctx->ncu)), dim3(kZThreads), 0, st, z);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(ctx, e, "z-adic pass launch");
    }
    return GF2X_OK;
}

// E(a): Split into 2^W words, BasisCvt over the bits (z-adic expansion, the
// word-level conversion; the per-word map runs inside the encoding), the
// encoding, FFT_LCH at beta_{m+64} over the 2^m elements.
int frob_forward(gf2x_ctx* ctx, const uint64_t* src, uint64_t nbits, uint64_t* words, int W, uint4* spec, int m,
                 hipStream_t st) {
    std::vector<Op> ops;
    emit_pack(ops, src, nbits, words, 1ull << W);
    int rc = run_ops(ctx, ops, st);
    if (rc) return rc;
    if ((rc = launch_zadic(ctx, zadic_passes(words, W, false), st))) return rc;
    ops.clear();
    emit_bc(ops, ctx->pool, words, 0, W, 0, single_params(ctx).bc_small);
    if ((rc = run_ops(ctx, ops, st))) return rc;
    const FrobEncode F{words, spec, (uint32_t)W, (uint32_t)m};
    hipLaunchKernelGGL(k_fencode, dim3(grid_for(frob_tiles((uint32_t)m), 4ull * ctx->ncu)), dim3(kFeThreads), 0, st, F,
                       (const uint4*)ctx->d_frob);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "encoding launch");
    return launch_sfft(ctx, sfft_passes(spec, nullptr, m, m, false, m + 64), st);
}

// The inverse: iFFT_LCH at beta_{m+64}, the inverse encoding and per-word
// map into 2^(m+1) words, iBasisCvt of the words, the z-adic recomposition;
// the first ceil(nc_bits/64) words of the polynomial go to c.  spec is
// overwritten.
int frob_inverse(gf2x_ctx* ctx, uint4* spec, int m, uint64_t* words, uint64_t* c, uint64_t nc_bits, hipStream_t st) {
    int rc = launch_sfft(ctx, sfft_passes(spec, nullptr, m, m, true, m + 64), st);
    if (rc) return rc;
    const FrobDecode F{spec, words, (uint32_t)m};
    hipLaunchKernelGGL(k_fdecode, dim3(grid_for(frob_tiles((uint32_t)m), 4ull * ctx->ncu)), dim3(kFdThreads), 0, st, F,
                       (const uint4*)ctx->d_frob);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "decoding launch");
    std::vector<Op> ops;
    emit_bc(ops, ctx->pool, words, 0, m + 1, 1, single_params(ctx).bc_small);
    if ((rc = run_ops(ctx, ops, st))) return rc;
    return launch_zadic(ctx, zadic_passes(words, m + 1, true, c, (nc_bits + 63) / 64), st);
}

int frob_mul(gf2x_ctx* ctx, const FrobSizes& s, const uint64_t* a, const uint64_t* b, uint64_t* c, hipStream_t st) {
    const FrobWorkspace w = frob_workspace(s);
    int rc = ensure_ws(ctx, w.bytes, st);
    if (rc) return rc;
    uint64_t* wa = (uint64_t*)(ctx->ws + w.off_wa);
    uint64_t* wb = (uint64_t*)(ctx->ws + w.off_wb);
    uint4* sa = (uint4*)(ctx->ws + w.off_sa);
    uint4* sb = (uint4*)(ctx->ws + w.off_sb);
    const uint64_t n = 1ull << s.m;
    if ((rc = frob_forward(ctx, a, s.na_bits, wa, s.w_a, sa, s.m, st))) return rc;
    if ((rc = frob_forward(ctx, b, s.nb_bits, wb, s.w_b, sb, s.m, st))) return rc;
    hipLaunchKernelGGL(k_spmul, dim3(grid_for((n + kSfLaneThreads - 1) / kSfLaneThreads, 16ull * ctx->ncu)),
                       dim3(kSfLaneThreads), 0, st, (const uint4*)sa, (const uint4*)sb, sb, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "Frobenius-variant pointmul launch");
    // the decoded words overwrite sa (2^(m+1) words = 16 n bytes)
    return frob_inverse(ctx, sb, s.m, (uint64_t*)sa, c, s.nc_bits, st);
}

extern "C" {

const char* gf2x_strerror(int status) {
    switch (status) {
        case GF2X_OK: return "ok";
        case GF2X_EINVAL: return "invalid argument";
        case GF2X_ERANGE: return "size out of range";
        case GF2X_ENOMEM: return "out of device memory";
        case GF2X_EDEVICE: return "HIP device error";
        default: return "unknown status";
    }
}

const char* gf2x_last_error(gf2x_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

size_t gf2x_out_words(uint64_t na_bits, uint64_t nb_bits) { return (size_t)make_sizes(na_bits, nb_bits).out_words; }

int gf2x_fft_log2(uint64_t na_bits, uint64_t nb_bits) {
    if (!na_bits || !nb_bits) return -1;
    return make_sizes(na_bits, nb_bits).m;
}

size_t gf2x_workspace_bytes(uint64_t na_bits, uint64_t nb_bits) {
    if (!na_bits || !nb_bits) return 0;
    return workspace_for(make_sizes(na_bits, nb_bits)).bytes;
}

size_t gf2x_workspace_bytes_w(uint64_t na_bits, uint64_t nb_bits, int w) {
    if (!na_bits || !nb_bits || (w != 64 && w != 128)) return 0;
    return workspace_for(make_sizes(na_bits, nb_bits, w)).bytes;
}

int gf2x_ctx_create(gf2x_ctx** out, int device) {
    if (!out) return GF2X_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return GF2X_EDEVICE;
    }
    gf2x_ctx* ctx = new gf2x_ctx();
    ctx->device = device;
    DeviceGuard g(device);
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
        ctx->ncu = ncu;

    HostTower T;
    std::vector<uint8_t> mt(65536);
    for (int a = 0; a < 256; ++a)
        for (int b = 0; b < 256; ++b) mt[a * 256 + b] = T.mt8[a][b];
    uint32_t lam[32][32];
    build_lambda(T, lam);
    memcpy(ctx->h_lam, lam, sizeof(lam));
    ctx->h_mt = mt;
    ctx->params.lam = ctx->h_lam;
    ctx->params.mt = ctx->h_mt.data();
    ReprTables R = build_repr(T);
    if (!R.ok) {
        delete ctx;
        return GF2X_EINVAL;
    }
    // changeRepr: the nibble tables of every mode; changeRepr back: the w = 64
    // byte tables, then the w = 128 nibble tables
    std::vector<uint4> phi(kPhinTotal), psi(kPsiTab64 + kPsiTab128);
    for (int i = 0; i < kPhinTotal; ++i) phi[i] = to_u4(R.phin[i]);
    for (int i = 0; i < kPsiTab64; ++i) psi[i] = to_u4(R.psi[i]);
    for (int i = 0; i < kPsiTab128; ++i) psi[kPsiTab64 + i] = to_u4(R.psin[i]);

    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_mt, 65536);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_lam, sizeof(lam));
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_phi, phi.size() * sizeof(uint4));
    const std::vector<uint32_t> ctab = build_const_tabs(T);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_psi, psi.size() * sizeof(uint4));
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_ctab, ctab.size() * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemcpy(ctx->d_ctab, ctab.data(), ctab.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->d_mt, mt.data(), 65536, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->d_lam, lam, sizeof(lam), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->d_phi, phi.data(), phi.size() * sizeof(uint4), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->d_psi, psi.data(), psi.size() * sizeof(uint4), hipMemcpyHostToDevice);
    std::vector<gcm_u128> cantor;
    if (!build_cantor_table(cantor)) {
        gf2x_ctx_destroy(ctx);
        return GF2X_EINVAL;
    }
    std::vector<uint4> cantor4(cantor.size());
    for (size_t i = 0; i < cantor.size(); ++i) cantor4[i] = to_u4((u128)cantor[i]);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_cantor, cantor4.size() * sizeof(uint4));
    if (e == hipSuccess)
        e = hipMemcpy(ctx->d_cantor, cantor4.data(), cantor4.size() * sizeof(uint4), hipMemcpyHostToDevice);
    std::vector<gcm_u128> fenc, fdec;
    std::vector<uint64_t> fwf, fwi;
    if (!build_frob_tables(cantor.data(), fenc, fdec, fwf, fwi)) {
        gf2x_ctx_destroy(ctx);
        return GF2X_EINVAL;
    }
    std::vector<uint4> frob(kFrobTabU4);
    for (int i = 0; i < kElemTab; ++i) {
        frob[kFrobEncOff + i] = to_u4((u128)fenc[i]);
        frob[kFrobDecOff + i] = to_u4((u128)fdec[i]);
    }
    memcpy(frob.data() + kFrobWordOff, fwf.data(), 8 * kWordTab);
    memcpy((char*)(frob.data() + kFrobWordOff) + 8 * kWordTab, fwi.data(), 8 * kWordTab);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_frob, frob.size() * sizeof(uint4));
    if (e == hipSuccess) e = hipMemcpy(ctx->d_frob, frob.data(), frob.size() * sizeof(uint4), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_layers, ctx->pool.host.size() * sizeof(BcLayer));
    if (e == hipSuccess)
        e = hipMemcpy(ctx->d_layers, ctx->pool.host.data(), ctx->pool.host.size() * sizeof(BcLayer), hipMemcpyHostToDevice);
    ctx->pool.base = ctx->d_layers;
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->own_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->aux_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_last, hipEventDisableTiming);
    if (e == hipSuccess) e = scratch_address(device, &ctx->scratch);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&ctx->persist_per_cu, k_persistent, kThreads, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        gf2x_ctx_destroy(ctx);
        return GF2X_EDEVICE;
    }
    *out = ctx;
    return GF2X_OK;
}

void gf2x_ctx_destroy(gf2x_ctx* ctx) {
    if (!ctx) return;
    DeviceGuard g(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->d_mt) (void)hipFree(ctx->d_mt);
    if (ctx->d_lam) (void)hipFree(ctx->d_lam);
    if (ctx->d_phi) (void)hipFree(ctx->d_phi);
    if (ctx->d_psi) (void)hipFree(ctx->d_psi);
    if (ctx->d_ctab) (void)hipFree(ctx->d_ctab);
    if (ctx->d_cantor) (void)hipFree(ctx->d_cantor);
    if (ctx->d_frob) (void)hipFree(ctx->d_frob);
    if (ctx->d_layers) (void)hipFree(ctx->d_layers);
    if (ctx->transient) batch_free(ctx->transient);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->io) (void)hipFree(ctx->io);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->own_stream);
    if (ctx->aux_stream) (void)hipStreamDestroy(ctx->aux_stream);
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    if (ctx->ev_last) (void)hipEventDestroy(ctx->ev_last);
    delete ctx;
}

int gf2x_trace_begin(gf2x_ctx* ctx, uint32_t kind_mask) {
    if (check_ctx(ctx)) return GF2X_EINVAL;
    ctx->trace_mask = kind_mask;
    return GF2X_OK;
}

int64_t gf2x_trace_read(gf2x_ctx* ctx, gf2x_trace_rec* out, size_t max) {
    if (check_ctx(ctx)) return GF2X_EINVAL;
    if (max && !out) return GF2X_EINVAL;
    DeviceGuard g(ctx->device);
    int64_t n = (int64_t)ctx->trace.size();
    int rc = GF2X_OK;
    for (size_t i = 0; i < ctx->trace.size(); ++i) {
        auto& p = ctx->trace[i];
        hipError_t e = hipEventSynchronize(p.stop);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.start, p.stop);
        if (e != hipSuccess && rc == GF2X_OK) rc = hip_fail(ctx, e, "trace read");
        p.rec.ms = ms;
        if (i < max) out[i] = p.rec;
        (void)hipEventDestroy(p.start);
        (void)hipEventDestroy(p.stop);
    }
    ctx->trace.clear();
    return rc ? rc : n;
}

}  // extern "C"

// Checks of a product's arguments shared by the product entry points.
int check_product(gf2x_ctx* ctx, const Sizes& s, const uint64_t* a, const uint64_t* b, const uint64_t* c) {
    if (!a || !b || !c) return fail(ctx, GF2X_EINVAL, "NULL operand or product pointer");
    if (s.m > kMaxLog2N) return fail(ctx, GF2X_ERANGE, "transform length above 2^32");
    if (ranges_overlap(c, 8 * s.out_words, a, 8 * s.n_a) || ranges_overlap(c, 8 * s.out_words, b, 8 * s.n_b))
        return fail(ctx, GF2X_EINVAL, "product overlaps an operand");
    return GF2X_OK;
}

// The whole product in one dispatch (k_single): its ops, planned with the
// tiles of the batch kernels (1024-thread blocks), go in the kernel
// arguments.  Returns 1, having done nothing, if the plan has more ops than
// the arguments hold.
constexpr int kTraceSingle = 8;  // trace kind of a whole-product launch
int mul_single(gf2x_ctx* ctx, const Sizes& s, const uint64_t* a, const uint64_t* b, uint64_t* c, char* ws,
               hipStream_t st) {
    std::vector<Op> ops;
    plan_mul(ops, ctx->pool, ctx->params, s, a, b, c, ws);
    if (ops.size() > (size_t)kSingleMaxOps) return 1;
    SingleArgs A;
    memset(&A, 0, sizeof(A));
    for (size_t i = 0; i < ops.size(); ++i) A.ops[i] = make_devop(ops[i]);
    A.nops = (int)ops.size();
    gf2x_ctx::Pending pend{};
    const bool traced = (ctx->trace_mask >> kTraceSingle) & 1u;
    if (traced) {
        pend.rec.kind = kTraceSingle;
        pend.rec.elements = 1ull << s.m;
        pend.rec.bytes_read = 8 * (s.n_a + s.n_b);
        pend.rec.bytes_written = 8 * s.out_words;
        hipError_t e = hipEventCreate(&pend.start);
        if (e == hipSuccess) e = hipEventCreate(&pend.stop);
        if (e != hipSuccess) return hip_fail(ctx, e, "trace event");
        hipExtLaunchKernelGGL(k_single, dim3(1), dim3(kThreads), 0, st, pend.start, pend.stop, 0, A,
                              (const uint8_t*)ctx->d_mt, (const uint32_t*)ctx->d_lam, (const uint4*)ctx->d_phi,
                              (const uint4*)ctx->d_psi, (const uint32_t*)ctx->d_ctab);
    } else {
        hipLaunchKernelGGL(k_single, dim3(1), dim3(kThreads), 0, st, A, (const uint8_t*)ctx->d_mt,
                           (const uint32_t*)ctx->d_lam, (const uint4*)ctx->d_phi, (const uint4*)ctx->d_psi,
                           (const uint32_t*)ctx->d_ctab);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "single-block product launch");
    if (traced) ctx->trace.push_back(pend);
    return GF2X_OK;
}

// The ops after the forward transforms of a small product as one k_tail
// launch when they are pointmul, one untruncated w = 64 inverse pass on a
// single tile with its whole BasisCvt inside, and Psi, on at most one
// pointmul tile of points (at 2^11 points pointmul and Psi on one block
// instead of two cost more than the two launches saved: 2^16-bit products
// 0.074 -> 0.077 ms); returns 1, having done nothing, for any other shape.
constexpr int kTraceTail = 9;  // trace kind of a k_tail launch
int run_tail(gf2x_ctx* ctx, const std::vector<Op>& rest, hipStream_t st, bool may_trace) {
    if (rest.size() != 3 || rest[0].kind != OpKind::Pmul || rest[1].kind != OpKind::Fft ||
        rest[2].kind != OpKind::Psi)
        return 1;
    const TailOp T{rest[0].pmul, rest[1].fft, rest[2].psi};
    const uint64_t N = 1ull << T.fft.log_m;
    if (T.pm.ah || T.psi.spech || !T.fft.inverse || T.fft.phi_in != kPhiNone || T.fft.lo != 0 ||
        T.fft.hi != T.fft.log_m || T.fft.log_tc != 0 || T.fft.pack != 0 || T.fft.ncosets != 1 ||
        T.fft.coset0 != 0 || N > (uint64_t)kPmulTile || fft_tiles(T.fft) != 1 || T.pm.n != N ||
        T.pm.n_out != N || T.pm.c != T.fft.dst || T.psi.spec != T.fft.dst || T.psi.nspec != N)
        return 1;
    gf2x_ctx::Pending pend{};
    const bool traced = may_trace && ((ctx->trace_mask >> kTraceTail) & 1u);
    if (traced) {
        gf2x_trace_rec r{};
        for (const Op& op : rest) {
            op_traffic(op, r);
            pend.rec.lookups += r.lookups;
        }
        pend.rec.kind = kTraceTail;
        pend.rec.elements = N;
        pend.rec.bytes_read = 32 * N;  // the two spectra; the result stays on chip
        pend.rec.bytes_written = 8 * T.psi.nwords;
        hipError_t e = hipEventCreate(&pend.start);
        if (e == hipSuccess) e = hipEventCreate(&pend.stop);
        if (e != hipSuccess) return hip_fail(ctx, e, "trace event");
        hipExtLaunchKernelGGL(k_tail, dim3(1), dim3(kThreads), 0, st, pend.start, pend.stop, 0, T,
                              (const uint8_t*)ctx->d_mt, (const uint32_t*)ctx->d_lam, (const uint32_t*)ctx->d_ctab,
                              (const uint4*)ctx->d_psi);
    } else {
        hipLaunchKernelGGL(k_tail, dim3(1), dim3(kThreads), 0, st, T, (const uint8_t*)ctx->d_mt,
                           (const uint32_t*)ctx->d_lam, (const uint32_t*)ctx->d_ctab, (const uint4*)ctx->d_psi);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "tail launch");
    if (traced) ctx->trace.push_back(pend);
    return GF2X_OK;
}

// A product planned by plan_mul (split: the ends of the two forward
// transforms) on one stream.  Below 2^kForkMinLog points the forward
// transforms are interleaved level by level, so that their FFT passes of one
// level share a launch (run_ops), and the last steps run as one launch when
// they fit one block (run_tail); otherwise op by op.
int run_product(gf2x_ctx* ctx, const std::vector<Op>& ops, const size_t* split, int m, hipStream_t st,
                bool may_trace) {
    if (!split[1] || m >= kForkMinLog) return run_ops(ctx, ops, st, may_trace);
    std::vector<Op> il;
    il.reserve(split[1]);
    size_t ia = 0, ib = split[0];
    while (ia < split[0] || ib < split[1]) {
        const uint32_t la = ia < split[0] ? ops[ia].level : ~0u, lb = ib < split[1] ? ops[ib].level : ~0u;
        const uint32_t l = la < lb ? la : lb;
        while (ia < split[0] && ops[ia].level == l) il.push_back(ops[ia++]);
        while (ib < split[1] && ops[ib].level == l) il.push_back(ops[ib++]);
    }
    int rc = run_ops(ctx, il, st, may_trace, true);
    if (rc) return rc;
    const std::vector<Op> rest(ops.begin() + split[1], ops.end());
    rc = run_tail(ctx, rest, st, may_trace);
    return rc == 1 ? run_ops(ctx, rest, st, may_trace, true) : rc;
}

// The product's ops on stream st with the workspace at ws (Alg. 5): small
// products in one dispatch, the others op by op.
int mul_on(gf2x_ctx* ctx, const Sizes& s, const uint64_t* a, const uint64_t* b, uint64_t* c, char* ws,
           hipStream_t st) {
    if (s.m <= ctx->single_max_log) {
        const int rc = mul_single(ctx, s, a, b, c, ws, st);
        if (rc != 1) return rc;
    }
    std::vector<Op> ops;
    size_t split[2] = {0, 0};
    plan_mul(ops, ctx->pool, single_params(ctx), s, a, b, c, ws, split);
    if (!split[1] || s.m < kForkMinLog) return run_product(ctx, ops, split, s.m, st, true);
    // The two forward transforms are independent: b's runs on the second
    // stream, between a fork event recorded here and a join event that a's
    // continuation waits for.  Up to 2^kForkMaxLog points the whole transforms
    // overlap; above, only their pack and BasisCvt launches do (each FFT pass
    // fills the device, and its launches stay alone).
    std::vector<Op> fa(ops.begin(), ops.begin() + split[0]), fb(ops.begin() + split[0], ops.begin() + split[1]),
        rest(ops.begin() + split[1], ops.end());
    std::vector<Op> fa_fft, fb_fft;
    if (s.m > kForkMaxLog) {
        auto cut = [](std::vector<Op>& v, std::vector<Op>& tail) {
            size_t i = 0;
            while (i < v.size() && v[i].kind != OpKind::Fft && v[i].kind != OpKind::Spine) ++i;
            tail.assign(v.begin() + i, v.end());
            v.resize(i);
        };
        cut(fa, fa_fft);
        cut(fb, fb_fft);
    }
    hipError_t e = hipEventRecord(ctx->ev_fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(ctx->aux_stream, ctx->ev_fork, 0);
    if (e != hipSuccess) return hip_fail(ctx, e, "fork");
    int rc = run_ops(ctx, fb, ctx->aux_stream);
    if (rc) return rc;
    e = hipEventRecord(ctx->ev_join, ctx->aux_stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "join");
    rc = run_ops(ctx, fa, st);
    if (rc) return rc;
    e = hipStreamWaitEvent(st, ctx->ev_join, 0);
    if (e != hipSuccess) return hip_fail(ctx, e, "join");
    if ((rc = run_ops(ctx, fa_fft, st))) return rc;
    if ((rc = run_ops(ctx, fb_fft, st))) return rc;
    return run_ops(ctx, rest, st);
}

extern "C" {

int gf2x_mul_dev(gf2x_ctx* ctx, const uint64_t* a, uint64_t na_bits, const uint64_t* b, uint64_t nb_bits,
                 uint64_t* c, void* stream) {
    if (check_ctx(ctx)) return GF2X_EINVAL;
    ctx->err.clear();
    Sizes s = make_sizes(na_bits, nb_bits, ctx->params.word_bits);
    if (!s.out_words) return GF2X_OK;
    int rc = check_product(ctx, s, a, b, c);
    if (rc) return rc;
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    const bool cap = stream_capturing(st);
    if ((rc = ws_enter(ctx, st, cap))) return rc;
    if ((rc = ensure_ws(ctx, workspace_for(s).bytes, st))) return rc;
    return ws_leave(ctx, st, cap, mul_on(ctx, s, a, b, c, ctx->ws, st));
}

int gf2x_mul_dev_static(gf2x_ctx* ctx, const uint64_t* a, uint64_t na_bits, const uint64_t* b, uint64_t nb_bits,
                        uint64_t* c, void* stream) {
    if (check_ctx(ctx)) return GF2X_EINVAL;
    ctx->err.clear();
    Sizes s = make_sizes(na_bits, nb_bits, ctx->params.word_bits);
    if (!s.out_words) return GF2X_OK;
    int rc = check_product(ctx, s, a, b, c);
    if (rc) return rc;
    const size_t need = workspace_for(s).bytes;
    if (need > (size_t)GF2X_STATIC_SCRATCH_BYTES)
        return fail(ctx, GF2X_ENOMEM, "product needs " + std::to_string(need) + " bytes of workspace; the static buffer holds " +
                                          std::to_string((size_t)GF2X_STATIC_SCRATCH_BYTES));
    if (!ctx->scratch) return fail(ctx, GF2X_EDEVICE, "no address for the static buffer on this device");
    DeviceGuard g(ctx->device);
    // every op on the caller's stream (no second stream, no events, no trace):
    // the ops write each workspace byte before they read it, so nothing in the
    // buffer has to start at zero
    std::vector<Op> ops;
    size_t split[2] = {0, 0};
    plan_mul(ops, ctx->pool, single_params(ctx), s, a, b, c, ctx->scratch, split);
    return run_product(ctx, ops, split, s.m, (hipStream_t)stream, false);
}

int gf2x_forward_dev(gf2x_ctx* ctx, const uint64_t* a, uint64_t na_bits, int log2n, void* spec, void* stream) {
    if (check_ctx(ctx)) return GF2X_EINVAL;
    ctx->err.clear();
    if (!a || !spec || na_bits == 0) return fail(ctx, GF2X_EINVAL, "NULL pointer or empty operand");
    if (log2n < 0 || log2n > kMaxLog2N) return fail(ctx, GF2X_ERANGE, "log2n out of range");
    uint64_t n = (na_bits + 63) / 64;
    int m_a = ceil_log2(n);
    if (m_a > log2n) return fail(ctx, GF2X_EINVAL, "spectrum shorter than the operand");
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    const bool cap = stream_capturing(st);
    int rc = ws_enter(ctx, st, cap);
    if (rc) return rc;
    if ((rc = ensure_ws(ctx, align256(8ull << m_a), st))) return rc;
    std::vector<Op> ops;
    emit_forward(ops, ctx->pool, single_params(ctx), a, na_bits, (uint64_t*)ctx->ws, m_a, (uint4*)spec, log2n,
                 1ull << log2n);
    return ws_leave(ctx, st, cap, run_ops(ctx, ops, st));
}

int gf2x_pointmul_dev(gf2x_ctx* ctx, const void* sa, const void* sb, void* sc, uint64_t n, void* stream) {
    if (check_ctx(ctx)) return GF2X_EINVAL;
    ctx->err.clear();
    if (n == 0) return GF2X_OK;
    if (!sa || !sb || !sc) return fail(ctx, GF2X_EINVAL, "NULL spectrum");
    DeviceGuard g(ctx->device);
    std::vector<Op> ops;
    emit_pmul(ops, (const uint4*)sa, (const uint4*)sb, (uint4*)sc, n);
    return run_ops(ctx, ops, (hipStream_t)stream);
}

int gf2x_inverse_dev(gf2x_ctx* ctx, void* spec, int log2n, uint64_t* c, uint64_t nc_bits, void* stream) {
    if (check_ctx(ctx)) return GF2X_EINVAL;
    ctx->err.clear();
    if (nc_bits == 0) return GF2X_OK;
    if (!spec || !c) return fail(ctx, GF2X_EINVAL, "NULL pointer");
    if (log2n < 0 || log2n > kMaxLog2N) return fail(ctx, GF2X_ERANGE, "log2n out of range");
    if (ranges_overlap(c, 8 * ((nc_bits + 63) / 64), spec, 16ull << log2n))
        return fail(ctx, GF2X_EINVAL, "output overlaps the spectrum");
    DeviceGuard g(ctx->device);
    std::vector<Op> ops;
    emit_inverse(ops, ctx->pool, single_params(ctx), (uint4*)spec, log2n, 1ull << log2n, c, nc_bits);
    return run_ops(ctx, ops, (hipStream_t)stream);
}

int gf2x_basiscvt_dev(gf2x_ctx* ctx, uint64_t* words, int log2n, int inverse, void* stream) {
    if (check_ctx(ctx)) return GF2X_EINVAL;
    ctx->err.clear();
    if (!words) return fail(ctx, GF2X_EINVAL, "NULL words");
    if (log2n < 0 || log2n > 40) return fail(ctx, GF2X_ERANGE, "log2n out of range");
    DeviceGuard g(ctx->device);
    std::vector<Op> ops;
    emit_bc(ops, ctx->pool, words, 0, log2n, inverse ? 1 : 0, 1);
    return run_ops(ctx, ops, (hipStream_t)stream);
}

int gf2x_simple_mul_dev(gf2x_ctx* ctx, const uint64_t* a, uint64_t na_bits, const uint64_t* b, uint64_t nb_bits,
                        uint64_t* c, void* stream) {
    if (check_ctx(ctx)) return GF2X_EINVAL;
    ctx->err.clear();
    const Sizes s = make_sizes(na_bits, nb_bits, 64);
    if (!s.out_words) return GF2X_OK;
    int rc = check_product(ctx, s, a, b, c);
    if (rc) return rc;
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    const bool cap = stream_capturing(st);
    if ((rc = ws_enter(ctx, st, cap))) return rc;
    return ws_leave(ctx, st, cap, simple_mul(ctx, a, na_bits, b, nb_bits, c, st));
}

int gf2x_simple_forward_dev(gf2x_ctx* ctx, const uint64_t* a, uint64_t na_bits, int log2n, void* spec,
                            void* stream) {
    if (check_ctx(ctx)) return GF2X_EINVAL;
    ctx->err.clear();
    if (!a || !spec || na_bits == 0) return fail(ctx, GF2X_EINVAL, "NULL pointer or empty operand");
    if (log2n < 0 || log2n > kMaxLog2N) return fail(ctx, GF2X_ERANGE, "log2n out of range");
    const int m_a = ceil_log2((na_bits + 63) / 64);
    if (m_a > log2n) return fail(ctx, GF2X_EINVAL, "spectrum shorter than the operand");
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    const bool cap = stream_capturing(st);
    int rc = ws_enter(ctx, st, cap);
    if (rc) return rc;
    if ((rc = ensure_ws(ctx, align256(8ull << m_a), st))) return rc;
    return ws_leave(ctx, st, cap, simple_forward(ctx, a, na_bits, (uint64_t*)ctx->ws, m_a, (uint4*)spec, log2n, st));
}

int gf2x_set_single_launch(gf2x_ctx* ctx, int max_log2n) {
    if (check_ctx(ctx)) return GF2X_EINVAL;
    if (max_log2n < -1 || max_log2n > kSingleMaxLog) return fail(ctx, GF2X_EINVAL, "single-launch bound out of range");
    ctx->single_max_log = max_log2n;
    return GF2X_OK;
}

int gf2x_set_fusion(gf2x_ctx* ctx, int mask, int single_max_log2n, int batch_max_log2n) {
    if (check_ctx(ctx)) return GF2X_EINVAL;
    if (mask < 0 || mask > 7) return fail(ctx, GF2X_EINVAL, "fusion mask outside 0..7");
    if (single_max_log2n < 0 || single_max_log2n > PlanParams::kMaxM || batch_max_log2n < 0 ||
        batch_max_log2n > PlanParams::kMaxM)
        return fail(ctx, GF2X_EINVAL, "fusion size bound outside 0..32");
    ctx->params.fuse_bc = mask;
    ctx->params.fuse_max_log = batch_max_log2n;
    ctx->fuse_single_max_log = single_max_log2n;
    return GF2X_OK;
}

int gf2x_frobenius_log2n(uint64_t na_bits, uint64_t nb_bits) {
    if (!na_bits || !nb_bits) return -1;
    return frob_sizes(na_bits, nb_bits).m;
}

size_t gf2x_frobenius_workspace_bytes(uint64_t na_bits, uint64_t nb_bits) {
    if (!na_bits || !nb_bits) return 0;
    return frob_workspace(frob_sizes(na_bits, nb_bits)).bytes;
}

int gf2x_frobenius_mul_dev(gf2x_ctx* ctx, const uint64_t* a, uint64_t na_bits, const uint64_t* b, uint64_t nb_bits,
                           uint64_t* c, void* stream) {
    if (check_ctx(ctx)) return GF2X_EINVAL;
    ctx->err.clear();
    const FrobSizes s = frob_sizes(na_bits, nb_bits);
    if (!s.out_words) return GF2X_OK;
    if (!a || !b || !c) return fail(ctx, GF2X_EINVAL, "NULL operand or product pointer");
    if (s.m > kMaxLog2N) return fail(ctx, GF2X_ERANGE, "more than 2^32 points");
    if (ranges_overlap(c, 8 * s.out_words, a, 8 * ((na_bits + 63) / 64)) ||
        ranges_overlap(c, 8 * s.out_words, b, 8 * ((nb_bits + 63) / 64)))
        return fail(ctx, GF2X_EINVAL, "product overlaps an operand");
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    const bool cap = stream_capturing(st);
    int rc = ws_enter(ctx, st, cap);
    if (rc) return rc;
    return ws_leave(ctx, st, cap, frob_mul(ctx, s, a, b, c, st));
}

int gf2x_frobenius_forward_dev(gf2x_ctx* ctx, const uint64_t* a, uint64_t na_bits, int log2n, void* spec,
                               void* stream) {
    if (check_ctx(ctx)) return GF2X_EINVAL;
    ctx->err.clear();
    if (!a || !spec || na_bits == 0) return fail(ctx, GF2X_EINVAL, "NULL pointer or empty operand");
    if (log2n < 0 || log2n > kMaxLog2N) return fail(ctx, GF2X_ERANGE, "log2n out of range");
    if (na_bits > (128ull << log2n)) return fail(ctx, GF2X_EINVAL, "operand longer than 128 bits per point");
    const int W = frob_ceil_log2((na_bits + 63) / 64);
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    const bool cap = stream_capturing(st);
    int rc = ws_enter(ctx, st, cap);
    if (rc) return rc;
    if ((rc = ensure_ws(ctx, align256(8ull << W), st))) return rc;
    return ws_leave(ctx, st, cap, frob_forward(ctx, a, na_bits, (uint64_t*)ctx->ws, W, (uint4*)spec, log2n, st));
}

int gf2x_frobenius_inverse_dev(gf2x_ctx* ctx, void* spec, int log2n, uint64_t* c, uint64_t nc_bits, void* stream) {
    if (check_ctx(ctx)) return GF2X_EINVAL;
    ctx->err.clear();
    if (nc_bits == 0) return GF2X_OK;
    if (!spec || !c) return fail(ctx, GF2X_EINVAL, "NULL pointer");
    if (log2n < 0 || log2n > kMaxLog2N) return fail(ctx, GF2X_ERANGE, "log2n out of range");
    if (nc_bits > (128ull << log2n)) return fail(ctx, GF2X_EINVAL, "more than 128 bits per point requested");
    if (ranges_overlap(c, 8 * ((nc_bits + 63) / 64), spec, 16ull << log2n))
        return fail(ctx, GF2X_EINVAL, "output overlaps the values");
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    const bool cap = stream_capturing(st);
    int rc = ws_enter(ctx, st, cap);
    if (rc) return rc;
    if ((rc = ensure_ws(ctx, align256(16ull << log2n), st))) return rc;
    return ws_leave(ctx, st, cap, frob_inverse(ctx, (uint4*)spec, log2n, (uint64_t*)ctx->ws, c, nc_bits, st));
}

int gf2x_mul_batch(gf2x_ctx* ctx, const gf2x_job* jobs, size_t njobs, void* stream) {
    if (check_ctx(ctx)) return GF2X_EINVAL;
    ctx->err.clear();
    if (njobs == 0) return GF2X_OK;
    if (!jobs) return fail(ctx, GF2X_EINVAL, "NULL job array");
    int rc = check_jobs(ctx, jobs, njobs);
    if (rc) return rc;
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    // the previous call's batch may still be running on its stream
    if (ctx->transient) {
        hipError_t e = hipStreamSynchronize(ctx->transient_stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
        batch_free(ctx->transient);
        ctx->transient = nullptr;
    }
    gf2x_batch* B = nullptr;
    rc = batch_build(ctx, jobs, njobs, GF2X_BATCH_STAGED, &B);
    if (rc) return rc;
    ctx->transient = B;
    ctx->transient_stream = st;
    return batch_launch_groups(B, st);
}

int gf2x_batch_create(gf2x_ctx* ctx, const gf2x_job* jobs, size_t njobs, int mode, gf2x_batch** out) {
    if (check_ctx(ctx) || !out) return GF2X_EINVAL;
    if (mode != GF2X_BATCH_STAGED && mode != GF2X_BATCH_PERSISTENT) return fail(ctx, GF2X_EINVAL, "unknown batch mode");
    ctx->err.clear();
    *out = nullptr;
    if (njobs && !jobs) return fail(ctx, GF2X_EINVAL, "NULL job array");
    int rc = check_jobs(ctx, jobs, njobs);
    if (rc) return rc;
    DeviceGuard g(ctx->device);
    return batch_build(ctx, jobs, njobs, mode, out);
}

int gf2x_batch_run(gf2x_batch* B, void* stream) {
    if (!B) return GF2X_EINVAL;
    gf2x_ctx* ctx = B->ctx;
    ctx->err.clear();
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    if (B->groups.empty()) return GF2X_OK;
    auto launch = [&](hipStream_t s) {
        return B->mode == GF2X_BATCH_PERSISTENT ? batch_launch_persistent(B, s) : batch_launch_groups(B, s);
    };
    if (!B->use_graph || ctx->trace_mask) return launch(st);
    if (!B->exec) {
        // record the launch sequence once on the context's own stream
        hipStream_t cs = ctx->own_stream;
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamBeginCapture");
        int rc = launch(cs);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(cs, &graph);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamEndCapture");
        B->graph = graph;
        e = hipGraphInstantiate(&B->exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipGraphInstantiate");
    }
    hipError_t e = hipGraphLaunch(B->exec, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipGraphLaunch");
    return GF2X_OK;
}

int gf2x_batch_info(const gf2x_batch* B, gf2x_batch_stats* st) {
    if (!B || !st) return GF2X_EINVAL;
    st->launches = 0;
    for (const auto& G : B->groups) st->launches += G.kind == OpKind::BcLayer ? (uint64_t)G.nops : 1;
    if (B->mode == GF2X_BATCH_PERSISTENT) st->launches = 2;  // state clear + the persistent kernel
    st->ops = B->plan.ops.size();
    st->ranks = B->plan.max_rank;
    st->workspace_bytes = B->plan.ws_bytes;
    uint64_t tiles = 0;
    for (const auto& G : B->groups) tiles += G.total;
    st->tiles = tiles;
    return GF2X_OK;
}

int gf2x_batch_set_spin_limit(gf2x_batch* B, uint32_t polls) {
    if (!B) return GF2X_EINVAL;
    B->spin_limit = polls;
    if (B->exec) {  // the limit is a kernel argument: record the graph again
        (void)hipGraphExecDestroy(B->exec);
        (void)hipGraphDestroy(B->graph);
        B->exec = nullptr;
        B->graph = nullptr;
    }
    return GF2X_OK;
}

int gf2x_batch_check(gf2x_batch* B) {
    if (!B) return GF2X_EINVAL;
    if (B->mode != GF2X_BATCH_PERSISTENT || !B->pdesc) return GF2X_OK;
    DeviceGuard g(B->ctx->device);
    uint32_t flag = 0;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(&flag, B->pdesc + B->play.state_off, 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(B->ctx, e, "gf2x_batch_check");
    if (flag) return fail(B->ctx, GF2X_EDEVICE, "persistent batch: a barrier wait timed out; results incomplete");
    return GF2X_OK;
}

void gf2x_batch_destroy(gf2x_batch* B) {
    if (!B) return;
    DeviceGuard g(B->ctx->device);
    (void)hipDeviceSynchronize();
    batch_free(B);
}

int gf2x_mul(const uint64_t* a, uint64_t na_bits, const uint64_t* b, uint64_t nb_bits, uint64_t* c) {
    Sizes s = make_sizes(na_bits, nb_bits);
    if (!s.out_words) return GF2X_OK;
    if (!a || !b || !c) return GF2X_EINVAL;
    if (ranges_overlap(c, 8 * s.out_words, a, 8 * s.n_a) || ranges_overlap(c, 8 * s.out_words, b, 8 * s.n_b))
        return GF2X_EINVAL;
    std::lock_guard<std::mutex> lock(g_default_mu);
    if (!g_default) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return GF2X_EDEVICE;
        int rc = gf2x_ctx_create(&g_default, dev);
        if (rc) return rc;
    }
    gf2x_ctx* ctx = g_default;
    DeviceGuard g(ctx->device);
    hipStream_t st = ctx->own_stream;
    size_t ba = align256(8 * s.n_a), bb = align256(8 * s.n_b), bc = align256(8 * s.out_words);
    if (ba + bb + bc > ctx->io_bytes) {
        if (ctx->io) (void)hipFree(ctx->io);
        ctx->io = nullptr;
        ctx->io_bytes = 0;
        if (hipMalloc((void**)&ctx->io, ba + bb + bc) != hipSuccess) {
            (void)hipGetLastError();
            return fail(ctx, GF2X_ENOMEM, "operand staging");
        }
        ctx->io_bytes = ba + bb + bc;
    }
    uint64_t* da = (uint64_t*)ctx->io;
    uint64_t* db = (uint64_t*)(ctx->io + ba);
    uint64_t* dc = (uint64_t*)(ctx->io + ba + bb);
    hipError_t e = hipMemcpyAsync(da, a, 8 * s.n_a, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(db, b, 8 * s.n_b, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "copy operands");
    int rc = gf2x_mul_dev(ctx, da, na_bits, db, nb_bits, dc, st);
    if (rc) return rc;
    e = hipMemcpyAsync(c, dc, 8 * s.out_words, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(ctx, e, "copy product");
    return GF2X_OK;
}

uint64_t gf2x_now_ns(void) { return now_ns(); }

int gf2x_server_create(gf2x_ctx* ctx, const gf2x_server_cfg* cfg, gf2x_server** out) {
    if (check_ctx(ctx) || !cfg || !out) return GF2X_EINVAL;
    ctx->err.clear();
    *out = nullptr;
    if (!cfg->arena_bytes || !cfg->max_active || !cfg->levels_per_iter || cfg->inflight < 1 || cfg->inflight > 4)
        return fail(ctx, GF2X_EINVAL, "server configuration: zero field or inflight outside 1..4");
    if (cfg->mode != GF2X_BATCH_STAGED && cfg->mode != GF2X_BATCH_PERSISTENT && cfg->mode != GF2X_SERVER_ADAPTIVE)
        return fail(ctx, GF2X_EINVAL, "server configuration: unknown mode");
    DeviceGuard g(ctx->device);
    gf2x_server* S = new gf2x_server();
    S->ctx = ctx;
    S->cfg = *cfg;
    hipError_t e = hipStreamCreateWithFlags(&S->st, hipStreamNonBlocking);
    if (e != hipSuccess) {
        server_free(S);
        return hip_fail(ctx, e, "server stream");
    }
    e = hipMalloc((void**)&S->arena, cfg->arena_bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        server_free(S);
        return fail(ctx, GF2X_ENOMEM, "server arena");
    }
    S->alloc.reset(cfg->arena_bytes);
    S->slots.resize(cfg->inflight);
    for (uint32_t i = 0; i < cfg->inflight; ++i) {
        e = hipEventCreateWithFlags(&S->slots[i].ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            server_free(S);
            return hip_fail(ctx, e, "server events");
        }
        int rc = server_ensure_slot(S, S->slots[i], 1 << 20);
        if (rc) {
            server_free(S);
            return rc;
        }
        S->free_slots.push_back((int)(cfg->inflight - 1 - i));
    }
    *out = S;
    return GF2X_OK;
}

int gf2x_server_submit(gf2x_server* S, const uint64_t* a, uint64_t na_bits, const uint64_t* b, uint64_t nb_bits,
                       uint64_t* c, uint64_t tag, void* stream) {
    if (!S) return GF2X_EINVAL;
    gf2x_ctx* ctx = S->ctx;
    ctx->err.clear();
    if (S->sticky) return fail(ctx, S->sticky, "server stopped after a device error");
    const Sizes s = make_sizes(na_bits, nb_bits, ctx->params.word_bits);
    const uint64_t t = now_ns();
    if (!s.out_words) {
        S->done.push_back(gf2x_done{tag, GF2X_OK, 0, t, t, t});
        ++S->stats.submitted;
        ++S->stats.completed;
        return GF2X_OK;
    }
    gf2x_job j{a, na_bits, b, nb_bits, c};
    int rc = check_jobs(ctx, &j, 1);
    if (rc) return rc;
    gf2x_server::Req r;
    r.a = a;
    r.b = b;
    r.c = c;
    r.na = na_bits;
    r.nb = nb_bits;
    r.w = s.w;
    r.tag = tag;
    r.t_submit = t;
    r.bytes = workspace_for(s).bytes;
    if (Arena::round(r.bytes) > S->alloc.capacity())
        return fail(ctx, GF2X_ENOMEM, "request footprint exceeds the server arena");
    DeviceGuard g(ctx->device);
    if (S->free_events.empty()) {
        hipEvent_t ev = nullptr;
        hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(ctx, e, "serving: submit event");
        S->all_events.push_back(ev);
        S->free_events.push_back(ev);
    }
    r.src = (hipStream_t)stream;
    r.ready = S->free_events.back();
    hipError_t e = hipEventRecord(r.ready, r.src);
    if (e != hipSuccess) return hip_fail(ctx, e, "serving: record on the submitter's stream");
    S->free_events.pop_back();
    S->queue.push_back(std::move(r));
    ++S->stats.submitted;
    return GF2X_OK;
}

int gf2x_server_step(gf2x_server* S, uint64_t until_ns) {
    if (!S) return GF2X_EINVAL;
    if (S->sticky) return S->sticky;
    DeviceGuard g(S->ctx->device);
    while (true) {
        int rc = server_retire(S);
        if (rc) return rc;
        const bool work = !S->queue.empty() || !S->active.empty();
        if (work && !S->free_slots.empty()) {
            bool launched = false;
            rc = server_iterate(S, launched);
            if (rc) {
                server_fail_all(S, rc);
                return rc;
            }
            if (launched) continue;
        }
        if (!work && S->inflight.empty()) return GF2X_OK;
        if (now_ns() >= until_ns) return GF2X_OK;
        std::this_thread::yield();
    }
}

size_t gf2x_server_poll(gf2x_server* S, gf2x_done* out, size_t max) {
    if (!S || !out) return 0;
    size_t n = 0;
    while (n < max && !S->done.empty()) {
        out[n++] = S->done.front();
        S->done.pop_front();
    }
    return n;
}

int gf2x_server_info(const gf2x_server* S, gf2x_server_stats* st) {
    if (!S || !st) return GF2X_EINVAL;
    *st = S->stats;
    st->queued = S->queue.size();
    st->active = S->active.size();
    st->arena_used = S->alloc.used();
    return GF2X_OK;
}

void gf2x_server_destroy(gf2x_server* S) {
    if (!S) return;
    DeviceGuard g(S->ctx->device);
    if (S->st) (void)hipStreamSynchronize(S->st);
    server_free(S);
}

int gf2x_set_schedule(gf2x_ctx* ctx, int m, int bottom_log, int col_rows_log) {
    if (check_ctx(ctx)) return GF2X_EINVAL;
    if (m < 1 || m > PlanParams::kMaxM || bottom_log < 1 || bottom_log > kFftTileLog || col_rows_log < 1 ||
        col_rows_log > kFftTileLog)
        return fail(ctx, GF2X_EINVAL, "schedule outside its range");
    ctx->params.fft_bottom_log[m] = (int8_t)bottom_log;
    ctx->params.fft_col_rows_log[m] = (int8_t)col_rows_log;
    return GF2X_OK;
}

int gf2x_get_schedule(gf2x_ctx* ctx, int m, int* bottom_log, int* col_rows_log) {
    if (check_ctx(ctx) || !bottom_log || !col_rows_log) return GF2X_EINVAL;
    if (m < 1 || m > PlanParams::kMaxM) return fail(ctx, GF2X_EINVAL, "m outside 1..32");
    *bottom_log = ctx->params.bottom(m);
    *col_rows_log = ctx->params.rows(m);
    return GF2X_OK;
}

int gf2x_autotune(gf2x_ctx* ctx, int m_lo, int m_hi, int reps, gf2x_tune_rec* out) {
    if (check_ctx(ctx)) return GF2X_EINVAL;
    ctx->err.clear();
    if (m_lo < 1 || m_hi > 26 || m_lo > m_hi || reps < 1) return fail(ctx, GF2X_EINVAL, "autotune range");
    DeviceGuard g(ctx->device);
    TuneBuffers T;
    size_t need = 0;
    for (int M = m_lo; M <= m_hi; ++M) {
        const int copies = M >= 21 ? 1 : 1 << (21 - M);
        need = std::max(need, (size_t)copies * (align256(8ull << M) + align256(16ull << M)));
    }
    hipError_t e = hipMalloc((void**)&T.scratch, need);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, GF2X_ENOMEM, "autotune scratch");
    }
    e = hipMemset(T.scratch, 0, need);
    if (e == hipSuccess) e = hipEventCreate(&T.e0);
    if (e == hipSuccess) e = hipEventCreate(&T.e1);
    if (e != hipSuccess) return hip_fail(ctx, e, "autotune setup");
    for (int M = m_lo; M <= m_hi; ++M) {
        const int copies = M >= 21 ? 1 : 1 << (21 - M);
        PlanParams pp = ctx->params;
        std::vector<std::vector<std::pair<int, int>>> seen;
        float best = 0, dflt = 0;
        const PlanParams dflt_pp;
        int best_b = dflt_pp.bottom(M), best_r = dflt_pp.rows(M), ncand = 0;
        // the default first, then the candidates; schedules with the same
        // passes are timed once
        std::vector<std::pair<int, int>> cands{{best_b, best_r}};
        for (int b = kFftTileLog; b >= 7; --b)
            for (int r = 3; r <= kFftTileLog; ++r) cands.push_back({b, r});
        for (auto [b, r] : cands) {
            pp.fft_bottom_log[M] = (int8_t)b;
            pp.fft_col_rows_log[M] = (int8_t)r;
            auto ranges = fft_pass_ranges(M, pp);
            bool dup = false;
            for (auto& x : seen) dup |= x == ranges;
            if (dup) continue;
            seen.push_back(ranges);
            float us = 0;
            int rc = tune_time(ctx, T, pp, M, copies, reps, us);
            if (rc) return rc;
            ++ncand;
            if (ncand == 1) dflt = us;
            if (ncand == 1 || us < best) {
                best = us;
                best_b = b;
                best_r = r;
            }
        }
        ctx->params.fft_bottom_log[M] = (int8_t)best_b;
        ctx->params.fft_col_rows_log[M] = (int8_t)best_r;
        if (out) out[M - m_lo] = gf2x_tune_rec{M, best_b, best_r, copies, ncand, dflt, best};
    }
    return GF2X_OK;
}

int gf2x_set_truncation(gf2x_ctx* ctx, int levels, int min_log2n, int max_terms) {
    if (check_ctx(ctx)) return GF2X_EINVAL;
    if (levels < 0 || levels > 16) return fail(ctx, GF2X_EINVAL, "truncation levels outside 0..16");
    if (min_log2n < 1 || min_log2n > 32) return fail(ctx, GF2X_EINVAL, "truncation size outside 1..32");
    if (max_terms < 0 || max_terms > 32) return fail(ctx, GF2X_EINVAL, "truncation terms outside 0..32");
    ctx->params.trunc_levels = levels;
    ctx->params.trunc_min_log = min_log2n;
    ctx->params.trunc_max_terms = max_terms;
    return GF2X_OK;
}

int gf2x_set_word_bits(gf2x_ctx* ctx, int w) {
    if (check_ctx(ctx)) return GF2X_EINVAL;
    if (w != 64 && w != 128) return fail(ctx, GF2X_EINVAL, "word width must be 64 or 128");
    ctx->params.word_bits = w;
    return GF2X_OK;
}

int gf2x_get_word_bits(gf2x_ctx* ctx) { return ctx ? ctx->params.word_bits : 0; }

uint64_t gf2x_eval_points(gf2x_ctx* ctx, uint64_t na_bits, uint64_t nb_bits) {
    if (!ctx) return 0;
    const Sizes s = make_sizes(na_bits, nb_bits, ctx->params.word_bits);
    if (!s.out_words) return 0;
    return eval_points(s, ctx->params);
}

int gf2x_lookup_rate(gf2x_ctx* ctx, double* lookups_per_s) {
    if (check_ctx(ctx) || !lookups_per_s) return GF2X_EINVAL;
    ctx->err.clear();
    DeviceGuard g(ctx->device);
    const unsigned blocks = 2u * (unsigned)std::max(1, ctx->ncu);
    uint32_t* out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc((void**)&out, (size_t)blocks * kThreads * sizeof(uint32_t));
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float ms = 0;
    hipStream_t st = ctx->own_stream;
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {  // the first run warms up
        e = hipEventRecord(e0, st);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_lookup_rate, dim3(blocks), dim3(kThreads), 0, st, (const uint8_t*)ctx->d_mt, out);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    }
    if (out) (void)hipFree(out);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(ctx, e, "lookup rate");
    *lookups_per_s = (double)blocks * kThreads * kLookupIters * 8 / (ms * 1e-3);
    return GF2X_OK;
}

}  // extern "C"
