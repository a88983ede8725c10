// Planning: sizes of a product and the op list that computes it (Alg. 5).
#pragma once
#include <algorithm>
#include <cstdint>
#include <vector>

#include "afft_ops.hpp"

namespace gf2x {

enum class OpKind : int { Pack, BcTile, BcLayer, Fft, Pmul, Psi, BcClass, Spine };

struct Op {
    OpKind kind;
    uint32_t level;  // dependency level inside one product: an op needs every op of lower level done
    PackOp pack;
    BcTileOp bct;
    BcLayerOp bcl;
    FftPass fft;
    PmulOp pmul;
    PsiOp psi;
    BcClassOp bcc;
    SpineOp spn;
};

inline int ceil_log2(uint64_t n) {
    int l = 0;
    while ((1ull << l) < n) ++l;
    return l;
}

// Sizes of one product (readings: operands converted at their own power-of-two
// length; N = max(2, 2^ceil(log2(n_a + n_b - 1))) evaluation points).
// Sizes of one product with Split into w-bit words (w = 64: TGF(2^128);
// w = 128: TGF(2^256), Alg. 5).
struct Sizes {
    uint64_t na_bits = 0, nb_bits = 0;
    uint64_t n_a = 0, n_b = 0;    // 64-bit words of the operands
    int w = 64;                   // word width of Split
    uint64_t k_a = 0, k_b = 0;    // w-bit words of the operands
    int m_a = 0, m_b = 0, m = 0;  // log2 of k'_a, k'_b (converted lengths), N
    uint64_t out_words = 0;       // ceil((na + nb - 1) / 64)
    uint64_t nc_bits = 0;         // na + nb - 1
};

inline Sizes make_sizes(uint64_t na_bits, uint64_t nb_bits, int w = 64) {
    Sizes s;
    s.na_bits = na_bits;
    s.nb_bits = nb_bits;
    s.w = w;
    if (!na_bits || !nb_bits) return s;
    s.n_a = (na_bits + 63) / 64;
    s.n_b = (nb_bits + 63) / 64;
    s.k_a = (na_bits + w - 1) / w;
    s.k_b = (nb_bits + w - 1) / w;
    s.m_a = ceil_log2(s.k_a);
    s.m_b = ceil_log2(s.k_b);
    s.m = ceil_log2(s.k_a + s.k_b - 1);
    if (s.m < 1) s.m = 1;
    s.nc_bits = na_bits + nb_bits - 1;
    s.out_words = (s.nc_bits + 63) / 64;
    return s;
}

// Flat layer list of BasisCvt on 2^m units of 2^log_u elements (Alg. 3 with
// Alg. 2 unrolled into in-place divisions by x^D + x^k): with K the largest
// power of two below m, VarSubs divides by y^(2^j) = x^(2^(K+j)) + x^(2^j) for
// j = m-K-1 .. 0 on every aligned block; then the series in y is converted
// with units of 2^K elements, and finally every block of 2^K.
inline void bc_layer_list(int m, int log_u, std::vector<BcLayer>& out) {
    if (m <= 1) return;
    int K = 1;
    while (2 * K < m) K *= 2;
    for (int j = m - K - 1; j >= 0; --j) out.push_back(BcLayer{(uint32_t)(K + j), (uint32_t)j, (uint32_t)log_u, 0});
    bc_layer_list(m - K, log_u + K, out);
    bc_layer_list(K, log_u, out);
}

inline uint64_t bc_span_log(const BcLayer& L) { return L.log_d + 1 + L.log_u; }

// Every layer list a tile op can run (BasisCvt of 2^m units of 2^log_u
// elements with both at most kPoolMax), stored once; ops point into it.
constexpr int kPoolMax = 16;
struct LayerPool {
    std::vector<BcLayer> host;
    uint32_t off[kPoolMax + 1][kPoolMax + 1];
    uint32_t cnt[kPoolMax + 1][kPoolMax + 1];
    const BcLayer* base = nullptr;  // where the executing side reads `host`
    LayerPool() {
        for (int m = 0; m <= kPoolMax; ++m)
            for (int u = 0; u <= kPoolMax; ++u) {
                std::vector<BcLayer> L;
                bc_layer_list(m, u, L);
                off[m][u] = (uint32_t)host.size();
                cnt[m][u] = (uint32_t)L.size();
                host.insert(host.end(), L.begin(), L.end());
            }
    }
    const BcLayer* get(int m, int log_u, uint32_t& n) const {
        n = cnt[m][log_u];
        return base + off[m][log_u];
    }
};

// FFT pass schedule, per transform size M (2^M points, M <= 32): the bottom
// pass covers layers [0, b) on contiguous tiles of 2^b elements, and the
// layers above it are split evenly into strided passes of at most 2^r rows.
struct PlanParams {
    static constexpr int kMaxM = 32;
    int8_t fft_bottom_log[kMaxM + 1];
    int8_t fft_col_rows_log[kMaxM + 1];
    // Truncated transforms: a product of n_c = n_a + n_b - 1 word coefficients
    // is evaluated at M points, n_c rounded up to a multiple of 2^g,
    // g = max(m - trunc_levels, kTruncMinLog), and further to the next M whose
    // count of 2^g blocks has at most trunc_max_terms set bits (0: any): each
    // set bit is a full block plus spine steps, and a third one (M = 7/8 N)
    // measured slower than no truncation (M = N when trunc_levels = 0 or
    // m < trunc_min_log).
    // The spine steps need the multipliers on the host: the 32 x 32 table
    // lam[i][t] = s_i(v_t) and the GF(256) product table (both owned by the
    // caller; no truncation while either is null).
    // Only transforms of at least 2^trunc_min_log points are truncated (each
    // step of the recursion is a pass of its own, which smaller transforms
    // do not repay).
    static constexpr int kTruncMinLog = 6;
    int trunc_levels = 3;
    int trunc_min_log = 23;
    int trunc_max_terms = 2;
    // word width of Split: 64 (TGF(2^128)) or 128 (TGF(2^256), never truncated)
    int word_bits = 64;
    // 1: BasisCvt on 32 KiB tiles (single products; see kBcSmallShift)
    int bc_small = 0;
    // a one-pass transform's cosets are packed into tiles only while at
    // least this many tiles remain (0: as many to a tile as fit; batches and
    // the server, whose launches hold the tiles of many products; single
    // products keep one tile per CU at least)
    uint32_t fft_pack_min_tiles = 0;
    // BasisCvt sub-conversions inside the FFT passes whose rows hold their
    // index bits (FftPass): kFuseForward in forward transforms, kFuseInverse
    // in inverse ones, kFuseAlign splits the strided passes of a transform at
    // BasisCvt's top level when that keeps their number
    // (transforms of at most 2^fuse_max_log points only).  By default only
    // transforms of one small pass fuse (at most 2^11 points), where the
    // launches saved dominate: above that BasisCvt's layer sweeps, bound by
    // LDS and barriers as the FFT layers are by LDS lookups, cost the FFT
    // kernel about what their own pass costs, and the HBM round trip saved
    // was already overlapped
    enum : int { kFuseForward = 1, kFuseInverse = 2, kFuseAlign = 4 };
    int fuse_bc = kFuseForward | kFuseInverse | kFuseAlign;
    int fuse_max_log = 11;
    const uint32_t* lam = nullptr;
    const uint8_t* mt = nullptr;
    PlanParams() {
        for (int m = 0; m <= kMaxM; ++m) {
            fft_bottom_log[m] = 12;
            fft_col_rows_log[m] = 6;
        }
    }
    int bottom(int M) const { return fft_bottom_log[std::min(std::max(M, 0), kMaxM)]; }
    int rows(int M) const { return fft_col_rows_log[std::min(std::max(M, 0), kMaxM)]; }
};

// An FFT pass (once per plane) that can run one BasisCvt sub-conversion on
// its tile: its rows are index bits [lo, hi), at tile-element bit log_tc.
struct BcSlot {
    std::vector<FftPass*> passes;
    int lo, hi, log_tc, nel_log;
    bool used;
};

struct BcPlanner {
    void* data;
    int wide;
    uint64_t n;         // elements
    int cap_log;        // LDS capacity of a tile, log2 elements
    const LayerPool* pool;
    std::vector<Op> ops;
    std::vector<BcSlot>* slots = nullptr;
    struct Fused {
        int m, log_u, slot;
    };
    std::vector<Fused> fused;  // conversions assigned to slots (assign_slots)

    // a conversion of 2^m units of 2^log_u elements that one tile op runs
    bool tileable(int m, int log_u) const {
        return m + log_u <= cap_log || (log_u > 0 && m + std::min(log_u, 3) <= cap_log);
    }
    static int top_k(int m) {
        int K = 1;
        while (2 * K < m) K *= 2;
        return K;
    }

    // Which conversions run inside FFT passes: the nodes cvt() can reach (the
    // split ones and the tile-sized ones below them) whose bits [log_u,
    // log_u + m) lie in a slot's rows, one per slot, the largest first, never
    // a node together with one inside it.
    void assign_slots(int m_root) {
        if (!slots) return;
        struct Node {
            int m, log_u, parent;
            bool taken, below;  // assigned; some node inside it assigned
        };
        std::vector<Node> nodes;
        auto collect = [&](auto&& self, int m, int log_u, int parent) -> void {
            if (m <= 1) return;
            const int id = (int)nodes.size();
            nodes.push_back(Node{m, log_u, parent, false, false});
            if (tileable(m, log_u)) return;
            const int K = top_k(m);
            self(self, m - K, log_u + K, id);
            self(self, K, log_u, id);
        };
        collect(collect, m_root, 0, -1);
        std::vector<int> order(nodes.size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return nodes[x].m > nodes[y].m; });
        for (int id : order) {
            Node& nd = nodes[id];
            if (nd.below) continue;
            bool above = false;
            for (int p = nd.parent; p >= 0; p = nodes[p].parent) above = above || nodes[p].taken;
            if (above) continue;
            for (size_t k = 0; k < slots->size(); ++k) {
                BcSlot& sl = (*slots)[k];
                if (sl.used || nd.log_u < sl.lo || nd.log_u + nd.m > sl.hi) continue;
                sl.used = true;
                nd.taken = true;
                for (int p = nd.parent; p >= 0; p = nodes[p].parent) nodes[p].below = true;
                fused.push_back(Fused{nd.m, nd.log_u, (int)k});
                break;
            }
        }
    }

    // run the conversion inside its pass if assign_slots gave it one
    bool fuse(int m, int log_u) {
        for (const Fused& f : fused) {
            if (f.m != m || f.log_u != log_u) continue;
            const BcSlot& sl = (*slots)[f.slot];
            const int u = log_u - sl.lo + sl.log_tc;
            uint32_t nl = 0;
            const BcLayer* L = pool->get(m, u, nl);
            for (FftPass* A : sl.passes) {
                A->bc_layers = L;
                A->bc_n = nl;
            }
            return true;
        }
        return false;
    }

    // the layers of BasisCvt on 2^m units of 2^log_u LDS elements, on tiles
    void tile_pass(int log_rows, int log_stride, int log_tc, int m, int log_u) {
        Op op{};
        op.kind = OpKind::BcTile;
        op.bct.data = data;
        op.bct.nelem = n;
        op.bct.log_rows = (uint32_t)log_rows;
        op.bct.log_stride = (uint32_t)log_stride;
        op.bct.log_tc = (uint32_t)log_tc;
        op.bct.wide = (uint32_t)wide;
        op.bct.layers = pool->get(m, log_u, op.bct.nlayers);
        if (op.bct.nlayers) ops.push_back(op);
    }

    void global_layer(const BcLayer& L) {
        for (int part = 0; part < 2; ++part) {
            Op g{};
            g.kind = OpKind::BcLayer;
            g.bcl.data = data;
            g.bcl.nelem = n;
            g.bcl.wide = (uint32_t)wide;
            g.bcl.which = (uint32_t)part;
            g.bcl.layer = L;
            ops.push_back(g);
        }
    }

    // BasisCvt on every aligned block of 2^m units of 2^log_u elements.
    void cvt(int m, int log_u) {
        if (m <= 1) return;
        if (fuse(m, log_u)) return;
        const int blk_log = m + log_u;
        if (blk_log <= cap_log) {
            // whole blocks fit: a contiguous tile holds 2^(T - blk_log) of them
            int T = std::min<int>(cap_log, ceil_log2(n));
            tile_pass(T, 0, 0, m, log_u);
            return;
        }
        if (log_u > 0 && m + std::min(log_u, 3) <= cap_log) {
            // strided "column" tiles: all 2^m rows of up to 2^log_tc columns
            int log_tc = std::min(log_u, cap_log - m);
            tile_pass(m, log_u, log_tc, m, log_tc);  // row units scaled to LDS elements
            return;
        }
        const int K = top_k(m);
        uint64_t P = (1ull << K) - 1;
        uint64_t Q = ((1ull << m) + P - 1) / P;
        if (Q <= (1ull << cap_log)) {
            const uint64_t W = std::max<uint64_t>(1, std::min<uint64_t>((1ull << cap_log) / Q, P << log_u));
            Op op{};
            op.kind = OpKind::BcClass;
            op.bcc.data = data;
            op.bcc.nelem = n;
            op.bcc.m = (uint32_t)m;
            op.bcc.K = (uint32_t)K;
            op.bcc.log_u = (uint32_t)log_u;
            op.bcc.w = (uint32_t)W;
            op.bcc.w_magic = ((1ull << 32) + W - 1) / W;
            op.bcc.q_rows = (uint32_t)Q;
            op.bcc.wide = (uint32_t)wide;
            ops.push_back(op);
        } else {
            for (int j = m - K - 1; j >= 0; --j) global_layer(BcLayer{(uint32_t)(K + j), (uint32_t)j, (uint32_t)log_u, 0});
        }
        cvt(m - K, log_u + K);
        cvt(K, log_u);
    }
};

// Append a planned BasisCvt op list, or its inverse: the list reversed, each
// tile and class op running its layers backwards.  A layer too tall for any
// tile is two global ops (its two parts, each an XOR involution); reversing
// the list already runs them in the opposite order, which is their inverse.
inline void append_bc(std::vector<Op>& ops, const std::vector<Op>& fwd, int inverse) {
    if (!inverse) {
        for (const Op& op : fwd) ops.push_back(op);
        return;
    }
    for (size_t i = fwd.size(); i-- > 0;) {
        Op op = fwd[i];
        if (op.kind == OpKind::BcTile) op.bct.inverse = 1;
        if (op.kind == OpKind::BcClass) op.bcc.inverse = 1;
        ops.push_back(op);
    }
}

// Emit BasisCvt (or its inverse) of 2^m elements at `data`.
inline void emit_bc(std::vector<Op>& ops, const LayerPool& pool, void* data, int wide, int m, int inverse,
                    int small = 0) {
    const int shift = !small ? 0 : m <= kBcTinyMaxLog ? kBcTinyShift : kBcSmallShift;
    BcPlanner P{data, wide, 1ull << m, (wide ? kBcTileLog128 : kBcTileLog64) - shift, &pool, {}};
    P.cvt(m, 0);
    append_bc(ops, P.ops, inverse);
}

// Layer ranges of the FFT passes: a contiguous bottom pass of up to 2^b
// elements, and strided passes of up to 2^r rows above it (b, r from the
// schedule for M, both at most the 2^12-element tile).
inline std::vector<std::pair<int, int>> fft_pass_ranges(int M, const PlanParams& pp) {
    std::vector<std::pair<int, int>> col;
    int bottom = std::min(M, std::max(1, std::min(pp.bottom(M), kFftTileLog)));
    int rem = M - bottom;
    int rows = std::max(1, std::min(pp.rows(M), kFftTileLog));
    int ncol = (rem + rows - 1) / rows;
    // BasisCvt's top level (Alg. 3: K the largest power of two below M)
    // converts index bits [K, M); a top pass of exactly those rows runs it
    // (FftPass), if that keeps the number of passes and leaves the top pass
    // at least 16 columns
    int K = 1;
    while (2 * K < M) K *= 2;
    int top = 0;
    if ((pp.fuse_bc & PlanParams::kFuseAlign) && M <= pp.fuse_max_log && ncol >= 2 && K > bottom && M - K <= kFftTileLog - 4 && K - bottom >= ncol - 1 &&
        (K - bottom + ncol - 2) / (ncol - 1) <= kFftTileLog) {
        top = M - K;
        rem -= top;
        --ncol;
    }
    int lo = bottom;
    for (int c = 0; c < ncol; ++c) {
        int sz = rem / ncol + (c < rem % ncol ? 1 : 0);
        col.push_back({lo, lo + sz});
        lo += sz;
    }
    if (top) col.push_back({K, M});
    std::vector<std::pair<int, int>> r;
    r.push_back({0, bottom});
    for (auto& p : col) r.push_back(p);
    return r;  // bottom first (inverse order); the forward FFT runs it reversed
}

inline uint32_t fft_log_tc(int lo, int hi) {
    if (lo == 0) return 0;
    return (uint32_t)std::min(lo, kFftTileLog - (hi - lo));
}

// FFT passes over the aligned blocks coset0 .. coset0 + ncosets - 1 of
// length 2^log_m of a transform of length 2^log_total at `spec`: forward
// (top layers first; the first pass reads the 2^log_m converted words at
// `words` and applies changeRepr, unless words is null) or inverse.
inline void emit_fft_block(std::vector<Op>& ops, const PlanParams& pp, const void* words, uint4* spec, int log_m,
                           uint32_t coset0, uint32_t ncosets, int log_total, bool inverse,
                           uint32_t phi_mode = kPhi64) {
    auto ranges = fft_pass_ranges(log_m, pp);
    const size_t nr = ranges.size();
    for (size_t q = 0; q < nr; ++q) {
        const size_t r = inverse ? q : nr - 1 - q;
        const bool phi = !inverse && words && q == 0;  // a pass with no layers still converts the words
        if (ranges[r].first == ranges[r].second && !phi) continue;
        Op op{};
        op.kind = OpKind::Fft;
        FftPass& A = op.fft;
        A.phi_in = phi ? phi_mode : kPhiNone;
        A.src = A.phi_in ? (const void*)words : (const void*)spec;
        A.dst = spec;
        A.log_m = (uint32_t)log_m;
        A.lo = (uint32_t)ranges[r].first;
        A.hi = (uint32_t)ranges[r].second;
        A.log_tc = fft_log_tc(ranges[r].first, ranges[r].second);
        A.ncosets = ncosets;
        A.coset0 = coset0;
        A.inverse = inverse ? 1u : 0u;
        A.log_total = (uint32_t)log_total;
        // a transform done in one pass that fills less than a tile: as many
        // cosets to a tile as fit (an aligned run of them: the tile's row bits
        // then carry the cosets' global index bits)
        if (nr == 1 && log_m < kFftTileLog) {
            uint32_t pk = 0;
            while (log_m + (int)pk < kFftTileLog && ((ncosets | coset0) & ((2u << pk) - 1)) == 0 &&
                   (ncosets >> (pk + 1)) >= pp.fft_pack_min_tiles)
                ++pk;
            A.pack = pk;
        }
        ops.push_back(op);
    }
}

// Forward transform of one operand: `words` holds 2^M converted words; the
// spectrum has 2^(M + log_cosets) elements (all cosets).
inline void emit_fft_forward(std::vector<Op>& ops, const PlanParams& pp, const uint64_t* words, uint4* spec, int M,
                             int log_cosets) {
    emit_fft_block(ops, pp, words, spec, M, 0, 1u << log_cosets, M + log_cosets, false);
}

inline void emit_fft_inverse(std::vector<Op>& ops, const PlanParams& pp, uint4* spec, int m) {
    emit_fft_block(ops, pp, nullptr, spec, m, 0, 1, m, true);
}

// ----------------------------------------------------- truncated transforms
// Points evaluated for a product of sizes s (see PlanParams).
inline uint64_t eval_points(const Sizes& s, const PlanParams& pp) {
    const uint64_t N = 1ull << s.m;
    if (s.w != 64 || pp.trunc_levels <= 0 || s.m < pp.trunc_min_log || !pp.lam || !pp.mt) return N;
    const int g = std::max(s.m - pp.trunc_levels, PlanParams::kTruncMinLog);
    if (g >= s.m) return N;
    const uint64_t nc = s.n_a + s.n_b - 1;
    uint64_t q = (nc + (1ull << g) - 1) >> g;  // blocks of 2^g points, at most 2^(m - g)
    if (pp.trunc_max_terms > 0)
        while (__builtin_popcountll(q) > pp.trunc_max_terms) q += q & (~q + 1);
    return q << g;
}

// lambda of layer i for the block starting at global index s (a multiple of 2^(i+1))
inline uint32_t host_lambda(const PlanParams& pp, int i, uint64_t s) {
    uint32_t l = 0;
    for (uint64_t b = s >> (i + 1); b; b &= b - 1) l ^= pp.lam[i * 32 + i + 1 + __builtin_ctzll(b)];
    return l;
}

inline void emit_spine(std::vector<Op>& ops, const PlanParams& pp, uint32_t mode, uint4* x, uint4* y, uint64_t n,
                       uint32_t lambda, const uint64_t* words = nullptr) {
    Op op{};
    op.kind = OpKind::Spine;
    SpineOp& S = op.spn;
    S.x = x;
    S.y = y;
    S.words = words;
    S.n = n;
    S.mode = mode;
    S.mu = make_mu_k(pp.mt, lambda);
    const int w = lambda ? 32 - __builtin_clz(lambda) : 0;
    S.width = (uint32_t)width_mode(w);
    ops.push_back(op);
}

// Values at the first Mb points of the block of 2^n points at global index s
// of a transform of length 2^log_total whose coefficients are in place
// (Alg. 1 truncated): at each level only the half-blocks holding needed
// points are transformed further; a half whose points are all beyond Mb only
// needs the u side of its butterfly.
inline void emit_fwd_spine(std::vector<Op>& ops, const PlanParams& pp, uint4* spec, uint64_t s, int n, uint64_t Mb,
                           int log_total) {
    if (Mb == (1ull << n)) {
        emit_fft_block(ops, pp, nullptr, spec, n, (uint32_t)(s >> n), 1, log_total, false);
        return;
    }
    const uint64_t h = 1ull << (n - 1);
    const uint32_t lam = host_lambda(pp, n - 1, s);
    if (Mb > h) {
        emit_spine(ops, pp, kSpineFwd, spec + s, spec + s + h, h, lam);
        emit_fwd_spine(ops, pp, spec, s, n - 1, h, log_total);
        emit_fwd_spine(ops, pp, spec, s + h, n - 1, Mb - h, log_total);
    } else {
        if (lam) emit_spine(ops, pp, kSpineHalf, spec + s, spec + s + h, h, lam);
        emit_fwd_spine(ops, pp, spec, s, n - 1, Mb, log_total);
    }
}

// Coefficients of the block of 2^n points at global index s from its values
// at the first mk points and its coefficients at the other positions, all in
// place (the inverse of the truncated Alg. 1).  Write the block's
// coefficients as halves (U, V), transformed by the top butterfly into
// U' = U + lambda V (first half) and V' = U' + V (second half).
//   mk <= h: U' is known beyond mk (U and V are), the first half is the same
//     problem one level down; then U = U' + lambda V.
//   mk > h: the first half is a full inverse transform (U'); V' = U' + V is
//     known beyond mk - h, the second half is the same problem one level down;
//     then the inverse butterfly V = V' + U', U = U' + lambda V.
inline void emit_inv_spine(std::vector<Op>& ops, const PlanParams& pp, uint4* spec, uint64_t s, int n, uint64_t mk,
                           int log_total) {
    if (mk == 0) return;
    if (mk == (1ull << n)) {
        emit_fft_block(ops, pp, nullptr, spec, n, (uint32_t)(s >> n), 1, log_total, true);
        return;
    }
    const uint64_t h = 1ull << (n - 1);
    const uint32_t lam = host_lambda(pp, n - 1, s);
    if (mk <= h) {
        if (lam && mk < h) emit_spine(ops, pp, kSpineHalf, spec + s + mk, spec + s + h + mk, h - mk, lam);
        emit_inv_spine(ops, pp, spec, s, n - 1, mk, log_total);
        if (lam) emit_spine(ops, pp, kSpineHalf, spec + s, spec + s + h, h, lam);
    } else {
        emit_fft_block(ops, pp, nullptr, spec, n - 1, (uint32_t)(s >> (n - 1)), 1, log_total, true);
        if (mk < 2 * h) emit_spine(ops, pp, kSpineAdd, spec + s + mk - h, spec + s + mk, 2 * h - mk, 0);
        emit_inv_spine(ops, pp, spec, s + h, n - 1, mk - h, log_total);
        emit_spine(ops, pp, kSpineInv, spec + s, spec + s + h, h, lam);
    }
}

inline void emit_pack(std::vector<Op>& ops, const uint64_t* src, uint64_t nbits, uint64_t* dst, uint64_t ndst) {
    Op op{};
    op.kind = OpKind::Pack;
    op.pack = PackOp{src, nbits, dst, ndst};
    ops.push_back(op);
}

// Slots of the FFT passes in `ffts` (the same pass list once per plane).
inline std::vector<BcSlot> bc_slots(const std::vector<std::vector<Op>*>& ffts) {
    std::vector<BcSlot> sl;
    if (ffts.empty()) return sl;
    const std::vector<Op>& f0 = *ffts[0];
    for (size_t k = 0; k < f0.size(); ++k) {
        if (f0[k].kind != OpKind::Fft) continue;
        const FftPass& A = f0[k].fft;
        BcSlot b{{}, (int)A.lo, (int)A.hi, (int)A.log_tc, (int)(A.hi - A.lo + A.pack + A.log_tc), false};
        for (std::vector<Op>* v : ffts) b.passes.push_back(&(*v)[k].fft);
        sl.push_back(b);
    }
    return sl;
}

// BasisCvt of 2^m elements at `data` planned around FFT passes (BcSlot):
// the sub-conversions whose bits lie in a pass's rows run in that pass, the
// rest are returned as ops, in forward order.
// (dir: PlanParams::kFuseForward or kFuseInverse, the direction of the
// transforms)
inline std::vector<Op> plan_bc_around(const LayerPool& pool, const PlanParams& pp, void* data, int wide, int m,
                                      const std::vector<std::vector<Op>*>& ffts, int dir) {
    const int shift = !pp.bc_small ? 0 : m <= kBcTinyMaxLog ? kBcTinyShift : kBcSmallShift;
    BcPlanner P{data, wide, 1ull << m, (wide ? kBcTileLog128 : kBcTileLog64) - shift, &pool, {}};
    std::vector<BcSlot> sl;
    int log_total = 0;
    for (const std::vector<Op>* v : ffts)
        for (const Op& op : *v)
            if (op.kind == OpKind::Fft) log_total = std::max(log_total, (int)op.fft.log_total);
    if ((pp.fuse_bc & dir) && log_total <= pp.fuse_max_log) {
        sl = bc_slots(ffts);
        P.slots = &sl;
        P.assign_slots(m);
    }
    P.cvt(m, 0);
    return P.ops;
}

// How the operand (nbits bits at src) enters its forward transform, the
// words at `words` (nwords 64-bit words) being its converted copy: a first
// BasisCvt op on contiguous tiles reads it in place of a packed copy, and with
// no BasisCvt op left the changeRepr passes read it; otherwise a pack op
// copies it (a class pass gathers rows far apart, where reading the operand
// itself, with its bounds and mask per word, measured slower than the copy).
// Appends the pack op (if any) and the BasisCvt ops.
inline void emit_operand_bc(std::vector<Op>& ops, std::vector<Op>& bc, const std::vector<std::vector<Op>*>& ffts,
                            const uint64_t* src, uint64_t nbits, uint64_t* words, uint64_t nwords) {
    if (nbits && !bc.empty() && bc[0].kind == OpKind::BcTile && bc[0].bct.log_stride == 0) {
        bc[0].bct.src = src;
        bc[0].bct.src_bits = nbits;
    } else if (nbits && bc.empty()) {
        for (std::vector<Op>* v : ffts)
            for (Op& op : *v)
                if (op.kind == OpKind::Fft && op.fft.phi_in != kPhiNone) {
                    op.fft.src = src;
                    op.fft.src_bits = nbits;
                }
    } else {
        emit_pack(ops, src, nbits, words, nwords);
    }
    ops.insert(ops.end(), bc.begin(), bc.end());
}

inline void emit_pmul(std::vector<Op>& ops, const uint4* a, const uint4* b, uint4* c, uint64_t n,
                      uint64_t n_out = 0) {
    Op op{};
    op.kind = OpKind::Pmul;
    op.pmul = PmulOp{a, b, c, n, n_out > n ? n_out : n};
    ops.push_back(op);
}

inline void emit_psi(std::vector<Op>& ops, const uint4* spec, uint64_t nspec, uint64_t* out, uint64_t nbits) {
    Op op{};
    op.kind = OpKind::Psi;
    op.psi = PsiOp{spec, nspec, out, (nbits + 63) / 64, nbits};
    ops.push_back(op);
}

// Workspace of one product: converted words of a and b, then the two spectra.
struct Workspace {
    size_t off_wa, off_wb, off_sa, off_sb, bytes;
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// (w = 128: words of 16 bytes, and each spectrum is two planes of N uint4)
inline Workspace workspace_for(const Sizes& s) {
    Workspace w{};
    const size_t wb = (size_t)s.w / 8, sb = 16 * ((size_t)s.w / 64);
    size_t o = 0;
    w.off_wa = o;
    o = align256(o + (wb << s.m_a));
    w.off_wb = o;
    o = align256(o + (wb << s.m_b));
    w.off_sa = o;
    o = align256(o + (sb << s.m));
    w.off_sb = o;
    o = align256(o + (sb << s.m));
    w.bytes = o;
    return w;
}

// Forward transform of one operand into an N-point spectrum (Split, BasisCvt
// on 64-bit words, changeRepr, FFT_LCH at 0).  `words` is scratch of 2^m_op words.
// Values at the first M of N = 2^m points: the cosets of length 2^m_op
// entirely below M are full transforms, the one holding M is truncated.
inline void emit_forward(std::vector<Op>& ops, const LayerPool& pool, const PlanParams& pp, const uint64_t* src,
                         uint64_t nbits, uint64_t* words, int m_op, uint4* spec, int m, uint64_t M) {
    if (M == (1ull << m)) {
        std::vector<Op> fft;
        emit_fft_forward(fft, pp, words, spec, m_op, m - m_op);
        std::vector<Op> bc = plan_bc_around(pool, pp, words, 0, m_op, {&fft}, PlanParams::kFuseForward);
        emit_operand_bc(ops, bc, {&fft}, src, nbits, words, 1ull << m_op);
        ops.insert(ops.end(), fft.begin(), fft.end());
        return;
    }
    // a truncated transform mixes the top bits of the converted words before
    // its FFT blocks (spine steps): BasisCvt runs whole, before it
    emit_pack(ops, src, nbits, words, 1ull << m_op);
    emit_bc(ops, pool, words, 0, m_op, 0, pp.bc_small);
    const uint64_t full = M >> m_op, rem = M - (full << m_op);
    if (full) emit_fft_block(ops, pp, words, spec, m_op, 0, (uint32_t)full, m, false);
    if (rem) {
        const uint64_t s0 = full << m_op;
        emit_spine(ops, pp, kSpinePhi, spec + s0, nullptr, 1ull << m_op, 0, words);
        emit_fwd_spine(ops, pp, spec, s0, m_op, rem, m);
    }
}

// Inverse transform of the values at the first M of N = 2^m points into
// nc_bits product bits (iFFT_LCH, iBasisCvt, changeRepr back,
// InterleavedCombine); positions M and beyond hold the (zero) coefficients
// there.
inline void emit_inverse(std::vector<Op>& ops, const LayerPool& pool, const PlanParams& pp, uint4* spec, int m,
                         uint64_t M, uint64_t* out, uint64_t nc_bits) {
    if (M == (1ull << m)) {
        std::vector<Op> fft;
        emit_fft_inverse(fft, pp, spec, m);
        const std::vector<Op> bc = plan_bc_around(pool, pp, spec, 1, m, {&fft}, PlanParams::kFuseInverse);
        ops.insert(ops.end(), fft.begin(), fft.end());
        append_bc(ops, bc, 1);
    } else {
        emit_inv_spine(ops, pp, spec, 0, m, M, m);  // pointmul wrote zeros at M and beyond
        emit_bc(ops, pool, spec, 1, m, 1, pp.bc_small);
    }
    emit_psi(ops, spec, 1ull << m, out, nc_bits);
}

// w = 128: the product over TGF(2^256).  A spectrum is two planes of N
// uint4 (the low and high TGF(2^128) halves of every point); multiplying by a
// subfield element acts on each half alone (Prop. 2), so each plane runs the
// w = 64 FFT passes with the same multipliers, the changeRepr pass keeping
// its half of the image of each 128-bit word.  BasisCvt and its inverse act
// on whole coefficients, so on 128-bit words, and on each plane alone.  Ops
// of the two planes are independent and share levels.
inline void plan_mul128(std::vector<Op>& ops, const LayerPool& pool, const PlanParams& pp, const Sizes& s,
                        const uint64_t* a, const uint64_t* b, uint64_t* c, char* ws, size_t* split = nullptr) {
    const Workspace w = workspace_for(s);
    const uint64_t N = 1ull << s.m;
    uint4* wa = (uint4*)(ws + w.off_wa);
    uint4* wb = (uint4*)(ws + w.off_wb);
    uint4* sa = (uint4*)(ws + w.off_sa);
    uint4* sb = (uint4*)(ws + w.off_sb);
    auto forward = [&](const uint64_t* src, uint64_t nbits, uint4* words, int m_op, uint4* spec) {
        std::vector<Op> pre, pl[2];
        for (int h = 0; h < 2; ++h)
            emit_fft_block(pl[h], pp, words, spec + h * N, m_op, 0, 1u << (s.m - m_op), s.m, false,
                           h ? kPhi128Hi : kPhi128Lo);
        std::vector<Op> bc = plan_bc_around(pool, pp, words, 1, m_op, {&pl[0], &pl[1]}, PlanParams::kFuseForward);
        emit_operand_bc(pre, bc, {&pl[0], &pl[1]}, src, nbits, (uint64_t*)words, 2ull << m_op);
        uint32_t l = 0;
        for (Op op : pre) {
            op.level = l++;
            ops.push_back(op);
        }
        for (size_t q = 0; q < pl[0].size(); ++q)
            for (int h = 0; h < 2; ++h) {
                Op op = pl[h][q];
                op.level = l + (uint32_t)q;
                ops.push_back(op);
            }
        return l + (uint32_t)pl[0].size();
    };
    const size_t a0 = ops.size();
    const uint32_t la = forward(a, s.na_bits, wa, s.m_a, sa);
    const size_t b0 = ops.size();
    const uint32_t lb = forward(b, s.nb_bits, wb, s.m_b, sb);
    if (split && a0 == 0) {
        split[0] = b0;
        split[1] = ops.size();
    }
    const uint32_t lp = std::max(la, lb);
    Op pm{};
    pm.kind = OpKind::Pmul;
    pm.pmul = PmulOp{sa, sb, sb, N, N, sa + N, sb + N, sb + N};
    pm.level = lp;
    ops.push_back(pm);
    std::vector<Op> inv[2];
    for (int h = 0; h < 2; ++h) {
        emit_fft_inverse(inv[h], pp, sb + h * N, s.m);
        const std::vector<Op> bc = plan_bc_around(pool, pp, sb + h * N, 1, s.m, {&inv[h]}, PlanParams::kFuseInverse);
        append_bc(inv[h], bc, 1);
    }
    for (size_t q = 0; q < inv[0].size(); ++q)
        for (int h = 0; h < 2; ++h) {
            Op op = inv[h][q];
            op.level = lp + 1 + (uint32_t)q;
            ops.push_back(op);
        }
    Op ps{};
    ps.kind = OpKind::Psi;
    ps.psi = PsiOp{sb, N, c, s.out_words, s.nc_bits, sb + N};
    ps.level = lp + 1 + (uint32_t)inv[0].size();
    ops.push_back(ps);
}

// The whole product c = a * b with the workspace at `ws`.  If `split` is
// given, split[0] and split[1] receive the ends of the forward transform of a
// (ops [0, split[0])) and of b (ops [split[0], split[1])).
inline void plan_mul(std::vector<Op>& ops, const LayerPool& pool, const PlanParams& pp, const Sizes& s, const uint64_t* a,
                     const uint64_t* b, uint64_t* c, char* ws, size_t* split = nullptr) {
    if (s.w == 128) {
        plan_mul128(ops, pool, pp, s, a, b, c, ws, split);
        return;
    }
    Workspace w = workspace_for(s);
    uint64_t* wa = (uint64_t*)(ws + w.off_wa);
    uint64_t* wb = (uint64_t*)(ws + w.off_wb);
    uint4* sa = (uint4*)(ws + w.off_sa);
    uint4* sb = (uint4*)(ws + w.off_sb);
    // the two forward transforms are independent and share levels
    const size_t a0 = ops.size();
    const uint64_t M = eval_points(s, pp);
    emit_forward(ops, pool, pp, a, s.na_bits, wa, s.m_a, sa, s.m, M);
    const size_t b0 = ops.size();
    emit_forward(ops, pool, pp, b, s.nb_bits, wb, s.m_b, sb, s.m, M);
    const size_t p0 = ops.size();
    for (size_t i = a0; i < b0; ++i) ops[i].level = (uint32_t)(i - a0);
    for (size_t i = b0; i < p0; ++i) ops[i].level = (uint32_t)(i - b0);
    const uint32_t lp = (uint32_t)std::max(b0 - a0, p0 - b0);
    if (split && a0 == 0) {
        split[0] = b0;
        split[1] = p0;
    }
    emit_pmul(ops, sa, sb, sb, M, 1ull << s.m);
    emit_inverse(ops, pool, pp, sb, s.m, M, c, s.nc_bits);
    for (size_t i = p0; i < ops.size(); ++i) ops[i].level = lp + (uint32_t)(i - p0);
}

// Number of dependency levels of a planned product.
inline uint32_t plan_levels(const std::vector<Op>& ops) {
    uint32_t l = 0;
    for (const Op& op : ops) l = std::max(l, op.level + 1);
    return l;
}

}  // namespace gf2x

namespace gf2x {

// ------------------------------------------------------------------ batches
// A batch of independent products is planned job by job; op r of every job
// has rank r.  Ops of one rank and kind run in one launch (a "group"), and
// groups launch rank by rank, so op r of a job starts after op r - 1 of the
// same job has finished.

struct BatchJob {
    const uint64_t* a;
    uint64_t na_bits;
    const uint64_t* b;
    uint64_t nb_bits;
    uint64_t* c;
};

struct BatchGroup {
    OpKind kind;
    int wide;
    std::vector<uint32_t> ops;  // indices into BatchPlan::ops
};

// A group's descriptor image: offsets of its op records and tile prefix sums
// (global BasisCvt layers are launched one by one, from host copies).
struct LaunchGroup {
    OpKind kind;
    int wide;
    size_t ops_off, prefix_off;
    int nops;
    uint64_t total;
    std::vector<BcLayerOp> layers;
};

struct BatchPlan {
    std::vector<Op> ops;
    std::vector<uint32_t> job_of;
    std::vector<uint32_t> rank_of;
    std::vector<BatchGroup> groups;
    std::vector<size_t> ws_off;  // per job
    size_t ws_bytes = 0;
    uint32_t max_rank = 0;
};

inline uint64_t op_tiles(const Op& op) {
    switch (op.kind) {
        case OpKind::Pack: return pack_tiles(op.pack);
        case OpKind::BcTile: return bc_tiles(op.bct);
        case OpKind::BcLayer: return 1;
        case OpKind::Fft: return fft_tiles(op.fft);
        case OpKind::Pmul: return pmul_tiles(op.pmul);
        case OpKind::Psi: return psi_tiles(op.psi);
        case OpKind::BcClass: return bc_class_tiles(op.bcc);
        case OpKind::Spine: return spine_tiles(op.spn);
    }
    return 0;
}

inline int op_wide(const Op& op) {
    if (op.kind == OpKind::BcTile) return (int)op.bct.wide;
    if (op.kind == OpKind::BcClass) return (int)op.bcc.wide;
    if (op.kind == OpKind::BcLayer) return (int)op.bcl.wide;
    return 0;
}

// Groups of ops[first..] by (rank, kind, wide), rank by rank; rank_of gives
// each op's rank, and ranks run from 0 to nranks - 1.
inline void group_by_rank(const std::vector<Op>& ops, const std::vector<uint32_t>& rank_of, size_t first,
                          uint32_t nranks, std::vector<BatchGroup>& out) {
    std::vector<std::vector<uint32_t>> by_rank(nranks);
    for (size_t i = first; i < ops.size(); ++i) by_rank[rank_of[i]].push_back((uint32_t)i);
    for (uint32_t r = 0; r < nranks; ++r) {
        std::vector<BatchGroup> g;
        for (uint32_t idx : by_rank[r]) {
            const Op& op = ops[idx];
            const int w = op_wide(op);
            BatchGroup* G = nullptr;
            for (auto& x : g)
                if (x.kind == op.kind && x.wide == w) G = &x;
            if (!G) {
                g.push_back(BatchGroup{op.kind, w, {}});
                G = &g.back();
            }
            G->ops.push_back(idx);
        }
        for (auto& x : g) out.push_back(std::move(x));
    }
}

// Workspace sizes first (ws == nullptr), then the ops with real addresses.
inline void plan_batch(BatchPlan& P, const LayerPool& pool, const PlanParams& pp, const BatchJob* jobs, size_t njobs,
                       char* ws) {
    P = BatchPlan();
    P.ws_off.assign(njobs, 0);
    size_t total = 0;
    for (size_t j = 0; j < njobs; ++j) {
        Sizes s = make_sizes(jobs[j].na_bits, jobs[j].nb_bits, pp.word_bits);
        P.ws_off[j] = total;
        if (s.out_words) total += workspace_for(s).bytes;
    }
    P.ws_bytes = total;
    if (!ws) return;
    for (size_t j = 0; j < njobs; ++j) {
        Sizes s = make_sizes(jobs[j].na_bits, jobs[j].nb_bits, pp.word_bits);
        if (!s.out_words) continue;
        const size_t first = P.ops.size();
        plan_mul(P.ops, pool, pp, s, jobs[j].a, jobs[j].b, jobs[j].c, ws + P.ws_off[j]);
        for (size_t i = first; i < P.ops.size(); ++i) {
            P.job_of.push_back((uint32_t)j);
            P.rank_of.push_back(P.ops[i].level);
            P.max_rank = std::max<uint32_t>(P.max_rank, P.ops[i].level + 1);
        }
    }
    group_by_rank(P.ops, P.rank_of, 0, P.max_rank, P.groups);
}

}  // namespace gf2x
