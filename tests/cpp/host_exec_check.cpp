// Host-side check of the planner and the kernel bodies: the op lists the
// library plans (single products, batches by level and kind, truncated
// transforms, BasisCvt tile and class passes) are executed sequentially on
// the CPU (thread 0 of 1, the same tile bodies the kernels run) and every
// product is compared with the oracle.  No GPU is involved.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "afft_plan.hpp"
#include "frobenius.hpp"
#include "simple.hpp"
#include "tower_host.hpp"

using namespace gf2x;

extern "C" int oracle_mul(const uint64_t* a, size_t na_bits, const uint64_t* b, size_t nb_bits, uint64_t* c,
                          int threads);

namespace {

std::vector<uint8_t> MT(65536);
std::vector<uint32_t> LAM(1024);
std::vector<uint4> PHIN(kPhinTotal), PSI(kPsiTab64 + kPsiTab128);
std::vector<uint2> MT3(768);
std::vector<uint32_t> CTAB;
LayerPool POOL;
PlanParams PP;

uint4 to_u4(u128 v) { return make_uint4((uint32_t)v, (uint32_t)(v >> 32), (uint32_t)(v >> 64), (uint32_t)(v >> 96)); }

bool init() {
    POOL.base = POOL.host.data();
    HostTower T;
    for (int a = 0; a < 256; ++a)
        for (int b = 0; b < 256; ++b) MT[a * 256 + b] = T.mt8[a][b];
    uint32_t lam[32][32];
    build_lambda(T, lam);
    memcpy(LAM.data(), lam, sizeof(lam));
    ReprTables R = build_repr(T);
    if (!R.ok) return false;
    for (int i = 0; i < kPhinTotal; ++i) PHIN[i] = to_u4(R.phin[i]);
    for (int i = 0; i < kPsiTab64; ++i) PSI[i] = to_u4(R.psi[i]);
    for (int i = 0; i < kPsiTab128; ++i) PSI[kPsiTab64 + i] = to_u4(R.psin[i]);
    CTAB = build_const_tabs(T);
    PP.lam = LAM.data();
    PP.mt = MT.data();
    build_mt3(0, 1, MT.data(), MT3.data());
    return true;
}

struct Scratch {
    std::vector<uint4> tl = std::vector<uint4>(1 << kFftTileLog), mu = std::vector<uint4>(kMuEntries),
                       mut = std::vector<uint4>(32);
    std::vector<uint64_t> l64 = std::vector<uint64_t>(1 << kBcTileLog64);
    std::vector<uint4> l128 = std::vector<uint4>(1 << kBcTileLog128);
};

void run_tile(const Op& op, uint64_t t, Scratch& S) {
    switch (op.kind) {
        case OpKind::Pack: pack_tile(0, 1, t, op.pack); break;
        case OpKind::BcTile:
            if (op.bct.wide)
                bc_tile<uint4>(0, 1, t, op.bct, S.l128.data());
            else
                bc_tile<uint64_t>(0, 1, t, op.bct, S.l64.data());
            break;
        case OpKind::BcLayer:
            if (op.bcl.wide)
                bc_part<uint4>(0, 1, (uint4*)op.bcl.data, op.bcl.nelem, op.bcl.layer, (int)op.bcl.which);
            else
                bc_part<uint64_t>(0, 1, (uint64_t*)op.bcl.data, op.bcl.nelem, op.bcl.layer, (int)op.bcl.which);
            break;
        case OpKind::Fft:
            fft_local_mu(0, 1, op.fft, MT.data(), LAM.data(), S.mu.data());
            fft_tile<kFftRL>(0, 1, t, op.fft, MT.data(), MT3.data(), LAM.data(), PHIN.data() + phin_off(op.fft.phi_in),
                             S.tl.data(), S.mu.data(),
                             S.mut.data());
            break;
        case OpKind::Pmul: pmul_tile(0, 1, t, op.pmul, MT.data(), CTAB.data()); break;
        case OpKind::Psi: psi_tile(0, 1, t, op.psi, PSI.data() + psi_tab_off(op.psi)); break;
        case OpKind::BcClass:
            if (op.bcc.wide)
                bc_class_tile<uint4>(0, 1, t, op.bcc, S.l128.data());
            else
                bc_class_tile<uint64_t>(0, 1, t, op.bcc, S.l64.data());
            break;
        case OpKind::Spine: spine_tile(0, 1, t, op.spn, MT.data(), PHIN.data()); break;
    }
}

void run_ops(const std::vector<Op>& ops) {
    Scratch S;
    for (const Op& op : ops) {
        const uint64_t n = op_tiles(op);
        for (uint64_t t = 0; t < n; ++t) run_tile(op, t, S);
    }
}

std::vector<uint64_t> rand_words(std::mt19937_64& g, uint64_t nbits) {
    std::vector<uint64_t> w((nbits + 63) / 64);
    for (auto& x : w) x = g();
    return w;
}

// one product through the planner, compared with the oracle
bool check_product(std::mt19937_64& g, uint64_t na, uint64_t nb) {
    Sizes s = make_sizes(na, nb, PP.word_bits);
    Workspace w = workspace_for(s);
    std::vector<char> ws(w.bytes, 0x5a);  // garbage: the plan must not read what it did not write
    auto a = rand_words(g, na), b = rand_words(g, nb);
    std::vector<uint64_t> c(s.out_words + 1, 0xdead), r(s.out_words + 1, 0);
    std::vector<Op> ops;
    plan_mul(ops, POOL, PP, s, a.data(), b.data(), c.data(), ws.data());
    run_ops(ops);
    oracle_mul(a.data(), na, b.data(), nb, r.data(), 4);
    const bool ok = memcmp(c.data(), r.data(), 8 * s.out_words) == 0 && c[s.out_words] == 0xdead;
    if (!ok)
        printf("MISMATCH %llu x %llu bits (w = %d, N = 2^%d, M = %llu, truncation %d)\n", (unsigned long long)na,
               (unsigned long long)nb, s.w, s.m, (unsigned long long)eval_points(s, PP), PP.trunc_levels);
    return ok;
}

// a batch run group by group, tiles mapped to ops by the prefix sums as the
// multi-op kernels do
bool check_batch(std::mt19937_64& g, int njobs) {
    std::vector<BatchJob> jobs(njobs);
    std::vector<std::vector<uint64_t>> A(njobs), B(njobs), C(njobs);
    for (int j = 0; j < njobs; ++j) {
        uint64_t na = 1 + g() % (1ull << (1 + g() % 17)), nb = 1 + g() % (1ull << (1 + g() % 17));
        A[j] = rand_words(g, na);
        B[j] = rand_words(g, nb);
        C[j].assign((na + nb - 1 + 63) / 64 + 1, 0xdead);
        jobs[j] = BatchJob{A[j].data(), na, B[j].data(), nb, C[j].data()};
    }
    BatchPlan P;
    plan_batch(P, POOL, PP, jobs.data(), njobs, nullptr);
    std::vector<char> ws(P.ws_bytes + 16, 0x5a);
    plan_batch(P, POOL, PP, jobs.data(), njobs, ws.data());
    Scratch S;
    for (const BatchGroup& G : P.groups) {
        std::vector<uint64_t> prefix(G.ops.size() + 1, 0);
        for (size_t i = 0; i < G.ops.size(); ++i) prefix[i + 1] = prefix[i] + op_tiles(P.ops[G.ops[i]]);
        int o = -1;
        for (uint64_t t = 0; t < prefix.back(); ++t) {
            o = op_of_tile(prefix.data(), (int)G.ops.size(), t, o);
            run_tile(P.ops[G.ops[o]], t - prefix[o], S);
        }
    }
    int bad = 0;
    for (int j = 0; j < njobs; ++j) {
        const uint64_t ow = (jobs[j].na_bits + jobs[j].nb_bits - 1 + 63) / 64;
        std::vector<uint64_t> r(ow + 1, 0);
        oracle_mul(A[j].data(), jobs[j].na_bits, B[j].data(), jobs[j].nb_bits, r.data(), 4);
        if (memcmp(r.data(), C[j].data(), 8 * ow) || C[j][ow] != 0xdead) ++bad;
    }
    if (bad) printf("batch MISMATCH in %d of %d jobs\n", bad, njobs);
    return bad == 0;
}

// BasisCvt as tile and class passes against the flat layer list, both directions
template <typename T>
T rnd_elem(std::mt19937_64& g);
template <>
uint64_t rnd_elem<uint64_t>(std::mt19937_64& g) {
    return g();
}
template <>
uint4 rnd_elem<uint4>(std::mt19937_64& g) {
    const uint64_t a = g(), b = g();
    return make_uint4((uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32));
}
bool same(uint64_t a, uint64_t b) { return a == b; }
bool same(uint4 a, uint4 b) { return a.x == b.x && a.y == b.y && a.z == b.z && a.w == b.w; }

template <typename T>
bool check_basiscvt(int m, int small) {
    std::mt19937_64 g(1000 + m);
    const uint64_t n = 1ull << m;
    std::vector<T> a(n), flat, orig;
    for (auto& x : a) x = rnd_elem<T>(g);
    flat = a;
    orig = a;
    const int wide = sizeof(T) == 16;
    std::vector<Op> ops;
    emit_bc(ops, POOL, a.data(), wide, m, 0, small);
    run_ops(ops);
    std::vector<BcLayer> L;
    bc_layer_list(m, 0, L);
    for (const BcLayer& l : L)
        for (int part = 0; part < 2; ++part) bc_part<T>(0, 1, flat.data(), n, l, part);
    bool ok = true;
    for (uint64_t i = 0; i < n && ok; ++i) ok = same(a[i], flat[i]);
    std::vector<Op> inv;
    emit_bc(inv, POOL, a.data(), wide, m, 1, small);
    run_ops(inv);
    for (uint64_t i = 0; i < n && ok; ++i) ok = same(a[i], orig[i]);
    if (!ok) printf("BasisCvt MISMATCH m = %d, %s, %s tiles\n", m, wide ? "128-bit" : "64-bit", small ? "small" : "large");
    return ok;
}

// BasisCvt planned on tiles of 2^cap_log elements, so small that some layers
// fit no class tile and run as global layer ops: forward against the flat
// layer list, then the inverse back to the input.
template <typename T>
bool check_basiscvt_cap(int m, int cap_log) {
    std::mt19937_64 g(2000 + m);
    const uint64_t n = 1ull << m;
    std::vector<T> a(n), flat, orig;
    for (auto& x : a) x = rnd_elem<T>(g);
    flat = a;
    orig = a;
    const int wide = sizeof(T) == 16;
    BcPlanner P{a.data(), wide, n, cap_log, &POOL, {}};
    P.cvt(m, 0);
    bool global = false;
    for (const Op& op : P.ops) global |= op.kind == OpKind::BcLayer;
    std::vector<Op> ops;
    append_bc(ops, P.ops, 0);
    run_ops(ops);
    std::vector<BcLayer> L;
    bc_layer_list(m, 0, L);
    for (const BcLayer& l : L)
        for (int part = 0; part < 2; ++part) bc_part<T>(0, 1, flat.data(), n, l, part);
    bool ok = global;
    for (uint64_t i = 0; i < n && ok; ++i) ok = same(a[i], flat[i]);
    std::vector<Op> inv;
    append_bc(inv, P.ops, 1);
    run_ops(inv);
    for (uint64_t i = 0; i < n && ok; ++i) ok = same(a[i], orig[i]);
    if (!ok)
        printf("BasisCvt with global layers MISMATCH m = %d, tiles of 2^%d, %s (global layers planned: %d)\n", m,
               cap_log, wide ? "128-bit" : "64-bit", (int)global);
    return ok;
}

// The XCD-aware block-to-tile order of the block-strided kernels visits every
// tile exactly once, for grids that are and are not multiples of 8 and tile
// counts with and without a partial last round.
bool check_xcd_order(std::mt19937_64& g) {
    std::vector<uint64_t> grids = {1, 7, 8, 16, 255, 256, 512, 1024, 2048};
    for (int i = 0; i < 20; ++i) grids.push_back(1 + g() % 3000);
    for (uint64_t grid : grids) {
        std::vector<uint64_t> counts = {0, 1, grid - 1, grid, grid + 1, 2 * grid, 8 * grid + 3, 5 * grid};
        for (int i = 0; i < 10; ++i) counts.push_back(g() % (20 * grid + 1));
        for (uint64_t nt : counts) {
            std::vector<uint8_t> seen(nt, 0);
            for (uint64_t b = 0; b < grid; ++b)
                for (uint64_t t = b; t < nt; t += grid) {
                    const uint64_t x = xcd_tile(t, grid, nt);
                    if (x >= nt || seen[x]++) {
                        printf("XCD order MISMATCH grid %llu, tiles %llu\n", (unsigned long long)grid,
                               (unsigned long long)nt);
                        return false;
                    }
                }
            for (uint64_t x = 0; x < nt; ++x)
                if (!seen[x]) {
                    printf("XCD order misses tile %llu (grid %llu, tiles %llu)\n", (unsigned long long)x,
                           (unsigned long long)grid, (unsigned long long)nt);
                    return false;
                }
        }
    }
    // blocks of one XCD (b mod 8 equal) take a contiguous run in a full round
    const uint64_t grid = 256, nt = 2048;
    for (uint64_t xcd = 0; xcd < 8; ++xcd)
        for (uint64_t j = 0; j + 1 < grid / 8; ++j)
            if (xcd_tile(xcd + 8 * (j + 1), grid, nt) != xcd_tile(xcd + 8 * j, grid, nt) + 1) {
                printf("XCD order: run of XCD %llu broken\n", (unsigned long long)xcd);
                return false;
            }
    return true;
}

// ---- the simple variant (Alg. 4): the FFT passes, pointmul and combine run
// here with the bodies the kernels run, workgroup by workgroup and phase by
// phase (every thread of a phase before any of the next, as the barriers do)
std::vector<uint4> CANTOR;

// The bottom pass: chunks of 64 groups of 2^G points, one group per thread
// (points past N are zero and not stored).
template <int G>
void run_sfft_groups(const SfftPass& P, uint4* T) {
    for (uint64_t c = 0; c < ((P.n + (1ull << (G + 6)) - 1) >> (G + 6)); ++c) {
        const uint64_t J0 = c << (G + 6);
        for (uint32_t g = 0; g < 64; ++g) {
            uint4 x[1 << G];
            for (int p = 0; p < (1 << G); ++p) {
                const uint64_t j = J0 + (g << G) + p;
                x[p] = j < P.n ? sfft_load(P, j) : make_uint4(0u, 0u, 0u, 0u);
            }
            if (P.inverse)
                sf_group_layers<G, true>(P, J0, g, x, T, CANTOR.data());
            else
                sf_group_layers<G, false>(P, J0, g, x, T, CANTOR.data());
            for (int p = 0; p < (1 << G); ++p) {
                const uint64_t j = J0 + (g << G) + p;
                if (j < P.n) P.x[j] = x[p];
            }
        }
    }
}

void run_sfft(const std::vector<SfftPass>& passes) {
    std::vector<uint4> tab(((1 << kSfTabL) - 1) * kSfTabStride), dat(1 << kSfTabPtsLog), T(16 * kSfLaneTabStride);
    for (const SfftPass& P : passes) {
        if (P.lo == 0) {
            if (P.c == 2)
                run_sfft_groups<2>(P, T.data());
            else
                run_sfft_groups<3>(P, T.data());
        } else {
            const uint32_t npts = 1u << (P.L + P.c), ntab = (1u << P.L) - 1;
            for (uint64_t g = 0; g < sf_tab_groups(P); ++g) {
                for (uint32_t e = 0; e < npts; ++e) dat[e] = sfft_load(P, sf_tab_point(P, g, e));
                for (uint32_t t = 0; t < ntab; ++t) sf_tab_table(P, g, t, CANTOR.data(), tab.data());
                for (int s = 0; s < P.L;)
                    if (sf_tab_quads(P, s)) {
                        for (uint32_t q = 0; q < npts / 4; ++q) sf_tab_quad(P, s, q, dat.data(), tab.data());
                        s += 2;
                    } else {
                        for (uint32_t q = 0; q < npts / 2; ++q) sf_tab_bfly(P, s, q, dat.data(), tab.data());
                        s += 1;
                    }
                for (uint32_t e = 0; e < npts; ++e) P.x[sf_tab_point(P, g, e)] = dat[e];
            }
        }
    }
}

// The pass plan of every transform size: the bottom pass first (inverse) or
// last (forward) with groups of 2^c, c = 2 or 3, and layers [0, min(M, c));
// strided passes of 1..kSfTabL layers covering the rest of [0, M) once, in
// order, each with 2^c consecutive points, c <= lo and L + c <= kSfTabPtsLog;
// groups of 4 exactly when N <= 2^kSfGroupSmallLog and they add no strided
// pass; the forward transform's first pass reads the words.
bool check_sfft_plan() {
    auto npass = [](int M, int G) { const int up = M - (M < G ? M : G); return (up + kSfTabL - 1) / kSfTabL; };
    uint4* x = (uint4*)0x1000;
    const uint64_t* words = (const uint64_t*)0x2000;
    for (int m = 0; m <= 32; ++m)
        for (int m_op = 0; m_op <= m; ++m_op)
            for (int inv = 0; inv < 2; ++inv) {
                if (inv && m_op != m) continue;
                const int M = inv ? m : m_op;
                std::vector<SfftPass> v = sfft_passes(x, words, m_op, m, inv != 0);
                if (!inv) std::reverse(v.begin(), v.end());
                const SfftPass& b = v[0];
                const int want_c = m <= kSfGroupSmallLog && npass(M, 2) == npass(M, 3) ? 2 : 3;
                bool ok = b.lo == 0 && b.c == want_c && b.L == (M < want_c ? M : want_c) && (int)v.size() == 1 + npass(M, b.c);
                int lo = b.L;
                for (size_t i = 1; i < v.size() && ok; ++i) {
                    const SfftPass& p = v[i];
                    ok = p.lo == lo && p.L >= 1 && p.L <= kSfTabL && p.c <= p.lo && p.L + p.c <= kSfTabPtsLog;
                    lo += p.L;
                }
                ok = ok && lo == M;
                for (const SfftPass& p : v) ok = ok && p.x == x && p.n == (1ull << m) && p.inverse == inv;
                const SfftPass& first = inv ? v.front() : v.back();
                ok = ok && (inv ? first.words == nullptr : first.words == words && first.wmask == (1ull << m_op) - 1);
                if (!ok) {
                    printf("SIMPLE PLAN WRONG: m %d, m_op %d, inverse %d\n", m, m_op, inv);
                    return false;
                }
            }
    return true;
}

bool check_simple_tables() {
    std::vector<gcm_u128> C;
    if (!build_cantor_table(C)) return false;
    CANTOR.resize(C.size());
    for (size_t i = 0; i < C.size(); ++i) CANTOR[i] = to_u4(C[i]);
    bool ok = C[0] == 1;
    for (int i = 1; i < kCantorBeta; ++i) ok &= (gcm_mul_host(C[i], C[i]) ^ C[i]) == C[i - 1] && !(C[i] & 1);
    // the table product against the shift-and-add product
    std::mt19937_64 g(7);
    std::vector<uint4> T(16), TL(16 * kSfLaneTabStride);
    for (int i = 0; i < 2000 && ok; ++i) {
        const gcm_u128 a = ((gcm_u128)g() << 64) | g(), b = ((gcm_u128)g() << 64) | g();
        gcm_build_tab(to_u4(a), T.data());
        gcm_build_tab<kSfLaneTabStride>(to_u4(a), TL.data());
        const uint4 r = gcm_mul_tab(T.data(), to_u4(b)), want = to_u4(gcm_mul_host(a, b));
        const uint4 rl = gcm_mul_tab_lane(TL.data(), to_u4(b));
        ok &= r.x == want.x && r.y == want.y && r.z == want.z && r.w == want.w;
        ok &= rl.x == want.x && rl.y == want.y && rl.z == want.z && rl.w == want.w;
    }
    if (!ok) printf("simple-variant tables or table product wrong\n");
    return ok;
}

bool check_simple_product(std::mt19937_64& g, uint64_t na, uint64_t nb) {
    const Sizes s = make_sizes(na, nb, 64);
    const Workspace w = workspace_for(s);
    std::vector<char> ws(w.bytes, 0x5a);
    auto a = rand_words(g, na), b = rand_words(g, nb);
    std::vector<uint64_t> c(s.out_words + 1, 0xdead), r(s.out_words + 1, 0);
    uint64_t* wa = (uint64_t*)(ws.data() + w.off_wa);
    uint64_t* wb = (uint64_t*)(ws.data() + w.off_wb);
    uint4* sa = (uint4*)(ws.data() + w.off_sa);
    uint4* sb = (uint4*)(ws.data() + w.off_sb);
    const uint64_t N = 1ull << s.m;
    std::vector<Op> ops;
    emit_pack(ops, a.data(), na, wa, 1ull << s.m_a);
    emit_bc(ops, POOL, wa, 0, s.m_a, 0, 1);
    emit_pack(ops, b.data(), nb, wb, 1ull << s.m_b);
    emit_bc(ops, POOL, wb, 0, s.m_b, 0, 1);
    run_ops(ops);
    run_sfft(sfft_passes(sa, wa, s.m_a, s.m, false));
    run_sfft(sfft_passes(sb, wb, s.m_b, s.m, false));
    std::vector<uint4> T(16 * kSfLaneTabStride);  // k_spmul's lane-interleaved table
    for (uint64_t j = 0; j < N; ++j) {
        gcm_build_tab<kSfLaneTabStride>(sa[j], T.data());
        sb[j] = gcm_mul_tab_lane(T.data(), sb[j]);
    }
    run_sfft(sfft_passes(sb, nullptr, s.m, s.m, true));
    ops.clear();
    emit_bc(ops, POOL, sb, 1, s.m, 1, 1);
    run_ops(ops);
    for (uint64_t k = 0; k < s.out_words; ++k) c[k] = sf_combine_word(sb, N, k, s.out_words, s.nc_bits);
    oracle_mul(a.data(), na, b.data(), nb, r.data(), 4);
    const bool ok = memcmp(c.data(), r.data(), 8 * s.out_words) == 0 && c[s.out_words] == 0xdead;
    if (!ok)
        printf("SIMPLE MISMATCH %llu x %llu bits (N = 2^%d)\n", (unsigned long long)na, (unsigned long long)nb, s.m);
    return ok;
}

// ---- the Frobenius-partition variant (App. C): z-adic passes, the word
// BasisCvt, encoding, the simple variant's passes at alpha = beta_{m+64},
// pointmul, and the inverse chain, run here with the kernels' bodies
std::vector<uint4> FROB;

void run_zadic(const std::vector<ZadicPass>& passes) {
    std::vector<uint64_t> lds(1 << kZTileLog);
    for (const ZadicPass& z : passes)
        for (uint64_t t = 0; t < zadic_tiles(z); ++t) zadic_tile(0, 1, t, z, lds.data());
}

bool init_frob() {
    if (CANTOR.empty() && !check_simple_tables()) return false;
    std::vector<gcm_u128> C, enc, dec;
    std::vector<uint64_t> wf, wi;
    if (!build_cantor_table(C) || !build_frob_tables(C.data(), enc, dec, wf, wi)) return false;
    FROB.assign(kFrobTabU4, make_uint4(0, 0, 0, 0));
    for (int i = 0; i < kElemTab; ++i) {
        FROB[kFrobEncOff + i] = to_u4((u128)enc[i]);
        FROB[kFrobDecOff + i] = to_u4((u128)dec[i]);
    }
    memcpy(FROB.data() + kFrobWordOff, wf.data(), 8 * kWordTab);
    memcpy((char*)(FROB.data() + kFrobWordOff) + 8 * kWordTab, wi.data(), 8 * kWordTab);
    return true;
}

void frob_forward_host(const uint64_t* src, uint64_t nbits, uint64_t* words, int W, uint4* spec, int m) {
    std::vector<Op> ops;
    emit_pack(ops, src, nbits, words, 1ull << W);
    run_ops(ops);
    run_zadic(zadic_passes(words, W, false));
    ops.clear();
    emit_bc(ops, POOL, words, 0, W, 0, 1);
    run_ops(ops);
    const FrobEncode F{words, spec, (uint32_t)W, (uint32_t)m};
    std::vector<uint64_t> lds(kFeStage);
    const uint64_t* wt = (const uint64_t*)(FROB.data() + kFrobWordOff);
    for (uint64_t t = 0; t < frob_tiles((uint32_t)m); ++t)
        frob_encode_tile(0, 1, t, F, FROB.data() + kFrobEncOff, wt, lds.data());
    run_sfft(sfft_passes(spec, nullptr, m, m, false, m + 64));
}

bool check_frob_product(std::mt19937_64& g, uint64_t na, uint64_t nb) {
    const FrobSizes s = frob_sizes(na, nb);
    const FrobWorkspace w = frob_workspace(s);
    std::vector<char> ws(w.bytes, 0x5a);
    auto a = rand_words(g, na), b = rand_words(g, nb);
    std::vector<uint64_t> c(s.out_words + 1, 0xdead), r(s.out_words + 1, 0);
    uint64_t* wa = (uint64_t*)(ws.data() + w.off_wa);
    uint64_t* wb = (uint64_t*)(ws.data() + w.off_wb);
    uint4* sa = (uint4*)(ws.data() + w.off_sa);
    uint4* sb = (uint4*)(ws.data() + w.off_sb);
    const uint64_t n = 1ull << s.m;
    frob_forward_host(a.data(), na, wa, s.w_a, sa, s.m);
    frob_forward_host(b.data(), nb, wb, s.w_b, sb, s.m);
    std::vector<uint4> T(16 * kSfLaneTabStride);  // k_spmul's lane-interleaved table
    for (uint64_t j = 0; j < n; ++j) {
        gcm_build_tab<kSfLaneTabStride>(sa[j], T.data());
        sb[j] = gcm_mul_tab_lane(T.data(), sb[j]);
    }
    run_sfft(sfft_passes(sb, nullptr, s.m, s.m, true, s.m + 64));
    uint64_t* words = (uint64_t*)sa;
    const FrobDecode F{sb, words, (uint32_t)s.m};
    std::vector<uint64_t> lds(kFeStage);
    const uint64_t* wt = (const uint64_t*)(FROB.data() + kFrobWordOff) + kWordTab;
    for (uint64_t t = 0; t < frob_tiles((uint32_t)s.m); ++t)
        frob_decode_tile(0, 1, t, F, FROB.data() + kFrobDecOff, wt, lds.data());
    std::vector<Op> ops;
    emit_bc(ops, POOL, words, 0, s.m + 1, 1, 1);
    run_ops(ops);
    run_zadic(zadic_passes(words, s.m + 1, true, c.data(), s.out_words));
    oracle_mul(a.data(), na, b.data(), nb, r.data(), 4);
    const bool ok = memcmp(c.data(), r.data(), 8 * s.out_words) == 0 && c[s.out_words] == 0xdead;
    if (!ok) {
        uint64_t k = 0;
        while (k < s.out_words && c[k] == r[k]) ++k;
        printf("FROBENIUS MISMATCH %llu x %llu bits (n = 2^%d), first bad word %llu of %llu\n",
               (unsigned long long)na, (unsigned long long)nb, s.m, (unsigned long long)k,
               (unsigned long long)s.out_words);
    }
    return ok;
}

// the z-adic expansion alone: recomposition inverts it, and the digits of a
// polynomial below x^64 (one word) are the polynomial itself
bool check_zadic(std::mt19937_64& g) {
    bool ok = true;
    for (int W = 0; W <= 17 && ok; ++W) {
        std::vector<uint64_t> x(1ull << W), y;
        for (auto& v : x) v = g();
        y = x;
        run_zadic(zadic_passes(y.data(), W, false));
        std::vector<uint64_t> z(1ull << W, 0);
        run_zadic(zadic_passes(y.data(), W, true, z.data(), z.size()));
        ok &= z == x;
        std::vector<uint64_t> one(1ull << W, 0);
        one[0] = x[0];
        run_zadic(zadic_passes(one.data(), W, false));
        ok &= one[0] == x[0];
        for (size_t k = 1; k < one.size(); ++k) ok &= one[k] == 0;
        if (!ok) printf("z-adic round trip or single-word digits wrong at W = %d\n", W);
    }
    return ok;
}

}  // namespace

int main(int argc, char** argv) {
    if (!init()) {
        printf("table construction failed\n");
        return 2;
    }
    const std::string what = argc > 1 ? argv[1] : "all";
    int bad = 0;
    std::mt19937_64 g(20261202);
    if (what == "all" || what == "products") {
        const uint64_t fixed[][2] = {{1, 1},         {64, 64},           {65, 64},           {1, 700},
                                     {1000, 999},    {64 * 33, 64 * 31}, {5000, 70},         {1 << 16, 1 << 16},
                                     {100000, 3},    {64 * 5000 + 7, 64 * 3000 + 1},        {1 << 20, 1 << 20},
                                     {1 << 21, 1 << 19}};
        for (auto& p : fixed) bad += !check_product(g, p[0], p[1]);
        for (int i = 0; i < 60; ++i) bad += !check_product(g, 1 + g() % (1ull << (1 + g() % 18)), 1 + g() % (1ull << (1 + g() % 18)));
        // the small BasisCvt tiles of single products
        PP.bc_small = 1;
        for (auto& p : fixed) bad += !check_product(g, p[0], p[1]);
        PP.bc_small = 0;
        // 2^17 and 2^18 points: the bottom layers' multipliers have 17 and 18
        // bits (TGF(2^32) with a high half in GF(256))
        bad += !check_product(g, 1 << 22, 1 << 22);
        bad += !check_product(g, (1 << 23) - 77, (1 << 22) + 5);
    }
    if (what == "all" || what == "fusion") {
        // BasisCvt sub-conversions inside FFT passes at every size (the default
        // fuses transforms of at most 2^11 points only): every mask, products
        // of one and several passes (single-product and batch tiles), the
        // 128-bit words, a batch
        PP.fuse_max_log = 32;
        const uint64_t fixed[][2] = {{1, 1},     {65, 64},      {1000, 999},  {64 * 33, 64 * 31}, {1 << 16, 1 << 16},
                                     {100000, 3}, {1 << 20, 1 << 20}, {1 << 21, 1 << 19}, {1 << 22, (1 << 22) - 3}};
        for (int mask = 1; mask <= 7; ++mask) {
            PP.fuse_bc = mask;
            for (int small = 0; small < 2; ++small) {
                PP.bc_small = small;
                for (auto& p : fixed) bad += !check_product(g, p[0], p[1]);
                for (int i = 0; i < 8; ++i)
                    bad += !check_product(g, 1 + g() % (1ull << (1 + g() % 18)), 1 + g() % (1ull << (1 + g() % 18)));
            }
            PP.bc_small = 0;
            PP.word_bits = 128;
            for (int i = 0; i < 4; ++i)
                bad += !check_product(g, 1 + g() % (1ull << (1 + g() % 18)), 1 + g() % (1ull << (1 + g() % 18)));
            PP.word_bits = 64;
            bad += !check_batch(g, 12);
        }
        PP.fuse_bc = 7;  // the default
        PP.fuse_max_log = 11;
    }
    if (what == "all" || what == "batch") bad += !check_batch(g, 60);
    if (what == "all" || what == "trunc") {
        PP.trunc_min_log = 1;
        for (int i = 0; i < 300; ++i) {
            PP.trunc_levels = i % 9;
            PP.trunc_max_terms = (i / 9) % 4;  // any count, 1, 2, 3 terms
            bad += !check_product(g, 1 + g() % (1ull << (1 + g() % 17)), 1 + g() % (1ull << (1 + g() % 17)));
        }
        PP.trunc_levels = 3;
        PP.trunc_max_terms = 0;
        bad += !check_batch(g, 40);
        PP.trunc_max_terms = 2;
        PP.trunc_min_log = 23;
    }
    if (what == "all" || what == "w128") {
        // Split into 128-bit words, products over TGF(2^256)
        PP.word_bits = 128;
        const uint64_t fixed[][2] = {{1, 1},     {128, 128}, {129, 128}, {64, 64},      {1, 700},
                                     {1000, 999}, {128 * 33, 128 * 31},  {5000, 70},   {1 << 16, 1 << 16},
                                     {100000, 3}, {1 << 20, 1 << 20},    {1 << 21, 1 << 19}};
        for (auto& p : fixed) bad += !check_product(g, p[0], p[1]);
        for (int i = 0; i < 40; ++i) bad += !check_product(g, 1 + g() % (1ull << (1 + g() % 18)), 1 + g() % (1ull << (1 + g() % 18)));
        bad += !check_batch(g, 30);
        PP.word_bits = 64;
    }
    if (what == "all" || what == "simple") {
        bad += !check_sfft_plan();
        // Alg. 4: bottom pass only (N <= 8), one and several strided passes
        // above it, operands far shorter than N, single words
        bad += !check_simple_tables();
        const uint64_t fixed[][2] = {{1, 1},      {64, 64},     {65, 64},         {1, 700},     {1000, 999},
                                     {5000, 70},  {64, 1 << 16}, {1 << 16, 1 << 16}, {100000, 3}, {1 << 19, 1 << 18},
                                     {64 * 4096 + 1, 64 * 4095}, {1 << 20, 1 << 20}, {1 << 22, 1 << 22},
                                     {(1 << 23) - 5, 1000}};
        for (auto& p : fixed) bad += !check_simple_product(g, p[0], p[1]);
        for (int i = 0; i < 30; ++i)
            bad += !check_simple_product(g, 1 + g() % (1ull << (1 + g() % 18)), 1 + g() % (1ull << (1 + g() % 18)));
    }
    if (what == "all" || what == "frobenius") {
        if (!init_frob()) {
            printf("Frobenius tables failed\n");
            return 2;
        }
        bad += !check_zadic(g);
        // n = 1 .. 2^13 points: the small-encoding path (n < 64), one and
        // several encoding tiles, one and several z-adic passes
        const uint64_t fixed[][2] = {{1, 1},       {64, 64},        {65, 64},       {1, 700},         {128, 1},
                                     {129, 1},     {100, 29},       {1000, 999},    {5000, 70},       {4096, 4097},
                                     {1 << 13, 1 << 13}, {(1 << 13) + 1, 1 << 13}, {64, 1 << 16}, {1 << 16, 1 << 16},
                                     {100000, 3},  {1 << 19, 1 << 18}, {(1 << 19) + 77, (1 << 19) - 5},
                                     {1 << 20, 1 << 20}};
        for (auto& p : fixed) bad += !check_frob_product(g, p[0], p[1]);
        for (int i = 0; i < 30; ++i)
            bad += !check_frob_product(g, 1 + g() % (1ull << (1 + g() % 18)), 1 + g() % (1ull << (1 + g() % 18)));
    }
    if (what == "all" || what == "xcd") bad += !check_xcd_order(g);
    if (what == "all" || what == "basiscvt") {
        // 22 and 23: the strided pass of 2^6 / 2^7-row columns above the
        // top class pass, as in products of 2^28-bit operands
        for (int small = 0; small < 2; ++small) {
            for (int m : {0, 1, 2, 5, 12, 13, 14, 16, 17, 20, 22}) bad += !check_basiscvt<uint64_t>(m, small);
            for (int m : {11, 12, 13, 16, 19, 23}) bad += !check_basiscvt<uint4>(m, small);
        }
        // every size on the tiles of single products (the smallest tiles up to
        // 2^kBcTinyMaxLog elements, then the 32 KiB ones)
        for (int m = 0; m <= kBcTinyMaxLog + 1; ++m) {
            bad += !check_basiscvt<uint64_t>(m, 1);
            bad += !check_basiscvt<uint4>(m, 1);
        }
        // layers too tall for any class tile (as for 2^29 words on 32 KiB
        // tiles) on small stand-in tiles
        bad += !check_basiscvt_cap<uint64_t>(16, 8);
        bad += !check_basiscvt_cap<uint4>(17, 8);
        bad += !check_basiscvt_cap<uint64_t>(16, 7);
    }
    printf(bad ? "host exec: %d failures\n" : "host exec ok\n", bad);
    return bad ? 1 : 0;
}
