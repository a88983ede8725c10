// Host-side tower-field arithmetic and the constant tables the kernels use.
//
// Tower field (Sec. 3.2 of Chen, Cheng, Kuo, Li, Yang, arXiv:1708.09746):
//   TGF(2^2) = GF(2)[x1]/(x1^2 + x1 + 1),
//   TGF(2^{2^k}) = TGF(2^{2^{k-1}})[xk]/(xk^2 + xk + x1 x2 ... x_{k-1}).
// Bit j of an element is the coefficient of the basis element v_j, the product
// of the generators x_{t+1} over the set bits t of j (Def. of (v_k)).  An element
// of TGF(2^W) is a0 + a1 X with X the top generator, a0 in the low W/2 bits and
// a1 in the high W/2 bits; X^2 = X + c_W where c_W (the product of all lower
// generators) is the half-field element with only bit W/2 - 1 set.
//
// Multiplication is the Karatsuba form of the defining relation:
//   t = a1 b1,  lo = a0 b0 + c_W t,  hi = (a0 + a1)(b0 + b1) + a0 b0.
#pragma once
#include <array>
#include <cstdint>
#include <cstring>
#include <vector>

namespace gf2x {

using u128 = unsigned __int128;

struct HostTower {
    uint8_t mt8[256][256];  // full GF(256) product table

    HostTower() {
        // GF(16) by the bit-level recursion, then GF(256) on top of it
        uint8_t m4[16][16];
        for (int a = 0; a < 16; ++a)
            for (int b = 0; b < 16; ++b) m4[a][b] = (uint8_t)rec(a, b, 4);
        for (int a = 0; a < 256; ++a)
            for (int b = 0; b < 256; ++b) {
                int a0 = a & 15, a1 = a >> 4, b0 = b & 15, b1 = b >> 4;
                int t = m4[a1][b1];
                int p0 = m4[a0][b0];
                int lo = p0 ^ m4[0x8][t];  // c_8 = x1 x2 = bit 3 of GF(16)
                int hi = m4[a0 ^ a1][b0 ^ b1] ^ p0;
                mt8[a][b] = (uint8_t)(lo | (hi << 4));
            }
    }

    // bit-level recursion for widths <= 4 (only used to seed the tables)
    static uint32_t rec(uint32_t a, uint32_t b, int w) {
        if (w == 1) return a & b & 1u;
        int h = w / 2;
        uint32_t m = (1u << h) - 1;
        uint32_t a0 = a & m, a1 = a >> h, b0 = b & m, b1 = b >> h;
        uint32_t t = rec(a1, b1, h);
        uint32_t p0 = rec(a0, b0, h);
        uint32_t lo = p0 ^ rec(1u << (h - 1), t, h);
        uint32_t hi = rec(a0 ^ a1, b0 ^ b1, h) ^ p0;
        return lo | (hi << h);
    }

    uint64_t mul(uint64_t a, uint64_t b, int w) const {
        if (w == 8) return mt8[a & 255][b & 255];
        if (w < 8) return rec((uint32_t)a, (uint32_t)b, w);
        int h = w / 2;
        uint64_t m = (h == 64) ? ~0ull : ((1ull << h) - 1);
        uint64_t a0 = a & m, a1 = a >> h, b0 = b & m, b1 = b >> h;
        uint64_t t = mul(a1, b1, h);
        uint64_t p0 = mul(a0, b0, h);
        uint64_t lo = p0 ^ mul(1ull << (h - 1), t, h);
        uint64_t hi = mul(a0 ^ a1, b0 ^ b1, h) ^ p0;
        return lo | (hi << h);
    }

    u128 mul128(u128 a, u128 b) const {
        uint64_t a0 = (uint64_t)a, a1 = (uint64_t)(a >> 64);
        uint64_t b0 = (uint64_t)b, b1 = (uint64_t)(b >> 64);
        uint64_t t = mul(a1, b1, 64);
        uint64_t p0 = mul(a0, b0, 64);
        uint64_t lo = p0 ^ mul(1ull << 63, t, 64);
        uint64_t hi = mul(a0 ^ a1, b0 ^ b1, 64) ^ p0;
        return (u128)lo | ((u128)hi << 64);
    }

    // s_i(x) = sum over subsets j of the bits of i of x^(2^j) (Tab. 1 pattern;
    // equivalently s_i = s_1 applied i times).  Evaluated by iterating s_1.
    uint64_t s_eval(int i, uint64_t x, int w) const {
        for (int r = 0; r < i; ++r) x = mul(x, x, w) ^ x;
        return x;
    }
};

// Butterfly multiplier basis: lambda[i][t] = s_i(v_t) for i, t < 32.  The
// multiplier of the layer-i block starting at index s is s_i(s̄), and since s_i
// is GF(2)-linear it is the XOR of lambda[i][t] over the set bits t of s
// (bits t <= i of a block start are zero, and s_i(v_t) = 0 for t < i).
inline void build_lambda(const HostTower& T, uint32_t lam[32][32]) {
    for (int i = 0; i < 32; ++i)
        for (int t = 0; t < 32; ++t) lam[i][t] = (uint32_t)T.s_eval(i, 1ull << t, 32);
}

// Constant multiples for the generic product (kConstTabWords words): the
// multiples by c64 = x1 ... x5 (bit 31) of the bytes of a TGF(2^32) element,
// T64[k][y] = c64 (y << 8k) (k < 4), then by c32 = x1 ... x4 (bit 15) of the
// bytes of a TGF(2^16) element, T32[k][y] = c32 (y << 8k) (k < 2) as packed
// halfwords, then the register tables of multiplication by c16 in GF(256).
inline std::vector<uint32_t> build_const_tabs(const HostTower& T) {
    std::vector<uint32_t> t(4 * 256 + 256 + 8, 0);
    for (int k = 0; k < 4; ++k)
        for (int y = 0; y < 256; ++y) t[256 * k + y] = (uint32_t)T.mul((uint64_t)y << (8 * k), 1ull << 31, 32);
    uint16_t* h = (uint16_t*)(t.data() + 1024);
    for (int k = 0; k < 2; ++k)
        for (int y = 0; y < 256; ++y) h[256 * k + y] = (uint16_t)T.mul((uint64_t)y << (8 * k), 1ull << 15, 16);
    // c16 = 0x80 times the 3-bit groups of a byte: T0[y] = c16 y, T1[y] = c16 (y << 3)
    // (y < 8, one byte each, two words per table), T2[y] = c16 (y << 6) (y < 4)
    const uint8_t* r = T.mt8[0x80];
    uint32_t* g = t.data() + 1280;
    for (int y = 0; y < 8; ++y) {
        g[y >> 2] |= (uint32_t)r[y] << (8 * (y & 3));
        g[2 + (y >> 2)] |= (uint32_t)r[y << 3] << (8 * (y & 3));
    }
    for (int y = 0; y < 4; ++y) g[4] |= (uint32_t)r[y << 6] << (8 * y);
    return t;
}

// Kronecker embedding (Sec. 2.1) and its inverse (Sec. 4.3): a 64-bit block u
// (a polynomial of degree < 64 in z) maps to u(theta) in TGF(2^128) with
// theta = x7 = v_64, which generates TGF(2^128) since it lies outside
// TGF(2^64).  Products of two images are images of the carry-less product
// (degree < 127 < 128), so the inverse map recovers 127-bit partial products.
//
// w = 128: a 128-bit block maps into TGF(2^256) = TGF(2^128)[x8]/(x8^2 + x8 +
// c256), c256 = x1 ... x7 (bit 127), at theta = x8, which lies outside
// TGF(2^128) and so generates TGF(2^256); elements are (lo, hi) halves.
struct ReprTables {
    // M4R-8 tables: phi[k][b] = image of byte b placed at byte k (k < 8),
    // psi[k][b] = preimage of byte b placed at byte k of the element (k < 16)
    std::vector<u128> phi;  // 8 * 256
    std::vector<u128> psi;  // 16 * 256
    u128 theta_pow[128];
    u128 psi_col[128];  // psi of the basis element v_j, as a 128-bit polynomial
    // M4R-4 tables.  phin: w = 64, phin[16 k + v] = Phi(v << 4k) (k < 16),
    // then w = 128, the low halves of Phi(v << 4k) (k < 32) at 256 + 16 k + v
    // and the high halves at 768 + 16 k + v.  psin: w = 128, the low halves
    // of Psi(v << 4k) (k < 64: nibble k of the element (lo, hi)) at 16 k + v,
    // the high halves at 1024 + 16 k + v.
    std::vector<u128> phin;  // 256 + 2 * 512
    std::vector<u128> psin;  // 2 * 1024
    bool ok = false;
};

// TGF(2^256) element as (lo, hi)
struct U256 {
    u128 lo, hi;
};
inline bool bit256(const U256& v, int b) { return b < 128 ? (v.lo >> b) & 1 : (v.hi >> (b - 128)) & 1; }
inline void xor256(U256& a, const U256& b) {
    a.lo ^= b.lo;
    a.hi ^= b.hi;
}

// w = 128 tables (see ReprTables); false if the powers of theta were dependent
inline bool build_repr256(const HostTower& T, ReprTables& R) {
    const u128 c256 = (u128)1 << 127;
    std::vector<U256> pw(256);
    pw[0] = U256{1, 0};
    for (int j = 1; j < 256; ++j) {
        // (lo + hi x8) x8 = hi c256 + (lo + hi) x8
        const U256& p = pw[j - 1];
        pw[j] = U256{T.mul128(p.hi, c256), p.lo ^ p.hi};
    }
    // invert the matrix with columns theta^j (Gauss-Jordan, fully reduced)
    std::vector<U256> val, comb;
    std::vector<int> piv;
    for (int j = 0; j < 256; ++j) {
        U256 v = pw[j], c{0, 0};
        if (j < 128) c.lo = (u128)1 << j; else c.hi = (u128)1 << (j - 128);
        for (size_t r = 0; r < piv.size(); ++r)
            if (bit256(v, piv[r])) { xor256(v, val[r]); xor256(c, comb[r]); }
        int pb = 255;
        while (pb >= 0 && !bit256(v, pb)) --pb;
        if (pb < 0) return false;
        for (size_t r = 0; r < piv.size(); ++r)
            if (bit256(val[r], pb)) { xor256(val[r], v); xor256(comb[r], c); }
        val.push_back(v);
        comb.push_back(c);
        piv.push_back(pb);
    }
    std::vector<U256> psi_col(256);
    for (int r = 0; r < 256; ++r) psi_col[piv[r]] = comb[r];
    R.phin.resize(256 + 2 * 512, 0);
    for (int k = 0; k < 16; ++k)
        for (int v = 0; v < 16; ++v) {
            u128 acc = 0;
            for (int t = 0; t < 4; ++t)
                if ((v >> t) & 1) acc ^= R.theta_pow[4 * k + t];
            R.phin[16 * k + v] = acc;
        }
    for (int k = 0; k < 32; ++k)
        for (int v = 0; v < 16; ++v) {
            U256 acc{0, 0};
            for (int t = 0; t < 4; ++t)
                if ((v >> t) & 1) xor256(acc, pw[4 * k + t]);
            R.phin[256 + 16 * k + v] = acc.lo;
            R.phin[768 + 16 * k + v] = acc.hi;
        }
    R.psin.assign(2 * 1024, 0);
    for (int k = 0; k < 64; ++k)
        for (int v = 0; v < 16; ++v) {
            U256 acc{0, 0};
            for (int t = 0; t < 4; ++t)
                if ((v >> t) & 1) xor256(acc, psi_col[4 * k + t]);
            R.psin[16 * k + v] = acc.lo;
            R.psin[1024 + 16 * k + v] = acc.hi;
        }
    return true;
}

inline ReprTables build_repr(const HostTower& T) {
    ReprTables R;
    u128 theta = (u128)1 << 64;
    R.theta_pow[0] = 1;
    for (int j = 1; j < 128; ++j) R.theta_pow[j] = T.mul128(R.theta_pow[j - 1], theta);
    // invert the matrix with columns theta^j: Gauss-Jordan on an augmented copy
    u128 rows_val[128], rows_comb[128];
    int npiv = 0;
    int pivbit[128];
    for (int j = 0; j < 128; ++j) {
        u128 v = R.theta_pow[j], comb = (u128)1 << j;
        for (int r = 0; r < npiv; ++r)
            if ((v >> pivbit[r]) & 1) { v ^= rows_val[r]; comb ^= rows_comb[r]; }
        if (v == 0) return R;  // dependent: not a generator
        int pb = 127;
        while (!((v >> pb) & 1)) --pb;
        for (int r = 0; r < npiv; ++r)
            if ((rows_val[r] >> pb) & 1) { rows_val[r] ^= v; rows_comb[r] ^= comb; }
        rows_val[npiv] = v; rows_comb[npiv] = comb; pivbit[npiv] = pb; ++npiv;
    }
    // fully reduced: each row has exactly its pivot bit set
    for (int r = 0; r < 128; ++r) R.psi_col[pivbit[r]] = rows_comb[r];
    R.phi.assign(8 * 256, 0);
    for (int k = 0; k < 8; ++k)
        for (int b = 0; b < 256; ++b) {
            u128 acc = 0;
            for (int t = 0; t < 8; ++t)
                if ((b >> t) & 1) acc ^= R.theta_pow[8 * k + t];
            R.phi[k * 256 + b] = acc;
        }
    R.psi.assign(16 * 256, 0);
    for (int k = 0; k < 16; ++k)
        for (int b = 0; b < 256; ++b) {
            u128 acc = 0;
            for (int t = 0; t < 8; ++t)
                if ((b >> t) & 1) acc ^= R.psi_col[8 * k + t];
            R.psi[k * 256 + b] = acc;
        }
    R.ok = build_repr256(T, R);
    return R;
}

}  // namespace gf2x
