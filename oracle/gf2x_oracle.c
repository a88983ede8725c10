/*
 * gf2x_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU multiplier for binary polynomials.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library; the GPU product path never calls it.
 *
 * What it computes (the problem statement of the paper, Sec. 2.1 "Multiplying
 * with Segmentation of Binary Polynomials", and the output line of Alg. 5):
 *     c(x) = a(x) * b(x) in GF(2)[x],   c_k = XOR_{i+j=k} a_i AND b_j.
 * The method of the paper reaches exactly this product, so the oracle is that
 * definition written out on 64-bit words, with no FFT and no field tower.
 *
 * Bit layout (shared convention with the library's C ABI, not shared code):
 * bit i of a polynomial is bit (i mod 64) of word floor(i / 64).  An operand
 * of n bits occupies ceil(n/64) words; bits >= n in the last word are ignored.
 * The product of an na-bit and an nb-bit operand has na+nb-1 coefficients and
 * is written as ceil((na+nb-1)/64) words, high bits zero.
 *
 * Pieces (each written from the definition, nothing shared with the GPU path):
 *   clmul64_bitloop   -- 64x64 -> 128 carry-less product, one bit at a time.
 *   clmul64_window    -- the same product with a 4-bit window table; tested
 *                        against the bit loop.
 *   schoolbook        -- word-level convolution with clmul64_window.
 *   karatsuba         -- (A0 + A1 X)(B0 + B1 X) = P0 + (P1 - P0 - P2) X + P2 X^2
 *                        over GF(2) (minus is XOR), with P1 = (A0+A1)(B0+B1);
 *                        falls back to schoolbook below a small threshold.
 *   oracle_mul        -- masks, splits unbalanced operands into chunks, and
 *                        fans the top Karatsuba levels out to POSIX threads.
 *   oracle_word       -- one output word, straight from the convolution sum
 *                        (for sampled checks at sizes where a full product
 *                        would take too long).
 *   oracle_mod        -- p(x) mod (x^64 + q(x)), for a randomized identity
 *                        check (a mod Q)(b mod Q) = c mod Q.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- clmul */

void oracle_clmul64_bitloop(uint64_t x, uint64_t y, uint64_t out[2])
{
    uint64_t lo = 0, hi = 0;
    for (int i = 0; i < 64; ++i) {
        if ((y >> i) & 1u) {
            lo ^= x << i;
            if (i) hi ^= x >> (64 - i);
        }
    }
    out[0] = lo;
    out[1] = hi;
}

static inline void clmul64_window(uint64_t x, uint64_t y, uint64_t *lo_out, uint64_t *hi_out)
{
    /* table[t] = x * t for the 16 polynomials t of degree < 4, as 67-bit values */
    uint64_t tlo[16], thi[16];
    tlo[0] = 0; thi[0] = 0;
    tlo[1] = x; thi[1] = 0;
    for (int t = 2; t < 16; t += 2) {
        tlo[t] = tlo[t >> 1] << 1;
        thi[t] = (thi[t >> 1] << 1) | (tlo[t >> 1] >> 63);
        tlo[t + 1] = tlo[t] ^ x;
        thi[t + 1] = thi[t];
    }
    uint64_t lo = 0, hi = 0;
    for (int i = 60; i >= 0; i -= 4) {
        /* shift the accumulator left by 4, then add the window product */
        hi = (hi << 4) | (lo >> 60);
        lo <<= 4;
        unsigned nib = (unsigned)(y >> i) & 15u;
        lo ^= tlo[nib];
        hi ^= thi[nib];
    }
    *lo_out = lo;
    *hi_out = hi;
}

void oracle_clmul64_window(uint64_t x, uint64_t y, uint64_t out[2])
{
    clmul64_window(x, y, &out[0], &out[1]);
}

/* ------------------------------------------------------------ schoolbook */

/* c[0 .. na+nb) ^= a * b  (c must already hold what is to be added to) */
static void schoolbook_acc(const uint64_t *a, size_t na, const uint64_t *b, size_t nb, uint64_t *c)
{
    for (size_t i = 0; i < na; ++i) {
        uint64_t ai = a[i];
        if (!ai) continue;
        for (size_t j = 0; j < nb; ++j) {
            uint64_t lo, hi;
            clmul64_window(ai, b[j], &lo, &hi);
            c[i + j] ^= lo;
            c[i + j + 1] ^= hi;
        }
    }
}

void oracle_mul_schoolbook(const uint64_t *a, size_t na, const uint64_t *b, size_t nb, uint64_t *c)
{
    memset(c, 0, (na + nb) * sizeof(uint64_t));
    schoolbook_acc(a, na, b, nb, c);
}

/* ------------------------------------------------------------- karatsuba */

#define KARA_THRESHOLD 12

/* c[0 .. 2n) = a[0..n) * b[0..n); tmp must hold kara_tmp_words(n) words */
static size_t kara_tmp_words(size_t n)
{
    if (n <= KARA_THRESHOLD) return 0;
    size_t h = (n + 1) / 2;
    /* sa (h) + sb (h) + P1 (2h) + recursion tmp for size h */
    return 4 * h + kara_tmp_words(h);
}

static void kara(const uint64_t *a, const uint64_t *b, size_t n, uint64_t *c, uint64_t *tmp)
{
    if (n <= KARA_THRESHOLD) {
        memset(c, 0, 2 * n * sizeof(uint64_t));
        schoolbook_acc(a, n, b, n, c);
        return;
    }
    size_t h = (n + 1) / 2; /* low half length */
    size_t l = n - h;       /* high half length, l <= h */
    uint64_t *sa = tmp, *sb = tmp + h, *p1 = tmp + 2 * h, *rest = tmp + 4 * h;

    /* P0 = A0 B0 -> c[0, 2h);  P2 = A1 B1 -> c[2h, 2h + 2l) */
    kara(a, b, h, c, rest);
    if (l == h) {
        kara(a + h, b + h, l, c + 2 * h, rest);
    } else {
        /* odd n: pad the high halves to h words */
        memcpy(sa, a + h, l * sizeof(uint64_t));
        memset(sa + l, 0, (h - l) * sizeof(uint64_t));
        memcpy(sb, b + h, l * sizeof(uint64_t));
        memset(sb + l, 0, (h - l) * sizeof(uint64_t));
        kara(sa, sb, h, p1, rest);
        memcpy(c + 2 * h, p1, 2 * l * sizeof(uint64_t)); /* top 2(h-l) words are zero */
    }
    /* P1 = (A0 + A1)(B0 + B1) */
    for (size_t i = 0; i < h; ++i) {
        sa[i] = a[i] ^ (i < l ? a[h + i] : 0);
        sb[i] = b[i] ^ (i < l ? b[h + i] : 0);
    }
    kara(sa, sb, h, p1, rest);
    /* middle term P1 + P0 + P2, added at X^h */
    for (size_t i = 0; i < 2 * h; ++i) {
        uint64_t p0 = c[i];
        uint64_t p2 = (i < 2 * l) ? c[2 * h + i] : 0;
        p1[i] ^= p0 ^ p2;
    }
    for (size_t i = 0; i < 2 * h; ++i) c[h + i] ^= p1[i];
}

/* Threaded top levels: each of the three sub-products runs in its own thread
 * down to `depth` levels, giving up to 3^depth concurrent leaves. */
struct kara_task {
    const uint64_t *a, *b;
    size_t n;
    uint64_t *c;
    int depth;
    int err;
};

static void kara_par(const uint64_t *a, const uint64_t *b, size_t n, uint64_t *c, int depth, int *err);

static void *kara_thread(void *p)
{
    struct kara_task *t = (struct kara_task *)p;
    kara_par(t->a, t->b, t->n, t->c, t->depth, &t->err);
    return NULL;
}

static void kara_par(const uint64_t *a, const uint64_t *b, size_t n, uint64_t *c, int depth, int *err)
{
    if (depth <= 0 || n <= 4 * KARA_THRESHOLD) {
        uint64_t *tmp = (uint64_t *)malloc((kara_tmp_words(n) + 1) * sizeof(uint64_t));
        if (!tmp) { *err = 1; return; }
        kara(a, b, n, c, tmp);
        free(tmp);
        return;
    }
    size_t h = (n + 1) / 2, l = n - h;
    uint64_t *buf = (uint64_t *)calloc(8 * h, sizeof(uint64_t));
    if (!buf) { *err = 1; return; }
    uint64_t *ah = buf, *bh = buf + h, *sa = buf + 2 * h, *sb = buf + 3 * h, *p1 = buf + 4 * h, *p2 = buf + 6 * h;
    memcpy(ah, a + h, l * sizeof(uint64_t));
    memcpy(bh, b + h, l * sizeof(uint64_t));
    for (size_t i = 0; i < h; ++i) { sa[i] = a[i] ^ ah[i]; sb[i] = b[i] ^ bh[i]; }

    struct kara_task t[3] = {
        {a, b, h, c, depth - 1, 0},
        {ah, bh, h, p2, depth - 1, 0},
        {sa, sb, h, p1, depth - 1, 0},
    };
    pthread_t th[3];
    int started[3] = {0, 0, 0};
    for (int i = 0; i < 3; ++i)
        started[i] = pthread_create(&th[i], NULL, kara_thread, &t[i]) == 0;
    for (int i = 0; i < 3; ++i) {
        if (started[i]) pthread_join(th[i], NULL);
        else kara_thread(&t[i]);
        if (t[i].err) *err = 1;
    }
    memcpy(c + 2 * h, p2, 2 * l * sizeof(uint64_t));
    for (size_t i = 0; i < 2 * h; ++i) p1[i] ^= c[i] ^ (i < 2 * l ? p2[i] : 0);
    for (size_t i = 0; i < 2 * h; ++i) c[h + i] ^= p1[i];
    free(buf);
}

/* ------------------------------------------------------------ public API */

size_t oracle_out_words(size_t na_bits, size_t nb_bits)
{
    if (na_bits == 0 || nb_bits == 0) return 0;
    return (na_bits + nb_bits - 1 + 63) / 64;
}

/* copy an operand into a fresh zero-padded buffer, masking bits >= nbits */
static uint64_t *load_masked(const uint64_t *a, size_t nbits, size_t nwords_alloc)
{
    size_t nw = (nbits + 63) / 64;
    uint64_t *r = (uint64_t *)calloc(nwords_alloc ? nwords_alloc : 1, sizeof(uint64_t));
    if (!r) return NULL;
    memcpy(r, a, nw * sizeof(uint64_t));
    if (nbits % 64) r[nw - 1] &= (~(uint64_t)0) >> (64 - nbits % 64);
    return r;
}

/*
 * c = a * b.  c receives oracle_out_words(na_bits, nb_bits) words.
 * threads <= 1 runs single-threaded; otherwise the top Karatsuba levels fan
 * out so that roughly `threads` leaves run at once.
 * Returns 0 on success, -1 on bad arguments, -3 on allocation failure.
 */
int oracle_mul(const uint64_t *a, size_t na_bits, const uint64_t *b, size_t nb_bits, uint64_t *c, int threads)
{
    size_t ow = oracle_out_words(na_bits, nb_bits);
    if (ow == 0) return 0;
    if (!a || !b || !c) return -1;
    size_t na = (na_bits + 63) / 64, nb = (nb_bits + 63) / 64;
    /* make a the longer operand */
    if (nb > na) {
        const uint64_t *tp = a; a = b; b = tp;
        size_t ts = na; na = nb; nb = ts;
        ts = na_bits; na_bits = nb_bits; nb_bits = ts;
    }
    size_t chunks = (na + nb - 1) / nb;
    uint64_t *A = load_masked(a, na_bits, chunks * nb);
    uint64_t *B = load_masked(b, nb_bits, nb);
    uint64_t *C = (uint64_t *)calloc(chunks * nb + nb + 1, sizeof(uint64_t));
    uint64_t *P = (uint64_t *)calloc(2 * nb, sizeof(uint64_t));
    if (!A || !B || !C || !P) { free(A); free(B); free(C); free(P); return -3; }

    int depth = 0;
    for (int t = 1; t < threads; t *= 3) depth++;
    int err = 0;
    for (size_t k = 0; k < chunks && !err; ++k) {
        kara_par(A + k * nb, B, nb, P, depth, &err);
        for (size_t i = 0; i < 2 * nb; ++i) C[k * nb + i] ^= P[i];
    }
    if (!err) {
        memcpy(c, C, ow * sizeof(uint64_t));
        size_t top = (na_bits + nb_bits - 1) % 64;
        if (top) c[ow - 1] &= (~(uint64_t)0) >> (64 - top);
    }
    free(A); free(B); free(C); free(P);
    return err ? -3 : 0;
}

/* Word k of a*b computed straight from the convolution sum:
 * bits [64k, 64k+64) collect lo(a_i b_j) for i+j = k and hi(a_i b_j) for
 * i+j = k-1.  Costs O(min(na, nb)) carry-less products. */
uint64_t oracle_word(const uint64_t *a, size_t na_bits, const uint64_t *b, size_t nb_bits, size_t k)
{
    size_t na = (na_bits + 63) / 64, nb = (nb_bits + 63) / 64;
    uint64_t mask_a = (na_bits % 64) ? ((~(uint64_t)0) >> (64 - na_bits % 64)) : ~(uint64_t)0;
    uint64_t mask_b = (nb_bits % 64) ? ((~(uint64_t)0) >> (64 - nb_bits % 64)) : ~(uint64_t)0;
    uint64_t r = 0;
    for (int part = 0; part < 2; ++part) {
        /* part 0: i + j = k (low words), part 1: i + j = k - 1 (high words) */
        if (part == 1 && k == 0) break;
        size_t s = k - (size_t)part;
        size_t ilo = (s >= nb) ? s - (nb - 1) : 0;
        size_t ihi = (s < na) ? s : na - 1;
        for (size_t i = ilo; i <= ihi && i < na; ++i) {
            size_t j = s - i;
            uint64_t ai = a[i], bj = b[j];
            if (i == na - 1) ai &= mask_a;
            if (j == nb - 1) bj &= mask_b;
            uint64_t lo, hi;
            clmul64_window(ai, bj, &lo, &hi);
            r ^= part ? hi : lo;
        }
    }
    size_t nbits = na_bits + nb_bits - 1;
    if (64 * k >= nbits) return 0;
    if (64 * (k + 1) > nbits) r &= (~(uint64_t)0) >> (64 - nbits % 64);
    return r;
}

/* p(x) mod Q(x), Q(x) = x^64 + q(x) with deg q < 64; p has nbits bits.
 * Horner over the words from the top: acc <- acc * x^64 + p_k (mod Q). */
static uint64_t mod_q_128(uint64_t lo, uint64_t hi, uint64_t q)
{
    /* reduce hi * x^64 + lo: x^64 == q, so hi*x^64 == hi*q, which is again
     * up to 127 bits; every fold lowers deg(hi) by 64 - deg(q) >= 1. */
    while (hi) {
        uint64_t plo, phi;
        clmul64_window(hi, q, &plo, &phi);
        lo ^= plo;
        hi = phi;
    }
    return lo;
}

uint64_t oracle_mod(const uint64_t *p, size_t nbits, uint64_t q)
{
    size_t nw = (nbits + 63) / 64;
    uint64_t acc = 0;
    for (size_t k = nw; k-- > 0;) {
        uint64_t w = p[k];
        if (k == nw - 1 && nbits % 64) w &= (~(uint64_t)0) >> (64 - nbits % 64);
        /* acc * x^64 + w  ==  (hi = acc, lo = w) */
        acc = mod_q_128(w, acc, q);
    }
    return acc;
}

/* (x mod Q)(y mod Q) mod Q for 64-bit residues */
uint64_t oracle_mulmod(uint64_t x, uint64_t y, uint64_t q)
{
    uint64_t lo, hi;
    clmul64_window(x, y, &lo, &hi);
    return mod_q_128(lo, hi, q);
}
