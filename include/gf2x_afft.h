/*
 * gf2x_afft.h -- multiplication of long binary polynomials on AMD MI355X
 * (gfx950) with the additive FFT over a tower field.
 *
 * Method: Chen, Cheng, Kuo, Li, Yang, "Faster Multiplication for Long Binary
 * Polynomials" (arXiv:1708.09746), Alg. 5 with w = 64 over TGF(2^128)
 * (w = 128 over TGF(2^256) as a per-context setting, gf2x_set_word_bits):
 * Split -> BasisCvt (Alg. 3) -> changeRepr -> FFT_LCH (Alg. 1) -> pointmul ->
 * iFFT_LCH -> iBasisCvt -> changeRepr back -> InterleavedCombine.
 *
 * Problem (Sec. 2.1): given a(x), b(x) in GF(2)[x] as bit sequences, return
 * c(x) = a(x) b(x).  Results are exact (bit for bit).
 *
 * Conventions shared by every entry point
 *   - Bit i of a polynomial is bit (i mod 64) of word floor(i / 64)
 *     (little-endian words).  An n-bit operand occupies ceil(n/64) words; bits
 *     at and above n in its last word are ignored.
 *   - The product of an na-bit and an nb-bit operand has na+nb-1 coefficients
 *     and is written as gf2x_out_words(na, nb) = ceil((na+nb-1)/64) words; bits
 *     at and above na+nb-1 in the last word are written as zero.
 *   - An operand of 0 bits is the zero polynomial: the product has 0 words,
 *     nothing is written and the call returns GF2X_OK.
 *   - Spectra (of the stage entry points, always w = 64) are arrays of
 *     TGF(2^128) elements, 16 bytes each: bit j of an
 *     element is the coefficient of the tower basis element v_j (Sec. 3.2,
 *     definition of (v_k)).  Spectrum entry j holds f(j̄), the value at the
 *     element whose tower representation is the integer j, of
 *     f(x) = sum_k Phi(a_k) x^k, where a_k is the k-th 64-bit word and
 *     Phi(u) = u(theta) is the polynomial u(z) evaluated at theta = x7, the
 *     tower element with only bit 64 set (Sec. 2.1 Kronecker segmentation;
 *     any generator of TGF(2^128) over GF(2) gives the same product).
 *   - Device pointers must be 8-byte aligned (words) or 16-byte aligned
 *     (spectra) and come from hipMalloc (or torch on ROCm).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     *_dev calls only enqueue work and return; completion is observed on the
 *     stream.  Calls on one context must be issued from one host thread.  A
 *     context's workspace is reused by its next call; a call that uses it
 *     (gf2x_mul_dev, gf2x_forward_dev, gf2x_simple_mul_dev,
 *     gf2x_simple_forward_dev) on a stream other than the previous such
 *     call's first makes its stream wait for everything that call enqueued
 *     (an event recorded at its end), so calls on mixed streams run one after
 *     the other.  Calls made while `stream` is being captured into a graph
 *     take no part in this ordering (the caller orders them).
 *
 * Status codes: every function returns GF2X_OK or a negative code and never
 * aborts.  gf2x_strerror() names a code; gf2x_last_error() gives the message
 * of the last failure on a context (HIP error text included).
 */
#ifndef GF2X_AFFT_H
#define GF2X_AFFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GF2X_OK = 0,
    GF2X_EINVAL = -1, /* NULL pointer with a nonzero size, bad length, overlap */
    GF2X_ERANGE = -2, /* transform length above 2^32 points (multiplier width) */
    GF2X_ENOMEM = -3, /* device workspace could not be allocated */
    GF2X_EDEVICE = -4 /* a HIP runtime error; see gf2x_last_error */
};

typedef struct gf2x_ctx gf2x_ctx;

/* Create a context on HIP device `device`: builds the constant tables (GF(256)
 * product table, butterfly multiplier basis lambda[i][t] = s_i(v_t) of
 * Sec. 4.4, the changeRepr tables of Sec. 4.3 for both word widths, the
 * constant-multiple tables of the pointwise tower product of Sec. 4.1) on the
 * host and uploads them.  The context owns them and a growable device
 * workspace; its word width starts at 64. */
int gf2x_ctx_create(gf2x_ctx **ctx, int device);

/* Release a context (synchronizes its device first). NULL is ignored. */
void gf2x_ctx_destroy(gf2x_ctx *ctx);

/* Words of the product of an na-bit and an nb-bit operand (0 if either is 0). */
size_t gf2x_out_words(uint64_t na_bits, uint64_t nb_bits);

/* log2 of the number of evaluation points N used for that product:
 * N = max(2, 2^ceil(log2(ceil(na/64) + ceil(nb/64) - 1))); -1 if either is 0. */
int gf2x_fft_log2(uint64_t na_bits, uint64_t nb_bits);

/* Device workspace bytes one product of these sizes needs (two N-point spectra
 * plus the converted operand words), with Split into 64-bit words. */
size_t gf2x_workspace_bytes(uint64_t na_bits, uint64_t nb_bits);
/* The same for a word width w of 64 or 128 bits (0 for any other w): the
 * footprint a server admits a request by on a context of that width. */
size_t gf2x_workspace_bytes_w(uint64_t na_bits, uint64_t nb_bits, int w);

/* c = a * b with HOST pointers; blocking.  Uses a process-wide context on the
 * current HIP device (created on first use, guarded by a mutex); copies the
 * operands to the device and the product back.  c receives
 * gf2x_out_words(na_bits, nb_bits) words and must not overlap a or b. */
int gf2x_mul(const uint64_t *a, uint64_t na_bits, const uint64_t *b, uint64_t nb_bits, uint64_t *c);

/* c = a * b with DEVICE pointers, enqueued on `stream` (Alg. 5).  a and b may
 * alias each other (squaring); c must not overlap either.  A small product
 * can be one kernel launch (gf2x_set_single_launch).  Below 2^15 points the
 * two forward transforms run interleaved on `stream`, their FFT passes of
 * one level sharing launches; for transforms of 2^15 points or more, part of
 * the forward
 * transform of b runs on a second stream owned by the context, forked from
 * `stream` and joined back to it by events: up to 2^19 points the whole
 * transform, above only its pack and BasisCvt.  The call stays ordered on
 * `stream` like any other. */
int gf2x_mul_dev(gf2x_ctx *ctx, const uint64_t *a, uint64_t na_bits, const uint64_t *b, uint64_t nb_bits,
                 uint64_t *c, void *stream);

/* The largest transform, 2^max_log2n points, that gf2x_mul_dev runs as one
 * launch (a single block running every stage of Alg. 5 in order, the ops in
 * the kernel arguments); -1 (the default) never does.  At most 12 (EINVAL
 * otherwise).  Results are the same either way; one launch saves the launch
 * gaps but runs every stage on one compute unit. */
int gf2x_set_single_launch(gf2x_ctx *ctx, int max_log2n);

/* Which BasisCvt sub-conversions run inside FFT passes (Alg. 3's recursion:
 * the conversion of the index bits [q, q + mb) commutes with the FFT layers
 * above them, with changeRepr and with the conversions of other bits, so a
 * pass whose tile rows hold those bits can run it before its layers, or, in
 * an inverse transform, its inverse after them).  Bits of mask: 1 in forward
 * transforms, 2 in inverse transforms, 4 split a transform's strided passes at
 * BasisCvt's top level when that keeps their number.  Only transforms of at
 * most 2^single_max_log2n points (single products: gf2x_mul_dev, the
 * no-allocation entry point, requests an idle server runs alone) or
 * 2^batch_max_log2n points (batches, serving iterations) fuse, and truncated
 * ones never do.  Default: mask 7, bounds 13 and 11.  There the launches
 * saved dominate (single products of 2^17 bits 0.13 -> 0.098 ms, 15 -> 4
 * launches; 2^18 bits 0.17 -> 0.16 ms; batches +1 % at 2^11 points, -2 % at
 * 2^12).  Above that a fused conversion's layer sweeps cost the FFT kernel
 * about what the conversion's own pass costs (both are bound by LDS, not by
 * the HBM round trip that fusion saves): products of 2^28 and 2^29 bits run
 * 0.5-1.5 % slower with mask 6.  Mask 0 runs every conversion as its own
 * pass.  Results are the same for every setting; EINVAL for a mask outside
 * 0..7 or a bound outside 0..32. */
int gf2x_set_fusion(gf2x_ctx *ctx, int mask, int single_max_log2n, int batch_max_log2n);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): c = a * b as
 * gf2x_mul_dev computes it (same result, same word width and truncation
 * settings of ctx), with the whole workspace in a fixed device buffer of
 * GF2X_STATIC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends (its address is looked up when a context is created
 * on that GPU).  The call allocates no device memory (no hipMalloc, hipFree
 * or other device-allocating routine) and creates no stream or event: every
 * kernel runs on `stream`, and it is never traced.  (Its host-side planning
 * builds a few small std::vector op lists on the host heap.)
 * A product whose workspace (gf2x_workspace_bytes_w at ctx's word width)
 * exceeds the buffer returns GF2X_ENOMEM with the sizes in gf2x_last_error;
 * with w = 64 that admits every product of at most 2^20 points, i.e.
 * operands of up to 2^25 bits each.  Every call on one GPU, from any
 * context, shares that GPU's buffer, so calls that overlap in time (other
 * streams, other host threads) race: the caller orders them, e.g. on one
 * stream.  The buffer keeps the last call's contents; no call needs it to
 * start zeroed.  Arguments, aliasing and errors otherwise as gf2x_mul_dev. */
#define GF2X_STATIC_SCRATCH_BYTES (64u << 20)
int gf2x_mul_dev_static(gf2x_ctx *ctx, const uint64_t *a, uint64_t na_bits, const uint64_t *b, uint64_t nb_bits,
                        uint64_t *c, void *stream);

/* Forward transform of one operand (Split, BasisCvt of Alg. 3 on 64-bit words,
 * changeRepr, FFT_LCH of Alg. 1 at alpha = 0): spec[j] = f(j̄) for
 * j < 2^log2n (see the spectrum convention above).  Requires
 * 2^log2n >= 2^ceil(log2(ceil(na/64))) and log2n <= 32.  spec is DEVICE memory of
 * 16 * 2^log2n bytes, written entirely. */
int gf2x_forward_dev(gf2x_ctx *ctx, const uint64_t *a, uint64_t na_bits, int log2n, void *spec, void *stream);

/* Pointwise product of two spectra in TGF(2^128) (pointmul of Alg. 5):
 * sc[j] = sa[j] * sb[j] for j < n.  sc may equal sa or sb. */
int gf2x_pointmul_dev(gf2x_ctx *ctx, const void *sa, const void *sb, void *sc, uint64_t n, void *stream);

/* Inverse transform (iFFT_LCH, iBasisCvt, changeRepr back, InterleavedCombine):
 * spec holds the values at all 2^log2n points of a polynomial
 * F(x) = sum_k F_k x^k of degree < 2^log2n with coefficients in TGF(2^128); the
 * call writes ceil(nc_bits/64) words of sum_k Psi(F_k) x^(64k), truncated to
 * nc_bits bits, where Psi is the inverse of the changeRepr map above (defined
 * on all of TGF(2^128), giving polynomials of degree < 128).  spec is
 * overwritten (used as scratch). */
int gf2x_inverse_dev(gf2x_ctx *ctx, void *spec, int log2n, uint64_t *c, uint64_t nc_bits, void *stream);

/* BasisCvt (Alg. 3) of 2^log2n 64-bit words in place: the words become the
 * coefficients g_k of the same polynomial in the novel basis X_k (Sec. 2.3.1,
 * Def. of X_k); inverse != 0 applies iBasisCvt.  The conversion only XORs
 * whole words, so it acts on each of the 64 bit positions independently. */
int gf2x_basiscvt_dev(gf2x_ctx *ctx, uint64_t *words, int log2n, int inverse, void *stream);

/* ---- the simple variant (Alg. 4) ----
 * The same product by the paper's simple method: the working field stays
 * GF(2^128) = GF(2)[x]/(x^128 + x^7 + x^2 + x + 1) in its polynomial basis
 * (Sec. 3.1), FFT_LCH evaluates at the points phi(j) of a Cantor basis
 * (Sec. 3.3: beta_0 = 1, beta_i^2 + beta_i = beta_{i-1}, each beta_i taken
 * as the root without an x^0 term; phi(j) = sum of beta_t over the set bits t
 * of j), and every butterfly and pointwise product is a full GF(2^128)
 * product.  A second, independent route to the product, for cross-checks:
 * it shares BasisCvt (Alg. 3) with the tower method and nothing else.
 *
 * gf2x_simple_mul_dev: c = a * b with DEVICE pointers, enqueued on `stream`;
 * the same sizes, output, aliasing rules and status codes as gf2x_mul_dev, and
 * the same product bits.  64-bit words and all N points always: the context's
 * word-width and truncation settings do not apply.  Uses the context's
 * workspace (gf2x_workspace_bytes(na_bits, nb_bits) bytes).
 *
 * gf2x_simple_forward_dev: spec[j] = f(phi(j)) for j < 2^log2n, where
 * f(y) = sum_k a_k y^k and the 64-bit word a_k is the field element of degree
 * < 64 with the same bits.  spec is DEVICE memory of 16 * 2^log2n bytes, an
 * element stored as two little-endian 64-bit halves (bit e of the 128 is the
 * coefficient of x^e), written entirely.  Requires
 * 2^log2n >= 2^ceil(log2(ceil(na_bits/64))) and log2n <= 32. */
int gf2x_simple_mul_dev(gf2x_ctx *ctx, const uint64_t *a, uint64_t na_bits, const uint64_t *b, uint64_t nb_bits,
                        uint64_t *c, void *stream);
int gf2x_simple_forward_dev(gf2x_ctx *ctx, const uint64_t *a, uint64_t na_bits, int log2n, void *spec,
                            void *stream);

/* One job of a batch: DEVICE pointers, same conventions as gf2x_mul_dev. */
typedef struct {
    const uint64_t *a;
    uint64_t na_bits;
    const uint64_t *b;
    uint64_t nb_bits;
    uint64_t *c;
} gf2x_job;

/* Independent products of uneven sizes, enqueued on `stream` (a one-shot
 * batch: see gf2x_batch_create).  `jobs` is HOST memory and may be reused as
 * soon as the call returns.  Each job's result is bit-identical to
 * gf2x_mul_dev on the same operands.  The plan is kept by the context until
 * its next gf2x_mul_batch call (which first waits for it). */
int gf2x_mul_batch(gf2x_ctx *ctx, const gf2x_job *jobs, size_t njobs, void *stream);

/* ---- the Frobenius-partition variant (App. C) ----
 * The same product with no Kronecker segmentation: a polynomial of fewer than
 * 128 n bits (n = 2^m) is represented by its values at the n points
 * beta_{m+64} + V_m of GF(2^128) (the field and Cantor basis of the simple
 * variant above; V_m = span(beta_0 .. beta_{m-1})), a bijection because the
 * Frobenius orbits of these points are disjoint and hold 128 points each
 * (App. C, the partition of the evaluation points).  The values are computed
 * as App. C's truncated FFT: BasisCvt (Alg. 3) over the bits, the "encoding"
 * (its first seven layers: value-vector element i = sum over j < 128 of bit
 * j n + i times P_j, P_j the product of beta_{64-t} over the set bits t of j,
 * since s_{m+t}(beta_{m+64}) = beta_{64-t}), then FFT_LCH (Alg. 1) at
 * alpha = beta_{m+64} over the n elements.  A product takes n = 2^m points
 * with m the least such that 128 n >= na + nb - 1, about half the points of
 * Alg. 4 with w = 64. */

/* m for the product of an na-bit and an nb-bit operand (-1 if either is 0). */
int gf2x_frobenius_log2n(uint64_t na_bits, uint64_t nb_bits);

/* Device workspace bytes of gf2x_frobenius_mul_dev for these sizes (0 if
 * either is 0): the operands' words and two n-point value vectors. */
size_t gf2x_frobenius_workspace_bytes(uint64_t na_bits, uint64_t nb_bits);

/* c = a * b with DEVICE pointers on `stream`, by the Frobenius partition:
 * the values of a and b at the n points, their pointwise products in
 * GF(2^128), then the inverse (iFFT_LCH at alpha, the inverse of the
 * encoding, iBasisCvt over the bits).  Conventions, aliasing, ordering and
 * errors as gf2x_mul_dev (ERANGE above 2^32 points); the context's word width
 * and truncation settings do not apply. */
int gf2x_frobenius_mul_dev(gf2x_ctx *ctx, const uint64_t *a, uint64_t na_bits, const uint64_t *b, uint64_t nb_bits,
                           uint64_t *c, void *stream);

/* The values of a (na_bits bits, na_bits <= 128 * 2^log2n, log2n <= 32) at
 * the 2^log2n points: spec[j] = a(beta_{m+64} + phi(j)), m = log2n, with
 * phi(j) the sum of beta_t over the set bits t of j; each element 16 bytes,
 * bit e the coefficient of x^e (as the simple variant's spectra).  spec is
 * DEVICE memory of 16 * 2^log2n bytes, written entirely. */
int gf2x_frobenius_forward_dev(gf2x_ctx *ctx, const uint64_t *a, uint64_t na_bits, int log2n, void *spec,
                               void *stream);

/* The inverse: given the values at the 2^log2n points of a polynomial of
 * fewer than 128 * 2^log2n bits, writes its first ceil(nc_bits/64) words to c
 * (nc_bits <= 128 * 2^log2n; bits at and above nc_bits of the polynomial are
 * dropped, those below kept).  spec is overwritten (used as scratch); c must
 * not overlap it. */
int gf2x_frobenius_inverse_dev(gf2x_ctx *ctx, void *spec, int log2n, uint64_t *c, uint64_t nc_bits, void *stream);

/* ---- tracing: per-kernel timing with HIP events (Sec. "Results" profiles the
 * same stages per component).  While a mask is set, every launch of a kernel
 * kind whose bit is in the mask carries two hipEvents in its own dispatch
 * (hipExtLaunchKernelGGL), so their interval is the kernel's execution time;
 * gf2x_trace_read() waits for them and returns one record per launch.  Kinds (bit = 1 << kind): 0 pack, 1 BasisCvt tile, 2 BasisCvt global
 * layer, 3 FFT pass, 4 pointmul, 5 changeRepr back + combine, 6 BasisCvt
 * VarSubs class pass, 7 truncated-transform step, 8 a whole product in one
 * launch (gf2x_set_single_launch: one block runs all its stages in order), 9
 * the last steps of a small product in one launch (pointmul, an inverse
 * transform of one tile with its BasisCvt, changeRepr back and combine).
 * Two FFT passes of one level of a small product (its two forward
 * transforms) can share one launch and one record. */
typedef struct {
    int kind;            /* one of the kinds above */
    uint64_t elements;   /* elements (words or 16-byte field elements) the launch covers */
    uint64_t bytes_read; /* bytes the launch must read from memory (algorithmic) */
    uint64_t bytes_written;
    uint64_t lookups;    /* LDS table reads of its subfield products (FFT passes; else 0) */
    float ms;            /* hipEventElapsedTime between the two events */
} gf2x_trace_rec;

/* Calibration: the rate of random byte lookups into a 64 KiB LDS table over
 * the whole device (one kernel, every CU busy, every address in bounds), the
 * unit that bounds the FFT passes.  Blocking. */
int gf2x_lookup_rate(gf2x_ctx *ctx, double *lookups_per_s);

/* Start recording launches of the kinds in `kind_mask` (0 stops; records kept). */
int gf2x_trace_begin(gf2x_ctx *ctx, uint32_t kind_mask);

/* Wait for the recorded events and copy up to `max` records into `out` (host
 * memory); returns the number of records available (may exceed max), or a
 * negative status.  The records are cleared afterwards. */
int64_t gf2x_trace_read(gf2x_ctx *ctx, gf2x_trace_rec *out, size_t max);

/* ---- reusable batches.  A batch fixes its jobs (device pointers and sizes)
 * at creation: the library plans every product, allocates the batch's own
 * workspace and uploads the op descriptors (synchronously).  Each run then
 * enqueues all products on `stream`: op r of every job runs in one launch per
 * kernel kind, rank after rank.  The first run records the launch sequence as
 * a hipGraph on the context's stream; later runs replay the graph.  The
 * operand and product buffers must stay valid while the batch exists; runs of
 * one batch must not overlap (they share its workspace). */
typedef struct gf2x_batch gf2x_batch;

typedef struct {
    uint64_t ops;             /* ops of all jobs */
    uint64_t ranks;           /* longest op list of a job */
    uint64_t launches;        /* kernel launches per run */
    uint64_t tiles;           /* work tiles per run */
    uint64_t workspace_bytes; /* device memory held by the batch */
} gf2x_batch_stats;

/* Execution modes: STAGED runs rank after rank, one launch per kernel kind;
 * PERSISTENT runs the whole batch in one launch of a persistent kernel (one
 * block per CU) whose blocks take (op, tile) items of a rank from a counter
 * and meet at a grid barrier between ranks (bounded wait: on timeout the run
 * stops early and gf2x_batch_check reports GF2X_EDEVICE).  The context checks
 * at creation that a CU can hold a block of that kernel (the occupancy
 * query); if none can, a persistent run fails with GF2X_EDEVICE before it
 * launches.  All blocks are then resident unless other work shares the
 * device, which the bounded wait turns into that error. */
enum { GF2X_BATCH_STAGED = 0, GF2X_BATCH_PERSISTENT = 1 };

int gf2x_batch_create(gf2x_ctx *ctx, const gf2x_job *jobs, size_t njobs, int mode, gf2x_batch **batch);
int gf2x_batch_run(gf2x_batch *batch, void *stream);
/* Waits for the device, then reports whether the last persistent run finished
 * every item (GF2X_OK) or stopped on a wait timeout (GF2X_EDEVICE). */
int gf2x_batch_check(gf2x_batch *batch);
/* Polls a persistent run's barrier wait may make before the run is abandoned
 * (default 2^26, about 4 s); 0 abandons it at the first wait. */
int gf2x_batch_set_spin_limit(gf2x_batch *batch, uint32_t polls);
int gf2x_batch_info(const gf2x_batch *batch, gf2x_batch_stats *stats);
/* Synchronizes the device, then frees the batch. NULL is ignored. */
void gf2x_batch_destroy(gf2x_batch *batch);

/* ---------------------------------------------------------------- schedules
 * FFT pass schedule per transform size 2^m: the bottom pass runs the layers
 * below bottom_log on contiguous tiles of 2^bottom_log points, and the layers
 * above are split evenly into strided passes of at most 2^col_rows_log rows
 * (both in 1..12; 2^12 points fill one LDS tile).  Every schedule computes the
 * same bits; schedules differ in the number of passes over memory and in tile
 * shape.  Default 12 and 6 for every m.  A schedule applies to products
 * planned after it is set (a gf2x_batch keeps the plan it was created with). */
typedef struct {
    int32_t m;            /* transform size 2^m */
    int32_t bottom_log;   /* chosen schedule */
    int32_t col_rows_log;
    int32_t copies;       /* transforms timed together */
    int32_t candidates;   /* distinct schedules timed */
    float us_default;     /* forward + inverse time per launch set, default schedule (us) */
    float us_best;        /* the same for the chosen schedule */
} gf2x_tune_rec;

/* EINVAL for m outside 1..32 or a value outside 1..12. */
int gf2x_set_schedule(gf2x_ctx *ctx, int m, int bottom_log, int col_rows_log);
int gf2x_get_schedule(gf2x_ctx *ctx, int m, int *bottom_log, int *col_rows_log);

/* Autotuner: for each m in [m_lo, m_hi] (1 <= m_lo <= m_hi <= 26) times every
 * distinct candidate schedule (bottom_log in 7..12, col_rows_log in 3..12,
 * capped at m) on a forward and an inverse FFT of max(1, 2^(21-m)) transforms
 * at once, one multi-op launch per pass as in batches, `reps` times each;
 * keeps the fastest in ctx and writes one record per m to `out` (NULL
 * allowed).  Blocking; uses a temporary device buffer (ENOMEM if it does
 * not fit). */
int gf2x_autotune(gf2x_ctx *ctx, int m_lo, int m_hi, int reps, gf2x_tune_rec *out);

/* --------------------------------------------------- truncated transforms
 * A product of n_c = ceil(na/64) + ceil(nb/64) - 1 word coefficients needs
 * N = 2^m >= n_c evaluation points; with truncation the two forward
 * transforms evaluate only the first M points, n_c rounded up to a multiple
 * of 2^g, g = max(m - levels, 6), and further to the next M whose count of
 * 2^g blocks has at most max_terms set bits (each set bit is a full block of
 * the recursion below; 0: any count), pointmul runs on M points, and the inverse
 * recovers the coefficients from those M values (the coefficients at M and
 * beyond are zero by the degree bound): the butterflies of Alg. 1 restricted
 * to the needed points, and their inverse run on the values below M and the
 * known coefficients above it.  Only transforms of at least 2^min_log2n
 * points are truncated: each step of the recursion is a pass of its own,
 * which smaller transforms do not repay.  levels = 0 turns truncation off
 * (M = N).  The default, 3 levels from 2^23 points on with at most 2 terms,
 * follows single-product timings on one MI355X: with n_c just above N/2,
 * M = 5/8 N takes 10 % (2^23 points) to 16 % (2^25) less time than M = N;
 * M = 3/4 N 5-11 % less; M = 7/8 N (three terms) 5-9 % more; at 2^22 points
 * and below truncation gains nothing or loses.  The product bits are the same
 * either way. */

/* Truncation for products planned afterwards: levels in 0..16, min_log2n in
 * 1..32, max_terms in 0..32 (EINVAL outside). */
int gf2x_set_truncation(gf2x_ctx *ctx, int levels, int min_log2n, int max_terms);
/* Points M a product of these sizes is evaluated at on ctx (0 if empty). */
uint64_t gf2x_eval_points(gf2x_ctx *ctx, uint64_t na_bits, uint64_t nb_bits);

/* ---- word width of Split (Alg. 5 with w = 64 or w = 128) ----
 * Alg. 5 splits the operands into w-bit words and multiplies in TGF(2^2w).
 * The default w = 64 works in TGF(2^128).  w = 128 works in TGF(2^256): half
 * as many points (one layer fewer), each a TGF(2^256) element, changeRepr of
 * 128-bit words at x8 (which generates TGF(2^256): it lies outside
 * TGF(2^128)), the pointwise products in TGF(2^256), and InterleavedCombine
 * of 255-bit partial products at 128-bit offsets.  The product bits are the
 * same for either width.  On the device a TGF(2^256) spectrum is two planes
 * of TGF(2^128) halves, transformed alone with the same multipliers (Prop. 2:
 * a subfield multiplier acts on each half).  w = 128 is never truncated.
 *
 * gf2x_set_word_bits: the width for products planned afterwards on ctx
 * (gf2x_mul_dev, batches built afterwards, and requests submitted afterwards
 * to a server), 64 or 128 (EINVAL otherwise).  The stage entry points
 * (gf2x_forward_dev ... gf2x_basiscvt_dev) and gf2x_workspace_bytes always
 * use w = 64.  gf2x_get_word_bits: the current width (0 for a NULL ctx). */
int gf2x_set_word_bits(gf2x_ctx *ctx, int w);
int gf2x_get_word_bits(gf2x_ctx *ctx);

/* ------------------------------------------------------------------ serving
 * A request loop with continuous batching (not part of the paper: a serving
 * pattern around its product).  Requests are products whose operands and
 * result buffer live in device memory owned by the caller, who keeps them
 * valid until the request completes.  Each request is admitted when its
 * device footprint (the two converted operands and the two N-point spectra,
 * gf2x_workspace_bytes) fits in the server's arena and a slot is free; its
 * state then stays on the device until it completes.  The engine runs
 * iterations: every admitted request advances by up to `levels_per_iter`
 * dependency levels of its product (fewer when `iter_tiles` bounds the
 * iteration's work, so that iterations stay short under load), the ops of all requests at one level run
 * together in multi-op launches (STAGED) or in one persistent launch per
 * iteration (PERSISTENT), and requests that arrive meanwhile join at the next
 * iteration as memory and slots free up.  Admission is first come, first
 * served.  A request's result is the same bits as gf2x_mul_dev gives it alone.
 *
 * A server borrows ctx's tables; ctx, the server and its requests are used
 * from one host thread.  Timestamps are CLOCK_MONOTONIC nanoseconds
 * (gf2x_now_ns). */
typedef struct gf2x_server gf2x_server;

typedef struct {
    uint64_t arena_bytes;     /* device memory for request state (one allocation) */
    uint32_t max_active;      /* admitted requests at most (slots) */
    uint32_t levels_per_iter; /* dependency levels each request advances per iteration (>= 1) */
    uint32_t inflight;        /* iterations queued on the device at once (1..4) */
    int32_t mode;             /* GF2X_BATCH_STAGED, GF2X_BATCH_PERSISTENT or GF2X_SERVER_ADAPTIVE */
    uint64_t iter_tiles;      /* work bound: an iteration stops adding levels (beyond the first)
                                 once its tiles would exceed this; 0 = no bound */
} gf2x_server_cfg;

/* Server mode GF2X_SERVER_ADAPTIVE: an iteration runs as one persistent
 * launch while at least GF2X_SERVER_ADAPTIVE_ACTIVE requests are admitted and
 * fewer than GF2X_SERVER_ADAPTIVE_BACKLOG wait in the queue (no launch tails:
 * the lowest latency under load), and staged otherwise (few requests: the
 * lowest latency alone; a long queue: the highest throughput).  Under light
 * load (nothing queued, at most two requests admitted) an iteration runs every
 * remaining level of the admitted requests; a lone request then runs as a
 * plain call does, one launch per op, with no descriptor upload. */
enum { GF2X_SERVER_ADAPTIVE = 2, GF2X_SERVER_ADAPTIVE_ACTIVE = 8, GF2X_SERVER_ADAPTIVE_BACKLOG = 1024 };

typedef struct {
    uint64_t tag;        /* the caller's tag from gf2x_server_submit */
    int32_t status;      /* GF2X_OK, or GF2X_EDEVICE when its iteration failed */
    uint32_t iterations; /* iterations the request took part in */
    uint64_t t_submit_ns, t_admit_ns, t_done_ns;
} gf2x_done;

typedef struct {
    uint64_t submitted, admitted, completed, iterations, launches;
    uint64_t queued, active;            /* now */
    uint64_t arena_used, arena_peak;    /* bytes */
    uint64_t active_peak;
} gf2x_server_stats;

uint64_t gf2x_now_ns(void);

/* Allocates the arena and per-iteration descriptor buffers on ctx's device.
 * ENOMEM if the arena does not fit; EINVAL for a zero field or a bad mode. */
int gf2x_server_create(gf2x_ctx *ctx, const gf2x_server_cfg *cfg, gf2x_server **server);

/* Queues c = a * b (device pointers, sizes in bits as for gf2x_mul_dev).
 * `stream` is the caller's stream that produced a and b (and last used c):
 * an event is recorded on it now, and the request's first work on the
 * server's own stream waits for it, so the request reads its operands and
 * writes c only after everything enqueued on `stream` before this call.
 * Work the caller enqueues later may read c once poll reports the request.
 * Returns at once: EINVAL for NULL pointers with nonzero sizes or overlap of
 * c with a or b, ERANGE for N > 2^32, ENOMEM if the request's footprint
 * exceeds the whole arena (it could never be admitted); the request is then
 * not queued.  An empty product is complete at once (nothing is written). */
int gf2x_server_submit(gf2x_server *server, const uint64_t *a, uint64_t na_bits, const uint64_t *b, uint64_t nb_bits,
                       uint64_t *c, uint64_t tag, void *stream);

/* Runs the engine until gf2x_now_ns() >= until_ns or there is nothing left
 * to do: records completions, admits queued requests, builds and launches
 * iterations (at most cfg.inflight queued at once).  Returns EDEVICE after a
 * device error (the requests involved complete with that status). */
int gf2x_server_step(gf2x_server *server, uint64_t until_ns);

/* Moves up to `max` completion records, oldest first, into out; returns how
 * many. */
size_t gf2x_server_poll(gf2x_server *server, gf2x_done *out, size_t max);

int gf2x_server_info(const gf2x_server *server, gf2x_server_stats *stats);

/* Waits for the device, then frees the server (queued requests are dropped).
 * NULL is ignored. */
void gf2x_server_destroy(gf2x_server *server);

/* Name of a status code. */
const char *gf2x_strerror(int status);

/* Message of the last failure on ctx ("" if none); valid until the next call. */
const char *gf2x_last_error(gf2x_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* GF2X_AFFT_H */
