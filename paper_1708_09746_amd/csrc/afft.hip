// GPU executor and C ABI of the additive-FFT GF(2)[x] multiplier (gfx950).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gf2x_afft.h"
#include "afft_plan.hpp"
#include "tower_host.hpp"

using namespace gf2x;

// ------------------------------------------------------------------ kernels

__global__ __launch_bounds__(kThreads) void k_pack(PackOp P) {
    const uint64_t nt = pack_tiles(P);
    for (uint64_t t = blockIdx.x; t < nt; t += gridDim.x) pack_tile(threadIdx.x, blockDim.x, t, P);
}

template <int WIDE>
__global__ __launch_bounds__(kThreads) void k_bc_tile(BcTileOp B) {
    __shared__ uint4 lds[1 << kBcTileLog128];  // 64 KiB
    const uint64_t nt = bc_tiles(B);
    for (uint64_t t = blockIdx.x; t < nt; t += gridDim.x) {
        if (WIDE)
            bc_tile<uint4>(threadIdx.x, blockDim.x, t, B, lds);
        else
            bc_tile<uint64_t>(threadIdx.x, blockDim.x, t, B, (uint64_t*)lds);
    }
}

template <int WIDE>
__global__ __launch_bounds__(kThreads) void k_bc_class(BcClassOp C) {
    __shared__ uint4 lds[1 << kBcTileLog128];  // 64 KiB
    const uint64_t nt = bc_class_tiles(C);
    for (uint64_t t = blockIdx.x; t < nt; t += gridDim.x) {
        if (WIDE)
            bc_class_tile<uint4>(threadIdx.x, blockDim.x, t, C, lds);
        else
            bc_class_tile<uint64_t>(threadIdx.x, blockDim.x, t, C, (uint64_t*)lds);
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

// Tiles of one FFT pass, block-strided; each block loads the tables and the
// pass's local mu-sets once, and prefetches the next tile's elements into
// registers while the current tile's layers run.
constexpr int kFftPrefetch = (1 << kFftTileLog) / kThreads;

__global__ __launch_bounds__(kThreads) void k_fft(FftPass A, const uint8_t* g_mt, const uint32_t* g_lam,
                                                  const uint4* g_phi) {
    __shared__ __align__(16) uint8_t mt[65536];
    __shared__ uint32_t lam[1024];
    __shared__ uint4 tl[1 << kFftTileLog];
    __shared__ uint4 mu[1 << kFftTileLog];
    __shared__ uint4 mu_tile[32];
    const int tid = threadIdx.x, nt = blockDim.x;
    copy_words(tid, nt, (uint32_t*)mt, (const uint32_t*)g_mt, 16384);
    copy_words(tid, nt, lam, g_lam, 1024);
    __syncthreads();
    fft_local_mu(tid, nt, A, mt, lam, mu);
    const uint64_t ntiles = fft_tiles(A);
    uint64_t t = blockIdx.x;
    if (t >= ntiles) return;
    FftTileGeom G = fft_geom(A, t);
    uint4 pre[kFftPrefetch];
#pragma unroll
    for (int j = 0; j < kFftPrefetch; ++j) {
        uint32_t e = tid + j * nt;
        if (e < G.nel) pre[j] = fft_load(A, g_phi, G, e);
    }
    while (true) {
#pragma unroll
        for (int j = 0; j < kFftPrefetch; ++j) {
            uint32_t e = tid + j * nt;
            if (e < G.nel) tl[e] = pre[j];
        }
        __syncthreads();
        const uint64_t tn = t + gridDim.x;
        FftTileGeom Gn = G;
        if (tn < ntiles) {
            Gn = fft_geom(A, tn);
#pragma unroll
            for (int j = 0; j < kFftPrefetch; ++j) {
                uint32_t e = tid + j * nt;
                if (e < Gn.nel) pre[j] = fft_load(A, g_phi, Gn, e);
            }
        }
        fft_tile_layers<1>(tid, nt, A, G, mt, lam, tl, mu, mu_tile);
        for (uint32_t e = tid; e < G.nel; e += nt) A.dst[G.gbase | fft_elem_index(A, G, e)] = tl[e];
        if (tn >= ntiles) break;
        __syncthreads();
        t = tn;
        G = Gn;
    }
}

__global__ __launch_bounds__(kThreads) void k_pmul(PmulOp P, const uint8_t* g_mt) {
    __shared__ __align__(16) uint8_t mt[65536];
    copy_words(threadIdx.x, blockDim.x, (uint32_t*)mt, (const uint32_t*)g_mt, 16384);
    __syncthreads();
    const uint64_t nt = pmul_tiles(P);
    for (uint64_t t = blockIdx.x; t < nt; t += gridDim.x) pmul_tile(threadIdx.x, blockDim.x, t, P, mt);
}

__global__ __launch_bounds__(kThreads) void k_psi(PsiOp P, const uint4* g_psi) {
    __shared__ uint4 tab[16 * 256];  // 64 KiB
    copy_words(threadIdx.x, blockDim.x, tab, g_psi, 16 * 256);
    __syncthreads();
    const uint64_t nt = psi_tiles(P);
    for (uint64_t t = blockIdx.x; t < nt; t += gridDim.x) psi_tile(threadIdx.x, blockDim.x, t, P, tab);
}

// ------------------------------------------------------------------ context

struct gf2x_ctx {
    int device = 0;
    int ncu = 256;
    uint8_t* d_mt = nullptr;
    uint32_t* d_lam = nullptr;
    uint4* d_phi = nullptr;
    uint4* d_psi = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    char* io = nullptr;  // operand/product staging for the host-pointer entry point
    size_t io_bytes = 0;
    hipStream_t own_stream = nullptr;
    std::string err;
    // tracing
    uint32_t trace_mask = 0;
    struct Pending {
        gf2x_trace_rec rec;
        hipEvent_t start, stop;
    };
    std::vector<Pending> trace;
};

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

int ensure_ws(gf2x_ctx* ctx, size_t bytes, hipStream_t st) {
    if (bytes <= ctx->ws_bytes) return GF2X_OK;
    // work already enqueued may still use the old buffer
    hipError_t e = hipStreamSynchronize(st);
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
            uint64_t n = 1ull << (op.fft.log_m + op.fft.log_cosets);
            r.elements = n;
            r.bytes_read = op.fft.phi_in ? 8 * n : 16 * n;
            r.bytes_written = 16 * n;
            break;
        }
        case OpKind::Pmul:
            r.elements = op.pmul.n;
            r.bytes_read = 32 * op.pmul.n;
            r.bytes_written = 16 * op.pmul.n;
            break;
        case OpKind::BcClass:
            r.elements = op.bcc.nelem;
            r.bytes_read = r.bytes_written = op.bcc.nelem * (op.bcc.wide ? 16 : 8);
            break;
        case OpKind::Psi:
            r.elements = op.psi.nwords;
            r.bytes_read = 16 * std::min(op.psi.nwords, op.psi.nspec);
            r.bytes_written = 8 * op.psi.nwords;
            break;
    }
}

int run_ops(gf2x_ctx* ctx, const std::vector<Op>& ops, hipStream_t st) {
    const uint64_t ncu = (uint64_t)ctx->ncu;
    for (const Op& op : ops) {
        gf2x_ctx::Pending pend{};
        const bool traced = (ctx->trace_mask >> (int)op.kind) & 1u;
        if (traced) {
            op_traffic(op, pend.rec);
            hipError_t e = hipEventCreate(&pend.start);
            if (e == hipSuccess) e = hipEventCreate(&pend.stop);
            if (e == hipSuccess) e = hipEventRecord(pend.start, st);
            if (e != hipSuccess) return hip_fail(ctx, e, "trace event");
        }
        switch (op.kind) {
            case OpKind::Pack:
                hipLaunchKernelGGL(k_pack, dim3(grid_for(pack_tiles(op.pack), 8 * ncu)), dim3(kThreads), 0, st, op.pack);
                break;
            case OpKind::BcTile:
                if (op.bct.wide)
                    hipLaunchKernelGGL(k_bc_tile<1>, dim3(grid_for(bc_tiles(op.bct), 2 * ncu)), dim3(kThreads), 0, st, op.bct);
                else
                    hipLaunchKernelGGL(k_bc_tile<0>, dim3(grid_for(bc_tiles(op.bct), 2 * ncu)), dim3(kThreads), 0, st, op.bct);
                break;
            case OpKind::BcLayer: {
                uint64_t items = op.bcl.nelem / 2;
                uint64_t blocks = (items + kThreads - 1) / kThreads;
                if (op.bcl.wide)
                    hipLaunchKernelGGL(k_bc_layer<1>, dim3(grid_for(blocks, 16 * ncu)), dim3(kThreads), 0, st, op.bcl);
                else
                    hipLaunchKernelGGL(k_bc_layer<0>, dim3(grid_for(blocks, 16 * ncu)), dim3(kThreads), 0, st, op.bcl);
                break;
            }
            case OpKind::Fft:
                hipLaunchKernelGGL(k_fft, dim3(grid_for(fft_tiles(op.fft), ncu)), dim3(kThreads), 0, st, op.fft,
                                   (const uint8_t*)ctx->d_mt, (const uint32_t*)ctx->d_lam, (const uint4*)ctx->d_phi);
                break;
            case OpKind::Pmul:
                hipLaunchKernelGGL(k_pmul, dim3(grid_for(pmul_tiles(op.pmul), 2 * ncu)), dim3(kThreads), 0, st, op.pmul,
                                   (const uint8_t*)ctx->d_mt);
                break;
            case OpKind::BcClass:
                if (op.bcc.wide)
                    hipLaunchKernelGGL(k_bc_class<1>, dim3(grid_for(bc_class_tiles(op.bcc), 2 * ncu)), dim3(kThreads), 0, st, op.bcc);
                else
                    hipLaunchKernelGGL(k_bc_class<0>, dim3(grid_for(bc_class_tiles(op.bcc), 2 * ncu)), dim3(kThreads), 0, st, op.bcc);
                break;
            case OpKind::Psi:
                hipLaunchKernelGGL(k_psi, dim3(grid_for(psi_tiles(op.psi), 2 * ncu)), dim3(kThreads), 0, st, op.psi,
                                   (const uint4*)ctx->d_psi);
                break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(ctx, e, "kernel launch");
        if (traced) {
            e = hipEventRecord(pend.stop, st);
            if (e != hipSuccess) return hip_fail(ctx, e, "trace event");
            ctx->trace.push_back(pend);
        }
    }
    return GF2X_OK;
}

constexpr int kMaxLog2N = 32;  // multipliers s_i(v_t) are tabulated for t < 32

int check_ctx(gf2x_ctx* ctx) { return ctx ? GF2X_OK : GF2X_EINVAL; }

std::mutex g_default_mu;
gf2x_ctx* g_default = nullptr;

}  // namespace

// ------------------------------------------------------------------ C ABI

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
    ReprTables R = build_repr(T);
    if (!R.ok) {
        delete ctx;
        return GF2X_EINVAL;
    }
    std::vector<uint4> phi(8 * 256), psi(16 * 256);
    for (int i = 0; i < 8 * 256; ++i) phi[i] = to_u4(R.phi[i]);
    for (int i = 0; i < 16 * 256; ++i) psi[i] = to_u4(R.psi[i]);

    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_mt, 65536);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_lam, sizeof(lam));
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_phi, phi.size() * sizeof(uint4));
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_psi, psi.size() * sizeof(uint4));
    if (e == hipSuccess) e = hipMemcpy(ctx->d_mt, mt.data(), 65536, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->d_lam, lam, sizeof(lam), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->d_phi, phi.data(), phi.size() * sizeof(uint4), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->d_psi, psi.data(), psi.size() * sizeof(uint4), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->own_stream, hipStreamNonBlocking);
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
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->io) (void)hipFree(ctx->io);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->own_stream);
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

int gf2x_mul_dev(gf2x_ctx* ctx, const uint64_t* a, uint64_t na_bits, const uint64_t* b, uint64_t nb_bits,
                 uint64_t* c, void* stream) {
    if (check_ctx(ctx)) return GF2X_EINVAL;
    ctx->err.clear();
    Sizes s = make_sizes(na_bits, nb_bits);
    if (!s.out_words) return GF2X_OK;
    if (!a || !b || !c) return fail(ctx, GF2X_EINVAL, "NULL operand or product pointer");
    if (s.m > kMaxLog2N) return fail(ctx, GF2X_ERANGE, "transform length above 2^32");
    if (ranges_overlap(c, 8 * s.out_words, a, 8 * s.n_a) || ranges_overlap(c, 8 * s.out_words, b, 8 * s.n_b))
        return fail(ctx, GF2X_EINVAL, "product overlaps an operand");
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    Workspace w = workspace_for(s);
    int rc = ensure_ws(ctx, w.bytes, st);
    if (rc) return rc;
    std::vector<Op> ops;
    plan_mul(ops, s, a, b, c, ctx->ws);
    return run_ops(ctx, ops, st);
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
    int rc = ensure_ws(ctx, align256(8ull << m_a), st);
    if (rc) return rc;
    std::vector<Op> ops;
    emit_forward(ops, a, na_bits, (uint64_t*)ctx->ws, m_a, (uint4*)spec, log2n);
    return run_ops(ctx, ops, st);
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
    emit_inverse(ops, (uint4*)spec, log2n, c, nc_bits);
    return run_ops(ctx, ops, (hipStream_t)stream);
}

int gf2x_basiscvt_dev(gf2x_ctx* ctx, uint64_t* words, int log2n, int inverse, void* stream) {
    if (check_ctx(ctx)) return GF2X_EINVAL;
    ctx->err.clear();
    if (!words) return fail(ctx, GF2X_EINVAL, "NULL words");
    if (log2n < 0 || log2n > 40) return fail(ctx, GF2X_ERANGE, "log2n out of range");
    DeviceGuard g(ctx->device);
    std::vector<Op> ops;
    emit_bc(ops, words, 0, log2n, inverse ? 1 : 0);
    return run_ops(ctx, ops, (hipStream_t)stream);
}

int gf2x_mul_batch(gf2x_ctx* ctx, const gf2x_job* jobs, size_t njobs, void* stream) {
    if (check_ctx(ctx)) return GF2X_EINVAL;
    ctx->err.clear();
    if (njobs == 0) return GF2X_OK;
    if (!jobs) return fail(ctx, GF2X_EINVAL, "NULL job array");
    std::vector<Sizes> sz(njobs);
    std::vector<size_t> off(njobs);
    size_t total = 0;
    for (size_t j = 0; j < njobs; ++j) {
        const gf2x_job& J = jobs[j];
        sz[j] = make_sizes(J.na_bits, J.nb_bits);
        if (!sz[j].out_words) continue;
        if (!J.a || !J.b || !J.c) return fail(ctx, GF2X_EINVAL, "NULL pointer in job " + std::to_string(j));
        if (sz[j].m > kMaxLog2N) return fail(ctx, GF2X_ERANGE, "job " + std::to_string(j) + " too long");
        off[j] = total;
        total += workspace_for(sz[j]).bytes;
    }
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    int rc = ensure_ws(ctx, total, st);
    if (rc) return rc;
    std::vector<Op> ops;
    for (size_t j = 0; j < njobs; ++j) {
        if (!sz[j].out_words) continue;
        plan_mul(ops, sz[j], jobs[j].a, jobs[j].b, jobs[j].c, ctx->ws + off[j]);
    }
    return run_ops(ctx, ops, st);
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

}  // extern "C"
