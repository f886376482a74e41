// Device side of the library (gfx950): evaluation-key upload and the gate
// bootstrapping pipeline.
//
//   K1 precombine      (0, const) + s1*c1 + s2*c2, then modulus switch to
//                      Z_2N (§4.1 Eqs. (6)-(11), Algs. 1-2)
//   K2 br_plain        blind rotation, exact 32-bit integer VALU products
//   K3 br_mfma         blind rotation, exact split-limb int8 MFMA products
//                      (mk_mfma.hip)
//   K4 extract_ks      sample extraction, + 1/8, multi-key key switching
//                      (§3.2 MKKeySwitch)
//
// All arithmetic is on Torus32 words and wraps mod 2^32; nothing on the GPU
// uses floating point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "mk_device_common.h"
#include "mk_internal.h"

namespace mk {

// ------------------------------------------------------------- helpers ---

int hip_fail(hipError_t e, const char *what) {
    return fail(MK_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define MK_HIP(call, what)                                   \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return hip_fail(e_, what);     \
    } while (0)

StageTimer::StageTimer(mk_ctx *c, int st, hipStream_t str) : ctx(c), stage(st), s(str) {
    if (ctx->dev.profiling < (st >= 4 ? 2 : 1)) return;
    if (hipEventCreate(&b) != hipSuccess || hipEventCreate(&e) != hipSuccess) {
        b = e = nullptr;
        return;
    }
    (void)hipEventRecord(b, s);
}

StageTimer::~StageTimer() {
    if (!b) return;
    (void)hipEventRecord(e, s);
    ctx->dev.events[stage].emplace_back((void *)b, (void *)e);
}

static void drain_events(mk_ctx *ctx) {
    DeviceKeys &D = ctx->dev;
    for (int st = 0; st < MK_PROFILE_SLOTS; ++st) {
        for (auto &pr : D.events[st]) {
            hipEvent_t b = (hipEvent_t)pr.first, e = (hipEvent_t)pr.second;
            float ms = 0;
            if (hipEventSynchronize(e) == hipSuccess && hipEventElapsedTime(&ms, b, e) == hipSuccess) {
                D.prof_ms[st] += ms;
                D.prof_launches[st] += 1;
            }
            (void)hipEventDestroy(b);
            (void)hipEventDestroy(e);
        }
        D.events[st].clear();
    }
}

int ensure_scratch(mk_ctx *ctx, size_t bytes) {
    DeviceKeys &D = ctx->dev;
    if (D.scratch_bytes >= bytes) return MK_OK;
    if (D.fixed_scratch) return fail(MK_EINTERNAL, "fixed scratch block too small (gate buffers)");
    if (D.scratch) {
        MK_HIP(hipDeviceSynchronize(), "scratch sync");
        (void)hipFree(D.scratch);
        D.scratch = nullptr;
        D.scratch_bytes = 0;
    }
    size_t sz = bytes + bytes / 4;
    hipError_t e = hipMalloc(&D.scratch, sz);
    if (e != hipSuccess) {
        D.scratch = nullptr;
        return fail(MK_ENOMEM, "device scratch allocation failed");
    }
    D.scratch_bytes = sz;
    return MK_OK;
}

static int check_uploaded(const mk_ctx *ctx) {
    if (!ctx->dev.uploaded) return fail(MK_ESTATE, "evaluation key not uploaded (mk_upload_eval_key)");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != ctx->dev.device)
        return fail(MK_ESTATE, "current HIP device differs from the upload device");
    return MK_OK;
}

// -------------------------------------------------------------- upload ---

void device_release(mk_ctx *ctx) {
    drain_events(ctx);
    DeviceKeys &D = ctx->dev;
    void *ptrs[] = {D.bk_ext, D.evk_ext, D.bk_win, D.evk_win, D.ks, D.ks_win, D.scratch, D.mfma_scratch,
                    D.ks_scratch, D.circ_scratch, D.status};
    bool any = false;
    for (void *p : ptrs) any |= p != nullptr;
    if (any) {
        (void)hipDeviceSynchronize();
        for (void *p : ptrs)
            if (p) (void)hipFree(p);
    }
    for (void *&st : D.aux_stream)
        if (st) (void)hipStreamDestroy((hipStream_t)st);
    for (void *&ev : D.aux_event)
        if (ev) (void)hipEventDestroy((hipEvent_t)ev);
    const int prof = D.profiling;
    const auto tuned = D.tuned_tiles;
    const auto tuned_parts = D.tuned_parts;
    const int f0 = D.force_tiles[0], f1 = D.force_tiles[1];
    const int rk = D.rot_kind, gp = D.graph_piece;
    D = DeviceKeys();
    D.rot_kind = rk;
    D.graph_piece = gp;
    D.profiling = prof;
    D.tuned_tiles = tuned;
    D.tuned_parts = tuned_parts;
    D.force_tiles[0] = f0;
    D.force_tiles[1] = f1;
}

template <class T>
static int dev_alloc_copy(T **dst, const std::vector<T> &src, hipStream_t s, const char *what) {
    if (hipMalloc((void **)dst, src.size() * sizeof(T)) != hipSuccess) {
        *dst = nullptr;
        return fail(MK_ENOMEM, std::string("device allocation failed: ") + what);
    }
    MK_HIP(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s), what);
    return MK_OK;
}

// Extended form [-K | K] of a key polynomial (plain path).
static void put_ext(uint32_t *dst, const uint32_t *K, int N) {
    for (int m = 0; m < N; ++m) {
        dst[m] = 0u - K[m];
        dst[N + m] = K[m];
    }
}

int device_upload(mk_ctx *ctx, void *stream) {
    const mk_params &P = ctx->p;
    for (int i = 0; i < P.k; ++i)
        if (!ctx->parties[i].present) return fail(MK_ESTATE, "mk_upload_eval_key: a party has no keys");
    device_release(ctx);
    hipStream_t s = (hipStream_t)stream;
    const int N = P.N, n = P.n, ell = P.bk_ell, k = P.k;
    // plain-path extended keys
    std::vector<uint32_t> bk_ext((size_t)k * n * 3 * ell * 2 * N);
    for (int i = 0; i < k; ++i)
        for (size_t poly = 0; poly < (size_t)n * 3 * ell; ++poly)
            put_ext(&bk_ext[((size_t)i * n * 3 * ell + poly) * 2 * N],
                    &ctx->parties[i].bk[poly * N], N);
    std::vector<uint32_t> evk((size_t)(k + 1) * ell * N);
    for (size_t x = 0; x < (size_t)ell * N; ++x) evk[x] = 0u - ctx->crs[x];
    for (int i = 0; i < k; ++i)
        std::memcpy(&evk[(size_t)(i + 1) * ell * N], ctx->parties[i].pk.data(), (size_t)ell * N * 4);
    std::vector<uint32_t> evk_ext((size_t)(k + 1) * ell * 2 * N);
    for (size_t poly = 0; poly < (size_t)(k + 1) * ell; ++poly)
        put_ext(&evk_ext[poly * 2 * N], &evk[poly * N], N);
    std::vector<uint32_t> ks;
    ks.reserve(k * ctx->parties[0].ks.size());
    for (int i = 0; i < k; ++i) ks.insert(ks.end(), ctx->parties[i].ks.begin(), ctx->parties[i].ks.end());

    int rc;
    DeviceKeys &D = ctx->dev;
    MK_HIP(hipGetDevice(&D.device), "hipGetDevice");
    if ((rc = dev_alloc_copy(&D.bk_ext, bk_ext, s, "bk_ext"))) return rc;
    if ((rc = dev_alloc_copy(&D.evk_ext, evk_ext, s, "evk_ext"))) return rc;
    if ((rc = dev_alloc_copy(&D.ks, ks, s, "ks"))) return rc;
    if ((rc = mfma_upload(ctx, evk, s))) return rc;
    if ((rc = ks_mfma_upload(ctx, s))) return rc;
    MK_HIP(hipStreamSynchronize(s), "upload sync");
    D.uploaded = true;
    return MK_OK;
}

// ---------------------------------------------------------- K1 kernels ---

// Constant, s1, s2 of each bootstrapped gate (§4.1; NOR and XNOR constants
// are the readings 3/8 and 1/2 that satisfy the truth table).
__constant__ uint32_t c_gate_const[6] = {0xA0000000u, 0xE0000000u, 0x20000000u,
                                         0x60000000u, 0x00000000u, 0x80000000u};
__constant__ int c_gate_s1[6] = {-1, 1, 1, -1, 2, -2};
__constant__ int c_gate_s2[6] = {-1, 1, 1, -1, -2, 2};

__global__ void precombine_kernel(const uint8_t *__restrict__ types,
                                  const uint32_t *__restrict__ in1,
                                  const uint32_t *__restrict__ in2, size_t stride,
                                  int words, int log2_2N, size_t total,
                                  uint32_t *__restrict__ abar, uint32_t *status) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const size_t g = idx / words;
    const int w = (int)(idx - g * words);
    // out-of-range types read as NAND and are reported through the status
    const int t = types[g] < 6 ? types[g] : 0;
    if (t != types[g] && w == 0) atomicOr(status, kStatusBadType);
    uint32_t x = (uint32_t)c_gate_s1[t] * in1[g * stride + w] +
                 (uint32_t)c_gate_s2[t] * in2[g * stride + w];
    if (w == 0) x += c_gate_const[t];
    abar[idx] = (x + (1u << (31 - log2_2N))) >> (32 - log2_2N);
}

__global__ void not_kernel(const uint32_t *__restrict__ in, uint32_t *out, size_t stride,
                           int words, size_t total) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const size_t g = idx / words;
    const int w = (int)(idx - g * words);
    const uint32_t v = in[g * stride + w];
    out[g * stride + w] = (w == 0 ? 0x40000000u : 0u) - v;
}

// ------------------------------------------------- K2: plain rotation ----
//
// One workgroup per gate, persistent over all k*n CMux steps; the
// accumulator (c_0..c_k) lives in LDS.  Each step:
//   1. P_j = X^-a ACC_j - ACC_j, decomposed into ell signed int8 digit polys.
//   2. stage 1: thread unit (j, m0) computes R consecutive outputs of
//      c'_j = sum_l u_{j,l} * d_l and w_j = sum_l u_{j,l} * b_{j,l}.
//   3. w = sum_j w_j, decomposed into v.
//   4. stage 2: units (o, m0): c'_0 += sum_l v_l * f0_l, c'_i += v * f1.
// Products: c_m = sum_p u_p K'[m-p] with K' read from the extended key
// [-K | K] through a 16-word sliding window (R = 8 outputs x 8 digits per
// window).  Each Torus32 product u*K is formed exactly mod 2^32 from two
// full-rate 24-bit multiply-adds: u*sext24(K) + 2^24 * u*((K + 2^23) >> 24).

constexpr int kR = 8;

struct BrPlainArgs {
    int k, n, N, ell, log2N, steps;
    const uint32_t *abar;     // [count][kn+1]
    const uint32_t *bk_ext;   // [k][n][3][ell][2N]
    const uint32_t *evk_ext;  // [k+1][ell][2N]
    uint32_t *acc_out;        // [count][(k+1)N]
};

// u * sext24(b) + c, wrapping mod 2^32: the 24-bit multiply gives the low 32
// bits of the product, and the sums are unsigned so that their intended
// wrap-around is defined.
__device__ __forceinline__ uint32_t mad24(int a, int b, uint32_t c) { return (uint32_t)__mul24(a, b) + c; }

// Accumulates the R outputs m0..m0+R-1 of sum_p u_p K'[m-p] for NK key
// polynomials that share the digit polynomial u.
template <int NK>
__device__ __forceinline__ void toeplitz_mac(const int8_t *__restrict__ U,
                                             const uint32_t *const *Kx, int N, int m0,
                                             uint32_t (&lo)[NK][kR], uint32_t (&hi)[NK][kR]) {
    for (int p0 = 0; p0 < N; p0 += 8) {
        const int base = N + m0 - p0 - 8;
        int win[NK][16], winh[NK][16];
#pragma unroll
        for (int q = 0; q < NK; ++q) {
            const uint4 *src = reinterpret_cast<const uint4 *>(Kx[q] + base);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const uint4 x = src[v];
                win[q][4 * v + 0] = (int)x.x;
                win[q][4 * v + 1] = (int)x.y;
                win[q][4 * v + 2] = (int)x.z;
                win[q][4 * v + 3] = (int)x.w;
            }
#pragma unroll
            for (int e = 0; e < 16; ++e) winh[q][e] = (int)(((uint32_t)win[q][e] + 0x800000u) >> 24);
        }
        const uint2 dd = *reinterpret_cast<const uint2 *>(U + p0);
#pragma unroll
        for (int pp = 0; pp < 8; ++pp) {
            const uint32_t word = pp < 4 ? dd.x : dd.y;
            const int u = (int)(int8_t)(word >> (8 * (pp & 3)));
#pragma unroll
            for (int q = 0; q < NK; ++q)
#pragma unroll
                for (int r = 0; r < kR; ++r) {
                    lo[q][r] = mad24(u, win[q][8 - pp + r], lo[q][r]);
                    hi[q][r] = mad24(u, winh[q][8 - pp + r], hi[q][r]);
                }
        }
    }
}

__global__ __launch_bounds__(512) void br_plain_kernel(BrPlainArgs a) {
    extern __shared__ uint32_t smem[];
    const int k = a.k, N = a.N, ell = a.ell, log2N = a.log2N;
    const int K1 = k + 1;
    uint32_t *acc = smem;                              // [k+1][N]
    uint32_t *wpart = acc + K1 * N;                    // [k+1][N]
    int8_t *dig = reinterpret_cast<int8_t *>(wpart + K1 * N);  // [k+1][ell][N]
    int8_t *vdig = dig + K1 * ell * N;                 // [ell][N]
    const int tid = threadIdx.x, T = blockDim.x;
    const size_t g = blockIdx.x;
    const uint32_t *ab = a.abar + g * (size_t)(k * a.n + 1);
    const uint32_t offset = decomp_offset(ell);

    const int b0 = (int)ab[0];
    for (int idx = tid; idx < K1 * N; idx += T) {
        uint32_t v = 0;
        if (idx < N) {
            const int s = idx + b0;
            const int src = s & (N - 1);
            const uint32_t tv = src < N / 2 ? 0xE0000000u : 0x20000000u;
            v = ((s >> log2N) & 1) ? 0u - tv : tv;
        }
        acc[idx] = v;
    }
    __syncthreads();

    const int units2 = 2 * (N / kR);
    for (int st = 0; st < a.steps; ++st) {
        const int party = st / a.n, bit = st - party * a.n;
        const int ashift = (int)ab[1 + st];
        if (ashift == 0) continue;  // X^0 ACC - ACC = 0 adds nothing
        // Slots j >= party+2 are still exactly zero (only c'_0 and c'_{1+i}
        // receive stage-2 output, and a zero slot has zero digits): skipped.
        const int live = min(K1, party + 2);
        // 1. rotate, subtract, decompose
        for (int idx = tid; idx < live * N; idx += T) {
            const int j = idx >> log2N, m = idx & (N - 1);
            const int s = m + ashift;
            const uint32_t src = acc[(j << log2N) + (s & (N - 1))];
            const uint32_t rot = ((s >> log2N) & 1) ? 0u - src : src;
            const uint32_t y = rot - acc[idx] + offset;
            for (int l = 0; l < ell; ++l)
                dig[(j * ell + l) * N + m] = (int8_t)((int)((y >> (24 - 8 * l)) & 255u) - 128);
        }
        __syncthreads();
        const uint32_t *bkbit = a.bk_ext + ((size_t)party * a.n + bit) * 3 * ell * 2 * N;
        // 2. stage 1
        for (int u = tid; u < live * (N / kR); u += T) {
            const int j = u / (N / kR), m0 = (u - j * (N / kR)) * kR;
            uint32_t lo[2][kR] = {}, hi[2][kR] = {};
            for (int l = 0; l < ell; ++l) {
                const uint32_t *Kx[2] = {bkbit + (size_t)(0 * ell + l) * 2 * N,
                                         a.evk_ext + (size_t)(j * ell + l) * 2 * N};
                toeplitz_mac<2>(dig + (j * ell + l) * N, Kx, N, m0, lo, hi);
            }
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                acc[j * N + m0 + r] += lo[0][r] + (hi[0][r] << 24);
                wpart[j * N + m0 + r] = lo[1][r] + (hi[1][r] << 24);
            }
        }
        __syncthreads();
        // 3. w = sum_j w_j, decomposed
        for (int m = tid; m < N; m += T) {
            uint32_t w = 0;
            for (int j = 0; j < live; ++j) w += wpart[j * N + m];
            const uint32_t y = w + offset;
            for (int l = 0; l < ell; ++l)
                vdig[l * N + m] = (int8_t)((int)((y >> (24 - 8 * l)) & 255u) - 128);
        }
        __syncthreads();
        // 4. stage 2
        for (int u = tid; u < units2; u += T) {
            const int o = u / (N / kR), m0 = (u - o * (N / kR)) * kR;
            uint32_t lo[1][kR] = {}, hi[1][kR] = {};
            for (int l = 0; l < ell; ++l) {
                const uint32_t *Kx[1] = {bkbit + (size_t)((1 + o) * ell + l) * 2 * N};
                toeplitz_mac<1>(vdig + l * N, Kx, N, m0, lo, hi);
            }
            uint32_t *dst = acc + (o == 0 ? 0 : (1 + party)) * N + m0;
#pragma unroll
            for (int r = 0; r < kR; ++r) dst[r] += lo[0][r] + (hi[0][r] << 24);
        }
        __syncthreads();
    }
    uint32_t *out = a.acc_out + g * (size_t)K1 * N;
    for (int idx = tid; idx < K1 * N; idx += T) out[idx] = acc[idx];
}

static int launch_br_plain(mk_ctx *ctx, const uint32_t *abar, uint32_t *acc, size_t count,
                           int steps, hipStream_t s) {
    const mk_params &P = ctx->p;
    BrPlainArgs a;
    a.k = P.k; a.n = P.n; a.N = P.N; a.ell = P.bk_ell;
    a.log2N = __builtin_ctz(P.N);
    a.steps = steps;
    a.abar = abar; a.bk_ext = ctx->dev.bk_ext; a.evk_ext = ctx->dev.evk_ext; a.acc_out = acc;
    const int K1 = P.k + 1;
    const size_t lds = (size_t)K1 * P.N * 8 + (size_t)K1 * P.bk_ell * P.N + (size_t)P.bk_ell * P.N;
    if (lds > 160 * 1024) return fail(MK_EPARAM, "plain rotation: LDS need exceeds 160 KiB");
    int threads = K1 * (P.N / kR);
    threads = std::min(512, (threads + 63) / 64 * 64);
    MK_HIP(hipFuncSetAttribute((const void *)br_plain_kernel,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
           "br_plain attribute");
    for (size_t off = 0; off < count; off += 65535) {
        const size_t c = std::min<size_t>(65535, count - off);
        BrPlainArgs b = a;
        b.abar = abar + off * (P.k * P.n + 1);
        b.acc_out = acc + off * K1 * P.N;
        StageTimer tm(ctx, 1, s);
        hipLaunchKernelGGL(br_plain_kernel, dim3((unsigned)c), dim3(threads), lds, s, b);
        MK_HIP(hipGetLastError(), "br_plain launch");
    }
    return MK_OK;
}

// -------------------------------------------- K4: extract + key switch ---
//
// One workgroup per gate.  For each party i the extracted mask
// a_i[q] = (q == 0 ? c_{1+i}[0] : -c_{1+i}[N-q]) is rounded to t base-B'
// digits (LDS), then thread r accumulates words tid + 256 r of the rows
// KS_i[q][p][v] with v != 0.  b = c_0[0] + 1/8 + the rows' b words.

constexpr int kKsThreads = 256;
constexpr int kKsWords = 4;  // words per thread: n + 1 <= 1024

struct KsArgs {
    int k, n, N, t, lb;
    const uint32_t *acc;  // [count][(k+1)N]
    const uint32_t *ks;   // [k][N][t][B'-1][n+1]
    uint32_t *out;
    size_t stride;
};

__global__ __launch_bounds__(kKsThreads) void extract_ks_kernel(KsArgs a) {
    extern __shared__ uint8_t kdig[];  // [N][t]
    const int tid = threadIdx.x;
    const size_t g = blockIdx.x;
    const int N = a.N, n = a.n, t = a.t, lb = a.lb;
    const int Bm1 = (1 << lb) - 1;
    const int prec = lb * t;
    const uint32_t *A = a.acc + g * (size_t)(a.k + 1) * N;
    uint32_t *out = a.out + g * a.stride;
    uint32_t bsum = 0;
    for (int i = 0; i < a.k; ++i) {
        const uint32_t *ci = A + (size_t)(1 + i) * N;
        for (int q = tid; q < N; q += kKsThreads) {
            const uint32_t aq = q == 0 ? ci[0] : 0u - ci[N - q];
            const uint32_t r = (aq + (1u << (31 - prec))) >> (32 - prec);
            for (int p = 0; p < t; ++p) kdig[q * t + p] = (uint8_t)((r >> (lb * (t - 1 - p))) & Bm1);
        }
        __syncthreads();
        uint32_t accw[kKsWords] = {};
        const uint32_t *base = a.ks + (size_t)i * N * t * Bm1 * (n + 1);
        for (int qp = 0; qp < N * t; ++qp) {
            const int v = kdig[qp];
            if (v == 0) continue;
            const uint32_t *row = base + ((size_t)qp * Bm1 + (v - 1)) * (n + 1);
#pragma unroll
            for (int r = 0; r < kKsWords; ++r) {
                const int w = tid + kKsThreads * r;
                if (w <= n) accw[r] += row[w];
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kKsWords; ++r) {
            const int w = tid + kKsThreads * r;
            if (w == 0) bsum += accw[r];
            else if (w <= n) out[1 + (size_t)i * n + (w - 1)] = accw[r];
        }
    }
    if (tid == 0) out[0] = A[0] + 0x20000000u + bsum;
}

int launch_extract_ks(mk_ctx *ctx, const uint32_t *acc, uint32_t *out, size_t count,
                             size_t stride, hipStream_t s) {
    const mk_params &P = ctx->p;
    KsArgs a;
    a.k = P.k; a.n = P.n; a.N = P.N; a.t = P.ks_t; a.lb = P.ks_log_base;
    a.ks = ctx->dev.ks; a.stride = stride;
    const size_t lds = (size_t)P.N * P.ks_t;
    MK_HIP(hipFuncSetAttribute((const void *)extract_ks_kernel,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
           "extract_ks attribute");
    for (size_t off = 0; off < count; off += 65535) {
        const size_t c = std::min<size_t>(65535, count - off);
        KsArgs b = a;
        b.acc = acc + off * (P.k + 1) * P.N;
        b.out = out + off * stride;
        StageTimer tm(ctx, 2, s);
        hipLaunchKernelGGL(extract_ks_kernel, dim3((unsigned)c), dim3(kKsThreads), lds, s, b);
        MK_HIP(hipGetLastError(), "extract_ks launch");
    }
    return MK_OK;
}

// ----------------------------------------------------------- pipeline ---

int run_blind_rotate(mk_ctx *ctx, const uint32_t *abar, uint32_t *acc, size_t count,
                     int steps, int path, hipStream_t s) {
    if (path == MK_PATH_I32) return launch_br_plain(ctx, abar, acc, count, steps, s);
    if (path == MK_PATH_MFMA_I8) return launch_br_mfma(ctx, abar, acc, count, steps, s);
    return fail(MK_EINVAL, "unknown path");
}

int run_key_switch(mk_ctx *ctx, const uint32_t *acc, uint32_t *out, size_t count, size_t stride, int path,
                   hipStream_t s) {
    if (path == MK_PATH_I32) return launch_extract_ks(ctx, acc, out, count, stride, s);
    if (path == MK_PATH_MFMA_I8)
        return ctx->dev.ks_win ? launch_ks_mfma(ctx, acc, out, count, stride, s)
                               : launch_extract_ks(ctx, acc, out, count, stride, s);
    return fail(MK_EINVAL, "unknown path");
}

int run_rotate_ks(mk_ctx *ctx, const uint32_t *abar, uint32_t *acc, uint32_t *out, size_t count, size_t stride,
                  int path, hipStream_t s) {
    const mk_params &P = ctx->p;
    const int steps = P.k * P.n;
    int rc;
    if (path != MK_PATH_MFMA_I8) {
        if ((rc = run_blind_rotate(ctx, abar, acc, count, steps, path, s))) return rc;
        return run_key_switch(ctx, acc, out, count, stride, path, s);
    }
    // one or two consecutive launches (mfma_rotation_split)
    const size_t first = mfma_rotation_split(ctx, count);
    for (size_t off = 0; off < count;) {
        const size_t n = off ? count - off : first;
        const uint32_t *ab = abar + off * lwe_words(P);
        uint32_t *ac = acc + off * (size_t)(P.k + 1) * P.N, *o = out + off * stride;
        bool done = false;
        if ((rc = launch_br_mfma(ctx, ab, ac, n, steps, s, o, stride, &done))) return rc;
        if (!done && (rc = run_key_switch(ctx, ac, o, n, stride, path, s))) return rc;
        off += n;
    }
    return MK_OK;
}

// Gates per rotation launch: larger batches (and wide circuit levels) run in
// chunks, which bounds the scratch memory and keeps the MFMA path's 32-bit
// digit offsets, K1 ell GP N < 2^31, in range.
size_t rotation_chunk(const mk_params &P) {
    const size_t lim = (((size_t)1 << 31) - 1) / ((size_t)(P.k + 1) * P.bk_ell * P.N) / 32 * 32;
    return std::max<size_t>(32, std::min<size_t>(lim, 65536));
}

int run_gates(mk_ctx *ctx, const uint8_t *types, const uint32_t *in1, const uint32_t *in2,
              uint32_t *out, size_t count, size_t stride, int path, hipStream_t s) {
    const mk_params &P = ctx->p;
    const size_t words = lwe_words(P);
    const size_t chunk = std::min(count, rotation_chunk(P));
    const size_t abar_bytes = (chunk * words * 4 + 255) / 256 * 256;
    const size_t acc_bytes = chunk * (P.k + 1) * P.N * 4;
    int rc = ensure_scratch(ctx, abar_bytes + acc_bytes);
    if (rc) return rc;
    uint32_t *abar = (uint32_t *)ctx->dev.scratch;
    uint32_t *acc = (uint32_t *)((char *)ctx->dev.scratch + abar_bytes);
    const int log2_2N = __builtin_ctz(2 * P.N);
    for (size_t c0 = 0; c0 < count; c0 += chunk) {
        const size_t cnt = std::min(chunk, count - c0), total = cnt * words;
        {
            StageTimer tm(ctx, 0, s);
            hipLaunchKernelGGL(precombine_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                               types + c0, in1 + c0 * stride, in2 + c0 * stride, stride, (int)words, log2_2N,
                               total, abar, ctx->dev.status);
        }
        MK_HIP(hipGetLastError(), "precombine launch");
        if ((rc = run_rotate_ks(ctx, abar, acc, out + c0 * stride, cnt, stride, path, s))) return rc;
    }
    return MK_OK;
}

}  // namespace mk

using namespace mk;

extern "C" {

int mk_upload_eval_key(mk_ctx *ctx, void *stream) {
    if (!ctx) return fail(MK_EINVAL, "mk_upload_eval_key: null context");
    return device_upload(ctx, stream);
}

int mk_set_profiling(mk_ctx *ctx, int level) {
    if (!ctx || level < 0 || level > 2) return fail(MK_EINVAL, "mk_set_profiling: bad argument");
    ctx->dev.profiling = level;
    return MK_OK;
}

int mk_get_profile(mk_ctx *ctx, double *ms, int64_t *launches, int reset) {
    if (!ctx) return fail(MK_EINVAL, "mk_get_profile: null context");
    drain_events(ctx);
    for (int st = 0; st < MK_PROFILE_SLOTS; ++st) {
        if (ms) ms[st] = ctx->dev.prof_ms[st];
        if (launches) launches[st] = ctx->dev.prof_launches[st];
        if (reset) {
            ctx->dev.prof_ms[st] = 0;
            ctx->dev.prof_launches[st] = 0;
        }
    }
    return MK_OK;
}

int mk_not(const mk_ctx *ctx, const uint32_t *in_dev, uint32_t *out_dev, size_t count,
           size_t stride, void *stream) {
    if (!ctx || (count && (!in_dev || !out_dev))) return fail(MK_EINVAL, "mk_not: null argument");
    const size_t words = lwe_words(ctx->p);
    if (stride < words) return fail(MK_EINVAL, "mk_not: stride < kn+1");
    if (!count) return MK_OK;
    const size_t total = count * words;
    hipLaunchKernelGGL(not_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, in_dev, out_dev, stride, (int)words, total);
    MK_HIP(hipGetLastError(), "not launch");
    return MK_OK;
}

int mk_bootstrap_gate(mk_ctx *ctx, const uint8_t *types, const uint32_t *in1,
                      const uint32_t *in2, uint32_t *out, size_t count, size_t stride,
                      int path, void *stream) {
    if (!ctx) return fail(MK_EINVAL, "mk_bootstrap_gate: null context");
    if (count && (!types || !in1 || !in2 || !out)) return fail(MK_EINVAL, "mk_bootstrap_gate: null pointer");
    if (stride < lwe_words(ctx->p)) return fail(MK_EINVAL, "mk_bootstrap_gate: stride < kn+1");
    if (path != MK_PATH_I32 && path != MK_PATH_MFMA_I8) return fail(MK_EINVAL, "mk_bootstrap_gate: bad path");
    int rc = check_uploaded(ctx);
    if (rc) return rc;
    if (!count) return MK_OK;
    return run_gates(ctx, types, in1, in2, out, count, stride, path, (hipStream_t)stream);
}

int mk_blind_rotate(mk_ctx *ctx, const uint32_t *abar_dev, uint32_t *acc_dev, size_t count,
                    int max_steps, int path, void *stream) {
    if (!ctx || (count && (!abar_dev || !acc_dev))) return fail(MK_EINVAL, "mk_blind_rotate: null argument");
    int rc = check_uploaded(ctx);
    if (rc) return rc;
    if (!count) return MK_OK;
    const int total = ctx->p.k * ctx->p.n;
    const int steps = (max_steps < 0 || max_steps > total) ? total : max_steps;
    return run_blind_rotate(ctx, abar_dev, acc_dev, count, steps, path, (hipStream_t)stream);
}

int mk_extract_keyswitch(mk_ctx *ctx, const uint32_t *acc_dev, uint32_t *out_dev, size_t count,
                         size_t stride, int path, void *stream) {
    if (!ctx || (count && (!acc_dev || !out_dev))) return fail(MK_EINVAL, "mk_extract_keyswitch: null argument");
    if (stride < lwe_words(ctx->p)) return fail(MK_EINVAL, "mk_extract_keyswitch: stride < kn+1");
    int rc = check_uploaded(ctx);
    if (rc) return rc;
    if (!count) return MK_OK;
    return run_key_switch(ctx, acc_dev, out_dev, count, stride, path, (hipStream_t)stream);
}

}  // extern "C"
