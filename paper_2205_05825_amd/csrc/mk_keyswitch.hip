// Key switching on the int8-MFMA path (§3.2 MKKeySwitch) as one exact
// integer GEMM per party.
//
// For party i the switched coefficients are
//     out_i[c] = sum_{q < N} sum_{p < t} KS_i[q][p][v_qp][c],   c = 0..n,
// where v_qp is digit p (most significant first, base 2^lb) of the rounded
// coefficient a_{i,q} of the extracted sample and KS_i[q][p][0] = 0.  With
// the one-hot code e[(q,p,v)][g] = [v_qp(g) = v] of gate g this is the
// product out_i = KS_i^T e over the index K = (q, p, v): an int8 x int8 ->
// int32 contraction once the Torus32 key entries are split into four signed
// limbs (as in the blind rotation), exact since |sum| <= N t 128 < 2^31.
// The one-hot operand never touches memory: each lane forms its 16 bytes
// from the rounded coefficient in registers.
//
// K-block kb (32 K values) covers coefficient q = kb / KBq, KBq =
// ceil(t 2^lb / 32) blocks per coefficient; its byte beta = 32 (kb % KBq) +
// j is (p, v) = (beta >> lb, beta & (2^lb - 1)).  Layouts:
//   tiles  i8  [k][CT][4 limbs][N KBq][64 lanes][16]   A fragments of
//              v_mfma_i32_32x32x32_i8: lane l holds output column
//              32 ct + l % 32 and the K bytes 16 (l / 32) .. + 15
//   R      u32 [k][N][GP]   rounded coefficients (lb t bits), gate fastest
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mk_device_common.h"

namespace mk {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

#define MK_HIP(call, what)                               \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

constexpr int kKsTile = 1024;      // bytes of one 32x32 int8 fragment
constexpr int kKsMR = 3;           // output column tiles per workgroup
constexpr int kKsRing = 8;         // K-blocks in flight per wave
constexpr uint32_t kKsWord3 = 0x00020000u;   // raw dword buffer
constexpr uint32_t kKsOut = 0x80000000u;     // offset beyond every block

struct KsShape {
    int k, N, n, t, lb, CT, KBq, GP;
};

static KsShape ks_shape(const mk_params &P, size_t GP) {
    KsShape s;
    s.k = P.k; s.N = P.N; s.n = P.n; s.t = P.ks_t; s.lb = P.ks_log_base;
    s.CT = (P.n + 1 + 31) / 32;
    s.KBq = (P.ks_t * (1 << P.ks_log_base) + 31) / 32;
    s.GP = (int)GP;
    return s;
}

// One thread per (party, column tile, limb, K-block, lane): 16 key bytes.
__global__ void ks_tiles_kernel(const uint32_t *__restrict__ ks, KsShape s, int8_t *__restrict__ out) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t KB = (size_t)s.N * s.KBq;
    const size_t total = (size_t)s.k * s.CT * 4 * KB * 64;
    if (idx >= total) return;
    const int lane = (int)(idx % 64);
    const size_t kb = (idx / 64) % KB;
    const int limb = (int)((idx / (64 * KB)) % 4);
    const int ct = (int)((idx / (64 * KB * 4)) % s.CT);
    const int i = (int)(idx / (64 * KB * 4 * s.CT));
    const int q = (int)(kb / s.KBq), sub = (int)(kb % s.KBq);
    const int c = ct * 32 + lane % 32, h = lane / 32;
    const int Bm1 = (1 << s.lb) - 1;
    const uint32_t *base = ks + (size_t)i * s.N * s.t * Bm1 * (s.n + 1);
    uint32_t w[4] = {0, 0, 0, 0};
    for (int b = 0; b < 16; ++b) {
        const int beta = 32 * sub + 16 * h + b;
        const int p = beta >> s.lb, v = beta & Bm1;
        uint32_t x = 0;
        if (p < s.t && v != 0 && c <= s.n)
            x = base[(((size_t)q * s.t + p) * Bm1 + (v - 1)) * (s.n + 1) + c];
        const uint32_t byte = (((x + 0x80808080u) >> (8 * limb)) & 255u) - 128u;  // signed limb
        w[b / 4] |= (byte & 255u) << (8 * (b % 4));
    }
    reinterpret_cast<uint4 *>(out)[idx] = make_uint4(w[0], w[1], w[2], w[3]);
}

int ks_mfma_upload(mk_ctx *ctx, hipStream_t s) {
    const mk_params &P = ctx->p;
    DeviceKeys &D = ctx->dev;
    const KsShape sh = ks_shape(P, 0);
    const size_t KB = (size_t)P.N * sh.KBq;
    const size_t per_party = (size_t)sh.CT * 4 * KB * kKsTile;
    // a party's tiles are addressed with 32-bit offsets; parameter sets
    // beyond that keep the int32 key switch on both paths (same result)
    if (per_party >= ((size_t)1 << 31)) return MK_OK;
    D.ks_win_bytes = (size_t)P.k * per_party;
    if (hipMalloc((void **)&D.ks_win, D.ks_win_bytes) != hipSuccess) {
        D.ks_win = nullptr;
        return fail(MK_ENOMEM, "device allocation failed: MFMA key-switching tiles");
    }
    const size_t threads = D.ks_win_bytes / 16;
    hipLaunchKernelGGL(ks_tiles_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, D.ks, sh,
                       D.ks_win);
    MK_HIP(hipGetLastError(), "key-switching tiles launch");
    return MK_OK;
}

// Sample extraction and rounding: R[i][q][g] = round(a_{i,q}) to lb t bits,
// a_{i,0} = c_{1+i}[0], a_{i,q} = -c_{1+i}[N-q]; out[g][0] = c_0[0] + 1/8
// (party blocks of q-chunk 0 of party 0 write it).  Block: 32 gates x 64
// coefficients of one party, transposed through LDS so that both the reads
// (along q) and the writes (along g) are coalesced.
__global__ __launch_bounds__(256) void ks_round_kernel(const uint32_t *__restrict__ acc, KsShape s,
                                                       size_t count, uint32_t *__restrict__ R,
                                                       uint32_t *__restrict__ out, size_t stride) {
    __shared__ uint32_t tile[32][65];
    const int i = blockIdx.z, q0 = blockIdx.y * 64, gt = blockIdx.x;
    const int tid = threadIdx.x, K1 = s.k + 1, N = s.N;
    const int prec = s.lb * s.t;
    {
        const int ql = tid % 64, grp = tid / 64;
        const int q = q0 + ql;
        for (int j = 0; j < 8; ++j) {
            const int gl = grp * 8 + j;
            const size_t g = (size_t)gt * 32 + gl;
            uint32_t r = 0;
            if (g < count && q < N) {
                const uint32_t *ci = acc + (g * K1 + 1 + i) * (size_t)N;
                const uint32_t a = q == 0 ? ci[0] : 0u - ci[N - q];
                r = (a + (1u << (31 - prec))) >> (32 - prec);
            }
            tile[gl][ql] = r;
        }
    }
    __syncthreads();
    {
        const int gl = tid % 32, qs = tid / 32;
        for (int j = 0; j < 8; ++j) {
            const int ql = qs + 8 * j, q = q0 + ql;
            if (q < N) R[((size_t)i * N + q) * s.GP + (size_t)gt * 32 + gl] = tile[gl][ql];
        }
    }
    if (i == 0 && blockIdx.y == 0 && tid < 32) {
        const size_t g = (size_t)gt * 32 + tid;
        if (g < count) out[g * stride] = acc[g * K1 * (size_t)N] + 0x20000000u;
    }
}

// One-hot B fragment of K-block (q, sub) for the lane's gate: bytes
// beta = 32 sub + 16 h + j, set where v = digit p of r.  LB2: base-4
// digits, one digit per 32-bit word.
template <bool LB2>
__device__ __forceinline__ v4i one_hot(uint32_t r, int t, int lb, int sub, int h) {
    v4i w;
    if constexpr (LB2) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int p = 8 * sub + 4 * h + j;
            const uint32_t d = p < t ? (r >> (2 * (t - 1 - p))) & 3u : 0u;
            w[j] = p < t ? (int)(1u << (8 * d)) : 0;
        }
    } else {
        const int mask = (1 << lb) - 1;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            uint32_t word = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int beta = 32 * sub + 16 * h + 4 * j + b;
                const int p = beta >> lb, v = beta & mask;
                if (p < t && (int)((r >> (lb * (t - 1 - p))) & (uint32_t)mask) == v) word |= 1u << (8 * b);
            }
            w[j] = (int)word;
        }
    }
    return w;
}

// Workgroup (party i, kKsMR column tiles, one gate tile); wave = key limb.
// Per K-block a wave loads kKsMR key tiles of its limb and one rounded
// coefficient per lane, forms the one-hot digits and issues kKsMR MFMAs;
// kKsRing K-blocks are in flight (ring slot kb mod kKsRing, the loop
// unrolled kKsRing times).  The four limb sums are combined through LDS,
// sum_t 2^(8t) S_t, and stored: column 0 is added atomically to out[g][0]
// (one addition per party, exact mod 2^32 in any order), columns 1..n go
// to out[g][1 + i n + c - 1].
//
// Tasks (party, column block, gate tile) are numbered with the gate tile
// fastest, and each XCD runs one contiguous range of them: workgroup b
// runs on XCD b mod nx (round-robin dispatch), so task = (b mod nx) per +
// b / nx.  A column block's key tiles (12 MB at the Table 7 shape) are then
// fetched by at most two XCDs' L2s, instead of by every XCD.
template <bool LB2>
__global__ __launch_bounds__(256, 2) void ks_gemm_kernel(const int8_t *__restrict__ tiles,
                                                         const uint32_t *__restrict__ R, KsShape s,
                                                         size_t count, uint32_t *__restrict__ out,
                                                         size_t stride, int nx, int per) {
    __shared__ __align__(16) uint4 red[2 * 4 * 4 * 64];
    const int GT = s.GP / 32, CB = (s.CT + kKsMR - 1) / kKsMR;
    int task = (int)(blockIdx.x % (unsigned)nx) * per + (int)(blockIdx.x / (unsigned)nx);
    if (task >= s.k * CB * GT) return;
    const int gt = task % GT;
    task /= GT;
    const int cb = task % CB, i = task / CB;
    const int lane = threadIdx.x & 63, h = lane >> 5, gl = lane & 31;
    const int limb = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
    const int KB = s.N * s.KBq;
    const int ct0 = cb * kKsMR;
    const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(tiles + (size_t)i * s.CT * 4 * KB * kKsTile), (short)0, s.CT * 4 * KB * kKsTile, kKsWord3);
    const __amdgpu_buffer_rsrc_t rr = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(R + (size_t)i * s.N * s.GP), (short)0, s.N * s.GP * 4, kKsWord3);
    uint32_t a_uni[kKsMR];  // byte offset of K-block 0 of each column tile
#pragma unroll
    for (int m = 0; m < kKsMR; ++m)
        a_uni[m] = ct0 + m < s.CT ? (uint32_t)(((ct0 + m) * 4 + limb) * KB) * kKsTile : kKsOut;
    const uint32_t lane16 = (uint32_t)lane * 16, r_lane = (uint32_t)(gt * 32 + gl) * 4;
    // loads past the last K-block read either unused in-range tiles or
    // out-of-range zeros; they are never multiplied
    auto ldA = [&](int m, int x) {
        return (v4i)__builtin_amdgcn_raw_buffer_load_b128(ra, a_uni[m] + (uint32_t)x * kKsTile + lane16, 0, 0);
    };
    auto ldR = [&](int q) {
        return (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rr, (uint32_t)q * (uint32_t)s.GP * 4 + r_lane, 0, 0);
    };
    v16i acc[kKsMR];
#pragma unroll
    for (int m = 0; m < kKsMR; ++m) acc[m] = v16i{};
    v4i sa[kKsRing][kKsMR];
    uint32_t sr[kKsRing];
    int lq = 0, lsub = 0;  // (q, sub) of the next K-block to load
    auto advance = [&](int &q, int &sub) {
        const int wrap = sub + 1 == s.KBq;
        sub = wrap ? 0 : sub + 1;
        q += wrap;
    };
#pragma unroll
    for (int x = 0; x < kKsRing; ++x) {
#pragma unroll
        for (int m = 0; m < kKsMR; ++m) sa[x][m] = ldA(m, x);
        sr[x] = ldR(lq);
        advance(lq, lsub);
        __builtin_amdgcn_sched_barrier(0);
    }
    int msub = 0;  // sub-block of the K-block being multiplied
    for (int kb0 = 0; kb0 < KB; kb0 += kKsRing) {  // KB is a multiple of kKsRing
#pragma unroll
        for (int u = 0; u < kKsRing; ++u) {
            const v4i b = one_hot<LB2>(sr[u], s.t, s.lb, msub, h);
            msub = msub + 1 == s.KBq ? 0 : msub + 1;
#pragma unroll
            for (int m = 0; m < kKsMR; ++m)
                acc[m] = __builtin_amdgcn_mfma_i32_32x32x32_i8(sa[u][m], b, acc[m], 0, 0, 0);
#pragma unroll
            for (int m = 0; m < kKsMR; ++m) sa[u][m] = ldA(m, kb0 + u + kKsRing);
            sr[u] = ldR(lq);
            advance(lq, lsub);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    // limb combination: tile m through buffer m % 2 ([4 limbs][4 quads][64])
    const size_t g = (size_t)gt * 32 + gl;
    const uint32_t sh = 8u * (uint32_t)limb;
#pragma unroll
    for (int m = 0; m < kKsMR; ++m) {
        uint4 *buf = red + (m & 1) * 4 * 4 * 64;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            buf[(limb * 4 + q) * 64 + lane] =
                make_uint4((uint32_t)acc[m][4 * q + 0] << sh, (uint32_t)acc[m][4 * q + 1] << sh,
                           (uint32_t)acc[m][4 * q + 2] << sh, (uint32_t)acc[m][4 * q + 3] << sh);
        __syncthreads();
        uint4 sum = buf[limb * 64 + lane];
#pragma unroll
        for (int x = 1; x < 4; ++x) {
            const uint4 v = buf[(x * 4 + limb) * 64 + lane];
            sum.x += v.x;
            sum.y += v.y;
            sum.z += v.z;
            sum.w += v.w;
        }
        // registers 4 limb .. 4 limb + 3: columns 32 ct + 8 limb + 4 h + e
        if (g < count) {
            const int c0 = (ct0 + m) * 32 + 8 * limb + 4 * h;
            const uint32_t vals[4] = {sum.x, sum.y, sum.z, sum.w};
            uint32_t *row = out + g * stride;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int c = c0 + e;
                if (c == 0) atomicAdd(row, vals[e]);
                else if (c <= s.n) row[(size_t)i * s.n + c] = vals[e];
            }
        }
    }
}

size_t ks_scratch_need(const mk_params &P, size_t count) {
    return (size_t)P.k * P.N * ((count + 31) / 32 * 32) * 4;
}

int launch_ks_mfma(mk_ctx *ctx, const uint32_t *acc, uint32_t *out, size_t count, size_t stride,
                   hipStream_t s) {
    const mk_params &P = ctx->p;
    DeviceKeys &D = ctx->dev;
    const size_t GP = (count + 31) / 32 * 32;
    const KsShape sh = ks_shape(P, GP);
    if (P.N < kKsRing || (size_t)P.N * GP * 4 >= ((size_t)1 << 31))
        return fail(MK_EINVAL, "int8-MFMA key switching: batch too large for one launch (split it)");
    const size_t need = ks_scratch_need(P, count);
    if (D.ks_scratch_bytes < need) {
        if (D.fixed_scratch) return fail(MK_EINTERNAL, "fixed scratch block too small (key switching)");
        if (D.ks_scratch) {
            MK_HIP(hipStreamSynchronize(s), "ks scratch sync");
            (void)hipFree(D.ks_scratch);
            D.ks_scratch = nullptr;
            D.ks_scratch_bytes = 0;
        }
        if (hipMalloc(&D.ks_scratch, need) != hipSuccess) {
            D.ks_scratch = nullptr;
            return fail(MK_ENOMEM, "device allocation failed: key-switching scratch");
        }
        D.ks_scratch_bytes = need;
    }
    uint32_t *R = (uint32_t *)D.ks_scratch;
    const int GT = (int)(GP / 32), CB = (sh.CT + kKsMR - 1) / kKsMR;
    StageTimer tm(ctx, 2, s);
    hipLaunchKernelGGL(ks_round_kernel, dim3((unsigned)GT, (unsigned)((P.N + 63) / 64), (unsigned)P.k),
                       dim3(256), 0, s, acc, sh, count, R, out, stride);
    MK_HIP(hipGetLastError(), "key-switching round launch");
    const int tasks = P.k * CB * GT, nx = std::max(1, D.num_xcd), per = (tasks + nx - 1) / nx;
    const unsigned blocks = (unsigned)(nx * per);
    if (P.ks_log_base == 2)
        hipLaunchKernelGGL(ks_gemm_kernel<true>, dim3(blocks), dim3(256), 0, s, D.ks_win, R, sh, count, out,
                           stride, nx, per);
    else
        hipLaunchKernelGGL(ks_gemm_kernel<false>, dim3(blocks), dim3(256), 0, s, D.ks_win, R, sh, count, out,
                           stride, nx, per);
    MK_HIP(hipGetLastError(), "key-switching GEMM launch");
    return MK_OK;
}

}  // namespace mk
