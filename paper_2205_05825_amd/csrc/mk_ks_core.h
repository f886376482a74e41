// Device building blocks of the int8-MFMA key switching (§3.2
// MKKeySwitch), shared by its own kernels (mk_keyswitch.hip) and by the
// persistent rotation, which can run it on each tile as soon as that tile's
// rotation is done (mk_persist.hip).
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
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mk {

typedef int ks_v4i __attribute__((ext_vector_type(4)));
typedef int ks_v16i __attribute__((ext_vector_type(16)));

constexpr int kKsTile = 1024;      // bytes of one 32x32 int8 fragment
constexpr int kKsMR = 3;           // output column tiles per task
constexpr int kKsRing = 8;         // K-blocks in flight per wave
constexpr uint32_t kKsWord3 = 0x00020000u;   // raw dword buffer
constexpr uint32_t kKsOut = 0x80000000u;     // offset beyond every block
constexpr int kKsRoundLds = 32 * 65 * 4;     // bytes of ks_round_unit's LDS tile
constexpr int kKsGemmLds = 2 * 4 * 4 * 64 * 16;  // bytes of ks_gemm_task's LDS

struct KsShape {
    int k, N, n, t, lb, CT, KBq, GP;
};

// Key switching that the persistent rotation runs on each of its tiles once
// the tile's last CMux step is done (tiles == nullptr: not fused).
struct KsFused {
    const int8_t *tiles;   // key tiles (layout above)
    uint32_t *R;           // rounded coefficients, [k][N][GP]
    uint32_t *out;         // output ciphertexts, `stride` words per gate
    size_t stride, count;
    KsShape s;
};

// Column blocks of kKsMR column tiles.
__host__ __device__ inline int ks_col_blocks(const KsShape &s) { return (s.CT + kKsMR - 1) / kKsMR; }

// Extraction and rounding of one unit (gate tile gt, coefficients q0 ..
// q0 + 63, party i) by 256 threads: R[i][q][g] = round(a_{i,q}) to lb t
// bits, with a_{i,0} = c_{1+i}[0] and a_{i,q} = -c_{1+i}[N-q]; the unit of
// party 0 at q0 = 0 also writes out[g][0] = c_0[0] + 1/8.  The 32 x 64 block
// is transposed through LDS (`tile`, kKsRoundLds bytes) so that both the
// reads (along q) and the writes (along g) are coalesced.  COH: the
// accumulator was written by other compute units in the same launch, so its
// words are read with device-scope loads (they bypass the unit's L1).
template <bool COH>
__device__ __forceinline__ void ks_round_unit(const uint32_t *__restrict__ acc, const KsShape &s, size_t count,
                                              uint32_t *__restrict__ R, uint32_t *__restrict__ out, size_t stride,
                                              int gt, int q0, int i, uint32_t *tile) {
    const int tid = threadIdx.x, K1 = s.k + 1, N = s.N;
    const int prec = s.lb * s.t;
    auto ld = [&](const uint32_t *p) -> uint32_t {
        if constexpr (COH) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else return *p;
    };
    {
        const int ql = tid % 64, grp = tid / 64;
        const int q = q0 + ql;
        for (int j = 0; j < 8; ++j) {
            const int gl = grp * 8 + j;
            const size_t g = (size_t)gt * 32 + gl;
            uint32_t r = 0;
            if (g < count && q < N) {
                const uint32_t *ci = acc + (g * K1 + 1 + i) * (size_t)N;
                const uint32_t a = q == 0 ? ld(ci) : 0u - ld(ci + (N - q));
                r = (a + (1u << (31 - prec))) >> (32 - prec);
            }
            tile[gl * 65 + ql] = r;
        }
    }
    __syncthreads();
    {
        const int gl = tid % 32, qs = tid / 32;
        for (int j = 0; j < 8; ++j) {
            const int ql = qs + 8 * j, q = q0 + ql;
            if (q < N) R[((size_t)i * N + q) * s.GP + (size_t)gt * 32 + gl] = tile[gl * 65 + ql];
        }
    }
    if (i == 0 && q0 == 0 && tid < 32) {
        const size_t g = (size_t)gt * 32 + tid;
        if (g < count) {
            const uint32_t b = ld(acc + g * K1 * (size_t)N) + 0x20000000u;
            // in the same launch the GEMM tasks add to this word with
            // device-scope atomics, so it is written at that scope too
            if constexpr (COH) __hip_atomic_store(out + g * stride, b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else out[g * stride] = b;
        }
    }
    __syncthreads();   // `tile` is reused by the next unit
}

// One-hot B fragment of K-block (q, sub) for the lane's gate: bytes
// beta = 32 sub + 16 h + j, set where v = digit p of r.  LB2: base-4
// digits, one digit per 32-bit word.
template <bool LB2>
__device__ __forceinline__ ks_v4i one_hot(uint32_t r, int t, int lb, int sub, int h) {
    ks_v4i w;
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

// Task (party i, column block cb, gate tile gt) by 256 threads; wave = key
// limb.  Per K-block a wave loads kKsMR key tiles of its limb and one
// rounded coefficient per lane, forms the one-hot digits and issues kKsMR
// MFMAs; kKsRing K-blocks are in flight (ring slot kb mod kKsRing, the loop
// unrolled kKsRing times).  The four limb sums are combined through LDS
// (`red`, kKsGemmLds bytes), sum_t 2^(8t) S_t, and stored: column 0 is
// added atomically to out[g][0] (one addition per party, exact mod 2^32 in
// any order), columns 1..n go to out[g][1 + i n + c - 1].  RAUX: cache
// policy of the loads of R (device scope when other compute units wrote it
// in the same launch).
template <bool LB2, int RAUX>
__device__ __forceinline__ void ks_gemm_task(const int8_t *__restrict__ tiles, const uint32_t *__restrict__ R,
                                             const KsShape &s, size_t count, uint32_t *__restrict__ out,
                                             size_t stride, int gt, int cb, int i, uint4 *red) {
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
        return (ks_v4i)__builtin_amdgcn_raw_buffer_load_b128(ra, a_uni[m] + (uint32_t)x * kKsTile + lane16, 0, 0);
    };
    auto ldR = [&](int q) {
        return (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rr, (uint32_t)q * (uint32_t)s.GP * 4 + r_lane, 0,
                                                              RAUX);
    };
    ks_v16i acc[kKsMR];
#pragma unroll
    for (int m = 0; m < kKsMR; ++m) acc[m] = ks_v16i{};
    ks_v4i sa[kKsRing][kKsMR];
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
            const ks_v4i b = one_hot<LB2>(sr[u], s.t, s.lb, msub, h);
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
    __syncthreads();   // `red` is reused by the next task
}

}  // namespace mk
