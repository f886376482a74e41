// Int8-MFMA blind rotation (K3) for gfx950.
//
// Every negacyclic product of a blind-rotation step is an exact integer
// contraction  c_m = sum_p K'[m-p] u_p  (mod 2^32), where u are signed int8
// gadget digits and K' is the key polynomial extended negacyclically
// (K'[s] = K[s] for s >= 0, -K[s+N] for s < 0).  Each Torus32 entry K'[s] is
// split into four signed 8-bit limbs, K'[s] = sum_t 2^(8t) L_t(K'[s]) mod 2^32
// with L_t(x) = byte_t(x + 0x80808080) - 128, so
//     c_m = sum_t 2^(8t) sum_p L_t(K'[m-p]) u_p   (mod 2^32)
// and each inner sum is an int8 x int8 -> int32 matrix product, exact because
// |sum| <= (k+1) * ell * N * 2^14 < 2^31 (checked at setup).
//
// Batched over G gates the products of one CMux step are GEMMs whose A
// operand is a key Toeplitz matrix shared by all gates and whose B operand
// holds the gates' digits (one column per gate).  A 32x32 tile of a Toeplitz
// matrix at block row mb and block column kb only depends on d = mb - kb, so
// the 2N/32 - 1 distinct tiles of every (key polynomial, limb) are stored
// once, in the exact register layout of v_mfma_i32_32x32x32_i8 (lane l holds
// row l%32 and the 16 K-values 16*(l/32)..+15), and loaded with one
// coalesced 16-byte read per lane.
//
// Per CMux step (party i, bit l) four kernels run:
//   rotdec : P_j = X^-a ACC_j - ACC_j per gate, decomposed into ell int8
//            digit polynomials stored as MFMA B fragments.
//   gemm1  : for every (unit, 64-row block, 32-gate tile): unit c'_j adds
//            sum_l T(d_l) U_{j,l} into ACC_j; unit w_j writes the partial
//            sum_l T(b_{j,l}) U_{j,l} to W_j.
//   wdec   : V = g^-1(sum_j W_j) as B fragments.
//   gemm2  : ACC_0 += sum_l T(f0_l) V_l ;  ACC_{1+i} += sum_l T(f1_l) V_l.
// Layouts (GP = gates padded to 32, GT = GP/32, NB = N/32, ND = 2 NB - 1):
//   acc  u32 [GP][k+1][N]                 W  u32 [k+1][GP][N]
//   U    i8  [k+1][ell][GT][NB][64][16]    V  i8  [ell][GT][NB][64][16]
//   bk   i8  [k][n][3][ell][4][ND][64][16]
//   evk  i8  [k+1][ell][4][ND][64][16]
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mk_device_common.h"

namespace mk {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kTileBytes = 1024;  // one 32x32 int8 fragment (64 lanes x 16 B)

#define MK_HIP(call, what)                               \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// ------------------------------------------------------------ upload ----

// Writes the ND diagonal tiles of 4 limbs for `npoly` polynomials given in
// extended form ext[poly][2N] = [-K | K].  One thread per (poly, limb, diag,
// lane) writes 16 bytes.
__global__ void diag_tiles_kernel(const uint32_t *__restrict__ ext, int N, size_t npoly,
                                  int8_t *__restrict__ out) {
    const int NB = N / 32, ND = 2 * NB - 1;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t total = npoly * 4 * ND * 64;
    if (idx >= total) return;
    const int lane = (int)(idx % 64);
    const int d = (int)((idx / 64) % ND);
    const int t = (int)((idx / (64 * ND)) % 4);
    const size_t poly = idx / (64 * (size_t)ND * 4);
    const uint32_t *e = ext + poly * 2 * N;
    const int i = lane % 32, h = lane / 32;
    uint32_t w[4] = {0, 0, 0, 0};
    for (int b = 0; b < 16; ++b) {
        const int s = 32 * (d - (NB - 1)) + i - (16 * h + b);   // in [-(N-1), N-1]
        const uint32_t x = e[N + s] + 0x80808080u;
        const uint32_t limb = ((x >> (8 * t)) & 255u) - 128u;   // int8 as byte
        w[b / 4] |= (limb & 255u) << (8 * (b % 4));
    }
    reinterpret_cast<uint4 *>(out)[idx] = make_uint4(w[0], w[1], w[2], w[3]);
}

int mfma_upload(mk_ctx *ctx, const std::vector<uint32_t> &evk, hipStream_t s) {
    (void)evk;
    const mk_params &P = ctx->p;
    DeviceKeys &D = ctx->dev;
    const int NB = P.N / 32, ND = 2 * NB - 1;
    const size_t bk_polys = (size_t)P.k * P.n * 3 * P.bk_ell;
    const size_t evk_polys = (size_t)(P.k + 1) * P.bk_ell;
    D.bk_win_bytes = bk_polys * 4 * ND * kTileBytes;
    D.evk_win_bytes = evk_polys * 4 * ND * kTileBytes;
    if (hipMalloc((void **)&D.bk_win, D.bk_win_bytes) != hipSuccess) {
        D.bk_win = nullptr;
        return fail(MK_ENOMEM, "device allocation failed: MFMA bootstrapping-key tiles");
    }
    if (hipMalloc((void **)&D.evk_win, D.evk_win_bytes) != hipSuccess) {
        D.evk_win = nullptr;
        return fail(MK_ENOMEM, "device allocation failed: MFMA evaluation-key tiles");
    }
    // the extended plain-path keys are already queued for upload on `s`
    const size_t per_poly = (size_t)4 * ND * 64;
    const size_t chunk = (size_t)1 << 20;  // polys per launch bound
    for (size_t p0 = 0; p0 < bk_polys; p0 += chunk) {
        const size_t np = std::min(chunk, bk_polys - p0);
        const size_t threads = np * per_poly;
        hipLaunchKernelGGL(diag_tiles_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s,
                           D.bk_ext + p0 * 2 * P.N, P.N, np, D.bk_win + p0 * 4 * ND * kTileBytes);
        MK_HIP(hipGetLastError(), "diag tiles (bk) launch");
    }
    const size_t threads = evk_polys * per_poly;
    hipLaunchKernelGGL(diag_tiles_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s,
                       D.evk_ext, P.N, evk_polys, D.evk_win);
    MK_HIP(hipGetLastError(), "diag tiles (evk) launch");
    return MK_OK;
}

// ----------------------------------------------------------- kernels ----

struct MfmaArgs {
    int k, n, N, ell, log2N, GP, G;
    uint32_t offset;          // gadget decomposition offset
    const uint32_t *abar;     // [G][kn+1]
    uint32_t *acc;            // [GP][k+1][N]
    uint32_t *W;              // [k+1][GP][N] partial sums w_j
    int8_t *U;                // [k+1][ell][GT][NB][64][16]
    int8_t *V;                // [ell][GT][NB][64][16]
    const int8_t *bk;         // [k][n][3][ell][4][ND][1024]
    const int8_t *evk;        // [k+1][ell][4][ND][1024]
};

// ACC_0 = X^-b v (v = -1/8 below N/2, +1/8 above), other polynomials 0.
__global__ void mfma_init_kernel(MfmaArgs a) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int K1 = a.k + 1, N = a.N;
    const size_t total = (size_t)a.GP * K1 * N;
    if (idx >= total) return;
    const int m = (int)(idx % N);
    const int j = (int)((idx / N) % K1);
    const int g = (int)(idx / ((size_t)K1 * N));
    uint32_t v = 0;
    if (j == 0 && g < a.G) {
        const int s = m + (int)a.abar[(size_t)g * (a.k * a.n + 1)];
        const uint32_t tv = (s & (N - 1)) < N / 2 ? 0xE0000000u : 0x20000000u;
        v = ((s >> a.log2N) & 1) ? 0u - tv : tv;
    }
    a.acc[idx] = v;
}

// Digit kernels.  A workgroup of 256 threads (4 waves) owns one 32-gate tile
// and a range of kDigKB K-blocks (32 kDigKB coefficients).  Phase 1: wave w
// handles gates w, w+4, .., w+28 and lane L the coefficients m0 + L + 64 q,
// so every load instruction reads 64 consecutive words of one gate's row and
// all 8 gates' loads are in flight together; the ell digit bytes go to LDS
// as [l][gate][coefficient] (rows padded by 16 bytes against bank
// conflicts).  Phase 2 writes whole 1 KB MFMA B fragments (lane L = 32 h +
// gate, 16 bytes = coefficients 32 kb + 16 h ..).
constexpr int kDigKB = 4;
constexpr int kDigCoef = 32 * kDigKB;          // coefficients per workgroup
constexpr int kDigRow = kDigCoef + 16;          // padded LDS row (bytes)
constexpr int kDigQ = kDigCoef / 64;            // coefficients per lane per gate

__device__ __forceinline__ void digits_to_lds(int8_t *lds, int ell, int g, int mm, uint32_t y) {
    for (int l = 0; l < ell; ++l)
        lds[(l * 32 + g) * kDigRow + mm] = (int8_t)((int)((y >> (24 - 8 * l)) & 255u) - 128);
}

__device__ __forceinline__ void lds_to_frags(const int8_t *lds, int ell, int8_t *dst_l0,
                                             size_t l_stride, int kb0) {
    // fragment (l, kb) lives at dst_l0 + l * l_stride + kb * 1024
    const int tid = threadIdx.x;
    const int nfr = ell * kDigKB;
    for (int f = tid / 64; f < nfr; f += 4) {
        const int l = f / kDigKB, kk = f % kDigKB;
        const int L = tid & 63, g = L & 31, h = L >> 5;
        const uint4 v = *reinterpret_cast<const uint4 *>(lds + (l * 32 + g) * kDigRow + 32 * kk + 16 * h);
        *reinterpret_cast<uint4 *>(dst_l0 + l * l_stride + (size_t)(kb0 + kk) * kTileBytes + L * 16) = v;
    }
}

// rotdec: item (j, gate tile, K-block group); P_j = X^-a ACC_j - ACC_j.
__global__ __launch_bounds__(256) void mfma_rotdec_kernel(MfmaArgs a, int step) {
    __shared__ __align__(16) int8_t lds[3 * 32 * kDigRow];  // ell <= 3 (ell*8 <= 30)
    const int N = a.N, K1 = a.k + 1, NB = N / 32, GT = a.GP / 32, KG = NB / kDigKB;
    int item = blockIdx.x;
    const int kg = item % KG;
    item /= KG;
    const int gt = item % GT;
    const int j = item / GT;
    const int m0 = kg * kDigCoef;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int stride = a.k * a.n + 1;
    uint32_t y[8][kDigQ];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int g = wave + 4 * i, gg = gt * 32 + g;
        const int shift = gg < a.G ? (int)a.abar[(size_t)gg * stride + 1 + step] : 0;
        const uint32_t *row = a.acc + ((size_t)gg * K1 + j) * N;
#pragma unroll
        for (int q = 0; q < kDigQ; ++q) {
            const int m = m0 + lane + 64 * q;
            const int s = m + shift;
            const uint32_t src = row[s & (N - 1)];
            const uint32_t rot = ((s >> a.log2N) & 1) ? 0u - src : src;
            y[i][q] = rot - row[m] + a.offset;
        }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int q = 0; q < kDigQ; ++q) digits_to_lds(lds, a.ell, wave + 4 * i, lane + 64 * q, y[i][q]);
    __syncthreads();
    lds_to_frags(lds, a.ell, a.U + ((size_t)j * a.ell * GT + gt) * NB * kTileBytes,
                 (size_t)GT * NB * kTileBytes, kg * kDigKB);
}

// wdec: item (gate tile, K-block group); V = g^-1(sum_j W_j).
__global__ __launch_bounds__(256) void mfma_wdec_kernel(MfmaArgs a, int live) {
    __shared__ __align__(16) int8_t lds[3 * 32 * kDigRow];
    const int N = a.N, NB = N / 32, GT = a.GP / 32, KG = NB / kDigKB;
    const int kg = blockIdx.x % KG;
    const int gt = blockIdx.x / KG;
    const int m0 = kg * kDigCoef;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t y[8][kDigQ];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int q = 0; q < kDigQ; ++q) y[i][q] = a.offset;
    for (int j = 0; j < live; ++j) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int gg = gt * 32 + wave + 4 * i;
            const uint32_t *row = a.W + ((size_t)j * a.GP + gg) * N + m0 + lane;
#pragma unroll
            for (int q = 0; q < kDigQ; ++q) y[i][q] += row[64 * q];
        }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int q = 0; q < kDigQ; ++q) digits_to_lds(lds, a.ell, wave + 4 * i, lane + 64 * q, y[i][q]);
    __syncthreads();
    lds_to_frags(lds, a.ell, a.V + (size_t)gt * NB * kTileBytes, (size_t)GT * NB * kTileBytes,
                 kg * kDigKB);
}

// Accumulates acc[r][t] += T_t(A)[rows of tile mb0+r] * B over all NB
// K-blocks, for the 4 limbs t.  The Toeplitz tile of (row tile mb, K-block
// kb) is diagonal tile mb - kb, so when kb advances every row tile inherits
// the previous tile of the row tile above it and only row tile 0 needs a new
// one: a register window of MR tiles per limb, one new tile per limb per
// K-block.  Loads run two K-blocks ahead of the MFMAs (a two-slot ring,
// unrolled so that every register index is static).  They are buffer loads:
// the descriptors bound every access to the operand blocks (out-of-range
// reads return 0), and, unlike plain loads, the compiler does not merge the
// ring's loop-carried loads back into a load at the point of use.
constexpr uint32_t kBufWord3 = 0x00020000u;  // raw dword buffer, gfx9 family

template <int MR, int NC>
__device__ __forceinline__ void toeplitz_gemm(const int8_t *A,  // [4][ND][1024]
                                              const int8_t *B,  // NC x [NB][1024], contiguous
                                              int nc_valid, int NB, int mb0, int lane,
                                              v16i (&acc)[MR][NC][4]) {
    const int ND = 2 * NB - 1;
    const __amdgpu_buffer_rsrc_t ra =
        __builtin_amdgcn_make_buffer_rsrc((void *)A, (short)0, 4 * ND * kTileBytes, kBufWord3);
    // gate tiles beyond nc_valid (ragged last group) read as zero
    const __amdgpu_buffer_rsrc_t rb =
        __builtin_amdgcn_make_buffer_rsrc((void *)B, (short)0, nc_valid * NB * kTileBytes, kBufWord3);
    auto ldA = [&](int t, int kb) {
        return (v4i)__builtin_amdgcn_raw_buffer_load_b128(
            ra, (t * ND + mb0 - kb + NB - 1) * kTileBytes + lane * 16, 0, 0);
    };
    auto ldB = [&](int c, int kb) {
        return (v4i)__builtin_amdgcn_raw_buffer_load_b128(
            rb, (c * NB + kb) * kTileBytes + lane * 16, 0, 0);
    };
    v4i win[MR][4];
#pragma unroll
    for (int r = 0; r < MR; ++r)
#pragma unroll
        for (int t = 0; t < 4; ++t) win[r][t] = ldA(t, -r);
    v4i b[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) b[c] = ldB(c, 0);
    // ring slot s holds the operands of K-block kb+1 (s = kb & 1)
    v4i pa0[4], pa1[4], pb0[NC], pb1[NC];
    {
        const int k1 = NB > 1 ? 1 : 0, k2 = NB > 2 ? 2 : NB - 1;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            pa0[t] = ldA(t, k1);
            pa1[t] = ldA(t, k2);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            pb0[c] = ldB(c, k1);
            pb1[c] = ldB(c, k2);
        }
    }
    auto step = [&](int kb, v4i (&pa)[4], v4i (&pb)[NC]) {
#pragma unroll
        for (int r = 0; r < MR; ++r)
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    acc[r][c][t] =
                        __builtin_amdgcn_mfma_i32_32x32x32_i8(win[r][t], b[c], acc[r][c][t], 0, 0, 0);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
#pragma unroll
            for (int r = MR - 1; r > 0; --r) win[r][t] = win[r - 1][t];
            win[0][t] = pa[t];
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) b[c] = pb[c];
        const int kf = kb + 3 < NB ? kb + 3 : NB - 1;  // clamped: stays in range
#pragma unroll
        for (int t = 0; t < 4; ++t) pa[t] = ldA(t, kf);
#pragma unroll
        for (int c = 0; c < NC; ++c) pb[c] = ldB(c, kf);
    };
    for (int kb = 0; kb < NB; kb += 2) {  // NB is even (N >= 64)
        step(kb, pa0, pb0);
        step(kb + 1, pa1, pb1);
    }
}

// The same contraction for a workgroup whose four waves share the row block
// and the key polynomial (one 32-gate tile per wave): the new diagonal tile
// of each K-block is loaded once per workgroup, limb t by wave t, into a
// three-slot LDS ring and read from there by every wave, which cuts the
// vector-memory traffic per MFMA by 2.5x.  One barrier per K-block: slot
// kb%3 receives the tiles of K-block kb+3 after every wave has read it as
// K-block kb's tiles in the previous iteration.  All four waves must call
// this (gate tiles beyond the batch read zeros through their descriptor).
template <int MR>
__device__ __forceinline__ void toeplitz_gemm_lds(const int8_t *A, const int8_t *B, int nc_valid,
                                                  int NB, int mb0, int lane, int wave,
                                                  int8_t *lds,  // 3 slots x 4 tiles x 1 KB
                                                  v16i (&acc)[MR][1][4]) {
    const int ND = 2 * NB - 1;
    const __amdgpu_buffer_rsrc_t ra =
        __builtin_amdgcn_make_buffer_rsrc((void *)A, (short)0, 4 * ND * kTileBytes, kBufWord3);
    const __amdgpu_buffer_rsrc_t rb =
        __builtin_amdgcn_make_buffer_rsrc((void *)B, (short)0, nc_valid * NB * kTileBytes, kBufWord3);
    auto ldA = [&](int t, int kb) {
        return (v4i)__builtin_amdgcn_raw_buffer_load_b128(
            ra, (t * ND + mb0 - kb + NB - 1) * kTileBytes + lane * 16, 0, 0);
    };
    auto ldB = [&](int kb) {
        return (v4i)__builtin_amdgcn_raw_buffer_load_b128(rb, kb * kTileBytes + lane * 16, 0, 0);
    };
    auto slot = [&](int kb, int t) {
        return reinterpret_cast<v4i *>(lds + (((kb % 3) * 4 + t) * 64 + lane) * 16);
    };
    v4i win[MR][4];
#pragma unroll
    for (int r = 0; r < MR; ++r)
#pragma unroll
        for (int t = 0; t < 4; ++t) win[r][t] = ldA(t, -r);
    v4i b = ldB(0);
    v4i pb0 = ldB(NB > 1 ? 1 : 0), pb1 = ldB(NB > 2 ? 2 : NB - 1);
    *slot(1, wave) = ldA(wave, NB > 1 ? 1 : 0);
    *slot(2, wave) = ldA(wave, NB > 2 ? 2 : NB - 1);
    __syncthreads();
    auto step = [&](int kb, v4i &pb) {
        const int kf = kb + 3 < NB ? kb + 3 : NB - 1;
        const v4i ta = ldA(wave, kf);        // lands in slot kb%3 after the MFMAs
#pragma unroll
        for (int r = 0; r < MR; ++r)
#pragma unroll
            for (int t = 0; t < 4; ++t)
                acc[r][0][t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(win[r][t], b, acc[r][0][t], 0, 0, 0);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
#pragma unroll
            for (int r = MR - 1; r > 0; --r) win[r][t] = win[r - 1][t];
            win[0][t] = *slot(kb + 1, t);
        }
        b = pb;
        pb = ldB(kb + 3 < NB ? kb + 3 : NB - 1);
        *slot(kb, wave) = ta;
        __syncthreads();
    };
    for (int kb = 0; kb < NB; kb += 2) {  // NB is even
        step(kb, pb0);
        step(kb + 1, pb1);
    }
}

// Recombines the limbs of output register e of row tile r, gate tile c.
template <int MR, int NC>
__device__ __forceinline__ uint32_t combine(const v16i (&acc)[MR][NC][4], int r, int c, int e) {
    return (uint32_t)acc[r][c][0][e] + ((uint32_t)acc[r][c][1][e] << 8) +
           ((uint32_t)acc[r][c][2][e] << 16) + ((uint32_t)acc[r][c][3][e] << 24);
}

constexpr int kWaves = 4;   // waves per workgroup

// Task decode shared by both GEMMs.  A wave owns MR row tiles (of 32 rows)
// of NC consecutive 32-gate tiles; a workgroup's four waves share the row
// block and the unit (so the key tiles they load are shared through the
// CU's L1) and cover 4 NC gate tiles.  The gate group is the fastest index:
// with 8 gate groups each XCD keeps one group's digits in its L2.
struct Task {
    int unit, rb, gt0, nc_valid;
};
template <int NC>
__device__ __forceinline__ Task decode_task(int GT, int RB) {
    const int GG = (GT + kWaves * NC - 1) / (kWaves * NC);
    int task = blockIdx.x;
    Task t;
    const int gg = task % GG;
    task /= GG;
    t.rb = task % RB;
    t.unit = task / RB;
    t.gt0 = (gg * kWaves + (int)(threadIdx.x / 64)) * NC;
    t.nc_valid = GT - t.gt0 < NC ? GT - t.gt0 : NC;
    return t;
}

// out[rows of the wave's tiles] (+)= limb-combined accumulators, for the
// valid gate tiles; `rmw` adds to the old contents.  Registers 4q..4q+3 of
// row tile r hold rows m..m+3 of one column (gate).
template <int MR, int NC>
__device__ __forceinline__ void store_tiles(uint32_t *base, size_t gate_stride, const Task &tk,
                                            int MRrows, int lane, const v16i (&acc)[MR][NC][4],
                                            bool rmw) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        if (c >= tk.nc_valid) break;
        const int g = (tk.gt0 + c) * 32 + (lane & 31);
        uint32_t *dst = base + (size_t)g * gate_stride;
#pragma unroll
        for (int r = 0; r < MR; ++r) {
            uint32_t *row = dst + 32 * (tk.rb * MRrows + r) + 4 * (lane / 32);
            uint4 old[4];
            if (rmw) {
#pragma unroll
                for (int q = 0; q < 4; ++q) old[q] = *reinterpret_cast<const uint4 *>(row + 8 * q);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint4 v = make_uint4(combine<MR, NC>(acc, r, c, 4 * q + 0),
                                     combine<MR, NC>(acc, r, c, 4 * q + 1),
                                     combine<MR, NC>(acc, r, c, 4 * q + 2),
                                     combine<MR, NC>(acc, r, c, 4 * q + 3));
                if (rmw) {
                    v.x += old[q].x;
                    v.y += old[q].y;
                    v.z += old[q].z;
                    v.w += old[q].w;
                }
                *reinterpret_cast<uint4 *>(row + 8 * q) = v;
            }
        }
    }
}

// Stage 1.  Unit u < live adds c'_u = sum_l T(d_l) U_{u,l} into ACC_u; unit
// u = live+j writes the partial w_j = sum_l T(b_{j,l}) U_{j,l} to Wp[j].
// Slots j >= live are identically zero (see launch_br_mfma) and skipped.
template <int MR, int NC, int OCC, bool SHARED>
__global__ __launch_bounds__(256, OCC) void mfma_gemm1_kernel(MfmaArgs a, int party, int bit, int live) {
    __shared__ __align__(16) int8_t lds[SHARED ? 3 * 4 * kTileBytes : 16];
    const int N = a.N, NB = N / 32, ND = 2 * NB - 1, K1 = a.k + 1, ell = a.ell;
    const int GT = a.GP / 32;
    const Task tk = decode_task<NC>(GT, NB / MR);
    if (!SHARED && tk.nc_valid <= 0) return;
    const int lane = threadIdx.x & 63;
    const int kind = tk.unit / live, j = tk.unit % live;
    v16i acc[MR][NC][4];
#pragma unroll
    for (int r = 0; r < MR; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[r][c][t] = v16i{};
    const size_t poly_tiles = (size_t)4 * ND * kTileBytes;
    for (int l = 0; l < ell; ++l) {
        const int8_t *A = kind == 0
            ? a.bk + ((((size_t)party * a.n + bit) * 3 + 0) * ell + l) * poly_tiles
            : a.evk + ((size_t)j * ell + l) * poly_tiles;
        const int8_t *B = a.U + ((size_t)(j * ell + l) * GT + tk.gt0) * NB * kTileBytes;
        if constexpr (SHARED)
            toeplitz_gemm_lds<MR>(A, B, tk.nc_valid > 0 ? 1 : 0, NB, tk.rb * MR, lane,
                                  (int)(threadIdx.x / 64), lds, acc);
        else
            toeplitz_gemm<MR, NC>(A, B, tk.nc_valid, NB, tk.rb * MR, lane, acc);
    }
    if (tk.nc_valid <= 0) return;
    uint32_t *base = kind == 0 ? a.acc + (size_t)j * N : a.W + (size_t)j * a.GP * N;
    const size_t gate_stride = kind == 0 ? (size_t)K1 * N : (size_t)N;
    store_tiles<MR, NC>(base, gate_stride, tk, MR, lane, acc, kind == 0);
}

// Stage 2.  Unit o: ACC_{o ? 1+party : 0} += sum_l T(f_o,l) V_l.
template <int MR, int NC, int OCC, bool SHARED>
__global__ __launch_bounds__(256, OCC) void mfma_gemm2_kernel(MfmaArgs a, int party, int bit) {
    __shared__ __align__(16) int8_t lds[SHARED ? 3 * 4 * kTileBytes : 16];
    const int N = a.N, NB = N / 32, ND = 2 * NB - 1, K1 = a.k + 1, ell = a.ell;
    const int GT = a.GP / 32;
    const Task tk = decode_task<NC>(GT, NB / MR);
    if (!SHARED && tk.nc_valid <= 0) return;
    const int lane = threadIdx.x & 63;
    const int o = tk.unit;
    v16i acc[MR][NC][4];
#pragma unroll
    for (int r = 0; r < MR; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[r][c][t] = v16i{};
    const size_t poly_tiles = (size_t)4 * ND * kTileBytes;
    for (int l = 0; l < ell; ++l) {
        const int8_t *A = a.bk + ((((size_t)party * a.n + bit) * 3 + 1 + o) * ell + l) * poly_tiles;
        const int8_t *B = a.V + ((size_t)l * GT + tk.gt0) * NB * kTileBytes;
        if constexpr (SHARED)
            toeplitz_gemm_lds<MR>(A, B, tk.nc_valid > 0 ? 1 : 0, NB, tk.rb * MR, lane,
                                  (int)(threadIdx.x / 64), lds, acc);
        else
            toeplitz_gemm<MR, NC>(A, B, tk.nc_valid, NB, tk.rb * MR, lane, acc);
    }
    if (tk.nc_valid <= 0) return;
    store_tiles<MR, NC>(a.acc + (size_t)(o == 0 ? 0 : 1 + party) * N, (size_t)K1 * N, tk, MR, lane,
                        acc, true);
}

// Tile configurations of the two GEMMs (rows per wave MR x gate tiles per
// wave NC, waves per SIMD OCC).  The autotuner picks one per batch shape.
struct GemmShape {
    int MR, NC;
};
constexpr GemmShape kShapes[] = {{2, 1}, {4, 1}, {2, 2}, {2, 1}, {4, 1}};
constexpr int kNumShapes = 5;

// Shapes 3 and 4 share each K-block's key tiles through LDS.
template <int V>
struct ShapeOf;
template <> struct ShapeOf<0> { static constexpr int MR = 2, NC = 1, OCC = 2; static constexpr bool SH = false; };
template <> struct ShapeOf<1> { static constexpr int MR = 4, NC = 1, OCC = 1; static constexpr bool SH = false; };
template <> struct ShapeOf<2> { static constexpr int MR = 2, NC = 2, OCC = 1; static constexpr bool SH = false; };
template <> struct ShapeOf<3> { static constexpr int MR = 2, NC = 1, OCC = 2; static constexpr bool SH = true; };
template <> struct ShapeOf<4> { static constexpr int MR = 4, NC = 1, OCC = 1; static constexpr bool SH = true; };

template <int V>
static void launch_g1(const MfmaArgs &a, int party, int bit, int live, int GT, int NB, hipStream_t s) {
    using S = ShapeOf<V>;
    const int GG = (GT + kWaves * S::NC - 1) / (kWaves * S::NC);
    const unsigned g = (unsigned)(2 * live * (NB / S::MR) * GG);
    hipLaunchKernelGGL((mfma_gemm1_kernel<S::MR, S::NC, S::OCC, S::SH>), dim3(g), dim3(64 * kWaves), 0, s,
                       a, party, bit, live);
}
template <int V>
static void launch_g2(const MfmaArgs &a, int party, int bit, int GT, int NB, hipStream_t s) {
    using S = ShapeOf<V>;
    const int GG = (GT + kWaves * S::NC - 1) / (kWaves * S::NC);
    const unsigned g = (unsigned)(2 * (NB / S::MR) * GG);
    hipLaunchKernelGGL((mfma_gemm2_kernel<S::MR, S::NC, S::OCC, S::SH>), dim3(g), dim3(64 * kWaves), 0, s,
                       a, party, bit);
}
static void gemm1(int v, const MfmaArgs &a, int party, int bit, int live, int GT, int NB, hipStream_t s) {
    switch (v) {
        case 1: launch_g1<1>(a, party, bit, live, GT, NB, s); break;
        case 2: launch_g1<2>(a, party, bit, live, GT, NB, s); break;
        case 3: launch_g1<3>(a, party, bit, live, GT, NB, s); break;
        case 4: launch_g1<4>(a, party, bit, live, GT, NB, s); break;
        default: launch_g1<0>(a, party, bit, live, GT, NB, s);
    }
}
static void gemm2(int v, const MfmaArgs &a, int party, int bit, int GT, int NB, hipStream_t s) {
    switch (v) {
        case 1: launch_g2<1>(a, party, bit, GT, NB, s); break;
        case 2: launch_g2<2>(a, party, bit, GT, NB, s); break;
        case 3: launch_g2<3>(a, party, bit, GT, NB, s); break;
        case 4: launch_g2<4>(a, party, bit, GT, NB, s); break;
        default: launch_g2<0>(a, party, bit, GT, NB, s);
    }
}

__global__ void mfma_copyout_kernel(const uint32_t *__restrict__ src, uint32_t *__restrict__ dst,
                                    size_t words) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < words) dst[idx] = src[idx];
}

static inline unsigned blocks(size_t threads, int per) { return (unsigned)((threads + per - 1) / per); }

// Allocates (grows) the MFMA scratch for `count` gates and fills the kernel
// arguments.
static int prepare(mk_ctx *ctx, const uint32_t *abar, size_t count, hipStream_t s, MfmaArgs &a) {
    const mk_params &P = ctx->p;
    if (P.N < kDigCoef) return fail(MK_EPARAM, "int8-MFMA path needs N >= 128");
    const size_t GP = (count + 31) / 32 * 32;
    const int K1 = P.k + 1, N = P.N, ell = P.bk_ell;
    const size_t acc_b = GP * K1 * N * 4, w_b = (size_t)K1 * GP * N * 4;
    const size_t u_b = (size_t)K1 * ell * GP * N, v_b = (size_t)ell * GP * N;
    DeviceKeys &D = ctx->dev;
    const size_t need = acc_b + w_b + u_b + v_b;
    if (D.mfma_scratch_bytes < need) {
        if (D.mfma_scratch) {
            MK_HIP(hipStreamSynchronize(s), "mfma scratch sync");
            (void)hipFree(D.mfma_scratch);
            D.mfma_scratch = nullptr;
            D.mfma_scratch_bytes = 0;
        }
        if (hipMalloc(&D.mfma_scratch, need) != hipSuccess) {
            D.mfma_scratch = nullptr;
            return fail(MK_ENOMEM, "device allocation failed: MFMA scratch");
        }
        D.mfma_scratch_bytes = need;
    }
    char *sp = (char *)D.mfma_scratch;
    a.k = P.k; a.n = P.n; a.N = N; a.ell = ell; a.log2N = __builtin_ctz(N);
    a.GP = (int)GP; a.G = (int)count;
    a.offset = decomp_offset(ell);
    a.abar = abar;
    a.acc = (uint32_t *)sp;
    a.W = (uint32_t *)(sp + acc_b);
    a.U = (int8_t *)(sp + acc_b + w_b);
    a.V = (int8_t *)(sp + acc_b + w_b + u_b);
    a.bk = D.bk_win;
    a.evk = D.evk_win;
    return MK_OK;
}

// Tile shapes for a batch of GT gate tiles: forced by mk_set_tiles, else the
// autotuned choice for this size, else shape 0.
static void shapes_for(const mk_ctx *ctx, int GT, int &v1, int &v2) {
    const DeviceKeys &D = ctx->dev;
    v1 = v2 = 0;
    auto it = D.tuned_tiles.find(GT);
    if (it != D.tuned_tiles.end()) {
        v1 = it->second.first;
        v2 = it->second.second;
    }
    if (D.force_tiles[0] >= 0) v1 = D.force_tiles[0];
    if (D.force_tiles[1] >= 0) v2 = D.force_tiles[1];
}

int launch_br_mfma(mk_ctx *ctx, const uint32_t *abar, uint32_t *acc_out, size_t count, int steps,
                   hipStream_t s) {
    const mk_params &P = ctx->p;
    MfmaArgs a;
    int rc = prepare(ctx, abar, count, s, a);
    if (rc) return rc;
    const int K1 = P.k + 1, N = P.N;
    const size_t GP = (size_t)a.GP;
    const int NB = N / 32, GT = (int)(GP / 32);
    int v1, v2;
    shapes_for(ctx, GT, v1, v2);
    {
        StageTimer tm(ctx, 1, s);
        hipLaunchKernelGGL(mfma_init_kernel, dim3(blocks(GP * K1 * N, 256)), dim3(256), 0, s, a);
        MK_HIP(hipGetLastError(), "mfma init launch");
        const int KG = NB / kDigKB;
        const unsigned wd_blocks = (unsigned)(GT * KG);
        for (int st = 0; st < steps; ++st) {
            const int party = st / P.n, bit = st % P.n;
            // ACC starts as (X^-b v, 0, .., 0) and during party i's steps only
            // c'_0 and c'_{1+i} receive stage-2 output, while c'_j = 0 whenever
            // ACC_j = 0 (its digits are all zero).  So slots j >= i+2 are still
            // exactly zero: their digits, products and partial sums are skipped.
            const int live = std::min(K1, party + 2);
            const unsigned rd_blocks = (unsigned)(live * GT * KG);
            {
                StageTimer t6(ctx, 6, s);
                hipLaunchKernelGGL(mfma_rotdec_kernel, dim3(rd_blocks), dim3(256), 0, s, a, st);
            }
            {
                StageTimer t4(ctx, 4, s);
                gemm1(v1, a, party, bit, live, GT, NB, s);
            }
            {
                StageTimer t7(ctx, 7, s);
                hipLaunchKernelGGL(mfma_wdec_kernel, dim3(wd_blocks), dim3(256), 0, s, a, live);
            }
            {
                StageTimer t5(ctx, 5, s);
                gemm2(v2, a, party, bit, GT, NB, s);
            }
        }
        MK_HIP(hipGetLastError(), "mfma step launch");
        hipLaunchKernelGGL(mfma_copyout_kernel, dim3(blocks(count * K1 * N, 256)), dim3(256), 0, s,
                           a.acc, acc_out, count * K1 * N);
        MK_HIP(hipGetLastError(), "mfma copyout launch");
    }
    return MK_OK;
}

// Times every tile shape of both GEMMs on the scratch buffers of a batch of
// `count` gates (contents irrelevant: only durations are read) and records
// the fastest for this batch size.
int autotune(mk_ctx *ctx, size_t count, hipStream_t s, int *v1_out, int *v2_out, float *ms_out) {
    const mk_params &P = ctx->p;
    MfmaArgs a;
    int rc = prepare(ctx, nullptr, count, s, a);
    if (rc) return rc;
    const int NB = P.N / 32, GT = a.GP / 32;
    const int party = P.k - 1, live = std::min(P.k + 1, party + 2);
    hipEvent_t e0, e1;
    MK_HIP(hipEventCreate(&e0), "autotune event");
    MK_HIP(hipEventCreate(&e1), "autotune event");
    constexpr int kReps = 4;
    float best[2] = {3.0e38f, 3.0e38f};
    int pick[2] = {0, 0};
    for (int which = 0; which < 2; ++which)
        for (int v = 0; v < kNumShapes; ++v) {
            if (NB % kShapes[v].MR) continue;
            auto run = [&]() {
                if (which == 0) gemm1(v, a, party, 0, live, GT, NB, s);
                else gemm2(v, a, party, 0, GT, NB, s);
            };
            run();  // warm-up
            (void)hipEventRecord(e0, s);
            for (int r = 0; r < kReps; ++r) run();
            (void)hipEventRecord(e1, s);
            float ms = 0;
            if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                return fail(MK_EDEVICE, "autotune timing failed");
            }
            if (ms_out) ms_out[which * kNumShapes + v] = ms / kReps;
            if (ms < best[which]) {
                best[which] = ms;
                pick[which] = v;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    MK_HIP(hipGetLastError(), "autotune launch");
    ctx->dev.tuned_tiles[GT] = {pick[0], pick[1]};
    if (v1_out) *v1_out = pick[0];
    if (v2_out) *v2_out = pick[1];
    return MK_OK;
}

}  // namespace mk

using namespace mk;

extern "C" {

int mk_autotune(mk_ctx *ctx, size_t count, void *stream, int32_t *gemm1_shape, int32_t *gemm2_shape,
                float *ms) {
    if (!ctx || !count) return fail(MK_EINVAL, "mk_autotune: bad argument");
    if (!ctx->dev.uploaded) return fail(MK_ESTATE, "evaluation key not uploaded (mk_upload_eval_key)");
    int v1 = 0, v2 = 0;
    const int rc = autotune(ctx, count, (hipStream_t)stream, &v1, &v2, ms);
    if (gemm1_shape) *gemm1_shape = v1;
    if (gemm2_shape) *gemm2_shape = v2;
    return rc;
}

int mk_set_tiles(mk_ctx *ctx, int gemm1_shape, int gemm2_shape) {
    if (!ctx || gemm1_shape < -1 || gemm1_shape >= kNumShapes || gemm2_shape < -1 ||
        gemm2_shape >= kNumShapes)
        return fail(MK_EINVAL, "mk_set_tiles: shape out of range");
    const int NB = ctx->p.N / 32;
    if ((gemm1_shape >= 0 && NB % kShapes[gemm1_shape].MR) ||
        (gemm2_shape >= 0 && NB % kShapes[gemm2_shape].MR))
        return fail(MK_EINVAL, "mk_set_tiles: shape does not divide N/32");
    ctx->dev.force_tiles[0] = gemm1_shape;
    ctx->dev.force_tiles[1] = gemm2_shape;
    return MK_OK;
}

int mk_get_tiles(const mk_ctx *ctx, size_t count, int32_t *gemm1_shape, int32_t *gemm2_shape) {
    if (!ctx) return fail(MK_EINVAL, "mk_get_tiles: null context");
    int v1, v2;
    shapes_for(ctx, (int)((count + 31) / 32), v1, v2);
    if (gemm1_shape) *gemm1_shape = v1;
    if (gemm2_shape) *gemm2_shape = v2;
    return MK_OK;
}

}  // extern "C"
