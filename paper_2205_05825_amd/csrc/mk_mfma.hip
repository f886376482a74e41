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
#include "mk_ks_core.h"
#include "mk_mfma_core.h"

namespace mk {


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

__global__ void mfma_rotdec_kernel(MfmaArgs a, int step);

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
    int prc = persist_probe(ctx, s);
    if (prc) return prc;
    // rotdec keeps 8 accumulator rows in LDS (128 KB at N = 4096)
    const int rows_lds = 8 * P.N * 4;
    if (rows_lds > 65536)
        MK_HIP(hipFuncSetAttribute((const void *)mfma_rotdec_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   rows_lds),
               "rotdec LDS attribute");
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

// rotdec: workgroup = (slot j, 8 consecutive gates).  The 8 rows ACC_j are
// read once, with 16-byte loads, into LDS; then every piece takes its 16
// plain and 16 rotated coefficients from there: P_j = X^-a ACC_j - ACC_j,
// (X^-a c)[m] = c[m + a] for m + a < N and -c[m + a - N] beyond.
constexpr int kRotdecThreads = 512;
__global__ __launch_bounds__(kRotdecThreads) void mfma_rotdec_kernel(MfmaArgs a, int step) {
    extern __shared__ __align__(16) uint32_t rows[];   // [8][N]
    const int N = a.N, K1 = a.k + 1, NB = N / 32, GT = a.GP / 32;
    const int groups = a.GP / 8;
    const int j = blockIdx.x / groups, g8 = blockIdx.x % groups;
    const int tid = threadIdx.x;
    {
        const int per_row = N / 4;  // uint4 per row
        for (int v = tid; v < 8 * per_row; v += kRotdecThreads) {
            const int gi = v / per_row, c4 = v % per_row;
            const size_t gate = (size_t)g8 * 8 + gi;
            reinterpret_cast<uint4 *>(rows)[v] =
                reinterpret_cast<const uint4 *>(a.acc + (gate * K1 + j) * N)[c4];
        }
    }
    const int gi = tid % 8;
    const int gate = g8 * 8 + gi;
    const int stride = a.k * a.n + 1;
    const int shift = gate < a.G ? (int)a.abar[(size_t)gate * stride + 1 + step] : 0;
    __syncthreads();
    const uint32_t *row = rows + gi * N;
    const int gt = gate / 32, L0 = gate % 32;
    const size_t l_stride = (size_t)GT * NB * kTileBytes;
    int8_t *base = a.U + ((size_t)j * a.ell * GT + gt) * NB * kTileBytes;
    for (int item = tid / 8; item < NB * 2; item += kRotdecThreads / 8) {  // item = (kb, h)
        const int kb = item / 2, h = item % 2;
        const int m0 = 32 * kb + 16 * h;
        uint32_t y[16];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint4 p = *reinterpret_cast<const uint4 *>(row + m0 + 4 * q);
            const uint32_t pv[4] = {p.x, p.y, p.z, p.w};
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int s = m0 + 4 * q + b + shift;
                const uint32_t src = row[s & (N - 1)];
                const uint32_t rot = ((s >> a.log2N) & 1) ? 0u - src : src;
                y[4 * q + b] = rot - pv[b] + a.offset;
            }
        }
        put_digits(base + (size_t)kb * kTileBytes + (32 * h + L0) * 16, l_stride, a.ell, y);
    }
}

// wdec: one thread per V fragment piece; V = g^-1(sum_j W_j) over the live
// partial rows (16-byte loads: a wave reads 32 gates x 128 bytes).
__global__ __launch_bounds__(256) void mfma_wdec_kernel(MfmaArgs a, int live) {
    const int N = a.N, NB = N / 32, GT = a.GP / 32;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)GT * NB * 64) return;
    const int L = (int)(idx % 64), kb = (int)((idx / 64) % NB), gt = (int)(idx / (64 * (size_t)NB));
    const int g = L % 32, h = L / 32;
    const size_t gate = (size_t)gt * 32 + g;
    const int m0 = 32 * kb + 16 * h;
    uint32_t y[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) y[e] = a.offset;
    for (int jj = 0; jj < live; ++jj) {
        const uint4 *src = reinterpret_cast<const uint4 *>(a.W + ((size_t)jj * a.GP + gate) * N + m0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint4 v = src[q];
            y[4 * q + 0] += v.x;
            y[4 * q + 1] += v.y;
            y[4 * q + 2] += v.z;
            y[4 * q + 3] += v.w;
        }
    }
    put_digits(a.V + ((size_t)gt * NB + kb) * kTileBytes + L * 16, (size_t)GT * NB * kTileBytes, a.ell, y);
}

// Stage 1.  Unit u < live adds c'_u = sum_l T(d_l) U_{u,l} into ACC_u; unit
// u = live+j writes the partial w_j = sum_l T(b_{j,l}) U_{j,l} to Wp[j].
// Slots j >= live are identically zero (see launch_br_mfma) and skipped.
template <int MR, int NC, int OCC>
__global__ __launch_bounds__(256, OCC) void mfma_gemm1_kernel(MfmaArgs a, int party, int bit, int live) {
    const int N = a.N, NB = N / 32, ND = 2 * NB - 1, K1 = a.k + 1, ell = a.ell;
    const int GT = a.GP / 32;
    const Task tk = decode_task<NC>(GT, NB / MR);
    if (tk.nc_valid <= 0) return;
    const int lane = threadIdx.x & 63;
    const int kind = tk.unit / live, j = tk.unit % live;
    const size_t poly_tiles = (size_t)4 * ND * kTileBytes;
    Operands o;
    o.A = kind == 0 ? a.bk + (((size_t)party * a.n + bit) * 3 + 0) * ell * poly_tiles
                    : a.evk + (size_t)j * ell * poly_tiles;
    o.B = a.U + ((size_t)j * ell * GT + tk.gt0) * NB * kTileBytes;
    o.b_poly = (uint32_t)((size_t)GT * NB * kTileBytes);
    o.ell = ell; o.NB = NB; o.mb0 = tk.rb * MR; o.nc_valid = tk.nc_valid;
    uint32_t *base = kind == 0 ? a.acc + (size_t)j * N : a.W + (size_t)j * a.GP * N;
    const size_t gate_stride = kind == 0 ? (size_t)K1 * N : (size_t)N;
    v16i acc[MR][NC][4];
#pragma unroll
    for (int r = 0; r < MR; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[r][c][t] = v16i{};
    if (kind == 0) {  // c'_j is added to ACC_j
        uint4 old[MR][NC][4];
        load_tiles<MR, NC>(base, gate_stride, tk, lane, old);
        toeplitz_gemm<MR, NC>(o, lane, acc, [&]() { seed_acc<MR, NC>(old, acc); });
    } else {
        toeplitz_gemm<MR, NC>(o, lane, acc, []() {});
    }
    store_tiles<MR, NC>(base, gate_stride, tk, lane, acc);
}

// Stage 2.  Unit o: ACC_{o ? 1+party : 0} += sum_l T(f_o,l) V_l.
template <int MR, int NC, int OCC>
__global__ __launch_bounds__(256, OCC) void mfma_gemm2_kernel(MfmaArgs a, int party, int bit) {
    const int N = a.N, NB = N / 32, ND = 2 * NB - 1, K1 = a.k + 1, ell = a.ell;
    const int GT = a.GP / 32;
    const Task tk = decode_task<NC>(GT, NB / MR);
    if (tk.nc_valid <= 0) return;
    const int lane = threadIdx.x & 63;
    const size_t poly_tiles = (size_t)4 * ND * kTileBytes;
    Operands o;
    o.A = a.bk + ((((size_t)party * a.n + bit) * 3 + 1 + tk.unit) * ell) * poly_tiles;
    o.B = a.V + (size_t)tk.gt0 * NB * kTileBytes;
    o.b_poly = (uint32_t)((size_t)GT * NB * kTileBytes);
    o.ell = ell; o.NB = NB; o.mb0 = tk.rb * MR; o.nc_valid = tk.nc_valid;
    uint32_t *base = a.acc + (size_t)(tk.unit == 0 ? 0 : 1 + party) * N;
    v16i acc[MR][NC][4];
#pragma unroll
    for (int r = 0; r < MR; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[r][c][t] = v16i{};
    uint4 old[MR][NC][4];
    load_tiles<MR, NC>(base, (size_t)K1 * N, tk, lane, old);
    toeplitz_gemm<MR, NC>(o, lane, acc, [&]() { seed_acc<MR, NC>(old, acc); });
    store_tiles<MR, NC>(base, (size_t)K1 * N, tk, lane, acc);
}

// ------------------------------------------------------- K-split GEMMs ----
//
// At small batches the GEMMs above occupy a few dozen CUs and their time is
// the length of one wave's MFMA chain (MR x 4 limbs x ell x (NB + MR - 1))
// plus the load latencies along it.  These variants split the contraction:
// a workgroup has ell x H waves for one (unit, row block, gate tile), wave
// (l, c) runs the skewed schedule over key polynomial l alone (its digit
// block and key tiles start at l) and, with H = 2, over half of its K-blocks
// (MR = 1 only), with a deeper prefetch.  The partial results, limbs already
// combined, are summed through LDS by wave 0, which also does the
// read-modify-write of the output.  The launch bounds ask for two
// workgroups per CU, which caps a wave at 256 registers.
constexpr int kSplitD = 4;  // prefetch depth of the K-split GEMMs

__device__ __forceinline__ Task decode_split(int GT, int RB) {
    int task = blockIdx.x;
    Task t;
    t.gt0 = task % GT;  // gate tile fastest: each XCD keeps its tiles' digits
    task /= GT;
    t.rb = task % RB;
    t.unit = task / RB;
    t.nc_valid = 1;
    return t;
}

template <int MR>
__device__ __forceinline__ void split_reduce_store(uint32_t *red, int w, int waves, int lane,
                                                   const v16i (&acc)[MR][1][4], uint32_t *base,
                                                   size_t gate_stride, const Task &tk) {
    uint32_t v[MR][16];
#pragma unroll
    for (int r = 0; r < MR; ++r)
#pragma unroll
        for (int e = 0; e < 16; ++e) v[r][e] = combine<MR, 1>(acc, r, 0, e);
    if (w > 0) {
#pragma unroll
        for (int r = 0; r < MR; ++r)
#pragma unroll
            for (int e = 0; e < 16; ++e) red[(((w - 1) * MR + r) * 16 + e) * 64 + lane] = v[r][e];
    }
    __syncthreads();
    if (w != 0) return;
    for (int i = 1; i < waves; ++i)
#pragma unroll
        for (int r = 0; r < MR; ++r)
#pragma unroll
            for (int e = 0; e < 16; ++e) v[r][e] += red[(((i - 1) * MR + r) * 16 + e) * 64 + lane];
#pragma unroll
    for (int r = 0; r < MR; ++r) {
        uint32_t *row = tile_row<MR>(base, gate_stride, tk, 0, r, lane);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            *reinterpret_cast<uint4 *>(row + 8 * q) =
                make_uint4(v[r][4 * q], v[r][4 * q + 1], v[r][4 * q + 2], v[r][4 * q + 3]);
    }
}

// Runs wave (l, c)'s part of the contraction; with `seed` (wave 0 of a
// read-modify-write unit) the old output values start the accumulators.
template <int MR, int H>
__device__ __forceinline__ void split_part(const Operands &o, int c, int lane, bool seed, uint32_t *base,
                                           size_t gate_stride, const Task &tk, v16i (&acc)[MR][1][4]) {
    static_assert(H == 1 || MR == 1, "K-block chunks need the one-row schedule");
    const int NB = o.NB;
    const int X0 = c * (NB / H), nsteps = H == 1 ? NB + MR - 1 : NB / H;
#pragma unroll
    for (int r = 0; r < MR; ++r)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[r][0][t] = v16i{};
    if (seed) {
        uint4 old[MR][1][4];
        load_tiles<MR, 1>(base, gate_stride, tk, lane, old);
        toeplitz_gemm<MR, 1, kSplitD>(o, lane, acc, [&]() { seed_acc<MR, 1>(old, acc); }, X0, nsteps);
    } else {
        toeplitz_gemm<MR, 1, kSplitD>(o, lane, acc, []() {}, X0, nsteps);
    }
}

// Stage 1, K-split: units as in mfma_gemm1_kernel.
template <int MR, int H>
__global__ __launch_bounds__(64 * kMaxEll * H, 2) void mfma_gemm1_split_kernel(MfmaArgs a, int party, int bit,
                                                                             int live) {
    __shared__ uint32_t red[(kMaxEll * H - 1) * MR * 16 * 64];
    const int N = a.N, NB = N / 32, ND = 2 * NB - 1, K1 = a.k + 1, ell = a.ell;
    const int GT = a.GP / 32;
    const Task tk = decode_split(GT, NB / MR);
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64)), l = w / H, c = w % H;
    const int kind = tk.unit / live, j = tk.unit % live;
    const size_t poly_tiles = (size_t)4 * ND * kTileBytes;
    Operands o;
    o.A = (kind == 0 ? a.bk + (((size_t)party * a.n + bit) * 3 + 0) * ell * poly_tiles
                     : a.evk + (size_t)j * ell * poly_tiles) +
          (size_t)l * poly_tiles;
    o.B = a.U + (((size_t)j * ell + l) * GT + tk.gt0) * NB * kTileBytes;
    o.b_poly = (uint32_t)((size_t)GT * NB * kTileBytes);
    o.ell = 1; o.NB = NB; o.mb0 = tk.rb * MR; o.nc_valid = 1;
    uint32_t *base = kind == 0 ? a.acc + (size_t)j * N : a.W + (size_t)j * a.GP * N;
    const size_t gate_stride = kind == 0 ? (size_t)K1 * N : (size_t)N;
    v16i acc[MR][1][4];
    split_part<MR, H>(o, c, lane, kind == 0 && w == 0, base, gate_stride, tk, acc);
    split_reduce_store<MR>(red, w, ell * H, lane, acc, base, gate_stride, tk);
}

// Stage 2, K-split: units as in mfma_gemm2_kernel.
template <int MR, int H>
__global__ __launch_bounds__(64 * kMaxEll * H, 2) void mfma_gemm2_split_kernel(MfmaArgs a, int party, int bit) {
    __shared__ uint32_t red[(kMaxEll * H - 1) * MR * 16 * 64];
    const int N = a.N, NB = N / 32, ND = 2 * NB - 1, K1 = a.k + 1, ell = a.ell;
    const int GT = a.GP / 32;
    const Task tk = decode_split(GT, NB / MR);
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64)), l = w / H, c = w % H;
    const size_t poly_tiles = (size_t)4 * ND * kTileBytes;
    Operands o;
    o.A = a.bk + ((((size_t)party * a.n + bit) * 3 + 1 + tk.unit) * ell + l) * poly_tiles;
    o.B = a.V + ((size_t)l * GT + tk.gt0) * NB * kTileBytes;
    o.b_poly = (uint32_t)((size_t)GT * NB * kTileBytes);
    o.ell = 1; o.NB = NB; o.mb0 = tk.rb * MR; o.nc_valid = 1;
    uint32_t *base = a.acc + (size_t)(tk.unit == 0 ? 0 : 1 + party) * N;
    const size_t gate_stride = (size_t)K1 * N;
    v16i acc[MR][1][4];
    split_part<MR, H>(o, c, lane, w == 0, base, gate_stride, tk, acc);
    split_reduce_store<MR>(red, w, ell * H, lane, acc, base, gate_stride, tk);
}

// Workgroup task of the limb-split GEMMs: (unit, row block, NC gate tiles),
// the gate group fastest (spread over the XCDs).
template <int NC>
__device__ __forceinline__ Task decode_limb_task(int GT, int RB) {
    const int GG = (GT + NC - 1) / NC;
    int task = blockIdx.x;
    Task t;
    const int gg = task % GG;
    task /= GG;
    t.rb = task % RB;
    t.unit = task / RB;
    t.gt0 = gg * NC;
    t.nc_valid = GT - t.gt0 < NC ? GT - t.gt0 : NC;
    return t;
}

// Stage 1, limb-split (units as in mfma_gemm1_kernel).
template <int MR, int NC, int OCC>
__global__ __launch_bounds__(256, OCC) void mfma_gemm1_limb_kernel(MfmaArgs a, int party, int bit, int live) {
    __shared__ __align__(16) uint4 red[2 * 4 * 4 * 64];
    const int N = a.N, NB = N / 32, ND = 2 * NB - 1, K1 = a.k + 1, ell = a.ell;
    const int GT = a.GP / 32;
    const Task tk = decode_limb_task<NC>(GT, NB / MR);
    const int lane = threadIdx.x & 63;
    const int t = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
    const int kind = tk.unit / live, j = tk.unit % live;
    const size_t poly_tiles = (size_t)4 * ND * kTileBytes;
    Operands o;
    o.A = kind == 0 ? a.bk + (((size_t)party * a.n + bit) * 3 + 0) * ell * poly_tiles
                    : a.evk + (size_t)j * ell * poly_tiles;
    o.B = a.U + ((size_t)j * ell * GT + tk.gt0) * NB * kTileBytes;
    o.b_poly = (uint32_t)((size_t)GT * NB * kTileBytes);
    o.ell = ell; o.NB = NB; o.mb0 = tk.rb * MR; o.nc_valid = tk.nc_valid;
    uint32_t *base = kind == 0 ? a.acc + (size_t)j * N : a.W + (size_t)j * a.GP * N;
    const size_t gate_stride = kind == 0 ? (size_t)K1 * N : (size_t)N;
    v16i acc[MR][NC];
#pragma unroll
    for (int r = 0; r < MR; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[r][c] = v16i{};
    const bool seed = kind == 0 && (t == 0 || t == 3);  // c'_j is added to ACC_j
    limb_gemm<MR, NC>(o, t, lane, acc, [&]() {
        if (seed) {
            load_old<MR, NC>(base, gate_stride, tk, lane, acc);
            seed_old<MR, NC>(t, acc);
        }
    });
    combine_store<MR, NC>(base, gate_stride, tk, t, lane, acc, red);
}

// Stage 2, limb-split: unit o adds sum_l T(f_o,l) V_l to ACC_{o ? 1+party : 0}.
template <int MR, int NC, int OCC>
__global__ __launch_bounds__(256, OCC) void mfma_gemm2_limb_kernel(MfmaArgs a, int party, int bit) {
    __shared__ __align__(16) uint4 red[2 * 4 * 4 * 64];
    const int N = a.N, NB = N / 32, ND = 2 * NB - 1, K1 = a.k + 1, ell = a.ell;
    const int GT = a.GP / 32;
    const Task tk = decode_limb_task<NC>(GT, NB / MR);
    const int lane = threadIdx.x & 63;
    const int t = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
    const size_t poly_tiles = (size_t)4 * ND * kTileBytes;
    Operands o;
    o.A = a.bk + ((((size_t)party * a.n + bit) * 3 + 1 + tk.unit) * ell) * poly_tiles;
    o.B = a.V + (size_t)tk.gt0 * NB * kTileBytes;
    o.b_poly = (uint32_t)((size_t)GT * NB * kTileBytes);
    o.ell = ell; o.NB = NB; o.mb0 = tk.rb * MR; o.nc_valid = tk.nc_valid;
    uint32_t *base = a.acc + (size_t)(tk.unit == 0 ? 0 : 1 + party) * N;
    v16i acc[MR][NC];
#pragma unroll
    for (int r = 0; r < MR; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[r][c] = v16i{};
    const bool seed = t == 0 || t == 3;
    limb_gemm<MR, NC>(o, t, lane, acc, [&]() {
        if (seed) {
            load_old<MR, NC>(base, (size_t)K1 * N, tk, lane, acc);
            seed_old<MR, NC>(t, acc);
        }
    });
    combine_store<MR, NC>(base, (size_t)K1 * N, tk, t, lane, acc, red);
}

// Tile configurations of the two GEMMs.  Limb-split shapes (LIMB): MR row
// tiles x NC gate tiles per workgroup, one limb per wave; shared-key shape:
// MR row tiles x NC gate tiles per wave, four limbs per wave, four gate
// tiles per workgroup.  OCC: workgroups per CU the register budget is sized
// for.  The autotuner picks one per batch shape.
struct GemmShape {
    int MR, NC;
};
constexpr GemmShape kShapes[] = {{8, 1}, {4, 2}, {4, 1}, {2, 1}, {8, 2}, {2, 1}, {1, 1}, {1, 1}};
constexpr int kNumShapes = 8;

template <int V>
struct ShapeOf;
template <> struct ShapeOf<0> { static constexpr int MR = 8, NC = 1, OCC = 2; static constexpr bool LIMB = true; };
template <> struct ShapeOf<1> { static constexpr int MR = 4, NC = 2, OCC = 2; static constexpr bool LIMB = true; };
template <> struct ShapeOf<2> { static constexpr int MR = 4, NC = 1, OCC = 3; static constexpr bool LIMB = true; };
template <> struct ShapeOf<3> { static constexpr int MR = 2, NC = 1, OCC = 2; static constexpr bool LIMB = false; };
template <> struct ShapeOf<4> { static constexpr int MR = 8, NC = 2, OCC = 1; static constexpr bool LIMB = true; };
// OCC = 0 marks the K-split kernels (ell x H waves per workgroup).
template <> struct ShapeOf<5> { static constexpr int MR = 2, NC = 1, OCC = 0, H = 1; static constexpr bool LIMB = false; };
template <> struct ShapeOf<6> { static constexpr int MR = 1, NC = 1, OCC = 0, H = 1; static constexpr bool LIMB = false; };
template <> struct ShapeOf<7> { static constexpr int MR = 1, NC = 1, OCC = 0, H = 2; static constexpr bool LIMB = false; };

template <int V>
static void launch_g1(const MfmaArgs &a, int party, int bit, int live, int GT, int NB, hipStream_t s) {
    using S = ShapeOf<V>;
    if constexpr (S::OCC == 0) {
        const unsigned g = (unsigned)(2 * live * (NB / S::MR) * GT);
        hipLaunchKernelGGL((mfma_gemm1_split_kernel<S::MR, S::H>), dim3(g), dim3(64 * a.ell * S::H), 0, s, a,
                           party, bit, live);
    } else if constexpr (S::LIMB) {
        const unsigned g = (unsigned)(2 * live * (NB / S::MR) * ((GT + S::NC - 1) / S::NC));
        hipLaunchKernelGGL((mfma_gemm1_limb_kernel<S::MR, S::NC, S::OCC>), dim3(g), dim3(256), 0, s, a, party,
                           bit, live);
    } else {
        const int GG = (GT + kWaves * S::NC - 1) / (kWaves * S::NC);
        const unsigned g = (unsigned)(2 * live * (NB / S::MR) * GG);
        hipLaunchKernelGGL((mfma_gemm1_kernel<S::MR, S::NC, S::OCC>), dim3(g), dim3(64 * kWaves), 0, s,
                           a, party, bit, live);
    }
}
template <int V>
static void launch_g2(const MfmaArgs &a, int party, int bit, int GT, int NB, hipStream_t s) {
    using S = ShapeOf<V>;
    if constexpr (S::OCC == 0) {
        const unsigned g = (unsigned)(2 * (NB / S::MR) * GT);
        hipLaunchKernelGGL((mfma_gemm2_split_kernel<S::MR, S::H>), dim3(g), dim3(64 * a.ell * S::H), 0, s, a,
                           party, bit);
    } else if constexpr (S::LIMB) {
        const unsigned g = (unsigned)(2 * (NB / S::MR) * ((GT + S::NC - 1) / S::NC));
        hipLaunchKernelGGL((mfma_gemm2_limb_kernel<S::MR, S::NC, S::OCC>), dim3(g), dim3(256), 0, s, a, party,
                           bit);
    } else {
        const int GG = (GT + kWaves * S::NC - 1) / (kWaves * S::NC);
        const unsigned g = (unsigned)(2 * (NB / S::MR) * GG);
        hipLaunchKernelGGL((mfma_gemm2_kernel<S::MR, S::NC, S::OCC>), dim3(g), dim3(64 * kWaves), 0, s,
                           a, party, bit);
    }
}
static void gemm1(int v, const MfmaArgs &a, int party, int bit, int live, int GT, int NB, hipStream_t s) {
    switch (v) {
        case 1: launch_g1<1>(a, party, bit, live, GT, NB, s); break;
        case 2: launch_g1<2>(a, party, bit, live, GT, NB, s); break;
        case 3: launch_g1<3>(a, party, bit, live, GT, NB, s); break;
        case 4: launch_g1<4>(a, party, bit, live, GT, NB, s); break;
        case 5: launch_g1<5>(a, party, bit, live, GT, NB, s); break;
        case 6: launch_g1<6>(a, party, bit, live, GT, NB, s); break;
        case 7: launch_g1<7>(a, party, bit, live, GT, NB, s); break;
        default: launch_g1<0>(a, party, bit, live, GT, NB, s);
    }
}
static void gemm2(int v, const MfmaArgs &a, int party, int bit, int GT, int NB, hipStream_t s) {
    switch (v) {
        case 1: launch_g2<1>(a, party, bit, GT, NB, s); break;
        case 2: launch_g2<2>(a, party, bit, GT, NB, s); break;
        case 3: launch_g2<3>(a, party, bit, GT, NB, s); break;
        case 4: launch_g2<4>(a, party, bit, GT, NB, s); break;
        case 5: launch_g2<5>(a, party, bit, GT, NB, s); break;
        case 6: launch_g2<6>(a, party, bit, GT, NB, s); break;
        case 7: launch_g2<7>(a, party, bit, GT, NB, s); break;
        default: launch_g2<0>(a, party, bit, GT, NB, s);
    }
}

__global__ void mfma_copyout_kernel(const uint32_t *__restrict__ src, uint32_t *__restrict__ dst,
                                    size_t words) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < words) dst[idx] = src[idx];
}

static inline unsigned blocks(size_t threads, int per) { return (unsigned)((threads + per - 1) / per); }

// Scratch bytes of the rotation for `count` gates: accumulator, partial
// sums W, digits U and V, and the persistent rotation's control words.
size_t mfma_scratch_need(const mk_params &P, size_t count) {
    const size_t GP = (count + 31) / 32 * 32;
    const size_t K1 = P.k + 1, N = P.N, ell = P.bk_ell;
    return GP * K1 * N * 4 + K1 * GP * N * 4 + K1 * ell * GP * N + ell * GP * N +
           persist_ctl_words((int)(GP / 32)) * 4;
}

// Control words of a part: right after its V digits.
static uint32_t *ctl_of(const MfmaArgs &a) {
    return (uint32_t *)(a.V + (size_t)a.ell * a.GP * a.N);
}

// Whether the persistent rotation runs a batch of GT gate tiles: by choice
// (mk_set_rotation), else at N = 1024 from one tile per XCD on (the team
// size then follows the batch width, persist_team_rows), and at other N from
// 2.5 tiles per XCD on.  Measured on MI355X at the Table 7 shape, stream-
// ordered against persistent (ms per batch, team size in brackets): 128
// gates 37.8 / 49.4 (32), 256 gates 50.6 / 45.6 (32), 384 gates 66.5 / 53.0
// (16), 512 gates 72.9 / 58.8 (16), 640 gates 81.7 / 76.6 (8), 768 gates
// 92.4 / 79.4 (8), 1024 gates 101.6 / 88.0 (8).  Below one tile per XCD
// whole XCDs would idle, while the stream-ordered kernels split a tile over
// many compute units.
bool use_persist(const mk_ctx *ctx, int GT) {
    const DeviceKeys &D = ctx->dev;
    if (D.rot_kind == MK_ROT_STREAM || D.num_xcd <= 0 || !persist_supported(ctx->p)) return false;
    if (D.rot_kind == MK_ROT_PERSISTENT) return true;
    return ctx->p.N == 1024 ? GT >= D.num_xcd : 2 * GT >= 5 * D.num_xcd;
}

// Gates of the first part when an automatic persistent rotation of `count`
// gates is better run as two consecutive launches, else `count`.  At N =
// 1024 an XCD holds U = (its compute units) / 8 teams of 8 workgroups; with
// more than U tiles on an XCD some teams run two or more tiles phase by
// phase.  When the tiles beyond the last full round are at most one per
// XCD, the batch runs as the full rounds, then the remainder as its own
// launch (teams of 32, or the stream-ordered kernels below one tile per
// XCD).  Measured at the Table 7 shape, one launch against two: 1100 gates
// 139.9 / 127.4 ms, 1280 gates 143.8 / 133.3; with larger remainders one
// launch is as fast or faster (1536 gates 147.3 / 146.6, 1792 gates
// 163.1 / 167.5, 2400 gates 225.1 / 228.5), since a team running two
// tiles pays its barriers and pipeline fills once for both.
size_t mfma_rotation_split(const mk_ctx *ctx, size_t count) {
    const DeviceKeys &D = ctx->dev;
    const int GT = (int)((count + 31) / 32);
    if (ctx->p.N != 1024 || D.rot_kind != MK_ROT_AUTO || D.team_rows || !use_persist(ctx, GT)) return count;
    const int round = D.num_xcd * std::max(1, D.num_cus / D.num_xcd / 8);   // tiles of one full round
    const int rem = GT % round;
    if (GT <= round || rem == 0 || rem > D.num_xcd) return count;
    return (size_t)(GT - rem) * 32;
}

// Sub-batches of a rotation: a batch can be split in two halves that run on
// two streams, so that one half's memory-bound digit kernels and GEMM tails
// overlap the other half's GEMMs.  The split is chosen by the autotuner per
// batch size; untuned batches are not split.
struct Split {
    int parts;
    size_t cnt[2], off[2];
};
static Split split_for(const mk_ctx *ctx, size_t count) {
    Split sp{1, {count, 0}, {0, 0}};
    const int GT = (int)((count + 31) / 32);
    auto it = ctx->dev.tuned_parts.find(GT);
    if (!ctx->dev.fixed_scratch && it != ctx->dev.tuned_parts.end() && it->second == 2 && GT >= 2) {
        sp.parts = 2;
        sp.cnt[0] = (size_t)((GT + 1) / 2) * 32;
        sp.cnt[1] = count - sp.cnt[0];
        sp.off[1] = sp.cnt[0];
    }
    return sp;
}

// Allocates (grows) the MFMA scratch for the parts of `sp` and fills their
// kernel arguments (part i: gates off[i] .. off[i] + cnt[i] - 1).
static int prepare(mk_ctx *ctx, const uint32_t *abar, const Split &sp, hipStream_t s, MfmaArgs *a) {
    const mk_params &P = ctx->p;
    if (P.N < 128) return fail(MK_EPARAM, "int8-MFMA path needs N >= 128");
    const int K1 = P.k + 1, N = P.N, ell = P.bk_ell;
    size_t need = 0;
    for (int i = 0; i < sp.parts; ++i) {
        const size_t GP = (sp.cnt[i] + 31) / 32 * 32;
        // the GEMMs address a key polynomial's digit block with 32-bit offsets
        if ((size_t)K1 * ell * GP * N >= ((size_t)1 << 31))
            return fail(MK_EINVAL, "int8-MFMA path: batch too large for one launch (split it)");
        need += mfma_scratch_need(P, sp.cnt[i]);
    }
    DeviceKeys &D = ctx->dev;
    if (D.mfma_scratch_bytes < need) {
        if (D.fixed_scratch) return fail(MK_EINTERNAL, "fixed scratch block too small (MFMA rotation)");
        if (D.mfma_scratch) {
            MK_HIP(hipDeviceSynchronize(), "mfma scratch sync");
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
    char *sp_base = (char *)D.mfma_scratch;
    for (int i = 0; i < sp.parts; ++i) {
        const size_t GP = (sp.cnt[i] + 31) / 32 * 32;
        const size_t acc_b = GP * K1 * N * 4, w_b = (size_t)K1 * GP * N * 4;
        const size_t u_b = (size_t)K1 * ell * GP * N;
        MfmaArgs &x = a[i];
        x.k = P.k; x.n = P.n; x.N = N; x.ell = ell; x.log2N = __builtin_ctz(N);
        x.GP = (int)GP; x.G = (int)sp.cnt[i];
        x.offset = decomp_offset(ell);
        x.abar = abar ? abar + sp.off[i] * ((size_t)P.k * P.n + 1) : nullptr;
        x.acc = (uint32_t *)sp_base;
        x.W = (uint32_t *)(sp_base + acc_b);
        x.U = (int8_t *)(sp_base + acc_b + w_b);
        x.V = (int8_t *)(sp_base + acc_b + w_b + u_b);
        x.bk = D.bk_win;
        x.evk = D.evk_win;
        sp_base += mfma_scratch_need(P, sp.cnt[i]);
    }
    return MK_OK;
}

// First shape whose row block divides N/32.
static int default_shape(int NB) {
    for (int v = 0; v < kNumShapes; ++v)
        if (NB % kShapes[v].MR == 0) return v;
    return kNumShapes - 1;
}

// Untuned shapes by batch size, from timings at N = 1024 on MI355X: K-split
// shapes while a launch covers few CUs, then the skewed shape, then the
// first limb-split shape that fits (stage 2, with a third of stage 1's
// products, keeps the skewed shape).
static void default_shapes(int NB, int GT, int &v1, int &v2) {
    v1 = GT <= 2 ? 6 : GT <= 4 ? 5 : GT <= 12 ? 3 : default_shape(NB);
    v2 = GT <= 4 ? 6 : GT <= 12 ? 5 : 3;
}

// Tile shapes for a batch of GT gate tiles: forced by mk_set_tiles, else the
// autotuned choice for this size, else the default.
static void shapes_for(const mk_ctx *ctx, int GT, int &v1, int &v2) {
    const DeviceKeys &D = ctx->dev;
    default_shapes(ctx->p.N / 32, GT, v1, v2);
    auto it = D.tuned_tiles.find(GT);
    if (it != D.tuned_tiles.end()) {
        v1 = it->second.first;
        v2 = it->second.second;
    }
    if (D.force_tiles[0] >= 0) v1 = D.force_tiles[0];
    if (D.force_tiles[1] >= 0) v2 = D.force_tiles[1];
}

// Enqueues CMux steps st0 .. st1-1 of every part, part i on stream ss[i].
static int enqueue_steps(mk_ctx *ctx, const MfmaArgs *a, int parts, hipStream_t *ss, int st0, int st1) {
    const mk_params &P = ctx->p;
    const int K1 = P.k + 1, NB = P.N / 32;
    const size_t rows_lds = (size_t)8 * P.N * 4;   // rotdec: 8 accumulator rows
    int GT[2], v1[2], v2[2];
    for (int i = 0; i < parts; ++i) {
        GT[i] = a[i].GP / 32;
        shapes_for(ctx, GT[i], v1[i], v2[i]);
    }
    for (int st = st0; st < st1; ++st) {
        const int party = st / P.n, bit = st % P.n;
        // ACC starts as (X^-b v, 0, .., 0) and during party i's steps only
        // c'_0 and c'_{1+i} receive stage-2 output, while c'_j = 0 whenever
        // ACC_j = 0 (its digits are all zero).  So slots j >= i+2 are still
        // exactly zero: their digits, products and partial sums are skipped.
        const int live = std::min(K1, party + 2);
        for (int i = 0; i < parts; ++i) {
            hipStream_t s = ss[i];
            {
                StageTimer t6(ctx, 6, s);
                hipLaunchKernelGGL(mfma_rotdec_kernel, dim3((unsigned)(live * GT[i] * 4)), dim3(kRotdecThreads),
                                   rows_lds, s, a[i], st);
            }
            {
                StageTimer t4(ctx, 4, s);
                gemm1(v1[i], a[i], party, bit, live, GT[i], NB, s);
            }
            {
                StageTimer t7(ctx, 7, s);
                hipLaunchKernelGGL(mfma_wdec_kernel, dim3((unsigned)(GT[i] * NB / 4)), dim3(256), 0, s,
                                   a[i], live);
            }
            {
                StageTimer t5(ctx, 5, s);
                gemm2(v2[i], a[i], party, bit, GT[i], NB, s);
            }
        }
        if (ctx->dev.capture) {
            int rc = capture_checkpoint(ctx, ss[0], 4 * parts);
            if (rc) return rc;
        }
    }
    MK_HIP(hipGetLastError(), "mfma step launch");
    return MK_OK;
}

// Streams for the parts: the caller's stream when not split; otherwise two
// auxiliary streams (default priority) that wait for the caller's stream
// and that the caller's stream later waits for (join_parts).
static int fork_parts(mk_ctx *ctx, int parts, hipStream_t s, hipStream_t *ss) {
    if (parts == 1) {
        ss[0] = s;
        return MK_OK;
    }
    DeviceKeys &D = ctx->dev;
    for (int i = 0; i < 2; ++i)
        if (!D.aux_stream[i])
            MK_HIP(hipStreamCreateWithFlags((hipStream_t *)&D.aux_stream[i], hipStreamNonBlocking), "aux stream");
    for (int i = 0; i < 3; ++i)
        if (!D.aux_event[i])
            MK_HIP(hipEventCreateWithFlags((hipEvent_t *)&D.aux_event[i], hipEventDisableTiming), "aux event");
    MK_HIP(hipEventRecord((hipEvent_t)D.aux_event[0], s), "fork record");
    for (int i = 0; i < 2; ++i) {
        ss[i] = (hipStream_t)D.aux_stream[i];
        MK_HIP(hipStreamWaitEvent(ss[i], (hipEvent_t)D.aux_event[0], 0), "fork wait");
    }
    return MK_OK;
}
static int join_parts(mk_ctx *ctx, int parts, hipStream_t s, hipStream_t *ss) {
    if (parts == 1) return MK_OK;
    DeviceKeys &D = ctx->dev;
    for (int i = 0; i < 2; ++i) {
        MK_HIP(hipEventRecord((hipEvent_t)D.aux_event[1 + i], ss[i]), "join record");
        MK_HIP(hipStreamWaitEvent(s, (hipEvent_t)D.aux_event[1 + i], 0), "join wait");
    }
    return MK_OK;
}

int launch_br_mfma(mk_ctx *ctx, const uint32_t *abar, uint32_t *acc_out, size_t count, int steps,
                   hipStream_t s, uint32_t *ks_out, size_t ks_stride, bool *ks_done) {
    const mk_params &P = ctx->p;
    Split sp = split_for(ctx, count);
    // per-kernel timing and graph capture see a single stream
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (ctx->dev.profiling >= 2 || hipStreamIsCapturing(s, &cap) != hipSuccess ||
        cap != hipStreamCaptureStatusNone)
        sp = Split{1, {count, 0}, {0, 0}};
    const bool persist = use_persist(ctx, (int)((count + 31) / 32));
    if (persist) sp = Split{1, {count, 0}, {0, 0}};
    MfmaArgs a[2];
    int rc = prepare(ctx, abar, sp, s, a);
    if (rc) return rc;
    const int K1 = P.k + 1, N = P.N;
    StageTimer tm(ctx, 1, s);
    if (persist) {
        hipLaunchKernelGGL(mfma_init_kernel, dim3(blocks((size_t)a[0].GP * K1 * N, 256)), dim3(256), 0, s, a[0]);
        MK_HIP(hipGetLastError(), "mfma init launch");
        // extraction and key switching inside the launch: each team runs
        // them on its own tiles right after their last CMux step
        const bool fuse = ks_out && ks_done && ctx->dev.ks_fuse && ctx->dev.ks_win && steps == P.k * P.n;
        KsFused kf;
        if (fuse && (rc = ks_fused_args(ctx, count, ks_out, ks_stride, s, &kf))) return rc;
        {
            StageTimer tp(ctx, 4, s);
            if ((rc = launch_persist(ctx, a[0], steps, ctl_of(a[0]), fuse ? &kf : nullptr, s))) return rc;
        }
        if (fuse) {
            *ks_done = true;
            return MK_OK;
        }
        const size_t words = count * K1 * N;
        hipLaunchKernelGGL(mfma_copyout_kernel, dim3(blocks(words, 256)), dim3(256), 0, s, a[0].acc, acc_out,
                           words);
        MK_HIP(hipGetLastError(), "mfma copyout launch");
        return MK_OK;
    }
    hipStream_t ss[2];
    if ((rc = fork_parts(ctx, sp.parts, s, ss))) return rc;
    for (int i = 0; i < sp.parts; ++i) {
        hipLaunchKernelGGL(mfma_init_kernel, dim3(blocks((size_t)a[i].GP * K1 * N, 256)), dim3(256), 0, ss[i],
                           a[i]);
        MK_HIP(hipGetLastError(), "mfma init launch");
    }
    if ((rc = enqueue_steps(ctx, a, sp.parts, ss, 0, steps))) return rc;
    for (int i = 0; i < sp.parts; ++i) {
        const size_t words = sp.cnt[i] * K1 * N;
        hipLaunchKernelGGL(mfma_copyout_kernel, dim3(blocks(words, 256)), dim3(256), 0, ss[i], a[i].acc,
                           acc_out + sp.off[i] * K1 * N, words);
        MK_HIP(hipGetLastError(), "mfma copyout launch");
    }
    return join_parts(ctx, sp.parts, s, ss);
}

// Times every tile shape of both GEMMs on the scratch buffers of `count`
// gates (contents irrelevant: only durations are read) and records the
// fastest for that batch size.
static int tune_shapes(mk_ctx *ctx, size_t count, hipStream_t s, hipEvent_t e0, hipEvent_t e1, int *pick,
                       float *ms_out) {
    const mk_params &P = ctx->p;
    MfmaArgs a;
    int rc = prepare(ctx, nullptr, Split{1, {count, 0}, {0, 0}}, s, &a);
    if (rc) return rc;
    const int NB = P.N / 32, GT = a.GP / 32;
    const int party = P.k - 1, live = std::min(P.k + 1, party + 2);
    constexpr int kReps = 4;
    float best[2] = {3.0e38f, 3.0e38f};
    default_shapes(NB, GT, pick[0], pick[1]);
    for (int which = 0; which < 2; ++which)
        for (int v = 0; v < kNumShapes; ++v) {
            if (NB % kShapes[v].MR) continue;
            auto run = [&]() {
                if (which == 0) gemm1(v, a, party, 0, live, GT, NB, s);
                else gemm2(v, a, party, 0, GT, NB, s);
            };
            run();  // warm-up
            MK_HIP(hipEventRecord(e0, s), "autotune record");
            for (int r = 0; r < kReps; ++r) run();
            MK_HIP(hipEventRecord(e1, s), "autotune record");
            float ms = 0;
            MK_HIP(hipEventSynchronize(e1), "autotune sync");
            MK_HIP(hipEventElapsedTime(&ms, e0, e1), "autotune timing");
            if (ms_out) ms_out[which * kNumShapes + v] = ms / kReps;
            if (ms < best[which]) {
                best[which] = ms;
                pick[which] = v;
            }
        }
    MK_HIP(hipGetLastError(), "autotune launch");
    ctx->dev.tuned_tiles[GT] = {pick[0], pick[1]};
    return MK_OK;
}

// Average time of `steps` CMux steps of party k-1 on `count` gates run as
// `parts` sub-batches (abar all zero: the shifts do not change the work).
static int time_steps(mk_ctx *ctx, size_t count, int parts, const uint32_t *abar, hipStream_t s,
                      hipEvent_t e0, hipEvent_t e1, float *ms) {
    const mk_params &P = ctx->p;
    Split sp{1, {count, 0}, {0, 0}};
    if (parts == 2) {
        const size_t GT = (count + 31) / 32;
        sp = Split{2, {(GT + 1) / 2 * 32, 0}, {0, (GT + 1) / 2 * 32}};
        sp.cnt[1] = count - sp.cnt[0];
    }
    MfmaArgs a[2];
    int rc = prepare(ctx, abar, sp, s, a);
    if (rc) return rc;
    hipStream_t ss[2];
    const int st0 = (P.k - 1) * P.n, nsteps = std::min(8, P.n);
    for (int rep = 0; rep < 2; ++rep) {  // first pass warms up
        MK_HIP(hipEventRecord(e0, s), "autotune record");
        if ((rc = fork_parts(ctx, sp.parts, s, ss)) || (rc = enqueue_steps(ctx, a, sp.parts, ss, st0, st0 + nsteps)) ||
            (rc = join_parts(ctx, sp.parts, s, ss)))
            return rc;
        MK_HIP(hipEventRecord(e1, s), "autotune record");
        MK_HIP(hipEventSynchronize(e1), "autotune sync");
    }
    MK_HIP(hipEventElapsedTime(ms, e0, e1), "autotune timing");
    *ms /= nsteps;
    return MK_OK;
}

// Tile shapes for `count` gates and for its half, then whether a batch of
// `count` runs faster whole or as two sub-batches on two streams.
int autotune(mk_ctx *ctx, size_t count, hipStream_t s, int *v1_out, int *v2_out, float *ms_out) {
    const mk_params &P = ctx->p;
    DeviceKeys &D = ctx->dev;
    count = std::min(count, rotation_chunk(P));  // larger batches run in chunks of this size
    hipEvent_t e0, e1;
    MK_HIP(hipEventCreate(&e0), "autotune event");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(MK_EDEVICE, "autotune event");
    }
    const int saved_prof = D.profiling;
    D.profiling = 0;
    int pick[2], pick_half[2];
    int rc = tune_shapes(ctx, count, s, e0, e1, pick, ms_out);
    const size_t GT = (count + 31) / 32;
    uint32_t *abar = nullptr;
    float whole = 0, split = 0;
    if (!rc && GT >= 2) {
        const size_t half = (GT + 1) / 2 * 32;
        rc = tune_shapes(ctx, half, s, e0, e1, pick_half, nullptr);
        const size_t words = count * ((size_t)P.k * P.n + 1);
        if (!rc && hipMalloc((void **)&abar, words * 4) != hipSuccess) {
            abar = nullptr;
            rc = fail(MK_ENOMEM, "autotune: device allocation failed");
        }
        if (!rc && hipMemsetAsync(abar, 0, words * 4, s) != hipSuccess) rc = fail(MK_EDEVICE, "autotune memset");
        if (!rc) rc = time_steps(ctx, count, 1, abar, s, e0, e1, &whole);
        if (!rc) rc = time_steps(ctx, count, 2, abar, s, e0, e1, &split);
        if (!rc) D.tuned_parts[(int)GT] = split < whole ? 2 : 1;
    }
    if (abar) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(abar);
    }
    D.profiling = saved_prof;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
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

int mk_set_split(mk_ctx *ctx, size_t count, int parts) {
    if (!ctx || !count || parts < 0 || parts > 2) return fail(MK_EINVAL, "mk_set_split: bad argument");
    const int GT = (int)((count + 31) / 32);
    if (parts == 0) ctx->dev.tuned_parts.erase(GT);
    else ctx->dev.tuned_parts[GT] = parts;
    return MK_OK;
}

int mk_get_split(const mk_ctx *ctx, size_t count, int32_t *parts) {
    if (!ctx || !parts) return fail(MK_EINVAL, "mk_get_split: bad argument");
    *parts = split_for(ctx, count).parts;
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
