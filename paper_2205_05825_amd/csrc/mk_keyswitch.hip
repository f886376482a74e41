// Key switching on the int8-MFMA path (§3.2 MKKeySwitch) as one exact
// integer GEMM per party: the key tiles are built at upload, then each
// batch runs an extraction-and-rounding kernel and the GEMM kernel (the
// arithmetic, layouts and exactness bound are described in mk_ks_core.h).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mk_device_common.h"
#include "mk_ks_core.h"

namespace mk {

#define MK_HIP(call, what)                               \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

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

// Extraction and rounding, one block per (gate tile, 64 coefficients,
// party): ks_round_unit.
__global__ __launch_bounds__(256) void ks_round_kernel(const uint32_t *__restrict__ acc, KsShape s,
                                                       size_t count, uint32_t *__restrict__ R,
                                                       uint32_t *__restrict__ out, size_t stride) {
    __shared__ uint32_t tile[32 * 65];
    ks_round_unit<false>(acc, s, count, R, out, stride, blockIdx.x, blockIdx.y * 64, blockIdx.z, tile);
}

// One ks_gemm_task per workgroup.  Tasks (party, column block, gate tile)
// are numbered with the gate tile fastest, and each XCD runs one contiguous
// range of them: workgroup b runs on XCD b mod nx (round-robin dispatch),
// so task = (b mod nx) per + b / nx.  A column block's key tiles (12 MB at
// the Table 7 shape) are then fetched by at most two XCDs' L2s, instead of
// by every XCD.
template <bool LB2>
__global__ __launch_bounds__(256, 2) void ks_gemm_kernel(const int8_t *__restrict__ tiles,
                                                         const uint32_t *__restrict__ R, KsShape s,
                                                         size_t count, uint32_t *__restrict__ out,
                                                         size_t stride, int nx, int per) {
    __shared__ __align__(16) uint4 red[kKsGemmLds / 16];
    const int GT = s.GP / 32, CB = ks_col_blocks(s);
    int task = (int)(blockIdx.x % (unsigned)nx) * per + (int)(blockIdx.x / (unsigned)nx);
    if (task >= s.k * CB * GT) return;
    const int gt = task % GT;
    task /= GT;
    ks_gemm_task<LB2, 0>(tiles, R, s, count, out, stride, gt, task % CB, task / CB, red);
}

size_t ks_scratch_need(const mk_params &P, size_t count) {
    return (size_t)P.k * P.N * ((count + 31) / 32 * 32) * 4;
}

// Grows the rounded-coefficient scratch R to `count` gates (never while the
// scratch is a caller-fixed block).
static int ensure_ks_scratch(mk_ctx *ctx, size_t count, hipStream_t s) {
    DeviceKeys &D = ctx->dev;
    const size_t need = ks_scratch_need(ctx->p, count);
    if (D.ks_scratch_bytes >= need) return MK_OK;
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
    return MK_OK;
}

static int ks_check(const mk_params &P, size_t GP) {
    if (P.N < kKsRing || (size_t)P.N * GP * 4 >= ((size_t)1 << 31))
        return fail(MK_EINVAL, "int8-MFMA key switching: batch too large for one launch (split it)");
    return MK_OK;
}

int ks_fused_args(mk_ctx *ctx, size_t count, uint32_t *out, size_t stride, hipStream_t s, KsFused *f) {
    const mk_params &P = ctx->p;
    DeviceKeys &D = ctx->dev;
    if (!D.ks_win) return fail(MK_EINTERNAL, "fused key switching without key-switching tiles");
    const size_t GP = (count + 31) / 32 * 32;
    int rc = ks_check(P, GP);
    if (!rc) rc = ensure_ks_scratch(ctx, count, s);
    if (rc) return rc;
    f->tiles = D.ks_win;
    f->R = (uint32_t *)D.ks_scratch;
    f->out = out;
    f->stride = stride;
    f->count = count;
    f->s = ks_shape(P, GP);
    return MK_OK;
}

int launch_ks_mfma(mk_ctx *ctx, const uint32_t *acc, uint32_t *out, size_t count, size_t stride,
                   hipStream_t s) {
    const mk_params &P = ctx->p;
    DeviceKeys &D = ctx->dev;
    const size_t GP = (count + 31) / 32 * 32;
    const KsShape sh = ks_shape(P, GP);
    int rc = ks_check(P, GP);
    if (!rc) rc = ensure_ks_scratch(ctx, count, s);
    if (rc) return rc;
    uint32_t *R = (uint32_t *)D.ks_scratch;
    const int GT = (int)(GP / 32), CB = ks_col_blocks(sh);
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
