// Declarations shared by the device translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "mk_internal.h"

namespace mk {

// Offset of the signed base-2^8 gadget decomposition with `ell` digits:
// 2^(31-8 ell) (rounding) + sum_p 2^(32-8p) * 2^7 (digit bias), so that
// digit_p = ((x + offset) >> (32-8p) & 255) - 128.
__host__ __device__ inline uint32_t decomp_offset(int ell) {
    uint32_t off = 1u << (31 - 8 * ell);
    for (int p = 1; p <= ell; ++p) off += 128u << (32 - 8 * p);
    return off;
}

int hip_fail(hipError_t e, const char *what);

// Bits of the context's sticky device status word (DeviceKeys::status).
constexpr uint32_t kStatusTimeout = 1u;   // a persistent rotation gave up waiting
constexpr uint32_t kStatusNoXcd = 2u;     // it ran on an XCD the probe did not see
constexpr uint32_t kStatusBadType = 4u;   // a gate type outside NAND..XNOR

// Brackets a kernel launch with profiling events when enabled.
struct StageTimer {
    StageTimer(mk_ctx *ctx, int stage, hipStream_t s);
    ~StageTimer();
    mk_ctx *ctx;
    int stage;
    hipStream_t s;
    hipEvent_t b = nullptr, e = nullptr;
};
int ensure_scratch(mk_ctx *ctx, size_t bytes);
// Gates per rotation launch (mk_device.hip): larger batches and circuit
// levels run in chunks of this size.
size_t rotation_chunk(const mk_params &P);

// Int8-MFMA path (mk_mfma.hip).
int mfma_upload(mk_ctx *ctx, const std::vector<uint32_t> &evk, hipStream_t s);
// With `ks_out` given and a full rotation (steps = k n) on the persistent
// schedule with key-switch fusion on, extraction and key switching into
// ks_out run inside the rotation's launch and *ks_done is set (acc is then
// left untouched); otherwise the caller runs them.
int launch_br_mfma(mk_ctx *ctx, const uint32_t *abar, uint32_t *acc, size_t count, int steps,
                   hipStream_t s, uint32_t *ks_out = nullptr, size_t ks_stride = 0, bool *ks_done = nullptr);
size_t mfma_scratch_need(const mk_params &P, size_t count);
// Whether a rotation of GT gate tiles runs on the persistent schedule.
bool use_persist(const mk_ctx *ctx, int GT);
// Gates of the first of two consecutive rotation launches for a batch of
// `count` (count itself when one launch is best).
size_t mfma_rotation_split(const mk_ctx *ctx, size_t count);
// Persistent rotation (mk_persist.hip).
struct MfmaArgs;
struct KsFused;
int persist_probe(mk_ctx *ctx, hipStream_t s);
size_t persist_ctl_words(int GT);
bool persist_supported(const mk_params &P);
int persist_team_rows(const mk_ctx *ctx, int GT);
int launch_persist(mk_ctx *ctx, const MfmaArgs &m, int steps, uint32_t *ctl, const KsFused *ks, hipStream_t s);
// Key switching as an int8-MFMA GEMM (mk_keyswitch.hip).
size_t ks_scratch_need(const mk_params &P, size_t count);
int ks_mfma_upload(mk_ctx *ctx, hipStream_t s);
int launch_ks_mfma(mk_ctx *ctx, const uint32_t *acc, uint32_t *out, size_t count, size_t stride,
                   hipStream_t s);
// Arguments of the key switching fused into a persistent rotation of
// `count` gates (grows the rounded-coefficient scratch).
int ks_fused_args(mk_ctx *ctx, size_t count, uint32_t *out, size_t stride, hipStream_t s, KsFused *f);
// During a graph capture: ends the current graph after enough kernels and
// begins the next one on the same stream (mk_engine.hip).
int capture_checkpoint(mk_ctx *ctx, hipStream_t s, int kernels);
// The whole gate pipeline on `count` gates (mk_device.hip).
int run_gates(mk_ctx *ctx, const uint8_t *types, const uint32_t *in1, const uint32_t *in2,
              uint32_t *out, size_t count, size_t stride, int path, hipStream_t s);
// Blind rotation of `count` gates, then sample extraction and key switching
// into `out` (fused into the rotation's launch where that applies).
int run_rotate_ks(mk_ctx *ctx, const uint32_t *abar, uint32_t *acc, uint32_t *out, size_t count, size_t stride,
                  int path, hipStream_t s);
// Sample extraction + key switching on the given path (mk_device.hip).
int run_key_switch(mk_ctx *ctx, const uint32_t *acc, uint32_t *out, size_t count, size_t stride, int path,
                   hipStream_t s);

}  // namespace mk
