// Gate bootstrapping that allocates nothing: mk_bootstrap_gate with every
// scratch buffer of the pipeline (modulus-switched inputs, accumulators,
// the MFMA rotation's partial sums, digit planes and control words, the key
// switch's rounded coefficients) placed in one fixed device array.
//
// The array is a file-scope __device__ variable, so every GPU the library
// runs on holds its own copy from module load until the process ends.  Its
// device address is looked up once per device (with that device current)
// and only that address is handed to kernels; the host-side name of the
// array is never used as a device pointer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "mk_device_common.h"

namespace mk {

constexpr size_t kNoAllocBytes = (size_t)64 << 20;   // MK_NOALLOC_SCRATCH_BYTES
constexpr int kNoAllocDevices = 64;

__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

std::mutex g_addr_mu;
void *g_addr[kNoAllocDevices] = {};

// Device address of `scratch` on the current device `dev`.
int scratch_address(int dev, void **out) {
    if (dev < 0 || dev >= kNoAllocDevices) return fail(MK_EINVAL, "mk_bootstrap_gate_noalloc: device index out of range");
    std::lock_guard<std::mutex> lock(g_addr_mu);
    if (!g_addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch symbol address");
        g_addr[dev] = p;
    }
    *out = g_addr[dev];
    return MK_OK;
}

inline size_t round256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

// Bytes of the three regions for a batch of `count` gates on `path` (the
// gate pipeline runs chunks of at most rotation_chunk gates, unsplit).
static void noalloc_layout(const mk_ctx *ctx, size_t count, int path, size_t sz[3]) {
    const mk_params &P = ctx->p;
    const size_t chunk = std::min(count, rotation_chunk(P));
    const size_t abar_b = (chunk * lwe_words(P) * 4 + 255) / 256 * 256;
    sz[0] = round256(abar_b + chunk * (P.k + 1) * P.N * 4);
    const bool mfma = path == MK_PATH_MFMA_I8;
    sz[1] = mfma ? round256(mfma_scratch_need(P, chunk)) : 0;
    sz[2] = mfma && ctx->dev.ks_win ? round256(ks_scratch_need(P, chunk)) : 0;
}

}  // namespace mk

using namespace mk;

extern "C" {

int mk_bootstrap_gate_noalloc(mk_ctx *ctx, const uint8_t *types, const uint32_t *in1, const uint32_t *in2,
                              uint32_t *out, size_t count, size_t stride, int path, void *stream) {
    if (!ctx) return fail(MK_EINVAL, "mk_bootstrap_gate_noalloc: null context");
    if (count && (!types || !in1 || !in2 || !out))
        return fail(MK_EINVAL, "mk_bootstrap_gate_noalloc: null pointer");
    if (stride < lwe_words(ctx->p)) return fail(MK_EINVAL, "mk_bootstrap_gate_noalloc: stride < kn+1");
    if (path != MK_PATH_I32 && path != MK_PATH_MFMA_I8)
        return fail(MK_EINVAL, "mk_bootstrap_gate_noalloc: bad path");
    DeviceKeys &D = ctx->dev;
    if (!D.uploaded) return fail(MK_ESTATE, "evaluation key not uploaded (mk_upload_eval_key)");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != D.device)
        return fail(MK_ESTATE, "current HIP device differs from the upload device");
    size_t sz[3];
    noalloc_layout(ctx, count, path, sz);
    if (sz[0] + sz[1] + sz[2] > kNoAllocBytes)
        return fail(MK_EINVAL, "mk_bootstrap_gate_noalloc: batch needs more scratch than the fixed 64 MiB "
                               "block (split the batch)");
    void *base = nullptr;
    int rc = scratch_address(dev, &base);
    if (rc) return rc;
    if (!count) return MK_OK;
    // point the context's scratch at the block for this call only; no
    // buffer is grown, the rotation is not split over streams, and no
    // profiling events are made
    void *save_p[3] = {D.scratch, D.mfma_scratch, D.ks_scratch};
    const size_t save_b[3] = {D.scratch_bytes, D.mfma_scratch_bytes, D.ks_scratch_bytes};
    const int save_prof = D.profiling;
    char *b = (char *)base;
    D.scratch = b;
    D.scratch_bytes = sz[0];
    D.mfma_scratch = sz[1] ? b + sz[0] : nullptr;
    D.mfma_scratch_bytes = sz[1];
    D.ks_scratch = sz[2] ? b + sz[0] + sz[1] : nullptr;
    D.ks_scratch_bytes = sz[2];
    D.fixed_scratch = true;
    D.profiling = 0;
    rc = run_gates(ctx, types, in1, in2, out, count, stride, path, (hipStream_t)stream);
    D.fixed_scratch = false;
    D.profiling = save_prof;
    D.scratch = save_p[0];
    D.scratch_bytes = save_b[0];
    D.mfma_scratch = save_p[1];
    D.mfma_scratch_bytes = save_b[1];
    D.ks_scratch = save_p[2];
    D.ks_scratch_bytes = save_b[2];
    return rc;
}

}  // extern "C"
