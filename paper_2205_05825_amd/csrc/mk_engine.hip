// Levelled evaluation of gate netlists (the k-bit operators of Algs. 3-6).
//
// Host analysis (once per call):
//   * each wire resolves to (base value, inverted?, constant?): NOT gates
//     (Eq. (8), no bootstrapping) and the constant wires are folded into the
//     consumers' pre-combination, which is exact mod 2^32:
//       s * NOT(c) = -s * c + s * (1/4 on b),  s * const(m) = s * m/4 on b;
//   * gates that no output depends on are dropped;
//   * every bootstrapped gate gets level 1 + max(level of its inputs);
//   * each level's outputs get one contiguous range of wire slots, allocated
//     first-fit over ranges freed after their last reader's level.
// Device work per level: pre-combination gathering both operands of every
// (gate, instance), one blind rotation over all of them, and extraction + key
// switching straight into the level's slot range.  Wire buffer layout:
// row (slot * batch + instance) of `stride` words.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <list>
#include <vector>

#include "mk_device_common.h"

namespace mk {

int run_blind_rotate(mk_ctx *ctx, const uint32_t *abar, uint32_t *acc, size_t count, int steps,
                     int path, hipStream_t s);

namespace {

struct CircDesc {
    int32_t slot1, slot2;  // -1: no ciphertext operand
    int32_t s1, s2;
    uint32_t cst;
    int32_t pad;
};

struct OutDesc {
    int32_t slot;  // -1: constant
    int32_t neg;
    uint32_t cst;  // constant bit when slot < 0
    int32_t pad;
};

__global__ void precombine_circuit_kernel(const CircDesc *__restrict__ desc,
                                          const uint32_t *__restrict__ wires, size_t batch,
                                          size_t stride, int words, int log2_2N, size_t total,
                                          uint32_t *__restrict__ abar) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const size_t item = idx / words;
    const int w = (int)(idx - item * words);
    const size_t g = item / batch, b = item - g * batch;
    const CircDesc d = desc[g];
    uint32_t x = w == 0 ? d.cst : 0u;
    if (d.slot1 >= 0) x += (uint32_t)d.s1 * wires[((size_t)d.slot1 * batch + b) * stride + w];
    if (d.slot2 >= 0) x += (uint32_t)d.s2 * wires[((size_t)d.slot2 * batch + b) * stride + w];
    abar[idx] = (x + (1u << (31 - log2_2N))) >> (32 - log2_2N);
}

__global__ void gather_outputs_kernel(const OutDesc *__restrict__ od,
                                      const uint32_t *__restrict__ wires, uint32_t *__restrict__ out,
                                      size_t batch, size_t stride, int words, size_t total) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const size_t item = idx / words;
    const int w = (int)(idx - item * words);
    const size_t o = item / batch, b = item - o * batch;
    const OutDesc d = od[o];
    uint32_t v;
    if (d.slot < 0) {
        v = w == 0 ? d.cst * 0x40000000u : 0u;
    } else {
        v = wires[((size_t)d.slot * batch + b) * stride + w];
        if (d.neg) v = (w == 0 ? 0x40000000u : 0u) - v;
    }
    out[item * stride + w] = v;
}

struct Ref {
    int base = -1;   // producing input/gate wire, -1 for a constant
    bool neg = false;
    int cval = 0;    // constant bit when base < 0
};

const int kGateS1[6] = {-1, 1, 1, -1, 2, -2};
const int kGateS2[6] = {-1, 1, 1, -1, -2, 2};
const uint32_t kGateConst[6] = {0xA0000000u, 0xE0000000u, 0x20000000u,
                                0x60000000u, 0x00000000u, 0x80000000u};

}  // namespace

struct CircuitPlan {
    std::vector<Ref> ref;                 // per wire
    std::vector<int> level;               // per wire (0 for inputs)
    std::vector<std::vector<int>> levels; // gate indices per level (1..L)
    std::vector<int> slot;                // per wire: slot index or -1
    std::vector<int> level_base;          // per level: first slot
    int total_slots = 0;
    int64_t live_gates = 0;
    int max_width = 0;
};

// Builds the plan; returns MK_OK or MK_EINVAL for a malformed netlist.
int plan_circuit(const mk_circuit *c, CircuitPlan &P) {
    if (!c || c->n_wires < 2 || c->n_inputs < 0 || c->n_outputs < 0 || c->n_gates < 0 ||
        (c->n_inputs && !c->inputs) || (c->n_outputs && !c->outputs) || (c->n_gates && !c->gates))
        return fail(MK_EINVAL, "mk_eval_circuit: malformed circuit header");
    const int W = c->n_wires;
    std::vector<int> kind(W, 0);  // 0 undefined, 1 constant, 2 input, 3 gate
    std::vector<int> producer(W, -1);
    kind[0] = kind[1] = 1;
    P.ref.assign(W, Ref());
    P.ref[0].cval = 0;
    P.ref[1].cval = 1;
    for (int i = 0; i < c->n_inputs; ++i) {
        const int w = c->inputs[i];
        if (w < 2 || w >= W || kind[w]) return fail(MK_EINVAL, "mk_eval_circuit: bad input wire");
        kind[w] = 2;
        P.ref[w].base = w;
    }
    for (int gi = 0; gi < c->n_gates; ++gi) {
        const mk_gate &g = c->gates[gi];
        if (g.type < 0 || g.type > MK_GATE_NOT) return fail(MK_EINVAL, "mk_eval_circuit: bad gate type");
        if (g.out < 2 || g.out >= W || kind[g.out]) return fail(MK_EINVAL, "mk_eval_circuit: bad gate output");
        if (g.in1 < 0 || g.in1 >= W || !kind[g.in1]) return fail(MK_EINVAL, "mk_eval_circuit: gate input undefined");
        if (g.type != MK_GATE_NOT && (g.in2 < 0 || g.in2 >= W || !kind[g.in2]))
            return fail(MK_EINVAL, "mk_eval_circuit: gate input undefined");
        kind[g.out] = 3;
        producer[g.out] = gi;
        if (g.type == MK_GATE_NOT) {
            Ref r = P.ref[g.in1];
            if (r.base < 0) r.cval ^= 1;
            else r.neg = !r.neg;
            P.ref[g.out] = r;
        } else {
            P.ref[g.out].base = g.out;
        }
    }
    for (int i = 0; i < c->n_outputs; ++i)
        if (c->outputs[i] < 0 || c->outputs[i] >= W || !kind[c->outputs[i]])
            return fail(MK_EINVAL, "mk_eval_circuit: bad output wire");
    // live bootstrapped gates: backwards from the outputs
    std::vector<char> needed(W, 0);
    for (int i = 0; i < c->n_outputs; ++i) {
        const int b = P.ref[c->outputs[i]].base;
        if (b >= 0) needed[b] = 1;
    }
    for (int gi = c->n_gates - 1; gi >= 0; --gi) {
        const mk_gate &g = c->gates[gi];
        if (g.type == MK_GATE_NOT || !needed[g.out]) continue;
        for (int in : {g.in1, g.in2}) {
            const int b = P.ref[in].base;
            if (b >= 0) needed[b] = 1;
        }
    }
    // levels
    P.level.assign(W, 0);
    int L = 0;
    for (int gi = 0; gi < c->n_gates; ++gi) {
        const mk_gate &g = c->gates[gi];
        if (g.type == MK_GATE_NOT || !needed[g.out]) continue;
        int lv = 0;
        for (int in : {g.in1, g.in2}) {
            const int b = P.ref[in].base;
            if (b >= 0) lv = std::max(lv, P.level[b]);
        }
        P.level[g.out] = lv + 1;
        L = std::max(L, lv + 1);
    }
    P.levels.assign(L + 1, {});
    for (int gi = 0; gi < c->n_gates; ++gi) {
        const mk_gate &g = c->gates[gi];
        if (g.type == MK_GATE_NOT || !needed[g.out]) continue;
        P.levels[P.level[g.out]].push_back(gi);
        ++P.live_gates;
    }
    for (int l = 1; l <= L; ++l) P.max_width = std::max(P.max_width, (int)P.levels[l].size());
    // last level that reads each base value (L+1 for circuit outputs)
    std::vector<int> lastuse(W, 0);
    for (int l = 1; l <= L; ++l)
        for (int gi : P.levels[l])
            for (int in : {c->gates[gi].in1, c->gates[gi].in2}) {
                const int b = P.ref[in].base;
                if (b >= 0) lastuse[b] = std::max(lastuse[b], l);
            }
    for (int i = 0; i < c->n_outputs; ++i) {
        const int b = P.ref[c->outputs[i]].base;
        if (b >= 0) lastuse[b] = L + 1;
    }
    // slot ranges: inputs first (range of level 0), then one range per level
    P.slot.assign(W, -1);
    P.level_base.assign(L + 1, 0);
    struct Range { int start, size, last; };
    std::list<std::pair<int, int>> free_list;  // (start, size), sorted by start
    std::vector<Range> live;
    int top = 0;
    auto alloc = [&](int size) {
        for (auto it = free_list.begin(); it != free_list.end(); ++it)
            if (it->second >= size) {
                const int st = it->first;
                it->first += size;
                it->second -= size;
                if (!it->second) free_list.erase(it);
                return st;
            }
        const int st = top;
        top += size;
        return st;
    };
    auto release = [&](int start, int size) {
        auto it = free_list.begin();
        while (it != free_list.end() && it->first < start) ++it;
        it = free_list.insert(it, {start, size});
        auto nx = std::next(it);
        if (nx != free_list.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_list.erase(nx);
        }
        if (it != free_list.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_list.erase(it);
            }
        }
    };
    {
        const int st = alloc(c->n_inputs);
        int last = 0;
        for (int i = 0; i < c->n_inputs; ++i) {
            P.slot[c->inputs[i]] = st + i;
            last = std::max(last, lastuse[c->inputs[i]]);
        }
        P.level_base[0] = st;
        live.push_back({st, c->n_inputs, last});
    }
    for (int l = 1; l <= L; ++l) {
        for (size_t r = 0; r < live.size();) {
            if (live[r].last <= l) {  // read at most by this level's pre-combination
                if (live[r].size) release(live[r].start, live[r].size);
                live[r] = live.back();
                live.pop_back();
            } else {
                ++r;
            }
        }
        const int n = (int)P.levels[l].size();
        const int st = alloc(n);
        int last = 0;
        for (int i = 0; i < n; ++i) {
            const int w = c->gates[P.levels[l][i]].out;
            P.slot[w] = st + i;
            last = std::max(last, lastuse[w]);
        }
        P.level_base[l] = st;
        live.push_back({st, n, last});
    }
    P.total_slots = top;
    return MK_OK;
}

static int alloc_circ_scratch(mk_ctx *ctx, size_t bytes) {
    DeviceKeys &D = ctx->dev;
    if (D.circ_scratch_bytes >= bytes) return MK_OK;
    if (D.circ_scratch) {
        if (hipDeviceSynchronize() != hipSuccess) return fail(MK_EDEVICE, "circuit scratch sync failed");
        (void)hipFree(D.circ_scratch);
        D.circ_scratch = nullptr;
        D.circ_scratch_bytes = 0;
    }
    if (hipMalloc(&D.circ_scratch, bytes) != hipSuccess) {
        D.circ_scratch = nullptr;
        return fail(MK_ENOMEM, "device allocation failed: circuit wire buffer");
    }
    D.circ_scratch_bytes = bytes;
    return MK_OK;
}

}  // namespace mk

using namespace mk;

extern "C" {

int mk_circuit_stats(const mk_circuit *c, int32_t *n_levels, int64_t *live_gates,
                     int32_t *max_width, int32_t *slots) {
    CircuitPlan P;
    int rc = plan_circuit(c, P);
    if (rc) return rc;
    if (n_levels) *n_levels = (int32_t)P.levels.size() - 1;
    if (live_gates) *live_gates = P.live_gates;
    if (max_width) *max_width = P.max_width;
    if (slots) *slots = P.total_slots;
    return MK_OK;
}

int mk_eval_circuit(mk_ctx *ctx, const mk_circuit *c, const uint32_t *in_dev, uint32_t *out_dev,
                    size_t batch, size_t stride, int path, void *stream) {
    if (!ctx) return fail(MK_EINVAL, "mk_eval_circuit: null context");
    if (path != MK_PATH_I32 && path != MK_PATH_MFMA_I8) return fail(MK_EINVAL, "mk_eval_circuit: bad path");
    const mk_params &Pm = ctx->p;
    const size_t words = lwe_words(Pm);
    if (stride < words) return fail(MK_EINVAL, "mk_eval_circuit: stride < kn+1");
    if (!ctx->dev.uploaded) return fail(MK_ESTATE, "evaluation key not uploaded (mk_upload_eval_key)");
    CircuitPlan P;
    int rc = plan_circuit(c, P);
    if (rc) return rc;
    if (!batch || !c->n_outputs) return MK_OK;
    if ((c->n_inputs && !in_dev) || !out_dev) return fail(MK_EINVAL, "mk_eval_circuit: null buffer");
    hipStream_t s = (hipStream_t)stream;
    const int L = (int)P.levels.size() - 1;
    // descriptors
    std::vector<CircDesc> desc;
    std::vector<size_t> desc_off(L + 2, 0);
    for (int l = 1; l <= L; ++l) {
        desc_off[l] = desc.size();
        for (int gi : P.levels[l]) {
            const mk_gate &g = c->gates[gi];
            CircDesc d{-1, -1, 0, 0, kGateConst[g.type], 0};
            const int sc[2] = {kGateS1[g.type], kGateS2[g.type]};
            const int ins[2] = {g.in1, g.in2};
            for (int q = 0; q < 2; ++q) {
                const Ref &r = P.ref[ins[q]];
                if (r.base < 0) {
                    d.cst += (uint32_t)(sc[q] * r.cval) * 0x40000000u;
                } else {
                    int sv = sc[q];
                    if (r.neg) {  // s * (1/4 - c)
                        d.cst += (uint32_t)sv * 0x40000000u;
                        sv = -sv;
                    }
                    (q == 0 ? d.slot1 : d.slot2) = P.slot[r.base];
                    (q == 0 ? d.s1 : d.s2) = sv;
                }
            }
            desc.push_back(d);
        }
    }
    desc_off[L + 1] = desc.size();
    std::vector<OutDesc> od(c->n_outputs);
    for (int i = 0; i < c->n_outputs; ++i) {
        const Ref &r = P.ref[c->outputs[i]];
        od[i] = r.base < 0 ? OutDesc{-1, 0, (uint32_t)r.cval, 0}
                           : OutDesc{P.slot[r.base], r.neg ? 1 : 0, 0, 0};
    }
    // device memory: wires | descriptors | output descriptors
    const size_t wire_b = ((size_t)P.total_slots * batch * stride * 4 + 255) / 256 * 256;
    const size_t desc_b = (desc.size() * sizeof(CircDesc) + 255) / 256 * 256;
    const size_t od_b = od.size() * sizeof(OutDesc);
    if ((rc = alloc_circ_scratch(ctx, wire_b + desc_b + od_b + 256))) return rc;
    // after the first enqueue, errors wait for the stream before returning so
    // that no queued copy still reads the host descriptor vectors
    auto bail = [&](int code, const char *msg) {
        (void)hipStreamSynchronize(s);
        return fail(code, msg);
    };
    char *base = (char *)ctx->dev.circ_scratch;
    uint32_t *wires = (uint32_t *)base;
    CircDesc *d_desc = (CircDesc *)(base + wire_b);
    OutDesc *d_od = (OutDesc *)(base + wire_b + desc_b);
    if (!desc.empty() && hipMemcpyAsync(d_desc, desc.data(), desc.size() * sizeof(CircDesc),
                                        hipMemcpyHostToDevice, s) != hipSuccess)
        return bail(MK_EDEVICE, "mk_eval_circuit: descriptor upload failed");
    if (hipMemcpyAsync(d_od, od.data(), od_b, hipMemcpyHostToDevice, s) != hipSuccess)
        return bail(MK_EDEVICE, "mk_eval_circuit: output descriptor upload failed");
    if (c->n_inputs &&
        hipMemcpyAsync(wires + (size_t)P.level_base[0] * batch * stride, in_dev,
                       (size_t)c->n_inputs * batch * stride * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return bail(MK_EDEVICE, "mk_eval_circuit: input copy failed");
    // per-level pipeline; gate scratch sized for the widest level
    const size_t maxc = (size_t)P.max_width * batch;
    const size_t abar_b = (maxc * words * 4 + 255) / 256 * 256;
    if ((rc = ensure_scratch(ctx, abar_b + maxc * (Pm.k + 1) * Pm.N * 4))) {
        (void)hipStreamSynchronize(s);
        return rc;
    }
    uint32_t *abar = (uint32_t *)ctx->dev.scratch;
    uint32_t *acc = (uint32_t *)((char *)ctx->dev.scratch + abar_b);
    const int log2_2N = __builtin_ctz(2 * Pm.N);
    for (int l = 1; l <= L; ++l) {
        const size_t count = P.levels[l].size() * batch;
        const size_t total = count * words;
        {
            StageTimer tm(ctx, 0, s);
            hipLaunchKernelGGL(precombine_circuit_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256),
                               0, s, d_desc + desc_off[l], (const uint32_t *)wires, batch, stride,
                               (int)words, log2_2N, total, abar);
        }
        if (hipGetLastError() != hipSuccess) return bail(MK_EDEVICE, "circuit precombine launch failed");
        if ((rc = run_blind_rotate(ctx, abar, acc, count, Pm.k * Pm.n, path, s)) ||
            (rc = run_key_switch(ctx, acc, wires + (size_t)P.level_base[l] * batch * stride, count, stride,
                                 path, s))) {
            (void)hipStreamSynchronize(s);
            return rc;
        }
    }
    const size_t total = (size_t)c->n_outputs * batch * words;
    {
        StageTimer tm(ctx, 3, s);
        hipLaunchKernelGGL(gather_outputs_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                           (const OutDesc *)d_od, (const uint32_t *)wires, out_dev, batch, stride,
                           (int)words, total);
    }
    if (hipGetLastError() != hipSuccess) return bail(MK_EDEVICE, "circuit output gather launch failed");
    // the host descriptor vectors must outlive the asynchronous copies
    if (hipStreamSynchronize(s) != hipSuccess) return fail(MK_EDEVICE, "mk_eval_circuit: stream sync failed");
    return MK_OK;
}

}  // extern "C"
