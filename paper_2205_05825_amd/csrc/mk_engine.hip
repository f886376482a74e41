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
// Device work per level, in chunks of at most one rotation launch:
// pre-combination gathering both operands of every (gate, instance), one
// blind rotation over all of them, and extraction + key switching straight
// into the level's slot range.  Wire buffer layout:
// row (slot * batch + instance) of `stride` words.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <list>
#include <new>
#include <string>
#include <vector>

#include "mk_device_common.h"

// A captured evaluation of one circuit on fixed buffers; owns its device
// memory (buf: wires+descriptors, gate scratch, rotation scratch, key-switch
// scratch) so that later calls on the context cannot move it.
struct mk_graph {
    mk_ctx *ctx = nullptr;
    // consecutive pieces of the captured sequence, replayed in order
    std::vector<hipGraph_t> graphs;
    std::vector<hipGraphExec_t> execs;
    void *buf[4] = {nullptr, nullptr, nullptr, nullptr};
    size_t bytes[4] = {0, 0, 0, 0};
    int levels = 0;
    int64_t gates = 0;
};

namespace mk {

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

// Items item0 .. item0 + total / words - 1 of a level (item = gate of the
// level x batch + instance) into abar (chunk-local).
__global__ void precombine_circuit_kernel(const CircDesc *__restrict__ desc,
                                          const uint32_t *__restrict__ wires, size_t batch,
                                          size_t stride, int words, int log2_2N, size_t item0, size_t total,
                                          uint32_t *__restrict__ abar) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const size_t item = item0 + idx / words;
    const int w = (int)(idx % words);
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
        // A range becomes free once the level that last reads it has
        // finished: a wide level runs in chunks, and an earlier chunk's
        // outputs must not overwrite wires that a later chunk still reads.
        for (size_t r = 0; r < live.size();) {
            if (live[r].last < l) {
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
    // Check the assignment: when level l writes a slot, the wire held there
    // before must have no reader at level l or later (a wide level runs in
    // chunks, so its gates read their inputs while its outputs are written).
    std::vector<int> holder(top, -1);
    for (int i = 0; i < c->n_inputs; ++i) holder[P.slot[c->inputs[i]]] = c->inputs[i];
    for (int l = 1; l <= L; ++l) {
        for (int gi : P.levels[l]) {
            const int h = holder[P.slot[c->gates[gi].out]];
            if (h >= 0 && lastuse[h] >= l)
                return fail(MK_EINTERNAL, "mk_eval_circuit: wire slot reused while still read (planner bug)");
        }
        for (int gi : P.levels[l]) holder[P.slot[c->gates[gi].out]] = c->gates[gi].out;
    }
    return MK_OK;
}

void graph_release(mk_graph *g);

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


// Host side of one circuit evaluation: the plan, the per-level
// pre-combination descriptors and the device buffer layout.
struct CircuitRun {
    CircuitPlan P;
    std::vector<CircDesc> desc;
    std::vector<size_t> desc_off;
    std::vector<OutDesc> od;
    size_t batch = 0, stride = 0, words = 0;
    size_t chunk = 0;  // gates per rotation launch within a level
    int path = 0, n_inputs = 0, n_outputs = 0;
    size_t wire_b = 0, desc_b = 0, od_b = 0, abar_b = 0, gate_b = 0;
    uint32_t *wires = nullptr;
    CircDesc *d_desc = nullptr;
    OutDesc *d_od = nullptr;
};

int build_run(mk_ctx *ctx, const mk_circuit *c, size_t batch, size_t stride, int path, CircuitRun &R,
              const char *who) {
    if (!ctx) return fail(MK_EINVAL, std::string(who) + ": null context");
    if (path != MK_PATH_I32 && path != MK_PATH_MFMA_I8) return fail(MK_EINVAL, std::string(who) + ": bad path");
    const mk_params &Pm = ctx->p;
    const size_t words = lwe_words(Pm);
    if (stride < words) return fail(MK_EINVAL, std::string(who) + ": stride < kn+1");
    if (!ctx->dev.uploaded) return fail(MK_ESTATE, "evaluation key not uploaded (mk_upload_eval_key)");
    int rc = plan_circuit(c, R.P);
    if (rc) return rc;
    CircuitPlan &P = R.P;
    R.batch = batch; R.stride = stride; R.words = words; R.path = path;
    R.n_inputs = c->n_inputs; R.n_outputs = c->n_outputs;
    const int L = (int)P.levels.size() - 1;
    R.desc_off.assign(L + 2, 0);
    for (int l = 1; l <= L; ++l) {
        R.desc_off[l] = R.desc.size();
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
            R.desc.push_back(d);
        }
    }
    R.desc_off[L + 1] = R.desc.size();
    R.od.resize(c->n_outputs);
    for (int i = 0; i < c->n_outputs; ++i) {
        const Ref &r = P.ref[c->outputs[i]];
        R.od[i] = r.base < 0 ? OutDesc{-1, 0, (uint32_t)r.cval, 0} : OutDesc{P.slot[r.base], r.neg ? 1 : 0, 0, 0};
    }
    R.wire_b = ((size_t)P.total_slots * batch * stride * 4 + 255) / 256 * 256;
    R.desc_b = (R.desc.size() * sizeof(CircDesc) + 255) / 256 * 256;
    R.od_b = R.od.size() * sizeof(OutDesc);
    R.chunk = rotation_chunk(Pm);  // wide levels run in chunks
    const size_t maxc = std::min((size_t)P.max_width * batch, R.chunk);
    R.abar_b = (maxc * words * 4 + 255) / 256 * 256;
    R.gate_b = R.abar_b + maxc * (Pm.k + 1) * Pm.N * 4;
    return MK_OK;
}

// Layout inside one block: wires | descriptors | output descriptors.
void set_run_buffers(CircuitRun &R, char *base) {
    R.wires = (uint32_t *)base;
    R.d_desc = (CircDesc *)(base + R.wire_b);
    R.d_od = (OutDesc *)(base + R.wire_b + R.desc_b);
}

int upload_descriptors(const CircuitRun &R, hipStream_t s) {
    if (!R.desc.empty() && hipMemcpyAsync(R.d_desc, R.desc.data(), R.desc.size() * sizeof(CircDesc),
                                          hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(MK_EDEVICE, "circuit descriptor upload failed");
    if (!R.od.empty() &&
        hipMemcpyAsync(R.d_od, R.od.data(), R.od_b, hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(MK_EDEVICE, "circuit output descriptor upload failed");
    return MK_OK;
}

__global__ void copy_words_kernel(const uint32_t *__restrict__ src, uint32_t *__restrict__ dst, size_t n) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n) dst[idx] = src[idx];
}

// Kernels of one chunk of a level outside the stepwise rotation (which
// reports its own): pre-combination, and for each of up to two rotation
// launches the accumulator set-up, control clear, persistent launch, copies,
// extraction and key switching, with some margin.
constexpr int kChunkKernels = 16;

// Device work of one evaluation, kernels only (so that it can be captured
// into a graph): inputs into their wire slots, every level's
// pre-combination, blind rotation and key switching, then the outputs.
// gate_scratch holds abar | accumulator for the widest level.
int enqueue_run(mk_ctx *ctx, const CircuitRun &R, uint32_t *gate_scratch, const uint32_t *in_dev,
                uint32_t *out_dev, hipStream_t s) {
    const mk_params &Pm = ctx->p;
    const CircuitPlan &P = R.P;
    const size_t batch = R.batch, stride = R.stride, words = R.words;
    const int L = (int)P.levels.size() - 1;
    if (R.n_inputs) {
        const size_t n = (size_t)R.n_inputs * batch * stride;
        hipLaunchKernelGGL(copy_words_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in_dev,
                           R.wires + (size_t)P.level_base[0] * batch * stride, n);
        if (hipGetLastError() != hipSuccess) return fail(MK_EDEVICE, "circuit input copy launch failed");
    }
    uint32_t *abar = gate_scratch;
    uint32_t *acc = (uint32_t *)((char *)gate_scratch + R.abar_b);
    const int log2_2N = __builtin_ctz(2 * Pm.N);
    int rc;
    for (int l = 1; l <= L; ++l) {
        const size_t count = P.levels[l].size() * batch;
        for (size_t c0 = 0; c0 < count; c0 += R.chunk) {
            const size_t cnt = std::min(R.chunk, count - c0);
            const size_t total = cnt * words;
            {
                StageTimer tm(ctx, 0, s);
                hipLaunchKernelGGL(precombine_circuit_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256),
                                   0, s, R.d_desc + R.desc_off[l], (const uint32_t *)R.wires, batch, stride,
                                   (int)words, log2_2N, c0, total, abar);
            }
            if (hipGetLastError() != hipSuccess) return fail(MK_EDEVICE, "circuit precombine launch failed");
            uint32_t *dst = R.wires + ((size_t)P.level_base[l] * batch + c0) * stride;
            if ((rc = run_rotate_ks(ctx, abar, acc, dst, cnt, stride, R.path, s)) ||
                (rc = capture_checkpoint(ctx, s, kChunkKernels)))
                return rc;
        }
    }
    const size_t total = (size_t)R.n_outputs * batch * words;
    {
        StageTimer tm(ctx, 3, s);
        hipLaunchKernelGGL(gather_outputs_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                           (const OutDesc *)R.d_od, (const uint32_t *)R.wires, out_dev, batch, stride,
                           (int)words, total);
    }
    if (hipGetLastError() != hipSuccess) return fail(MK_EDEVICE, "circuit output gather launch failed");
    return MK_OK;
}

// A capture is cut into consecutive graphs of about `piece` kernel nodes
// (default 1024; one stream-ordered rotation step is 4): each piece stays
// far from the node counts at which building one graph for a whole operator
// failed (one level of a 2-party Table 7 rotation alone is 4480 kernels),
// and pieces replayed in order on one stream are equivalent to the whole
// sequence.  No piece may exceed kGraphMaxKernels, the largest one tested.
constexpr int kGraphMinKernels = 64;
constexpr int kGraphMaxKernels = 4096;

struct CaptureState {
    mk_graph *g;
    int kernels;
    int piece;
};

int capture_checkpoint(mk_ctx *ctx, hipStream_t s, int kernels) {
    CaptureState *cs = (CaptureState *)ctx->dev.capture;
    if (!cs) return MK_OK;
    cs->kernels += kernels;
    if (cs->kernels > kGraphMaxKernels)
        return fail(MK_EINVAL, "graph capture: a piece exceeds 4096 kernels (untested size)");
    if (cs->kernels < cs->piece) return MK_OK;
    hipGraph_t piece = nullptr;
    if (hipStreamEndCapture(s, &piece) != hipSuccess || !piece)
        return fail(MK_EDEVICE, "graph capture: ending a piece failed");
    cs->g->graphs.push_back(piece);
    cs->kernels = 0;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(MK_EDEVICE, "graph capture: starting a piece failed");
    return MK_OK;
}

void graph_release(mk_graph *g) {
    for (hipGraphExec_t e : g->execs)
        if (e) (void)hipGraphExecDestroy(e);
    for (hipGraph_t gr : g->graphs)
        if (gr) (void)hipGraphDestroy(gr);
    g->execs.clear();
    g->graphs.clear();
    bool any = false;
    for (void *p : g->buf) any |= p != nullptr;
    if (any) (void)hipDeviceSynchronize();
    for (void *&p : g->buf) {
        if (p) (void)hipFree(p);
        p = nullptr;
    }
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

int mk_set_graph_piece(mk_ctx *ctx, int kernels) {
    if (!ctx || kernels < kGraphMinKernels || kernels > kGraphMaxKernels)
        return fail(MK_EINVAL, "mk_set_graph_piece: kernels outside [64, 4096]");
    ctx->dev.graph_piece = kernels;
    return MK_OK;
}

int mk_circuit_slots(const mk_circuit *c, int32_t *slot, int32_t *level) {
    CircuitPlan P;
    int rc = plan_circuit(c, P);
    if (rc) return rc;
    for (int w = 0; w < c->n_wires; ++w) {
        const bool live = P.slot[w] >= 0;
        if (slot) slot[w] = P.slot[w];
        if (level) level[w] = live ? P.level[w] : -1;
    }
    return MK_OK;
}

int mk_eval_circuit(mk_ctx *ctx, const mk_circuit *c, const uint32_t *in_dev, uint32_t *out_dev,
                    size_t batch, size_t stride, int path, void *stream) {
    CircuitRun R;
    int rc = build_run(ctx, c, batch, stride, path, R, "mk_eval_circuit");
    if (rc) return rc;
    if (!batch || !c->n_outputs) return MK_OK;
    if ((c->n_inputs && !in_dev) || !out_dev) return fail(MK_EINVAL, "mk_eval_circuit: null buffer");
    hipStream_t s = (hipStream_t)stream;
    if ((rc = alloc_circ_scratch(ctx, R.wire_b + R.desc_b + R.od_b + 256))) return rc;
    set_run_buffers(R, (char *)ctx->dev.circ_scratch);
    // after the first enqueue, errors wait for the stream before returning so
    // that no queued copy still reads the host descriptor vectors
    if ((rc = upload_descriptors(R, s))) {
        (void)hipStreamSynchronize(s);
        return rc;
    }
    if ((rc = ensure_scratch(ctx, R.gate_b))) {
        (void)hipStreamSynchronize(s);
        return rc;
    }
    rc = enqueue_run(ctx, R, (uint32_t *)ctx->dev.scratch, in_dev, out_dev, s);
    // the host descriptor vectors must outlive the asynchronous copies
    const bool synced = hipStreamSynchronize(s) == hipSuccess;
    if (rc) return rc;
    if (!synced) return fail(MK_EDEVICE, "mk_eval_circuit: stream sync failed");
    return MK_OK;
}

int mk_circuit_graph_create(mk_ctx *ctx, const mk_circuit *c, const uint32_t *in_dev, uint32_t *out_dev,
                            size_t batch, size_t stride, int path, mk_graph **graph) {
    if (!graph) return fail(MK_EINVAL, "mk_circuit_graph_create: null graph pointer");
    *graph = nullptr;
    CircuitRun R;
    int rc = build_run(ctx, c, batch, stride, path, R, "mk_circuit_graph_create");
    if (rc) return rc;
    if (!batch || !c->n_outputs) return fail(MK_EINVAL, "mk_circuit_graph_create: empty batch or circuit");
    if ((c->n_inputs && !in_dev) || !out_dev) return fail(MK_EINVAL, "mk_circuit_graph_create: null buffer");
    mk_graph *g = new (std::nothrow) mk_graph();
    if (!g) return fail(MK_ENOMEM, "mk_circuit_graph_create: out of host memory");
    g->ctx = ctx;
    g->levels = (int)R.P.levels.size() - 1;
    g->gates = R.P.live_gates * (int64_t)batch;
    auto abandon = [&](int code) {
        graph_release(g);
        delete g;
        return code;
    };
    // graph-owned device memory: wires | descriptors, the gate pipeline's
    // scratch and, on the MFMA path, the rotation's and key switch's scratch
    const size_t maxc = std::min((size_t)R.P.max_width * batch, R.chunk);
    const size_t sizes[4] = {R.wire_b + R.desc_b + R.od_b + 256, R.gate_b,
                             path == MK_PATH_MFMA_I8 ? mfma_scratch_need(ctx->p, maxc) : 0,
                             path == MK_PATH_MFMA_I8 ? ks_scratch_need(ctx->p, maxc) : 0};
    for (int i = 0; i < 4; ++i) {
        g->bytes[i] = sizes[i];
        if (sizes[i] && hipMalloc(&g->buf[i], sizes[i]) != hipSuccess) {
            g->buf[i] = nullptr;
            return abandon(fail(MK_ENOMEM, "mk_circuit_graph_create: device allocation failed"));
        }
    }
    set_run_buffers(R, (char *)g->buf[0]);
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
        return abandon(fail(MK_EDEVICE, "mk_circuit_graph_create: stream creation failed"));
    if ((rc = upload_descriptors(R, cs)) || hipStreamSynchronize(cs) != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return abandon(rc ? rc : fail(MK_EDEVICE, "mk_circuit_graph_create: descriptor upload failed"));
    }
    // capture with the context's scratch pointing at the graph's buffers (no
    // allocation can happen inside the capture) and profiling off
    DeviceKeys &D = ctx->dev;
    void *save_p[3] = {D.scratch, D.mfma_scratch, D.ks_scratch};
    size_t save_b[3] = {D.scratch_bytes, D.mfma_scratch_bytes, D.ks_scratch_bytes};
    const int save_prof = D.profiling;
    D.scratch = g->buf[1]; D.scratch_bytes = g->bytes[1];
    D.mfma_scratch = g->buf[2]; D.mfma_scratch_bytes = g->bytes[2];
    D.ks_scratch = g->buf[3]; D.ks_scratch_bytes = g->bytes[3];
    D.profiling = 0;
    CaptureState state{g, 0, D.graph_piece};
    D.capture = &state;
    rc = MK_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        rc = fail(MK_EDEVICE, "mk_circuit_graph_create: capture failed to start");
    } else {
        rc = enqueue_run(ctx, R, (uint32_t *)g->buf[1], in_dev, out_dev, cs);
        // end whatever capture is open (also after an error inside a piece)
        hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(cs, &st) == hipSuccess && st != hipStreamCaptureStatusNone) {
            hipGraph_t piece = nullptr;
            const hipError_t e = hipStreamEndCapture(cs, &piece);
            if (piece) g->graphs.push_back(piece);
            if (!rc && e != hipSuccess) rc = fail(MK_EDEVICE, "mk_circuit_graph_create: capture failed");
        }
    }
    D.capture = nullptr;
    D.scratch = save_p[0]; D.scratch_bytes = save_b[0];
    D.mfma_scratch = save_p[1]; D.mfma_scratch_bytes = save_b[1];
    D.ks_scratch = save_p[2]; D.ks_scratch_bytes = save_b[2];
    D.profiling = save_prof;
    (void)hipStreamDestroy(cs);
    if (rc) return abandon(rc);
    for (hipGraph_t piece : g->graphs) {
        hipGraphExec_t e = nullptr;
        if (hipGraphInstantiate(&e, piece, nullptr, nullptr, 0) != hipSuccess)
            return abandon(fail(MK_EDEVICE, "mk_circuit_graph_create: instantiation failed"));
        g->execs.push_back(e);
    }
    *graph = g;
    return MK_OK;
}

int mk_graph_launch(mk_graph *g, void *stream) {
    if (!g || g->execs.empty()) return fail(MK_EINVAL, "mk_graph_launch: null graph");
    for (hipGraphExec_t e : g->execs)
        if (hipGraphLaunch(e, (hipStream_t)stream) != hipSuccess)
            return fail(MK_EDEVICE, "mk_graph_launch: launch failed");
    return MK_OK;
}

int mk_graph_info(const mk_graph *g, int32_t *n_levels, int64_t *gates, int32_t *pieces) {
    if (!g) return fail(MK_EINVAL, "mk_graph_info: null graph");
    if (n_levels) *n_levels = g->levels;
    if (gates) *gates = g->gates;
    if (pieces) *pieces = (int32_t)g->execs.size();
    return MK_OK;
}

int mk_graph_destroy(mk_graph *g) {
    if (!g) return MK_OK;
    graph_release(g);
    delete g;
    return MK_OK;
}

}  // extern "C"
