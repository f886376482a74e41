// Persistent int8-MFMA blind rotation: all k*n CMux steps of a batch in one
// launch (the batching of a circuit level, §3.1 and the "parallel
// optimization" of §5.3-§5.4, realised on one GPU).
//
// Each 32-gate tile of the batch is run by a team of S = 2 RB workgroups
// (RB = N/32 / MR row blocks of MR 32-row tiles).  A workgroup's four waves
// hold the four key limbs of one contraction task (seamless limb-split
// schedule, mk_mfma_core.h).  One CMux step (party i, bit l, live slots L =
// min(k+1, i+2)) is three phases, separated by team barriers:
//   R   P_j = X^-a ACC_j - ACC_j, decomposed into ell digit planes U_j
//       (gadget base 2^8), for j < L; units of 4 gates x one slot, spread
//       evenly over the members.
//   S1  members 0..RB-1 (row block rb = member) contract
//           w = sum_{j<L} sum_l T(b_{j,l}) U_{j,l}
//       over all L*ell key polynomials in one accumulation, and decompose w
//       into the digit planes V; members RB..2RB-1 (rb = member - RB) add
//       c'_j = sum_l T(d_l) U_{j,l} into ACC_j for every j < L, as one
//       seamless stream of L*ell polynomials cut into L segments (a row
//       tile hands its finished c'_j to LDS and restarts for c'_{j+1}
//       without draining the pipeline).  Both halves contract L*ell
//       polynomials.
//   S2  ACC_{o ? 1+i : 0} += sum_l T(f_o,l) V_l, one (o, rb) task per member
//       (the same segmented stream as the c' half, with one segment).
// This is the hybrid product of the uni-encrypted bootstrapping key (§3.2)
// with the evaluation key (b_0 = -a, b_1..b_k), in the same order as the
// stream-ordered kernels, hence bit-identical to them.  When an XCD owns
// more tiles than teams fit on it, a team runs c tiles, phase by phase.
// After the last step a gate launch can also run sample extraction and key
// switching (§3.2 MKKeySwitch) on the team's tiles: rounding units, one
// barrier, then the one-hot int8 GEMM tasks (mk_ks_core.h), so the final
// accumulators never leave the XCD's L2 before they are switched.
//
// Teams are pinned to one XCD: a workgroup reads the XCD it runs on from
// the hardware (XCC_ID), registers there, and forms teams with the
// workgroups registered before it on the same XCD; every tile is owned by
// one XCD.  The data a team exchanges (accumulator rows, digit planes)
// therefore stays in one L2, and loads of it use the device-scope cache
// policy, which bypasses the compute unit's L1 (whose lines are not kept
// coherent with other compute units' stores).  A barrier is: every wave
// waits for its stores to complete, then one device-scope atomic increment
// per workgroup and a bounded spin until the team's count is reached.  A
// workgroup that waits too long sets an abort flag that every other one
// observes, and the host sees the error in the context's status word.
//
// Teams are formed in registration order, so a team only ever waits for its
// own members, which registered before any later team's: earlier teams
// finish without waiting for later ones and no co-residency is assumed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <set>
#include <vector>

#include "mk_device_common.h"
#include "mk_ks_core.h"
#include "mk_mfma_core.h"

namespace mk {

#define MK_HIP(call, what)                               \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

typedef __attribute__((address_space(3))) void lds_void;

constexpr int kPThreads = 256;     // 4 waves, one key limb each
constexpr int kCtlHeader = 64;     // control words before the first team's block
constexpr int kCtlPerTeam = 64;    // one barrier counter per team (256 B apart)
constexpr int kHdrAbort = 0, kHdrReg = 16;  // kHdrReg + x: workgroups registered on XCD x
constexpr int kRGates = 4;         // gates per R unit
constexpr int kMaxRUnits = 4;      // R units held in LDS at once
constexpr int kLimbTileBytes = 4 * 4 * 64 * 16;     // one row tile's four limbs in LDS

// Prefetch depths and workgroups per compute unit of the contraction for
// N = 32 NB with row blocks of MR row tiles (team size S = 2 NB / MR; the
// rings of the seamless schedule must divide NB, see slide_gemm).  At N =
// 1024 three team sizes are built: MR = 8 (S = 8) for batches of at least
// three tiles per XCD, and MR = 4 (S = 16) and MR = 2 (S = 32) so that
// narrower batches still spread each tile over most of an XCD's compute
// units.
template <int NB, int MR>
struct PersistCfg;
template <> struct PersistCfg<4, 2> { static constexpr int D = 2, OCC = 2, PF = 2; };
template <> struct PersistCfg<8, 4> { static constexpr int D = 4, OCC = 2, PF = 4; };
template <> struct PersistCfg<16, 4> { static constexpr int D = 4, OCC = 2, PF = 4; };
template <> struct PersistCfg<32, 8> { static constexpr int D = 6, OCC = 1, PF = 10; };
template <> struct PersistCfg<32, 4> { static constexpr int D = 6, OCC = 1, PF = 10; };
template <> struct PersistCfg<32, 2> { static constexpr int D = 6, OCC = 1, PF = 10; };
template <> struct PersistCfg<64, 8> { static constexpr int D = 6, OCC = 1, PF = 4; };

struct PersistArgs {
    MfmaArgs m;
    uint32_t *ctl;       // control block, zeroed before the launch
    uint32_t *status;    // sticky status word of the context
    int nx;              // XCDs in use (dense indices 0..nx-1)
    int c;               // tiles per team
    int teams_max;       // teams of the XCD with the most tiles
    int steps;           // CMux steps run
    int8_t xmap[16];     // XCC_ID -> dense XCD index, -1 if unused
    uint32_t spin_limit;
    KsFused ks;          // key switching after the last step (ks.tiles != nullptr)
};

__device__ __forceinline__ uint32_t ld_dev(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t add_dev(uint32_t *p, uint32_t v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ v4i ld_coherent(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return (v4i)__builtin_amdgcn_raw_buffer_load_b128(r, off, 0, kCoherent);
}

// Team barrier: every member's stores have completed before it counts
// itself; returns false on abort or timeout.
__device__ bool team_sync(const PersistArgs &p, uint32_t *ctr, uint32_t target, int *sh_flag) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        add_dev(ctr, 1u);
        bool ok = false;
        for (uint32_t s = 0; s < p.spin_limit; ++s) {
            if (ld_dev(ctr) >= target) {
                ok = true;
                break;
            }
            if ((s & 63) == 63 && ld_dev(p.ctl + kHdrAbort)) break;
            __builtin_amdgcn_s_sleep(1);
        }
        if (!ok && !ld_dev(p.ctl + kHdrAbort)) {
            add_dev(p.ctl + kHdrAbort, 1u);
            __hip_atomic_fetch_or(p.status, kStatusTimeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        *sh_flag = ok;
    }
    __syncthreads();
    return *sh_flag != 0;
}

// R for units u0, u0 + stride, ... < nunits (at most kMaxRUnits of them) of
// this step, unit = (tile, slot j, 4-gate quad q) from unit_of(u).  Their
// accumulator rows are copied straight into LDS (each wave moves 1 KB per
// load, all in flight at once), then each thread forms 16-byte fragment
// pieces of the ell digit planes from 16 plain and 16 rotated coefficients:
// (X^-a c)[m] = c[m + a] for m + a < N and -c[m + a - N] beyond (a < 2N).
template <class UnitOf>
__device__ void rotdec_batch(const PersistArgs &p, int u0, int stride, int nunits, int step, UnitOf unit_of,
                             uint32_t *rows) {
    const MfmaArgs &a = p.m;
    const int N = a.N, K1 = a.k + 1, NB = N / 32, GT = a.GP / 32, tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64)), lane = tid & 63;
    int nu = 0;
    for (int u = u0; u < nunits && nu < kMaxRUnits; u += stride, ++nu) {
        int t, j, q;
        unit_of(u, t, j, q);
        const __amdgpu_buffer_rsrc_t racc = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(a.acc + (size_t)t * 32 * K1 * N), (short)0, 32 * K1 * N * 4, kBufWord3);
        uint32_t *dst = rows + (size_t)nu * kRGates * N;
        if (N >= 256) {
            // kRGates rows of N words (4 N bytes): N / 256 loads of 1 KB each
            const int per_row = N / 256;
            for (int x = wave; x < kRGates * per_row; x += 4) {
                const int gi = x / per_row, part = x % per_row;
                const uint32_t src = (uint32_t)((((kRGates * q + gi) * K1 + j) * N + 256 * part) * 4) + 16u * lane;
                __builtin_amdgcn_raw_ptr_buffer_load_lds(racc, (lds_void *)(dst + (size_t)gi * N + 256 * part), 16,
                                                         src, 0, 0, kCoherent);
            }
        } else {
            // rows shorter than one 1 KB load: through registers
            for (int v = tid; v < kRGates * N / 4; v += kPThreads) {
                const int gi = v / (N / 4), c4 = v % (N / 4);
                const v4i x4 = ld_coherent(racc, (uint32_t)((((kRGates * q + gi) * K1 + j) * N + 4 * c4) * 4));
                reinterpret_cast<uint4 *>(dst)[v] = make_uint4(x4[0], x4[1], x4[2], x4[3]);
            }
        }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const int stride_ab = a.k * a.n + 1;
    const size_t l_stride = (size_t)GT * NB * kTileBytes;
    for (int item = tid; item < nu * kRGates * NB * 2; item += kPThreads) {  // (unit, kb, h, gate)
        const int k = item / (kRGates * NB * 2), rem = item % (kRGates * NB * 2);
        const int gi = rem % kRGates, kb = rem / (2 * kRGates), h = (rem / kRGates) % 2;
        int t, j, q;
        unit_of(u0 + k * stride, t, j, q);
        const int gate = t * 32 + kRGates * q + gi;
        const int shift = gate < a.G ? (int)a.abar[(size_t)gate * stride_ab + 1 + step] : 0;
        const uint32_t *row = rows + ((size_t)k * kRGates + gi) * N;
        const int m0 = 32 * kb + 16 * h;
        uint32_t y[16];
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            const uint4 pl = *reinterpret_cast<const uint4 *>(row + m0 + 4 * qq);
            const uint32_t pv[4] = {pl.x, pl.y, pl.z, pl.w};
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int s = m0 + 4 * qq + b + shift;
                const uint32_t src = row[s & (N - 1)];
                const uint32_t rot = ((s >> a.log2N) & 1) ? 0u - src : src;
                y[4 * qq + b] = rot - pv[b] + a.offset;
            }
        }
        int8_t *base = a.U + ((size_t)j * a.ell * GT + t) * NB * kTileBytes;
        put_digits(base + (size_t)kb * kTileBytes + (32 * h + gate % 32) * 16, l_stride, a.ell, y);
    }
    __syncthreads();   // the rows are reused by the next batch or task
}

template <class UnitOf>
__device__ void pass_rotdec(const PersistArgs &p, int u0, int stride, int nunits, int step, UnitOf unit_of,
                            uint32_t *rows) {
    for (int b = u0; b < nunits; b += kMaxRUnits * stride) rotdec_batch(p, b, stride, nunits, step, unit_of, rows);
}

// Limb combination in one LDS round: every wave writes all MR of its limb
// tiles, shifted by 8 t (limb t weighs 2^(8t)), then after one barrier wave
// t sums quad t (registers 4t..4t+3, i.e. words 8t..8t+3 of its lane's row
// within each 32-row tile) over the four limbs.  `red` holds MR x 16 KB.
template <int MR>
__device__ __forceinline__ void limb_sums(const v16i (&acc)[MR][1], int t, int lane, uint4 *red,
                                          uint4 (&sum)[MR]) {
    const uint32_t sh = 8u * (uint32_t)t;
#pragma unroll
    for (int i = 0; i < MR; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            red[((i * 4 + t) * 4 + q) * 64 + lane] =
                make_uint4((uint32_t)acc[i][0][4 * q + 0] << sh, (uint32_t)acc[i][0][4 * q + 1] << sh,
                           (uint32_t)acc[i][0][4 * q + 2] << sh, (uint32_t)acc[i][0][4 * q + 3] << sh);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MR; ++i) {
        uint4 v = red[((i * 4 + 0) * 4 + t) * 64 + lane];
#pragma unroll
        for (int l = 1; l < 4; ++l) {
            const uint4 x = red[((i * 4 + l) * 4 + t) * 64 + lane];
            v.x += x.x;
            v.y += x.y;
            v.z += x.z;
            v.w += x.w;
        }
        sum[i] = v;
    }
}

// The ell digits of w into V: a thread's 4 consecutive coefficients
// 32 kb + 8 t + 4 h .. + 3 of its lane's gate are bytes 8 (t & 1) + 4 h ..
// + 3 of fragment piece (kb, lane 32 (t >> 1) + g) of each digit plane.
template <int MR>
__device__ __forceinline__ void store_v_digits(const MfmaArgs &a, int tile, int rb, int t, int lane,
                                               const uint4 (&sum)[MR]) {
    const int NB = a.N / 32, GT = a.GP / 32;
    const int h = lane >> 5, g = lane & 31;
#pragma unroll
    for (int i = 0; i < MR; ++i) {
        const uint32_t y[4] = {sum[i].x + a.offset, sum[i].y + a.offset, sum[i].z + a.offset, sum[i].w + a.offset};
        const int kb = rb * MR + i;
        int8_t *dst = a.V + ((size_t)tile * NB + kb) * kTileBytes + (32 * (t >> 1) + g) * 16 + 8 * (t & 1) + 4 * h;
#pragma unroll
        for (int l = 0; l < kMaxEll; ++l) {
            if (l >= a.ell) break;
            uint32_t wd = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) wd |= ((((y[e] >> (24 - 8 * l)) & 255u) - 128u) & 255u) << (8 * e);
            *reinterpret_cast<uint32_t *>(dst + (size_t)l * GT * NB * kTileBytes) = wd;
        }
    }
}

// One contraction task on tile t, row block rb, wave w = key limb: kind 0 =
// c'_j into ACC_j for every live slot j (one seamless stream of live x ell
// polynomials, one segment per slot), 1 = w into V, 2 = stage-2 unit o into
// ACC_{o ? 1+party : 0} (a stream of ell polynomials, one segment).  The
// read-modify-write kinds hand each finished row to LDS and add the old
// row, prefetched while the row's last products run, when they store it.
template <int NB, int MR>
__device__ __forceinline__ void task_gemm(const PersistArgs &p, int kind, int j_or_o, int t, int rb, int party,
                                          int bit, int live, uint4 *red) {
    constexpr int ND = 2 * NB - 1;
    using Cfg = PersistCfg<NB, MR>;
    const MfmaArgs &a = p.m;
    const int N = a.N, K1 = a.k + 1, ell = a.ell, GT = a.GP / 32;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
    const size_t poly_tiles = (size_t)4 * ND * kTileBytes;
    const size_t bkbit = ((size_t)party * a.n + bit) * 3;
    const size_t gate_stride = (size_t)K1 * N;
    Operands o;
    o.b_poly = (uint32_t)((size_t)GT * NB * kTileBytes);
    o.NB = NB;
    o.mb0 = rb * MR;
    o.nc_valid = 1;
    v16i acc[MR][1];
#pragma unroll
    for (int r = 0; r < MR; ++r) acc[r][0] = v16i{};
    if (kind == 0 || kind == 2) {
        // kind 0: d_l against U_{j,l} for j < live: polynomial p = j ell + l,
        // segment j into slot j; kind 2: f_{o,l} against V_l, one segment
        // into slot 0 (o = 0) or 1 + party (o = 1)
        const int out_slot = kind == 0 ? 0 : (j_or_o == 0 ? 0 : 1 + party);
        const int seg_step = kind == 0 ? 1 : 0;
        if (kind == 0) {
            o.A = a.bk + bkbit * ell * poly_tiles;
            o.B = a.U + (size_t)t * NB * kTileBytes;
            o.ell = live * ell;
        } else {
            o.A = a.bk + ((bkbit + 1 + j_or_o) * ell) * poly_tiles;
            o.B = a.V + (size_t)t * NB * kTileBytes;
            o.ell = ell;
        }
        // the tile's gates: lane g's row tile r of slot s starts at word
        // g K1 N + s N + 32 (rb MR + r); wave w owns words 8 w + 4 h .. + 3
        const __amdgpu_buffer_rsrc_t racc = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(a.acc + (size_t)t * 32 * gate_stride), (short)0, (int)(32 * gate_stride * 4), kBufWord3);
        const uint32_t lane_word =
            (uint32_t)((size_t)(lane & 31) * gate_stride + 32 * rb * MR + 8 * w + 4 * (lane >> 5));
        uint32_t *tile_acc = a.acc + (size_t)t * 32 * gate_stride;
        // a segment's rows go to LDS one by one as they finish (row r in
        // slot r, [wave][quad][lane]); after the segment's last iteration,
        // one barrier, then wave w sums quad w of the four limbs of every
        // row, limb l weighted 2^(8 l), onto the row's old value.  A second
        // barrier before the first put keeps a segment's puts clear of the
        // previous segment's reads.
        uint4 *slots = red;
        slide_gemm_seg<MR, NB, Cfg::D, kCoherent, Cfg::PF>(
            o, ell, w, lane, acc,
            [&](int r, int s) {
                const int slot = out_slot + seg_step * s;
                return ld_coherent(racc, (lane_word + (uint32_t)(slot * N + 32 * r)) * 4u);
            },
            [&](int r) {
                if (r == MR - 1) __syncthreads();
                uint4 *slot = slots + r * (4 * 4 * 64);
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    slot[(w * 4 + q) * 64 + lane] =
                        make_uint4((uint32_t)acc[r][0][4 * q + 0], (uint32_t)acc[r][0][4 * q + 1],
                                   (uint32_t)acc[r][0][4 * q + 2], (uint32_t)acc[r][0][4 * q + 3]);
            },
            [&](int s, const v4i (&old)[MR]) {
                __syncthreads();
#pragma unroll
                for (int r = 0; r < MR; ++r) {
                    const uint4 *slot = slots + r * (4 * 4 * 64);
                    uint4 v = make_uint4((uint32_t)old[r][0], (uint32_t)old[r][1], (uint32_t)old[r][2],
                                         (uint32_t)old[r][3]);
#pragma unroll
                    for (int l = 0; l < 4; ++l) {
                        const uint4 x = slot[(l * 4 + w) * 64 + lane];
                        v.x += x.x << (8 * l);
                        v.y += x.y << (8 * l);
                        v.z += x.z << (8 * l);
                        v.w += x.w << (8 * l);
                    }
                    *reinterpret_cast<uint4 *>(tile_acc + lane_word + (size_t)(out_slot + seg_step * s) * N + 32 * r) = v;
                }
            });
        __syncthreads();   // the slots are reused by the next task
        return;
    }
    // kind 1: w = sum over the live slots of b_{j,l} against U_{j,l}, its
    // limbs combined and decomposed into V
    o.A = a.evk;                                   // b_{j,l}, j < live, flattened
    o.B = a.U + (size_t)t * NB * kTileBytes;       // U_{j,l}, same order
    o.ell = live * ell;
    slide_gemm<MR, NB, Cfg::D, kCoherent>(o, w, lane, acc, []() {});
    uint4 sum[MR];
    limb_sums<MR>(acc, w, lane, red, sum);
    store_v_digits<MR>(a, t, rb, w, lane, sum);
    __syncthreads();   // red is reused by the next task
}

template <int NB, int MR>
__global__ __launch_bounds__(kPThreads, (PersistCfg<NB, MR>::OCC)) void persist_rotation_kernel(PersistArgs p) {
    // R units keep their accumulator rows here, contraction tasks their limb
    // combination buffer; a workgroup runs one at a time
    extern __shared__ __align__(16) uint32_t smem[];
    uint32_t *rows = smem;
    uint4 *red = reinterpret_cast<uint4 *>(smem);
    __shared__ int sh[2];
    constexpr int RB = NB / MR, S = 2 * RB;
    const int GT = p.m.GP / 32;
    if (threadIdx.x == 0) {
        const int xcc = __builtin_amdgcn_s_getreg((31 << 11) | 20) & 15;  // HW_REG_XCC_ID
        const int x = p.xmap[xcc];
        sh[0] = x;
        sh[1] = x >= 0 ? (int)add_dev(p.ctl + kHdrReg + x, 1u) : 0;
        if (x < 0) __hip_atomic_fetch_or(p.status, kStatusNoXcd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    const int x = sh[0], m = sh[1];
    if (x < 0 || x >= GT) return;                  // an XCD without tiles
    const int ntx = (GT - x + p.nx - 1) / p.nx;    // this XCD's tiles x + nx i, i < ntx
    const int team = m / S, r = m % S;
    if (team * p.c >= ntx) return;                 // more workgroups than teams
    const int c = min(p.c, ntx - team * p.c);      // tiles of this team
    const int tile0 = team * p.c;                  // index among the XCD's tiles
    uint32_t *ctr = p.ctl + kCtlHeader + (size_t)(x * p.teams_max + team) * kCtlPerTeam;
    const int K1 = p.m.k + 1, n = p.m.n;
    constexpr int Q = 32 / kRGates;                // R units per (tile, slot)
    uint32_t target = 0;
    for (int st = 0; st < p.steps; ++st) {
        const int party = st / n, bit = st - party * n;
        const int L = min(K1, party + 2);
        // R: c tiles x L slots x Q units over the S members
        pass_rotdec(p, r, S, c * L * Q, st,
                    [&](int u, int &t, int &j, int &q) {
                        t = x + (tile0 + u / (L * Q)) * p.nx;
                        j = (u / Q) % L;
                        q = u % Q;
                    },
                    rows);
        target += S;
        if (!team_sync(p, ctr, target, &sh[0])) return;
        // S1 (phase 1) and S2 (phase 2); one call site for every contraction
        // task keeps a single copy of it
        for (int ph = 1; ph <= 2; ++ph) {
            // one task of this member per tile: S1 w or c'_0..c'_{L-1}, S2 (o, rb)
            for (int ti = 0; ti < c; ++ti) {
                const int kind = ph == 2 ? 2 : (r < RB ? 1 : 0);
                const int jo = ph == 2 ? r / RB : 0;
                const int rb = ph == 2 ? r % RB : (r < RB ? r : r - RB);
                task_gemm<NB, MR>(p, kind, jo, x + (tile0 + ti) * p.nx, rb, party, bit, L, red);
            }
            target += S;
            if (!team_sync(p, ctr, target, &sh[0])) return;
        }
    }
    if (!p.ks.tiles) return;
    // Extraction and key switching of the team's tiles, whose accumulators
    // are final after the last barrier: rounding units (tile, party, 64
    // coefficients), one barrier, then GEMM tasks (tile, party, column
    // block), both spread over the members.  The accumulators and the
    // rounded coefficients were written by other members, so they are read
    // with device-scope loads.
    const KsShape &ks = p.ks.s;
    const int QB = (ks.N + 63) / 64, units = ks.k * QB;
    for (int u = r; u < c * units; u += S)
        ks_round_unit<true>(p.m.acc, ks, p.ks.count, p.ks.R, p.ks.out, p.ks.stride,
                            x + (tile0 + u / units) * p.nx, (u % units % QB) * 64, u % units / QB, smem);
    target += S;
    if (!team_sync(p, ctr, target, &sh[0])) return;
    const int CB = ks_col_blocks(ks), tasks = ks.k * CB;
    for (int u = r; u < c * tasks; u += S) {
        const int gt = x + (tile0 + u / tasks) * p.nx, cb = u % tasks % CB, i = u % tasks / CB;
        if (ks.lb == 2) ks_gemm_task<true, kCoherent>(p.ks.tiles, p.ks.R, ks, p.ks.count, p.ks.out, p.ks.stride,
                                                      gt, cb, i, red);
        else ks_gemm_task<false, kCoherent>(p.ks.tiles, p.ks.R, ks, p.ks.count, p.ks.out, p.ks.stride, gt, cb,
                                            i, red);
    }
}

__global__ void zero_words_kernel(uint32_t *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ void xcc_probe_kernel(uint32_t *out) {
    if (threadIdx.x == 0) out[blockIdx.x] = __builtin_amdgcn_s_getreg((31 << 11) | 20) & 15;
}

// XCDs of the device: every workgroup of a large probe grid records the
// XCC_ID it runs on; the ids seen are numbered densely.
int persist_probe(mk_ctx *ctx, hipStream_t s) {
    DeviceKeys &D = ctx->dev;
    hipDeviceProp_t prop;
    MK_HIP(hipGetDeviceProperties(&prop, D.device), "device properties");
    D.num_cus = prop.multiProcessorCount;
    const int G = 16 * prop.multiProcessorCount;
    uint32_t *buf = nullptr;
    MK_HIP(hipMalloc((void **)&buf, (size_t)G * 4), "xcc probe buffer");
    hipLaunchKernelGGL(xcc_probe_kernel, dim3(G), dim3(64), 0, s, buf);
    std::vector<uint32_t> ids(G);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(ids.data(), buf, (size_t)G * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(buf);
    if (e != hipSuccess) return hip_fail(e, "xcc probe");
    std::set<uint32_t> seen(ids.begin(), ids.end());
    std::memset(D.xmap, -1, sizeof(D.xmap));
    int x = 0;
    for (uint32_t id : seen) D.xmap[id & 15] = (int8_t)x++;
    D.num_xcd = x;
    if (!D.status) {
        MK_HIP(hipMalloc((void **)&D.status, 4), "status word");
        hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, s, D.status, 1);
        MK_HIP(hipGetLastError(), "status clear");
    }
    return MK_OK;
}

// Row tiles per contraction task (MR) of the persistent rotation of GT gate
// tiles: forced by mk_set_team_rows, else, at N = 1024, the smallest team
// that keeps every compute unit of an XCD busy.  An XCD with 1 or 2 tiles
// runs teams of 32 (MR = 2) or 16 (MR = 4) workgroups, from 3 tiles on
// teams of 8 (MR = 8, the most MFMAs per key tile).  Other rings have one
// size.
int persist_team_rows(const mk_ctx *ctx, int GT) {
    const mk_params &P = ctx->p;
    const DeviceKeys &D = ctx->dev;
    const int NB = P.N / 32;
    if (NB != 32) return NB == 4 ? 2 : NB == 64 ? 8 : 4;
    if (D.team_rows) return D.team_rows;
    const int nx = std::max(1, D.num_xcd), cus = D.num_cus / nx;
    const int ntx = (GT + nx - 1) / nx;
    if (ntx <= 1 && cus >= 32) return 2;
    if (ntx <= 2 && cus >= 16) return 4;
    return 8;
}

// Teams number at most the tiles plus one per XCD.
size_t persist_ctl_words(int GT) { return (size_t)kCtlHeader + (size_t)(GT + 16) * kCtlPerTeam; }

bool persist_supported(const mk_params &P) {
    const int NB = P.N / 32;
    return (NB == 4 || NB == 8 || NB == 16 || NB == 32 || NB == 64) && P.bk_ell <= kMaxEll;
}

template <int NB, int MR>
static int launch_nb(mk_ctx *ctx, PersistArgs &pa, hipStream_t s) {
    const DeviceKeys &D = ctx->dev;
    auto kern = persist_rotation_kernel<NB, MR>;
    const size_t lds = std::max<size_t>({(size_t)kMaxRUnits * kRGates * NB * 32 * 4, (size_t)MR * kLimbTileBytes,
                                         (size_t)kKsRoundLds, (size_t)kKsGemmLds});
    if (lds > 65536)
        MK_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
               "persistent rotation LDS attribute");
    int occ = 0;
    MK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)kern, kPThreads, lds),
           "persistent rotation occupancy");
    occ = std::max(1, std::min(occ, PersistCfg<NB, MR>::OCC));
    constexpr int S = 2 * (NB / MR);
    const int per_xcd = occ * (D.num_cus / D.num_xcd);   // workgroups an XCD holds at once
    if (S > per_xcd) return fail(MK_EPARAM, "persistent rotation: a team does not fit on one XCD");
    const int GT = pa.m.GP / 32;
    const int ntx_max = (GT + D.num_xcd - 1) / D.num_xcd;
    const int fit = per_xcd / S;                          // teams an XCD holds at once
    pa.c = (ntx_max + fit - 1) / fit;
    pa.teams_max = (ntx_max + pa.c - 1) / pa.c;
    // round-robin dispatch gives each XCD grid / nx workgroups
    const int grid = D.num_xcd * pa.teams_max * S;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kPThreads), lds, s, pa);
    MK_HIP(hipGetLastError(), "persistent rotation launch");
    return MK_OK;
}

// Runs CMux steps 0 .. steps-1 of the batch described by `m` (accumulator
// already initialised) as one persistent launch; with `ks`, the whole
// rotation followed by extraction and key switching into ks->out.
int launch_persist(mk_ctx *ctx, const MfmaArgs &m, int steps, uint32_t *ctl, const KsFused *ks, hipStream_t s) {
    const mk_params &P = ctx->p;
    DeviceKeys &D = ctx->dev;
    if (!persist_supported(P)) return fail(MK_EPARAM, "persistent rotation: parameters out of range");
    if (D.num_xcd <= 0 || D.num_cus < D.num_xcd) return fail(MK_ESTATE, "persistent rotation: XCDs not probed");
    if (steps <= 0) return MK_OK;
    PersistArgs pa;
    pa.m = m;
    pa.ctl = ctl;
    pa.status = D.status;
    pa.nx = D.num_xcd;
    pa.steps = steps;
    std::memcpy(pa.xmap, D.xmap, sizeof(pa.xmap));
    pa.spin_limit = 1u << 24;
    std::memset(&pa.ks, 0, sizeof(pa.ks));
    if (ks) {
        if (steps != P.k * P.n || ks->count != (size_t)m.G)
            return fail(MK_EINTERNAL, "fused key switching needs the whole rotation of the batch");
        pa.ks = *ks;
    }
    const int words = (int)persist_ctl_words(m.GP / 32);
    hipLaunchKernelGGL(zero_words_kernel, dim3((words + 255) / 256), dim3(256), 0, s, ctl, words);
    MK_HIP(hipGetLastError(), "persistent control clear");
    switch (P.N / 32) {
        case 4: return launch_nb<4, 2>(ctx, pa, s);
        case 8: return launch_nb<8, 4>(ctx, pa, s);
        case 16: return launch_nb<16, 4>(ctx, pa, s);
        case 32:
            switch (persist_team_rows(ctx, m.GP / 32)) {
                case 2: return launch_nb<32, 2>(ctx, pa, s);
                case 4: return launch_nb<32, 4>(ctx, pa, s);
                default: return launch_nb<32, 8>(ctx, pa, s);
            }
        default: return launch_nb<64, 8>(ctx, pa, s);
    }
}

}  // namespace mk

using namespace mk;

extern "C" {

int mk_set_rotation(mk_ctx *ctx, int kind) {
    if (!ctx || kind < MK_ROT_AUTO || kind > MK_ROT_PERSISTENT)
        return fail(MK_EINVAL, "mk_set_rotation: bad argument");
    ctx->dev.rot_kind = kind;
    return MK_OK;
}

int mk_set_team_rows(mk_ctx *ctx, int rows) {
    if (!ctx || (rows != 0 && rows != 2 && rows != 4 && rows != 8))
        return fail(MK_EINVAL, "mk_set_team_rows: rows must be 0, 2, 4 or 8");
    if (rows && ctx->p.N != 1024) return fail(MK_EINVAL, "mk_set_team_rows: team sizes are selectable at N = 1024 only");
    ctx->dev.team_rows = rows;
    return MK_OK;
}

int mk_get_team_rows(const mk_ctx *ctx, size_t count, int32_t *rows) {
    if (!ctx || !rows) return fail(MK_EINVAL, "mk_get_team_rows: null argument");
    const int GT = (int)((count + 31) / 32);
    *rows = use_persist(ctx, GT) ? persist_team_rows(ctx, GT) : 0;
    return MK_OK;
}

int mk_set_ks_fusion(mk_ctx *ctx, int on) {
    if (!ctx || (on != 0 && on != 1)) return fail(MK_EINVAL, "mk_set_ks_fusion: bad argument");
    ctx->dev.ks_fuse = on;
    return MK_OK;
}

int mk_device_status(mk_ctx *ctx, void *stream) {
    if (!ctx) return fail(MK_EINVAL, "mk_device_status: null context");
    DeviceKeys &D = ctx->dev;
    if (!D.uploaded || !D.status) return fail(MK_ESTATE, "evaluation key not uploaded (mk_upload_eval_key)");
    hipStream_t s = (hipStream_t)stream;
    uint32_t st = 0;
    MK_HIP(hipStreamSynchronize(s), "mk_device_status: stream sync");
    MK_HIP(hipMemcpy(&st, D.status, 4, hipMemcpyDeviceToHost), "mk_device_status: read");
    if (!st) return MK_OK;
    hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, s, D.status, 1);
    MK_HIP(hipGetLastError(), "mk_device_status: clear");
    MK_HIP(hipStreamSynchronize(s), "mk_device_status: clear sync");
    if (st & kStatusTimeout)
        return fail(MK_EDEVICE, "persistent rotation: a workgroup timed out waiting for its team (outputs invalid)");
    if (st & kStatusNoXcd) return fail(MK_EDEVICE, "persistent rotation: ran on an XCD the upload probe did not see");
    return fail(MK_EINVAL, "mk_bootstrap_gate: a gate type outside NAND..XNOR was evaluated as NAND");
}

}  // extern "C"
