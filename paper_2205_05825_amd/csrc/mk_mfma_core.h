// Device building blocks of the int8-MFMA blind rotation, shared by the
// stream-ordered kernels (mk_mfma.hip) and the persistent rotation
// (mk_persist.hip).
//
// A negacyclic product c_m = sum_p K'[m-p] u_p (mod 2^32) of int8 gadget
// digits u with a Torus32 key polynomial K (K'[s] = K[s] for s >= 0 and
// -K[s+N] for s < 0) is computed as sum_t 2^(8t) sum_p L_t(K'[m-p]) u_p with
// the key split into four signed 8-bit limbs L_t(x) = byte_t(x + 0x80808080)
// - 128; each inner sum is an exact int8 x int8 -> int32 contraction.  Key
// Toeplitz tiles (32x32, one per diagonal and limb) and digit tiles are
// stored as 1 KB fragments in the register layout of v_mfma_i32_32x32x32_i8.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace mk {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kTileBytes = 1024;

// Calls f(std::integral_constant<int, I>) for I = B .. E - 1.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}  // one 32x32 int8 fragment (64 lanes x 16 B)

// Digit kernels.  Fragment piece (slot or V, l, gate tile, K-block kb, lane
// L = 32 h + g) is the 16 bytes of digit l of coefficients 32 kb + 16 h ..
// + 15 of gate 32 gt + g: one thread computes one piece for all ell digits
// from 16 consecutive coefficients and writes ell 16-byte stores, so a wave
// writes whole 1 KB fragments (wdec) or 128-byte runs of them (rotdec).
constexpr int kMaxEll = 3;   // ell * 8 <= 30

__device__ __forceinline__ void put_digits(int8_t *dst_l0, size_t l_stride, int ell, const uint32_t (&y)[16]) {
    // digit l of y = byte (3 - l) of y (the offset folds in rounding and
    // the +128 bias), minus 128
#pragma unroll
    for (int l = 0; l < kMaxEll; ++l) {
        if (l >= ell) break;
        uint32_t w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            uint32_t v = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b)
                v |= ((((y[4 * q + b] >> (24 - 8 * l)) & 255u) - 128u) & 255u) << (8 * b);
            w[q] = v;
        }
        *reinterpret_cast<uint4 *>(dst_l0 + l * l_stride) = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

// ------------------------------------------------------------- GEMMs ----
//
// A wave computes MR row tiles (32 output coefficients each) of NC gate
// tiles: acc[r][c][t] accumulates sum_l T_t(A_l) B_l over the ell key
// polynomials A_l and the NB K-blocks, for the 4 limbs t.  The Toeplitz
// tile at (row tile mb, K-block kb) is diagonal tile mb - kb.
//
// Skewed schedule: at step x, row tile r works on K-block x + r, whose tile
// is diagonal mb0 - x =: s(x) for every r, so all MR row tiles share one key
// tile per limb per step and the digit tiles slide past them instead.  For
// each l the steps run x = -(MR-1) .. NB-1 (P = NB + MR - 1 steps); a row
// tile whose K-block lies outside [0, NB) meets a digit tile that reads as
// zero.  Flattened over l, step X = l P + y (y = x + MR - 1) loads the key
// tiles alpha(X) = s_l(x) and the digit tiles beta(X) = B_l[K-block y] (zero
// for y >= NB), and row tile r multiplies alpha(X) by beta(X - MR + 1 + r):
// the stream is uniform across the l boundaries (the MR - 1 zero digit tiles
// at the end of each l are exactly what the first steps of the next l see),
// so the load pipeline never drains between key polynomials.
//
// Loads are buffer loads through wave-uniform descriptors: accesses are
// bounded by the operand blocks, reads out of range return 0 (used for the
// zero tiles), and, unlike plain loads, the compiler does not merge the
// rings' loads back into a load at the point of use.
constexpr uint32_t kBufWord3 = 0x00020000u;  // raw dword buffer, gfx9 family
constexpr uint32_t kOutOfRange = 0x80000000u;  // offset beyond every block
// Cache policy of loads that must see stores made by other compute units of
// the same XCD during one launch: device scope (sc1) bypasses the compute
// unit's vector L1, whose lines are not kept coherent with other units'
// stores, and reads the XCD's L2.
constexpr int kCoherent = 16;

struct Operands {
    const int8_t *A;   // [ell][4][ND][1024] key tiles
    const int8_t *B;   // digit tiles of l = 0 and the wave's first gate tile
    uint32_t b_poly;   // bytes between the digit tiles of consecutive l
    int ell, NB, mb0, nc_valid;
};

// Position in the flattened step stream: the byte offsets of limb 0 of
// alpha and of gate tile 0 of beta there, and rem = P - y, the steps left
// in the current key polynomial.  Advancing is branch-free and costs a few
// scalar instructions (the wrap to the next l is one select), so the
// compiler keeps every load of the unrolled loop in one basic block and its
// load counters exact.  Past the last polynomial both offsets run beyond
// their descriptors' ranges and the loads return zeros.
struct Cursor {
    uint32_t a, b;
    int rem;
};

// Digit K-block of step y is y - dshift (0 for the skewed schedule, MR - 1
// for the windowed one).  Only the skewed schedule multiplies digit tiles
// outside [0, NB), which must read as zero (zero_edges).
struct Streams {
    __amdgpu_buffer_rsrc_t ra, rb;
    int NB, ND, P, MRm1, dshift, nc_valid;
    uint32_t lane16, a_wrap, b_wrap, limb_stride, tile_stride, b_poly, mb0;
    __device__ __forceinline__ Streams(const Operands &o, int MR, int lane, int dshift_) {
        const int ell = o.ell;
        NB = o.NB; ND = 2 * NB - 1; P = NB + MR - 1; MRm1 = MR - 1; dshift = dshift_;
        nc_valid = o.nc_valid; lane16 = (uint32_t)lane * 16; b_poly = o.b_poly; mb0 = (uint32_t)o.mb0;
        limb_stride = (uint32_t)ND * kTileBytes;
        tile_stride = (uint32_t)NB * kTileBytes;
        // offset change from (l, P-1) to (l+1, 0) beyond the usual step
        a_wrap = (uint32_t)(4 * ND + P) * kTileBytes;
        b_wrap = b_poly - (uint32_t)P * kTileBytes;
        ra = __builtin_amdgcn_make_buffer_rsrc((void *)o.A, (short)0, ell * 4 * ND * kTileBytes, kBufWord3);
        const int nv = nc_valid > 0 ? nc_valid : 0;
        rb = __builtin_amdgcn_make_buffer_rsrc((void *)o.B, (short)0,
                                               (int)((ell - 1) * b_poly + nv * NB * kTileBytes), kBufWord3);
    }
    __device__ __forceinline__ Cursor at(int X) const {  // setup only (divides)
        const int l = X / P, y = X - l * P;
        Cursor q;
        q.a = (uint32_t)((4 * l * ND + (int)mb0 - (y - MRm1) + NB - 1) * kTileBytes);
        q.b = (uint32_t)l * b_poly + (uint32_t)((y - dshift) * kTileBytes);
        q.rem = P - y;
        return q;
    }
    __device__ __forceinline__ void next(Cursor &q) const {
        q.a -= kTileBytes;
        q.b += kTileBytes;
        q.rem -= 1;
        // all ones when rem reached 0 (integer mask: no lane-mask selects)
        const uint32_t m = (uint32_t)((q.rem - 1) >> 31);
        q.a += a_wrap & m;
        q.b += b_wrap & m;
        q.rem += P & (int)m;
    }
    // per-wave vector offsets: limb t of alpha, gate tile c of beta (gate
    // tiles beyond the batch read zeros)
    __device__ __forceinline__ uint32_t key_lane(int t) const { return t * limb_stride + lane16; }
    __device__ __forceinline__ uint32_t dig_lane(int c) const {
        return c < nc_valid ? c * tile_stride + lane16 : kOutOfRange + lane16;
    }
    __device__ __forceinline__ v4i key(const Cursor &q, uint32_t vlane) const {
        return (v4i)__builtin_amdgcn_raw_buffer_load_b128(ra, q.a + vlane, 0, 0);
    }
    // digit K-block y - dshift; with zero_edges, K-blocks outside [0, NB)
    // (y >= NB for the skewed schedule) read as zero
    // Quarter `t` of the digit tile at the cursor: 4 bytes per lane, bytes
    // 256 t + 4 lane of the 1 KB fragment (zero outside the operand block).
    template <int AUX = 0>
    __device__ __forceinline__ uint32_t digit_quarter(const Cursor &q, uint32_t vq) const {
        return (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rb, q.b + vq, 0, AUX);
    }
    // AUX: cache-policy bits of the load (kCoherent for digits that other
    // compute units wrote during the same launch)
    template <bool zero_edges, int AUX = 0>
    __device__ __forceinline__ v4i digits(const Cursor &q, uint32_t vlane) const {
        uint32_t uni = q.b;
        if constexpr (zero_edges) uni |= q.rem > P - NB ? 0u : kOutOfRange;
        return (v4i)__builtin_amdgcn_raw_buffer_load_b128(rb, uni + vlane, 0, AUX);
    }
};

constexpr int kWaves = 4;   // waves per workgroup

// Task decode shared by both GEMMs.  A wave owns MR row tiles (of 32 rows)
// of NC consecutive 32-gate tiles; a workgroup's four waves share the row
// block and the unit (so the key tiles they load are shared through the
// CU's L1 or LDS) and cover 4 NC gate tiles.  The gate group is the fastest
// index: with 8 gate groups each XCD keeps one group's digits in its L2.
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
    // readfirstlane: the wave index is uniform, so are the operand pointers
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
    t.gt0 = (gg * kWaves + wave) * NC;
    t.nc_valid = GT - t.gt0 < NC ? GT - t.gt0 : NC;
    return t;
}

// Output register e of row tile r, gate tile c holds row 32 (rb MR + r) +
// 8 (e / 4) + 4 (lane / 32) + e % 4 of gate 32 (gt0 + c) + lane % 32, so
// registers 4q..4q+3 are four consecutive words of one gate's row.
template <int MR>
__device__ __forceinline__ uint32_t *tile_row(uint32_t *base, size_t gate_stride, const Task &tk,
                                              int c, int r, int lane) {
    const int g = (tk.gt0 + c) * 32 + (lane & 31);
    return base + (size_t)g * gate_stride + 32 * (tk.rb * MR + r) + 4 * (lane / 32);
}

// ---------------------------------------------------- limb-split GEMMs ----
//
// The workgroup's four waves compute the four limb products of the same MR
// row tiles x NC gate tiles: wave t accumulates S_t = sum_l T_t(A_l) B_l
// (one accumulator tile per row tile and gate tile) and the limbs are
// combined, sum_t 2^(8t) S_t, through LDS at the end.  Per step a wave
// loads one key tile and NC digit tiles for MR NC MFMAs; the digit tiles
// are shared by the four waves through the CU's L1.
//
// Windowed schedule over a flattened stream: per key polynomial l the steps
// run y = 0 .. P - 1 (P = NB + MR - 1); step y loads s_l(y - MR + 1) of limb
// t (s(x) = diagonal tile mb0 - x) and the digit tiles of K-block
// y - MR + 1, and for y >= MR - 1, i.e. K-block kb = y - MR + 1 >= 0, row
// tile r multiplies s(kb - r), loaded r steps earlier, by the digit tiles
// of K-block kb.  The first MR - 1 steps of every l only fill the window,
// so the load pipeline runs on through the l boundaries.  Rings: key tiles
// in RA = 2 MR slots (window MR, prefetch D <= MR - 1), digit tiles in
// RB = D + 1 slots (prefetch D), s(X) and beta(X) in slot X mod RA / RB,
// the loop unrolled RA times so that every slot index is a compile-time
// constant; with equal prefetch distances one cursor drives both streams.
template <int MR, int NC, int DAUX = 0, class Init>
__device__ __forceinline__ void limb_gemm(const Operands &o, int t, int lane, v16i (&acc)[MR][NC],
                                          Init init) {
    // keys and digits are prefetched the same D steps ahead, so one cursor
    // serves both streams (D = MR - 1, or 3 with two gate tiles to spare
    // registers)
    constexpr int D = NC == 1 ? MR - 1 : 3, RA = 2 * MR, RB = D + 1, U = RA;
    static_assert(U % RB == 0, "ring sizes must divide the unroll");
    const Streams S(o, MR, lane, MR - 1);
    const int P = S.P, steps = o.ell * P, W = MR - 1;
    const uint32_t vk = S.key_lane(t);
    uint32_t vd[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) vd[c] = S.dig_lane(c);
    v4i win[RA], sb[RB][NC];
    Cursor q = S.at(0);
    // alpha(0..D-1) and beta(0..D-1), in the order the loop issues them
#pragma unroll
    for (int x = 0; x < D; ++x) {
        win[x] = S.key(q, vk);
#pragma unroll
        for (int c = 0; c < NC; ++c) sb[x][c] = S.digits<false, DAUX>(q, vd[c]);
        S.next(q);
        __builtin_amdgcn_sched_barrier(0);
    }
    init();  // may load and set acc, once the prologue's loads are in flight
    int ys = 0;  // y of the current step
    // Step X first loads alpha(X + D) over alpha(X - MR - 1) and beta(X + D)
    // over beta(X - 1), then multiplies.
    auto step = [&](int u) {  // u = X mod U
        win[(u + D) % RA] = S.key(q, vk);
#pragma unroll
        for (int c = 0; c < NC; ++c) sb[(u + D) % RB][c] = S.digits<false, DAUX>(q, vd[c]);
        S.next(q);
        if (ys >= W) {
#pragma unroll
            for (int r = 0; r < MR; ++r)
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    acc[r][c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(win[(u - r + RA) % RA], sb[u % RB][c],
                                                                      acc[r][c], 0, 0, 0);
        }
        ys = ys + 1 == P ? 0 : ys + 1;
        __builtin_amdgcn_sched_barrier(0);
    };
    int X = 0;
    for (; X + U <= steps; X += U) {
#pragma unroll
        for (int u = 0; u < U; ++u) step(u);
    }
#pragma unroll
    for (int u = 0; u < U - 1; ++u)
        if (X + u < steps) step(u);
}

// Seamless limb-split contraction.  Wave t holds key limb t of MR row
// tiles (rows mb0 .. mb0 + MR - 1) of one gate tile; the K range is the
// flattened sequence F = l NB + kb of (key polynomial l, K-block kb).  At
// global step X, row tile r multiplies K-block F = X + r: the Toeplitz tile
// of polynomial l = F / NB there is diagonal mb0 - X + l NB, the same for
// every row that is on polynomial l.  So one key tile serves all rows of a
// step, two where the rows straddle a polynomial boundary, and one new digit
// tile enters per step: no step waits for a window to refill at the start
// of a polynomial, unlike the windowed schedule, and only the MR - 1 steps
// at each end of the whole stream multiply zero tiles.  The steps are
// unrolled by polynomial (iteration i covers X = i NB .. i NB + NB - 1; in
// it, rows with x + r >= NB already work on polynomial i + 1), so every ring
// slot is a compile-time constant:
//   main keys  (polynomial i, step x)      ring RK, slot x % RK
//   next keys  (polynomial i + 1, x >= NB - MR + 1)  MR - 1 slots
//   digits     (local K index c = x + r)   ring RB, slot c % RB
// with every tile loaded D steps before its first use.  Iteration -1 runs
// only the steps that load the first tiles and multiply polynomial 0's
// leading rows.  Key and digit loads of polynomials outside [0, ell) read
// zeros.  DAUX is the digits' cache policy.
__host__ __device__ constexpr int pow2_at_least(int v) {
    int m = 1;
    while (m < v) m *= 2;
    return m;
}
template <int MR, int NB, int D, int DAUX, int NC, bool SEG, int PF, class Init, class Pre, class Put, class Settle>
__device__ __forceinline__ void slide_core(const Operands &o, int seg, int t, int lane, v16i (&acc)[MR][NC], Init init,
                                           Pre pre, Put put, Settle settle) {
    constexpr int ND = 2 * NB - 1;
    constexpr int RK = pow2_at_least(D + 1), RB = pow2_at_least(MR + D);
    constexpr int RN = MR > 1 ? MR - 1 : 1;
    constexpr int X0 = NB - MR + 1;   // first step whose rows straddle polynomials
    static_assert(NB % RK == 0 && NB % RB == 0 && D + MR - 1 < NB && D < X0, "ring sizes for this N");
    const int ell = o.ell;
    const int nv = o.nc_valid > 0 ? o.nc_valid : 0;
    const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
        (void *)o.A, (short)0, (SEG ? seg : ell) * 4 * ND * kTileBytes, kBufWord3);
    const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(
        (void *)o.B, (short)0, (int)((ell - 1) * o.b_poly + nv * NB * kTileBytes), kBufWord3);
    const uint32_t lane16 = (uint32_t)lane * 16;
    const uint32_t kpoly = 4u * ND * kTileBytes;
    const uint32_t klimb = (uint32_t)t * ND * kTileBytes + lane16;
    // per-gate-tile digit offsets (gate tiles beyond the batch read zeros)
    uint32_t vd[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) vd[c] = c < o.nc_valid ? (uint32_t)c * NB * kTileBytes + lane16 : kOutOfRange;
    // byte offsets of polynomial p's main-row key at x = 0, its next-row key
    // at x = 0 (the term - x KB is added per step), and its digit block;
    // with segments, polynomial p multiplies key p mod seg
    auto kpos = [&](int p) -> uint32_t { return (uint32_t)(SEG ? p % seg : p) * kpoly; };
    auto kmain = [&](int p) -> uint32_t {
        return (p >= 0 && p < ell) ? kpos(p) + klimb + (uint32_t)(o.mb0 + NB - 1) * kTileBytes : kOutOfRange;
    };
    auto knext = [&](int p) -> uint32_t {   // p = polynomial of the next rows
        return (p >= 0 && p < ell) ? kpos(p) + klimb + (uint32_t)(o.mb0 + 2 * NB - 1) * kTileBytes
                                   : kOutOfRange;
    };
    // digit block of polynomial p, gate tile g (zeros outside the operand)
    auto dpoly = [&](int p, int g) -> uint32_t {
        return (p >= 0 && p < ell && vd[g] != kOutOfRange) ? (uint32_t)p * o.b_poly + vd[g] : kOutOfRange;
    };
    v4i km[RK], kn[RN], dg[RB][NC];
    // offsets of iteration i (current) and i + 1 (next)
    uint32_t km_i, km_n, kn_i, dg_i[NC], dg_n[NC];
    auto set_iter = [&](int i) {
        km_i = kmain(i);
        km_n = kmain(i + 1);
        kn_i = knext(i + 1);
#pragma unroll
        for (int g = 0; g < NC; ++g) {
            dg_i[g] = dpoly(i, g);
            dg_n[g] = dpoly(i + 1, g);
        }
    };
    auto ldk = [&](uint32_t off) -> v4i { return (v4i)__builtin_amdgcn_raw_buffer_load_b128(ra, off, 0, 0); };
    auto ldd = [&](uint32_t off) -> v4i { return (v4i)__builtin_amdgcn_raw_buffer_load_b128(rb, off, 0, DAUX); };
    // loads issued at step x of an iteration: main key of step x + D, next
    // key of step x + D if that straddles, digits of c = x + MR - 1 + D
    auto issue = [&](auto xc) {
        constexpr int x = decltype(xc)::value;
        constexpr int xk = x + D;
        if constexpr (xk < NB) km[xk % RK] = ldk(km_i - (uint32_t)xk * kTileBytes);
        else km[xk % RK] = ldk(km_n - (uint32_t)(xk - NB) * kTileBytes);
        if constexpr (xk >= X0 && xk < NB) kn[xk - X0] = ldk(kn_i - (uint32_t)xk * kTileBytes);
        constexpr int c = x + MR - 1 + D;
#pragma unroll
        for (int g = 0; g < NC; ++g) {
            if constexpr (c < NB) dg[c % RB][g] = ldd(dg_i[g] + (uint32_t)c * kTileBytes);
            else dg[c % RB][g] = ldd(dg_n[g] + (uint32_t)(c - NB) * kTileBytes);
        }
    };
    // multiplications of step x: rows on polynomial i (main, skipped in the
    // leading iteration) and rows already on polynomial i + 1 (in the last
    // iteration their key tiles read as zero).  The row whose K range ends
    // at this step (x = NB - 1 - r) goes first, so that its result is ready
    // while the step's other products run.
    auto mult = [&](auto xc, auto lead) {
        constexpr int x = decltype(xc)::value;
        constexpr int r0 = (NB - 1 - x >= 0 && NB - 1 - x < MR) ? NB - 1 - x : 0;
#pragma unroll
        for (int k = 0; k < MR; ++k)
#pragma unroll
            for (int g = 0; g < NC; ++g) {
                const int r = (k + r0) % MR;
                if (x + r < NB) {
                    if constexpr (!decltype(lead)::value)
                        acc[r][g] = __builtin_amdgcn_mfma_i32_32x32x32_i8(km[x % RK], dg[(x + r) % RB][g], acc[r][g],
                                                                          0, 0, 0);
                } else {
                    // reached only for x >= X0 (r <= MR - 1)
                    acc[r][g] = __builtin_amdgcn_mfma_i32_32x32x32_i8(kn[x >= X0 ? x - X0 : 0], dg[(x + r) % RB][g],
                                                                      acc[r][g], 0, 0, 0);
                }
            }
    };
    // iteration -1: steps X0 - D .. NB - 1 (loads from the first; the
    // leading rows of polynomial 0 multiply from X0 on)
    set_iter(-1);
    static_for<X0 - D, NB>([&](auto xc) {
        constexpr int x = decltype(xc)::value;
        issue(xc);
        if constexpr (x >= X0) {
            if constexpr (x == X0) init();   // once the first loads are in flight
            mult(xc, std::true_type{});
        }
        __builtin_amdgcn_sched_barrier(0);
    });
    [[maybe_unused]] v4i old[MR];
    int s = 0, left = seg;   // segments: segment of iteration i, iterations left in it
    for (int i = 0; i < ell; ++i) {
        set_iter(i);
        // segment boundary: rows finish segment s in this iteration
        [[maybe_unused]] bool last = false;
        if constexpr (SEG) last = --left == 0;
        static_for<0, NB>([&](auto xc) {
            constexpr int x = decltype(xc)::value;
            issue(xc);
            if constexpr (SEG) {
                // row rp finishes PF steps from now: fetch what settle needs
                constexpr int rp = NB - 1 - (x + PF);
                if constexpr (rp >= 0 && rp < MR)
                    if (last) old[rp] = pre(rp, s);
            }
            mult(xc, std::false_type{});
            if constexpr (SEG) {
                // row rf multiplied the last K-block of the segment at this step
                constexpr int rf = NB - 1 - x;
                if constexpr (rf >= 0 && rf < MR)
                    if (last) {
                        put(rf);
                        acc[rf][0] = v16i{};
                    }
            }
            __builtin_amdgcn_sched_barrier(0);
        });
        if constexpr (SEG)
            if (last) {
                settle(s, old);
                ++s;
                left = seg;
            }
    }
}

template <int MR, int NB, int D, int DAUX, int NC = 1, class Init>
__device__ __forceinline__ void slide_gemm(const Operands &o, int t, int lane, v16i (&acc)[MR][NC], Init init) {
    slide_core<MR, NB, D, DAUX, NC, false, 0>(o, 0, t, lane, acc, init, [](int, int) { return v4i{}; },
                                              [](int) {}, [](int, const v4i (&)[MR]) {});
}

// The seamless contraction over o.ell = S seg polynomials cut into S
// segments of seg: polynomial p multiplies key polynomial p mod seg (the
// same key for every segment) and digit block p.  Row tile r finishes
// segment s at step NB - 1 - r of the segment's last iteration: right after
// that multiplication put(r) takes the row's limb accumulators (acc[r]),
// which restart from zero for segment s + 1 with the row's next product
// (one step later).  After the iteration, settle(s, old) completes the
// segment's rows; old[r] is what pre(r, s) returned, PF steps before row
// r's put (a load in flight meanwhile).  Rows finish one per step, from
// r = MR - 1 to 0.
template <int MR, int NB, int D, int DAUX, int PF, class Pre, class Put, class Settle>
__device__ __forceinline__ void slide_gemm_seg(const Operands &o, int seg, int t, int lane, v16i (&acc)[MR][1],
                                               Pre pre, Put put, Settle settle) {
    static_assert(NB - MR - PF >= 0, "the first prefetch must fall inside the segment's last iteration");
    slide_core<MR, NB, D, DAUX, 1, true, PF>(o, seg, t, lane, acc, []() {}, pre, put, settle);
}

// Limb-split contraction whose digit tiles reach the four waves through
// LDS, for digits other compute units wrote during the same launch (loaded
// with policy DAUX): each wave loads one quarter of a tile (4 bytes per
// lane), writes it to a ring of four 1 KB LDS slots two steps ahead of use,
// and after the step's barrier every wave reads the next tile whole.  So a
// digit tile costs the workgroup one 1 KB read from L2 instead of four.  Step
// X: load alpha(X + D) and quarter beta(X + D); write quarter beta(X + 2)
// into slot (X + 2) % 4; multiply with beta(X) (read at the end of step X -
// 1); barrier; read beta(X + 1) from slot (X + 1) % 4.  The slot written at
// step X was last read at the end of step X - 3, before the barrier of step
// X - 2.  `lds` holds 4 KB.
template <int MR, int DAUX, class Init>
__device__ __forceinline__ void limb_gemm_lds(const Operands &o, int t, int lane, v16i (&acc)[MR][1], Init init,
                                              uint32_t *lds) {
    constexpr int D = MR - 1 > 3 ? MR - 1 : 3;
    constexpr int RA = (2 * MR >= D + MR) ? 2 * MR : 2 * (D + MR), RQ = D + 1;
    constexpr int U = RA > RQ ? RA : RQ;
    static_assert(U % RA == 0 && U % RQ == 0 && U % 4 == 0, "ring sizes must divide the unroll");
    const Streams S(o, MR, lane, MR - 1);
    const int P = S.P, steps = o.ell * P, W = MR - 1;
    const uint32_t vk = S.key_lane(t);
    const uint32_t vq = 256u * (uint32_t)t + 4u * (uint32_t)lane;
    v4i win[RA], bt[2];
    uint32_t qr[RQ];
    Cursor q = S.at(0);
#pragma unroll
    for (int x = 0; x < D; ++x) {
        win[x] = S.key(q, vk);
        qr[x] = S.digit_quarter<DAUX>(q, vq);
        S.next(q);
        __builtin_amdgcn_sched_barrier(0);
    }
    // beta(0) and beta(1) into slots 0 and 1, then beta(0) to registers
    lds[0 * 256 + 64 * t + lane] = qr[0];
    lds[1 * 256 + 64 * t + lane] = qr[1];
    __syncthreads();
    bt[0] = *reinterpret_cast<const v4i *>(lds + 4 * lane);
    init();  // may load and set acc, once the prologue's loads are in flight
    int ys = 0;  // y of the current step
    auto step = [&](int u) {  // u = X mod U
        win[(u + D) % RA] = S.key(q, vk);
        qr[(u + D) % RQ] = S.digit_quarter<DAUX>(q, vq);
        S.next(q);
        lds[((u + 2) % 4) * 256 + 64 * t + lane] = qr[(u + 2) % RQ];
        if (ys >= W) {
#pragma unroll
            for (int r = 0; r < MR; ++r)
                acc[r][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(win[(u - r + RA) % RA], bt[u & 1], acc[r][0],
                                                                  0, 0, 0);
        }
        ys = ys + 1 == P ? 0 : ys + 1;
        __syncthreads();
        bt[(u + 1) & 1] = *reinterpret_cast<const v4i *>(lds + ((u + 1) % 4) * 256 + 4 * lane);
        __builtin_amdgcn_sched_barrier(0);
    };
    int X = 0;
    for (; X + U <= steps; X += U) {
#pragma unroll
        for (int u = 0; u < U; ++u) step(u);
    }
#pragma unroll
    for (int u = 0; u < U - 1; ++u)
        if (X + u < steps) step(u);
}

// Read-modify-write seed: the old output tiles start wave 0's accumulators
// (low 24 bits) and wave 3's (high 8 bits), which keeps every limb sum
// inside int32 and makes the combined sum old + product.  Loaded after the
// contraction's first loads are issued, so both latencies overlap.
template <int MR, int NC>
__device__ __forceinline__ void load_old(const uint32_t *base, size_t gate_stride, const Task &tk,
                                         int lane, v16i (&acc)[MR][NC]) {
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int r = 0; r < MR; ++r) {
            const uint32_t *row = tile_row<MR>(const_cast<uint32_t *>(base), gate_stride, tk,
                                               c < tk.nc_valid ? c : 0, r, lane);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint4 v = *reinterpret_cast<const uint4 *>(row + 8 * q);
                acc[r][c][4 * q + 0] = (int)v.x;
                acc[r][c][4 * q + 1] = (int)v.y;
                acc[r][c][4 * q + 2] = (int)v.z;
                acc[r][c][4 * q + 3] = (int)v.w;
            }
        }
}
template <int MR, int NC>
__device__ __forceinline__ void seed_old(int t, v16i (&acc)[MR][NC]) {
#pragma unroll
    for (int r = 0; r < MR; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int e = 0; e < 16; ++e)
                acc[r][c][e] = t == 0 ? (int)((uint32_t)acc[r][c][e] & 0xFFFFFFu)
                                      : (int)((uint32_t)acc[r][c][e] >> 24);
}

// Combines the four waves' limb sums and stores the valid gate tiles.  Tile
// i = (r, c) passes through LDS buffer i % 2 ([4 limbs][4 quads][64 lanes]
// of uint4): wave t writes its registers shifted by 8t, and after the
// barrier sums the four limbs of quad t, i.e. words 8t..8t+3 of its lane's
// rows, and stores them.  The second buffer lets tile i+1 be written while
// tile i is still being read; tile i+2 reuses buffer i % 2 only after the
// barrier of tile i+1, which every wave passes after its reads of tile i.
template <int MR, int NC>
__device__ __forceinline__ void combine_store(uint32_t *base, size_t gate_stride, const Task &tk, int t,
                                              int lane, const v16i (&acc)[MR][NC], uint4 *red) {
#pragma unroll
    for (int i = 0; i < MR * NC; ++i) {
        const int r = i / NC, c = i % NC;
        uint4 *buf = red + (i & 1) * 4 * 4 * 64;
        const uint32_t sh = 8u * (uint32_t)t;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            buf[(t * 4 + q) * 64 + lane] =
                make_uint4((uint32_t)acc[r][c][4 * q + 0] << sh, (uint32_t)acc[r][c][4 * q + 1] << sh,
                           (uint32_t)acc[r][c][4 * q + 2] << sh, (uint32_t)acc[r][c][4 * q + 3] << sh);
        __syncthreads();
        uint4 sum = buf[t * 64 + lane];
#pragma unroll
        for (int s = 1; s < 4; ++s) {
            const uint4 v = buf[(s * 4 + t) * 64 + lane];
            sum.x += v.x;
            sum.y += v.y;
            sum.z += v.z;
            sum.w += v.w;
        }
        if (c < tk.nc_valid) *reinterpret_cast<uint4 *>(tile_row<MR>(base, gate_stride, tk, c, r, lane) + 8 * t) = sum;
    }
}

// Register rings of R = MR + D slots (D = max(MR, 2) steps of prefetch):
// alpha(X) and beta(X) live in slot X mod R.  The loop is unrolled R times
// so that every slot index is a compile-time constant (no register moves);
// after step X's MFMAs the slots of alpha(X - MR + 1) and beta(X - MR + 1),
// no longer needed, receive alpha(X + D + 1) and beta(X + D + 1).
// DP overrides the prefetch depth; steps X0 .. X0 + nsteps - 1 of the
// stream are run (default: all of them).  A start X0 > 0 needs MR = 1, whose
// steps use no digit tile of an earlier step.
template <int MR, int NC, int DP = 0, int DAUX = 0, class Init>
__device__ __forceinline__ void toeplitz_gemm(const Operands &o, int lane, v16i (&acc)[MR][NC][4],
                                              Init init, int X0 = 0, int nsteps = -1) {
    constexpr int D = DP > 0 ? DP : (MR > 2 ? MR : 2), R = MR + D;
    const Streams S(o, MR, lane, 0);
    const int steps = nsteps >= 0 ? nsteps : o.ell * S.P;
    uint32_t vk[4], vd[NC];
#pragma unroll
    for (int t = 0; t < 4; ++t) vk[t] = S.key_lane(t);
#pragma unroll
    for (int c = 0; c < NC; ++c) vd[c] = S.dig_lane(c);
    v4i sa[R][4], sb[R][NC];
#pragma unroll
    for (int i = 1; i < MR; ++i)
#pragma unroll
        for (int c = 0; c < NC; ++c) sb[R - i][c] = v4i{};  // beta(-i) = 0
    Cursor q = S.at(X0);
#pragma unroll
    for (int x = 0; x <= D; ++x) {
#pragma unroll
        for (int t = 0; t < 4; ++t) sa[x][t] = S.key(q, vk[t]);
#pragma unroll
        for (int c = 0; c < NC; ++c) sb[x][c] = S.digits<true, DAUX>(q, vd[c]);
        S.next(q);
        __builtin_amdgcn_sched_barrier(0);  // issue in ring order
    }
    init();  // sets acc, once the prologue's loads are in flight
    auto step = [&](int u) {  // u = X mod R
#pragma unroll
        for (int r = 0; r < MR; ++r)
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    acc[r][c][t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                        sa[u][t], sb[(u - MR + 1 + r + R) % R][c], acc[r][c][t], 0, 0, 0);
#pragma unroll
        for (int t = 0; t < 4; ++t) sa[(u + D + 1) % R][t] = S.key(q, vk[t]);
#pragma unroll
        for (int c = 0; c < NC; ++c) sb[(u + D + 1) % R][c] = S.digits<true, DAUX>(q, vd[c]);
        S.next(q);
        // keep the scheduler from sinking these loads towards their use
        __builtin_amdgcn_sched_barrier(0);
    };
    // branch-free main loop (keeps the load counters exact), then the tail
    int X = 0;
    for (; X + R <= steps; X += R) {
#pragma unroll
        for (int u = 0; u < R; ++u) step(u);
    }
#pragma unroll
    for (int u = 0; u < R - 1; ++u)
        if (X + u < steps) step(u);
}

// Read-modify-write without a dependent load at the end: the old output
// values are loaded before the contraction starts (load_tiles) and become
// the accumulators' initial values once its first loads are in flight
// (seed_acc): the low 24 bits go to limb 0's accumulator and the high 8 bits
// to limb 3's, which keeps every limb sum inside int32 (|sum| < 2^30 by the
// setup bound) and recombines to the old value plus the product.
template <int MR, int NC>
__device__ __forceinline__ void load_tiles(const uint32_t *base, size_t gate_stride, const Task &tk,
                                           int lane, uint4 (&old)[MR][NC][4]) {
    // gate tiles beyond the batch (LDS shapes' idle waves) are never stored:
    // their accumulators start at 0; ragged tiles re-read tile 0
    if (tk.nc_valid <= 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int r = 0; r < MR; ++r)
#pragma unroll
                for (int q = 0; q < 4; ++q) old[r][c][q] = make_uint4(0, 0, 0, 0);
        return;
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int r = 0; r < MR; ++r) {
            const uint32_t *row = tile_row<MR>(const_cast<uint32_t *>(base), gate_stride, tk,
                                               c < tk.nc_valid ? c : 0, r, lane);
#pragma unroll
            for (int q = 0; q < 4; ++q) old[r][c][q] = *reinterpret_cast<const uint4 *>(row + 8 * q);
        }
}
template <int MR, int NC>
__device__ __forceinline__ void seed_acc(const uint4 (&old)[MR][NC][4], v16i (&acc)[MR][NC][4]) {
#pragma unroll
    for (int r = 0; r < MR; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t w[4] = {old[r][c][q].x, old[r][c][q].y, old[r][c][q].z, old[r][c][q].w};
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    acc[r][c][0][4 * q + i] = (int)(w[i] & 0xFFFFFFu);
                    acc[r][c][3][4 * q + i] = (int)(w[i] >> 24);
                }
            }
}

// Recombines the limbs of output register e of row tile r, gate tile c.
template <int MR, int NC>
__device__ __forceinline__ uint32_t combine(const v16i (&acc)[MR][NC][4], int r, int c, int e) {
    return (uint32_t)acc[r][c][0][e] + ((uint32_t)acc[r][c][1][e] << 8) +
           ((uint32_t)acc[r][c][2][e] << 16) + ((uint32_t)acc[r][c][3][e] << 24);
}

// out[rows of the wave's tiles] = limb-combined accumulators, for the valid
// gate tiles.
template <int MR, int NC>
__device__ __forceinline__ void store_tiles(uint32_t *base, size_t gate_stride, const Task &tk,
                                            int lane, const v16i (&acc)[MR][NC][4]) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        if (c >= tk.nc_valid) break;
#pragma unroll
        for (int r = 0; r < MR; ++r) {
            uint32_t *row = tile_row<MR>(base, gate_stride, tk, c, r, lane);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                *reinterpret_cast<uint4 *>(row + 8 * q) =
                    make_uint4(combine<MR, NC>(acc, r, c, 4 * q + 0), combine<MR, NC>(acc, r, c, 4 * q + 1),
                               combine<MR, NC>(acc, r, c, 4 * q + 2), combine<MR, NC>(acc, r, c, 4 * q + 3));
        }
    }
}

// Arguments of the rotation kernels.  Layouts (GP = gates padded to 32, GT =
// GP/32, NB = N/32, ND = 2 NB - 1):
//   acc  u32 [GP][k+1][N]                 W  u32 [k+1][GP][N]
//   U    i8  [k+1][ell][GT][NB][64][16]    V  i8  [ell][GT][NB][64][16]
//   bk   i8  [k][n][3][ell][4][ND][64][16]
//   evk  i8  [k+1][ell][4][ND][64][16]
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

}  // namespace mk
