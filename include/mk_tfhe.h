/*
 * mk_tfhe.h - C ABI of the MI355X (gfx950) multi-key TFHE gate-bootstrapping
 * library.
 *
 * The operations follow the paper's statement of the problem (Jiang et al.,
 * "Privacy-Preserving Distributed Machine Learning Made Faster"):
 *   §3.2  MKTFHE.Setup / KeyGen / SymEnc / SymDec / MKKeySwitch / NAND,
 *   §4.1  the bootstrapped AND/OR/NOR/XOR/XNOR gates, Eqs. (6)-(11), and the
 *         free NOT, Eq. (8),
 *   §4.3-§4.5  k-bit two's-complement adder, multiplier, subtractor and
 *         divider (Algs. 3-6), evaluated as layered gate netlists.
 * The scheme's internals, which the paper does not print, follow the
 * MKTFHE scheme it builds on (Chen, Chillotti, Song 2019): uni-encryption
 * bootstrapping keys, hybrid-product blind rotation, sample extraction and
 * per-party key switching.
 *
 * Conventions
 *   Torus32   a torus value x in [0,1) is the uint32_t round(x * 2^32).
 *   LWE ciphertext of k parties: words (b, a_1[0..n), ..., a_k[0..n)),
 *             kn+1 words, phase b + sum_i <a_i, s_i>; bit m is encoded as
 *             phase m/4.  Arrays of ciphertexts have a row stride of
 *             `stride` words (stride >= kn+1).
 *   Ownership the context owns all key material (host and device) and its
 *             device scratch; the caller owns every ciphertext buffer.
 *   Streams   device entry points are asynchronous on the given hipStream_t
 *             (passed as void*, NULL = default stream); host entry points are
 *             synchronous.  Device calls on one context share its scratch
 *             buffers, so calls on the same context must not overlap: issue
 *             them on one stream, or order the streams.  Contexts are
 *             independent of each other.  A context must not be used from two
 *             threads at once.
 *   Errors    0 on success, a negative MK_E* code otherwise; no exception
 *             crosses the ABI.  mk_last_error() returns a thread-local message
 *             describing the most recent failure on the calling thread.
 */
#ifndef MK_TFHE_H
#define MK_TFHE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ----------------------------------------------------------- codes ---- */
#define MK_OK 0
#define MK_EINVAL -1   /* bad argument (null pointer, range, size)        */
#define MK_ENOMEM -2   /* host or device allocation failed                */
#define MK_EDEVICE -3  /* a HIP call or kernel launch failed              */
#define MK_ESTATE -4   /* keys missing / evaluation key not uploaded      */
#define MK_EPARAM -5   /* parameters unsupported (see mk_setup)           */
#define MK_EINTERNAL -6 /* an internal consistency check failed          */

/* Gate types.  NAND..XNOR are bootstrapped (§4.1); NOT is free (Eq. (8)). */
#define MK_GATE_NAND 0
#define MK_GATE_AND 1
#define MK_GATE_OR 2
#define MK_GATE_NOR 3
#define MK_GATE_XOR 4
#define MK_GATE_XNOR 5
#define MK_GATE_NOT 6

/* Blind-rotation implementations (bit-identical results). */
#define MK_PATH_I32 0     /* exact 32-bit integer VALU products            */
#define MK_PATH_MFMA_I8 1 /* exact split-limb int8 MFMA products           */

/* ------------------------------------------------------- parameters ---- */
/*
 * Parameter set (symbols of Table 7 plus the party count k of §3.1).
 *   k              parties, 1..8
 *   n              LWE dimension
 *   N              ring dimension, a power of two in [16, 4096]
 *   bk_log_base    log2 of the gadget base B (must be 8: digits are int8)
 *   bk_ell         gadget length, with bk_log_base*bk_ell <= 30
 *   ks_log_base    log2 of the key-switching base B' (1..4)
 *   ks_t           key-switching digits, ks_log_base*ks_t <= 30
 *   *_noise_log2   noise standard deviation 2^-s in torus units for the
 *                  public/bootstrapping keys, key-switching keys and fresh
 *                  encryptions (1 <= s <= 40)
 * mk_setup rejects with MK_EPARAM sets for which the int8 contraction could
 * overflow its int32 accumulators: (k+1)*bk_ell*N*2^14 must be < 2^31.
 */
typedef struct mk_params {
    int32_t k, n, N;
    int32_t bk_log_base, bk_ell;
    int32_t ks_log_base, ks_t;
    int32_t bk_noise_log2, ks_noise_log2, lwe_noise_log2;
} mk_params;

typedef struct mk_ctx mk_ctx;

/* Circuit netlist for mk_eval_circuit (Algs. 3-6 are such netlists).
 * Wires 0 and 1 are the constants 0 and 1 (noiseless trivial ciphertexts);
 * wires 2..n_wires-1 are inputs or gate outputs.  Gates must be in
 * topological order; a gate of type MK_GATE_NOT ignores in2. */
typedef struct mk_gate {
    int32_t type, in1, in2, out;
} mk_gate;

typedef struct mk_circuit {
    int32_t n_wires;
    int32_t n_inputs;
    const int32_t *inputs;   /* wire id of each input                     */
    int32_t n_outputs;
    const int32_t *outputs;  /* wire id of each output                    */
    int32_t n_gates;
    const mk_gate *gates;
} mk_circuit;

/* ------------------------------------------------ setup and keys (host) -- */

/* §3.2 MKTFHE.Setup: validate `p` and sample the common reference string
 * a in T_N[X]^bk_ell from `seed`.  *out receives a new context (free it with
 * mk_free).  Errors: MK_EINVAL (null), MK_EPARAM (unsupported parameters),
 * MK_ENOMEM. */
int mk_setup(const mk_params *p, uint64_t seed, mk_ctx **out);

/* §3.2 MKTFHE.KeyGen for party `party` (0..k-1): LWE key s, ring key z,
 * public key pk = -z*a + e, bootstrapping key (a uni-encryption of every bit
 * of s under z), and key-switching key from z to s, all derived from `seed`
 * by the library's Philox4x64-10 streams.  Host only.  Errors: MK_EINVAL. */
int mk_keygen(mk_ctx *ctx, int party, uint64_t seed);

/* Serialise the keys of `party` (or the CRS with party = -1) into `buf`.
 * With buf == NULL only *len is set to the required size.  Layout (little
 * endian): "MKK1", int32 version=1, the 10 int32 of mk_params, int32 party,
 * then for party -1: crs u32[ell][N]; for a party: s u8[n], z u8[N],
 * pk u32[ell][N], bk u32[n][3][ell][N] (components d, f0, f1),
 * ks u32[N][t][B'-1][n+1] (rows (b, a)).  Errors: MK_EINVAL, MK_ESTATE. */
int mk_export_keys(const mk_ctx *ctx, int party, void *buf, size_t *len);

/* Load keys written by mk_export_keys (same parameters required).  Errors:
 * MK_EINVAL (size, magic or parameter mismatch). */
int mk_import_keys(mk_ctx *ctx, int party, const void *buf, size_t len);

/* The server-side "reconstruction" of the parties' keys into the evaluation
 * key (Alg. 7/8 step 1): copies the bootstrapping keys, the public keys
 * (as b_0 = -a, b_1..b_k) and the key-switching keys to the current HIP
 * device, in the layouts of both blind-rotation paths.  Synchronous on
 * `stream`.  Errors: MK_ESTATE (a party has no keys), MK_ENOMEM, MK_EDEVICE. */
int mk_upload_eval_key(mk_ctx *ctx, void *stream);

/* §3.2 MKTFHE.SymEnc by `party` of `count` bits (0/1), extended to k slots
 * (the other parties' slots are zero).  Randomness comes from `seed`
 * (message j uses stream index j).  out_host: count rows of stride_words
 * words (host memory).  Errors: MK_EINVAL, MK_ESTATE. */
int mk_encrypt(const mk_ctx *ctx, int party, const uint8_t *bits, size_t count,
               uint64_t seed, uint32_t *out_host, size_t stride_words);

/* §3.2 MKTFHE.SymDec with every party's secret key: bit = 1 iff the phase
 * is in [1/8, 5/8).  ct_host: host rows.  Errors: MK_EINVAL, MK_ESTATE. */
int mk_decrypt(const mk_ctx *ctx, const uint32_t *ct_host, size_t count,
               size_t stride_words, uint8_t *bits);

/* Noiseless ciphertexts of `bits` (b = bit/4, a = 0), host memory. */
int mk_trivial(const mk_ctx *ctx, const uint8_t *bits, size_t count,
               uint32_t *out_host, size_t stride_words);

/* ------------------------------------------------- device entry points -- */

/* MKNOT, Eq. (8): out = (0, 1/4) - in for `count` device rows; no
 * bootstrapping.  in/out may alias.  Errors: MK_EINVAL, MK_EDEVICE. */
int mk_not(const mk_ctx *ctx, const uint32_t *in_dev, uint32_t *out_dev,
           size_t count, size_t stride, void *stream);

/* Bootstrapped gates of §4.1 (Eqs. (6)-(11)) on `count` independent pairs:
 * out[g] = Boots_{types[g]}(in1[g], in2[g]).  All pointers are device
 * memory; rows have `stride` words.  Pipeline: pre-combination and modulus
 * switch, blind rotation (path MK_PATH_I32 or MK_PATH_MFMA_I8, identical
 * bits), sample extraction, multi-key key switching.  Batches larger than
 * one rotation launch takes (65536 gates, fewer when (k+1)*bk_ell*N*65536
 * reaches 2^31) run as consecutive chunks on `stream`.  `out` must not alias
 * the inputs.  The gate types are device memory, so they are checked on
 * the device: a type outside MK_GATE_NAND..MK_GATE_XNOR is evaluated as NAND
 * and recorded in the context's status word, which mk_device_status then
 * reports as MK_EINVAL.  Errors: MK_EINVAL (sizes, null pointers, path),
 * MK_ESTATE (mk_upload_eval_key not called), MK_ENOMEM, MK_EDEVICE. */
int mk_bootstrap_gate(mk_ctx *ctx, const uint8_t *gate_types_dev,
                      const uint32_t *in1_dev, const uint32_t *in2_dev,
                      uint32_t *out_dev, size_t count, size_t stride, int path,
                      void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as mk_bootstrap_gate, bit for bit, with every scratch buffer
 * in one fixed block of MK_NOALLOC_SCRATCH_BYTES per GPU (a static device
 * array that each GPU the library runs on holds until the process ends).
 * The call allocates and frees nothing; it does not split a batch over
 * streams and records no profiling events.  The block holds about 1000
 * gates at the Table 7 shape on MK_PATH_MFMA_I8 (about 61 KB per gate,
 * counted in 32-gate tiles); larger batches are refused with MK_EINVAL
 * before any work (split them).  Every call on one GPU, from any context,
 * uses the same block and leaves its contents behind: calls that may
 * overlap on one GPU (different streams, threads or contexts) race and
 * must be ordered by the caller.  Arguments, layouts and the other errors
 * are those of mk_bootstrap_gate. */
#define MK_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int mk_bootstrap_gate_noalloc(mk_ctx *ctx, const uint8_t *gate_types_dev,
                              const uint32_t *in1_dev, const uint32_t *in2_dev,
                              uint32_t *out_dev, size_t count, size_t stride,
                              int path, void *stream);

/* Evaluates `batch` independent instances of a netlist (Algs. 3-6).
 * in_dev: [n_inputs][batch][stride] words, out_dev: [n_outputs][batch]
 * [stride] words (device memory).  NOT gates and the constant wires are
 * folded into the consumers' pre-combination (exact mod 2^32), gates that no
 * output depends on are skipped, and the remaining gates are levelled by
 * bootstrapping depth; every level runs as one batch of all its gates over
 * all instances (in chunks, as in mk_bootstrap_gate, when wider than one
 * rotation launch).  The call returns after the work on `stream` has
 * completed.
 * Errors as mk_bootstrap_gate, plus MK_EINVAL for a malformed netlist
 * (undefined or redefined wires, gates out of topological order). */
int mk_eval_circuit(mk_ctx *ctx, const mk_circuit *c, const uint32_t *in_dev,
                    uint32_t *out_dev, size_t batch, size_t stride, int path,
                    void *stream);

/* An operator's whole level sequence captured as one HIP graph (the
 * batched, layered evaluation of mk_eval_circuit, replayed without host
 * work).  mk_circuit_graph_create plans `c` for `batch` instances, takes
 * the tile shapes tuned for each level's size at that moment, allocates the
 * graph's own device buffers (wires, descriptors and every scratch buffer
 * of the path, so later calls on the context cannot move them) and
 * captures, on a stream of its own, the evaluation reading in_dev and
 * writing out_dev (layouts as in mk_eval_circuit); in_dev and out_dev must
 * stay valid for the graph's lifetime.  The capture is cut into consecutive
 * pieces of about 1024 kernels (256 CMux steps), since a single graph of a
 * whole operator (thousands of kernels per level) is beyond what graph
 * instantiation handles.  Each mk_graph_launch on `stream` replays the
 * pieces in order and so evaluates the circuit on the current contents of
 * in_dev (the evaluation key must stay uploaded).  Launches of one graph
 * must not overlap (they share its buffers).  mk_graph_info reports the
 * number of levels, of bootstrapped gates per launch and of pieces (any
 * pointer may be NULL); mk_graph_destroy waits for the device and frees
 * everything.  Errors: those of mk_eval_circuit, plus
 * MK_EDEVICE when capture or instantiation fails. */
typedef struct mk_graph mk_graph;
int mk_circuit_graph_create(mk_ctx *ctx, const mk_circuit *c, const uint32_t *in_dev,
                            uint32_t *out_dev, size_t batch, size_t stride, int path,
                            mk_graph **graph);
int mk_graph_launch(mk_graph *graph, void *stream);
int mk_graph_info(const mk_graph *graph, int32_t *n_levels, int64_t *gates, int32_t *pieces);
int mk_graph_destroy(mk_graph *graph);

/* Graph piece size: mk_circuit_graph_create cuts its capture after about
 * `kernels` kernel nodes (default 1024).  Larger pieces mean fewer graph
 * launches per replay.  Values outside [64, 4096] (4096 kernels per graph
 * is the largest piece the test suite replays) are refused with MK_EINVAL;
 * a capture whose piece would still exceed 4096 kernels fails the same
 * way.  Takes effect for graphs created afterwards.  Host-only. */
int mk_set_graph_piece(mk_ctx *ctx, int kernels);

/* Host-side analysis of a netlist as mk_eval_circuit levels it: number of
 * bootstrapping levels, bootstrapped gates actually evaluated, widest level,
 * and wire slots needed per instance.  Any output pointer may be NULL.
 * Errors: MK_EINVAL for a malformed netlist. */
int mk_circuit_stats(const mk_circuit *c, int32_t *n_levels, int64_t *live_gates,
                     int32_t *max_width, int32_t *slots);

/* The wire-slot assignment behind mk_circuit_stats: for every wire w <
 * c->n_wires, slot[w] is the slot (per instance) that holds its ciphertext
 * (-1 for constants, NOT outputs and gates no output depends on) and
 * level[w] its bootstrapping level (0 for inputs, -1 where slot is -1).
 * A level's outputs never take a slot that a gate of that level or a later
 * one still reads; the planner checks this itself (MK_EINTERNAL otherwise).
 * Either pointer may be NULL; each array holds n_wires entries.
 * Errors: MK_EINVAL for a malformed netlist. */
int mk_circuit_slots(const mk_circuit *c, int32_t *slot, int32_t *level);

/* Stage entry points (the same kernels as mk_bootstrap_gate, exposed so that
 * each step can be checked on its own).
 *   mk_blind_rotate: abar_dev holds `count` rows of kn+1 uint32 values in
 *     [0, 2N) (modulus-switched b, a_1..a_k); acc_dev receives count rows of
 *     (k+1)*N words (the RLWE accumulator c_0..c_k) after the first
 *     `max_steps` CMux steps (all k*n when max_steps < 0).  This stage call
 *     is not chunked: on MK_PATH_MFMA_I8, MK_EINVAL when
 *     (k+1)*bk_ell*N*count (count rounded up to 32) reaches 2^31.
 *   mk_extract_keyswitch: acc_dev rows of (k+1)*N words -> out_dev LWE rows
 *     (sample extraction, + 1/8, key switching); MK_PATH_I32 sums the
 *     selected key-switching rows with 32-bit adds, MK_PATH_MFMA_I8 runs the
 *     same sums as a one-hot int8-MFMA GEMM per party (kept on 32-bit adds
 *     when a party's tile set would exceed 2 GiB).  Both are exact. */
int mk_blind_rotate(mk_ctx *ctx, const uint32_t *abar_dev, uint32_t *acc_dev,
                    size_t count, int max_steps, int path, void *stream);
int mk_extract_keyswitch(mk_ctx *ctx, const uint32_t *acc_dev,
                         uint32_t *out_dev, size_t count, size_t stride,
                         int path, void *stream);

/* Netlist builders (§4.3-§4.5).  Each writes into caller-provided arrays
 * sized by a first call with gates == NULL (which only sets *n_gates and
 * *n_wires).  Input wires: operand a bits (LSB first) then operand b bits;
 * output wires: result bits LSB first.  Operators:
 *   MK_OP_ADD   k-bit adder, carry-in 0, 5k gates (Alg. 3)
 *   MK_OP_SUB   k-bit subtractor: k XORs with 1, adder with carry-in 1, 6k
 *               gates (Alg. 5)
 *   MK_OP_MUL   signed k x k -> 2k-bit Baugh-Wooley array (Alg. 4's role)
 *   MK_OP_DIV   signed k-bit / k-bit truncating division: k quotient bits
 *               then k remainder bits, results mod 2^k (Alg. 6's role)
 *   MK_OP_DIV2  the same with a 2k-bit dividend (2k + k inputs)
 * kbits must be in [1, 64] ([2, 64] for MUL and DIV).  Errors: MK_EINVAL. */
#define MK_OP_ADD 0
#define MK_OP_SUB 1
#define MK_OP_MUL 2
#define MK_OP_DIV 3
#define MK_OP_DIV2 4
int mk_build_operator(int op, int kbits, mk_gate *gates, int32_t *n_gates,
                      int32_t *n_wires, int32_t *inputs, int32_t *outputs);

/* One fixed-point gradient-descent step of linear regression (§4.6) on Q8.8
 * int16 values: r_i = sum_j mulq(x_ij, w_j) - y_i, g_j = sum_i mulq(x_ij,
 * r_i), w_j' = w_j - (g_j >> shift), with mulq(a,b) = bits 8..23 of a*b and
 * sums mod 2^16.  Inputs: x (m*d values row-major), y (m), w (d), 16 bits
 * each LSB first; outputs: w' (d values).  Sizing as mk_build_operator.
 * Errors: MK_EINVAL (m*d > 4096, shift > 15). */
int mk_build_lr_step(int m, int d, int shift, mk_gate *gates, int32_t *n_gates,
                     int32_t *n_wires, int32_t *inputs, int32_t *outputs);

/* Closed-form one-feature linear regression (§3.4 Eqs. (2)-(3), Alg. 7) on
 * m pairs of signed 8-bit integers.  Sums are taken mod 2^16 and divisions
 * truncate toward zero (the divider array of MK_OP_DIV/DIV2):
 *   S_x = sum x_i, S_y = sum y_i; xbar = S_x / m, ybar = S_y / m (low 8 bits);
 *   dx_i = x_i - xbar, dy_i = y_i - ybar (mod 2^8);
 *   num = sum dy_i dx_i, den = sum dx_i dx_i (8 x 8 -> 16-bit products);
 *   slope = (num 2^frac) / den (32-bit dividend);
 *   intercept = (S_y 2^frac - slope S_x) / m (32-bit dividend, 16x16 product).
 * The centred sums equal Eq. (2)'s numerator and denominator in exact
 * arithmetic and keep the rounding of xbar, ybar small.  Inputs: x_0..x_{m-1}
 * then y_0..y_{m-1}, 8 bits each LSB first; outputs: slope then intercept,
 * 16 bits each, both with `frac` fractional bits.  The constant m enters as
 * constant wires.  Sizing as mk_build_operator.  Errors: MK_EINVAL (m outside
 * [1, 4096], frac outside [0, 15]). */
int mk_build_lr_formula(int m, int frac, mk_gate *gates, int32_t *n_gates, int32_t *n_wires,
                        int32_t *inputs, int32_t *outputs);

/* The comparison design of Table 2 (left column): gate `type` (NAND..XNOR,
 * or MK_GATE_NOT) built from bootstrapped NAND gates only, NOT included
 * (NOT a = NAND(a, a)); inputs a, b (b unused by NOT), one output.  Same
 * two-call convention as mk_build_operator.  Errors: MK_EINVAL. */
int mk_build_naive_gate(int type, mk_gate *gates, int32_t *n_gates, int32_t *n_wires,
                        int32_t *inputs, int32_t *outputs);

/* Kernel timing.  With level 1, every pipeline stage is bracketed by HIP
 * events recorded on the caller's stream; level 2 also brackets each kernel
 * of the int8-MFMA rotation; level 0 turns timing off.  mk_get_profile waits
 * for the events and returns accumulated milliseconds and launch counts for
 * MK_PROFILE_SLOTS slots: [0] pre-combination, [1] blind rotation (whole),
 * [2] extraction + key switching, [3] circuit bookkeeping, [4] MFMA stage-1
 * GEMM or the persistent rotation kernel, [5] MFMA stage-2 GEMM, [6] rotate
 * + decompose, [7] w decompose.
 * reset != 0 clears the accumulators.  Errors: MK_EINVAL. */
#define MK_PROFILE_SLOTS 8
int mk_set_profiling(mk_ctx *ctx, int level);
int mk_get_profile(mk_ctx *ctx, double *ms, int64_t *launches, int reset);

/* Tile shapes of the int8-MFMA rotation's two GEMM kernels.  Limb-split
 * shapes, where a workgroup's four waves hold the four key limbs of one
 * output block: 0 = 256 rows x 32 gates, 1 = 128 rows x 64 gates, 2 = 128
 * rows x 32 gates, 4 = 256 rows x 64 gates; shape 3 = one wave per 64 rows
 * x 32 gates with all four limbs; K-split shapes 5 (64 rows), 6 (32 rows)
 * and 7 (32 rows, each key polynomial's K range in two halves) x 32 gates,
 * where each of the workgroup's waves takes one part of the contraction
 * and their sums are added in LDS (short chains for small batches).
 * Results are identical for every shape; only speed differs.  Without
 * tuning a batch of GT 32-gate tiles uses gemm1 shape 6 (GT <= 2), 5
 * (GT <= 4), 3 (GT <= 12), else the first shape whose row count divides N;
 * gemm2 shape 6 (GT <= 4), 5 (GT <= 12), else 3.
 *   mk_autotune   times every shape of both kernels on the scratch buffers of
 *                 a batch of `count` gates (at most one rotation launch: larger
 *                 counts tune the chunk size they run in; synchronous on
 *                 `stream`) and
 *                 records the fastest for that batch size; ms (optional,
 *                 2 * MK_TILE_SHAPES floats) receives the average times,
 *                 gemm1 shapes first (0 for shapes that do not divide N/32).
 *                 It then tunes the shapes for half the batch and times a
 *                 few CMux steps of the whole batch run in one piece and as
 *                 two sub-batches on two streams (one's digit kernels and
 *                 GEMM tails overlapping the other's GEMMs), and records
 *                 the faster batch split for this size.
 *   mk_set_tiles  forces shapes (-1 = use the tuned or default shape).
 *   mk_get_tiles  reports the shapes a batch of `count` gates would use.
 *   mk_set_split  records the split of batches of `count` gates: 1 (whole),
 *                 2 (two sub-batches; needs count > 32) or 0 (forget).
 *   mk_get_split  reports it (1 unless tuned or set).  Splitting is skipped
 *                 at profiling level 2 and while `stream` is being captured
 *                 into a graph; results are identical either way.
 * Errors: MK_EINVAL, MK_ESTATE (key not uploaded), MK_ENOMEM, MK_EDEVICE. */
#define MK_TILE_SHAPES 8
int mk_autotune(mk_ctx *ctx, size_t count, void *stream, int32_t *gemm1_shape,
                int32_t *gemm2_shape, float *ms);
int mk_set_tiles(mk_ctx *ctx, int gemm1_shape, int gemm2_shape);
int mk_set_split(mk_ctx *ctx, size_t count, int parts);
int mk_get_split(const mk_ctx *ctx, size_t count, int32_t *parts);
int mk_get_tiles(const mk_ctx *ctx, size_t count, int32_t *gemm1_shape,
                 int32_t *gemm2_shape);

/* Schedule of the int8-MFMA blind rotation (§3.1: a level's gates are
 * independent, so all of them run together).  Both schedules give
 * bit-identical results.
 *   MK_ROT_STREAM      every CMux step is four stream-ordered kernels
 *                      (rotate + decompose, stage-1 GEMM, w decompose,
 *                      stage-2 GEMM), tile shapes as for mk_set_tiles.
 *   MK_ROT_PERSISTENT  all k*n CMux steps of a batch in one launch: every
 *                      32-gate tile is owned by one XCD, where a team of
 *                      workgroups runs it, meeting at a barrier after each
 *                      phase of a CMux step (rotate + decompose, stage 1,
 *                      stage 2).  Needs N in {128, 256, 512, 1024, 2048}.
 *   MK_ROT_AUTO        the persistent schedule where it is faster: at
 *                      N = 1024 for batches of at least one tile per XCD
 *                      (256 gates on MI355X), with teams sized to the batch
 *                      (mk_set_team_rows), at other N from 2.5 tiles per
 *                      XCD; stream-ordered kernels below (default).
 * Errors: MK_EINVAL. */
#define MK_ROT_AUTO -1
#define MK_ROT_STREAM 0
#define MK_ROT_PERSISTENT 1
int mk_set_rotation(mk_ctx *ctx, int kind);

/* Where the int8-MFMA path runs sample extraction and key switching (§3.2
 * MKKeySwitch) after a persistent rotation: on = 1 (default) inside the
 * rotation's own launch, each team of workgroups switching its own 32-gate
 * tiles right after their last CMux step; on = 0 as two separate kernels
 * after the launch (the only form after stream-ordered rotations).  Results
 * are identical either way.  Errors: MK_EINVAL. */
int mk_set_ks_fusion(mk_ctx *ctx, int on);

/* Team size of the persistent rotation at N = 1024: each 32-gate tile is
 * run by 2 * 32 / rows workgroups, each contracting `rows` 32-row tiles per
 * task.  rows = 0 (default) picks by batch width: 2 (teams of 32, a whole
 * XCD per tile) when no XCD has more than one tile, 4 (teams of 16) at two
 * tiles per XCD, 8 (teams of 8, the most MFMAs per key tile loaded) from
 * three on.  rows = 2, 4 or 8 forces that size (tuning and tests).  Every
 * size gives the same words.  mk_get_team_rows reports the size a rotation
 * of `count` gates runs with (also at other N, where it is fixed), or 0 when
 * it runs on the stream-ordered kernels (always before mk_upload_eval_key,
 * which finds the XCDs).
 * Errors: MK_EINVAL (other values, or rows != 0 at N != 1024). */
int mk_set_team_rows(mk_ctx *ctx, int rows);
int mk_get_team_rows(const mk_ctx *ctx, size_t count, int32_t *rows);

/* Waits for `stream`, then reports and clears the context's device status
 * word, which device entry points set when they meet a condition they can
 * only detect on the GPU: MK_OK; MK_EINVAL if mk_bootstrap_gate met a gate
 * type outside NAND..XNOR since the last call; MK_EDEVICE if a persistent
 * rotation gave up waiting for another workgroup (its outputs are then
 * invalid) or ran on an XCD the upload's probe did not see.  Errors:
 * MK_EINVAL (null context), MK_ESTATE (key not uploaded), MK_EDEVICE. */
int mk_device_status(mk_ctx *ctx, void *stream);

/* Thread-local description of the last error on this thread. */
const char *mk_last_error(void);

/* Releases the context, its host keys and device memory. */
void mk_free(mk_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* MK_TFHE_H */
