// Internal declarations shared by the host and device translation units of
// the library.  Not part of the C ABI.
#pragma once

#include <cstddef>
#include <cstdint>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "mk_tfhe.h"

namespace mk {

// Sets the thread-local error message and returns `code`.
int fail(int code, const std::string &msg);

struct HostPartyKeys {
    bool present = false;
    std::vector<uint8_t> s;      // [n]
    std::vector<uint8_t> z;      // [N]
    std::vector<uint32_t> pk;    // [ell][N]
    std::vector<uint32_t> bk;    // [n][3][ell][N]
    std::vector<uint32_t> ks;    // [N][t][B'-1][n+1]
};

// Device copies of the evaluation key, built by mk_upload_eval_key.
struct DeviceKeys {
    bool uploaded = false;
    int device = -1;
    // Plain path: every key polynomial K stored in extended form [-K | K]
    // (2N words) so that the negacyclic Toeplitz entry T[m][p] = K'[m-p] is
    // the word at index N + m - p.
    uint32_t *bk_ext = nullptr;   // [k][n][3][ell][2N]
    uint32_t *evk_ext = nullptr;  // [k+1][ell][2N]
    // Int8-MFMA path: limb-planar windows (see mk_device.hip).
    int8_t *bk_win = nullptr;
    int8_t *evk_win = nullptr;
    size_t bk_win_bytes = 0, evk_win_bytes = 0;
    uint32_t *ks = nullptr;       // [k][N][t][B'-1][n+1]
    int8_t *ks_win = nullptr;     // MFMA key-switching tiles (mk_keyswitch.hip)
    size_t ks_win_bytes = 0;
    // Profiling: event pairs per stage, accumulated on mk_get_profile.
    int profiling = 0;
    std::vector<std::pair<void *, void *>> events[MK_PROFILE_SLOTS];
    double prof_ms[MK_PROFILE_SLOTS] = {};
    int64_t prof_launches[MK_PROFILE_SLOTS] = {};
    // Scratch for the gate pipeline and for the MFMA rotation, grown on demand.
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    void *mfma_scratch = nullptr;
    size_t mfma_scratch_bytes = 0;
    void *ks_scratch = nullptr;     // rounded coefficients of the MFMA key switch
    size_t ks_scratch_bytes = 0;
    // Set while the scratch pointers above point into a caller-fixed block
    // (the allocation-free entry point): nothing is grown or split then.
    bool fixed_scratch = false;
    void *circ_scratch = nullptr;   // circuit wire buffer and descriptors
    size_t circ_scratch_bytes = 0;
    // GEMM tile shapes of the MFMA rotation: autotuned per batch size (in
    // 32-gate tiles) and optionally forced (-1 = not forced).
    std::map<int, std::pair<int, int>> tuned_tiles;
    int force_tiles[2] = {-1, -1};
    // Sub-batches of the MFMA rotation (1 or 2, run on aux streams), tuned
    // per batch size in 32-gate tiles; streams and events made on first use.
    std::map<int, int> tuned_parts;
    // Graph capture in progress (mk_circuit_graph_create): the capture is cut
    // into consecutive graphs of at most about kGraphSteps CMux steps.
    void *capture = nullptr;
    int graph_piece = 1024;   // kernels per captured piece (mk_set_graph_piece)
    void *aux_stream[2] = {nullptr, nullptr};
    void *aux_event[3] = {nullptr, nullptr, nullptr};
    // Persistent rotation (mk_persist.hip): compute units, the XCDs found
    // by the upload's probe (XCC_ID -> dense index), a sticky device status
    // word, and the schedule choice (-1 automatic, 0 stream-ordered kernels,
    // 1 persistent).
    int num_cus = 0, num_xcd = 0;
    int8_t xmap[16] = {};
    uint32_t *status = nullptr;
    int rot_kind = -1;
    // Extraction and key switching inside the persistent rotation's launch
    // (mk_set_ks_fusion): 1 on, 0 separate kernels.
    int ks_fuse = 1;
    // Row tiles per contraction task of the persistent rotation at N = 1024
    // (mk_set_team_rows): 0 chosen by batch width, else 2, 4 or 8.
    int team_rows = 0;
};

}  // namespace mk

struct mk_ctx {
    mk_params p{};
    uint64_t crs_seed = 0;
    std::vector<uint32_t> crs;   // [ell][N]
    std::vector<mk::HostPartyKeys> parties;
    mk::DeviceKeys dev;
};

namespace mk {

inline size_t lwe_words(const mk_params &p) { return (size_t)p.k * p.n + 1; }
inline int ks_base(const mk_params &p) { return 1 << p.ks_log_base; }
inline size_t ks_rows(const mk_params &p) {
    return (size_t)p.N * p.ks_t * (ks_base(p) - 1);
}

// Device side (mk_device.hip).
int device_upload(mk_ctx *ctx, void *stream);
void device_release(mk_ctx *ctx);

}  // namespace mk
