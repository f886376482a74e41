// Host side of the library: parameter validation, the Philox4x64-10 streams
// and sampler, §3.2 Setup/KeyGen/SymEnc/SymDec, key serialisation.
//
// Randomness: Philox4x64-10 (Salmon et al., SC'11) keyed by
// (seed, party << 32 | object) with counter (block, index, 0, 0); u32 draw j
// of a stream is the low (j even) or high (j odd) half of 64-bit word j/2.
// Noise with standard deviation 2^-s is floor((sum of 12 draws - 6*2^32 +
// 2^(s-1)) / 2^s): an integer Irwin-Hall(12) sample.
#include <cstring>
#include <new>
#include <thread>

#include "mk_internal.h"

namespace mk {

static thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

namespace {

enum : uint32_t {
    OBJ_CRS = 1, OBJ_SK_LWE = 2, OBJ_SK_RLWE = 3, OBJ_PK_E = 4, OBJ_BK_R = 5,
    OBJ_BK_E1 = 6, OBJ_BK_F1 = 7, OBJ_BK_E2 = 8, OBJ_KS_A = 9, OBJ_KS_E = 10,
    OBJ_ENC_A = 11, OBJ_ENC_E = 12
};
constexpr uint32_t kPublicParty = 0xFFFF;

// One Philox4x64 block: ten rounds with the key bumped between rounds.
inline void philox_block(uint64_t c0, uint64_t c1, uint64_t k0, uint64_t k1,
                         uint64_t out[4]) {
    uint64_t x0 = c0, x1 = c1, x2 = 0, x3 = 0;
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B97F4A7C15ULL;
            k1 += 0xBB67AE8584CAA73BULL;
        }
        const unsigned __int128 p0 = (unsigned __int128)0xD2E7470EE14C6C93ULL * x0;
        const unsigned __int128 p1 = (unsigned __int128)0xCA5A826395121157ULL * x2;
        const uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        const uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        const uint64_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
        x0 = y0; x1 = lo1; x2 = y2; x3 = lo0;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

// Sequential reader of one u32 stream.
class Stream {
  public:
    Stream(uint64_t seed, uint32_t party, uint32_t obj, uint64_t idx)
        : k0_(seed), k1_(((uint64_t)party << 32) | obj), idx_(idx) {}
    uint32_t next() {
        if (pos_ == 8) {
            uint64_t w[4];
            philox_block(block_++, idx_, k0_, k1_, w);
            for (int i = 0; i < 4; ++i) {
                buf_[2 * i] = (uint32_t)w[i];
                buf_[2 * i + 1] = (uint32_t)(w[i] >> 32);
            }
            pos_ = 0;
        }
        return buf_[pos_++];
    }
    uint32_t noise(int s) {
        int64_t acc = 0;
        for (int i = 0; i < 12; ++i) acc += next();
        acc -= 6LL * (1LL << 32);
        acc += 1LL << (s - 1);
        return (uint32_t)(acc >> s);  // arithmetic shift = floor division
    }

  private:
    uint64_t k0_, k1_, idx_;
    uint64_t block_ = 0;
    uint32_t buf_[8];
    int pos_ = 8;
};

// out += sign * bin * K in Z[X]/(X^N+1), bin a 0/1 polynomial.
void add_binary_times(uint32_t *out, const uint8_t *bin, const uint32_t *K, int N,
                      bool negate) {
    for (int p = 0; p < N; ++p) {
        if (!bin[p]) continue;
        // X^p * K: coefficient m gets K[m-p] for m >= p, -K[N+m-p] for m < p.
        if (!negate) {
            for (int m = p; m < N; ++m) out[m] += K[m - p];
            for (int m = 0; m < p; ++m) out[m] -= K[N + m - p];
        } else {
            for (int m = p; m < N; ++m) out[m] -= K[m - p];
            for (int m = 0; m < p; ++m) out[m] += K[N + m - p];
        }
    }
}

template <class F>
void parallel_for(size_t count, F &&f) {
    unsigned nt = std::thread::hardware_concurrency();
    if (nt == 0) nt = 1;
    if (nt > 16) nt = 16;
    if (count < 2 * nt) nt = 1;
    if (nt == 1) {
        for (size_t i = 0; i < count; ++i) f(i);
        return;
    }
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t)
        th.emplace_back([&, t] {
            for (size_t i = t; i < count; i += nt) f(i);
        });
    for (auto &x : th) x.join();
}

int check_params(const mk_params &p) {
    if (p.k < 1 || p.k > 8) return fail(MK_EPARAM, "k must be in [1, 8]");
    if (p.n < 1 || p.n > 1023) return fail(MK_EPARAM, "n must be in [1, 1023]");
    if (p.N < 16 || p.N > 4096 || (p.N & (p.N - 1)))
        return fail(MK_EPARAM, "N must be a power of two in [16, 4096]");
    if (p.bk_log_base != 8) return fail(MK_EPARAM, "bk_log_base must be 8 (int8 digits)");
    if (p.bk_ell < 1 || p.bk_ell * p.bk_log_base > 30)
        return fail(MK_EPARAM, "bk_ell * bk_log_base must be in [8, 30]");
    if (p.ks_log_base < 1 || p.ks_log_base > 4)
        return fail(MK_EPARAM, "ks_log_base must be in [1, 4]");
    if (p.ks_t < 1 || p.ks_t * p.ks_log_base > 30)
        return fail(MK_EPARAM, "ks_t * ks_log_base must be in [1, 30]");
    for (int s : {p.bk_noise_log2, p.ks_noise_log2, p.lwe_noise_log2})
        if (s < 1 || s > 40) return fail(MK_EPARAM, "noise log2 must be in [1, 40]");
    // exactness of the int8 contraction: |sum| <= (k+1)*ell*N*2^14 < 2^31
    const double bound = (double)(p.k + 1) * p.bk_ell * p.N * 16384.0;
    if (bound >= 2147483648.0)
        return fail(MK_EPARAM, "(k+1)*ell*N*2^14 must be < 2^31");
    return MK_OK;
}

void gen_party(const mk_params &P, const std::vector<uint32_t> &crs, int party,
               uint64_t seed, HostPartyKeys &K) {
    const int n = P.n, N = P.N, ell = P.bk_ell, t = P.ks_t;
    const int Bm1 = ks_base(P) - 1;
    K.s.resize(n);
    K.z.resize(N);
    {
        Stream st(seed, party, OBJ_SK_LWE, 0);
        for (int i = 0; i < n; ++i) K.s[i] = st.next() & 1;
        Stream sz(seed, party, OBJ_SK_RLWE, 0);
        for (int i = 0; i < N; ++i) K.z[i] = sz.next() & 1;
    }
    // public key: b_l = -z * a_l + e_l
    K.pk.assign((size_t)ell * N, 0);
    for (int l = 0; l < ell; ++l) {
        uint32_t *b = &K.pk[(size_t)l * N];
        Stream se(seed, party, OBJ_PK_E, l);
        for (int m = 0; m < N; ++m) b[m] = se.noise(P.bk_noise_log2);
        add_binary_times(b, K.z.data(), &crs[(size_t)l * N], N, true);
    }
    // bootstrapping key: uni-encryption (d, f0, f1) of each bit of s under z
    K.bk.assign((size_t)n * 3 * ell * N, 0);
    parallel_for((size_t)n, [&](size_t j) {
        std::vector<uint8_t> r(N);
        Stream sr(seed, party, OBJ_BK_R, j);
        for (int m = 0; m < N; ++m) r[m] = sr.next() & 1;
        for (int l = 0; l < ell; ++l) {
            const uint32_t g = 1u << (32 - P.bk_log_base * (l + 1));
            const uint64_t idx = (uint64_t)j * ell + l;
            uint32_t *d = &K.bk[(((size_t)j * 3 + 0) * ell + l) * N];
            uint32_t *f0 = &K.bk[(((size_t)j * 3 + 1) * ell + l) * N];
            uint32_t *f1 = &K.bk[(((size_t)j * 3 + 2) * ell + l) * N];
            Stream s1(seed, party, OBJ_BK_E1, idx);
            for (int m = 0; m < N; ++m) d[m] = s1.noise(P.bk_noise_log2);
            add_binary_times(d, r.data(), &crs[(size_t)l * N], N, false);
            d[0] += (uint32_t)K.s[j] * g;
            Stream sf(seed, party, OBJ_BK_F1, idx);
            for (int m = 0; m < N; ++m) f1[m] = sf.next();
            Stream s2(seed, party, OBJ_BK_E2, idx);
            for (int m = 0; m < N; ++m) f0[m] = s2.noise(P.bk_noise_log2) + (uint32_t)r[m] * g;
            add_binary_times(f0, K.z.data(), f1, N, true);
        }
    });
    // key-switching key: KS[q][p][v] = LWE_s(v * z_q * 2^(32 - lb*(p+1)))
    const size_t rows = ks_rows(P);
    K.ks.assign(rows * (n + 1), 0);
    parallel_for(rows, [&](size_t row) {
        const int q = (int)(row / ((size_t)t * Bm1));
        const int p = (int)((row / Bm1) % t);
        const uint32_t v = (uint32_t)(row % Bm1) + 1;
        uint32_t *dst = &K.ks[row * (n + 1)];
        Stream sa(seed, party, OBJ_KS_A, row);
        uint32_t dot = 0;
        for (int i = 0; i < n; ++i) {
            dst[1 + i] = sa.next();
            dot += dst[1 + i] * (uint32_t)K.s[i];
        }
        Stream se(seed, party, OBJ_KS_E, row);
        const uint32_t msg = v * (uint32_t)K.z[q] * (uint32_t)(1ULL << (32 - P.ks_log_base * (p + 1)));
        dst[0] = msg - dot + se.noise(P.ks_noise_log2);
    });
    K.present = true;
}

// --- serialisation ---
constexpr uint32_t kMagic = 0x314B4B4Du;  // "MKK1"

size_t export_size(const mk_params &P, int party) {
    size_t hdr = 4 + 4 + 10 * 4 + 4;
    if (party < 0) return hdr + (size_t)P.bk_ell * P.N * 4;
    return hdr + (size_t)P.n + P.N + (size_t)P.bk_ell * P.N * 4 +
           (size_t)P.n * 3 * P.bk_ell * P.N * 4 + ks_rows(P) * (P.n + 1) * 4;
}

void put(uint8_t *&dst, const void *src, size_t bytes) {
    std::memcpy(dst, src, bytes);
    dst += bytes;
}
void get(const uint8_t *&src, void *dst, size_t bytes) {
    std::memcpy(dst, src, bytes);
    src += bytes;
}

}  // namespace
}  // namespace mk

using namespace mk;

extern "C" {

const char *mk_last_error(void) { return g_err.c_str(); }

int mk_setup(const mk_params *p, uint64_t seed, mk_ctx **out) {
    if (!p || !out) return fail(MK_EINVAL, "mk_setup: null argument");
    *out = nullptr;
    int rc = check_params(*p);
    if (rc) return rc;
    mk_ctx *ctx = new (std::nothrow) mk_ctx();
    if (!ctx) return fail(MK_ENOMEM, "mk_setup: out of host memory");
    ctx->p = *p;
    ctx->crs_seed = seed;
    ctx->crs.resize((size_t)p->bk_ell * p->N);
    for (int l = 0; l < p->bk_ell; ++l) {
        Stream st(seed, kPublicParty, OBJ_CRS, l);
        for (int m = 0; m < p->N; ++m) ctx->crs[(size_t)l * p->N + m] = st.next();
    }
    ctx->parties.resize(p->k);
    *out = ctx;
    return MK_OK;
}

int mk_keygen(mk_ctx *ctx, int party, uint64_t seed) {
    if (!ctx) return fail(MK_EINVAL, "mk_keygen: null context");
    if (party < 0 || party >= ctx->p.k) return fail(MK_EINVAL, "mk_keygen: party out of range");
    try {
        gen_party(ctx->p, ctx->crs, party, seed, ctx->parties[party]);
    } catch (const std::bad_alloc &) {
        return fail(MK_ENOMEM, "mk_keygen: out of host memory");
    }
    ctx->dev.uploaded = false;
    return MK_OK;
}

int mk_export_keys(const mk_ctx *ctx, int party, void *buf, size_t *len) {
    if (!ctx || !len) return fail(MK_EINVAL, "mk_export_keys: null argument");
    const mk_params &P = ctx->p;
    if (party < -1 || party >= P.k) return fail(MK_EINVAL, "mk_export_keys: party out of range");
    if (party >= 0 && !ctx->parties[party].present)
        return fail(MK_ESTATE, "mk_export_keys: party has no keys");
    const size_t need = export_size(P, party);
    if (!buf) {
        *len = need;
        return MK_OK;
    }
    if (*len < need) return fail(MK_EINVAL, "mk_export_keys: buffer too small");
    uint8_t *d = (uint8_t *)buf;
    const uint32_t magic = kMagic, version = 1;
    const int32_t pty = party;
    put(d, &magic, 4);
    put(d, &version, 4);
    put(d, &P, sizeof(mk_params));
    put(d, &pty, 4);
    if (party < 0) {
        put(d, ctx->crs.data(), ctx->crs.size() * 4);
    } else {
        const HostPartyKeys &K = ctx->parties[party];
        put(d, K.s.data(), K.s.size());
        put(d, K.z.data(), K.z.size());
        put(d, K.pk.data(), K.pk.size() * 4);
        put(d, K.bk.data(), K.bk.size() * 4);
        put(d, K.ks.data(), K.ks.size() * 4);
    }
    *len = need;
    return MK_OK;
}

int mk_import_keys(mk_ctx *ctx, int party, const void *buf, size_t len) {
    if (!ctx || !buf) return fail(MK_EINVAL, "mk_import_keys: null argument");
    const mk_params &P = ctx->p;
    if (party < -1 || party >= P.k) return fail(MK_EINVAL, "mk_import_keys: party out of range");
    if (len != export_size(P, party)) return fail(MK_EINVAL, "mk_import_keys: size mismatch");
    const uint8_t *s = (const uint8_t *)buf;
    uint32_t magic, version;
    mk_params q;
    int32_t pty;
    get(s, &magic, 4);
    get(s, &version, 4);
    get(s, &q, sizeof(mk_params));
    get(s, &pty, 4);
    if (magic != kMagic || version != 1) return fail(MK_EINVAL, "mk_import_keys: bad magic");
    if (std::memcmp(&q, &P, sizeof(mk_params)) != 0 || pty != party)
        return fail(MK_EINVAL, "mk_import_keys: parameter or party mismatch");
    try {
        if (party < 0) {
            get(s, ctx->crs.data(), ctx->crs.size() * 4);
        } else {
            HostPartyKeys &K = ctx->parties[party];
            K.s.resize(P.n);
            K.z.resize(P.N);
            K.pk.resize((size_t)P.bk_ell * P.N);
            K.bk.resize((size_t)P.n * 3 * P.bk_ell * P.N);
            K.ks.resize(ks_rows(P) * (P.n + 1));
            get(s, K.s.data(), K.s.size());
            get(s, K.z.data(), K.z.size());
            get(s, K.pk.data(), K.pk.size() * 4);
            get(s, K.bk.data(), K.bk.size() * 4);
            get(s, K.ks.data(), K.ks.size() * 4);
            K.present = true;
        }
    } catch (const std::bad_alloc &) {
        return fail(MK_ENOMEM, "mk_import_keys: out of host memory");
    }
    ctx->dev.uploaded = false;
    return MK_OK;
}

int mk_encrypt(const mk_ctx *ctx, int party, const uint8_t *bits, size_t count,
               uint64_t seed, uint32_t *out_host, size_t stride_words) {
    if (!ctx || (count && (!bits || !out_host))) return fail(MK_EINVAL, "mk_encrypt: null argument");
    const mk_params &P = ctx->p;
    if (party < 0 || party >= P.k) return fail(MK_EINVAL, "mk_encrypt: party out of range");
    if (stride_words < lwe_words(P)) return fail(MK_EINVAL, "mk_encrypt: stride < kn+1");
    const HostPartyKeys &K = ctx->parties[party];
    if (!K.present) return fail(MK_ESTATE, "mk_encrypt: party has no keys");
    parallel_for(count, [&](size_t j) {
        uint32_t *row = out_host + j * stride_words;
        std::memset(row, 0, lwe_words(P) * 4);
        uint32_t *a = row + 1 + (size_t)party * P.n;
        Stream sa(seed, party, OBJ_ENC_A, j);
        uint32_t dot = 0;
        for (int i = 0; i < P.n; ++i) {
            a[i] = sa.next();
            dot += a[i] * (uint32_t)K.s[i];
        }
        Stream se(seed, party, OBJ_ENC_E, j);
        row[0] = (uint32_t)(bits[j] & 1) * 0x40000000u - dot + se.noise(P.lwe_noise_log2);
    });
    return MK_OK;
}

int mk_decrypt(const mk_ctx *ctx, const uint32_t *ct_host, size_t count,
               size_t stride_words, uint8_t *bits) {
    if (!ctx || (count && (!ct_host || !bits))) return fail(MK_EINVAL, "mk_decrypt: null argument");
    const mk_params &P = ctx->p;
    if (stride_words < lwe_words(P)) return fail(MK_EINVAL, "mk_decrypt: stride < kn+1");
    for (int i = 0; i < P.k; ++i)
        if (!ctx->parties[i].present) return fail(MK_ESTATE, "mk_decrypt: a party has no keys");
    for (size_t j = 0; j < count; ++j) {
        const uint32_t *row = ct_host + j * stride_words;
        uint32_t ph = row[0];
        for (int i = 0; i < P.k; ++i) {
            const uint32_t *a = row + 1 + (size_t)i * P.n;
            const uint8_t *s = ctx->parties[i].s.data();
            for (int q = 0; q < P.n; ++q) ph += a[q] * (uint32_t)s[q];
        }
        bits[j] = (ph >= 0x20000000u && ph < 0xA0000000u) ? 1 : 0;
    }
    return MK_OK;
}

int mk_trivial(const mk_ctx *ctx, const uint8_t *bits, size_t count, uint32_t *out_host,
               size_t stride_words) {
    if (!ctx || (count && (!bits || !out_host))) return fail(MK_EINVAL, "mk_trivial: null argument");
    if (stride_words < lwe_words(ctx->p)) return fail(MK_EINVAL, "mk_trivial: stride < kn+1");
    for (size_t j = 0; j < count; ++j) {
        uint32_t *row = out_host + j * stride_words;
        std::memset(row, 0, lwe_words(ctx->p) * 4);
        row[0] = (uint32_t)(bits[j] & 1) * 0x40000000u;
    }
    return MK_OK;
}

void mk_free(mk_ctx *ctx) {
    if (!ctx) return;
    device_release(ctx);
    delete ctx;
}

}  // extern "C"
