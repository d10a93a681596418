// Host core of the FDFB library: parameter checks, seeded key generation,
// rotation polynomials, device key layouts, scratch pool and the stream-
// ordered orchestration of the bootstrap (Sec. 3.2, Fig. 2 "Bootstrap").
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <memory>
#include <mutex>
#include <numeric>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "fdfb.h"
#include "internal.h"
#include "kernels.h"
#include "pipeline_plan.h"

namespace fdfbi {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

}  // namespace fdfbi

using fdfbi::fail;
using fdfbi::g_last_error;

namespace {

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t _e = (expr);                                                                \
        if (_e != hipSuccess)                                                                  \
            return fail(FDFB_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e));      \
    } while (0)

// --------------------------------------------------------------------------
// Counter-based SplitMix64 (Steele, Lea & Flood, OOPSLA 2014; finaliser of
// Vigna's reference splitmix64.c).  Stream `tag` of seed `seed` starts at
// state fin(seed + tag * gamma); its k-th output is fin(state + (k+1) gamma).
// --------------------------------------------------------------------------
class CounterRng {
  public:
    static constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
    CounterRng(uint64_t seed, uint64_t tag) : state0_(fin(seed + tag * kGamma)) {}
    uint64_t word(uint64_t k) const { return fin(state0_ + (k + 1) * kGamma); }
    uint32_t uniform32(uint64_t k) const { return static_cast<uint32_t>(word(k) >> 32); }
    uint32_t bit(uint64_t k) const { return static_cast<uint32_t>(word(k) >> 63); }
    // Rounded N(0, sigma^2): Box-Muller on outputs 2k and 2k+1.
    int64_t gaussian(uint64_t k, double sigma) const
    {
        if (sigma == 0.0) return 0;
        const double u1 = static_cast<double>((word(2 * k) >> 11) + 1) * (1.0 / 9007199254740992.0);
        const double u2 = static_cast<double>(word(2 * k + 1) >> 11) * (1.0 / 9007199254740992.0);
        const double z = std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
        return static_cast<int64_t>(std::nearbyint(z * sigma));
    }

  private:
    static uint64_t fin(uint64_t z)
    {
        z ^= z >> 30;
        z *= 0xBF58476D1CE4E5B9ull;
        z ^= z >> 27;
        z *= 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    uint64_t state0_;
};

enum StreamTag : uint64_t {
    kTagS = 1, kTagSF = 2, kTagBrkA = 3, kTagBrkE = 4, kTagPkA = 5, kTagPkE = 6,
    kTagKsA = 7, kTagKsE = 8, kTagEncA = 9, kTagEncE = 10
};

inline uint32_t gadget_word(uint32_t log2B, uint32_t ell, uint32_t j)
{
    return 1u << (32 - ell * log2B + log2B * j);
}

unsigned worker_count()
{
    unsigned h = std::thread::hardware_concurrency();
    return std::max(1u, std::min(h ? h : 1u, 16u));
}

template <class F>
void parallel_for(size_t count, F &&f)
{
    const unsigned nt = worker_count();
    if (count < 2 || nt == 1) {
        for (size_t k = 0; k < count; ++k) f(k);
        return;
    }
    std::atomic<size_t> next{0};
    std::vector<std::thread> pool;
    for (unsigned w = 0; w < nt; ++w)
        pool.emplace_back([&] {
            for (size_t k; (k = next.fetch_add(1)) < count;) f(k);
        });
    for (auto &th : pool) th.join();
}

// b <- a * sf + noise with binary sf: a sum of negacyclic rotations of a.
void times_binary_key(const uint32_t *a, const std::vector<uint32_t> &sf, uint32_t N, uint32_t *b)
{
    for (uint32_t p = 0; p < N; ++p) {
        if (!sf[p]) continue;
        for (uint32_t m = 0; m < p; ++m) b[m] -= a[m + N - p];
        for (uint32_t m = p; m < N; ++m) b[m] += a[m - p];
    }
}

// Balanced signed byte limbs of a 32-bit word: w = sum_l limb_l 256^l mod 2^32.
inline void balanced_limbs(uint32_t w, int8_t out[4])
{
    int64_t v = w;
    for (int l = 0; l < 4; ++l) {
        const int64_t lo = ((v & 0xFF) ^ 0x80) - 0x80;
        out[l] = static_cast<int8_t>(lo);
        v = (v - lo) >> 8;
    }
}

}  // namespace

namespace {

bool is_pow2(uint32_t x) { return x && !(x & (x - 1)); }

fdfbk::Geometry geometry_of(const fdfb_params &P);

// The plain blind rotation keeps the accumulator, the key of one CMux and the
// digits in LDS.
bool plain_br_fits(const fdfb_params &P)
{
    const size_t R = 2 * P.g_ell;
    return 8ull * P.N + 8ull * R * P.N + 4ull * R * P.N <= 160 * 1024;
}

int check_params(const fdfb_params &P)
{
    if (!is_pow2(P.N) || P.N < 64 || P.N > 2048) return fail(FDFB_EINVAL, "N must be a power of two in [64, 2048]");
    if (P.n < 1 || P.n > 4096) return fail(FDFB_EINVAL, "n must be in [1, 4096]");
    if (P.log2_t < 1 || (1u << P.log2_t) > P.N) return fail(FDFB_EINVAL, "t must be a power of two with 2 <= t <= N");
    struct G { uint32_t b, l; const char *name; } gs[] = {
        {P.g_log2B, P.g_ell, "gadget"}, {P.ks_log2B, P.ks_ell, "key switch"},
        {P.pk_log2B, P.pk_ell, "packing key"}};
    for (auto &g : gs)
        if (g.b < 1 || g.l < 1 || g.b * g.l > 32)
            return fail(FDFB_EINVAL, std::string(g.name) + ": need 1 <= ell, 1 <= log2B, ell*log2B <= 32");
    if (P.g_log2B > 14) return fail(FDFB_EINVAL, "gadget base above 2^14 is not supported");
    if (P.ks_ell > 8 || P.pk_ell > 8) return fail(FDFB_EINVAL, "key switching ell above 8 is not supported");
    if (P.ks_log2B > 16 || P.pk_log2B > 16) return fail(FDFB_EINVAL, "key switching base above 2^16 is not supported");
    if (P.boot_log2B == 0) {  // one signed digit in [-t/2, t/2)
        if (P.boot_ell != 1 || P.log2_t > 7)
            return fail(FDFB_EINVAL, "a signed boot digit needs boot_ell = 1 and t <= 128");
    } else if (P.boot_log2B > 7 || P.boot_ell < 1 || P.boot_ell * P.boot_log2B < P.log2_t) {
        return fail(FDFB_EINVAL, "boot digits must cover t: boot_ell * boot_log2B >= log2_t, log2B in [1,7]");
    }
    if (!(P.sigma_lwe >= 0) || !(P.sigma_glwe >= 0) || !(P.sigma_pk >= 0) || !(P.sigma_ks >= 0))
        return fail(FDFB_EINVAL, "noise deviations must be non-negative");
    if (!plain_br_fits(P) && !fdfbk::br_mfma_supported(geometry_of(P)))
        return fail(FDFB_EINVAL, "no blind-rotation kernel for this ring degree and gadget");
    return FDFB_OK;
}

fdfbk::Geometry geometry_of(const fdfb_params &P)
{
    fdfbk::Geometry G{};
    G.n = P.n; G.N = P.N; G.log2_t = P.log2_t;
    G.g_log2B = P.g_log2B; G.g_ell = P.g_ell; G.g_chunks = fdfbk::digit_chunks(P.g_log2B);
    G.ks_log2B = P.ks_log2B; G.ks_ell = P.ks_ell;
    G.pk_log2B = P.pk_log2B; G.pk_ell = P.pk_ell;
    G.boot_log2B = P.boot_log2B; G.boot_ell = P.boot_ell;
    return G;
}

// Keys of Theorem "Correctness of the Bootstrapping" (Sec. 3.2):
//   brK[i] = RGSW(𝔰, s[i]); pK[i][j] = RLWE(𝔰, s_F[i] g_j); ksK[i][j] = LWE(s, s_F[i] g_j).
void generate_keys(fdfb_ctx &c)
{
    const fdfb_params &P = c.P;
    const uint32_t n = P.n, N = P.N, R = 2 * P.g_ell;
    const uint64_t seed = c.seed;
    c.s.resize(n);
    c.sf.resize(N);
    const CounterRng rs(seed, kTagS), rsf(seed, kTagSF);
    for (uint32_t i = 0; i < n; ++i) c.s[i] = rs.bit(i);
    for (uint32_t p = 0; p < N; ++p) c.sf[p] = rsf.bit(p);

    c.brk.assign((size_t)n * R * 2 * N, 0);
    const CounterRng ra(seed, kTagBrkA), re(seed, kTagBrkE);
    parallel_for((size_t)n * R, [&](size_t row_id) {
        const uint32_t i = row_id / R, r = row_id % R;
        uint32_t *b = &c.brk[row_id * 2 * N], *a = b + N;
        for (uint32_t p = 0; p < N; ++p) {
            a[p] = ra.uniform32(row_id * N + p);
            b[p] = static_cast<uint32_t>(re.gaussian(row_id * N + p, P.sigma_glwe));
        }
        times_binary_key(a, c.sf, N, b);
        const uint32_t comp = r / P.g_ell, j = r % P.g_ell;
        (comp == 0 ? b : a)[0] += c.s[i] * gadget_word(P.g_log2B, P.g_ell, j);
    });

    c.pk.assign((size_t)N * P.pk_ell * 2 * N, 0);
    const CounterRng pa(seed, kTagPkA), pe(seed, kTagPkE);
    parallel_for((size_t)N * P.pk_ell, [&](size_t row_id) {
        const uint32_t i = row_id / P.pk_ell, j = row_id % P.pk_ell;
        uint32_t *b = &c.pk[row_id * 2 * N], *a = b + N;
        for (uint32_t p = 0; p < N; ++p) {
            a[p] = pa.uniform32(row_id * N + p);
            b[p] = static_cast<uint32_t>(pe.gaussian(row_id * N + p, P.sigma_pk));
        }
        times_binary_key(a, c.sf, N, b);
        b[0] += c.sf[i] * gadget_word(P.pk_log2B, P.pk_ell, j);
    });

    c.ksk.assign((size_t)N * P.ks_ell * (n + 1), 0);
    const CounterRng ka(seed, kTagKsA), ke(seed, kTagKsE);
    parallel_for((size_t)N * P.ks_ell, [&](size_t row_id) {
        const uint32_t i = row_id / P.ks_ell, j = row_id % P.ks_ell;
        uint32_t *row = &c.ksk[row_id * (n + 1)];
        uint32_t acc = 0;
        for (uint32_t q = 0; q < n; ++q) {
            row[1 + q] = ka.uniform32(row_id * n + q);
            acc += row[1 + q] * c.s[q];
        }
        row[0] = acc + static_cast<uint32_t>(ke.gaussian(row_id, P.sigma_ks)) +
                 c.sf[i] * gadget_word(P.ks_log2B, P.ks_ell, j);
    });
}

// Rotation polynomials (Sec. 3.3, Theorem "rotation polynomial"): for every
// rotation y in [0, 2N), coefficient 0 of rotP_0 X^y (y < N) or rotP_1 X^y
// (y >= N) is f(m) for the m that owns y.  The windows are the y within
// N/t (cyclically) of the centres 2N m / t; with t | N they are exactly
// half a centre spacing wide and meet at the midpoints, which the larger m
// owns (the later write of the construction in Fig. 2).
void setup_polynomial(const uint32_t *f, uint32_t t, uint32_t N, int32_t *p0, int32_t *p1)
{
    std::fill(p0, p0 + N, 0);
    std::fill(p1, p1 + N, 0);
    const uint32_t spacing = 2 * N / t, half = N / t;  // t is a power of two dividing N
    for (uint32_t y = 0; y < 2 * N; ++y) {
        const uint32_t below = y / spacing, r = y % spacing;  // the centre at or below y, and y's offset
        uint32_t m;
        if (r < half) m = below;
        else if (r > half) m = (below + 1) % t;      // the centre above (m = 0 again past 2N)
        else m = below + 1 < t ? below + 1 : below;  // a midpoint: the larger m
        const int32_t v = static_cast<int32_t>(f[m]);
        // coefficient 0 of X^y p reads p_0 (y = 0) or -p_{N-y}; X^y = -X^{y-N} for y >= N
        if (y < N) (y == 0 ? p0[0] : p0[N - y]) = y == 0 ? v : -v;
        else (y == N ? p1[0] : p1[2 * N - y]) = y == N ? -v : v;
    }
}

// Key operand of the MFMA blind rotation, as byte planes: block (i, r', j)
// holds 4 planes of N + 64 bytes, plane l = limb l of K'~[x] for x < N + 64,
// where K' is the key polynomial of virtual row r' for output component j,
// times 2^(7h) for digit chunk h, and K'~ its negacyclic extension.  Lane
// (s, l, g) of k-block kb reads bytes 64 kb + 16 (g + s) .. +15 of plane l.
std::vector<int8_t> build_brk_fragments(const fdfb_ctx &c)
{
    const fdfb_params &P = c.P;
    const uint32_t N = P.N, ell = P.g_ell, CH = fdfbk::digit_chunks(P.g_log2B);
    const uint32_t RPC = ell * CH, RV = 2 * RPC, R = 2 * ell, PL = N + 64;
    std::vector<int8_t> out((size_t)P.n * RV * 2 * 4 * PL);
    parallel_for((size_t)P.n * RV, [&](size_t id) {
        const uint32_t i = id / RV, rv = id % RV;
        const uint32_t comp_in = rv / RPC, rr = rv % RPC, jd = rr / CH, h = rr % CH;
        const uint32_t row = comp_in * ell + jd;
        for (uint32_t j = 0; j < 2; ++j) {
            const uint32_t *K = &c.brk[(((size_t)i * R + row) * 2 + j) * N];
            int8_t *dst = &out[(id * 2 + j) * 4 * PL];
            for (uint32_t x = 0; x < PL; ++x) {
                uint32_t w = (x < N) ? K[x] : 0u - K[x - N];  // PL <= 2N
                w <<= 7 * h;
                int8_t limbs[4];
                balanced_limbs(w, limbs);
                for (uint32_t l = 0; l < 4; ++l) dst[l * PL + x] = limbs[l];
            }
        }
    });
    return out;
}

// Lane-ordered B fragments of the MFMA key switch: block (kb, tile) holds,
// for lane L and byte t, limb L % 4 of key word K[i][j][4 tile + L/4 % 4]
// with j * din + i = 64 kb + 16 (L / 16) + t; words past out_len are zero.
std::vector<int8_t> build_ks_fragments(const uint32_t *key, uint32_t din, uint32_t ell, uint32_t out_len)
{
    const uint32_t nkb = din * ell / 64, wtiles = (out_len + 63) / 64 * 16;
    std::vector<int8_t> out((size_t)nkb * wtiles * 1024);
    parallel_for((size_t)nkb * wtiles, [&](size_t id) {
        const uint32_t kb = id / wtiles, tile = id % wtiles;
        for (uint32_t L = 0; L < 64; ++L) {
            const uint32_t col = L & 15, w = 4 * tile + (col >> 2), l = col & 3;
            int8_t *dst = &out[(id * 64 + L) * 16];
            for (uint32_t t = 0; t < 16; ++t) {
                const uint32_t k = 64 * kb + 16 * (L >> 4) + t, j = k / din, i = k % din;
                int8_t limbs[4] = {0, 0, 0, 0};
                if (w < out_len) balanced_limbs(key[((size_t)i * ell + j) * out_len + w], limbs);
                dst[t] = limbs[l];
            }
        }
    });
    return out;
}

// Key operand of the Karatsuba blind rotation, in the lane order of the MFMA
// B operand: block (i, r', p, j, kb) holds for lane L and byte t limb L % 4 of
// K'~[64 kb + 16 (L / 16) + (L / 4 % 4) + t], where K' is the half-ring key
// polynomial of product p (K_e[x] = K[2x], K_o[x] = K[2x+1], or K_e + K_o)
// times 2^(7h) for digit chunk h, and K'~ its negacyclic extension in
// Z[Y]/(Y^M + 1), M = N/2.
std::vector<int8_t> build_brk_kara(const fdfb_ctx &c)
{
    const fdfb_params &P = c.P;
    const uint32_t N = P.N, M = N / 2, ell = P.g_ell, CH = fdfbk::digit_chunks(P.g_log2B);
    const uint32_t RPC = ell * CH, RV = 2 * RPC, R = 2 * ell, NKB = M / 64;
    std::vector<int8_t> out((size_t)P.n * RV * 3 * 2 * NKB * 1024);
    parallel_for((size_t)P.n * RV, [&](size_t id) {
        const uint32_t i = id / RV, rv = id % RV;
        const uint32_t comp_in = rv / RPC, rr = rv % RPC, jd = rr / CH, h = rr % CH;
        const uint32_t row = comp_in * ell + jd;
        std::vector<uint32_t> ext(M + 64);
        for (uint32_t j = 0; j < 2; ++j) {
            const uint32_t *K = &c.brk[(((size_t)i * R + row) * 2 + j) * N];
            for (uint32_t p = 0; p < 3; ++p) {
                for (uint32_t x = 0; x < M + 64; ++x) {  // M + 64 <= 2M
                    const uint32_t xx = x < M ? x : x - M;
                    uint32_t w = p == 0 ? K[2 * xx] : p == 1 ? K[2 * xx + 1] : K[2 * xx] + K[2 * xx + 1];
                    if (x >= M) w = 0u - w;
                    ext[x] = w << (7 * h);
                }
                int8_t *dst = &out[((id * 3 + p) * 2 + j) * NKB * 1024];
                for (uint32_t kb = 0; kb < NKB; ++kb)
                    for (uint32_t L = 0; L < 64; ++L) {
                        const uint32_t sft = (L >> 2) & 3, l = L & 3, gg = L >> 4;
                        for (uint32_t t = 0; t < 16; ++t) {
                            int8_t limbs[4];
                            balanced_limbs(ext[64 * kb + 16 * gg + sft + t], limbs);
                            dst[(kb * 64 + L) * 16 + t] = limbs[l];
                        }
                    }
            }
        }
    });
    return out;
}

// Offset correction of the Karatsuba form: the kernel multiplies V = D - O,
// with O = 64 on even and 63 on odd coefficients for 7-bit digit chunks (0
// for narrower chunks), so sum_r O_r * K'_r (negacyclic, mod 2^32) is added
// back per step.  Stored per (i, j) in even/odd order.  With s_c / t_c the
// partial / total sums of K' over coefficients of parity c,
//   (O * K')[m] = o_e (2 s_same - t_same) + o_o (2 s_other - t_other).
std::vector<uint32_t> build_brk_kara_corr(const fdfb_ctx &c)
{
    const fdfb_params &P = c.P;
    const uint32_t N = P.N, M = N / 2, ell = P.g_ell, CH = fdfbk::digit_chunks(P.g_log2B);
    const uint32_t RPC = ell * CH, RV = 2 * RPC, R = 2 * ell;
    std::vector<uint32_t> out((size_t)P.n * 2 * N);
    parallel_for((size_t)P.n * 2, [&](size_t id) {
        const uint32_t i = id / 2, j = id % 2;
        std::vector<uint32_t> W(N, 0), Kp(N);
        for (uint32_t rv = 0; rv < RV; ++rv) {
            const uint32_t comp_in = rv / RPC, rr = rv % RPC, jd = rr / CH, h = rr % CH;
            if (7 * (h + 1) > P.g_log2B) continue;  // narrow chunk: no offset
            const uint32_t oe = 64, oo = 63;
            const uint32_t *K = &c.brk[(((size_t)i * R + comp_in * ell + jd) * 2 + j) * N];
            uint32_t tot[2] = {0, 0}, part[2] = {0, 0};
            for (uint32_t x = 0; x < N; ++x) {
                Kp[x] = K[x] << (7 * h);
                tot[x & 1] += Kp[x];
            }
            for (uint32_t m = 0; m < N; ++m) {
                part[m & 1] += Kp[m];
                const uint32_t same = 2 * part[m & 1] - tot[m & 1];
                const uint32_t other = 2 * part[(m & 1) ^ 1] - tot[(m & 1) ^ 1];
                W[m] += oe * same + oo * other;
            }
        }
        for (uint32_t m = 0; m < N; ++m) out[id * N + (m & 1) * M + (m >> 1)] = W[m];
    });
    return out;
}

// First upload of a device array (the pointer must still be null).
template <class T>
int dev_upload(T **dst, const T *src, size_t count)
{
    *dst = nullptr;
    HIP_TRY(hipMalloc((void **)dst, std::max<size_t>(count, 1) * sizeof(T)));
    if (count) HIP_TRY(hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice));
    return FDFB_OK;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

void fdfb_ctx::release_scratch()
{
    bool any = !retired.empty();
    for (auto &p : pools) any = any || p.base;
    if (any) (void)hipDeviceSynchronize();  // launches on any stream may still use the blocks
    for (auto &p : pools)
        if (p.base) (void)hipFree(p.base);
    for (void *p : retired) (void)hipFree(p);
    pools.clear();
    retired.clear();
}

fdfb_ctx::~fdfb_ctx()
{
    for (hipEvent_t e : prof_events) (void)hipEventDestroy(e);
    release_scratch();
    for (void *p : {(void *)d_brk, (void *)d_pk, (void *)d_ksk, d_brk_frag, (void *)d_brk_corr, d_brk_direct,
                    d_pk_frag, d_ksk_frag, (void *)d_luts, (void *)d_err})
        if (p) (void)hipFree(p);
}

namespace fdfbi {

int ensure_device(fdfb_ctx &c)
{
    if (c.abort_flag.load()) return fail(FDFB_EABORTED, "abort flag raised");
    if (!c.on_device) {
        int rc;
        if ((rc = dev_upload(&c.d_brk, c.brk.data(), c.brk.size()))) return rc;
        const fdfb_params &P = c.P;
        if (fdfbk::keyswitch_mfma_supported(P.pk_log2B, P.pk_ell, P.N)) {
            std::vector<int8_t> fr = build_ks_fragments(c.pk.data(), P.N, P.pk_ell, 2 * P.N);
            int8_t *p = nullptr;
            if ((rc = dev_upload(&p, fr.data(), fr.size()))) return rc;
            c.d_pk_frag = p;
        } else if ((rc = dev_upload(&c.d_pk, c.pk.data(), c.pk.size()))) {
            return rc;
        }
        if (fdfbk::keyswitch_mfma_supported(P.ks_log2B, P.ks_ell, P.N)) {
            std::vector<int8_t> fr = build_ks_fragments(c.ksk.data(), P.N, P.ks_ell, P.n + 1);
            int8_t *p = nullptr;
            if ((rc = dev_upload(&p, fr.data(), fr.size()))) return rc;
            c.d_ksk_frag = p;
        } else if ((rc = dev_upload(&c.d_ksk, c.ksk.data(), c.ksk.size()))) {
            return rc;
        }
        if (c.mfma_ok) {
            std::vector<int8_t> fr = build_brk_kara(c);
            int8_t *p = nullptr;
            if ((rc = dev_upload(&p, fr.data(), fr.size()))) return rc;
            c.d_brk_frag = p;
            std::vector<uint32_t> corr = build_brk_kara_corr(c);
            if ((rc = dev_upload(&c.d_brk_corr, corr.data(), corr.size()))) return rc;
        }
        const uint32_t zero = 0;
        if ((rc = dev_upload(&c.d_err, &zero, 1))) return rc;
        c.on_device = true;
    }
    if (c.dev_nluts != c.nluts) {
        // Entries of registered tables never change, so only new tables are
        // copied.  A full buffer is replaced by a larger one and kept alive
        // until the context is freed: work already enqueued, or captured in a
        // HIP graph, keeps reading the old buffer's (unchanged) entries.
        const size_t per = 2 * (size_t)c.P.N;
        if ((size_t)c.nluts > c.d_luts_cap) {
            const size_t cap = std::max<size_t>({(size_t)c.nluts, 2 * c.d_luts_cap, 16});
            int32_t *nb = nullptr;
            HIP_TRY(hipMalloc((void **)&nb, cap * per * sizeof(int32_t)));
            const hipError_t e = hipMemcpy(nb, c.lut_polys.data(), (size_t)c.nluts * per * sizeof(int32_t),
                                           hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                (void)hipFree(nb);
                return fail(FDFB_EDEVICE, std::string("table upload: ") + hipGetErrorString(e));
            }
            if (c.d_luts) c.retired.push_back(c.d_luts);
            c.d_luts = nb;
            c.d_luts_cap = cap;
        } else {
            HIP_TRY(hipMemcpy(c.d_luts + (size_t)c.dev_nluts * per, &c.lut_polys[(size_t)c.dev_nluts * per],
                              (size_t)(c.nluts - c.dev_nluts) * per * sizeof(int32_t), hipMemcpyHostToDevice));
        }
        c.dev_nluts = c.nluts;
    }
    return FDFB_OK;
}

bool device_ready(const fdfb_ctx &c, uint32_t flags)
{
    return c.on_device && c.dev_nluts == c.nluts && (!(flags & FDFB_DIRECT) || c.d_brk_direct);
}

int ensure_form(fdfb_ctx &c, uint32_t flags)
{
    if ((flags & FDFB_DIRECT) && !c.d_brk_direct) {
        std::vector<int8_t> fr = build_brk_fragments(c);
        int8_t *p = nullptr;
        if (int rc = dev_upload(&p, fr.data(), fr.size())) return rc;
        c.d_brk_direct = p;
    }
    return FDFB_OK;
}

// words of each scratch buffer, in the order of ScratchView
static void scratch_words(const fdfb_params &P, uint32_t B, uint32_t L, size_t w[7])
{
    const size_t n1 = P.n + 1, N = P.N, eb = P.boot_ell, E = (size_t)B * L;
    w[0] = B * n1;            // ctN
    w[1] = B * eb * 2 * N;    // acc_sign
    w[2] = B * eb * (N + 1);  // cbits
    w[3] = B * eb * 2 * N;    // rbits
    w[4] = E * 2 * N;         // accf
    w[5] = E * (N + 1);       // cq
    w[6] = kWorkWords;        // work counters
}

size_t scratch_bytes(const fdfb_params &P, uint32_t B, uint32_t L)
{
    size_t w[7], total = 0;
    scratch_words(P, B, L, w);
    for (size_t k : w) total += align256(4 * k);
    return total;
}

ScratchView carve_scratch(const fdfb_params &P, uint32_t B, uint32_t L, void *base)
{
    size_t w[7];
    scratch_words(P, B, L, w);
    ScratchView v;
    uint32_t **bufs[7] = {&v.ctN, &v.acc_sign, &v.cbits, &v.rbits, &v.accf, &v.cq, &v.work};
    char *p = static_cast<char *>(base);
    for (int k = 0; k < 7; ++k) {
        *bufs[k] = reinterpret_cast<uint32_t *>(p);
        p += align256(4 * w[k]);
    }
    return v;
}

int pool_block(fdfb_ctx &c, void *stream, size_t need, void **base)
{
    StreamScratch *ps = nullptr;
    for (auto &p : c.pools)
        if (p.stream == stream) ps = &p;
    if (!ps) {
        c.pools.push_back(StreamScratch{stream, nullptr, 0});
        ps = &c.pools.back();
    }
    if (ps->bytes < need) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing((hipStream_t)stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
            return fail(FDFB_EINVAL, "this stream has no scratch for this batch size and cannot allocate under "
                                     "graph capture: make one call with at least this batch on the stream first");
        size_t bytes = std::max(need, 2 * ps->bytes);
        void *nb = nullptr;
        hipError_t e = hipMalloc(&nb, bytes);
        if (e != hipSuccess && bytes > need) e = hipMalloc(&nb, bytes = need);
        if (e != hipSuccess)
            return fail(e == hipErrorOutOfMemory ? FDFB_ENOMEM : FDFB_EDEVICE,
                        std::string("scratch allocation: ") + hipGetErrorString(e));
        if (ps->base) c.retired.push_back(ps->base);
        ps->base = nb;
        ps->bytes = bytes;
    }
    *base = ps->base;
    return FDFB_OK;
}

int pool_scratch(fdfb_ctx &c, void *stream, uint32_t B, uint32_t L, ScratchView *out)
{
    if ((uint64_t)B * L > 0xFFFFFFFFu) return fail(FDFB_EINVAL, "too many table evaluations in one call");
    void *base = nullptr;
    if (int rc = pool_block(c, stream, scratch_bytes(c.P, B, L), &base)) return rc;
    *out = carve_scratch(c.P, B, L, base);
    return FDFB_OK;
}

// One batched blind rotation in the form `flags` select; the Karatsuba form
// is issued with the tuned plan for A accumulators (work: one device word for
// a queue plan's counter).
hipError_t run_br(fdfb_ctx &c, uint32_t *acc, const uint32_t *ctN, uint32_t A, uint32_t per,
                  uint32_t flags, uint32_t *work, hipStream_t st)
{
    if (flags & FDFB_DIRECT) return fdfbk::launch_br_mfma(c.geom, acc, ctN, A, per, c.d_brk_direct, st);
    if (!(flags & FDFB_PLAIN) && c.mfma_ok) {
        fdfbk::BrPlan plan = tuned_plan(c.geom, A);
        if (plan.form == fdfbk::kFormQueue && !work) plan = fdfbk::BrPlan{};
        return fdfbk::launch_br_kara(c.geom, acc, ctN, A, per, c.d_brk_frag, c.d_brk_corr, plan, work, st);
    }
    return fdfbk::launch_br_plain(c.geom, acc, ctN, A, per, c.d_brk, st);
}

// LWE -> LWE (ksK) or LWE -> RLWE (pK) switching of B samples of dimension N,
// on int8 MFMA when the key was uploaded as fragments.
hipError_t run_ks(fdfb_ctx &c, bool packing, const uint32_t *in, uint32_t B, uint32_t *out, hipStream_t st)
{
    const fdfb_params &P = c.P;
    const int lb = packing ? P.pk_log2B : P.ks_log2B, ell = packing ? P.pk_ell : P.ks_ell;
    const uint32_t out_len = packing ? 2 * P.N : P.n + 1;
    const void *frag = packing ? c.d_pk_frag : c.d_ksk_frag;
    if (frag) return fdfbk::launch_keyswitch_mfma(in, B, P.N, frag, lb, ell, out_len, out, st);
    return fdfbk::launch_keyswitch(in, B, P.N, packing ? c.d_pk : c.d_ksk, lb, ell, out_len, out, st);
}

// The requested blind-rotation form must exist for the context's parameters.
int check_form(const fdfb_ctx &c, uint32_t flags)
{
    if ((flags & FDFB_PLAIN) && (flags & FDFB_DIRECT))
        return fail(FDFB_EINVAL, "FDFB_PLAIN and FDFB_DIRECT are exclusive");
    if ((flags & FDFB_PLAIN) ? !plain_br_fits(c.P)
        : (flags & FDFB_DIRECT) ? !c.mfma_ok
        : !(c.mfma_ok || plain_br_fits(c.P)))
        return fail(FDFB_ENOTSUP, "this blind-rotation form does not support the parameter set");
    return FDFB_OK;
}

#define K_TRY(expr)                                                                            \
    do {                                                                                       \
        hipError_t _e = (expr);                                                                \
        if (_e != hipSuccess)                                                                  \
            return fail(FDFB_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e));      \
    } while (0)

int enqueue_bootstrap(fdfb_ctx &c, const ScratchView &sc, const uint32_t *d_cts, const int32_t *d_ids,
                      uint32_t B, uint32_t *d_out, uint32_t flags, hipStream_t st, uint32_t L, bool profile)
{
    if (!device_ready(c, flags)) return fail(FDFB_EINVAL, "keys and tables are not resident on the device");
    const uint32_t E = B * L;  // table evaluations, sample-major: e = b L + l
    const fdfbk::Geometry &G = c.geom;
    const uint32_t eb = G.boot_ell;
    const uint32_t half = 1u << (31 - G.log2_t);
    hipEvent_t ev[FDFB_NPHASES + 1] = {};
    const bool prof = profile && c.profiling;
    if (prof) {
        for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
        c.prof_events.insert(c.prof_events.end(), ev, ev + FDFB_NPHASES + 1);
    }
    auto mark = [&](int k) { return prof ? hipEventRecord(ev[k], st) : hipSuccess; };
    K_TRY(mark(0));
    // 1. ModSwitch q -> 2N, sign accumulators
    K_TRY(fdfbk::launch_modswitch(G, d_cts, B, sc.ctN, st));
    K_TRY(fdfbk::launch_init_sign(G, sc.ctN, B, sc.acc_sign, st));
    K_TRY(mark(1));
    // 2. the ell_boot sign blind rotations of every sample, one batched pass
    K_TRY(run_br(c, sc.acc_sign, sc.ctN, B * eb, eb, flags, sc.work, st));
    K_TRY(mark(2));
    // 3. bit samples: SampleExtract + L_boot^i Delta/2
    K_TRY(fdfbk::launch_extract(G, sc.acc_sign, B * eb, eb, half, sc.cbits, st));
    K_TRY(mark(3));
    // 4. BuildAcc: LWE -> RLWE switching, then the public mux (one accumulator
    //    per table; the bit samples are shared by the tables of a sample)
    K_TRY(run_ks(c, true, sc.cbits, B * eb, sc.rbits, st));
    K_TRY(mark(4));
    K_TRY(fdfbk::launch_pubmux(G, sc.rbits, sc.ctN, d_ids, E, L, c.d_luts, c.nluts, c.d_err, sc.accf, st));
    K_TRY(mark(5));
    // 5. function blind rotations, L per sample
    K_TRY(run_br(c, sc.accf, sc.ctN, E, L, flags, sc.work, st));
    K_TRY(mark(6));
    // 6. SampleExtract, then LWE(N) -> LWE(n) unless the extracted form is requested
    if (flags & FDFB_OUT_EXTRACTED) {
        K_TRY(fdfbk::launch_extract(G, sc.accf, E, 1, 0, d_out, st));
    } else {
        K_TRY(fdfbk::launch_extract(G, sc.accf, E, 1, 0, sc.cq, st));
        K_TRY(run_ks(c, false, sc.cq, E, d_out, st));
    }
    K_TRY(mark(7));
    return FDFB_OK;
}

bool queue_eligible(const fdfb_ctx &c, uint32_t flags)
{
    return !(flags & (FDFB_PLAIN | FDFB_DIRECT)) && c.mfma_ok && fdfbk::br_queue_supported(c.geom);
}

// The steps of one job before, between and after its blind rotations.
static int job_front(const fdfb_job &j, const ScratchView &sc, hipStream_t st)
{
    K_TRY(fdfbk::launch_modswitch(j.ctx->geom, j.d_cts, j.B, sc.ctN, st));
    K_TRY(fdfbk::launch_init_sign(j.ctx->geom, sc.ctN, j.B, sc.acc_sign, st));
    return FDFB_OK;
}

static int job_mid(const fdfb_job &j, const ScratchView &sc, hipStream_t st)
{
    fdfb_ctx &c = *j.ctx;
    const fdfbk::Geometry &G = c.geom;
    K_TRY(fdfbk::launch_extract(G, sc.acc_sign, j.B * G.boot_ell, G.boot_ell, 1u << (31 - G.log2_t), sc.cbits, st));
    K_TRY(run_ks(c, true, sc.cbits, j.B * G.boot_ell, sc.rbits, st));
    K_TRY(fdfbk::launch_pubmux(G, sc.rbits, sc.ctN, j.d_lut_ids, j.B, 1, c.d_luts, c.nluts, c.d_err, sc.accf, st));
    return FDFB_OK;
}

static int job_back(const fdfb_job &j, const ScratchView &sc, hipStream_t st)
{
    fdfb_ctx &c = *j.ctx;
    if (j.flags & FDFB_OUT_EXTRACTED) {
        K_TRY(fdfbk::launch_extract(c.geom, sc.accf, j.B, 1, 0, j.d_out, st));
    } else {
        K_TRY(fdfbk::launch_extract(c.geom, sc.accf, j.B, 1, 0, sc.cq, st));
        K_TRY(run_ks(c, false, sc.cq, j.B, j.d_out, st));
    }
    return FDFB_OK;
}

// Queue descriptor of accumulators [a0, a0 + A) of job j's sign rotations
// (a0 a multiple of the accumulators per sample) or of its function rotation.
static fdfbk::BrJobDesc job_desc(const fdfb_job &j, const ScratchView &sc, bool sign, uint32_t a0, uint32_t A)
{
    const fdfb_ctx &c = *j.ctx;
    const uint32_t per = sign ? c.geom.boot_ell : 1, N = c.P.N;
    fdfbk::BrJobDesc x;
    x.G = c.geom;
    x.acc = (sign ? sc.acc_sign : sc.accf) + (size_t)a0 * 2 * N;
    x.ctN = sc.ctN + (size_t)(a0 / per) * (c.P.n + 1);
    x.A = A;
    x.per = per;
    x.bfrag = c.d_brk_frag;
    x.corr = c.d_brk_corr;
    return x;
}

int enqueue_multi(const fdfb_job *jobs, uint32_t njobs, const ScratchView *views, uint32_t *counters,
                  uint32_t ncounters, bool use_queue, hipStream_t st)
{
    // eligible jobs of one phase, as queue descriptors
    auto descs = [&](bool sign, std::vector<fdfbk::BrJobDesc> &d, std::vector<uint32_t> &others) {
        d.clear();
        others.clear();
        for (uint32_t k = 0; k < njobs; ++k) {
            const fdfb_job &j = jobs[k];
            if (!j.B) continue;
            if (use_queue && queue_eligible(*j.ctx, j.flags))
                d.push_back(job_desc(j, views[k], sign, 0, sign ? j.B * j.ctx->geom.boot_ell : j.B));
            else
                others.push_back(k);
        }
    };
    std::vector<fdfbk::BrJobDesc> d;
    std::vector<uint32_t> others;
    // ModSwitch and sign accumulators of every job
    for (uint32_t k = 0; k < njobs; ++k)
        if (jobs[k].B)
            if (int rc = job_front(jobs[k], views[k], st)) return rc;
    // the sign rotations of all jobs
    descs(true, d, others);
    uint32_t launches = 0;
    K_TRY(fdfbk::br_queue_launches(d.data(), (int)d.size(), &launches));
    if (2 * launches > ncounters) return fail(FDFB_EINVAL, "too many job groups for one submission");
    K_TRY(fdfbk::launch_br_queue(d.data(), (int)d.size(), counters, launches, st));
    for (uint32_t k : others) {
        const fdfb_job &j = jobs[k];
        K_TRY(run_br(*j.ctx, views[k].acc_sign, views[k].ctN, j.B * j.ctx->geom.boot_ell, j.ctx->geom.boot_ell,
                     j.flags, views[k].work, st));
    }
    // bit samples, packing key switch, public mux of every job
    for (uint32_t k = 0; k < njobs; ++k)
        if (jobs[k].B)
            if (int rc = job_mid(jobs[k], views[k], st)) return rc;
    // the function rotations of all jobs
    descs(false, d, others);
    K_TRY(fdfbk::launch_br_queue(d.data(), (int)d.size(), counters + launches, ncounters - launches, st));
    for (uint32_t k : others) {
        const fdfb_job &j = jobs[k];
        K_TRY(run_br(*j.ctx, views[k].accf, views[k].ctN, j.B, 1, j.flags, views[k].work, st));
    }
    // SampleExtract and the final key switch of every job
    for (uint32_t k = 0; k < njobs; ++k)
        if (jobs[k].B)
            if (int rc = job_back(jobs[k], views[k], st)) return rc;
    return FDFB_OK;
}

int enqueue_pipeline(const fdfb_job *jobs, uint32_t njobs, const ScratchView *views, uint32_t *counters,
                     uint32_t ncounters, uint32_t rounds, hipStream_t st)
{
    // resident workgroups of the persistent kernel for these jobs
    std::vector<fdfbk::BrJobDesc> all;
    std::vector<fdfbp::Job> pj(njobs);
    for (uint32_t k = 0; k < njobs; ++k) {
        const fdfbk::Geometry &G = jobs[k].ctx->geom;
        pj[k] = {jobs[k].B, (uint32_t)G.boot_ell, G.N > 1024};
        if (jobs[k].B) all.push_back(job_desc(jobs[k], views[k], false, 0, jobs[k].B));
    }
    uint32_t cap = 0;
    K_TRY(fdfbk::br_queue_slots(all.data(), (int)all.size(), &cap));
    if (!cap) return FDFB_OK;
    std::vector<fdfbk::BrJobDesc> d;
    for (const fdfbp::Launch &L : fdfbp::schedule(pj, cap, rounds)) {
        for (uint32_t k : L.fronts)
            if (int rc = job_front(jobs[k], views[k], st)) return rc;
        d.clear();
        for (const fdfbp::Range &r : L.ranges) d.push_back(job_desc(jobs[r.job], views[r.job], r.sign, r.a0, r.A));
        uint32_t launches = 0;
        K_TRY(fdfbk::br_queue_launches(d.data(), (int)d.size(), &launches));
        if (launches > ncounters) return fail(FDFB_EINVAL, "too many job groups for one launch");
        K_TRY(fdfbk::launch_br_queue(d.data(), (int)d.size(), counters, ncounters, st));
        for (uint32_t k : L.backs)
            if (int rc = job_back(jobs[k], views[k], st)) return rc;
        for (uint32_t k : L.mids)
            if (int rc = job_mid(jobs[k], views[k], st)) return rc;
    }
    return FDFB_OK;
}

}  // namespace fdfbi

using namespace fdfbi;

// ============================================================================
// C ABI
// ============================================================================
// FDFB_TRACE set (and not "0") when a context is created: record the phase
// events of every bootstrap call on it and print their summary on fdfb_free.
static void apply_trace_env(fdfb_ctx &c)
{
    const char *v = std::getenv("FDFB_TRACE");
    if (v && *v && std::strcmp(v, "0") != 0) c.profiling = c.trace = true;
}

using Lock = std::lock_guard<std::recursive_mutex>;

// A multi-job submission captured in a HIP graph, with its own scratch.
struct fdfb_graph {
    std::vector<fdfb_job> jobs;
    void *scratch = nullptr;
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool uses_queue = false;
    ~fdfb_graph()
    {
        if (stream) (void)hipStreamSynchronize(stream);
        if (exec) {
            (void)hipDeviceSynchronize();  // replays on any stream may still run
            (void)hipGraphExecDestroy(exec);
        }
        if (graph) (void)hipGraphDestroy(graph);
        if (stream) (void)hipStreamDestroy(stream);
        if (scratch) (void)hipFree(scratch);
    }
};

// Keys, tables and the requested form resident on the device.
static int prepare(fdfb_ctx &c, uint32_t flags)
{
    int rc = ensure_device(c);
    if (!rc) rc = ensure_form(c, flags);
    return rc;
}

// Arguments shared by the bootstrap entry points.
static int check_batch(const fdfb_ctx *c, const void *d_cts, const void *d_ids, const void *d_out, uint32_t flags)
{
    if (c->abort_flag.load()) return fail(FDFB_EABORTED, "abort flag raised");
    if (!d_cts || !d_ids || !d_out) return fail(FDFB_EINVAL, "null buffer");
    if (flags & ~kAllFlags) return fail(FDFB_EINVAL, "unknown flag");
    return check_form(*c, flags);
}

extern "C" {

const char *fdfb_last_error(void) { return g_last_error.c_str(); }

int fdfb_keygen_from_seed(const fdfb_params *params, uint64_t seed, fdfb_ctx **out)
{
    return guarded([&]() -> int {
        if (!params || !out) return fail(FDFB_EINVAL, "null argument");
        *out = nullptr;
        int rc = check_params(*params);
        if (rc) return rc;
        std::unique_ptr<fdfb_ctx> c(new fdfb_ctx());
        apply_trace_env(*c);
        c->P = *params;
        c->seed = seed;
        c->geom = geometry_of(*params);
        c->mfma_ok = fdfbk::br_mfma_supported(c->geom);
        generate_keys(*c);
        *out = c.release();
        return FDFB_OK;
    });
}

int fdfb_register_lut(fdfb_ctx *c, const uint32_t *table, int32_t *lut_id)
{
    return guarded([&]() -> int {
        if (!c || !table || !lut_id) return fail(FDFB_EINVAL, "null argument");
        Lock lk(c->mu);
        const uint32_t t = 1u << c->P.log2_t, N = c->P.N;
        for (uint32_t m = 0; m < t; ++m)
            if (table[m] >= t) return fail(FDFB_EINVAL, "table value out of range [0, t)");
        if (c->nluts == INT32_MAX) return fail(FDFB_EINVAL, "too many tables");
        std::vector<int32_t> poly(2 * (size_t)N);
        setup_polynomial(table, t, N, poly.data(), poly.data() + N);
        c->lut_tables.insert(c->lut_tables.end(), table, table + t);
        c->lut_polys.insert(c->lut_polys.end(), poly.begin(), poly.end());
        *lut_id = c->nluts++;
        return FDFB_OK;
    });
}

int fdfb_bootstrap_batch(fdfb_ctx *c, const uint32_t *d_cts, const int32_t *d_lut_ids, uint32_t B,
                         uint32_t *d_out, uint32_t flags, void *stream)
{
    return fdfb_bootstrap_multi_lut(c, d_cts, d_lut_ids, B, 1, d_out, flags, stream);
}

int fdfb_bootstrap_multi_lut(fdfb_ctx *c, const uint32_t *d_cts, const int32_t *d_lut_ids, uint32_t B,
                             uint32_t L, uint32_t *d_out, uint32_t flags, void *stream)
{
    return guarded([&]() -> int {
        if (!c) return fail(FDFB_EINVAL, "null context");
        if (L == 0) return fail(FDFB_EINVAL, "at least one table per sample");
        if (B == 0) return c->abort_flag.load() ? fail(FDFB_EABORTED, "abort flag raised") : FDFB_OK;
        Lock lk(c->mu);
        int rc = check_batch(c, d_cts, d_lut_ids, d_out, flags);
        if (!rc) rc = prepare(*c, flags);
        ScratchView sc;
        if (!rc) rc = pool_scratch(*c, stream, B, L, &sc);
        if (rc) return rc;
        return enqueue_bootstrap(*c, sc, d_cts, d_lut_ids, B, d_out, flags, (hipStream_t)stream, L);
    });
}

int fdfb_tfhe_bootstrap_batch(fdfb_ctx *c, const uint32_t *d_cts, const int32_t *d_lut_ids, uint32_t B,
                              uint32_t *d_out, uint32_t flags, void *stream)
{
    return guarded([&]() -> int {
        if (!c) return fail(FDFB_EINVAL, "null context");
        if (B == 0) return c->abort_flag.load() ? fail(FDFB_EABORTED, "abort flag raised") : FDFB_OK;
        Lock lk(c->mu);
        int rc = check_batch(c, d_cts, d_lut_ids, d_out, flags);
        if (!rc) rc = prepare(*c, flags);
        ScratchView sc;
        if (!rc) rc = pool_scratch(*c, stream, B, 1, &sc);
        if (rc) return rc;
        const fdfbk::Geometry &G = c->geom;
        const hipStream_t st = (hipStream_t)stream;
        K_TRY(fdfbk::launch_modswitch(G, d_cts, B, sc.ctN, st));
        K_TRY(fdfbk::launch_init_tfhe(G, sc.ctN, d_lut_ids, B, c->d_luts, c->nluts, c->d_err, sc.accf, st));
        K_TRY(run_br(*c, sc.accf, sc.ctN, B, 1, flags, sc.work, st));
        if (flags & FDFB_OUT_EXTRACTED) {
            K_TRY(fdfbk::launch_extract(G, sc.accf, B, 1, 0, d_out, st));
        } else {
            K_TRY(fdfbk::launch_extract(G, sc.accf, B, 1, 0, sc.cq, st));
            K_TRY(run_ks(*c, false, sc.cq, B, d_out, st));
        }
        return FDFB_OK;
    });
}

// Validate the jobs of a multi-job submission (contexts locked by the
// caller) and upload what they need.
static int check_jobs(const fdfb_job *jobs, uint32_t njobs)
{
    if (njobs > kMaxJobs) return fail(FDFB_EINVAL, "at most " + std::to_string(kMaxJobs) + " jobs per submission");
    for (uint32_t k = 0; k < njobs; ++k) {
        const fdfb_job &j = jobs[k];
        if (j.ctx->abort_flag.load()) return fail(FDFB_EABORTED, "abort flag raised");
        if (j.B == 0) continue;
        if (int rc = check_batch(j.ctx, j.d_cts, j.d_lut_ids, j.d_out, j.flags)) return rc;
    }
    for (uint32_t k = 0; k < njobs; ++k)
        if (jobs[k].B)
            if (int rc = prepare(*jobs[k].ctx, jobs[k].flags)) return rc;
    return FDFB_OK;
}

// Locks of every distinct context of a job list, taken in address order (no
// lock-order cycles between concurrent submissions).
static int lock_jobs(const fdfb_job *jobs, uint32_t njobs, std::vector<std::unique_lock<std::recursive_mutex>> &locks)
{
    if (njobs && !jobs) return fail(FDFB_EINVAL, "null jobs");
    std::vector<fdfb_ctx *> ctxs;
    for (uint32_t k = 0; k < njobs; ++k) {
        if (!jobs[k].ctx) return fail(FDFB_EINVAL, "null context in job");
        ctxs.push_back(jobs[k].ctx);
    }
    std::sort(ctxs.begin(), ctxs.end());
    ctxs.erase(std::unique(ctxs.begin(), ctxs.end()), ctxs.end());
    for (fdfb_ctx *c : ctxs) locks.emplace_back(c->mu);
    return FDFB_OK;
}

// The persistent queue takes the blind rotations of a submission when its
// eligible jobs span more than one context (a single context's rotations
// already fill the device in rounds of the resident capacity).
static bool multi_uses_queue(const fdfb_job *jobs, uint32_t njobs)
{
    const fdfb_ctx *first = nullptr;
    for (uint32_t k = 0; k < njobs; ++k) {
        if (!jobs[k].B || !queue_eligible(*jobs[k].ctx, jobs[k].flags)) continue;
        if (first && jobs[k].ctx != first) return true;
        first = jobs[k].ctx;
    }
    return false;
}

// Scratch of every job: one block per context on `stream`, each job of that
// context at its own offset; the work counters of the submission follow the
// first job's scratch.
static int multi_scratch(const fdfb_job *jobs, uint32_t njobs, void *stream, std::vector<ScratchView> &views,
                         uint32_t **counters)
{
    views.assign(njobs, ScratchView{});
    *counters = nullptr;
    std::vector<fdfb_ctx *> done;
    for (uint32_t k = 0; k < njobs; ++k) {
        fdfb_ctx *c = jobs[k].ctx;
        if (!jobs[k].B || std::find(done.begin(), done.end(), c) != done.end()) continue;
        done.push_back(c);
        size_t total = 0;
        for (uint32_t m = k; m < njobs; ++m)
            if (jobs[m].ctx == c && jobs[m].B) total += scratch_bytes(c->P, jobs[m].B);
        void *base = nullptr;
        if (int rc = pool_block(*c, stream, total, &base)) return rc;
        size_t off = 0;
        for (uint32_t m = k; m < njobs; ++m)
            if (jobs[m].ctx == c && jobs[m].B) {
                views[m] = carve_scratch(c->P, jobs[m].B, 1, static_cast<char *>(base) + off);
                off += scratch_bytes(c->P, jobs[m].B);
                if (!*counters) *counters = views[m].work;
            }
    }
    return FDFB_OK;
}

int fdfb_bootstrap_multi(const fdfb_job *jobs, uint32_t njobs, void *stream)
{
    return fdfb_bootstrap_multi_ex(jobs, njobs, -1, stream);
}

int fdfb_bootstrap_multi_ex(const fdfb_job *jobs, uint32_t njobs, int use_queue, void *stream)
{
    return guarded([&]() -> int {
        if (use_queue < -1 || use_queue > 1) return fail(FDFB_EINVAL, "use_queue must be -1, 0 or 1");
        std::vector<std::unique_lock<std::recursive_mutex>> locks;
        if (int rc = lock_jobs(jobs, njobs, locks)) return rc;
        if (int rc = check_jobs(jobs, njobs)) return rc;
        std::vector<ScratchView> views;
        uint32_t *counters = nullptr;
        if (int rc = multi_scratch(jobs, njobs, stream, views, &counters)) return rc;
        if (!counters) return FDFB_OK;  // no samples
        const bool queue = use_queue < 0 ? multi_uses_queue(jobs, njobs) : use_queue == 1;
        return enqueue_multi(jobs, njobs, views.data(), counters, kWorkWords, queue, (hipStream_t)stream);
    });
}

int fdfb_bootstrap_pipeline(const fdfb_job *jobs, uint32_t njobs, uint32_t rounds, void *stream)
{
    return guarded([&]() -> int {
        if (rounds > kMaxPipelineRounds)
            return fail(FDFB_EINVAL, "rounds must be at most " + std::to_string(kMaxPipelineRounds));
        std::vector<std::unique_lock<std::recursive_mutex>> locks;
        if (int rc = lock_jobs(jobs, njobs, locks)) return rc;
        if (njobs > kMaxJobs) return fail(FDFB_EINVAL, "at most " + std::to_string(kMaxJobs) + " jobs per submission");
        for (uint32_t k = 0; k < njobs; ++k)
            if (jobs[k].B && !queue_eligible(*jobs[k].ctx, jobs[k].flags))
                return fail(FDFB_EINVAL, "job " + std::to_string(k) +
                                             ": its blind rotations are not in a form the work-queue kernel takes");
        if (int rc = check_jobs(jobs, njobs)) return rc;
        std::vector<ScratchView> views;
        uint32_t *counters = nullptr;
        if (int rc = multi_scratch(jobs, njobs, stream, views, &counters)) return rc;
        if (!counters) return FDFB_OK;  // no samples
        return enqueue_pipeline(jobs, njobs, views.data(), counters, kWorkWords, rounds ? rounds : 4,
                                (hipStream_t)stream);
    });
}

int fdfb_multi_graph_create(const fdfb_job *jobs, uint32_t njobs, int use_queue, fdfb_graph **out)
{
    return guarded([&]() -> int {
        if (!out) return fail(FDFB_EINVAL, "null argument");
        *out = nullptr;
        if (use_queue < -1 || use_queue > 1) return fail(FDFB_EINVAL, "use_queue must be -1, 0 or 1");
        std::vector<std::unique_lock<std::recursive_mutex>> locks;
        if (int rc = lock_jobs(jobs, njobs, locks)) return rc;
        if (int rc = check_jobs(jobs, njobs)) return rc;
        std::unique_ptr<fdfb_graph> g(new fdfb_graph());
        g->jobs.assign(jobs, jobs + njobs);
        // the graph's own scratch: every job at its own offset
        size_t total = 0;
        for (uint32_t k = 0; k < njobs; ++k)
            if (jobs[k].B) total += scratch_bytes(jobs[k].ctx->P, jobs[k].B);
        if (!total) return fail(FDFB_EINVAL, "no samples to capture");
        HIP_TRY(hipMalloc(&g->scratch, total));
        std::vector<ScratchView> views(njobs);
        uint32_t *counters = nullptr;
        size_t off = 0;
        for (uint32_t k = 0; k < njobs; ++k)
            if (jobs[k].B) {
                views[k] = carve_scratch(jobs[k].ctx->P, jobs[k].B, 1, static_cast<char *>(g->scratch) + off);
                off += scratch_bytes(jobs[k].ctx->P, jobs[k].B);
                if (!counters) counters = views[k].work;
            }
        const bool queue = use_queue < 0 ? multi_uses_queue(jobs, njobs) : use_queue == 1;
        hipStream_t st = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        g->stream = st;
        // one eager pass sets every kernel's attributes (none may change under capture)
        if (int rc = enqueue_multi(jobs, njobs, views.data(), counters, kWorkWords, queue, st)) return rc;
        HIP_TRY(hipStreamSynchronize(st));
        HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        int rc = enqueue_multi(jobs, njobs, views.data(), counters, kWorkWords, queue, st);
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(st, &graph);
        g->graph = graph;
        if (rc) return rc;
        if (ec != hipSuccess) return fail(FDFB_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ec));
        HIP_TRY(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
        g->uses_queue = queue;
        *out = g.release();
        return FDFB_OK;
    });
}

int fdfb_graph_launch(fdfb_graph *g, void *stream)
{
    return guarded([&]() -> int {
        if (!g || !g->exec) return fail(FDFB_EINVAL, "null graph");
        for (const fdfb_job &j : g->jobs)
            if (j.ctx->abort_flag.load()) return fail(FDFB_EABORTED, "abort flag raised");
        HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream));
        return FDFB_OK;
    });
}

int fdfb_graph_info(const fdfb_graph *g, uint32_t *uses_queue, size_t *scratch_bytes_out)
{
    return guarded([&]() -> int {
        if (!g || !uses_queue || !scratch_bytes_out) return fail(FDFB_EINVAL, "null argument");
        *uses_queue = g->uses_queue ? 1 : 0;
        size_t total = 0;
        for (const fdfb_job &j : g->jobs)
            if (j.B) total += scratch_bytes(j.ctx->P, j.B);
        *scratch_bytes_out = total;
        return FDFB_OK;
    });
}

void fdfb_graph_free(fdfb_graph *g)
{
    delete g;
}

int fdfb_keyswitch(fdfb_ctx *c, const uint32_t *d_in, uint32_t B, uint32_t *d_out, void *stream)
{
    return guarded([&]() -> int {
        if (!c) return fail(FDFB_EINVAL, "null context");
        if (B == 0) return FDFB_OK;
        if (!d_in || !d_out) return fail(FDFB_EINVAL, "null buffer");
        Lock lk(c->mu);
        int rc = ensure_device(*c);
        if (rc) return rc;
        K_TRY(run_ks(*c, false, d_in, B, d_out, (hipStream_t)stream));
        return FDFB_OK;
    });
}

int fdfb_modswitch(fdfb_ctx *c, const uint32_t *d_cts, uint32_t B, uint32_t *d_ctN, void *stream)
{
    return guarded([&]() -> int {
        if (!c) return fail(FDFB_EINVAL, "null context");
        if (B == 0) return FDFB_OK;
        if (!d_cts || !d_ctN) return fail(FDFB_EINVAL, "null buffer");
        Lock lk(c->mu);
        int rc = ensure_device(*c);
        if (rc) return rc;
        K_TRY(fdfbk::launch_modswitch(c->geom, d_cts, B, d_ctN, (hipStream_t)stream));
        return FDFB_OK;
    });
}

int fdfb_blind_rotate(fdfb_ctx *c, uint32_t *d_acc, const uint32_t *d_ctN, uint32_t A,
                      uint32_t accs_per_ct, uint32_t flags, void *stream)
{
    return guarded([&]() -> int {
        if (!c) return fail(FDFB_EINVAL, "null context");
        if (A == 0) return FDFB_OK;
        if (!d_acc || !d_ctN || accs_per_ct == 0) return fail(FDFB_EINVAL, "null buffer or accs_per_ct = 0");
        if (flags & ~kAllFlags) return fail(FDFB_EINVAL, "unknown flag");
        Lock lk(c->mu);
        if (int rc = check_form(*c, flags)) return rc;
        if (int rc = prepare(*c, flags)) return rc;
        void *work = nullptr;  // a queue plan's counter, in this stream's scratch block
        if (int rc = pool_block(*c, stream, kWorkWords * 4, &work)) return rc;
        K_TRY(run_br(*c, d_acc, d_ctN, A, accs_per_ct, flags, static_cast<uint32_t *>(work), (hipStream_t)stream));
        return FDFB_OK;
    });
}

int fdfb_sample_extract(fdfb_ctx *c, const uint32_t *d_acc, uint32_t A, uint32_t *d_lwe, void *stream)
{
    return guarded([&]() -> int {
        if (!c) return fail(FDFB_EINVAL, "null context");
        if (A == 0) return FDFB_OK;
        if (!d_acc || !d_lwe) return fail(FDFB_EINVAL, "null buffer");
        K_TRY(fdfbk::launch_extract(c->geom, d_acc, A, 1, 0, d_lwe, (hipStream_t)stream));
        return FDFB_OK;
    });
}

int fdfb_packing_keyswitch(fdfb_ctx *c, const uint32_t *d_in, uint32_t A, uint32_t *d_out, void *stream)
{
    return guarded([&]() -> int {
        if (!c) return fail(FDFB_EINVAL, "null context");
        if (A == 0) return FDFB_OK;
        if (!d_in || !d_out) return fail(FDFB_EINVAL, "null buffer");
        Lock lk(c->mu);
        int rc = ensure_device(*c);
        if (rc) return rc;
        K_TRY(run_ks(*c, true, d_in, A, d_out, (hipStream_t)stream));
        return FDFB_OK;
    });
}

int fdfb_pubmux(fdfb_ctx *c, const uint32_t *d_rlwe, const uint32_t *d_ctN, const int32_t *d_lut_ids,
                uint32_t B, uint32_t *d_acc, void *stream)
{
    return guarded([&]() -> int {
        if (!c) return fail(FDFB_EINVAL, "null context");
        if (B == 0) return FDFB_OK;
        if (!d_rlwe || !d_ctN || !d_lut_ids || !d_acc) return fail(FDFB_EINVAL, "null buffer");
        Lock lk(c->mu);
        int rc = ensure_device(*c);
        if (rc) return rc;
        K_TRY(fdfbk::launch_pubmux(c->geom, d_rlwe, d_ctN, d_lut_ids, B, 1, c->d_luts, c->nluts, c->d_err, d_acc,
                                   (hipStream_t)stream));
        return FDFB_OK;
    });
}

int fdfb_affine(const int32_t *d_W, const uint32_t *d_in, uint32_t rows, uint32_t cols, uint32_t width,
                uint32_t *d_out, void *stream)
{
    return guarded([&]() -> int {
        if (rows == 0 || width == 0) return FDFB_OK;
        if (!d_W || (cols && !d_in) || !d_out) return fail(FDFB_EINVAL, "null buffer");
        K_TRY(fdfbk::launch_affine(d_W, d_in, rows, cols, width, d_out, (hipStream_t)stream));
        return FDFB_OK;
    });
}

int fdfb_lincomb2(const uint32_t *d_x, const uint32_t *d_y, int32_t wx, int32_t wy, uint32_t B, uint32_t width,
                  uint32_t *d_out, void *stream)
{
    return guarded([&]() -> int {
        if (B == 0 || width == 0) return FDFB_OK;
        if (!d_x || !d_y || !d_out) return fail(FDFB_EINVAL, "null buffer");
        if ((uint64_t)B * width > 0xFFFFFFFFu) return fail(FDFB_EINVAL, "B * width must fit 32 bits");
        K_TRY(fdfbk::launch_lincomb2(d_x, d_y, wx, wy, B * width, d_out, (hipStream_t)stream));
        return FDFB_OK;
    });
}

int fdfb_encrypt_debug(fdfb_ctx *c, const uint32_t *m, uint32_t B, uint64_t seed, uint32_t *cts)
{
    return guarded([&]() -> int {
        if (!c || (B && (!m || !cts))) return fail(FDFB_EINVAL, "null argument");
        Lock lk(c->mu);
        const uint32_t n = c->P.n, t = 1u << c->P.log2_t, delta = 1u << (32 - c->P.log2_t);
        const CounterRng ra(seed, kTagEncA), re(seed, kTagEncE);
        for (uint32_t b = 0; b < B; ++b)
            if (m[b] >= t) return fail(FDFB_EINVAL, "message out of range [0, t)");
        for (uint32_t b = 0; b < B; ++b) {
            uint32_t *ct = cts + (size_t)b * (n + 1), dot = 0;
            for (uint32_t q = 0; q < n; ++q) {
                ct[1 + q] = ra.uniform32((uint64_t)b * n + q);
                dot += ct[1 + q] * c->s[q];
            }
            ct[0] = dot + delta * m[b] + static_cast<uint32_t>(re.gaussian(b, c->P.sigma_lwe));
        }
        return FDFB_OK;
    });
}

int fdfb_decrypt_debug(fdfb_ctx *c, const uint32_t *cts, uint32_t B, uint32_t dim, uint32_t *m_out,
                       int64_t *err_out)
{
    return guarded([&]() -> int {
        if (!c || (B && (!cts || !m_out))) return fail(FDFB_EINVAL, "null argument");
        Lock lk(c->mu);
        const std::vector<uint32_t> *key = nullptr;
        if (dim == c->P.n) key = &c->s;
        else if (dim == c->P.N) key = &c->sf;
        else return fail(FDFB_EINVAL, "dim must be n or N");
        const uint32_t sh = 32 - c->P.log2_t, tmask = (1u << c->P.log2_t) - 1;
        for (uint32_t b = 0; b < B; ++b) {
            const uint32_t *ct = cts + (size_t)b * (dim + 1);
            uint32_t ph = ct[0];
            for (uint32_t q = 0; q < dim; ++q) ph -= ct[1 + q] * (*key)[q];
            const uint32_t mm = (uint32_t)(((uint64_t)ph + (1ull << (sh - 1))) >> sh) & tmask;
            m_out[b] = mm;
            if (err_out) err_out[b] = (int64_t)(int32_t)(ph - (mm << sh));
        }
        return FDFB_OK;
    });
}

// --- serialisation ----------------------------------------------------------
static const char kMagic[8] = {'F', 'D', 'F', 'B', 'K', 'E', 'Y', '1'};
static constexpr size_t kHead = sizeof(kMagic) + sizeof(fdfb_params) + 8 + 8 * 6;

int fdfb_export_keys(const fdfb_ctx *cc, void *buf, size_t *len)
{
    return guarded([&]() -> int {
        if (!cc || !len) return fail(FDFB_EINVAL, "null argument");
        fdfb_ctx *c = const_cast<fdfb_ctx *>(cc);  // the lock only
        Lock lk(c->mu);
        const uint64_t counts[] = {c->s.size(), c->sf.size(), c->brk.size(), c->pk.size(), c->ksk.size(),
                                   c->lut_tables.size()};
        size_t need = kHead;
        for (uint64_t k : counts) need += 4 * k;
        if (!buf) {
            *len = need;
            return FDFB_OK;
        }
        if (*len < need) {
            *len = need;
            return fail(FDFB_EINVAL, "buffer too small");
        }
        char *p = static_cast<char *>(buf);
        auto put = [&](const void *src, size_t n) { std::memcpy(p, src, n); p += n; };
        put(kMagic, 8);
        put(&c->P, sizeof(fdfb_params));
        put(&c->seed, 8);
        put(counts, sizeof(counts));
        put(c->s.data(), 4 * counts[0]);
        put(c->sf.data(), 4 * counts[1]);
        put(c->brk.data(), 4 * counts[2]);
        put(c->pk.data(), 4 * counts[3]);
        put(c->ksk.data(), 4 * counts[4]);
        put(c->lut_tables.data(), 4 * counts[5]);
        *len = need;
        return FDFB_OK;
    });
}

int fdfb_import_keys(const void *buf, size_t len, fdfb_ctx **out)
{
    return guarded([&]() -> int {
        if (!buf || !out) return fail(FDFB_EINVAL, "null argument");
        *out = nullptr;
        const char *p = static_cast<const char *>(buf);
        if (len < kHead || std::memcmp(p, kMagic, 8)) return fail(FDFB_EINVAL, "not an fdfb key blob");
        fdfb_params P;
        std::memcpy(&P, p + 8, sizeof(P));
        int rc = check_params(P);
        if (rc) return rc;
        uint64_t seed, counts[6];
        std::memcpy(&seed, p + 8 + sizeof(P), 8);
        std::memcpy(counts, p + 16 + sizeof(P), sizeof(counts));
        const uint32_t n = P.n, N = P.N, t = 1u << P.log2_t;
        const uint64_t want[] = {n, N, (uint64_t)n * 2 * P.g_ell * 2 * N, (uint64_t)N * P.pk_ell * 2 * N,
                                 (uint64_t)N * P.ks_ell * (n + 1)};
        for (int k = 0; k < 5; ++k)
            if (counts[k] != want[k]) return fail(FDFB_EINVAL, "key blob sizes do not match its parameters");
        if (counts[5] % t) return fail(FDFB_EINVAL, "malformed table section");
        // every section must lie inside the blob: compare counts against the
        // bytes left, never sum them (a forged count must not wrap)
        size_t left = len - kHead;
        for (uint64_t k : counts) {
            if (k > left / 4) return fail(FDFB_EINVAL, "truncated key blob");
            left -= 4 * k;
        }
        std::unique_ptr<fdfb_ctx> c(new fdfb_ctx());
        apply_trace_env(*c);
        c->P = P;
        c->seed = seed;
        c->geom = geometry_of(P);
        c->mfma_ok = fdfbk::br_mfma_supported(c->geom);
        const char *q = p + kHead;
        auto take = [&](std::vector<uint32_t> &v, uint64_t k) {
            v.resize(k);
            std::memcpy(v.data(), q, 4 * k);
            q += 4 * k;
        };
        take(c->s, counts[0]);
        take(c->sf, counts[1]);
        take(c->brk, counts[2]);
        take(c->pk, counts[3]);
        take(c->ksk, counts[4]);
        for (uint32_t v : c->s)
            if (v > 1) return fail(FDFB_EINVAL, "secret key s is not binary");
        for (uint32_t v : c->sf)
            if (v > 1) return fail(FDFB_EINVAL, "secret key s_F is not binary");
        std::vector<uint32_t> tables;
        take(tables, counts[5]);
        for (size_t k = 0; k < tables.size(); k += t) {
            int32_t id;
            if ((rc = fdfb_register_lut(c.get(), &tables[k], &id))) return rc;
        }
        *out = c.release();
        return FDFB_OK;
    });
}

int fdfb_get_key(const fdfb_ctx *cc, uint32_t which, uint32_t *host, size_t *count)
{
    return guarded([&]() -> int {
        if (!cc || !count) return fail(FDFB_EINVAL, "null argument");
        fdfb_ctx *c = const_cast<fdfb_ctx *>(cc);  // the lock only
        Lock lk(c->mu);
        const std::vector<uint32_t> *v[] = {&c->s, &c->sf, &c->brk, &c->pk, &c->ksk};
        if (which > 4) return fail(FDFB_EINVAL, "which must be 0..4");
        const size_t need = v[which]->size();
        if (!host) { *count = need; return FDFB_OK; }
        if (*count < need) { *count = need; return fail(FDFB_EINVAL, "buffer too small"); }
        std::memcpy(host, v[which]->data(), 4 * need);
        *count = need;
        return FDFB_OK;
    });
}

int fdfb_get_rotation_polys(const fdfb_ctx *cc, int32_t lut_id, int32_t *host)
{
    return guarded([&]() -> int {
        if (!cc || !host) return fail(FDFB_EINVAL, "null argument");
        fdfb_ctx *c = const_cast<fdfb_ctx *>(cc);  // the lock only
        Lock lk(c->mu);
        if (lut_id < 0 || lut_id >= c->nluts) return fail(FDFB_EINVAL, "unknown lut_id");
        const size_t per = 2 * (size_t)c->P.N;
        std::memcpy(host, &c->lut_polys[(size_t)lut_id * per], per * sizeof(int32_t));
        return FDFB_OK;
    });
}

int fdfb_profile(fdfb_ctx *c, int enable)
{
    return guarded([&]() -> int {
        if (!c) return fail(FDFB_EINVAL, "null context");
        Lock lk(c->mu);
        c->profiling = enable != 0;
        return FDFB_OK;
    });
}

int fdfb_profile_read(fdfb_ctx *c, double *ms, uint32_t *calls)
{
    return guarded([&]() -> int {
        if (!c || !ms || !calls) return fail(FDFB_EINVAL, "null argument");
        Lock lk(c->mu);
        const size_t per = FDFB_NPHASES + 1;
        for (int k = 0; k < FDFB_NPHASES; ++k) ms[k] = 0.0;
        *calls = (uint32_t)(c->prof_events.size() / per);
        int rc = FDFB_OK;
        for (size_t base = 0; base + per <= c->prof_events.size() && rc == FDFB_OK; base += per) {
            hipError_t e = hipEventSynchronize(c->prof_events[base + per - 1]);
            if (e != hipSuccess) { rc = fail(FDFB_EDEVICE, hipGetErrorString(e)); break; }
            for (int k = 0; k < FDFB_NPHASES; ++k) {
                float t = 0.f;
                e = hipEventElapsedTime(&t, c->prof_events[base + k], c->prof_events[base + k + 1]);
                if (e != hipSuccess) { rc = fail(FDFB_EDEVICE, hipGetErrorString(e)); break; }
                ms[k] += t;
            }
        }
        for (hipEvent_t e : c->prof_events) (void)hipEventDestroy(e);
        c->prof_events.clear();
        return rc;
    });
}

int fdfb_br_launches(fdfb_ctx *c, uint32_t A, uint32_t per_ct, uint32_t flags, uint32_t *launches)
{
    return guarded([&]() -> int {
        if (!c || !launches) return fail(FDFB_EINVAL, "null argument");
        if (per_ct == 0) return fail(FDFB_EINVAL, "per_ct must be at least 1");
        Lock lk(c->mu);
        int rc = check_form(*c, flags);
        if (rc) return rc;
        if ((rc = ensure_device(*c))) return rc;
        *launches = A ? 1 : 0;
        if (A && !(flags & (FDFB_PLAIN | FDFB_DIRECT)) && c->mfma_ok)
            K_TRY(fdfbk::br_kara_launches(c->geom, A, per_ct, tuned_plan(c->geom, A), launches));
        return FDFB_OK;
    });
}

int fdfb_device_errors(fdfb_ctx *c, int clear, uint32_t *bits)
{
    return guarded([&]() -> int {
        if (!c || !bits) return fail(FDFB_EINVAL, "null argument");
        Lock lk(c->mu);
        *bits = 0;
        if (!c->d_err) return FDFB_OK;
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipMemcpy(bits, c->d_err, sizeof(uint32_t), hipMemcpyDeviceToHost));
        if (clear && *bits) {
            const uint32_t zero = 0;
            HIP_TRY(hipMemcpy(c->d_err, &zero, sizeof(uint32_t), hipMemcpyHostToDevice));
        }
        return FDFB_OK;
    });
}

static_assert(FDFB_NOALLOC_SCRATCH_BYTES == fdfbk::kNoallocScratchBytes, "one size for the static scratch");

// Largest batch whose scratch fits the static buffer (scratch_bytes grows with B).
static uint32_t noalloc_max_batch(const fdfb_params &P)
{
    uint32_t lo = 0, hi = 1u << 24;
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo + 1) / 2;
        if (scratch_bytes(P, mid, 1) <= FDFB_NOALLOC_SCRATCH_BYTES) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

int fdfb_noalloc_max_batch(const fdfb_ctx *c, uint32_t *max_B)
{
    return guarded([&]() -> int {
        if (!c || !max_B) return fail(FDFB_EINVAL, "null argument");
        *max_B = noalloc_max_batch(c->P);
        return FDFB_OK;
    });
}

int fdfb_bootstrap_batch_noalloc(fdfb_ctx *c, const uint32_t *d_cts, const int32_t *d_lut_ids, uint32_t B,
                                 uint32_t *d_out, uint32_t flags, void *stream)
{
    return guarded([&]() -> int {
        if (!c) return fail(FDFB_EINVAL, "null context");
        if (B == 0) return c->abort_flag.load() ? fail(FDFB_EABORTED, "abort flag raised") : FDFB_OK;
        Lock lk(c->mu);
        if (int rc = check_batch(c, d_cts, d_lut_ids, d_out, flags)) return rc;
        const uint32_t maxB = noalloc_max_batch(c->P);
        if (B > maxB)
            return fail(FDFB_EINVAL, "batch of " + std::to_string(B) + " exceeds the static scratch (at most " +
                                         std::to_string(maxB) + " samples for this parameter set)");
        if (!device_ready(*c, flags))
            return fail(FDFB_EINVAL, "context not prepared for these flags: call fdfb_prepare (or one "
                                     "fdfb_bootstrap_batch) first");
        void *base = nullptr;
        K_TRY(fdfbk::noalloc_scratch(&base));
        const ScratchView sc = carve_scratch(c->P, B, 1, base);
        return enqueue_bootstrap(*c, sc, d_cts, d_lut_ids, B, d_out, flags, (hipStream_t)stream, 1, false);
    });
}

int fdfb_prepare(fdfb_ctx *c, uint32_t flags)
{
    return guarded([&]() -> int {
        if (!c) return fail(FDFB_EINVAL, "null context");
        if (flags & ~kAllFlags) return fail(FDFB_EINVAL, "unknown flag");
        Lock lk(c->mu);
        if (int rc = check_form(*c, flags)) return rc;
        return prepare(*c, flags);
    });
}

int fdfb_release_scratch(fdfb_ctx *c)
{
    return guarded([&]() -> int {
        if (!c) return fail(FDFB_EINVAL, "null context");
        Lock lk(c->mu);
        c->release_scratch();
        return FDFB_OK;
    });
}

int fdfb_measure_mfma_peak(double *tera_ops, double *ms)
{
    return guarded([&]() -> int {
        if (!tera_ops || !ms) return fail(FDFB_EINVAL, "null argument");
        uint32_t blocks = 0;
        K_TRY(fdfbk::mfma_stream_capacity(&blocks));
        const uint32_t iters = 32768;  // about 25 ms at 4.3 POPS with every wave slot filled
        int32_t *out = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        auto done = [&](int rc) {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            if (out) (void)hipFree(out);
            return rc;
        };
        hipError_t e = hipMalloc(&out, (size_t)blocks * 64 * sizeof(int32_t));
        if (e == hipSuccess) e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        if (e == hipSuccess) e = fdfbk::launch_mfma_stream(blocks, 256, out, nullptr);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
        if (e == hipSuccess) e = fdfbk::launch_mfma_stream(blocks, iters, out, nullptr);
        if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        if (e != hipSuccess)
            return done(fail(FDFB_EDEVICE, std::string("mfma calibration: ") + hipGetErrorString(e)));
        const double ops = (double)blocks * iters * fdfbk::mfma_stream_chains() * (16.0 * 16 * 64 * 2);
        *ms = t;
        *tera_ops = t > 0 ? ops / (t * 1e-3) / 1e12 : 0.0;
        return done(FDFB_OK);
    });
}

void fdfb_set_abort(fdfb_ctx *c, int raised)
{
    if (c) c->abort_flag.store(raised ? 1 : 0);
}

void fdfb_free(fdfb_ctx *c)
{
    if (!c) return;
    (void)guarded([&]() -> int {
        if (c->trace) {
            static const char *const names[FDFB_NPHASES] = {"modswitch_init", "sign_br",     "extract_bits",
                                                            "packing_ks",     "pubmux",      "function_br",
                                                            "output"};
            double ms[FDFB_NPHASES];
            uint32_t calls = 0;
            if (fdfb_profile_read(c, ms, &calls) == FDFB_OK && calls) {
                std::fprintf(stderr, "fdfb trace: %u bootstrap calls, ms per call:", calls);
                for (int k = 0; k < FDFB_NPHASES; ++k) std::fprintf(stderr, " %s %.3f", names[k], ms[k] / calls);
                std::fprintf(stderr, "\n");
            }
        }
        return FDFB_OK;
    });
    delete c;
}

}  // extern "C"
