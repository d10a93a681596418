/*
 * FDFB oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU implementation of full-domain functional
 * bootstrapping (Kluczniak & Schild, "FDFB: Full Domain Functional
 * Bootstrapping Towards Practical Fully Homomorphic Encryption",
 * arXiv 2109.02731) with ciphertext modulus q = Q = 2^32, so every ring
 * coefficient is a uint32_t and reduction mod q is the natural wrap of
 * unsigned arithmetic.  GLWE rank is 1 (RLWE).
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this file.  It shares no code, header, table or helper with the
 * GPU library; the two meet only in the seeded plaintext inputs and in the
 * counter-based generator below, which each side implements on its own from
 * the published SplitMix64 definition.
 *
 * Every function cites the passage of the paper it follows.  Where the paper
 * is silent or inconsistent the reading taken is stated at the function
 * (readings R1..R9, listed together in the design notes).
 *
 * Parity status: every function below is pinned by a CPU test against an
 * independent fact (brute force, closed form, exact identity or the
 * noise-free limit) except where a header says "parity unpinned".  The noise
 * is pinned separately, stage by stage: every key's noise deviation, and the
 * variance each stage of the bootstrap adds, against the error analysis of
 * Sec. 2 and Theorem "Correctness of the Bootstrapping", two-sided, with a
 * different deviation for each key; the failure probability of Sec. 4 is
 * pinned to Table II.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Parameters.  Same meaning as the library's, declared independently.       */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint32_t n, N, log2_t;
    uint32_t g_log2B, g_ell;     /* blind-rotation key gadget (L_RGSW)      */
    uint32_t ks_log2B, ks_ell;   /* LWE(N) -> LWE(n) key switching key      */
    uint32_t pk_log2B, pk_ell;   /* LWE(N) -> RLWE packing key              */
    uint32_t boot_log2B, boot_ell; /* public-mux digits (L_boot)            */
    double sigma_lwe, sigma_glwe, sigma_pk, sigma_ks;
} or_params;

static uint32_t ilog2u(uint32_t x) { uint32_t r = 0; while ((1u << r) < x) ++r; return r; }

/* ------------------------------------------------------------------------ */
/* Counter-based SplitMix64 (Steele, Lea & Flood 2014; the finaliser as in   */
/* Vigna's reference splitmix64.c).  Output #idx of the stream started at    */
/* state mix(seed + stream * gamma).  Not part of the paper: the paper leaves */
/* the sampler open, and bit-exact comparison needs one fixed definition.    */
/* ------------------------------------------------------------------------ */
#define OR_GAMMA 0x9E3779B97F4A7C15ull

static uint64_t or_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t or_draw(uint64_t seed, uint64_t stream, uint64_t idx)
{
    uint64_t s0 = or_mix64(seed + stream * OR_GAMMA);
    return or_mix64(s0 + (idx + 1) * OR_GAMMA);
}

/* Rounded Gaussian of standard deviation sigma (Box-Muller, first output). */
int64_t or_gauss(uint64_t seed, uint64_t stream, uint64_t idx, double sigma)
{
    if (sigma == 0.0) return 0;
    uint64_t r1 = or_draw(seed, stream, 2 * idx);
    uint64_t r2 = or_draw(seed, stream, 2 * idx + 1);
    double u1 = (double)((r1 >> 11) + 1) * (1.0 / 9007199254740992.0); /* (0,1] */
    double u2 = (double)(r2 >> 11) * (1.0 / 9007199254740992.0);       /* [0,1) */
    double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    return (int64_t)nearbyint(z * sigma);
}

/* Stream tags (domain separation of the randomness). */
enum { ST_S = 1, ST_SF = 2, ST_BRK_A = 3, ST_BRK_E = 4, ST_PK_A = 5, ST_PK_E = 6,
       ST_KS_A = 7, ST_KS_E = 8, ST_ENC_A = 9, ST_ENC_E = 10 };

static uint32_t draw_u32(uint64_t seed, uint64_t stream, uint64_t idx)
{
    return (uint32_t)(or_draw(seed, stream, idx) >> 32);
}
static uint32_t draw_bit(uint64_t seed, uint64_t stream, uint64_t idx)
{
    return (uint32_t)(or_draw(seed, stream, idx) >> 63);
}

/* ------------------------------------------------------------------------ */
/* Ring R_{N,q} = Z_q[X]/(X^N + 1), Sec. 2 "Notation".                       */
/* ------------------------------------------------------------------------ */

/* c = a * b in R_{N,q}: schoolbook product, then X^N = -1 folds the upper   */
/* half back with a sign flip.                                               */
void or_negacyclic_mul(const uint32_t *a, const uint32_t *b, uint32_t *c, uint32_t N)
{
    for (uint32_t m = 0; m < N; ++m) {
        uint32_t acc = 0;
        for (uint32_t p = 0; p <= m; ++p) acc += a[p] * b[m - p];
        for (uint32_t p = m + 1; p < N; ++p) acc -= a[p] * b[N + m - p];
        c[m] = acc;
    }
}

/* out = p * X^e, e in [0, 2N).  The monomials form a cyclic group of order  */
/* 2N with X^N = -1 (Sec. 1.2, "FHEW/TFHE Bootstrapping").                   */
void or_monomial_mul(const uint32_t *p, uint32_t e, uint32_t *out, uint32_t N)
{
    e %= 2 * N;
    for (uint32_t m = 0; m < N; ++m) {
        /* coefficient m of X^e * p collects p[j] with j + e == m (mod 2N) */
        uint32_t j = (m + 2 * N - e) % (2 * N);
        out[m] = (j < N) ? p[j] : (uint32_t)(0u - p[j - N]);
    }
}

/* Same for small signed integer polynomials (rotation polynomials). */
static void monomial_mul_i64(const int64_t *p, uint32_t e, int64_t *out, uint32_t N)
{
    e %= 2 * N;
    for (uint32_t m = 0; m < N; ++m) {
        uint32_t j = (m + 2 * N - e) % (2 * N);
        out[m] = (j < N) ? p[j] : -p[j - N];
    }
}

/* ------------------------------------------------------------------------ */
/* Decomposition, Sec. 2 Def. "Gadget Matrix" and Def. "Decomposition".      */
/* Reading R1 (approximate gadget): with ell*log2B < 32 the gadget is         */
/* g_j = 2^(32 - ell*log2B) * L^(j-1), j = 1..ell, and x is first rounded     */
/* (half up) to its top ell*log2B bits; with ell*log2B = 32 this is exactly   */
/* the paper's powers-of-L vector and unsigned digits in [0, L).             */
/* digits[j] for j = 0..ell-1 multiplies g_{j+1}.                           */
/* ------------------------------------------------------------------------ */
void or_decomp(uint32_t x, uint32_t log2B, uint32_t ell, uint32_t *digits)
{
    uint32_t drop = 32 - ell * log2B;
    uint32_t top = x;
    if (drop > 0) top = (uint32_t)(x + (1u << (drop - 1))) >> drop;
    uint32_t mask = (log2B == 32) ? 0xFFFFFFFFu : ((1u << log2B) - 1);
    for (uint32_t j = 0; j < ell; ++j) digits[j] = (top >> (log2B * j)) & mask;
}

uint32_t or_gadget(uint32_t log2B, uint32_t ell, uint32_t j)
{
    return 1u << (32 - ell * log2B + log2B * j);
}

/* ------------------------------------------------------------------------ */
/* Modulus switching, App. A Fig. "ModSwitch": x -> round(q' x / q), here     */
/* q = 2^32 and q' = 2^w.  Reading R2: ties round up.                         */
/* ------------------------------------------------------------------------ */
uint32_t or_modswitch(uint32_t x, uint32_t log2_qout)
{
    uint32_t sh = 32 - log2_qout;
    uint64_t v = ((uint64_t)x + (1ull << (sh - 1))) >> sh; /* round(x / 2^sh) */
    return (uint32_t)(v & ((1ull << log2_qout) - 1));      /* mod q'          */
}

/* ------------------------------------------------------------------------ */
/* Sample extraction, App. A Fig. "SampleExtract" with k = 1 (the constant   */
/* coefficient): b' = b_0, a'_0 = a_0, a'_j = -a_{N-j} for j >= 1, because   */
/* NSgn(0) = -1 (the source defines its >= as a strict >).  Reading R3.      */
/* out = [b', a'_0 .. a'_{N-1}].                                             */
/* ------------------------------------------------------------------------ */
void or_sample_extract(const uint32_t *rlwe /* [2][N], b first */, uint32_t N, uint32_t *out)
{
    const uint32_t *b = rlwe, *a = rlwe + N;
    out[0] = b[0];
    out[1] = a[0];
    for (uint32_t j = 1; j < N; ++j) out[1 + j] = (uint32_t)(0u - a[N - j]);
}

/* ------------------------------------------------------------------------ */
/* Key switching, App. A Fig. "KeySwitch":                                    */
/*   A = Decomp(a);  c_out = [b, 0] - sum_i sum_j A[i,j] * K[i,j].            */
/* K[i][j] is a GLWE sample stored flat in `out_len` words (for LWE targets   */
/* out_len = n'+1; for RLWE targets out_len = 2N with b-polynomial first).   */
/* ------------------------------------------------------------------------ */
void or_keyswitch(const uint32_t *ct, uint32_t din, const uint32_t *K, uint32_t log2B,
                  uint32_t ell, uint32_t out_len, uint32_t *out)
{
    uint32_t dig[32];
    memset(out, 0, sizeof(uint32_t) * out_len);
    out[0] = ct[0];
    for (uint32_t i = 0; i < din; ++i) {
        or_decomp(ct[1 + i], log2B, ell, dig);
        for (uint32_t j = 0; j < ell; ++j) {
            const uint32_t *row = K + ((size_t)i * ell + j) * out_len;
            for (uint32_t w = 0; w < out_len; ++w) out[w] -= dig[j] * row[w];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* External product, Sec. 2 Def. "External Product" and App. A:              */
/*   extProd(C, d) = Decomp(d^T) . C                                        */
/* C is an RGSW sample with 2*ell rows, row r = c*ell + j holding the GLWE   */
/* row [b, a] (2 polynomials), matching G = I_2 (x) g.                       */
/* ------------------------------------------------------------------------ */
void or_extprod(const uint32_t *C, const uint32_t *d /* [2][N] */, uint32_t N,
                uint32_t log2B, uint32_t ell, uint32_t *out /* [2][N] */)
{
    uint32_t *dig = (uint32_t *)malloc(sizeof(uint32_t) * N * ell);
    uint32_t *tmp = (uint32_t *)malloc(sizeof(uint32_t) * N);
    uint32_t dg[32];
    memset(out, 0, sizeof(uint32_t) * 2 * N);
    for (uint32_t c = 0; c < 2; ++c) {
        for (uint32_t m = 0; m < N; ++m) {
            or_decomp(d[c * N + m], log2B, ell, dg);
            for (uint32_t j = 0; j < ell; ++j) dig[j * N + m] = dg[j];
        }
        for (uint32_t j = 0; j < ell; ++j) {
            const uint32_t *row = C + (size_t)(c * ell + j) * 2 * N;
            for (uint32_t comp = 0; comp < 2; ++comp) {
                or_negacyclic_mul(dig + j * N, row + comp * N, tmp, N);
                for (uint32_t m = 0; m < N; ++m) out[comp * N + m] += tmp[m];
            }
        }
    }
    free(dig);
    free(tmp);
}

/* CMux, App. A Fig. "CMux gate": d = g - h; out = extProd(C, d) + h. */
void or_cmux(const uint32_t *C, const uint32_t *g, const uint32_t *h, uint32_t N,
             uint32_t log2B, uint32_t ell, uint32_t *out)
{
    uint32_t *d = (uint32_t *)malloc(sizeof(uint32_t) * 2 * N);
    for (uint32_t m = 0; m < 2 * N; ++m) d[m] = g[m] - h[m];
    or_extprod(C, d, N, log2B, ell, out);
    for (uint32_t m = 0; m < 2 * N; ++m) out[m] += h[m];
    free(d);
}

/* ------------------------------------------------------------------------ */
/* Blind rotation, App. A Fig. "Blind Rotation" with u = {1} (binary s):     */
/*   for i in [n]: acc <- CMux(brK[i], acc * X^(-a[i]), acc).                */
/* ctN = [b, a_1..a_n] in Z_{2N}; acc is updated in place.                   */
/* ------------------------------------------------------------------------ */
void or_blind_rotate(const or_params *P, const uint32_t *brk, const uint32_t *ctN, uint32_t *acc)
{
    uint32_t N = P->N, R = 2 * P->g_ell;
    uint32_t *g = (uint32_t *)malloc(sizeof(uint32_t) * 2 * N);
    uint32_t *o = (uint32_t *)malloc(sizeof(uint32_t) * 2 * N);
    for (uint32_t i = 0; i < P->n; ++i) {
        uint32_t e = (2 * N - ctN[1 + i] % (2 * N)) % (2 * N); /* X^{-a} = X^{2N-a} */
        or_monomial_mul(acc, e, g, N);
        or_monomial_mul(acc + N, e, g + N, N);
        or_cmux(brk + (size_t)i * R * 2 * N, g, acc, N, P->g_log2B, P->g_ell, o);
        memcpy(acc, o, sizeof(uint32_t) * 2 * N);
    }
    free(g);
    free(o);
}

/* ------------------------------------------------------------------------ */
/* Rotation polynomials, Sec. 3.3 (Theorem "rotation polynomial"; Fig. 2    */
/* builds them window by window).  The property they must have: for every   */
/* y in the window of m -- the y whose cyclic distance mod 2N from           */
/* round(2N/t) m is at most ceil(N/t) -- coefficient 0 of rotP_0 X^y         */
/* (y < N) or of rotP_1 X^y (y >= N) equals f(m).  Each y in [0, 2N) is     */
/* taken in turn: its owner m is found and the one coefficient that         */
/* coefficient 0 of the product reads is set; y in no window leaves it 0.   */
/* Reading R4: the table holds f(m) unscaled (the theorem states            */
/* coefficient = f(m)); the scale Delta is applied once, in PubMux.         */
/* Reading R5: neighbouring windows overlap at their ends; there the        */
/* larger m owns y (the construction's later write).                        */
/* ------------------------------------------------------------------------ */
void or_setup_polynomial(const uint32_t *lut, uint32_t t, uint32_t N, int32_t *p0, int32_t *p1)
{
    memset(p0, 0, sizeof(int32_t) * N);
    memset(p1, 0, sizeof(int32_t) * N);
    const int64_t w = (int64_t)((N + t - 1) / t);       /* ceil(N/t)    */
    const int64_t step = (int64_t)((2 * N + t / 2) / t); /* round(2N/t)  */
    const int64_t twoN = 2 * (int64_t)N;
    for (int64_t y = 0; y < twoN; ++y) {
        int64_t owner = -1;
        for (int64_t m = (int64_t)t - 1; m >= 0 && owner < 0; --m) {
            const int64_t d = ((y - step * m) % twoN + twoN) % twoN;
            if (d <= w || d >= twoN - w) owner = m;      /* cyclic distance <= w */
        }
        if (owner < 0) continue;
        const int32_t v = (int32_t)lut[owner];
        /* coefficient 0 of X^y p: p_0 for y = 0, -p_{N-y} for 0 < y < N     */
        /* (X^N = -1); for y >= N, X^y p = -X^(y-N) p                         */
        if (y < (int64_t)N) {
            if (y == 0) p0[0] = v;
            else p0[N - y] = -v;
        } else {
            const int64_t z = y - N;
            if (z == 0) p1[0] = -v;
            else p1[N - z] = v;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Key generation.                                                           */
/*  * s in {0,1}^n and the RLWE key 𝔰 in {0,1}^N (reading R6: both binary); */
/*    s_F = KeyExtract(𝔰) = Coefs(𝔰) (Sec. 2 Def. "Sample Extraction").    */
/*  * GLWE sample of mu: [a*𝔰 + e + mu, a] (Sec. 2 Def. "Generalized LWE").  */
/*  * brK[i] = RGSW(𝔰, s[i]) (App. A Fig. "BRKeyGen", u = {1}); RGSW rows are */
/*    GLWE(0) + s[i] * G with G = I_2 (x) g (Def. "Generalized-GSW Sample"). */
/*  * pK[i][j] = RLWE(𝔰, s_F[i] g_j), ksK[i][j] = LWE(s, s_F[i] g_j)          */
/*    (App. A Fig. "KeySwitchSetup"; Theorem "Correctness of the            */
/*    Bootstrapping" fixes which keys are switched).                         */
/* Layouts: brk[n][2*g_ell][2][N]; pk[N][pk_ell][2][N]; ksk[N][ks_ell][n+1]. */
/* ------------------------------------------------------------------------ */
static void glwe_zero(const or_params *P, const uint32_t *sf, uint64_t seed, uint64_t sa,
                      uint64_t se, uint64_t base, double sigma, uint32_t *out, uint32_t *tmp)
{
    uint32_t N = P->N;
    uint32_t *b = out, *a = out + N;
    for (uint32_t p = 0; p < N; ++p) a[p] = draw_u32(seed, sa, base * N + p);
    or_negacyclic_mul(a, sf, tmp, N);
    for (uint32_t p = 0; p < N; ++p)
        b[p] = tmp[p] + (uint32_t)or_gauss(seed, se, base * N + p, sigma);
}

void or_keygen(const or_params *P, uint64_t seed, uint32_t *s, uint32_t *sf, uint32_t *brk,
               uint32_t *pk, uint32_t *ksk)
{
    uint32_t n = P->n, N = P->N;
    uint32_t *tmp = (uint32_t *)malloc(sizeof(uint32_t) * N);
    for (uint32_t i = 0; i < n; ++i) s[i] = draw_bit(seed, ST_S, i);
    for (uint32_t p = 0; p < N; ++p) sf[p] = draw_bit(seed, ST_SF, p);

    uint32_t R = 2 * P->g_ell;
    for (uint32_t i = 0; i < n; ++i)
        for (uint32_t r = 0; r < R; ++r) {
            uint32_t *row = brk + ((size_t)i * R + r) * 2 * N;
            glwe_zero(P, sf, seed, ST_BRK_A, ST_BRK_E, (uint64_t)i * R + r, P->sigma_glwe, row, tmp);
            uint32_t c = r / P->g_ell, j = r % P->g_ell;
            row[c * N] += s[i] * or_gadget(P->g_log2B, P->g_ell, j);
        }

    for (uint32_t i = 0; i < N; ++i)
        for (uint32_t j = 0; j < P->pk_ell; ++j) {
            uint32_t *row = pk + ((size_t)i * P->pk_ell + j) * 2 * N;
            glwe_zero(P, sf, seed, ST_PK_A, ST_PK_E, (uint64_t)i * P->pk_ell + j, P->sigma_pk, row, tmp);
            row[0] += sf[i] * or_gadget(P->pk_log2B, P->pk_ell, j);
        }

    for (uint32_t i = 0; i < N; ++i)
        for (uint32_t j = 0; j < P->ks_ell; ++j) {
            uint64_t idx = (uint64_t)i * P->ks_ell + j;
            uint32_t *row = ksk + idx * (n + 1);
            uint32_t dot = 0;
            for (uint32_t q = 0; q < n; ++q) {
                row[1 + q] = draw_u32(seed, ST_KS_A, idx * n + q);
                dot += row[1 + q] * s[q];
            }
            row[0] = dot + (uint32_t)or_gauss(seed, ST_KS_E, idx, P->sigma_ks)
                   + sf[i] * or_gadget(P->ks_log2B, P->ks_ell, j);
        }
    free(tmp);
}

/* ------------------------------------------------------------------------ */
/* Regev encryption / decryption (Sec. 1.2 "Regev Encryption", Sec. 2        */
/* Def. "Phase and Error"): b = <a,s> + Delta*m + e, m = round(t*phase/q).   */
/* ------------------------------------------------------------------------ */
void or_encrypt(const or_params *P, const uint32_t *s, uint32_t m, uint64_t seed, uint64_t index,
                uint32_t *ct)
{
    uint32_t n = P->n, dot = 0;
    for (uint32_t q = 0; q < n; ++q) {
        ct[1 + q] = draw_u32(seed, ST_ENC_A, index * n + q);
        dot += ct[1 + q] * s[q];
    }
    uint32_t delta = 1u << (32 - P->log2_t);
    ct[0] = dot + delta * m + (uint32_t)or_gauss(seed, ST_ENC_E, index, P->sigma_lwe);
}

uint32_t or_phase(const uint32_t *ct, const uint32_t *key, uint32_t dim)
{
    uint32_t ph = ct[0];
    for (uint32_t q = 0; q < dim; ++q) ph -= ct[1 + q] * key[q];
    return ph;
}

uint32_t or_decrypt(const uint32_t *ct, const uint32_t *key, uint32_t dim, uint32_t log2_t,
                    int64_t *err)
{
    uint32_t ph = or_phase(ct, key, dim);
    uint32_t sh = 32 - log2_t;
    uint32_t m = (uint32_t)(((uint64_t)ph + (1ull << (sh - 1))) >> sh) & ((1u << log2_t) - 1);
    if (err) *err = (int64_t)(int32_t)(ph - (m << sh));
    return m;
}

/* ------------------------------------------------------------------------ */
/* Public mux, Sec. 3.1 Fig. 1 "PubMux":                                     */
/*   p = p_1 - p_0;  digits of p;  c_out = [Delta p_0, 0] + sum_i p[i] c_i.  */
/* Reading R7: Delta * t = 0 mod 2^32, so only p mod t matters; the digits   */
/* are the unsigned base-L_boot digits of (p mod t), ell_boot = ceil(log_L t)*/
/* of them (boot_ell).                                                       */
/* Variant (boot_log2B = 0, boot_ell = 1): one signed digit, the centred     */
/* representative of (p mod t) in [-t/2, t/2); Delta * t = 0 mod 2^32 keeps  */
/* the plaintext Delta * p_bit, with one sign rotation instead of ell_boot.  */
/* c: ell_boot RLWE samples [2][N]; p0, p1 small signed polynomials.         */
/* ------------------------------------------------------------------------ */
void or_pubmux(const or_params *P, const uint32_t *c, const int64_t *p0, const int64_t *p1,
               uint32_t *out)
{
    uint32_t N = P->N, t = 1u << P->log2_t, delta = 1u << (32 - P->log2_t);
    uint32_t L = 1u << P->boot_log2B;
    uint32_t *dig = (uint32_t *)malloc(sizeof(uint32_t) * N);
    uint32_t *tmp = (uint32_t *)malloc(sizeof(uint32_t) * N);
    for (uint32_t m = 0; m < N; ++m) {
        out[m] = delta * (uint32_t)p0[m];
        out[N + m] = 0;
    }
    for (uint32_t i = 0; i < P->boot_ell; ++i) {
        uint32_t Li = 1;
        for (uint32_t k = 0; k < i; ++k) Li *= L;
        for (uint32_t m = 0; m < N; ++m) {
            int64_t p = p1[m] - p0[m];
            uint64_t pm = (uint64_t)(((p % (int64_t)t) + (int64_t)t) % (int64_t)t);
            if (P->boot_log2B == 0) {
                int64_t cen = (int64_t)pm >= (int64_t)(t / 2) ? (int64_t)pm - (int64_t)t : (int64_t)pm;
                dig[m] = (uint32_t)cen; /* two's complement, mod 2^32 */
            } else {
                dig[m] = (uint32_t)((pm / Li) % L);
            }
        }
        for (uint32_t comp = 0; comp < 2; ++comp) {
            or_negacyclic_mul(dig, c + ((size_t)i * 2 + comp) * N, tmp, N);
            for (uint32_t m = 0; m < N; ++m) out[comp * N + m] += tmp[m];
        }
    }
    free(dig);
    free(tmp);
}

/* ------------------------------------------------------------------------ */
/* Full domain functional bootstrapping, Sec. 3.2 Fig. 2 "Bootstrap", with:  */
/*  * sgnP = 1 - sum_{i=2}^{N} X^{i-1};                                      */
/*  * Delta = Delta_{Q,t} = 2^32 / t;                                        */
/*  * Reading R8 (selection): the sign rotation yields bit = 1 exactly when  */
/*    the phase lies in [0, N), and there the function rotation must use    */
/*    rotP_0 (Theorem "Correctness of the Bootstrapping" and Theorem         */
/*    "rotation polynomial"); PubMux returns p_bit, so it is called with     */
/*    (p_0, p_1) := (rotP_1 X^b, rotP_0 X^b).                               */
/*  * ell_boot sign rotations as in reading R7.                             */
/*  * Q = q, so the final ModSwitch(Q -> q) is the identity.                */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint32_t *ctN;       /* [n+1]            */
    uint32_t *acc_sign;  /* [ell_boot][2][N] after the sign rotations      */
    uint32_t *c_bits;    /* [ell_boot][N+1]  extracted sign samples        */
    uint32_t *r_bits;    /* [ell_boot][2][N] after LWE -> RLWE switching   */
    uint32_t *acc_f;     /* [2][N]           built accumulator             */
    uint32_t *acc_f_br;  /* [2][N]           after the function rotation   */
    uint32_t *c_q;       /* [N+1]            extracted output under s_F    */
} or_dumps;

#define OR_OUT_EXTRACTED 1u

void or_fdfb(const or_params *P, const uint32_t *brk, const uint32_t *pk, const uint32_t *ksk,
             const int32_t *rotP0, const int32_t *rotP1, const uint32_t *ct, uint32_t flags,
             uint32_t *out, or_dumps *dump)
{
    uint32_t n = P->n, N = P->N, ellb = P->boot_ell;
    uint32_t log2_2N = ilog2u(2 * N);
    uint32_t delta = 1u << (32 - P->log2_t);
    uint32_t half = delta >> 1;
    uint32_t L = 1u << P->boot_log2B;

    uint32_t *ctN = (uint32_t *)malloc(sizeof(uint32_t) * (n + 1));
    for (uint32_t q = 0; q <= n; ++q) ctN[q] = or_modswitch(ct[q], log2_2N);
    uint32_t bN = ctN[0];

    uint32_t *sgn = (uint32_t *)malloc(sizeof(uint32_t) * N);
    uint32_t *sgnb = (uint32_t *)malloc(sizeof(uint32_t) * N);
    sgn[0] = 1;
    for (uint32_t p = 1; p < N; ++p) sgn[p] = 0xFFFFFFFFu; /* -1 */
    or_monomial_mul(sgn, bN, sgnb, N);

    uint32_t *acc = (uint32_t *)malloc(sizeof(uint32_t) * 2 * N);
    uint32_t *cb = (uint32_t *)malloc(sizeof(uint32_t) * ellb * (N + 1));
    uint32_t *rb = (uint32_t *)malloc(sizeof(uint32_t) * ellb * 2 * N);
    uint32_t scale = half;
    for (uint32_t i = 0; i < ellb; ++i) {
        for (uint32_t m = 0; m < N; ++m) {
            acc[m] = scale * sgnb[m];
            acc[N + m] = 0;
        }
        or_blind_rotate(P, brk, ctN, acc);
        if (dump && dump->acc_sign) memcpy(dump->acc_sign + (size_t)i * 2 * N, acc, 8 * (size_t)N);
        uint32_t *ci = cb + (size_t)i * (N + 1);
        or_sample_extract(acc, N, ci);
        ci[0] += scale;
        scale *= L;
    }

    /* BuildAcc (Fig. 1): switch every bit sample to RLWE, then PubMux. */
    for (uint32_t i = 0; i < ellb; ++i)
        or_keyswitch(cb + (size_t)i * (N + 1), N, pk, P->pk_log2B, P->pk_ell, 2 * N,
                     rb + (size_t)i * 2 * N);

    int64_t *r0 = (int64_t *)malloc(sizeof(int64_t) * N), *r1 = (int64_t *)malloc(sizeof(int64_t) * N);
    int64_t *pA = (int64_t *)malloc(sizeof(int64_t) * N), *pB = (int64_t *)malloc(sizeof(int64_t) * N);
    for (uint32_t m = 0; m < N; ++m) { r0[m] = rotP0[m]; r1[m] = rotP1[m]; }
    monomial_mul_i64(r1, bN, pA, N); /* rotP'_1 */
    monomial_mul_i64(r0, bN, pB, N); /* rotP'_0 */
    or_pubmux(P, rb, pA, pB, acc);
    if (dump && dump->acc_f) memcpy(dump->acc_f, acc, 8 * (size_t)N);

    or_blind_rotate(P, brk, ctN, acc);
    if (dump && dump->acc_f_br) memcpy(dump->acc_f_br, acc, 8 * (size_t)N);

    uint32_t *cq = (uint32_t *)malloc(sizeof(uint32_t) * (N + 1));
    or_sample_extract(acc, N, cq);
    if (dump && dump->c_q) memcpy(dump->c_q, cq, 4 * (size_t)(N + 1));
    if (flags & OR_OUT_EXTRACTED) memcpy(out, cq, 4 * (size_t)(N + 1));
    else or_keyswitch(cq, N, ksk, P->ks_log2B, P->ks_ell, n + 1, out);

    if (dump) {
        if (dump->ctN) memcpy(dump->ctN, ctN, 4 * (size_t)(n + 1));
        if (dump->c_bits) memcpy(dump->c_bits, cb, 4 * (size_t)ellb * (N + 1));
        if (dump->r_bits) memcpy(dump->r_bits, rb, 4 * (size_t)ellb * 2 * N);
    }
    free(ctN); free(sgn); free(sgnb); free(acc); free(cb); free(rb);
    free(r0); free(r1); free(pA); free(pB); free(cq);
}

/* ------------------------------------------------------------------------ */
/* TFHE-style (half domain) bootstrap, App. A Fig. "TFHE Bootstrapping":     */
/* one rotation of [rotP * X^b, 0] (rotP already scaled), extract, switch.   */
/* ------------------------------------------------------------------------ */
void or_tfhe_bootstrap(const or_params *P, const uint32_t *brk, const uint32_t *ksk,
                       const uint32_t *rotP /* scaled, [N] */, const uint32_t *ct, uint32_t flags,
                       uint32_t *out)
{
    uint32_t n = P->n, N = P->N;
    uint32_t *ctN = (uint32_t *)malloc(sizeof(uint32_t) * (n + 1));
    for (uint32_t q = 0; q <= n; ++q) ctN[q] = or_modswitch(ct[q], ilog2u(2 * N));
    uint32_t *acc = (uint32_t *)calloc(2 * N, sizeof(uint32_t));
    or_monomial_mul(rotP, ctN[0], acc, N);
    or_blind_rotate(P, brk, ctN, acc);
    uint32_t *cq = (uint32_t *)malloc(sizeof(uint32_t) * (N + 1));
    or_sample_extract(acc, N, cq);
    if (flags & OR_OUT_EXTRACTED) memcpy(out, cq, 4 * (size_t)(N + 1));
    else or_keyswitch(cq, N, ksk, P->ks_log2B, P->ks_ell, n + 1, out);
    free(ctN); free(acc); free(cq);
}

/* ------------------------------------------------------------------------ */
/* Affine map on LWE samples, Sec. 2 Lemma "Linear Homomorphism of GLWE     */
/* samples" with scalar weights: out[r] = sum_c W[r][c] * ct[c] (mod 2^32).  */
/* ------------------------------------------------------------------------ */
void or_affine(const int32_t *W, uint32_t rows, uint32_t cols, const uint32_t *cts, uint32_t width,
               uint32_t *out)
{
    for (uint32_t r = 0; r < rows; ++r) {
        uint32_t *o = out + (size_t)r * width;
        memset(o, 0, 4 * (size_t)width);
        for (uint32_t c = 0; c < cols; ++c) {
            uint32_t w = (uint32_t)W[(size_t)r * cols + c];
            const uint32_t *x = cts + (size_t)c * width;
            for (uint32_t k = 0; k < width; ++k) o[k] += w * x[k];
        }
    }
}
