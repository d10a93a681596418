// HIP kernels of the FDFB path for gfx950 (MI355X).
//
// Arithmetic is exact: every ring coefficient is a uint32_t and wraps mod
// 2^32 (q = Q = 2^32).  The blind rotation has three forms that give
// identical bits:
//  * Karatsuba (default): k_br_kara1w (N <= 1024, one wavefront per
//    accumulator), k_br_kara1w2 (N = 1024, rounds that put two wavefronts on
//    every SIMD) and k_br_kara (N = 2048, two wavefronts per output
//    component).  Each external product splits the ring into even and odd
//    halves and computes three half-size Toeplitz contractions on int8 MFMA
//    (16x16x64) with 8-bit key limbs and int32 accumulation, recombined mod
//    2^32;
//  * k_br_mfma -- the direct form: one full-size contraction per digit row;
//  * k_br_plain -- one accumulator per workgroup, uint32 multiply-add on the
//    vector ALUs (the comparison form).
// Key switching (k_keyswitch_mfma), the public mux (k_pubmux) and the
// element-wise steps complete the bootstrap.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "kernels.h"

namespace fdfbk {

typedef int v4i __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// ModSwitch(x, 2^32 -> 2N) = round(2N x / 2^32) mod 2N, ties up
// (App. A Fig. "ModSwitch").
// ---------------------------------------------------------------------------
__global__ void k_modswitch(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                            uint32_t total, uint32_t sh, uint32_t mask)
{
    uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x < total) out[x] = ((in[x] + (1u << (sh - 1))) >> sh) & mask;
}

// ---------------------------------------------------------------------------
// Sign accumulators (Fig. 2 "Bootstrap", sign phase):
// acc_{b,i} = [L_boot^i (Delta/2) sgnP X^{b_N}, 0], sgnP = 1 - X - ... - X^{N-1}.
// ---------------------------------------------------------------------------
__global__ void k_init_sign(const uint32_t *__restrict__ ctN, uint32_t *__restrict__ acc,
                            uint32_t B, int n, int N, int ellb, uint32_t half, uint32_t Lb)
{
    const uint32_t a = blockIdx.y;  // accumulator index b * ellb + i
    const uint32_t b = a / ellb, i = a % ellb;
    uint32_t scale = half;
    for (uint32_t k = 0; k < i; ++k) scale *= Lb;
    const uint32_t e = ctN[(size_t)b * (n + 1)];
    uint32_t *row = acc + (size_t)a * 2 * N;
    for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < N; m += gridDim.x * blockDim.x) {
        // coefficient m of sgnP * X^e collects sgnP[j], j = m - e (mod 2N)
        uint32_t j = (uint32_t)(m + 2 * N - (int)e) % (2 * N);
        int32_t v = (j < (uint32_t)N) ? (j == 0 ? 1 : -1) : (j == (uint32_t)N ? -1 : 1);
        row[m] = scale * (uint32_t)v;
        row[N + m] = 0;
    }
}

// ---------------------------------------------------------------------------
// SampleExtract(acc, 1) (App. A Fig. "SampleExtract"): b' = b_0,
// a'_0 = a_0, a'_j = -a_{N-j}; optionally + add_base L_boot^(a mod per) on b'.
// ---------------------------------------------------------------------------
__global__ void k_extract(const uint32_t *__restrict__ acc, uint32_t *__restrict__ lwe, int N,
                          uint32_t per, uint32_t add_base, uint32_t Lb)
{
    const uint32_t a = blockIdx.y;
    const uint32_t *row = acc + (size_t)a * 2 * N;
    uint32_t *o = lwe + (size_t)a * (N + 1);
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j <= N; j += gridDim.x * blockDim.x) {
        uint32_t v;
        if (j == 0) {
            uint32_t add = 0;
            if (add_base) {
                add = add_base;
                for (uint32_t k = 0; k < a % per; ++k) add *= Lb;
            }
            v = row[0] + add;
        } else if (j == 1) {
            v = row[N];
        } else {
            v = 0u - row[N + (N - (j - 1))];
        }
        o[j] = v;
    }
}

// ---------------------------------------------------------------------------
// Key switching (App. A Fig. "KeySwitch"), LWE(din) -> GLWE flattened to
// out_len words:  out = [b, 0, ...] - sum_i sum_j Decomp(a_i)_j K[i][j].
// Workgroup: KS_TB samples x 256 output words.  The samples' digits of one
// chunk of input coordinates are staged in LDS (16 bits each: bases up to
// 2^16); each key word is read once per workgroup and used for all KS_TB
// samples.
// ---------------------------------------------------------------------------
constexpr int KS_TB = 16;
constexpr int KS_CHUNK = 128;

__global__ __launch_bounds__(256) void k_keyswitch(const uint32_t *__restrict__ in, uint32_t B,
                                                   uint32_t din, const uint32_t *__restrict__ key,
                                                   int log2B, int ell, uint32_t out_len,
                                                   uint32_t *__restrict__ out)
{
    __shared__ uint16_t dig[KS_CHUNK * 8 * KS_TB];  // [coord][j][sample], ell <= 8
    const uint32_t w = blockIdx.x * 256 + threadIdx.x;
    const uint32_t b0 = blockIdx.y * KS_TB;
    const uint32_t drop = 32 - ell * log2B;
    const uint32_t mask = (1u << log2B) - 1;
    uint32_t acc[KS_TB];
#pragma unroll
    for (int c = 0; c < KS_TB; ++c) acc[c] = 0;

    for (uint32_t i0 = 0; i0 < din; i0 += KS_CHUNK) {
        const uint32_t cnt = min((uint32_t)KS_CHUNK, din - i0);
        __syncthreads();
        for (uint32_t x = threadIdx.x; x < cnt * KS_TB; x += 256) {
            const uint32_t ii = x / KS_TB, c = x % KS_TB;
            const uint32_t b = b0 + c;
            uint32_t v = (b < B) ? in[(size_t)b * (din + 1) + 1 + i0 + ii] : 0u;
            uint32_t top = drop ? (v + (1u << (drop - 1))) >> drop : v;
            for (int j = 0; j < ell; ++j) dig[(ii * 8 + j) * KS_TB + c] = (top >> (log2B * j)) & mask;
        }
        __syncthreads();
        if (w < out_len) {
            for (uint32_t ii = 0; ii < cnt; ++ii) {
                for (int j = 0; j < ell; ++j) {
                    const uint32_t k = key[((size_t)(i0 + ii) * ell + j) * out_len + w];
                    const uint16_t *dg = dig + (ii * 8 + j) * KS_TB;
#pragma unroll
                    for (int c = 0; c < KS_TB; ++c) acc[c] += (uint32_t)dg[c] * k;
                }
            }
        }
    }
    if (w < out_len) {
#pragma unroll
        for (int c = 0; c < KS_TB; ++c) {
            const uint32_t b = b0 + c;
            if (b < B) {
                uint32_t init = (w == 0) ? in[(size_t)b * (din + 1)] : 0u;
                out[(size_t)b * out_len + w] = init - acc[c];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Key switching on int8 MFMA: the same sum as k_keyswitch as a GEMM
//   C[b][(w, l)] = sum_k dig[b][k] * limb_l(K[k][w]),  k = j * din + i
// (digit j of input coordinate i), with the key split into balanced byte
// limbs and stored as lane-ordered 1 KB B fragments per (k-block, 4 words).
// Workgroup: 64 samples x 64 output words; wavefront w takes words
// [16 w, 16 w + 16) for all 64 samples (4 x 4 MFMA tiles).  Digits of a
// 64-coordinate chunk are staged in LDS as bytes; int32 sums are exact
// (din ell 15 128 < 2^31) and limbs recombine mod 2^32 by DPP quad sums.
// ---------------------------------------------------------------------------
template <int ELL>
__global__ __launch_bounds__(256) void k_keyswitch_mfma(const uint32_t *__restrict__ in, uint32_t B,
                                                        uint32_t din, const v4i *__restrict__ kfrag,
                                                        int log2B, uint32_t out_len, uint32_t wtiles,
                                                        uint32_t *__restrict__ out)
{
    constexpr int ROW = 80;  // bytes per staged sample row (64 digits + pad, conflict-free reads)
    __shared__ __attribute__((aligned(16))) uint8_t dig[ELL][64][ROW];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t s0 = blockIdx.y * 64;
    const uint32_t wt0 = blockIdx.x * 16 + wv * 4;  // first 4-word tile of this wavefront
    const uint32_t drop = 32 - ELL * log2B;
    const uint32_t dmask = (1u << log2B) - 1;
    const int ri = lane & 15, g = lane >> 4;
    v4i C[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) C[a][b] = v4i{0, 0, 0, 0};

    for (uint32_t c0 = 0; c0 < din; c0 += 64) {
        v4i Bf[ELL][4];
#pragma unroll
        for (int j = 0; j < ELL; ++j) {
            const uint32_t kb = (j * din + c0) / 64;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) Bf[j][nt] = kfrag[((size_t)kb * wtiles + wt0 + nt) * 64 + lane];
        }
        __syncthreads();  // the previous chunk's digits are no longer read
        for (int task = threadIdx.x; task < 64 * 16; task += 256) {
            const uint32_t sl = task >> 4, cq = (task & 15) * 4;
            const uint32_t b = s0 + sl;
            uint32_t x[4] = {0, 0, 0, 0};
            if (b < B) {
                const uint32_t *src = in + (size_t)b * (din + 1) + 1 + c0 + cq;
                x[0] = src[0]; x[1] = src[1]; x[2] = src[2]; x[3] = src[3];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) x[u] = drop ? (x[u] + (1u << (drop - 1))) >> drop : x[u];
            if (b >= B) x[0] = x[1] = x[2] = x[3] = 0;
#pragma unroll
            for (int j = 0; j < ELL; ++j) {
                const uint32_t sh = log2B * j;
                const uint32_t w = ((x[0] >> sh) & dmask) | (((x[1] >> sh) & dmask) << 8) |
                                   (((x[2] >> sh) & dmask) << 16) | (((x[3] >> sh) & dmask) << 24);
                *(uint32_t *)&dig[j][sl][cq] = w;
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < ELL; ++j) {
            v4i Af[4];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) Af[mt] = *(const v4i *)&dig[j][mt * 16 + ri][16 * g];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
                    C[mt][nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(Af[mt], Bf[j][nt], C[mt][nt], 0, 0, 0);
        }
    }
    // recombine limbs: column = (word within tile, limb); rows = samples
    const int limb = lane & 3, wq = (lane >> 2) & 3;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int x = (int)((uint32_t)C[mt][nt][v] << (8 * limb));
                x += __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false);
                x += __builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, false);
                const uint32_t b = s0 + mt * 16 + 4 * g + v;
                const uint32_t w = (wt0 + nt) * 4 + wq;
                if (limb == 0 && b < B && w < out_len) {
                    const uint32_t init = (w == 0) ? in[(size_t)b * (din + 1)] : 0u;
                    out[(size_t)b * out_len + w] = init - (uint32_t)x;
                }
            }
}

// ---------------------------------------------------------------------------
// Affine map on LWE samples (Sec. 2 Lemma "Linear Homomorphism of GLWE
// samples" with scalar weights): out[r] = sum_c W[r][c] in[c] (mod 2^32),
// every coordinate of the samples at once.  Workgroup: AF_ROWS output rows x
// 256 words; each input word is read once per workgroup.
// ---------------------------------------------------------------------------
constexpr int AF_ROWS = 8;

__global__ __launch_bounds__(256) void k_affine(const int32_t *__restrict__ W, const uint32_t *__restrict__ in,
                                                uint32_t rows, uint32_t cols, uint32_t width,
                                                uint32_t *__restrict__ out)
{
    const uint32_t k = blockIdx.x * 256 + threadIdx.x;
    const uint32_t r0 = blockIdx.y * AF_ROWS;
    if (k >= width) return;
    uint32_t acc[AF_ROWS];
#pragma unroll
    for (int r = 0; r < AF_ROWS; ++r) acc[r] = 0;
    for (uint32_t c = 0; c < cols; ++c) {
        const uint32_t x = in[(size_t)c * width + k];
#pragma unroll
        for (int r = 0; r < AF_ROWS; ++r)
            if (r0 + r < rows) acc[r] += (uint32_t)W[(size_t)(r0 + r) * cols + c] * x;
    }
#pragma unroll
    for (int r = 0; r < AF_ROWS; ++r)
        if (r0 + r < rows) out[(size_t)(r0 + r) * width + k] = acc[r];
}

// Two-term linear combination of LWE samples (the same Lemma): out = wx x + wy y,
// word by word; x and y may be the same buffer.
__global__ __launch_bounds__(256) void k_lincomb2(const uint32_t *__restrict__ x, const uint32_t *__restrict__ y,
                                                  uint32_t wx, uint32_t wy, uint32_t count,
                                                  uint32_t *__restrict__ out)
{
    const uint32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k < count) out[k] = wx * x[k] + wy * y[k];
}

// ---------------------------------------------------------------------------
// PubMux of the bootstrap (Sec. 3.1 Fig. 1 with the selection of Fig. 2):
//   p_A = rotP_1 X^{b_N}, p_B = rotP_0 X^{b_N}, delta = (p_B - p_A) mod t,
//   acc = [Delta p_A, 0] + sum_i digit_i(delta) * R_i.
// One workgroup per sample; digits stored as a signed negacyclic extension
// so that every product term is a plain read.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_pubmux(const uint32_t *__restrict__ rlwe,
                                                const uint32_t *__restrict__ ctN,
                                                const int32_t *__restrict__ lut_ids,
                                                const int32_t *__restrict__ luts, int nluts,
                                                uint32_t *__restrict__ err, uint32_t *__restrict__ acc, int n,
                                                int N, int log2_t, int boot_log2B, int ellb, uint32_t per)
{
    extern __shared__ uint8_t smem[];
    int8_t *dx = (int8_t *)smem;                              // [ellb][2N]
    uint32_t *pa = (uint32_t *)(smem + ((ellb * 2 * N + 15) & ~15));  // [N] Delta * p_A
    const uint32_t eidx = blockIdx.x;  // table evaluation: sample eidx / per, its own table
    const uint32_t b = eidx / per;
    const int id = lut_ids[eidx];
    uint32_t *o = acc + (size_t)eidx * 2 * N;
    if (id < 0 || id >= nluts) {  // unknown table: all-zero output, reported in *err
        if (threadIdx.x == 0) atomicOr(err, 1u);
        for (int m = threadIdx.x; m < 2 * N; m += blockDim.x) o[m] = 0;
        return;
    }
    const int32_t *r0 = luts + (size_t)id * 2 * N, *r1 = r0 + N;
    const uint32_t e = ctN[(size_t)b * (n + 1)];
    const int t = 1 << log2_t;
    const uint32_t delta = 1u << (32 - log2_t);
    for (int m = threadIdx.x; m < N; m += blockDim.x) {
        uint32_t j = (uint32_t)(m + 2 * N - (int)e) % (2 * N);
        int32_t va = (j < (uint32_t)N) ? r1[j] : -r1[j - N];
        int32_t vb = (j < (uint32_t)N) ? r0[j] : -r0[j - N];
        int32_t p = (vb - va) % t;
        if (p < 0) p += t;
        for (int i = 0; i < ellb; ++i) {
            // unsigned base-L_boot digits, or (boot_log2B = 0) one centred digit
            int32_t d = boot_log2B ? (p >> (boot_log2B * i)) & ((1 << boot_log2B) - 1) : (p >= t / 2 ? p - t : p);
            dx[i * 2 * N + N + m] = (int8_t)d;   // position m
            dx[i * 2 * N + m] = (int8_t)(-d);    // position m - N
        }
        pa[m] = delta * (uint32_t)va;
    }
    __syncthreads();
    const uint32_t *R = rlwe + (size_t)b * ellb * 2 * N;
    for (int m = threadIdx.x; m < N; m += blockDim.x) {
        // each product digit x word mod 2^32 as digit x low half + (digit x high half) << 16:
        // the digits and the 16-bit halves fit the full-rate signed 24-bit multiplier, and
        // the two sums recombine exactly mod 2^32
        uint32_t lo0 = 0, hi0 = 0, lo1 = 0, hi1 = 0;
        for (int i = 0; i < ellb; ++i) {
            const int8_t *d = dx + i * 2 * N + N + m;  // d[-p] = digit at m - p
            const uint32_t *rb = R + (size_t)i * 2 * N, *ra = rb + N;
#pragma unroll 16
            for (int p = 0; p < N; ++p) {
                const int dv = d[-p];
                const uint32_t wb = rb[p], wa = ra[p];
                lo0 += (uint32_t)__mul24(dv, (int)(wb & 0xFFFFu));
                hi0 += (uint32_t)__mul24(dv, (int)(wb >> 16));
                lo1 += (uint32_t)__mul24(dv, (int)(wa & 0xFFFFu));
                hi1 += (uint32_t)__mul24(dv, (int)(wa >> 16));
            }
        }
        o[m] = pa[m] + lo0 + (hi0 << 16);
        o[N + m] = lo1 + (hi1 << 16);
    }
}

// ---------------------------------------------------------------------------
// TFHE-style accumulator (App. A Fig. "TFHE Bootstrapping"): [Delta rotP_0
// X^{b_N}, 0] for the table of each sample (zero for an unknown table).
// ---------------------------------------------------------------------------
__global__ void k_init_tfhe(const uint32_t *__restrict__ ctN, const int32_t *__restrict__ lut_ids,
                            const int32_t *__restrict__ luts, int nluts, uint32_t *__restrict__ err,
                            uint32_t *__restrict__ acc, int n, int N, int log2_t)
{
    const uint32_t b = blockIdx.y;
    const int id = lut_ids[b];
    if ((id < 0 || id >= nluts) && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(err, 1u);
    const uint32_t e = ctN[(size_t)b * (n + 1)];
    const uint32_t delta = 1u << (32 - log2_t);
    uint32_t *row = acc + (size_t)b * 2 * N;
    for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < N; m += gridDim.x * blockDim.x) {
        uint32_t v = 0;
        if (id >= 0 && id < nluts) {
            const int32_t *r0 = luts + (size_t)id * 2 * N;
            const uint32_t j = (uint32_t)(m + 2 * N - (int)e) % (2 * N);  // coefficient m of X^e r0
            v = delta * (uint32_t)((j < (uint32_t)N) ? r0[j] : -r0[j - N]);
        }
        row[m] = v;
        row[N + m] = 0;
    }
}

// ---------------------------------------------------------------------------
// Plain blind rotation (App. A Fig. "Blind Rotation"): one accumulator per
// workgroup, schoolbook uint32 negacyclic products on the vector ALUs.
// LDS: accumulator [2][N] u32, digits as signed extension [R][2N] int16,
// key of the current iteration [R][2][N] u32.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_br_plain(uint32_t *__restrict__ acc_g,
                                                  const uint32_t *__restrict__ ctN,
                                                  uint32_t accs_per_ct, int n, int N, int log2B,
                                                  int ell, const uint32_t *__restrict__ brk)
{
    extern __shared__ uint8_t smem[];
    const int R = 2 * ell;
    uint32_t *accL = (uint32_t *)smem;                   // [2][N]
    uint32_t *keyL = accL + 2 * N;                       // [R][2][N]
    int16_t *dx = (int16_t *)(keyL + (size_t)R * 2 * N);  // [R][2N]
    const uint32_t a_idx = blockIdx.x;
    uint32_t *row = acc_g + (size_t)a_idx * 2 * N;
    const uint32_t *crow = ctN + (size_t)(a_idx / accs_per_ct) * (n + 1) + 1;
    const uint32_t drop = 32 - ell * log2B;
    const uint32_t mask = (1u << log2B) - 1;
    for (int x = threadIdx.x; x < 2 * N; x += blockDim.x) accL[x] = row[x];
    for (int i = 0; i < n; ++i) {
        const uint32_t a = crow[i];
        if (a == 0) continue;  // X^0: the CMux adds extProd(C, 0) = 0
        __syncthreads();
        const uint32_t *kg = brk + (size_t)i * R * 2 * N;
        for (int x = threadIdx.x; x < R * 2 * N; x += blockDim.x) keyL[x] = kg[x];
        for (int x = threadIdx.x; x < 2 * N; x += blockDim.x) {
            const int c = x / N, m = x % N;
            // coefficient m of X^{-a} acc_c is acc_c[m + a] with sign flips
            uint32_t e = (uint32_t)m + a;
            uint32_t v = (e < (uint32_t)N) ? accL[c * N + e]
                         : (e < 2u * N) ? 0u - accL[c * N + e - N] : accL[c * N + e - 2 * N];
            uint32_t diff = v - accL[c * N + m];
            uint32_t top = drop ? (diff + (1u << (drop - 1))) >> drop : diff;
            for (int j = 0; j < ell; ++j) {
                int16_t d = (int16_t)((top >> (log2B * j)) & mask);
                dx[(c * ell + j) * 2 * N + N + m] = d;
                dx[(c * ell + j) * 2 * N + m] = (int16_t)(-d);
            }
        }
        __syncthreads();
        for (int x = threadIdx.x; x < N; x += blockDim.x) {
            uint32_t o0 = 0, o1 = 0;
            for (int r = 0; r < R; ++r) {
                const int16_t *d = dx + r * 2 * N + N + x;  // d[-p]: digit at x - p
                const uint32_t *k0 = keyL + (size_t)r * 2 * N, *k1 = k0 + N;
                for (int p = 0; p < N; ++p) {
                    const uint32_t dv = (uint32_t)(int32_t)d[-p];
                    o0 += dv * k0[p];
                    o1 += dv * k1[p];
                }
            }
            accL[x] += o0;
            accL[N + x] += o1;
        }
    }
    __syncthreads();
    for (int x = threadIdx.x; x < 2 * N; x += blockDim.x) row[x] = accL[x];
}

// ---------------------------------------------------------------------------
// Batched blind rotation on int8 MFMA, direct form (FDFB_DIRECT; the default
// is the Karatsuba form k_br_kara below).
//
// One workgroup owns one accumulator for the whole loop over i (the CMux
// chain is sequential in i, independent across accumulators); its
// wavefronts produce output component j (b or a), one wavefront per
// component for N <= 1024 and two (each half of the output rows) for
// N = 2048, where key fragments also stream in chunks of 16 k-blocks.  For one
// CMux the external product out_j = sum_r D_r * K_{r,j} (negacyclic) is a
// GEMM over the digit rows r:
//   C[m][col] = sum_p T(D_r)[m][p] * Bk[p][col],  T(D)[m][p] = D~[m - p]
// where D~ is the negacyclic extension of the digit polynomial
// (D~[x - N] = -D[x]) and the 16 columns are col = s*4 + l:
//   s in 0..3   key shifted by 16 s, so one A tile of 16 rows yields 64 rows,
//   l in 0..3   balanced signed byte limb of the 32-bit key word.
// B fragments come from key byte planes built on the host (per (i, r, j) one
// plane per limb of the negacyclic extension; lane (s, l, g) reads 16
// aligned bytes of plane l) and are double-buffered in registers: the next
// unit's fragments are in flight while the current unit runs.  A fragments are windows of a
// reversed copy of D~ in LDS, aligned per lane with v_alignbyte; a Toeplitz
// fragment depends only on the diagonal m0 - p0, so each one is built once
// per diagonal and used for every tile on it.  Each wavefront writes the
// digits of its own component; digit sets alternate between iterations so a
// single barrier per CMux orders writers and readers.  int32 accumulation is
// exact (|sum| < 2 ell CH N 127 128 < 2^31) and limbs are recombined mod 2^32
// with DPP quad sums.
// ---------------------------------------------------------------------------
template <int N, int ELL, int CH>
struct BrMfma {
    static constexpr int RPC = ELL * CH;             // virtual digit rows per component
    static constexpr int RV = 2 * RPC;               // virtual digit rows per CMux
    static constexpr int WPC = N > 1024 ? 2 : 1;     // wavefronts per output component
    static constexpr int WAVES = 2 * WPC;
    static constexpr int NT = N / 64 / WPC;          // 64-row output tiles per wavefront
    static constexpr int NKB = N / 64;               // k-blocks of 64 per digit row
    static constexpr int KC = NKB < 16 ? NKB : 16;   // k-blocks per key chunk
    static constexpr int NCH = NKB / KC;             // key chunks per digit row
    static constexpr int UNITS = RV * NCH;           // (row, chunk) units per CMux
    static constexpr int DLOC = 64 * (NT - 1);       // largest local diagonal
    static constexpr int NDIAG = NT + KC - 1;        // local diagonals per unit
    static constexpr int DIG_WORDS = N / 2;          // one digit row: 2N bytes
    static constexpr size_t LDS_BYTES = 4 * (2 * (size_t)N + 2 * (size_t)RV * DIG_WORDS);
    static constexpr int PLV = (N + 64) / 16;        // one key limb plane, in 16-byte units
};

template <int N, int ELL, int CH>
__global__ __launch_bounds__(256, 2) void k_br_mfma(uint32_t *__restrict__ acc_g,
                                                    const uint32_t *__restrict__ ctN,
                                                    uint32_t accs_per_ct, int n,
                                                    const v4i *__restrict__ bfrag, int log2B)
{
    using G = BrMfma<N, ELL, CH>;
    extern __shared__ uint8_t smem[];
    uint32_t *accL = (uint32_t *)smem;                  // [2][N]
    uint32_t *digL = accL + 2 * N;                      // [2 sets][RV][DIG_WORDS]
    auto dig = [&](int set, int r) { return digL + (set * G::RV + r) * G::DIG_WORDS; };

    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int jc = wv / G::WPC;                          // output component of this wavefront
    const int hw = wv % G::WPC;                          // its half of the tiles / coefficients
    const uint32_t a_idx = blockIdx.x;
    uint32_t *row = acc_g + (size_t)a_idx * 2 * N;
    for (int x = threadIdx.x; x < 2 * N; x += 64 * G::WAVES) accL[x] = row[x];
    const uint32_t *crow = ctN + (size_t)(a_idx / accs_per_ct) * (n + 1) + 1;

    const uint32_t drop = 32 - ELL * log2B;
    // A-fragment addressing: lane (i = lane%16, g = lane/16) of the fragment on
    // diagonal d reads bytes Rv[N-1-d-i+16g .. +15] of the reversed extension
    // Rv[z] = D~[N-1-z]: 5 aligned words, shifted by sh = (3 - i) mod 4.
    const int ri = lane & 15, g = lane >> 4;
    const int sh = (3 - ri) & 3;
    const int S0 = N - 1 - ri + 16 * g;
    // recombination: this lane's output column (shift s, limb l)
    const int limb = lane & 3, ss = (lane >> 2) & 3;
    // B fragments of unit u = (row, chunk) for this wavefront's component:
    // lane (s, l, g) reads 16 bytes of limb plane l at 64 kb + 16 (g + s)
    const int lane_v = (lane & 3) * G::PLV + (lane >> 4) + ((lane >> 2) & 3);
    auto frag = [&](int i, int u) {
        const int r = u / G::NCH, c = u % G::NCH;
        return bfrag + ((size_t)(i * G::RV + r) * 2 + jc) * 4 * G::PLV + lane_v + c * G::KC * 4;
    };
    auto next_live = [&](int i) {
        int k = i + 1;
        while (k < n && __builtin_amdgcn_readfirstlane(crow[k]) == 0) ++k;
        return k;
    };

    int i = next_live(-1);
    v4i B0[G::KC], B1[G::KC];
    {
        const v4i *bp = frag(i < n ? i : 0, 0);
#pragma unroll
        for (int kb = 0; kb < G::KC; ++kb) B0[kb] = bp[kb * 4];
    }
    int set = 0;
    __syncthreads();
    while (i < n) {
        const uint32_t a = __builtin_amdgcn_readfirstlane(crow[i]);
        const int inext = next_live(i);

        // digits of (X^{-a} acc_j - acc_j), written reversed and extended.
        // Coefficient m of X^{-a} acc is acc[(m + a) mod N], negated when
        // (m + a) mod 2N lies in [N, 2N).  Lane q handles m = 4q..4q+3: the
        // four rotated words come from two aligned quads of acc (conflict-free
        // 16-byte reads) and a wave-uniform shift rho = a mod 4 picks them.
        {
            const uint32_t rho = a & 3, qa0 = a >> 2;
            const uint4 *acc4 = (const uint4 *)&accL[jc * N];
#pragma unroll
            for (int qq = 0; qq < N / 256 / G::WPC; ++qq) {
                const uint32_t q = lane + 64 * (qq + hw * (N / 256 / G::WPC));
                const uint32_t Qa = (q + qa0) & (N / 2 - 1), Qb = (Qa + 1) & (N / 2 - 1);
                const uint4 A4 = acc4[Qa & (N / 4 - 1)], B4 = acc4[Qb & (N / 4 - 1)];
                const uint4 O4 = acc4[q];
                const uint32_t sa = (Qa & (N / 4)) ? 0xFFFFFFFFu : 0u;
                const uint32_t sb = (Qb & (N / 4)) ? 0xFFFFFFFFu : 0u;
                uint32_t w[8] = {(A4.x ^ sa) - sa, (A4.y ^ sa) - sa, (A4.z ^ sa) - sa, (A4.w ^ sa) - sa,
                                 (B4.x ^ sb) - sb, (B4.y ^ sb) - sb, (B4.z ^ sb) - sb, (B4.w ^ sb) - sb};
                uint32_t rot[4];
                switch (rho) {  // wave-uniform
                case 0: rot[0] = w[0]; rot[1] = w[1]; rot[2] = w[2]; rot[3] = w[3]; break;
                case 1: rot[0] = w[1]; rot[1] = w[2]; rot[2] = w[3]; rot[3] = w[4]; break;
                case 2: rot[0] = w[2]; rot[1] = w[3]; rot[2] = w[4]; rot[3] = w[5]; break;
                default: rot[0] = w[3]; rot[1] = w[4]; rot[2] = w[5]; rot[3] = w[6]; break;
                }
                const uint32_t own[4] = {O4.x, O4.y, O4.z, O4.w};
                uint32_t top[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint32_t diff = rot[u] - own[u];
                    top[u] = drop ? (diff + (1u << (drop - 1))) >> drop : diff;
                }
#pragma unroll
                for (int jj = 0; jj < ELL; ++jj) {
#pragma unroll
                    for (int h = 0; h < CH; ++h) {
                        const uint32_t off = log2B * jj + 7 * h;
                        const uint32_t wdt = (7 * (h + 1) <= log2B) ? 7u : (uint32_t)log2B - 7 * h;
                        // bytes in memory order: coefficient 4q+3 first (reversed layout)
                        uint32_t pos = __builtin_amdgcn_ubfe(top[3], off, wdt);
                        pos |= __builtin_amdgcn_ubfe(top[2], off, wdt) << 8;
                        pos |= __builtin_amdgcn_ubfe(top[1], off, wdt) << 16;
                        pos |= __builtin_amdgcn_ubfe(top[0], off, wdt) << 24;
                        // bytewise 0 - x for x in [0, 127], no carries between bytes
                        const uint32_t neg = (0x80808080u - pos) ^ 0x80808080u;
                        uint32_t *rv = dig(set, jc * G::RPC + jj * CH + h);
                        rv[N / 4 - q - 1] = pos;
                        rv[N / 2 - q - 1] = neg;
                    }
                }
            }
        }
        __syncthreads();

        v4i C[G::NT];
#pragma unroll
        for (int t = 0; t < G::NT; ++t) C[t] = v4i{0, 0, 0, 0};

        auto one_unit = [&](const int u, v4i(&Bc)[G::KC], v4i(&Bn)[G::KC]) {
            // prefetch the next unit (or the next live iteration's first unit);
            // the scheduling barrier keeps the loads here, a full unit ahead
            const v4i *np = (u + 1 < G::UNITS) ? frag(i, u + 1) : frag(inext < n ? inext : i, 0);
#pragma unroll
            for (int kb = 0; kb < G::KC; ++kb) Bn[kb] = np[kb * 4];
            __builtin_amdgcn_sched_barrier(0);
            // Toeplitz fragments, one per diagonal, ping-ponged: the words of
            // diagonal dd+1 are read and aligned while diagonal dd's MFMAs run.
            // Local diagonal dl = 64 (alpha' - kb') maps to d = dl + 64 (hw NT - c KC).
            const int r = u / G::NCH, c = u % G::NCH;
            const int dshift = 64 * (hw * G::NT - c * G::KC);
            const uint32_t *ab = dig(set, r) + (S0 - dshift - sh - G::DLOC) / 4;
            v4i Af[2];
            uint32_t wn[5];
            auto read_words = [&](const int dd, uint32_t(&w)[5]) {
                const uint32_t *wp = ab + 16 * dd;  // (DLOC - dl) / 4
#pragma unroll
                for (int k = 0; k < 5; ++k) w[k] = wp[k];
            };
            auto align = [&](const uint32_t(&w)[5], v4i &A) {
#pragma unroll
                for (int k = 0; k < 4; ++k) A[k] = (int)__builtin_amdgcn_alignbyte(w[k + 1], w[k], sh);
            };
            read_words(0, wn);
            align(wn, Af[0]);
#pragma unroll
            for (int dd = 0; dd < G::NDIAG; ++dd) {
                const int dl = G::DLOC - 64 * dd;
                if (dd + 1 < G::NDIAG) read_words(dd + 1, wn);
#pragma unroll
                for (int kb = 0; kb < G::KC; ++kb) {
                    const int m0 = dl + 64 * kb;  // local tile row
                    if (m0 >= 0 && m0 <= 64 * (G::NT - 1))
                        C[m0 / 64] = __builtin_amdgcn_mfma_i32_16x16x64_i8(Af[dd & 1], Bc[kb], C[m0 / 64], 0, 0, 0);
                }
                if (dd + 1 < G::NDIAG) align(wn, Af[(dd + 1) & 1]);
            }
        };
        // units in pairs so the two fragment register sets alternate statically
#pragma unroll 1
        for (int u = 0; u < G::UNITS; u += 2) {
            one_unit(u, B0, B1);
            one_unit(u + 1, B1, B0);
        }

        // limbs -> uint32 (mod 2^32): sum_l C_l << 8l over the lane quad
#pragma unroll
        for (int t = 0; t < G::NT; ++t) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int x = (int)((uint32_t)C[t][v] << (8 * limb));
                x += __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false);  // quad xor 1
                x += __builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, false);  // quad xor 2
                if (limb == 0) {
                    const int m = 64 * (hw * G::NT + t) + 16 * ss + 4 * g + v;
                    accL[jc * N + m] += (uint32_t)x;
                }
            }
        }
        if (G::WPC > 1) __syncthreads();  // both halves of acc_j feed the next digits
        set ^= 1;
        i = inext;
    }
    __syncthreads();
    for (int x = threadIdx.x; x < 2 * N; x += 64 * G::WAVES) row[x] = accL[x];
}

// ---------------------------------------------------------------------------
// Blind rotation with one level of Karatsuba over the even/odd split.
// With Y = X^2 (Y^(N/2) = -1) a polynomial is a = a_e(Y) + X a_o(Y), and
//   (a b)_e = a_e b_e + Y a_o b_o
//   (a b)_o = (a_e + a_o)(b_e + b_o) - a_e b_e - a_o b_o,
// three negacyclic products of size M = N/2 instead of four quarter-size
// blocks of the full product.  The digit operand of the middle product is
// a_e + a_o, which must fit int8: 7-bit digits are offset to V_e = D_e - 64
// and V_o = D_o - 63 (V_e, V_o, V_e + V_o and their negations all lie in
// [-127, 127]), and sum_r O_r * K_r, the product of the offset polynomials
// with the key rows, is added back each step from a table built with the
// key.  Narrower digit chunks need no offset.  The three products
// accumulate in three register sets over all digit rows; the accumulator
// is kept in LDS in even/odd order, where X^(-a) acts on each half as a
// negacyclic rotation of size M (and swaps the halves for odd a).
// Each product is the Toeplitz GEMM of k_br_mfma at size M (A fragments
// built once per diagonal, 16 B columns = 4 key shifts x 4 balanced limbs,
// units of 8 k-blocks with the next unit's B fragments in flight), with one
// change of tiling: output row i of a tile at m0 is coefficient
// m0 - 1 + 4i + s for key shift s in {0, 1, 2, 3}, which makes every lane's
// 16 A bytes start on a dword (four LDS words, no byte alignment) and puts
// the shifts in the lane-ordered B fragments built on the host.
// ---------------------------------------------------------------------------
template <int V> struct IC { static constexpr int value = V; };
template <int I, int END> struct StaticFor {
    template <class F> __device__ __attribute__((always_inline)) static void run(F &&f)
    {
        f(IC<I>{});
        StaticFor<I + 1, END>::run(f);
    }
};
template <int END> struct StaticFor<END, END> {
    template <class F> __device__ __attribute__((always_inline)) static void run(F &&) {}
};

// WPC_: wavefronts per output component (by default 1 up to N = 1024, 2 above;
// 4 at N = 2048 for the split form of small rounds)
template <int N, int ELL, int CH, int WPC_ = (N > 1024 ? 2 : 1)>
struct BrKara {
    static constexpr int M = N / 2;                   // size of the half rings
    static constexpr int RPC = ELL * CH;              // virtual digit rows per component
    static constexpr int RV = 2 * RPC;                // virtual digit rows per CMux
    static constexpr int WPC = WPC_;                  // wavefronts per output component
    static constexpr int WAVES = 2 * WPC;
    static constexpr int NT = M / 64 / WPC;           // output tiles per wavefront and product
    static constexpr int NKB = M / 64;                // k-blocks per product
    static constexpr int KC = NKB < 8 ? NKB : 8;      // k-blocks per key chunk
    static constexpr int NCH = NKB / KC;              // key chunks per product
    static constexpr int UPR = 3 * NCH;               // units per digit row
    static constexpr int RSTEP = (UPR % 2) ? 2 : 1;   // rows per loop step (even unit count)
    static constexpr int USTEP = RSTEP * UPR;
    static constexpr int DLOC = 64 * (NT - 1);        // largest local diagonal
    static constexpr int NDIAG = NT + KC - 1;         // local diagonals per unit
    static constexpr int SEQ_WORDS = M / 2;           // one reversed extension: 2M bytes
    static constexpr int DSETS = 1;                   // one digit set: a barrier follows the accumulate
    static constexpr size_t LDS_BYTES = 4 * (2 * (size_t)N + (size_t)DSETS * RV * 3 * SEQ_WORDS);
    // k_br_kara1w2: rows of V_e and V_o only (V_e + V_o overwrites V_e after P_e)
    static constexpr size_t LDS2W_BYTES = 4 * (2 * (size_t)N + (size_t)RV * 2 * SEQ_WORDS);
    static constexpr int QPW = M / 4 / WPC;           // coefficient quads per wavefront and half
    static_assert(RV % RSTEP == 0 && USTEP % 2 == 0, "unit sequence must alternate evenly");
};

// Four consecutive coefficients 4q..4q+3 of rot_beta(src) in R_M:
// rot_beta(p)[m] = p[(m + beta) mod M], negated when (m + beta) mod 2M >= M.
template <int M>
__device__ __attribute__((always_inline)) inline void kara_rot4(const uint4 *src, uint32_t q, uint32_t beta,
                                                                 uint32_t (&rot)[4])
{
    const uint32_t rho = beta & 3, qa0 = beta >> 2;
    const uint32_t Qa = (q + qa0) & (M / 2 - 1), Qb = (Qa + 1) & (M / 2 - 1);
    const uint4 A4 = src[Qa & (M / 4 - 1)], B4 = src[Qb & (M / 4 - 1)];
    const uint32_t sa = (Qa & (M / 4)) ? 0xFFFFFFFFu : 0u;
    const uint32_t sb = (Qb & (M / 4)) ? 0xFFFFFFFFu : 0u;
    const uint32_t w[8] = {(A4.x ^ sa) - sa, (A4.y ^ sa) - sa, (A4.z ^ sa) - sa, (A4.w ^ sa) - sa,
                           (B4.x ^ sb) - sb, (B4.y ^ sb) - sb, (B4.z ^ sb) - sb, (B4.w ^ sb) - sb};
    switch (rho) {  // wave-uniform
    case 0: rot[0] = w[0]; rot[1] = w[1]; rot[2] = w[2]; rot[3] = w[3]; break;
    case 1: rot[0] = w[1]; rot[1] = w[2]; rot[2] = w[3]; rot[3] = w[4]; break;
    case 2: rot[0] = w[2]; rot[1] = w[3]; rot[2] = w[4]; rot[3] = w[5]; break;
    default: rot[0] = w[3]; rot[1] = w[4]; rot[2] = w[5]; rot[3] = w[6]; break;
    }
}

// One accumulator (row, 2N words) rotated by the whole workgroup (64 WAVES
// threads), its ModSwitched coefficients a_1..a_n at crow; LDS at smem.
template <int N, int ELL, int CH, int WPC = BrKara<N, ELL, CH>::WPC>
__device__ __attribute__((always_inline)) inline void br_kara_run(uint8_t *smem, uint32_t *__restrict__ row,
                                                                 const uint32_t *__restrict__ crow, int n,
                                                                 const v4i *__restrict__ bfrag,
                                                                 const uint32_t *__restrict__ corr, int log2B)
{
    using G = BrKara<N, ELL, CH, WPC>;
    constexpr int M = G::M;
    uint32_t *accL = (uint32_t *)smem;  // [2][N]: per component, even half then odd half
    uint32_t *digL = accL + 2 * N;      // [DSETS][RV][3 products][SEQ_WORDS]
    auto seq = [&](int set, int r, int p) { return digL + ((set * G::RV + r) * 3 + p) * G::SEQ_WORDS; };

    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int jc = wv / G::WPC;  // output component of this wavefront
    const int hw = wv % G::WPC;  // its half of the tiles / coefficients
    for (int x = threadIdx.x; x < 2 * N; x += 64 * G::WAVES) {
        const int m = x & (N - 1);
        accL[(x & ~(N - 1)) + (m & 1) * M + (m >> 1)] = row[x];
    }
    const uint32_t drop = 32 - ELL * log2B;

    // Output row i of a tile starting at m0, for key shift s, is coefficient
    // m0 - 1 + 4 i + s, so lane (i, g) of the A fragment on diagonal d reads
    // bytes Rv[M - d - 4i + 16g ..+15] of the reversed extension
    // Rv[z] = V~[M - 1 - z]: four dword-aligned LDS words, no byte shifts.
    const int ri = lane & 15, g = lane >> 4;
    const int S0 = M - 4 * ri + 16 * g;
    const int limb = lane & 3, ss = (lane >> 2) & 3;
    auto frag = [&](int i, int r, int p, int c) {
        return bfrag + (((((size_t)i * G::RV + r) * 3 + p) * 2 + jc) * G::NKB + c * G::KC) * 64 + lane;
    };
    auto next_live = [&](int i) {
        int k = i + 1;
        while (k < n && __builtin_amdgcn_readfirstlane(crow[k]) == 0) ++k;
        return k;
    };

    int i = next_live(-1);
    v4i B0[G::KC], B1[G::KC];
    {
        const v4i *bp = frag(i < n ? i : 0, 0, 0, 0);
#pragma unroll
        for (int kb = 0; kb < G::KC; ++kb) B0[kb] = bp[kb * 64];
    }
    int set = 0;
    __syncthreads();
    while (i < n) {
        const uint32_t a = __builtin_amdgcn_readfirstlane(crow[i]);
        const int inext = next_live(i);

        // digits of (X^{-a} acc_j - acc_j) for both halves; per digit row the
        // sequences V_e, V_o and V_e + V_o, each as a reversed negacyclic
        // extension of size M (bytes in memory order: coefficient 4q+3 first).
        {
            const uint32_t al = a >> 1, odd_a = a & 1;
            const uint32_t *accJ = accL + jc * N;
            const uint4 *srcE = (const uint4 *)(accJ + (odd_a ? M : 0));
            const uint4 *srcO = (const uint4 *)(accJ + (odd_a ? 0 : M));
            const uint4 *ownE = (const uint4 *)accJ, *ownO = (const uint4 *)(accJ + M);
#pragma unroll
            for (int qq = 0; qq < (G::QPW + 63) / 64; ++qq) {
                if (G::QPW % 64 != 0 && qq * 64 + lane >= G::QPW) break;
                const uint32_t q = hw * G::QPW + qq * 64 + lane;
                uint32_t rE[4], rO[4];
                kara_rot4<M>(srcE, q, al, rE);
                kara_rot4<M>(srcO, q, al + odd_a, rO);
                const uint4 E4 = ownE[q], O4 = ownO[q];
                const uint32_t oE[4] = {E4.x, E4.y, E4.z, E4.w}, oO[4] = {O4.x, O4.y, O4.z, O4.w};
                uint32_t tE[4], tO[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint32_t dE = rE[u] - oE[u], dO = rO[u] - oO[u];
                    tE[u] = drop ? (dE + (1u << (drop - 1))) >> drop : dE;
                    tO[u] = drop ? (dO + (1u << (drop - 1))) >> drop : dO;
                }
#pragma unroll
                for (int jj = 0; jj < ELL; ++jj) {
#pragma unroll
                    for (int h = 0; h < CH; ++h) {
                        const uint32_t off = log2B * jj + 7 * h;
                        const bool full = 7 * (h + 1) <= log2B;
                        const uint32_t wdt = full ? 7u : (uint32_t)log2B - 7 * h;
                        // byte constants: offsets (64, 63) for 7-bit digits, none otherwise
                        const uint32_t oe = full ? 64u : 0u, oo = full ? 63u : 0u;
                        const uint32_t cE = (128u - oe) * 0x01010101u, nE = (128u + oe) * 0x01010101u;
                        const uint32_t cO = (128u - oo) * 0x01010101u, nO = (128u + oo) * 0x01010101u;
                        const uint32_t cS = (128u - oe - oo) * 0x01010101u, nS = (128u + oe + oo) * 0x01010101u;
                        uint32_t pe = __builtin_amdgcn_ubfe(tE[3], off, wdt);
                        pe |= __builtin_amdgcn_ubfe(tE[2], off, wdt) << 8;
                        pe |= __builtin_amdgcn_ubfe(tE[1], off, wdt) << 16;
                        pe |= __builtin_amdgcn_ubfe(tE[0], off, wdt) << 24;
                        uint32_t po = __builtin_amdgcn_ubfe(tO[3], off, wdt);
                        po |= __builtin_amdgcn_ubfe(tO[2], off, wdt) << 8;
                        po |= __builtin_amdgcn_ubfe(tO[1], off, wdt) << 16;
                        po |= __builtin_amdgcn_ubfe(tO[0], off, wdt) << 24;
                        const uint32_t ps = pe + po;  // bytes <= 254, no carries
                        // bytewise x - o and o - x: (x + 128 - o) ^ 0x80, (128 + o - x) ^ 0x80
                        const int r = jc * G::RPC + jj * CH + h;
                        uint32_t *sE = seq(set, r, 0), *sO = seq(set, r, 1), *sS = seq(set, r, 2);
                        sE[M / 4 - q - 1] = (pe + cE) ^ 0x80808080u;
                        sE[M / 2 - q - 1] = (nE - pe) ^ 0x80808080u;
                        sO[M / 4 - q - 1] = (po + cO) ^ 0x80808080u;
                        sO[M / 2 - q - 1] = (nO - po) ^ 0x80808080u;
                        sS[M / 4 - q - 1] = (ps + cS) ^ 0x80808080u;
                        sS[M / 2 - q - 1] = (nS - ps) ^ 0x80808080u;
                    }
                }
            }
        }
        __syncthreads();

        // the offset correction of this step, for the coefficients this lane accumulates
        uint32_t wE[G::NT], wO[G::NT];
        {
            const uint32_t *cp = corr + ((size_t)i * 2 + jc) * N;
#pragma unroll
            for (int t = 0; t < G::NT; ++t) {
                const int m = (64 * (hw * G::NT + t) + 16 * g + 4 * limb + ss - 1) & (M - 1);
                wE[t] = cp[m];
                wO[t] = cp[M + m];
            }
        }

        v4i C[3][G::NT];
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int t = 0; t < G::NT; ++t) C[p][t] = v4i{0, 0, 0, 0};

        auto one_unit = [&](const int r, auto P_, const int c, v4i(&Bc)[G::KC], v4i(&Bn)[G::KC],
                            const v4i *np) {
            constexpr int p = decltype(P_)::value;
#pragma unroll
            for (int kb = 0; kb < G::KC; ++kb) Bn[kb] = np[kb * 64];
            __builtin_amdgcn_sched_barrier(0);
            // local diagonal dl = 64 (t - kb) is global d = dl + dshift
            const int dshift = 64 * (hw * G::NT - c * G::KC);
            // dword-aligned, not 16-byte aligned: read as four dwords
            const uint32_t *ab = seq(set, r, p) + (S0 - dshift - G::DLOC) / 4;
            auto afrag = [&](const int dd, v4i &A) {
#pragma unroll
                for (int k = 0; k < 4; ++k) A[k] = (int)ab[16 * dd + k];
            };
            v4i Af[2];
            afrag(0, Af[0]);
#pragma unroll
            for (int dd = 0; dd < G::NDIAG; ++dd) {
                const int dl = G::DLOC - 64 * dd;
                if (dd + 1 < G::NDIAG) afrag(dd + 1, Af[(dd + 1) & 1]);
#pragma unroll
                for (int kb = 0; kb < G::KC; ++kb) {
                    const int m0 = dl + 64 * kb;
                    if (m0 >= 0 && m0 <= 64 * (G::NT - 1))
                        C[p][m0 / 64] =
                            __builtin_amdgcn_mfma_i32_16x16x64_i8(Af[dd & 1], Bc[kb], C[p][m0 / 64], 0, 0, 0);
                }
            }
        };

#pragma unroll 1
        for (int r = 0; r < G::RV; r += G::RSTEP) {
            StaticFor<0, G::USTEP>::run([&](auto U_) {
                constexpr int u = decltype(U_)::value;
                constexpr int rr = u / G::UPR, p = (u % G::UPR) / G::NCH, c = u % G::NCH;
                const v4i *np;
                if constexpr (u + 1 < G::USTEP) {
                    constexpr int u2 = u + 1;
                    np = frag(i, r + u2 / G::UPR, (u2 % G::UPR) / G::NCH, u2 % G::NCH);
                } else {
                    np = (r + G::RSTEP < G::RV) ? frag(i, r + G::RSTEP, 0, 0)
                                                : frag(inext < n ? inext : i, 0, 0, 0);
                }
                if constexpr (u % 2 == 0) one_unit(r + rr, IC<p>{}, c, B0, B1, np);
                else one_unit(r + rr, IC<p>{}, c, B1, B0, np);
            });
        }

        // limbs -> uint32 (mod 2^32) by a reduce-scatter over the lane quad:
        // lane with limb l ends with the full sum of row v = l of the tile.
        const bool p1 = lane & 1, h1 = lane & 2;
        auto rs = [&](const uint32_t (&z)[4]) -> uint32_t {
            const uint32_t y0 = z[0] << (8 * limb), y1 = z[1] << (8 * limb);
            const uint32_t y2 = z[2] << (8 * limb), y3 = z[3] << (8 * limb);
            const uint32_t za = (p1 ? y1 : y0) + (uint32_t)__builtin_amdgcn_mov_dpp((int)(p1 ? y0 : y1), 0xB1, 0xF, 0xF, false);
            const uint32_t zb = (p1 ? y3 : y2) + (uint32_t)__builtin_amdgcn_mov_dpp((int)(p1 ? y2 : y3), 0xB1, 0xF, 0xF, false);
            return (h1 ? zb : za) + (uint32_t)__builtin_amdgcn_mov_dpp((int)(h1 ? za : zb), 0x4E, 0xF, 0xF, false);
        };
        // row v of lane (s, l, g) is coefficient 64 t + mb of the product, with
        // mb = 16 g + 4 v + s - 1; after the reduce-scatter v = l.  Only
        // coefficient -1 (tile 0 of the first half, mb = -1) wraps: it is
        // -(coefficient M - 1).
        const int mb = 16 * g + 4 * limb + ss - 1;
        uint32_t *accE = accL + jc * N, *accO = accE + M;
#pragma unroll
        for (int t = 0; t < G::NT; ++t) {
            const int m = 64 * (hw * G::NT + t) + mb;
            uint32_t zo[4], z1[4], z2[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                z1[v] = (uint32_t)C[0][t][v];
                z2[v] = (uint32_t)C[1][t][v];
                zo[v] = (uint32_t)C[2][t][v] - z1[v] - z2[v];
            }
            const uint32_t xo = rs(zo), x1 = rs(z1), x2 = rs(z2);
            if (t == 0 && hw == 0 && mb < 0) {
                atomicAdd(&accO[M - 1], wO[t] - xo);  // (a b)_o = P_s - P_e - P_o
                atomicAdd(&accE[M - 1], wE[t] - x1);  // (a b)_e = P_e + Y P_o
            } else {
                atomicAdd(&accO[m], xo + wO[t]);
                atomicAdd(&accE[m], x1 + wE[t]);
            }
            atomicAdd(&accE[m + 1], x2);  // m + 1 <= M - 1: no wrap
        }
        __syncthreads();  // the next digits overwrite the set all wavefronts have just read
        if (G::DSETS > 1) set ^= 1;
        i = inext;
    }
    __syncthreads();
    for (int x = threadIdx.x; x < 2 * N; x += 64 * G::WAVES) {
        const int m = x & (N - 1);
        row[x] = accL[(x & ~(N - 1)) + (m & 1) * M + (m >> 1)];
    }
}

template <int N, int ELL, int CH, int WPC = BrKara<N, ELL, CH>::WPC>
__global__ __launch_bounds__(128 * WPC, 4 / WPC) void k_br_kara(uint32_t *__restrict__ acc_g,
                                                    const uint32_t *__restrict__ ctN, uint32_t a_base,
                                                    uint32_t accs_per_ct, int n,
                                                    const v4i *__restrict__ bfrag,
                                                    const uint32_t *__restrict__ corr, int log2B)
{
    extern __shared__ uint8_t smem[];
    const uint32_t a_idx = a_base + blockIdx.x;  // accumulator; sample a_idx / accs_per_ct
    br_kara_run<N, ELL, CH, WPC>(smem, acc_g + (size_t)a_idx * 2 * N,
                                 ctN + (size_t)(a_idx / accs_per_ct) * (n + 1) + 1, n, bfrag, corr, log2B);
}

// ---------------------------------------------------------------------------
// One-wavefront form of k_br_kara for N <= 1024: a single wavefront owns the
// accumulator and computes both output components, so each Toeplitz A
// fragment feeds the MFMAs of both components and no workgroup barrier is
// needed (all LDS traffic of an accumulator is in one wavefront's program
// order).  Same digits, products, layouts and results as k_br_kara.
// ---------------------------------------------------------------------------
template <int N, int ELL, int CH>
__global__ __launch_bounds__(64, 1) void k_br_kara1w(uint32_t *__restrict__ acc_g,
                                                    const uint32_t *__restrict__ ctN, uint32_t a_base,
                                                    uint32_t accs_per_ct, int n,
                                                    const v4i *__restrict__ bfrag,
                                                    const uint32_t *__restrict__ corr, int log2B)
{
    using G = BrKara<N, ELL, CH>;
    static_assert(G::WPC == 1, "one wavefront per accumulator needs N <= 1024");
    constexpr int M = G::M;
    extern __shared__ uint8_t smem[];
    uint32_t *accL = (uint32_t *)smem;  // [2][N]: per component, even half then odd half
    uint32_t *digL = accL + 2 * N;      // [RV][3 products][SEQ_WORDS]
    auto seq = [&](int r, int p) { return digL + (r * 3 + p) * G::SEQ_WORDS; };

    const int lane = threadIdx.x & 63;
    const uint32_t a_idx = a_base + blockIdx.x;  // accumulator; sample a_idx / accs_per_ct
    uint32_t *row = acc_g + (size_t)a_idx * 2 * N;
    for (int x = lane; x < 2 * N; x += 64) {
        const int m = x & (N - 1);
        accL[(x & ~(N - 1)) + (m & 1) * M + (m >> 1)] = row[x];
    }
    const uint32_t *crow = ctN + (size_t)(a_idx / accs_per_ct) * (n + 1) + 1;
    const uint32_t drop = 32 - ELL * log2B;
    const int ri = lane & 15, g = lane >> 4;
    const int S0 = M - 4 * ri + 16 * g;
    const int limb = lane & 3, ss = (lane >> 2) & 3;
    // B fragments of unit (row r, product p, chunk c), component 0; component 1 follows
    auto frag = [&](int i, int r, int p, int c) {
        return bfrag + (((((size_t)i * G::RV + r) * 3 + p) * 2) * G::NKB + c * G::KC) * 64 + lane;
    };
    constexpr int JSTRIDE = G::NKB * 64;
    auto next_live = [&](int i) {
        int k = i + 1;
        while (k < n && __builtin_amdgcn_readfirstlane(crow[k]) == 0) ++k;
        return k;
    };

    int i = next_live(-1);
    v4i B0[2][G::KC], B1[2][G::KC];
    {
        const v4i *bp = frag(i < n ? i : 0, 0, 0, 0);
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int kb = 0; kb < G::KC; ++kb) B0[j][kb] = bp[j * JSTRIDE + kb * 64];
    }
    __syncthreads();
    while (i < n) {
        const uint32_t a = __builtin_amdgcn_readfirstlane(crow[i]);
        const int inext = next_live(i);

        // digits of (X^{-a} acc_c - acc_c) for both components, as in k_br_kara
        {
            const uint32_t al = a >> 1, odd_a = a & 1;
#pragma unroll
            for (int jc = 0; jc < 2; ++jc) {
                const uint32_t *accJ = accL + jc * N;
                const uint4 *srcE = (const uint4 *)(accJ + (odd_a ? M : 0));
                const uint4 *srcO = (const uint4 *)(accJ + (odd_a ? 0 : M));
                const uint4 *ownE = (const uint4 *)accJ, *ownO = (const uint4 *)(accJ + M);
#pragma unroll
                for (int qq = 0; qq < (G::QPW + 63) / 64; ++qq) {
                    if (G::QPW % 64 != 0 && qq * 64 + lane >= G::QPW) break;
                    const uint32_t q = qq * 64 + lane;
                    uint32_t rE[4], rO[4];
                    kara_rot4<M>(srcE, q, al, rE);
                    kara_rot4<M>(srcO, q, al + odd_a, rO);
                    const uint4 E4 = ownE[q], O4 = ownO[q];
                    const uint32_t oE[4] = {E4.x, E4.y, E4.z, E4.w}, oO[4] = {O4.x, O4.y, O4.z, O4.w};
                    uint32_t tE[4], tO[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const uint32_t dE = rE[u] - oE[u], dO = rO[u] - oO[u];
                        tE[u] = drop ? (dE + (1u << (drop - 1))) >> drop : dE;
                        tO[u] = drop ? (dO + (1u << (drop - 1))) >> drop : dO;
                    }
#pragma unroll
                    for (int jj = 0; jj < ELL; ++jj) {
#pragma unroll
                        for (int h = 0; h < CH; ++h) {
                            const uint32_t off = log2B * jj + 7 * h;
                            const bool full = 7 * (h + 1) <= log2B;
                            const uint32_t wdt = full ? 7u : (uint32_t)log2B - 7 * h;
                            const uint32_t oe = full ? 64u : 0u, oo = full ? 63u : 0u;
                            const uint32_t cE = (128u - oe) * 0x01010101u, nE = (128u + oe) * 0x01010101u;
                            const uint32_t cO = (128u - oo) * 0x01010101u, nO = (128u + oo) * 0x01010101u;
                            const uint32_t cS = (128u - oe - oo) * 0x01010101u, nS = (128u + oe + oo) * 0x01010101u;
                            uint32_t pe = __builtin_amdgcn_ubfe(tE[3], off, wdt);
                            pe |= __builtin_amdgcn_ubfe(tE[2], off, wdt) << 8;
                            pe |= __builtin_amdgcn_ubfe(tE[1], off, wdt) << 16;
                            pe |= __builtin_amdgcn_ubfe(tE[0], off, wdt) << 24;
                            uint32_t po = __builtin_amdgcn_ubfe(tO[3], off, wdt);
                            po |= __builtin_amdgcn_ubfe(tO[2], off, wdt) << 8;
                            po |= __builtin_amdgcn_ubfe(tO[1], off, wdt) << 16;
                            po |= __builtin_amdgcn_ubfe(tO[0], off, wdt) << 24;
                            const uint32_t ps = pe + po;
                            const int r = jc * G::RPC + jj * CH + h;
                            uint32_t *sE = seq(r, 0), *sO = seq(r, 1), *sS = seq(r, 2);
                            sE[M / 4 - q - 1] = (pe + cE) ^ 0x80808080u;
                            sE[M / 2 - q - 1] = (nE - pe) ^ 0x80808080u;
                            sO[M / 4 - q - 1] = (po + cO) ^ 0x80808080u;
                            sO[M / 2 - q - 1] = (nO - po) ^ 0x80808080u;
                            sS[M / 4 - q - 1] = (ps + cS) ^ 0x80808080u;
                            sS[M / 2 - q - 1] = (nS - ps) ^ 0x80808080u;
                        }
                    }
                }
            }
        }
        __syncthreads();  // one wavefront: orders the digit writes before the fragment reads

        v4i C[3][2][G::NT];
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int t = 0; t < G::NT; ++t) C[p][j][t] = v4i{0, 0, 0, 0};

        auto one_unit = [&](const int r, auto P_, const int c, v4i(&Bc)[2][G::KC], v4i(&Bn)[2][G::KC],
                            const v4i *np) {
            constexpr int p = decltype(P_)::value;
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int kb = 0; kb < G::KC; ++kb) Bn[j][kb] = np[j * JSTRIDE + kb * 64];
            __builtin_amdgcn_sched_barrier(0);
            const int dshift = -64 * c * G::KC;
            const uint32_t *ab = seq(r, p) + (S0 - dshift - G::DLOC) / 4;
            auto afrag = [&](const int dd, v4i &A) {
#pragma unroll
                for (int k = 0; k < 4; ++k) A[k] = (int)ab[16 * dd + k];
            };
            v4i Af[2];
            afrag(0, Af[0]);
#pragma unroll
            for (int dd = 0; dd < G::NDIAG; ++dd) {
                const int dl = G::DLOC - 64 * dd;
                if (dd + 1 < G::NDIAG) afrag(dd + 1, Af[(dd + 1) & 1]);
#pragma unroll
                for (int kb = 0; kb < G::KC; ++kb) {
                    const int m0 = dl + 64 * kb;
                    if (m0 >= 0 && m0 <= 64 * (G::NT - 1)) {
#pragma unroll
                        for (int j = 0; j < 2; ++j)
                            C[p][j][m0 / 64] = __builtin_amdgcn_mfma_i32_16x16x64_i8(Af[dd & 1], Bc[j][kb],
                                                                                    C[p][j][m0 / 64], 0, 0, 0);
                    }
                }
            }
        };

#pragma unroll 1
        for (int r = 0; r < G::RV; r += G::RSTEP) {
            StaticFor<0, G::USTEP>::run([&](auto U_) {
                constexpr int u = decltype(U_)::value;
                constexpr int rr = u / G::UPR, p = (u % G::UPR) / G::NCH, c = u % G::NCH;
                const v4i *np;
                if constexpr (u + 1 < G::USTEP) {
                    constexpr int u2 = u + 1;
                    np = frag(i, r + u2 / G::UPR, (u2 % G::UPR) / G::NCH, u2 % G::NCH);
                } else {
                    np = (r + G::RSTEP < G::RV) ? frag(i, r + G::RSTEP, 0, 0)
                                                : frag(inext < n ? inext : i, 0, 0, 0);
                }
                if constexpr (u % 2 == 0) one_unit(r + rr, IC<p>{}, c, B0, B1, np);
                else one_unit(r + rr, IC<p>{}, c, B1, B0, np);
            });
        }

        // recombine both components (reduce-scatter over the lane quad) and add
        // the offset correction of this step
        const bool p1 = lane & 1, h1 = lane & 2;
        auto rs = [&](const uint32_t (&z)[4]) -> uint32_t {
            const uint32_t y0 = z[0] << (8 * limb), y1 = z[1] << (8 * limb);
            const uint32_t y2 = z[2] << (8 * limb), y3 = z[3] << (8 * limb);
            const uint32_t za = (p1 ? y1 : y0) + (uint32_t)__builtin_amdgcn_mov_dpp((int)(p1 ? y0 : y1), 0xB1, 0xF, 0xF, false);
            const uint32_t zb = (p1 ? y3 : y2) + (uint32_t)__builtin_amdgcn_mov_dpp((int)(p1 ? y2 : y3), 0xB1, 0xF, 0xF, false);
            return (h1 ? zb : za) + (uint32_t)__builtin_amdgcn_mov_dpp((int)(h1 ? za : zb), 0x4E, 0xF, 0xF, false);
        };
        const int mb = 16 * g + 4 * limb + ss - 1;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            uint32_t *accE = accL + j * N, *accO = accE + M;
            const uint32_t *cp = corr + ((size_t)i * 2 + j) * N;
#pragma unroll
            for (int t = 0; t < G::NT; ++t) {
                const int m = 64 * t + mb;
                const int mc = m & (M - 1);
                const uint32_t wE = cp[mc], wO = cp[M + mc];
                uint32_t zo[4], z1[4], z2[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    z1[v] = (uint32_t)C[0][j][t][v];
                    z2[v] = (uint32_t)C[1][j][t][v];
                    zo[v] = (uint32_t)C[2][j][t][v] - z1[v] - z2[v];
                }
                const uint32_t xo = rs(zo), x1 = rs(z1), x2 = rs(z2);
                // LDS atomic adds: lanes of one instruction touch distinct words,
                // but later statements touch words of other lanes (m + 1), which
                // plain read-modify-writes could reorder
                if (t == 0 && mb < 0) {
                    atomicAdd(&accO[M - 1], wO - xo);  // coefficient -1 is -(coefficient M - 1)
                    atomicAdd(&accE[M - 1], wE - x1);
                } else {
                    atomicAdd(&accO[m], xo + wO);
                    atomicAdd(&accE[m], x1 + wE);
                }
                atomicAdd(&accE[m + 1], x2);  // Y P_o
            }
        }
        __syncthreads();  // the accumulate completes before the next digits read it
        i = inext;
    }
    __syncthreads();
    for (int x = lane; x < 2 * N; x += 64) {
        const int m = x & (N - 1);
        row[x] = accL[(x & ~(N - 1)) + (m & 1) * M + (m >> 1)];
    }
}

// ---------------------------------------------------------------------------
// k_br_kara1w with two wavefronts per SIMD, for rounds that fill the device:
// the three products run one after another and are folded into the
// accumulator in turn, so that registers (one product's tiles) and LDS (two
// digit sequences per row, V_e + V_o written over V_e once P_e is done) leave
// room for a second wavefront, whose MFMAs run while the first computes
// digits or waits.  A round that does not fill every SIMD twice uses
// k_br_kara1w instead: its register use allows one wavefront per SIMD, so the
// dispatcher cannot stack two on one SIMD while another idles.  Same digits,
// products and results as k_br_kara1w.
// WV = 2 gives each accumulator two wavefronts, each with the digit rows of
// one input component (its digits, its products, its folds; the step's
// correction is added by the first), with one key buffer that is refilled
// block by block; two barriers per step.  It halves the time of a step for
// rounds small enough to give every wavefront a SIMD of its own.
// ---------------------------------------------------------------------------
// One accumulator (row) rotated by WV wavefronts whose threads are numbered
// tid = 0 .. 64 WV - 1, LDS at smem.  SKIP: steps with a_i = 0 are skipped
// (their CMux adds exactly zero); without it every step runs, so that
// wavefronts of one workgroup rotating different accumulators meet the same
// barriers.  The result is stored only if `store`.
template <int N, int ELL, int CH, int WV, bool SKIP>
__device__ __attribute__((always_inline)) inline void br_kara1w2_run(uint8_t *smem, uint32_t *__restrict__ row,
                                                                    const uint32_t *__restrict__ crow, int n,
                                                                    const v4i *__restrict__ bfrag,
                                                                    const uint32_t *__restrict__ corr, int log2B,
                                                                    int tid, bool store)
{
    using G = BrKara<N, ELL, CH>;
    static_assert(G::WPC == 1, "one wavefront per accumulator needs N <= 1024");
    constexpr int M = G::M;
    uint32_t *accL = (uint32_t *)smem;  // [2][N]: per component, even half then odd half
    uint32_t *digL = accL + 2 * N;      // [RV][V_e (then V_e + V_o), V_o][SEQ_WORDS]
    auto seq = [&](int r, int p) { return digL + (r * 2 + (p & 1)) * G::SEQ_WORDS; };

    static_assert(WV == 1 || WV == 2, "one wavefront, or one per component's digit rows");
    constexpr int RW = G::RV / WV;  // digit rows per wavefront: those of component hw when WV = 2
    const int lane = tid & 63;
    const int hw = WV == 1 ? 0 : __builtin_amdgcn_readfirstlane(tid >> 6);
    const int r0 = hw * RW;  // first digit row of this wavefront
    for (int x = tid; x < 2 * N; x += 64 * WV) {
        const int m = x & (N - 1);
        accL[(x & ~(N - 1)) + (m & 1) * M + (m >> 1)] = row[x];
    }
    const uint32_t drop = 32 - ELL * log2B;
    const int ri = lane & 15, g = lane >> 4;
    const int S0 = M - 4 * ri + 16 * g;
    const int limb = lane & 3, ss = (lane >> 2) & 3;
    // B fragments of unit (row r, product p, chunk c), component 0; component 1 follows
    auto frag = [&](int i, int r, int p, int c) {
        return bfrag + (((((size_t)i * G::RV + r) * 3 + p) * 2) * G::NKB + c * G::KC) * 64 + lane;
    };
    constexpr int JSTRIDE = G::NKB * 64;
    auto next_live = [&](int i) {
        int k = i + 1;
        if constexpr (SKIP)
            while (k < n && __builtin_amdgcn_readfirstlane(crow[k]) == 0) ++k;
        return k;
    };

    int i = next_live(-1);
    v4i B0[2][G::KC], B1[2][G::KC];
    {
        const v4i *bp = frag(i < n ? i : 0, r0, 0, 0);
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int kb = 0; kb < G::KC; ++kb) B0[j][kb] = bp[j * JSTRIDE + kb * 64];
    }
    __syncthreads();
    while (i < n) {
        const uint32_t a = __builtin_amdgcn_readfirstlane(crow[i]);
        const int inext = next_live(i);

        // digits of (X^{-a} acc_c - acc_c) for both components, as in k_br_kara
        {
            const uint32_t al = a >> 1, odd_a = a & 1;
#pragma unroll
            for (int jc0 = 0; jc0 < 2 / WV; ++jc0) {
                const int jc = WV == 1 ? jc0 : hw;
                const uint32_t *accJ = accL + jc * N;
                const uint4 *srcE = (const uint4 *)(accJ + (odd_a ? M : 0));
                const uint4 *srcO = (const uint4 *)(accJ + (odd_a ? 0 : M));
                const uint4 *ownE = (const uint4 *)accJ, *ownO = (const uint4 *)(accJ + M);
#pragma unroll
                for (int qq = 0; qq < (G::QPW + 63) / 64; ++qq) {
                    if (G::QPW % 64 != 0 && qq * 64 + lane >= G::QPW) break;
                    const uint32_t q = qq * 64 + lane;
                    uint32_t rE[4], rO[4];
                    kara_rot4<M>(srcE, q, al, rE);
                    kara_rot4<M>(srcO, q, al + odd_a, rO);
                    const uint4 E4 = ownE[q], O4 = ownO[q];
                    const uint32_t oE[4] = {E4.x, E4.y, E4.z, E4.w}, oO[4] = {O4.x, O4.y, O4.z, O4.w};
                    uint32_t tE[4], tO[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const uint32_t dE = rE[u] - oE[u], dO = rO[u] - oO[u];
                        tE[u] = drop ? (dE + (1u << (drop - 1))) >> drop : dE;
                        tO[u] = drop ? (dO + (1u << (drop - 1))) >> drop : dO;
                    }
#pragma unroll
                    for (int jj = 0; jj < ELL; ++jj) {
#pragma unroll
                        for (int h = 0; h < CH; ++h) {
                            const uint32_t off = log2B * jj + 7 * h;
                            const bool full = 7 * (h + 1) <= log2B;
                            const uint32_t wdt = full ? 7u : (uint32_t)log2B - 7 * h;
                            const uint32_t oe = full ? 64u : 0u, oo = full ? 63u : 0u;
                            const uint32_t cE = (128u - oe) * 0x01010101u, nE = (128u + oe) * 0x01010101u;
                            const uint32_t cO = (128u - oo) * 0x01010101u, nO = (128u + oo) * 0x01010101u;
                            uint32_t pe = __builtin_amdgcn_ubfe(tE[3], off, wdt);
                            pe |= __builtin_amdgcn_ubfe(tE[2], off, wdt) << 8;
                            pe |= __builtin_amdgcn_ubfe(tE[1], off, wdt) << 16;
                            pe |= __builtin_amdgcn_ubfe(tE[0], off, wdt) << 24;
                            uint32_t po = __builtin_amdgcn_ubfe(tO[3], off, wdt);
                            po |= __builtin_amdgcn_ubfe(tO[2], off, wdt) << 8;
                            po |= __builtin_amdgcn_ubfe(tO[1], off, wdt) << 16;
                            po |= __builtin_amdgcn_ubfe(tO[0], off, wdt) << 24;
                            const int r = jc * G::RPC + jj * CH + h;
                            uint32_t *sE = seq(r, 0), *sO = seq(r, 1);
                            sE[M / 4 - q - 1] = (pe + cE) ^ 0x80808080u;
                            sE[M / 2 - q - 1] = (nE - pe) ^ 0x80808080u;
                            sO[M / 4 - q - 1] = (po + cO) ^ 0x80808080u;
                            sO[M / 2 - q - 1] = (nO - po) ^ 0x80808080u;
                        }
                    }
                }
            }
        }
        __syncthreads();  // digits written, and every read of the accumulator done before a fold

        // One product at a time: its MFMA accumulators (both components) are
        // folded into the LDS accumulator before the next product starts, which
        // keeps the kernel within the registers of two wavefronts per SIMD.
        v4i C[2][G::NT];
        // first A word of unit (row r, product p, key chunk c) for this lane
        auto abase = [&](int r, int p, int c) { return seq(r, p) + (S0 + 64 * c * G::KC - G::DLOC) / 4; };
        auto one_unit = [&](const int r, auto P_, const int c, v4i(&Bc)[2][G::KC], v4i(&Bn)[2][G::KC],
                            const v4i *np) {
            constexpr int p = decltype(P_)::value;
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int kb = 0; kb < G::KC; ++kb) Bn[j][kb] = np[j * JSTRIDE + kb * 64];
            __builtin_amdgcn_sched_barrier(0);
            const uint32_t *ab = abase(r, p, c);
            auto afrag = [&](const int dd, v4i &A) {
#pragma unroll
                for (int k = 0; k < 4; ++k) A[k] = (int)ab[16 * dd + k];
            };
            v4i Af[2];
            afrag(0, Af[0]);
#pragma unroll
            for (int dd = 0; dd < G::NDIAG; ++dd) {
                const int dl = G::DLOC - 64 * dd;
                if (dd + 1 < G::NDIAG) afrag(dd + 1, Af[(dd + 1) & 1]);
#pragma unroll
                for (int kb = 0; kb < G::KC; ++kb) {
                    const int m0 = dl + 64 * kb;
                    if (m0 >= 0 && m0 <= 64 * (G::NT - 1)) {
#pragma unroll
                        for (int j = 0; j < 2; ++j)
                            C[j][m0 / 64] = __builtin_amdgcn_mfma_i32_16x16x64_i8(Af[dd & 1], Bc[j][kb], C[j][m0 / 64],
                                                                                 0, 0, 0);
                    }
                }
            }
        };

        const bool p1 = lane & 1, h1 = lane & 2;
        auto rs = [&](const v4i &zc) -> uint32_t {  // limbs recombined mod 2^32, reduce-scatter over the quad
            const uint32_t y0 = (uint32_t)zc[0] << (8 * limb), y1 = (uint32_t)zc[1] << (8 * limb);
            const uint32_t y2 = (uint32_t)zc[2] << (8 * limb), y3 = (uint32_t)zc[3] << (8 * limb);
            const uint32_t za = (p1 ? y1 : y0) + (uint32_t)__builtin_amdgcn_mov_dpp((int)(p1 ? y0 : y1), 0xB1, 0xF, 0xF, false);
            const uint32_t zb = (p1 ? y3 : y2) + (uint32_t)__builtin_amdgcn_mov_dpp((int)(p1 ? y2 : y3), 0xB1, 0xF, 0xF, false);
            return (h1 ? zb : za) + (uint32_t)__builtin_amdgcn_mov_dpp((int)(h1 ? za : zb), 0x4E, 0xF, 0xF, false);
        };
        const int mb = 16 * g + 4 * limb + ss - 1;
        constexpr int RS2 = (G::NCH % 2) ? 2 : 1;  // rows per unrolled group: an even number of units
        constexpr int UG = RS2 * G::NCH;
        static_assert(G::RV % RS2 == 0, "rows split into whole groups");

        StaticFor<0, 3>::run([&](auto P_) {
            constexpr int p = decltype(P_)::value;
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int t = 0; t < G::NT; ++t) C[j][t] = v4i{0, 0, 0, 0};
            if constexpr (WV == 1) {
#pragma unroll 1
                for (int r = 0; r < G::RV; r += RS2) {
                    StaticFor<0, UG>::run([&](auto U_) {
                        constexpr int u = decltype(U_)::value;
                        constexpr int rr = u / G::NCH, c = u % G::NCH;
                        const v4i *np;  // key fragments of the next unit
                        if constexpr (u + 1 < UG) {
                            constexpr int u2 = u + 1;
                            np = frag(i, r + u2 / G::NCH, p, u2 % G::NCH);
                        } else {
                            const bool more = r + RS2 < G::RV;
                            if constexpr (p < 2) np = more ? frag(i, r + RS2, p, 0) : frag(i, 0, p + 1, 0);
                            else np = more ? frag(i, r + RS2, p, 0) : frag(inext < n ? inext : i, 0, 0, 0);
                        }
                        if constexpr (u % 2 == 0) one_unit(r + rr, IC<p>{}, c, B0, B1, np);
                        else one_unit(r + rr, IC<p>{}, c, B1, B0, np);
                    });
                }
            } else {
                // this wavefront's rows, with one key buffer: each key block is
                // reloaded for the next unit once its last diagonal is done
#pragma unroll 1
                for (int rr = 0; rr < RW; ++rr) {
                    StaticFor<0, G::NCH>::run([&](auto C_) {
                        constexpr int c = decltype(C_)::value;
                        const v4i *np;
                        if constexpr (c + 1 < G::NCH) np = frag(i, r0 + rr, p, c + 1);
                        else if (rr + 1 < RW) np = frag(i, r0 + rr + 1, p, 0);
                        else if constexpr (p < 2) np = frag(i, r0, p + 1, 0);
                        else np = frag(inext < n ? inext : i, r0, 0, 0);
                        const uint32_t *ab = abase(r0 + rr, p, c);
                        auto afrag = [&](const int dd, v4i &A) {
#pragma unroll
                            for (int k = 0; k < 4; ++k) A[k] = (int)ab[16 * dd + k];
                        };
                        v4i Af[2];
                        afrag(0, Af[0]);
#pragma unroll
                        for (int dd = 0; dd < G::NDIAG; ++dd) {
                            const int dl = G::DLOC - 64 * dd;
                            if (dd + 1 < G::NDIAG) afrag(dd + 1, Af[(dd + 1) & 1]);
#pragma unroll
                            for (int kb = 0; kb < G::KC; ++kb) {
                                const int m0 = dl + 64 * kb;
                                if (m0 >= 0 && m0 <= 64 * (G::NT - 1)) {
#pragma unroll
                                    for (int j = 0; j < 2; ++j)
                                        C[j][m0 / 64] = __builtin_amdgcn_mfma_i32_16x16x64_i8(Af[dd & 1], B0[j][kb],
                                                                                             C[j][m0 / 64], 0, 0, 0);
                                }
                            }
                            // key block kb is last used by diagonal kb + NT - 1
                            if (dd >= G::NT - 1) {
                                const int kd = dd - (G::NT - 1);
#pragma unroll
                                for (int j = 0; j < 2; ++j) B0[j][kd] = np[j * JSTRIDE + kd * 64];
                            }
                        }
                    });
                }
            }
            if constexpr (p == 0) {
                // V_e + V_o (bytewise, no carry between bytes) replaces V_e: every
                // read of V_e was issued above, and one wavefront's LDS operations
                // are performed in order
#pragma unroll
                for (int x = lane * 4; x < RW * G::SEQ_WORDS; x += 256) {
                    const int rr = r0 + x / G::SEQ_WORDS, w = x % G::SEQ_WORDS;
                    uint4 *pe4 = (uint4 *)(seq(rr, 0) + w);
                    const uint4 e4 = *pe4, o4 = *(const uint4 *)(seq(rr, 1) + w);
                    auto add8 = [](uint32_t a, uint32_t b) {
                        return ((a & 0x7F7F7F7Fu) + (b & 0x7F7F7F7Fu)) ^ ((a ^ b) & 0x80808080u);
                    };
                    *pe4 = uint4{add8(e4.x, o4.x), add8(e4.y, o4.y), add8(e4.z, o4.z), add8(e4.w, o4.w)};
                }
            }
            // fold product p: (ab)_e = P_e + Y P_o, (ab)_o = P_s - P_e - P_o; the
            // offset correction of the step rides with P_e.  Coefficient -1 of the
            // tiling is -(coefficient M - 1).  LDS atomic adds: lanes of one
            // instruction touch distinct words, but later statements touch words
            // of other lanes (m + 1), which plain read-modify-writes could reorder.
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                uint32_t *accE = accL + j * N, *accO = accE + M;
#pragma unroll
                for (int t = 0; t < G::NT; ++t) {
                    const int m = 64 * t + mb;
                    const bool wrap = t == 0 && mb < 0;
                    const uint32_t x = rs(C[j][t]);
                    if constexpr (p == 0) {
                        const uint32_t *cp = corr + ((size_t)i * 2 + j) * N;
                        const int mc = m & (M - 1);
                        // the correction of the whole step, added once
                        const uint32_t wE = hw == 0 ? cp[mc] : 0u, wO = hw == 0 ? cp[M + mc] : 0u;
                        atomicAdd(&accE[wrap ? M - 1 : m], wrap ? wE - x : wE + x);
                        atomicAdd(&accO[wrap ? M - 1 : m], wrap ? wO + x : wO - x);
                    } else if constexpr (p == 1) {
                        atomicAdd(&accE[m + 1], x);
                        atomicAdd(&accO[wrap ? M - 1 : m], wrap ? x : 0u - x);
                    } else {
                        atomicAdd(&accO[wrap ? M - 1 : m], wrap ? 0u - x : x);
                    }
                }
            }
        });
        __syncthreads();  // the accumulate completes before the next digits read it
        i = inext;
    }
    __syncthreads();
    if (store)
        for (int x = tid; x < 2 * N; x += 64 * WV) {
            const int m = x & (N - 1);
            row[x] = accL[(x & ~(N - 1)) + (m & 1) * M + (m >> 1)];
        }
}

template <int N, int ELL, int CH, int WV>
__global__ __launch_bounds__(64 * WV) __attribute__((amdgpu_waves_per_eu(2))) void k_br_kara1w2(uint32_t *__restrict__ acc_g,
                                                    const uint32_t *__restrict__ ctN, uint32_t a_base,
                                                    uint32_t accs_per_ct, int n,
                                                    const v4i *__restrict__ bfrag,
                                                    const uint32_t *__restrict__ corr, int log2B)
{
    extern __shared__ uint8_t smem[];
    const uint32_t a_idx = a_base + blockIdx.x;  // accumulator; sample a_idx / accs_per_ct
    br_kara1w2_run<N, ELL, CH, WV, true>(smem, acc_g + (size_t)a_idx * 2 * N,
                                         ctN + (size_t)(a_idx / accs_per_ct) * (n + 1) + 1, n, bfrag, corr,
                                         log2B, (int)threadIdx.x, true);
}

// ---------------------------------------------------------------------------
// Persistent work-queue blind rotation: one launch rotates the accumulators
// of several jobs (contexts with their own keys, tables and samples) of two
// ring degrees at once.  Resident workgroups (4 wavefronts, two per CU) pull
// items from a device counter until the queue is empty.  An item of a "wide"
// job (N = 2048, geometry B) is one accumulator rotated by the whole
// workgroup (br_kara_run); an item of a narrow job (geometry A, N <= 1024)
// is four accumulators, one per wavefront (br_kara1w2_run), which run every
// step so that all four meet the same barriers (a step with a_i = 0 adds
// exactly zero).  A wavefront past the end of its job repeats the job's last
// accumulator without storing it.  Wide items come first in the queue (the
// longer items start first).  Results equal those of the per-job launches,
// bit for bit.
// ---------------------------------------------------------------------------
template <int NA, int LA, int CA, int NB, int LB, int CB>
struct BrQueueGeom {
    using GA = BrKara<NA, LA, CA>;
    using GB = BrKara<NB, LB, CB>;
    static_assert(GA::WPC == 1 && GB::WAVES == 4, "narrow: one wavefront per accumulator; wide: four");
    static constexpr size_t LDS_A = GA::LDS2W_BYTES;  // per wavefront
    static constexpr size_t LDS = 4 * LDS_A > GB::LDS_BYTES ? 4 * LDS_A : GB::LDS_BYTES;
};

template <int NA, int LA, int CA, int NB, int LB, int CB>
__global__ __launch_bounds__(256, 2) void k_br_queue(const BrQueue q, uint32_t *__restrict__ counter)
{
    using Q = BrQueueGeom<NA, LA, CA, NB, LB, CB>;
    extern __shared__ uint8_t smem[];
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    for (;;) {
        // the workgroup's next item, broadcast through LDS word 0 (free here:
        // every wavefront has passed the last barrier of the previous item)
        __syncthreads();
        if (threadIdx.x == 0) *(volatile uint32_t *)smem = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t item = __builtin_amdgcn_readfirstlane(*(volatile uint32_t *)smem);
        __syncthreads();
        if (item >= q.items) break;  // uniform: every wavefront leaves
        uint32_t j = 0;
        while (j + 1 < q.njobs && item >= q.job[j + 1].first_item) ++j;
        const BrQueueJob &J = q.job[j];
        const uint32_t k = item - J.first_item;
        const v4i *bfrag = (const v4i *)J.bfrag;
        if (J.wide) {
            br_kara_run<NB, LB, CB>(smem, J.acc + (size_t)k * 2 * NB, J.ctN + (size_t)(k / J.per) * (J.n + 1) + 1,
                                    (int)J.n, bfrag, J.corr, (int)J.log2B);
        } else {
            uint32_t a = 4 * k + wave;
            const bool store = a < J.accs;
            if (!store) a = J.accs - 1;
            br_kara1w2_run<NA, LA, CA, 1, false>(smem + wave * Q::LDS_A, J.acc + (size_t)a * 2 * NA,
                                                 J.ctN + (size_t)(a / J.per) * (J.n + 1) + 1, (int)J.n, bfrag,
                                                 J.corr, (int)J.log2B, (int)threadIdx.x & 63, store);
        }
    }
}

// Fill n words with v (resets the queue counters; a kernel rather than a
// memset so that it can sit in a captured HIP graph).
__global__ void k_fill(uint32_t *__restrict__ p, uint32_t n, uint32_t v)
{
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) p[x] = v;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static int ilog2i(int x) { int r = 0; while ((1 << r) < x) ++r; return r; }

// One-time set-up per device (function attributes and occupancy belong to a
// device): make(dev, &value) runs once per device, under a lock; devices past
// the table are set up on every call.
template <typename T>
struct PerDevice {
    static constexpr int kDevices = 64;
    std::mutex mu;
    bool have[kDevices] = {};
    T val[kDevices] = {};
    template <typename F>
    hipError_t get(T *out, F make)
    {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        std::lock_guard<std::mutex> lock(mu);
        const bool tab = dev >= 0 && dev < kDevices;
        if (tab && have[dev]) {
            *out = val[dev];
            return hipSuccess;
        }
        T v{};
        e = make(dev, &v);
        if (e != hipSuccess) return e;
        if (tab) {
            val[dev] = v;
            have[dev] = true;
        }
        *out = v;
        return hipSuccess;
    }
};

hipError_t launch_modswitch(const Geometry &G, const uint32_t *cts, uint32_t B, uint32_t *ctN,
                            hipStream_t s)
{
    const uint32_t total = B * (uint32_t)(G.n + 1);
    if (!total) return hipSuccess;
    const uint32_t sh = 32 - ilog2i(2 * G.N);
    hipLaunchKernelGGL(k_modswitch, dim3((total + 255) / 256), dim3(256), 0, s, cts, ctN, total, sh,
                       (uint32_t)(2 * G.N - 1));
    return hipGetLastError();
}

hipError_t launch_init_sign(const Geometry &G, const uint32_t *ctN, uint32_t B, uint32_t *acc,
                            hipStream_t s)
{
    if (!B) return hipSuccess;
    const uint32_t half = 1u << (31 - G.log2_t);
    hipLaunchKernelGGL(k_init_sign, dim3((G.N + 255) / 256, B * G.boot_ell), dim3(256), 0, s, ctN,
                       acc, B, G.n, G.N, G.boot_ell, half, 1u << G.boot_log2B);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Calibration: a stream of independent int8 MFMAs from registers (no memory
// traffic, operands with random-looking bytes), to measure the dense int8 rate
// the device sustains on such data.  Thirty-two accumulator chains per
// wavefront, three wavefronts per SIMD, keep the matrix pipe fed; the sums are
// stored so that nothing is optimised away.  The chains are kept in the
// architectural registers (two wavefronts per SIMD requested): with them in
// the accumulation registers the compiler moved chains between registers
// around the MFMAs, which waited on each other's results and held the pipe at
// about 72% occupancy instead of 96%.
// ---------------------------------------------------------------------------
constexpr int kStreamChains = 32;
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_mfma_stream(
    uint32_t iters, int32_t *__restrict__ out)
{
    // operand bytes spread like random digits and key limbs (a multiplicative hash of the lane)
    const uint32_t h = (blockIdx.x * 64u + threadIdx.x + 1u) * 0x9E3779B1u;
    const v4i a = {(int)h, (int)(h * 0x85EBCA77u), (int)(h * 0xC2B2AE3Du), (int)(h * 0x27D4EB2Fu)};
    const v4i b = {(int)(h ^ 0x165667B1u), (int)(h * 0xD3A2646Cu), (int)(h * 0xFD7046C5u), (int)(h * 0xB55A4F09u)};
    v4i c[kStreamChains];
#pragma unroll
    for (int k = 0; k < kStreamChains; ++k) c[k] = v4i{k, 0, 0, 0};
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kStreamChains; ++k) c[k] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c[k], 0, 0, 0);
    }
    int32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kStreamChains; ++k) sum += c[k][0] + c[k][1] + c[k][2] + c[k][3];
    out[(size_t)blockIdx.x * 64 + threadIdx.x] = sum;
}

uint32_t mfma_stream_chains() { return kStreamChains; }

hipError_t mfma_stream_capacity(uint32_t *blocks)
{
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_mfma_stream, 64, 0);
    if (e != hipSuccess) return e;
    *blocks = (uint32_t)std::max(1, per_cu * cus);
    return hipSuccess;
}

hipError_t launch_mfma_stream(uint32_t blocks, uint32_t iters, int32_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_mfma_stream, dim3(blocks), dim3(64), 0, s, iters, out);
    return hipGetLastError();
}

hipError_t launch_init_tfhe(const Geometry &G, const uint32_t *ctN, const int32_t *lut_ids, uint32_t B,
                            const int32_t *luts, int nluts, uint32_t *err, uint32_t *acc, hipStream_t s)
{
    if (!B) return hipSuccess;
    hipLaunchKernelGGL(k_init_tfhe, dim3((G.N + 255) / 256, B), dim3(256), 0, s, ctN, lut_ids, luts, nluts, err,
                       acc, G.n, G.N, G.log2_t);
    return hipGetLastError();
}

hipError_t launch_extract(const Geometry &G, const uint32_t *acc, uint32_t A, uint32_t per,
                          uint32_t add_base, uint32_t *lwe, hipStream_t s)
{
    if (!A) return hipSuccess;
    hipLaunchKernelGGL(k_extract, dim3((G.N + 1 + 255) / 256, A), dim3(256), 0, s, acc, lwe, G.N, per,
                       add_base, 1u << G.boot_log2B);
    return hipGetLastError();
}

hipError_t launch_keyswitch(const uint32_t *in, uint32_t B, uint32_t din, const uint32_t *key,
                            int log2B, int ell, uint32_t out_len, uint32_t *out, hipStream_t s)
{
    if (!B) return hipSuccess;
    if (ell > 8 || log2B > 16) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_keyswitch, dim3((out_len + 255) / 256, (B + KS_TB - 1) / KS_TB), dim3(256),
                       0, s, in, B, din, key, log2B, ell, out_len, out);
    return hipGetLastError();
}

bool keyswitch_mfma_supported(int log2B, int ell, uint32_t din)
{
    return log2B <= 7 && ell >= 1 && ell <= 8 && din % 64 == 0;
}

hipError_t launch_keyswitch_mfma(const uint32_t *in, uint32_t B, uint32_t din, const void *kfrag, int log2B,
                                 int ell, uint32_t out_len, uint32_t *out, hipStream_t s)
{
    if (!B) return hipSuccess;
    const uint32_t words_pad = (out_len + 63) / 64 * 64;
    const dim3 grid(words_pad / 64, (B + 63) / 64);
    const v4i *kf = (const v4i *)kfrag;
    switch (ell) {
#define KS_CASE(L)                                                                                   \
    case L:                                                                                          \
        hipLaunchKernelGGL(k_keyswitch_mfma<L>, grid, dim3(256), 0, s, in, B, din, kf, log2B, out_len, \
                           words_pad / 4, out);                                                      \
        break;
        KS_CASE(1) KS_CASE(2) KS_CASE(3) KS_CASE(4) KS_CASE(5) KS_CASE(6) KS_CASE(7) KS_CASE(8)
#undef KS_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_affine(const int32_t *W, const uint32_t *in, uint32_t rows, uint32_t cols, uint32_t width,
                         uint32_t *out, hipStream_t s)
{
    if (!rows || !width) return hipSuccess;
    hipLaunchKernelGGL(k_affine, dim3((width + 255) / 256, (rows + AF_ROWS - 1) / AF_ROWS), dim3(256), 0, s, W, in,
                       rows, cols, width, out);
    return hipGetLastError();
}

hipError_t launch_lincomb2(const uint32_t *x, const uint32_t *y, int32_t wx, int32_t wy, uint32_t count,
                           uint32_t *out, hipStream_t s)
{
    if (!count) return hipSuccess;
    hipLaunchKernelGGL(k_lincomb2, dim3((count + 255) / 256), dim3(256), 0, s, x, y, (uint32_t)wx, (uint32_t)wy,
                       count, out);
    return hipGetLastError();
}

hipError_t launch_pubmux(const Geometry &G, const uint32_t *rlwe, const uint32_t *ctN,
                         const int32_t *lut_ids, uint32_t E, uint32_t per, const int32_t *luts, int nluts,
                         uint32_t *err, uint32_t *acc, hipStream_t s)
{
    if (!E) return hipSuccess;
    if (!per) return hipErrorInvalidValue;
    const size_t lds = ((size_t)(G.boot_ell * 2 * G.N + 15) & ~(size_t)15) + 4 * (size_t)G.N;
    hipLaunchKernelGGL(k_pubmux, dim3(E), dim3(256), lds, s, rlwe, ctN, lut_ids, luts, nluts, err, acc,
                       G.n, G.N, G.log2_t, G.boot_log2B, G.boot_ell, per);
    return hipGetLastError();
}

hipError_t launch_br_plain(const Geometry &G, uint32_t *acc, const uint32_t *ctN, uint32_t A,
                           uint32_t accs_per_ct, const uint32_t *brk_raw, hipStream_t s)
{
    if (!A) return hipSuccess;
    const int R = 2 * G.g_ell;
    const size_t lds = 4 * (size_t)2 * G.N + 4 * (size_t)R * 2 * G.N + 2 * (size_t)R * 2 * G.N;
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    static PerDevice<bool> attr;
    bool ok = false;
    hipError_t e0 = attr.get(&ok, [](int, bool *v) {
        *v = true;
        return hipFuncSetAttribute((const void *)k_br_plain, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    });
    if (e0 != hipSuccess) return e0;
    hipLaunchKernelGGL(k_br_plain, dim3(A), dim3(256), lds, s, acc, ctN, accs_per_ct, G.n, G.N,
                       G.g_log2B, G.g_ell, brk_raw);
    return hipGetLastError();
}

template <int N, int ELL, int CH>
static hipError_t launch_br_mfma_t(const Geometry &G, uint32_t *acc, const uint32_t *ctN, uint32_t A,
                                   uint32_t accs_per_ct, const void *brk_frag, hipStream_t s)
{
    using GM = BrMfma<N, ELL, CH>;
    static PerDevice<bool> attr;
    bool ok = false;
    hipError_t e0 = attr.get(&ok, [](int, bool *v) {
        *v = true;
        return hipFuncSetAttribute((const void *)k_br_mfma<N, ELL, CH>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)GM::LDS_BYTES);
    });
    if (e0 != hipSuccess) return e0;
    hipLaunchKernelGGL((k_br_mfma<N, ELL, CH>), dim3(A), dim3(64 * GM::WAVES), GM::LDS_BYTES, s, acc, ctN,
                       accs_per_ct, G.n, (const v4i *)brk_frag, G.g_log2B);
    return hipGetLastError();
}

// Instantiations of the batched blind rotation: (N, ell, digit chunks).
#define FDFB_BR_MFMA_CASES(X) \
    X(256, 2, 2)              \
    X(256, 4, 2)              \
    X(1024, 3, 1)             \
    X(2048, 2, 2)             \
    X(2048, 4, 1)

// The blind-rotation kernel of the Karatsuba form for (N, ell, CH): one
// wavefront per accumulator for N <= 1024, else two per output component.
template <int N, int ELL, int CH>
static const void *br_kara_kernel()
{
    if constexpr (BrKara<N, ELL, CH>::WPC == 1) return (const void *)k_br_kara1w<N, ELL, CH>;
    else return (const void *)k_br_kara<N, ELL, CH>;
}
template <int N, int ELL, int CH>
static constexpr int br_kara_threads()
{
    return BrKara<N, ELL, CH>::WPC == 1 ? 64 : 64 * BrKara<N, ELL, CH>::WAVES;
}
// k_br_kara1w2 is instantiated at N = 1024: rounds with more accumulators
// than SIMDs run it with one wavefront per accumulator, rounds of at most one
// accumulator per two SIMDs with two wavefronts per accumulator.
template <int N, int ELL, int CH>
static constexpr bool br_kara_two()
{
    return N == 1024;
}

// Resident capacity of the batched blind rotation on the current device.
struct KaraFit {
    uint32_t cap1 = 0;  // workgroups of br_kara_kernel resident at once
    uint32_t cap2 = 0;  // of k_br_kara1w2<.., 1> (0 when it is not used)
    uint32_t capS = 0;  // of the split form k_br_kara<.., 4> (N = 2048; 0 otherwise)
    uint32_t round() const { return cap2 > cap1 ? cap2 : cap1; }
};

static hipError_t kernel_capacity(const void *k, int threads, size_t lds, int cus, uint32_t *cap)
{
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    int per_cu = 0;
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, threads, lds);
    if (e != hipSuccess) return e;
    *cap = (uint32_t)std::max(1, per_cu) * (uint32_t)cus;
    return hipSuccess;
}

template <int N, int ELL, int CH>
static hipError_t br_kara_fit(KaraFit *out)
{
    using GK = BrKara<N, ELL, CH>;
    static PerDevice<KaraFit> fits;
    return fits.get(out, [](int dev, KaraFit *f) {
        int cus = 0;
        hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = kernel_capacity(br_kara_kernel<N, ELL, CH>(), br_kara_threads<N, ELL, CH>(), GK::LDS_BYTES, cus,
                                &f->cap1);
        if constexpr (GK::WPC == 2)
            if (e == hipSuccess)
                e = kernel_capacity((const void *)k_br_kara<N, ELL, CH, 4>, 512, GK::LDS_BYTES, cus, &f->capS);
        if constexpr (br_kara_two<N, ELL, CH>()) {
            if (e == hipSuccess)
                e = kernel_capacity((const void *)k_br_kara1w2<N, ELL, CH, 1>, 64, GK::LDS2W_BYTES, cus, &f->cap2);
            if (e == hipSuccess)  // attribute only: rounds of WV = 2 are sized from cap1
                e = hipFuncSetAttribute((const void *)k_br_kara1w2<N, ELL, CH, 2>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)GK::LDS2W_BYTES);
        }
        return e;
    });
}

// The kernel a round of cnt accumulators runs under `form`: the fixed rule
// for kFormAuto (see launch_br_kara_t), else the form itself where it exists.
template <int N, int ELL, int CH>
static uint32_t round_form(uint32_t form, uint32_t cnt, const KaraFit &fit)
{
    if constexpr (br_kara_two<N, ELL, CH>()) {
        if (form == kFormAuto) return cnt > fit.cap1 ? kForm1W2 : (2 * cnt <= fit.cap1 ? kForm2W : kForm1W);
        return form;
    } else if constexpr (BrKara<N, ELL, CH>::WPC == 2) {
        // a round whose four wavefronts per accumulator would leave at least half of the
        // SIMDs empty splits each accumulator over eight
        if (form == kFormAuto) return 4 * cnt <= fit.cap1 ? kFormSplit : kForm1W;
        return form == kFormSplit ? kFormSplit : kForm1W;
    } else {
        return kForm1W;
    }
}

// Accumulators per round of a plan: the plan's own round size, else the
// resident capacity of its form (for kFormAuto the larger capacity).
static uint32_t plan_round(const BrPlan &plan, const KaraFit &fit)
{
    if (plan.round) return plan.round;
    switch (plan.form) {
    case kForm1W: return fit.cap1;
    case kForm1W2: return fit.cap2 ? fit.cap2 : fit.cap1;
    case kForm2W: return std::max(1u, fit.cap1 / 2);
    case kFormSplit: return fit.capS ? fit.capS : fit.cap1;
    default: return fit.round();
    }
}

template <int N, int ELL, int CH>
static hipError_t launch_br_kara_t(const Geometry &G, uint32_t *acc, const uint32_t *ctN, uint32_t A,
                                   uint32_t accs_per_ct, const void *brk_frag, const uint32_t *corr,
                                   const BrPlan &plan, hipStream_t s)
{
    using GK = BrKara<N, ELL, CH>;
    // Launch in rounds of the resident capacity: the workgroups of one launch
    // start together and walk the key in step, so a key block is fetched into
    // each XCD's L2 once and shared, where a second round started by
    // completions would drift and re-fetch.  A round may begin inside a
    // sample's group of accumulators (a_base), so no round is left short.
    // The fixed rule (kFormAuto) by round size: at N = 1024, more accumulators
    // than one wavefront per SIMD holds run two wavefronts per SIMD
    // (k_br_kara1w2 with one wavefront per accumulator), a round that gives
    // every wavefront of two per accumulator a SIMD runs those, the rest one
    // wavefront per SIMD; at N = 2048 a round of at most a quarter of the
    // capacity runs the split form (eight wavefronts per accumulator).
    KaraFit fit;
    hipError_t e0 = br_kara_fit<N, ELL, CH>(&fit);
    if (e0 != hipSuccess) return e0;
    const uint32_t R = plan_round(plan, fit);
    for (uint32_t a0 = 0; a0 < A; a0 += R) {
        const uint32_t cnt = std::min(R, A - a0);
        const uint32_t form = round_form<N, ELL, CH>(plan.form, cnt, fit);
        if constexpr (br_kara_two<N, ELL, CH>()) {
            if (form == kForm1W2)
                hipLaunchKernelGGL((k_br_kara1w2<N, ELL, CH, 1>), dim3(cnt), dim3(64), GK::LDS2W_BYTES, s, acc,
                                   ctN, a0, accs_per_ct, G.n, (const v4i *)brk_frag, corr, G.g_log2B);
            else if (form == kForm2W)
                hipLaunchKernelGGL((k_br_kara1w2<N, ELL, CH, 2>), dim3(cnt), dim3(128), GK::LDS2W_BYTES, s, acc,
                                   ctN, a0, accs_per_ct, G.n, (const v4i *)brk_frag, corr, G.g_log2B);
        }
        if constexpr (GK::WPC == 2)
            if (form == kFormSplit)
                hipLaunchKernelGGL((k_br_kara<N, ELL, CH, 4>), dim3(cnt), dim3(512), GK::LDS_BYTES, s, acc, ctN, a0,
                                   accs_per_ct, G.n, (const v4i *)brk_frag, corr, G.g_log2B);
        if (form == kForm1W) {
            if constexpr (GK::WPC == 1)
                hipLaunchKernelGGL((k_br_kara1w<N, ELL, CH>), dim3(cnt), dim3(64), GK::LDS_BYTES, s, acc, ctN, a0,
                                   accs_per_ct, G.n, (const v4i *)brk_frag, corr, G.g_log2B);
            else
                hipLaunchKernelGGL((k_br_kara<N, ELL, CH>), dim3(cnt), dim3(64 * GK::WAVES), GK::LDS_BYTES, s, acc,
                                   ctN, a0, accs_per_ct, G.n, (const v4i *)brk_frag, corr, G.g_log2B);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Geometries of the persistent work-queue kernel: narrow (one wavefront per
// accumulator) and wide (four), and the pairs it is instantiated for.
#define FDFB_QUEUE_NARROW(X) X(1024, 3, 1) X(256, 2, 2)
#define FDFB_QUEUE_WIDE(X) X(2048, 2, 2) X(2048, 4, 1)

struct QueueKey {
    int N, ell, ch;
    bool operator==(const QueueKey &o) const { return N == o.N && ell == o.ell && ch == o.ch; }
};
static QueueKey queue_key(const Geometry &G) { return {G.N, G.g_ell, digit_chunks(G.g_log2B)}; }
static bool queue_narrow(const QueueKey &k)
{
#define X(n_, l_, c_) if (k.N == n_ && k.ell == l_ && k.ch == c_) return true;
    FDFB_QUEUE_NARROW(X)
#undef X
    return false;
}
static bool queue_wide(const QueueKey &k)
{
#define X(n_, l_, c_) if (k.N == n_ && k.ell == l_ && k.ch == c_) return true;
    FDFB_QUEUE_WIDE(X)
#undef X
    return false;
}

bool br_queue_supported(const Geometry &G)
{
    const QueueKey k = queue_key(G);
    return queue_narrow(k) || queue_wide(k);
}

// Resident workgroups of one k_br_queue instantiation on the current device.
template <int NA, int LA, int CA, int NB, int LB, int CB>
static hipError_t br_queue_capacity(uint32_t *cap)
{
    using Q = BrQueueGeom<NA, LA, CA, NB, LB, CB>;
    static PerDevice<uint32_t> caps;
    return caps.get(cap, [](int dev, uint32_t *c) {
        int cus = 0;
        hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = kernel_capacity((const void *)k_br_queue<NA, LA, CA, NB, LB, CB>, 256, Q::LDS, cus, c);
        return e;
    });
}

// One launch group: a narrow and a wide geometry and the jobs of either.
struct QueueGroup {
    QueueKey narrow{0, 0, 0}, wide{0, 0, 0};
    std::vector<int> jobs;
};

static std::vector<QueueGroup> queue_groups(const BrJobDesc *jobs, int njobs)
{
    std::vector<QueueKey> nk, wk;
    for (int j = 0; j < njobs; ++j) {
        if (!jobs[j].A) continue;
        const QueueKey k = queue_key(jobs[j].G);
        auto &v = queue_wide(k) ? wk : nk;
        if (std::find(v.begin(), v.end(), k) == v.end()) v.push_back(k);
    }
    std::vector<QueueGroup> groups;
    const size_t pairs = std::max(nk.size(), wk.size());
    for (size_t g = 0; g < pairs; ++g) {
        // keys pair up in order; a class with fewer keys lends its first key
        // (whose body then simply gets no items)
        QueueKey a = g < nk.size() ? nk[g] : QueueKey{1024, 3, 1};
        QueueKey b = g < wk.size() ? wk[g] : QueueKey{2048, 2, 2};
        // wide jobs first, so that the longer items start first
        std::vector<int> mine;
        for (int pass = 0; pass < 2; ++pass)
            for (int j = 0; j < njobs; ++j) {
                if (!jobs[j].A) continue;
                const QueueKey k = queue_key(jobs[j].G);
                if ((pass == 0 && g < wk.size() && k == b) || (pass == 1 && g < nk.size() && k == a))
                    mine.push_back(j);
            }
        for (size_t lo = 0; lo < mine.size(); lo += kQueueJobs) {
            QueueGroup qg;
            qg.narrow = a;
            qg.wide = b;
            qg.jobs.assign(mine.begin() + lo, mine.begin() + std::min(mine.size(), lo + kQueueJobs));
            groups.push_back(qg);
        }
    }
    return groups;
}

hipError_t br_queue_launches(const BrJobDesc *jobs, int njobs, uint32_t *launches)
{
    for (int j = 0; j < njobs; ++j)
        if (jobs[j].A && !br_queue_supported(jobs[j].G)) return hipErrorInvalidValue;
    *launches = (uint32_t)queue_groups(jobs, njobs).size();
    return hipSuccess;
}

template <int NA, int LA, int CA, int NB, int LB, int CB>
static hipError_t launch_queue_t(const BrQueue &q, uint32_t *counter, hipStream_t s)
{
    using Q = BrQueueGeom<NA, LA, CA, NB, LB, CB>;
    uint32_t cap = 0;
    hipError_t e = br_queue_capacity<NA, LA, CA, NB, LB, CB>(&cap);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, s, counter, 1u, 0u);
    hipLaunchKernelGGL((k_br_queue<NA, LA, CA, NB, LB, CB>), dim3(std::min(cap, q.items)), dim3(256), Q::LDS, s, q,
                       counter);
    return hipGetLastError();
}

hipError_t launch_br_queue(const BrJobDesc *jobs, int njobs, uint32_t *counters, uint32_t ncounters,
                           hipStream_t s)
{
    for (int j = 0; j < njobs; ++j)
        if (jobs[j].A && !br_queue_supported(jobs[j].G)) return hipErrorInvalidValue;
    const std::vector<QueueGroup> groups = queue_groups(jobs, njobs);
    if (groups.size() > ncounters) return hipErrorInvalidValue;
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        const QueueGroup &qg = groups[gi];
        BrQueue q{};
        uint32_t items = 0;
        for (int j : qg.jobs) {
            const BrJobDesc &d = jobs[j];
            const bool wide = d.G.N > 1024;
            BrQueueJob &J = q.job[q.njobs++];
            J.acc = d.acc;
            J.ctN = d.ctN;
            J.bfrag = d.bfrag;
            J.corr = d.corr;
            J.accs = d.A;
            J.per = d.per;
            J.n = (uint32_t)d.G.n;
            J.log2B = (uint32_t)d.G.g_log2B;
            J.wide = wide;
            J.first_item = items;
            items += wide ? d.A : (d.A + 3) / 4;
        }
        q.items = items;
        if (!items) continue;
        hipError_t e = hipErrorInvalidValue;
        bool found = false;
#define XW(nb_, lb_, cb_)                                                                              \
    if (!found && qg.wide == QueueKey{nb_, lb_, cb_}) {                                                 \
        found = true;                                                                                  \
        e = launch_queue_t<na_, la_, ca_, nb_, lb_, cb_>(q, counters + gi, s);                         \
    }
#define XN(n_, l_, c_)                                                                                 \
    if (!found && qg.narrow == QueueKey{n_, l_, c_}) {                                                  \
        constexpr int na_ = n_, la_ = l_, ca_ = c_;                                                    \
        FDFB_QUEUE_WIDE(XW)                                                                            \
    }
        FDFB_QUEUE_NARROW(XN)
#undef XN
#undef XW
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

bool br_mfma_supported(const Geometry &G)
{
    const int ch = digit_chunks(G.g_log2B);
#define X(n_, l_, c_) if (G.N == n_ && G.g_ell == l_ && ch == c_) return true;
    FDFB_BR_MFMA_CASES(X)
#undef X
    return false;
}

hipError_t br_queue_slots(const BrJobDesc *jobs, int njobs, uint32_t *items)
{
    for (int j = 0; j < njobs; ++j)
        if (jobs[j].A && !br_queue_supported(jobs[j].G)) return hipErrorInvalidValue;
    uint32_t best = 0;
    for (const QueueGroup &qg : queue_groups(jobs, njobs)) {
        uint32_t cap = 0;
        hipError_t e = hipErrorInvalidValue;
        bool found = false;
#define XW(nb_, lb_, cb_)                                                                              \
    if (!found && qg.wide == QueueKey{nb_, lb_, cb_}) {                                                 \
        found = true;                                                                                  \
        e = br_queue_capacity<na_, la_, ca_, nb_, lb_, cb_>(&cap);                                     \
    }
#define XN(n_, l_, c_)                                                                                 \
    if (!found && qg.narrow == QueueKey{n_, l_, c_}) {                                                  \
        constexpr int na_ = n_, la_ = l_, ca_ = c_;                                                    \
        FDFB_QUEUE_WIDE(XW)                                                                            \
    }
        FDFB_QUEUE_NARROW(XN)
#undef XN
#undef XW
        if (e != hipSuccess) return e;
        best = best ? std::min(best, cap) : cap;
    }
    *items = best;
    return hipSuccess;
}

hipError_t launch_br_mfma(const Geometry &G, uint32_t *acc, const uint32_t *ctN, uint32_t A,
                          uint32_t accs_per_ct, const void *brk_frag, hipStream_t s)
{
    if (!A) return hipSuccess;
    const int ch = digit_chunks(G.g_log2B);
#define X(n_, l_, c_) \
    if (G.N == n_ && G.g_ell == l_ && ch == c_) return launch_br_mfma_t<n_, l_, c_>(G, acc, ctN, A, accs_per_ct, brk_frag, s);
    FDFB_BR_MFMA_CASES(X)
#undef X
    return hipErrorInvalidValue;
}

static hipError_t fit_of(const Geometry &G, KaraFit *fit)
{
    const int ch = digit_chunks(G.g_log2B);
#define X(n_, l_, c_) \
    if (G.N == n_ && G.g_ell == l_ && ch == c_) return br_kara_fit<n_, l_, c_>(fit);
    FDFB_BR_MFMA_CASES(X)
#undef X
    return hipErrorInvalidValue;
}

bool br_plan_valid(const Geometry &G, const BrPlan &plan)
{
    if (!br_mfma_supported(G)) return false;
    switch (plan.form) {
    case kFormAuto:
    case kForm1W: return true;
    case kForm1W2:
    case kForm2W: return G.N == 1024 && G.g_ell == 3 && digit_chunks(G.g_log2B) == 1;
    case kFormQueue: return br_queue_supported(G) && plan.round == 0;
    case kFormSplit: return G.N > 1024;
    default: return false;
    }
}

int br_plan_candidates(const Geometry &G, BrPlan *out, int max)
{
    const BrPlan all[] = {{kFormAuto, 0}, {kForm1W, 0}, {kForm1W2, 0}, {kForm2W, 0}, {kFormQueue, 0}, {kFormSplit, 0}};
    int k = 0;
    KaraFit fit;
    const bool have_fit = fit_of(G, &fit) == hipSuccess;
    for (const BrPlan &p : all) {
        if (!br_plan_valid(G, p)) continue;
        if (k < max) out[k] = p;
        ++k;
        // the same form in rounds of half its capacity (more rounds, fewer
        // workgroups walking the key together)
        if (have_fit && (p.form == kForm1W || p.form == kForm1W2 || p.form == kFormSplit)) {
            const uint32_t half = plan_round(p, fit) / 2;
            if (half) {
                if (k < max) out[k] = BrPlan{p.form, half};
                ++k;
            }
        }
    }
    return k;
}

hipError_t br_kara_launches(const Geometry &G, uint32_t A, uint32_t accs_per_ct, const BrPlan &plan,
                            uint32_t *launches)
{
    *launches = 0;
    if (!A) return hipSuccess;
    if (plan.form == kFormQueue) {
        *launches = 1;
        return hipSuccess;
    }
    (void)accs_per_ct;  // a round may split a sample's accumulators
    KaraFit fit;
    hipError_t e = fit_of(G, &fit);
    if (e != hipSuccess) return e;
    const uint32_t R = plan_round(plan, fit);
    *launches = (A + R - 1) / R;
    return hipSuccess;
}

hipError_t launch_br_kara(const Geometry &G, uint32_t *acc, const uint32_t *ctN, uint32_t A,
                          uint32_t accs_per_ct, const void *brk_frag, const uint32_t *corr, const BrPlan &plan,
                          uint32_t *work, hipStream_t s)
{
    if (!A) return hipSuccess;
    if (!br_plan_valid(G, plan)) return hipErrorInvalidValue;
    if (plan.form == kFormQueue) {
        if (!work) return hipErrorInvalidValue;
        BrJobDesc d;
        d.G = G;
        d.acc = acc;
        d.ctN = ctN;
        d.A = A;
        d.per = accs_per_ct;
        d.bfrag = brk_frag;
        d.corr = corr;
        return launch_br_queue(&d, 1, work, 1, s);
    }
    const int ch = digit_chunks(G.g_log2B);
#define X(n_, l_, c_) \
    if (G.N == n_ && G.g_ell == l_ && ch == c_) \
        return launch_br_kara_t<n_, l_, c_>(G, acc, ctN, A, accs_per_ct, brk_frag, corr, plan, s);
    FDFB_BR_MFMA_CASES(X)
#undef X
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Static scratch of the allocation-free bootstrap: one buffer per GPU, part
// of the code object, so it exists from library load until the process
// ends.  Host code must never pass `scratch` itself to a kernel (in host code
// it names a host-side stand-in); it uses the device address looked up once
// per device with hipGetSymbolAddress.
// ---------------------------------------------------------------------------
static __device__ __align__(256) uint8_t scratch[kNoallocScratchBytes];

hipError_t noalloc_scratch(void **ptr)
{
    static PerDevice<void *> addr;
    return addr.get(ptr, [](int, void **out) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        *out = p;
        return hipSuccess;
    });
}

}  // namespace fdfbk
