/*
 * fdfb.h -- C ABI of the MI355X full-domain functional bootstrapping library.
 *
 * The library computes the full-domain functional bootstrap of Kluczniak &
 * Schild (arXiv 2109.02731, Sec. 3.2, Fig. 2 "Bootstrap") over LWE / RLWE
 * samples with ciphertext modulus q = Q = 2^32: every coefficient is a
 * uint32_t and arithmetic wraps mod 2^32.  The GLWE rank is 1 (RLWE).
 *
 * Conventions shared by every entry point
 *  - Return value: 0 on success or a negative FDFB_E* code.  No entry point
 *    aborts the process; the text of the last error of the calling thread is
 *    returned by fdfb_last_error().
 *  - LWE samples are stored [b, a_1 .. a_d] (b first, Sec. 2 Def. "Generalized
 *    Learning With Errors"), row-major, one row per sample.
 *  - RLWE samples are stored [b_0 .. b_{N-1}, a_0 .. a_{N-1}].
 *  - "d_" pointers are device (HBM) pointers owned by the caller, valid on the
 *    given stream; "host" pointers are ordinary host memory.  `stream` is a
 *    hipStream_t passed as void* (NULL = the null stream).  Device work is
 *    enqueued asynchronously on `stream`; the call returns once it is queued.
 *  - A context (fdfb_ctx) owns the evaluation keys in device memory and the
 *    secret keys in host memory (for the *_debug calls).  Every call on a
 *    context takes the context's lock, so any thread may call at any time;
 *    calls that enqueue device work are ordered on their own streams only.
 *    Distinct contexts are independent.
 *  - Device scratch of direct calls comes from a pool per (context, stream):
 *    calls on one stream reuse its block in stream order, calls on different
 *    streams never share one.  A block that must grow is replaced, and the
 *    replaced block stays allocated until fdfb_release_scratch or fdfb_free,
 *    so work already enqueued or captured in a HIP graph never reads freed
 *    memory.
 *  - Results are bit-identical for identical inputs whatever the batch size,
 *    batch composition, kernel form (Karatsuba, direct or plain) or stream.
 */
#ifndef FDFB_H
#define FDFB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FDFB_OK 0
#define FDFB_EINVAL (-1)   /* invalid argument or parameter set            */
#define FDFB_ENOMEM (-2)   /* host or device allocation failed             */
#define FDFB_EDEVICE (-3)  /* a HIP runtime call failed (text in last_error) */
#define FDFB_EABORTED (-4) /* the host abort flag was raised               */
#define FDFB_ENOTSUP (-5)  /* parameter set not supported by the kernels   */

/* flags of fdfb_bootstrap_batch / fdfb_blind_rotate */
#define FDFB_OUT_EXTRACTED 0x1u /* return c_Q (dimension N, key s_F) instead of
                                   the key-switched sample (Sec. 3.4, "Computing
                                   in Z_t": affine maps on c_Q before switching) */
#define FDFB_PLAIN 0x2u         /* run the plain one-sample-per-workgroup
                                   VALU kernels instead of the batched MFMA ones */
#define FDFB_DIRECT 0x4u        /* batched MFMA blind rotation without the
                                   Karatsuba split: one N-size Toeplitz product
                                   per digit row (a comparison form with the same
                                   results; its key layout is built on first use).
                                   Exclusive with FDFB_PLAIN (FDFB_EINVAL). */

/*
 * Parameter set.  q = Q = 2^32 is fixed.  Gadget bases are powers of two,
 * L = 2^log2B; when ell*log2B < 32 the gadget is g_j = 2^(32-ell*log2B) L^(j-1)
 * and values are rounded (half up) to their top ell*log2B bits before the
 * unsigned digit decomposition (Sec. 2 Def. "Decomposition").
 *   n, N      LWE dimension and ring degree (N a power of two, 64..2048)
 *   log2_t    plaintext modulus t = 2^log2_t, 2 <= t <= N
 *   g_*       blind-rotation key gadget (L_RGSW)
 *   ks_*      key switching key LWE(s_F, N) -> LWE(s, n)
 *   pk_*      packing key LWE(s_F, N) -> RLWE(s_F)
 *   boot_*    public-mux digits: base L_boot, ell_boot = ceil(log_Lboot t);
 *             boot_log2B = 0 with boot_ell = 1 (t <= 128) selects one signed
 *             digit in [-t/2, t/2): one sign rotation per bootstrap
 *   sigma_*   noise standard deviations in units of 1 (q = 2^32): fresh LWE
 *             samples, blind-rotation key, packing key, key switching key
 */
typedef struct fdfb_params {
    uint32_t n, N, log2_t;
    uint32_t g_log2B, g_ell;
    uint32_t ks_log2B, ks_ell;
    uint32_t pk_log2B, pk_ell;
    uint32_t boot_log2B, boot_ell;
    double sigma_lwe, sigma_glwe, sigma_pk, sigma_ks;
} fdfb_params;

typedef struct fdfb_ctx fdfb_ctx;

/*
 * Key generation from a 64-bit seed (Sec. 3.2 Theorem "Correctness of the
 * Bootstrapping": brK = BRKeyGen(s, 𝔰), pK = KeySwitchSetup(s_F -> 𝔰),
 * ksK = KeySwitchSetup(s_F -> s); App. A Figs. "BRKeyGen", "KeySwitchSetup").
 * Secrets s in {0,1}^n and 𝔰 in {0,1}^N are uniform binary; s_F = Coefs(𝔰).
 * Randomness: counter-based SplitMix64 (one stream per purpose) and rounded
 * Box-Muller Gaussians; the exact stream layout is fixed so that any
 * implementation of the same definition reproduces the keys bit for bit.
 * Host only: no device memory is touched until the first device call.
 * On success *out owns the new context (release with fdfb_free).
 * Errors: FDFB_EINVAL for an unsupported parameter set, FDFB_ENOMEM.
 */
int fdfb_keygen_from_seed(const fdfb_params *params, uint64_t seed, fdfb_ctx **out);

/*
 * Register a lookup table f: Z_t -> Z_t (host array table[t], values in
 * [0, t)) and build its rotation polynomials rotP_0, rotP_1 (Sec. 3.3,
 * Fig. 2 "SetupPolynomial"; the table is stored unscaled, Delta = 2^32/t is
 * applied once inside the public mux).  *lut_id receives a small index
 * (0, 1, 2, ...) used by fdfb_bootstrap_batch.  Errors: FDFB_EINVAL when a
 * value is >= t, FDFB_ENOMEM.
 */
int fdfb_register_lut(fdfb_ctx *ctx, const uint32_t *table, int32_t *lut_id);

/*
 * Full-domain functional bootstrap of B LWE samples (Sec. 3.2, Fig. 2):
 * ModSwitch to Z_2N; ell_boot sign blind rotations; SampleExtract;
 * BuildAcc = packing key switch + public mux of rotP_1 X^b / rotP_0 X^b
 * (Sec. 3.1, Fig. 1); the function blind rotation; SampleExtract; the final
 * key switch (ModSwitch Q -> q is the identity since Q = q).
 *   d_cts      device uint32[B][n+1], inputs under s
 *   d_lut_ids  device int32[B], each a registered lut_id
 *   d_out      device uint32[B][n+1] (under s), or uint32[B][N+1] (under
 *              s_F) when FDFB_OUT_EXTRACTED is set
 *   flags      FDFB_OUT_EXTRACTED | FDFB_PLAIN | FDFB_DIRECT (FDFB_ENOTSUP when the plain form
 *              cannot hold the parameter set, e.g. N = 2048 with ell = 4)
 * Scratch comes from the context's block for `stream`, replaced by a larger
 * one (hipMalloc) the first time a larger B is seen on that stream.  B = 0 is
 * a no-op.  After one call with at least this B on the same stream (keys
 * uploaded, scratch sized), the call enqueues kernels only and can be
 * captured into a HIP graph; a graph replays into the scratch block of the
 * stream it was captured on, so replays must not overlap other calls on
 * that stream.
 * Errors: FDFB_EINVAL (null pointer with B > 0), FDFB_ENOMEM, FDFB_EDEVICE,
 * FDFB_EABORTED.  lut_ids are read on the device: an id that is not a
 * registered table gives that sample an all-zero accumulator (its output is
 * not a bootstrap of anything) and sets FDFB_DEVERR_LUT_ID in the context's
 * device error bits (fdfb_device_errors).
 */
int fdfb_bootstrap_batch(fdfb_ctx *ctx, const uint32_t *d_cts, const int32_t *d_lut_ids,
                         uint32_t B, uint32_t *d_out, uint32_t flags, void *stream);

/*
 * Same as fdfb_bootstrap_batch, for callers that cannot allocate memory
 * (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc): the scratch lives in one static device buffer of the library
 * (FDFB_NOALLOC_SCRATCH_BYTES per GPU, held from library load until the
 * process ends) instead of the context's pool, and the call makes no
 * allocation of any kind.  Inputs, outputs, flags and results are those of
 * fdfb_bootstrap_batch, bit for bit.  Limits and errors:
 *  - the context must already be prepared for these flags (keys, every
 *    registered table and, with FDFB_DIRECT, the direct key layout resident
 *    on the device, e.g. by one earlier fdfb_bootstrap_batch or by
 *    fdfb_prepare): FDFB_EINVAL otherwise;
 *  - fdfb_noalloc_max_batch gives the largest B whose scratch fits the
 *    buffer; a larger B is FDFB_EINVAL (nothing is enqueued);
 *  - every call on a GPU shares that GPU's buffer: calls whose device work
 *    may overlap (different streams without ordering, or replays of graphs
 *    that captured this call) race and give undefined results.  Calls in one
 *    stream's order are safe.  No part of the buffer needs to start at zero.
 */
#define FDFB_NOALLOC_SCRATCH_BYTES (64u << 20)
int fdfb_bootstrap_batch_noalloc(fdfb_ctx *ctx, const uint32_t *d_cts, const int32_t *d_lut_ids,
                                 uint32_t B, uint32_t *d_out, uint32_t flags, void *stream);

/* Largest B fdfb_bootstrap_batch_noalloc accepts for this context's
 * parameter set (host only, no device call). */
int fdfb_noalloc_max_batch(const fdfb_ctx *ctx, uint32_t *max_B);

/* Upload everything a call with these flags needs (keys, registered tables,
 * the direct key layout for FDFB_DIRECT) without enqueuing work, so that
 * later calls only enqueue kernels.  Errors: FDFB_ENOMEM, FDFB_EDEVICE. */
int fdfb_prepare(fdfb_ctx *ctx, uint32_t flags);

/*
 * Several functions of one input (Sec. "Application of Functional
 * Bootstrapping", multiple univariate functions with the same input: the
 * sign accumulators depend on the input only, so they are computed once and
 * reused by every table):
 * for each sample, ell_boot sign blind rotations, then per table a public
 * mux and a function blind rotation.  ell_boot + L blind rotations per
 * sample instead of L (ell_boot + 1).
 *   d_lut_ids  int32 [B][L], table l of sample b at b L + l
 *   d_out      uint32 [B][L][n+1] (or [B][L][N+1] with FDFB_OUT_EXTRACTED);
 *              output (b, l) is bit-identical to fdfb_bootstrap_batch of
 *              sample b with table d_lut_ids[b L + l]
 * L = 0 is FDFB_EINVAL; B = 0 is a no-op.  Scratch grows with B L.  Other
 * arguments and errors as fdfb_bootstrap_batch.
 */
int fdfb_bootstrap_multi_lut(fdfb_ctx *ctx, const uint32_t *d_cts, const int32_t *d_lut_ids, uint32_t B,
                             uint32_t L, uint32_t *d_out, uint32_t flags, void *stream);

/*
 * TFHE-style half-domain bootstrap (App. A Fig. "TFHE Bootstrapping"), the
 * one-rotation yardstick for FDFB on the same kernels: acc = [Delta rotP_0
 * X^{b_N}, 0] with rotP_0 of the sample's registered table, one blind
 * rotation, SampleExtract, then the key switch (or the extracted sample with
 * FDFB_OUT_EXTRACTED).  The result encrypts f(m) only for m < t/2; for
 * m >= t/2 it encrypts -f(m - t/2), the limitation the full-domain bootstrap
 * removes.  Arguments, layouts and errors as fdfb_bootstrap_batch.
 */
int fdfb_tfhe_bootstrap_batch(fdfb_ctx *ctx, const uint32_t *d_cts, const int32_t *d_lut_ids, uint32_t B,
                              uint32_t *d_out, uint32_t flags, void *stream);

/* One job of fdfb_bootstrap_multi: a batch on its own context (its own
 * parameter set, e.g. a different N). */
typedef struct fdfb_job {
    fdfb_ctx *ctx;
    const uint32_t *d_cts;
    const int32_t *d_lut_ids;
    uint32_t B;
    uint32_t *d_out;
    uint32_t flags;
} fdfb_job;

/*
 * Bootstrap several jobs (mixed parameter sets, ring degrees and lookup
 * tables; up to 256 jobs) as one stream-ordered submission, phase by phase
 * (Fig. 2's steps for all jobs together).  The blind rotations of every job
 * in the default (Karatsuba) form whose geometry the persistent kernel takes
 * (N = 1024 with gadget 2^7 x 3 or N = 256 with 2^8 x 2, together with
 * N = 2048 with 2^10 x 2 or 2^7 x 4) run in one persistent work-queue launch
 * per phase and pair of geometries (16 jobs per launch): resident
 * workgroups pull (job, accumulators) items from a device counter until
 * the queue is empty.  Other jobs rotate in their own launches.  The queue
 * is used when eligible jobs span more than one context (a single context's
 * rotations already fill the device).  Outputs are bit-identical to
 * fdfb_bootstrap_batch on each job.  Every job is validated before anything
 * is enqueued.  Scratch: one block per context and stream, each job of the
 * context at its own offset.  Errors as fdfb_bootstrap_batch, and
 * FDFB_EINVAL for more than 256 jobs.
 */
int fdfb_bootstrap_multi(const fdfb_job *jobs, uint32_t njobs, void *stream);

/* fdfb_bootstrap_multi with the rotation form chosen by the caller:
 * use_queue = 1 puts every eligible job in the persistent queue, 0 rotates
 * each job in its own launches, -1 is fdfb_bootstrap_multi's rule.  The
 * outputs are the same bits either way. */
int fdfb_bootstrap_multi_ex(const fdfb_job *jobs, uint32_t njobs, int use_queue, void *stream);

/*
 * Bootstrap a sequence of jobs (batches) as a software pipeline on one
 * stream: job k's function rotation shares persistent work-queue launches
 * with the sign rotations of the jobs after it, so that every launch holds
 * whole rounds of the kernel's resident capacity (two wavefronts per SIMD)
 * although one batch's function rotation alone fills only half of it.  Each
 * launch takes the function rotations of the jobs whose public mux is
 * enqueued, then the next jobs' sign rotations in job order (a job's may be
 * split between launches at whole samples) up to `rounds` rounds of the
 * resident capacity (0: 4; at most 64); the jobs' outputs follow the launch
 * that rotates them, in job order.  The steps of each job are those of
 * Fig. 2 (Sec. 3.2) and its outputs are bit-identical to
 * fdfb_bootstrap_batch on the job.  Every job's blind rotations must be in
 * the default form and of a geometry the persistent kernel takes (see
 * fdfb_bootstrap_multi): FDFB_EINVAL otherwise, before anything is enqueued.
 * Scratch, limits and other errors as fdfb_bootstrap_multi.
 */
int fdfb_bootstrap_pipeline(const fdfb_job *jobs, uint32_t njobs, uint32_t rounds, void *stream);

/*
 * A multi-job submission captured once into a HIP graph and replayed with one
 * launch (hipGraphLaunch): the whole bootstrap of every job, with the
 * persistent work-queue rotations (use_queue as in fdfb_bootstrap_multi_ex).
 * The graph owns its scratch (allocated here); the jobs' buffers, contexts
 * and registered tables must stay valid while the graph exists, and each
 * replay reads the jobs' inputs and writes their outputs at the pointers
 * given here.  Creation runs the submission once eagerly on a private stream
 * (setting every kernel's attributes) before capturing it, so the outputs
 * are written by then.  Replays of one graph must not overlap each other
 * (they share its scratch).  Errors: as fdfb_bootstrap_multi, FDFB_EDEVICE
 * when capture or instantiation fails.
 */
typedef struct fdfb_graph fdfb_graph;
int fdfb_multi_graph_create(const fdfb_job *jobs, uint32_t njobs, int use_queue, fdfb_graph **out);
/* Replay the graph on `stream` (one graph launch).  FDFB_EABORTED if a job's
 * context has its abort flag raised. */
int fdfb_graph_launch(fdfb_graph *graph, void *stream);
/* Whether the graph's rotations use the persistent queue, and its scratch bytes. */
int fdfb_graph_info(const fdfb_graph *graph, uint32_t *uses_queue, size_t *scratch_bytes);
/* Wait for the device, then release the graph and its scratch (NULL is a no-op). */
void fdfb_graph_free(fdfb_graph *graph);

/*
 * LWE -> LWE key switch with ksK (App. A Fig. "KeySwitch"):
 * d_in uint32[B][N+1] under s_F -> d_out uint32[B][n+1] under s.
 */
int fdfb_keyswitch(fdfb_ctx *ctx, const uint32_t *d_in, uint32_t B, uint32_t *d_out, void *stream);

/* Free every scratch block of the context, current and replaced (waits for
 * the whole device first).  HIP graphs that captured calls on this context
 * must not be replayed afterwards: their scratch is gone. */
int fdfb_release_scratch(fdfb_ctx *ctx);

/* Device error bits of the context (FDFB_DEVERR_*), set by kernels on
 * invalid data found on the device (e.g. an unregistered lut_id).  Waits for
 * the whole device, stores the bits in *bits and clears them if `clear`.
 * Errors: FDFB_EINVAL on null pointers, FDFB_EDEVICE. */
#define FDFB_DEVERR_LUT_ID 0x1u
int fdfb_device_errors(fdfb_ctx *ctx, int clear, uint32_t *bits);

/* ---- single procedures of the path, for tests and custom pipelines ----- */

/* ModSwitch(ct, q, 2N) of every coordinate (App. A Fig. "ModSwitch"):
 * d_cts uint32[B][n+1] -> d_ctN uint32[B][n+1] with values in [0, 2N). */
int fdfb_modswitch(fdfb_ctx *ctx, const uint32_t *d_cts, uint32_t B, uint32_t *d_ctN, void *stream);

/*
 * BlindRotate (App. A Fig. "Blind Rotation", u = {1}): for every accumulator
 * a in [A], acc_a <- CMux(brK[i], acc_a X^(-a_i), acc_a) for i = 1..n, where
 * a_i comes from row (a / accs_per_ct) of d_ctN.  d_acc uint32[A][2][N] is
 * updated in place; d_ctN uint32[A/accs_per_ct][n+1] (values in [0, 2N)).
 * flags: FDFB_PLAIN selects the VALU kernel, FDFB_DIRECT the MFMA kernel
 * without the Karatsuba split.
 */
int fdfb_blind_rotate(fdfb_ctx *ctx, uint32_t *d_acc, const uint32_t *d_ctN, uint32_t A,
                      uint32_t accs_per_ct, uint32_t flags, void *stream);

/* SampleExtract(acc, 1) (App. A Fig. "SampleExtract"):
 * d_acc uint32[A][2][N] -> d_lwe uint32[A][N+1]. */
int fdfb_sample_extract(fdfb_ctx *ctx, const uint32_t *d_acc, uint32_t A, uint32_t *d_lwe,
                        void *stream);

/* LWE -> RLWE key switch with the packing key pK (App. A Fig. "KeySwitch"):
 * d_in uint32[A][N+1] under s_F -> d_out uint32[A][2][N] under 𝔰. */
int fdfb_packing_keyswitch(fdfb_ctx *ctx, const uint32_t *d_in, uint32_t A, uint32_t *d_out,
                           void *stream);

/*
 * PubMux (Sec. 3.1 Fig. 1) of the bootstrap: for every sample b,
 * acc_b = [Delta p_A, 0] + sum_i digit_i((p_B - p_A) mod t) * R_{b,i} with
 * p_A = rotP_1 X^(b_N), p_B = rotP_0 X^(b_N) of lut d_lut_ids[b] and b_N the
 * first entry of row b of d_ctN.  d_rlwe uint32[B][ell_boot][2][N],
 * d_acc uint32[B][2][N].
 */
int fdfb_pubmux(fdfb_ctx *ctx, const uint32_t *d_rlwe, const uint32_t *d_ctN,
                const int32_t *d_lut_ids, uint32_t B, uint32_t *d_acc, void *stream);

/*
 * Affine map on LWE samples (Sec. 2 Lemma "Linear Homomorphism of GLWE
 * samples"; Sec. 3.4 "Computing in Z_t"): out[r] = sum_c W[r][c] * in[c]
 * (mod 2^32) coordinate-wise, with no bootstrap.
 *   d_W    device int32[rows][cols] weights
 *   d_in   device uint32[cols][width] samples (width = dimension + 1)
 *   d_out  device uint32[rows][width]
 * Needs no context.  Errors: FDFB_EINVAL for null buffers with rows > 0.
 */
int fdfb_affine(const int32_t *d_W, const uint32_t *d_in, uint32_t rows, uint32_t cols, uint32_t width,
                uint32_t *d_out, void *stream);

/* Pairwise linear combination of LWE samples (same Lemma):
 * d_out[b] = wx d_x[b] + wy d_y[b] (mod 2^32), coordinate-wise, for B
 * samples of `width` words each (d_x and d_y may alias).  Needs no context.
 * Errors: FDFB_EINVAL for null buffers or B * width >= 2^32. */
int fdfb_lincomb2(const uint32_t *d_x, const uint32_t *d_y, int32_t wx, int32_t wy, uint32_t B, uint32_t width,
                  uint32_t *d_out, void *stream);

/* ---- debug helpers (host memory, use the secret keys) ------------------ */

/* Encrypt B messages m[b] in [0, t) under s: b = <a, s> + Delta m + e with a
 * uniform and e ~ round(N(0, sigma_lwe^2)) drawn from `seed` (sample b uses
 * counter range b).  cts_host uint32[B][n+1]. */
int fdfb_encrypt_debug(fdfb_ctx *ctx, const uint32_t *m, uint32_t B, uint64_t seed,
                       uint32_t *cts_host);

/* Decrypt B samples of dimension dim (n: key s; N: key s_F):
 * m_out[b] = round(t * phase / 2^32) mod t (Sec. 1.2 "Regev Encryption");
 * err_out (nullable) receives the centred error phase - Delta m. */
int fdfb_decrypt_debug(fdfb_ctx *ctx, const uint32_t *cts_host, uint32_t B, uint32_t dim,
                       uint32_t *m_out, int64_t *err_out);

/*
 * Serialise the context (parameters, seed, secrets, raw keys and registered
 * tables) into buf.  *len: in = capacity of buf, out = bytes needed.  With
 * buf == NULL only the size is reported.  Errors: FDFB_EINVAL when the
 * capacity is too small.
 */
int fdfb_export_keys(const fdfb_ctx *ctx, void *buf, size_t *len);

/* Rebuild a context from fdfb_export_keys output.  Every section length is
 * checked against the parameters and against the bytes present before any
 * copy.  Errors: FDFB_EINVAL for a wrong magic, unsupported parameters,
 * inconsistent or truncated sections, non-binary secrets or table values
 * >= t; FDFB_ENOMEM. */
int fdfb_import_keys(const void *buf, size_t len, fdfb_ctx **out);

/* Copy one raw key array to host memory (for key-equality checks):
 * which = 0 s [n], 1 s_F [N], 2 brK [n][2 g_ell][2][N], 3 pK [N][pk_ell][2][N],
 * 4 ksK [N][ks_ell][n+1].  *count: in = capacity (words), out = words needed. */
int fdfb_get_key(const fdfb_ctx *ctx, uint32_t which, uint32_t *host, size_t *count);

/* Copy the rotation polynomials of a registered table to host memory:
 * host int32[2][N] = rotP_0, rotP_1 (unscaled table values, Sec. 3.3).
 * Errors: FDFB_EINVAL for a null pointer or an unknown lut_id. */
int fdfb_get_rotation_polys(const fdfb_ctx *ctx, int32_t lut_id, int32_t *host);

/* ---- serving engine ----------------------------------------------------- */

/*
 * Continuous batching of bootstrap requests (the batched form of
 * fdfb_bootstrap_batch applied to whatever requests are waiting).  A
 * scheduler thread keeps a FIFO of waiting requests; whenever one of the
 * server's streams is free it forms a batch from the oldest waiting request
 * and the later ones that share its context and flags, in arrival order (at
 * most max_batch samples), admits it only
 * if its device scratch fits in the memory budget next to the batches in
 * flight, gathers the inputs, bootstraps them and scatters the outputs.
 * Memory admission: the server owns one device arena of mem_budget bytes;
 * every batch carves its staging buffers and bootstrap scratch from it
 * (first fit) and returns them when it retires, so mem_budget bounds the
 * device memory serving uses besides the contexts' keys.  A batch that does
 * not fit is shortened to the longest prefix of its requests that does, or
 * waits for running batches to retire.  Batches on different streams
 * overlap on the device.  Each output is bit-identical to a standalone
 * fdfb_bootstrap_batch of that request.  A failure fails the requests of
 * its batch only.  Contexts may still be used directly (calls take the
 * context's lock) and tables may be registered at any time.
 */
typedef struct fdfb_server fdfb_server;

typedef struct fdfb_serving_stats {
    uint64_t requests_done, bootstraps_done, batches;
    uint64_t max_in_flight_bytes; /* peak admitted bytes (staging + scratch) */
    uint64_t arena_bytes;         /* size of the admission arena */
    double seconds;               /* since creation */
} fdfb_serving_stats;

/* ctxs[nctx]: parameter sets served (requests name them by index);
 * max_batch: largest batch (and request) in samples; mem_budget: bytes of
 * the admission arena (at least one batch of max_batch samples of every
 * context, else FDFB_EINVAL with the size needed in fdfb_last_error);
 * nstreams: 1..8 device streams.  Uploads keys and allocates the arena.
 * Errors: FDFB_EINVAL, FDFB_ENOMEM, FDFB_EDEVICE. */
int fdfb_server_create(fdfb_ctx *const *ctxs, uint32_t nctx, uint32_t max_batch, size_t mem_budget,
                       uint32_t nstreams, fdfb_server **out);

/* Enqueue a request of B samples (1 <= B <= max_batch) of context ctx_index:
 * same buffers and flags as fdfb_bootstrap_batch, device memory owned by the
 * caller.  The inputs are read only after the work enqueued on `stream`
 * before this call (an event recorded here), so they may still be being
 * produced there; outputs are written before the request completes and must
 * not be touched until then.  Thread-safe; returns at once with *req_id. */
int fdfb_server_submit(fdfb_server *srv, uint32_t ctx_index, const uint32_t *d_cts,
                       const int32_t *d_lut_ids, uint32_t B, uint32_t *d_out, uint32_t flags,
                       void *stream, uint64_t *req_id);

/* *done = 1 once the request's outputs are in place (0 while pending). */
int fdfb_server_poll(fdfb_server *srv, uint64_t req_id, int *done);

/* Block until the request completes; latency_s (nullable) receives the time
 * from submission to observed completion.  Forgets the request id. */
int fdfb_server_wait(fdfb_server *srv, uint64_t req_id, double *latency_s);

int fdfb_server_stats(fdfb_server *srv, fdfb_serving_stats *out);

/* Finish the waiting and running requests, then release the server. */
void fdfb_server_destroy(fdfb_server *srv);

/* ---- autotuning of the blind rotation ----------------------------------- */

/*
 * How a batched blind rotation of A accumulators is issued.  form:
 *   FDFB_FORM_AUTO   the fixed rule by launch round size
 *   FDFB_FORM_1W     one wavefront per accumulator, all three Karatsuba
 *                    products at once (four wavefronts per accumulator at
 *                    N = 2048)
 *   FDFB_FORM_1W2    one wavefront per accumulator, two per SIMD, products
 *                    one after another (N = 1024, gadget 2^7 x 3)
 *   FDFB_FORM_2W     two wavefronts per accumulator (N = 1024, gadget 2^7 x 3)
 *   FDFB_FORM_QUEUE  the persistent work-queue kernel, one launch
 *   FDFB_FORM_SPLIT  eight wavefronts per accumulator instead of four, each
 *                    with a quarter of one output component's tiles: for
 *                    rounds too small to fill the device (N = 2048)
 * round: accumulators per launch round (0 = the form's resident capacity;
 * ignored by the queue).  ms: measured milliseconds per rotation (0 if none).
 * Every plan gives the same output bits.
 */
#define FDFB_FORM_AUTO 0u
#define FDFB_FORM_1W 1u
#define FDFB_FORM_1W2 2u
#define FDFB_FORM_2W 3u
#define FDFB_FORM_QUEUE 4u
#define FDFB_FORM_SPLIT 5u
typedef struct fdfb_br_plan {
    uint32_t form, round;
    double ms;
} fdfb_br_plan;

/* The plans the kernels offer for the context's geometry.  *count: in =
 * capacity of plans (may be 0 with plans = NULL), out = number of plans.
 * Errors: FDFB_ENOTSUP without a batched rotation, FDFB_EINVAL when the
 * buffer is too small (*count then holds the number needed). */
int fdfb_br_plans(fdfb_ctx *ctx, fdfb_br_plan *plans, uint32_t *count);

/* Time every plan on A accumulators (per accumulators per sample, random
 * contents, the context's keys), each once to warm up and then `reps` times
 * on a private stream, and record the fastest for (this device's compute
 * units, N, ell, digit chunks, n, A) in the process-wide table; later
 * rotations of that size and geometry use it (every entry point, every
 * context with the same geometry).  With the environment variable
 * FDFB_TUNE_CACHE set to a path, the table is read from that file at first
 * use and written back after each tuning run.  *best receives the chosen
 * plan and its time; tried (nullable, capacity *ntried) every plan timed.
 * Allocates and frees timing buffers; synchronises its stream.
 * Errors: FDFB_EINVAL, FDFB_ENOTSUP, FDFB_ENOMEM, FDFB_EDEVICE. */
int fdfb_autotune(fdfb_ctx *ctx, uint32_t A, uint32_t per, uint32_t reps, fdfb_br_plan *best,
                  fdfb_br_plan *tried, uint32_t *ntried);

/* Tune the two rotation phases of a bootstrap batch where they run: every
 * plan is timed as part of whole batches of B samples with L tables each
 * (random samples, table 0, which must be registered), first for the sign
 * rotations (B ell_boot accumulators) with the function rotation's plan
 * fixed, then for the function rotation (B L accumulators); each phase's
 * fastest plan is recorded as fdfb_autotune records it.  Timing a phase
 * inside the batch catches what isolated timing misses (a launch that
 * follows other kernels may be placed unevenly on the SIMDs).  sign_best,
 * func_best: the plans chosen, with the batch time in ms; tried (nullable,
 * capacity *ntried) every batch timing.  When both phases have the same
 * accumulator count one plan is searched for both.  Errors: as
 * fdfb_autotune, FDFB_EINVAL without a registered table. */
int fdfb_autotune_bootstrap(fdfb_ctx *ctx, uint32_t B, uint32_t L, uint32_t reps, fdfb_br_plan *sign_best,
                            fdfb_br_plan *func_best, fdfb_br_plan *tried, uint32_t *ntried);

/* Record a plan for A accumulators of the context's geometry (plan = NULL
 * removes the entry, back to the fixed rule), or read the plan in use. */
int fdfb_br_set_plan(fdfb_ctx *ctx, uint32_t A, const fdfb_br_plan *plan);
int fdfb_br_get_plan(fdfb_ctx *ctx, uint32_t A, fdfb_br_plan *plan);

/* Write the table to a file / merge a file into it / empty it. */
int fdfb_tune_save(const char *path);
int fdfb_tune_load(const char *path);
int fdfb_tune_clear(void);

/* ---- per-phase device timing ------------------------------------------- */

/* Phases of fdfb_bootstrap_batch, in order. */
#define FDFB_PHASE_MODSWITCH_INIT 0 /* ModSwitch + sign accumulators          */
#define FDFB_PHASE_SIGN_BR 1        /* ell_boot sign blind rotations (batched) */
#define FDFB_PHASE_EXTRACT_BITS 2   /* SampleExtract of the sign rotations     */
#define FDFB_PHASE_PACKING_KS 3     /* LWE -> RLWE switching (BuildAcc)        */
#define FDFB_PHASE_PUBMUX 4         /* public mux (BuildAcc)                   */
#define FDFB_PHASE_FUNCTION_BR 5    /* function blind rotation                 */
#define FDFB_PHASE_OUTPUT 6         /* SampleExtract + final key switch        */
#define FDFB_NPHASES 7

/* Enable (1) or disable (0) timing: while enabled, every fdfb_bootstrap_batch
 * call records a hipEvent at each phase boundary on its stream.  A context
 * created while the environment variable FDFB_TRACE is set (to anything but
 * "0") starts with timing enabled, and fdfb_free prints the milliseconds per
 * call of each phase, over the calls not yet read, to stderr (a diagnostic:
 * the events of every call are kept until then). */
int fdfb_profile(fdfb_ctx *ctx, int enable);

/* Wait for the recorded events, add the elapsed milliseconds of each phase
 * over all recorded calls into ms[FDFB_NPHASES] (overwritten), store the
 * number of calls in *calls, and forget the events. */
int fdfb_profile_read(fdfb_ctx *ctx, double *ms, uint32_t *calls);

/* Number of kernel launches one batched blind rotation of `accumulators`
 * accumulators (`per_ct` consecutive ones per ciphertext, 1 <= per_ct)
 * takes on the current device, for matching per-launch profiles: the MFMA
 * form is issued in rounds of the device's resident workgroup capacity (or
 * of the tuned plan's round size; a queue plan is one launch), the plain and
 * direct forms in one launch.  0 accumulators take 0 launches.
 * FDFB_EINVAL on a null pointer or per_ct = 0, FDFB_EDEVICE on a HIP error. */
int fdfb_br_launches(fdfb_ctx *ctx, uint32_t accumulators, uint32_t per_ct, uint32_t flags,
                     uint32_t *launches);

/* Calibration of the roofline: run a stream of independent int8 MFMAs
 * (v_mfma_i32_16x16x64_i8, operands in registers, no memory traffic) on every
 * resident workgroup slot of the current device, synchronously on the null
 * stream, and store the sustained dense int8 rate in *tera_ops (10^12 ops/s,
 * a multiply-add counting 2) and the timed launch's duration in *ms.  It
 * allocates and frees a small output buffer.  FDFB_EINVAL on a null pointer,
 * FDFB_EDEVICE on a HIP error. */
int fdfb_measure_mfma_peak(double *tera_ops, double *ms);

/* Raise or clear the abort flag; while raised, device entry points return
 * FDFB_EABORTED without enqueuing work. */
void fdfb_set_abort(fdfb_ctx *ctx, int raised);

/* Release a context and its device memory (NULL is a no-op). */
void fdfb_free(fdfb_ctx *ctx);

/* Text of the last error on the calling thread ("" if none). */
const char *fdfb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FDFB_H */
