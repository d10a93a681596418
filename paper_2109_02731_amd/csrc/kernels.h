// Kernel launchers of the FDFB library (host side of the HIP kernels).
// All pointers are device pointers; every launcher enqueues on `stream`.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdfbk {

struct Geometry {
    int n, N, log2_t;
    int g_log2B, g_ell, g_chunks;  // chunks: 7-bit pieces per gadget digit (MFMA form)
    int ks_log2B, ks_ell;
    int pk_log2B, pk_ell;
    int boot_log2B, boot_ell;
};

// Number of 7-bit chunks an unsigned digit of log2B bits needs on the int8 MFMA path.
inline int digit_chunks(int log2B) { return (log2B + 6) / 7; }

// True when the batched MFMA blind rotation has an instantiation for G.
bool br_mfma_supported(const Geometry &G);

hipError_t launch_modswitch(const Geometry &G, const uint32_t *cts, uint32_t B, uint32_t *ctN,
                            hipStream_t s);
hipError_t launch_init_sign(const Geometry &G, const uint32_t *ctN, uint32_t B, uint32_t *acc,
                            hipStream_t s);
// [Delta rotP_0 X^{b_N}, 0] per sample (TFHE-style accumulator).
// An id outside [0, nluts) gives a zero accumulator and sets bit 0 of *err.
hipError_t launch_init_tfhe(const Geometry &G, const uint32_t *ctN, const int32_t *lut_ids, uint32_t B,
                            const int32_t *luts, int nluts, uint32_t *err, uint32_t *acc, hipStream_t s);
hipError_t launch_br_plain(const Geometry &G, uint32_t *acc, const uint32_t *ctN, uint32_t A,
                           uint32_t accs_per_ct, const uint32_t *brk_raw, hipStream_t s);
hipError_t launch_br_mfma(const Geometry &G, uint32_t *acc, const uint32_t *ctN, uint32_t A,
                          uint32_t accs_per_ct, const void *brk_frag, hipStream_t s);
// One job of the persistent work-queue blind rotation (device pointers).
// Items [first_item, next job's first_item) belong to it: one accumulator per
// item for a wide job (N = 2048), four for a narrow one.
struct BrQueueJob {
    uint32_t *acc;          // [accs][2][N]
    const uint32_t *ctN;    // [accs / per][n + 1]
    const void *bfrag;      // Karatsuba key fragments
    const uint32_t *corr;   // offset correction
    uint32_t accs, per, n, log2B, wide, first_item;
};
constexpr int kQueueJobs = 16;
struct BrQueue {
    BrQueueJob job[kQueueJobs];
    uint32_t njobs, items;
};
// A blind-rotation job for launch_br_queue.
struct BrJobDesc {
    Geometry G;
    uint32_t *acc;
    const uint32_t *ctN;
    uint32_t A, per;
    const void *bfrag;
    const uint32_t *corr;
};
// True when the persistent kernel can take a job of this geometry.
bool br_queue_supported(const Geometry &G);
// Rotate every job's accumulators with persistent work-queue launches: jobs
// are grouped into launches of one narrow and one wide geometry (at most
// kQueueJobs jobs each); counters: one device word per launch (reset by a
// kernel before it), at least br_queue_launches(...) of them.
hipError_t br_queue_launches(const BrJobDesc *jobs, int njobs, uint32_t *launches);
hipError_t launch_br_queue(const BrJobDesc *jobs, int njobs, uint32_t *counters, uint32_t ncounters,
                           hipStream_t s);
// Workgroups of the persistent kernel resident at once for these jobs (each
// takes one work item at a time: four accumulators of a narrow geometry or
// one of a wide one; the least over the launches the jobs form; 0 when there
// are none).
hipError_t br_queue_slots(const BrJobDesc *jobs, int njobs, uint32_t *items);

// How one batched blind rotation of the Karatsuba form is issued: the
// kernel form and the accumulators per launch round (0: the form's resident
// capacity).  kFormAuto is the fixed rule by round size; kForm1W one
// wavefront per accumulator with all three products at once (k_br_kara1w,
// or the four-wavefront k_br_kara at N = 2048); kForm1W2 one wavefront per
// accumulator, two per SIMD (k_br_kara1w2, N = 1024); kForm2W two wavefronts
// per accumulator (k_br_kara1w2, N = 1024); kFormQueue the persistent
// work-queue kernel in one launch; kFormSplit eight wavefronts per
// accumulator, each with a quarter of one output component's tiles
// (k_br_kara with four wavefronts per component, N = 2048).
enum BrForm : uint32_t { kFormAuto = 0, kForm1W = 1, kForm1W2 = 2, kForm2W = 3, kFormQueue = 4, kFormSplit = 5 };
struct BrPlan {
    uint32_t form = kFormAuto;
    uint32_t round = 0;
};
// The plans that exist for G (at most max written; returns how many exist).
int br_plan_candidates(const Geometry &G, BrPlan *out, int max);
bool br_plan_valid(const Geometry &G, const BrPlan &plan);
// Karatsuba form of the batched blind rotation (same instantiations as
// launch_br_mfma): brk_frag from build_brk_kara, corr the offset table;
// work: one device word for the queue counter (kFormQueue only).
hipError_t launch_br_kara(const Geometry &G, uint32_t *acc, const uint32_t *ctN, uint32_t A,
                          uint32_t accs_per_ct, const void *brk_frag, const uint32_t *corr, const BrPlan &plan,
                          uint32_t *work, hipStream_t s);
// Kernel launches launch_br_kara issues for A accumulators under `plan`
// (rounds of the resident capacity; a round may begin inside a sample's
// accumulators; the queue is one launch).
hipError_t br_kara_launches(const Geometry &G, uint32_t A, uint32_t accs_per_ct, const BrPlan &plan,
                            uint32_t *launches);
// add_base != 0: sample b of accumulator a gets add_base * L_boot^(a % per) added.
hipError_t launch_extract(const Geometry &G, const uint32_t *acc, uint32_t A, uint32_t per,
                          uint32_t add_base, uint32_t *lwe, hipStream_t s);
hipError_t launch_keyswitch(const uint32_t *in, uint32_t B, uint32_t din, const uint32_t *key,
                            int log2B, int ell, uint32_t out_len, uint32_t *out, hipStream_t s);
// Key switching as an int8 MFMA GEMM over key fragments built by
// build_keyswitch_fragments (requires log2B <= 7 and din % 64 == 0).
bool keyswitch_mfma_supported(int log2B, int ell, uint32_t din);
hipError_t launch_keyswitch_mfma(const uint32_t *in, uint32_t B, uint32_t din, const void *kfrag, int log2B,
                                 int ell, uint32_t out_len, uint32_t *out, hipStream_t s);
hipError_t launch_affine(const int32_t *W, const uint32_t *in, uint32_t rows, uint32_t cols, uint32_t width,
                         uint32_t *out, hipStream_t s);
// out[k] = wx x[k] + wy y[k] (mod 2^32) for k < count.
hipError_t launch_lincomb2(const uint32_t *x, const uint32_t *y, int32_t wx, int32_t wy, uint32_t count,
                           uint32_t *out, hipStream_t s);
// E table evaluations; evaluation e uses sample e / per (its RLWE bit samples
// and ModSwitched sample) and table lut_ids[e]; an id outside [0, nluts)
// gives a zero accumulator and sets bit 0 of *err.
hipError_t launch_pubmux(const Geometry &G, const uint32_t *rlwe, const uint32_t *ctN,
                         const int32_t *lut_ids, uint32_t E, uint32_t per, const int32_t *luts, int nluts,
                         uint32_t *err, uint32_t *acc, hipStream_t s);

// Calibration stream of independent int8 MFMAs: one 64-thread workgroup per
// block, mfma_stream_chains() chains of iters v_mfma_i32_16x16x64_i8 each; out
// holds blocks * 64 int32.  mfma_stream_capacity gives the workgroups
// resident at once.
uint32_t mfma_stream_chains();
hipError_t mfma_stream_capacity(uint32_t *blocks);
hipError_t launch_mfma_stream(uint32_t blocks, uint32_t iters, int32_t *out, hipStream_t s);

// Static device buffer of the allocation-free bootstrap (bytes per GPU) and
// its device address on the current device (looked up once per device).
constexpr size_t kNoallocScratchBytes = 64u << 20;
hipError_t noalloc_scratch(void **ptr);

}  // namespace fdfbk
