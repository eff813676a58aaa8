// Internal declarations shared by the device kernels and the C-ABI host code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/nmfkl.h"

namespace nmfkl {

// Width of one tile chunk: the number of consecutive (permuted) coordinates whose
// fixed-factor values a lane holds in registers at a time.
constexpr int kChunk = 8;
// Chunk width of the long-segment kernels and of the chunk-major copy they read.
constexpr int kChunkMajorW = 4;
static_assert(kChunkMajorW == 2 || kChunkMajorW == 4, "chunk-major copies are allocated for r rounded up to 4");

// Philox-4x64 with 10 rounds (Salmon et al., SC'11), shared by the host permutation entry
// point and the on-device permutation kernel.
__host__ __device__ inline void philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2],
                                              uint64_t out[4]) {
    uint64_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
#pragma unroll
    for (int rnd = 0; rnd < 10; ++rnd) {
        const uint64_t a = 0xD2E7470EE14C6C93ull * x0;   // low halves of the two products
        const uint64_t b = 0xCA5A826395121157ull * x2;
#if defined(__HIP_DEVICE_COMPILE__)
        const uint64_t ah = __umul64hi(0xD2E7470EE14C6C93ull, x0);
        const uint64_t bh = __umul64hi(0xCA5A826395121157ull, x2);
#else
        const uint64_t ah = (uint64_t)(((unsigned __int128)0xD2E7470EE14C6C93ull * x0) >> 64);
        const uint64_t bh = (uint64_t)(((unsigned __int128)0xCA5A826395121157ull * x2) >> 64);
#endif
        const uint64_t y0 = bh ^ x1 ^ k0, y2 = ah ^ x3 ^ k1;
        x0 = y0; x1 = b; x2 = y2; x3 = a;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

// Fisher-Yates order of 0..r-1 for (seed, t, stream); word w selects floor(w*(i+1)/2^64).
__host__ __device__ inline void coordinate_order(uint64_t seed, uint64_t t, uint64_t stream, int r,
                                                 int32_t* ids) {
    for (int i = 0; i < r; ++i) ids[i] = i;
    uint64_t words[4];
    const uint64_t key[2] = {seed, 0};
    uint64_t block = 0;
    int next = 4;
    for (int i = r - 1; i >= 1; --i) {
        if (next == 4) {
            const uint64_t ctr[4] = {block, t, stream, 0};
            philox4x64_10(ctr, key, words);
            ++block;
            next = 0;
        }
        const uint64_t w = words[next++];
#if defined(__HIP_DEVICE_COMPILE__)
        const int j = (int)__umul64hi(w, (uint64_t)(i + 1));
#else
        const int j = (int)(((unsigned __int128)w * (uint64_t)(i + 1)) >> 64);
#endif
        const int32_t tmp = ids[i];
        ids[i] = ids[j];
        ids[j] = tmp;
    }
}

// One permuted-copy / column-sum job: the fixed factor A (P x r) of one problem's half, or
// a factor of the objective in its natural order.  Jobs of a launch cover consecutive block
// ranges [first_block, first_block + nblocks) of the permute launch and [first_sum,
// first_sum + r) of the finalize launch.
struct PermJob {
    const float* A;       // P x r, point-major
    float* Ap;            // permuted copy, row stride Sp (nullptr: sums only)
    double* partials;     // nblocks x r float64 partial sums
    double* sums;         // r column sums (permuted order), written by the finalize launch
    int32_t* ids;         // the order used, stored by the job's first block (nullptr: not stored)
    int64_t P;
    int64_t rpb;          // rows per block
    uint64_t seed;        // Philox key of the order
    uint64_t stream;      // Philox stream of the order
    int32_t r, Sp;
    int32_t first_block, nblocks;
    int32_t first_sum;
    int32_t identity;     // 1: natural order, 0: the order of (seed, t, stream)
    int32_t bf16;         // 1: the copy holds bfloat16 values (round to nearest even) and the
                          //    column sums are those of the rounded values
    int32_t pad;
    float* Apc;           // nullptr, or a second copy in chunk-major order: the values of permuted
                          // columns Wc..Wc+W-1 of row p at Apc[(c * P + p) * W ..], W =
                          // kChunkMajorW (zero beyond r; bfloat16 when bf16)
};

// One half-sweep's per-launch arguments (kernels read them from a device table).
struct SweepArgs {
    const int64_t* ptr;     // segment pointers (CSC for the F-half, CSR for the W-half)
    const int32_t* idx;     // point ids of the nonzeros
    const float* val;       // values of the nonzeros
    const float* Ap;        // fixed factor, columns permuted into this sweep's order, row stride Sp
                            // (float32, or bfloat16 when tile_bf16)
    const double* sumA;     // its column sums, permuted order
    const int32_t* ids;     // the order: permuted column s is original column ids[s]
    float* X;               // the factor being updated (point-major, row stride r)
    const double* Min;      // model values at the nonzeros on entry ...
    const int32_t* Mmap;    // ... read as Min[Mmap[q]] when Mmap != nullptr, else Min[q]
    double* Mout;           // model values on exit, in this segment order
    unsigned long long* stats;  // optional counters (6), nullptr when off
    int32_t Sp;
    int32_t r;
    float alpha, beta, eps_log, eps_g, eps_x;
    int32_t t_max, j_max, literal_break, guard;
    int32_t tile_bf16;      // 1: Ap holds bfloat16 values (row stride Sp elements)
    int32_t model_from_tiles;  // 1: each segment computes its model values from the tiles and x
                               //    (Min unused); Mout may be null (no write-back)
    const float* Apc;       // nullptr, or the chunk-major copy (PermJob::Apc) read by the
                            // long-segment kernels
    int64_t Prows;          // rows of the fixed factor (the chunk stride of Apc)
};

// Fold-in launch arguments (the method parameters travel in a SweepArgs).
struct FoldinArgs {
    const int64_t* ptr;      // document pointers
    const int32_t* idx;      // word ids
    const float* val;        // counts
    const float* W;          // n x r, natural order
    const double* sumW;      // r column sums of W
    const double* rowsumW;   // n row sums of W
    double totW;             // sum of sumW
    const int32_t* perm;     // [max_passes][r] orders of the passes
    float* F;                // ndocs x r results
    int32_t* passes;         // passes run per document
    double* kl;              // final KL per document
    int r;
    int max_passes;
    double tol;
    unsigned* done;          // nullptr, or per-document completion words (host-coherent memory):
                             // done[d] = done_tag once F, passes and kl of document d are written
    unsigned done_tag;
};

// Fold-in variants: 0: 16 lanes x 4, 1: 64 x 4, 2: 256 x 4, 3: 256 x 8 nonzeros (blocks of
// 256 threads), 4: 512 lanes x 10 nonzeros (one document per 512-thread block).
constexpr int kFoldinVariants = 5;
constexpr int kFoldinCapacity[kFoldinVariants] = {64, 256, 1024, 2048, 5120};

// A block of the fused binned launch: variant and its slice of the segment list.
struct BlockWork {
    int32_t variant;   // index into the (lanes per segment, elements per lane) table
    int32_t first;     // first entry in the segment list
    int32_t count;     // number of segments for this block
    int32_t prob;      // entry of the argument table (problem of a batch)
};

// The (G lanes per segment, E elements per lane) variants of the fused launch.
struct Variant { int G, E; };
constexpr int kNumVariants = 14;
constexpr Variant kVariants[kNumVariants] = {{8, 3}, {8, 4}, {16, 3}, {16, 4},  {32, 3}, {32, 4}, {64, 3},
                                             {64, 4}, {64, 5}, {64, 6}, {64, 8}, {256, 3}, {256, 4}, {256, 8}};
constexpr int kFusedThreads = 256;
constexpr int kMaxFusedLength = 2048;   // 256 * 8 (the last variant, for 1025..2048 only)

// Segments longer than kMaxFusedLength: blocks of kCoopThreads threads x kCoopE nonzeros
// (kCoopBlocksPerCU blocks per compute unit), B = ceil(L / kCoopCapacity) of them per
// segment, cooperating through cross-block exchanges.
constexpr int kCoopThreads = 256;
constexpr int kCoopBlocksPerCU = 2;
constexpr int kCoopE = 20;
constexpr int kCoopCapacity = kCoopThreads * kCoopE;
// A queue of many waves uses blocks twice as wide, one per compute unit: the same nonzeros
// per unit, half as many partners in each cross-block exchange.
constexpr int kWideThreads = 512;
constexpr int kWideBlocksPerCU = 1;
constexpr int kWideCapacity = kWideThreads * kCoopE;

// A block of a long-segment launch.
struct LongWork {
    int32_t seg;    // segment id
    int32_t part;   // this block's part, 0 <= part < B
    int32_t B;      // blocks cooperating on the segment
    int32_t group;  // index of the segment's reduction slot in this launch
    int32_t prob;   // entry of the argument table (problem of a batch)
    int32_t pad;
};

// Launch wrappers (defined with the kernels).  All enqueue on `stream`.
// Permuted copies and partial column sums of njobs jobs (nblocks = total permute blocks).
// The order of outer iteration t = t_arg + (t_dev ? *t_dev : 0) is computed on the device.
hipError_t launch_permute_jobs(const PermJob* jobs, int njobs, int nblocks, int64_t t_arg,
                               const int64_t* t_dev, hipStream_t stream);
// Column sums of njobs jobs from their partials (nsum = total of the jobs' r).
hipError_t launch_finalize_jobs(const PermJob* jobs, int njobs, int nsum, hipStream_t stream);
hipError_t launch_model_terms(const double* M, const float* val, int64_t nnz, double* partials,
                              int nblocks, hipStream_t stream);
// tab: device table of SweepArgs; each block uses tab[work.prob].  stats: false when no
// entry of the table collects statistics (the launch then keeps no counters).
hipError_t launch_sweep_fused(const SweepArgs* tab, const BlockWork* work, const int32_t* segs,
                              int nblocks, bool lookahead, bool stats, hipStream_t stream);
// Partial sums a cooperating block publishes per reduction (at most S1 and S2 of every
// coordinate of an 8-wide chunk), one tagged 64-bit word each.
constexpr int kCoopValues = 2 * kChunk;
// Long segments over several co-resident blocks: one cooperative launch of `grid` blocks
// that take the nparts parts of the work list through a ticket counter.  Zeroes the groups'
// tagged partial words and the counter first (2 * pmax * kCoopValues words per group, pmax =
// largest B in the list, then one counter word).  cooperative = false: ordinary launch of
// the same grid (inside a captured graph), which relies on the grid fitting the device's
// co-resident capacity; the waits stay bounded.  wide: one part per block of kWideThreads
// (grid == nparts; the parts were cut at kWideCapacity).
hipError_t launch_sweep_long(const SweepArgs* tab, const LongWork* work, int nparts, int grid,
                             unsigned long long* words, int ngroups, unsigned* err, int pmax, bool cooperative,
                             bool wide, hipStream_t stream);
// Co-resident blocks of the cooperative long-segment kernel per compute unit (0 on failure).
int long_kernel_blocks_per_cu();
// ... and of its wide form.
int wide_kernel_blocks_per_cu();
hipError_t launch_model_objective(const int64_t* csc_ptr, const int32_t* csc_idx,
                                  const float* csc_val, int m, const float* W, const float* F, int r,
                                  double* Mcsc, double* partials, int nblocks, hipStream_t stream);
hipError_t launch_sum_f64(const double* in, int count, double* out, hipStream_t stream);
// dst[q] = src[map[q]], q < count.
hipError_t launch_gather_f64(const double* src, const int32_t* map, int64_t count, double* dst,
                             hipStream_t stream);
// *p = v (a kernel, so that it can precede a graph launch without a host-memory copy).
hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t stream);
hipError_t launch_validate_ptr(const int64_t* ptr, int64_t Q, int64_t nnz, unsigned* flags,
                               hipStream_t stream);
hipError_t launch_validate_entries(const int64_t* ptr, const int32_t* idx, const float* val,
                                   int64_t Q, int64_t P, int64_t nnz, unsigned* flags,
                                   hipStream_t stream);
hipError_t launch_validate_factor(const float* A, int64_t count, unsigned* flags, unsigned bit,
                                  hipStream_t stream);
hipError_t launch_build_maps(const int64_t* csr_ptr, const int32_t* csr_idx, const float* csr_val,
                             const int64_t* csc_ptr, const int32_t* csc_idx, const float* csc_val,
                             int64_t n, int64_t nnz, int32_t* csr2csc, int32_t* csc2csr,
                             unsigned* flags, hipStream_t stream);

hipError_t launch_foldin(const FoldinArgs& f, const SweepArgs& a, int variant, const int32_t* docs,
                         int ndocs, hipStream_t stream);
hipError_t launch_row_sums(const float* W, int64_t n, int r, double* out, hipStream_t stream);
// *out += the number of exact zeros among A[0..count).
hipError_t launch_count_zeros(const float* A, int64_t count, unsigned long long* out, hipStream_t stream);

// Validation flag bits.
enum : unsigned {
    kBadPtr = 1u, kBadIndex = 2u, kBadOrder = 4u, kBadValue = 8u, kBadTranspose = 16u,
    kBadW = 32u, kBadF = 64u
};

}  // namespace nmfkl
