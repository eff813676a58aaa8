// C ABI of the NMF-KL coordinate-descent library: handle life cycle, validation, nnz
// binning, and the enqueue sequence of each half-sweep and of the objective.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "nmfkl_internal.hpp"

using namespace nmfkl;

namespace {

thread_local std::string g_create_error;

enum ModelState { kModelNone = 0, kModelCscFresh, kModelCsc, kModelCsr };

struct BinPlan {
    BlockWork* work = nullptr;  // device: blocks of the fused launch
    int32_t* segs = nullptr;    // device
    int nblocks = 0;
    // long segments: one cooperative launch of at most the co-residency capacity whose blocks
    // take parts through a ticket counter (one part per block when all fit at once)
    LongWork* long_work = nullptr;  // device: the launch's parts
    // nblocks: parts; grid: blocks; wide: blocks of kWideThreads (parts of kWideCapacity)
    struct Round { int first, nblocks, ngroups, pmax, grid; bool wide; };
    std::vector<Round> rounds;
    int max_groups = 0, max_pmax = 0;
    // algorithmic (gather-model) bytes and updates of the fused and of the long launches
    double fused_bytes = 0, fused_updates = 0, long_bytes = 0, long_updates = 0;
};

// The segments of one problem's half, for planning: host copy of the segment pointers.
struct SegSource {
    const std::vector<int64_t>* ptr;
    int r;
    int prob;   // entry of the argument table
};

// Entries of a handle's device argument table (by the storage order of the model values
// the half reads) and of its permute-job table.
enum { kArgFfromCsr = 0, kArgFfromCsc = 1, kArgWfromCsc = 2, kArgWfromCsr = 3, kNumArgs = 4 };
enum { kJobF = 0, kJobW = 1, kJobSumW = 2, kJobSumF = 3, kNumJobs = 4 };

}  // namespace

struct nmfkl_handle {
    nmfkl_problem prob{};
    nmfkl_params prm{};
    hipStream_t stream = nullptr;
    int device = 0;
    int Sp = 0;
    // scratch
    float* Ap = nullptr;          // permuted padded copy of the fixed factor
    float* Apc = nullptr;         // its chunk-major copy (halves with long segments only)
    bool long_half[2] = {false, false};  // the F-half / W-half has segments for the long kernels
    double* sumA = nullptr;       // its column sums (permuted order)
    double* partials = nullptr;   // per-block column-sum partials
    int sum_blocks = 0;
    int32_t* ids = nullptr;       // the current order
    double* Mcsc = nullptr;       // model values at the nonzeros (float64), CSC order
    double* Mcsr = nullptr;       // ... CSR order
    int32_t* csc2csr = nullptr;
    int32_t* csr2csc = nullptr;
    double* obj_partials = nullptr;
    int obj_blocks = 0;
    // device results read back together by the objective: [total, 2 x r natural-order sums,
    // error flags], with a pinned host mirror of the same layout
    double* dres = nullptr;
    double* host_res = nullptr;
    double* sums2 = nullptr;      // dres + 1
    double* dscal = nullptr;      // dres
    unsigned long long* stats = nullptr;
    unsigned long long* coop_words = nullptr;  // tagged cross-block partial sums of long segments
    unsigned* dev_err = nullptr;       // device-side error flags (bounded waits), in dres's last word
    int long_capacity = 0;             // co-resident blocks of the cooperative long-segment kernel
    int wide_capacity = 0;             // co-resident blocks of its wide form
    BinPlan binF, binW;
    std::vector<int64_t> hptr_csc, hptr_csr;  // host copies of the segment pointers
    // out-of-core V (params.out_of_core): chunks of whole columns (F-half) / rows (W-half)
    // streamed from host memory through two device staging buffers
    struct Chunk {
        int64_t seg0, seg1;        // segment range
        int64_t nnz0, nnz1;        // nonzero range
        int64_t lptr;              // offset of its rebased pointers in h_lptr
        BinPlan plan;
    };
    bool ooc = false;
    std::vector<Chunk> chunks[2];  // [0] columns (CSC), [1] rows (CSR)
    int64_t* h_lptr = nullptr;     // pinned host: rebased pointers of every chunk of both halves
    int64_t* d_ptr[2] = {nullptr, nullptr};
    int32_t* d_idx[2] = {nullptr, nullptr};
    float* d_val[2] = {nullptr, nullptr};
    SweepArgs* ooc_args = nullptr;  // device: one entry per chunk (half 0 chunks, then half 1)
    double* d_chunk_obj = nullptr;  // per-chunk objective partial sums
    hipStream_t copy_stream = nullptr;
    hipEvent_t ev_copied[2] = {nullptr, nullptr}, ev_used[2] = {nullptr, nullptr};
    bool used_recorded[2] = {false, false};
    int64_t staged_bytes = 0;       // H2D bytes of V moved (timing/measurement)
    SweepArgs* argtab = nullptr;       // device: kNumArgs sweep-argument entries
    PermJob* jobtab = nullptr;         // device: kNumJobs permute jobs
    // timing (params.collect_timings): event pairs per launch group, resolved on demand
    struct Pending { int kind; hipEvent_t a, b; bool shared_a; };  // shared_a: a is the previous record's b
    std::vector<Pending> pending;
    std::vector<hipEvent_t> event_pool;
    nmfkl_timings timings{};
    int model = kModelNone;
    bool objective_pending = false;    // nmfkl_objective_enqueue's value not read yet
    std::string err;
};

namespace {

int fail(nmfkl_handle* h, int code, const std::string& msg) {
    if (h) h->err = msg;
    else g_create_error = msg;
    return code;
}

int hip_fail(nmfkl_handle* h, hipError_t e, const char* what) {
    return fail(h, NMFKL_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

size_t results_words(int r) { return 2 + 2 * (size_t)r; }

// The results block [total, 2 x r sums, error flags] on the device and its pinned mirror.
hipError_t alloc_results(nmfkl_handle* h) {
    const size_t n = results_words(h->prob.r);
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&h->dres), n * sizeof(double));
    if (e != hipSuccess) return e;
    e = hipHostMalloc(reinterpret_cast<void**>(&h->host_res), n * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) return e;
    h->dscal = h->dres;
    h->sums2 = h->dres + 1;
    h->dev_err = reinterpret_cast<unsigned*>(h->dres + 1 + 2 * (size_t)h->prob.r);
    return hipSuccess;
}

#define HIP_TRY(h, expr)                                   \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess) return hip_fail(h, e_, #expr); \
    } while (0)

template <class T>
hipError_t dalloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
}

// ---- timing helpers -------------------------------------------------------------------
// The timing events only ever give elapsed times, so they skip the system-scope fence of an
// ordinary event record (a cache writeback and invalidation between launch groups, which the
// next group would pay for): 3.005 -> 2.986 ms per corpus iteration with timings on.
hipError_t take_event(nmfkl_handle* h, hipEvent_t* ev) {
    if (!h->event_pool.empty()) {
        *ev = h->event_pool.back();
        h->event_pool.pop_back();
        return hipSuccess;
    }
    return hipEventCreateWithFlags(ev, hipEventDisableSystemFence);
}

// Starts a timed launch group; returns the index of the pending record or -1 when off.
int timer_begin(nmfkl_handle* h, int kind) {
    if (!h->prm.collect_timings) return -1;
    nmfkl_handle::Pending p{kind, nullptr, nullptr, false};
    if (take_event(h, &p.a) != hipSuccess || take_event(h, &p.b) != hipSuccess) return -1;
    if (hipEventRecord(p.a, h->stream) != hipSuccess) return -1;
    h->pending.push_back(p);
    return (int)h->pending.size() - 1;
}

void timer_end(nmfkl_handle* h, int idx) {
    if (idx < 0) return;
    (void)hipEventRecord(h->pending[idx].b, h->stream);
}

// Ends timed group prev (if any) and starts one of `kind` with the same event, for groups
// that follow each other on the stream.
int timer_switch(nmfkl_handle* h, int prev, int kind) {
    if (prev < 0) return timer_begin(h, kind);
    if (hipEventRecord(h->pending[prev].b, h->stream) != hipSuccess) return -1;
    nmfkl_handle::Pending p{kind, h->pending[prev].b, nullptr, true};
    if (take_event(h, &p.b) != hipSuccess) return -1;
    h->pending.push_back(p);
    return (int)h->pending.size() - 1;
}

hipError_t resolve_timings(nmfkl_handle* h) {
    if (h->pending.empty()) return hipSuccess;
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return e;
    for (auto& p : h->pending) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            h->timings.k[p.kind].ms_total += ms;
            h->timings.k[p.kind].launches += 1;
        }
        if (!p.shared_a) h->event_pool.push_back(p.a);
        h->event_pool.push_back(p.b);
    }
    h->pending.clear();
    return hipSuccess;
}

void release(nmfkl_handle* h) {
    for (auto& p : h->pending) {
        if (!p.shared_a) h->event_pool.push_back(p.a);
        h->event_pool.push_back(p.b);
    }
    h->pending.clear();
    for (hipEvent_t ev : h->event_pool) (void)hipEventDestroy(ev);
    h->event_pool.clear();
    auto f = [](void* p) { if (p) (void)hipFree(p); };
    f(h->Ap); f(h->Apc); f(h->sumA); f(h->partials); f(h->ids); f(h->Mcsc); f(h->Mcsr);
    f(h->csc2csr); f(h->csr2csc); f(h->obj_partials); f(h->dres); f(h->stats);
    f(h->binF.work); f(h->binF.segs); f(h->binW.work); f(h->binW.segs);
    f(h->binF.long_work); f(h->binW.long_work);
    f(h->coop_words); f(h->argtab); f(h->jobtab);
    if (h->host_res) (void)hipHostFree(h->host_res);
    for (int k = 0; k < 2; ++k) {
        for (auto& c : h->chunks[k]) {
            auto g = [](void* q) { if (q) (void)hipFree(q); };
            g(c.plan.work); g(c.plan.segs); g(c.plan.long_work);
        }
        f(h->d_ptr[k]); f(h->d_idx[k]); f(h->d_val[k]);
        if (h->ev_copied[k]) (void)hipEventDestroy(h->ev_copied[k]);
        if (h->ev_used[k]) (void)hipEventDestroy(h->ev_used[k]);
    }
    f(h->ooc_args); f(h->d_chunk_obj);
    if (h->h_lptr) (void)hipHostFree(h->h_lptr);
    if (h->copy_stream) (void)hipStreamDestroy(h->copy_stream);
}

// Variant for a segment of length L in the fused launch (-1: too long).  Segments of
// 1025..2048 nonzeros take the last variant (256 x 8, LDS form).  bin_shift > 0 maps a shorter
// segment to the smallest variant holding L << bin_shift nonzeros (more lanes per nonzero;
// 256 x 4 at most).
// pow2_only (tuning bit 2): only the variants of 4 and 8 nonzeros per lane, i.e. power-of-two
// capacities (a segment that fits E = 3, 5 or 6 gets the next variant of the same lane count,
// whose extra elements stay empty: the same sums in the same order).
int variant_for(int64_t L, int bin_shift, bool pow2_only = false) {
    if (L > kMaxFusedLength) return -1;
    if (L > kMaxFusedLength / 2) return kNumVariants - 1;   // 256 x 8 (LDS form) for 1025..2048
    const int64_t Ls = L << bin_shift;
    for (int v = 0; v < kNumVariants - 1; ++v) {
        if (pow2_only && (kVariants[v].E & (kVariants[v].E - 1)) != 0) continue;
        if (Ls <= (int64_t)kVariants[v].G * kVariants[v].E) return v;
    }
    return kNumVariants - 2;
}

void free_plan(BinPlan* p) {
    auto f = [](void* q) { if (q) (void)hipFree(q); };
    f(p->work); f(p->segs); f(p->long_work);
    *p = BinPlan{};
}

// Segments up to kMaxFusedLength: grouped by variant (longest variants first, so that long
// blocks start early); inside a variant each problem's segments are sorted longest first and
// cut into blocks of kFusedThreads / G segments of that problem, and the blocks of all
// problems are ordered by their first segment, longest first.  Longer segments: one
// cooperative launch that works through them as a queue, largest first.
// A queue of more than this many waves of the co-resident capacity runs on the wide blocks:
// on the corpus (3.5 waves) two blocks of 256 per unit are faster (long_W 1.32 ms against
// 1.53 ms with wide blocks), on the large corpus (about 50 waves) the wide blocks are (long_W
// 125 ms against 137 ms in a measuring harness).
constexpr int kWideQueueWaves = 8;

int plan_bins(const std::vector<SegSource>& src, int long_capacity, int wide_capacity,
              int bin_shift, bool problem_major, BinPlan* plan, std::string* err, bool pow2_only = false) {
    struct LongSeg { int32_t q, prob; int64_t len; };
    const size_t ns = src.size();
    std::vector<std::vector<std::vector<int32_t>>> groups(kNumVariants, std::vector<std::vector<int32_t>>(ns));
    std::vector<LongSeg> longs;
    for (size_t i = 0; i < ns; ++i) {
        const std::vector<int64_t>& ptr = *src[i].ptr;
        const double r = src[i].r;
        const int64_t Q = (int64_t)ptr.size() - 1;
        for (int64_t q = 0; q < Q; ++q) {
            const int64_t L = ptr[q + 1] - ptr[q];
            const double bytes = (double)L * (8.0 + 4.0 * r) + 8.0 + 8.0 * r;
            const int v = variant_for(L, bin_shift, pow2_only);
            if (v < 0) {
                longs.push_back(LongSeg{(int32_t)q, src[i].prob, L});
                plan->long_bytes += bytes;
                plan->long_updates += (double)L * r;
            } else {
                groups[v][i].push_back((int32_t)q);
                plan->fused_bytes += bytes;
                plan->fused_updates += (double)L * r;
            }
        }
    }
    std::vector<int32_t> segs;
    std::vector<BlockWork> work;
    struct Blk { int64_t key; size_t src, first; int count; int v; };
    std::vector<Blk> all;
    for (int v = kNumVariants - 1; v >= 0; --v) {
        const int spb = kFusedThreads / kVariants[v].G;
        std::vector<Blk> blks;
        for (size_t i = 0; i < ns; ++i) {
            const std::vector<int64_t>& ptr = *src[i].ptr;
            auto len = [&](int32_t q) { return ptr[q + 1] - ptr[q]; };
            auto& g = groups[v][i];
            std::stable_sort(g.begin(), g.end(), [&](int32_t a, int32_t b) { return len(a) > len(b); });
            for (size_t k = 0; k < g.size(); k += spb)
                blks.push_back(Blk{len(g[k]), i, k, (int)std::min<size_t>(spb, g.size() - k), v});
        }
        std::stable_sort(blks.begin(), blks.end(), [](const Blk& a, const Blk& b) { return a.key > b.key; });
        all.insert(all.end(), blks.begin(), blks.end());
    }
    // problem-major: the blocks of one problem together (variants longest first inside it), so
    // that the launch works on few problems' fixed factors at a time (cache locality)
    if (problem_major)
        std::stable_sort(all.begin(), all.end(), [](const Blk& a, const Blk& b) { return a.src < b.src; });
    for (const Blk& b : all) {
        BlockWork w;
        w.variant = b.v;
        w.first = (int32_t)segs.size();
        w.count = b.count;
        w.prob = src[b.src].prob;
        for (int k = 0; k < b.count; ++k) segs.push_back(groups[b.v][b.src][b.first + k]);
        work.push_back(w);
    }
    auto dev_fail = [&](hipError_t e, const char* what) {
        *err = std::string(what) + ": " + hipGetErrorString(e);
        return NMFKL_E_DEVICE;
    };
    hipError_t e;
    plan->nblocks = (int)work.size();
    if ((e = dalloc(&plan->work, work.size())) != hipSuccess) return dev_fail(e, "plan allocation");
    if ((e = dalloc(&plan->segs, segs.size())) != hipSuccess) return dev_fail(e, "plan allocation");
    if (!work.empty() &&
        (e = hipMemcpy(plan->work, work.data(), work.size() * sizeof(BlockWork), hipMemcpyHostToDevice)) != hipSuccess)
        return dev_fail(e, "plan upload");
    if (!segs.empty() &&
        (e = hipMemcpy(plan->segs, segs.data(), segs.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess)
        return dev_fail(e, "plan upload");

    std::stable_sort(longs.begin(), longs.end(), [](const LongSeg& a, const LongSeg& b) { return a.len > b.len; });
    std::vector<LongWork> lw;
    auto blocks_of = [](const LongSeg& l) { return (int)((l.len + kCoopCapacity - 1) / kCoopCapacity); };
    const std::vector<LongSeg>& queued = longs;
    // Longer segments take B = ceil(L / kCoopCapacity) co-resident blocks each and share one
    // cooperative launch that works through them as a queue, largest B first.  A queue of many
    // waves runs on the wide blocks (parts of kWideCapacity: half as many partners per exchange, whose
    // compute times spread when the chunk slices exceed the L2); a short queue keeps two
    // narrow blocks per unit, whose exchanges overlap the other block's compute.  Both hold
    // the same nonzeros per unit, so a segment that does not fit one fits neither.
    auto wide_blocks_of = [](const LongSeg& l) { return (int)((l.len + kWideCapacity - 1) / kWideCapacity); };
    if (!queued.empty()) {
        int64_t parts = 0;
        for (const LongSeg& l : queued) parts += blocks_of(l);
        const bool wide = parts > (int64_t)kWideQueueWaves * long_capacity;
        const int cap = wide ? wide_capacity : long_capacity;
        BinPlan::Round cur{(int)lw.size(), 0, 0, 0, 0, wide};
        for (const LongSeg& l : queued) {
            const int B = wide ? wide_blocks_of(l) : blocks_of(l);
            if (B > cap) {
                *err = "a segment of " + std::to_string(l.len) + " nonzeros needs " + std::to_string(B) +
                       " co-resident blocks; this device holds " + std::to_string(cap);
                return NMFKL_E_UNSUPPORTED;
            }
            // B = 1 parts exchange nothing: they share group 0
            const int group = B > 1 ? cur.ngroups++ : 0;
            for (int p = 0; p < B; ++p) lw.push_back(LongWork{l.q, p, B, group, l.prob, 0});
            cur.nblocks += B;
            cur.pmax = std::max(cur.pmax, B);
        }
        cur.ngroups = std::max(cur.ngroups, 1);
        cur.grid = std::min(cur.nblocks, cap);
        plan->rounds.push_back(cur);
    }
    for (const auto& r : plan->rounds) {
        plan->max_groups = std::max(plan->max_groups, r.ngroups);
        plan->max_pmax = std::max(plan->max_pmax, r.pmax);
    }
    if (!lw.empty()) {
        if ((e = dalloc(&plan->long_work, lw.size())) != hipSuccess) return dev_fail(e, "plan allocation");
        if ((e = hipMemcpy(plan->long_work, lw.data(), lw.size() * sizeof(LongWork), hipMemcpyHostToDevice)) !=
            hipSuccess)
            return dev_fail(e, "plan upload");
    }
    return NMFKL_OK;
}

int check_params(const nmfkl_params* p, std::string* why) {
    auto bad = [&](const char* m) { *why = m; return NMFKL_E_INVAL; };
    if (!(p->alpha_W >= 0) || !(p->alpha_F >= 0) || !(p->beta_W >= 0) || !(p->beta_F >= 0))
        return bad("alpha and beta must be >= 0");
    if (!std::isfinite(p->alpha_W + p->alpha_F + p->beta_W + p->beta_F))
        return bad("alpha and beta must be finite");
    if (!(p->eps_log >= 0) || !(p->eps_g >= 0) || !(p->eps_x >= 0) || !std::isfinite(p->eps_log + p->eps_g + p->eps_x))
        return bad("eps_log, eps_g, eps_x must be finite and >= 0");
    if (p->t_max < 1 || p->t_max > 1000000) return bad("t_max must be in [1, 1e6]");
    if (p->j_max < 0 || p->j_max > 64) return bad("j_max must be in [0, 64]");
    if (p->foldin_max_passes < 1) return bad("foldin_max_passes must be >= 1");
    if (!(p->foldin_tol >= 0)) return bad("foldin_tol must be >= 0");
    if (p->bin_shift < 0 || p->bin_shift > 3) return bad("bin_shift must be in [0, 3]");
    if (p->tile_bf16 != 0 && p->tile_bf16 != 1) return bad("tile_bf16 must be 0 or 1");
    if (p->out_of_core != 0 && p->out_of_core != 1) return bad("out_of_core must be 0 or 1");
    if (p->ooc_chunk_nnz < 0) return bad("ooc_chunk_nnz must be >= 0");
    return NMFKL_OK;
}

SweepArgs sweep_args(nmfkl_handle* h, bool fhalf) {
    SweepArgs a{};
    const nmfkl_problem& pr = h->prob;
    a.ptr = fhalf ? pr.csc_ptr : pr.csr_ptr;
    a.idx = fhalf ? pr.csc_idx : pr.csr_idx;
    a.val = fhalf ? pr.csc_val : pr.csr_val;
    a.Ap = h->Ap;
    a.sumA = h->sumA;
    a.ids = h->ids;
    a.X = fhalf ? pr.F : pr.W;
    a.stats = h->prm.collect_stats ? h->stats : nullptr;
    a.Sp = h->Sp;
    a.r = pr.r;
    a.alpha = (float)(fhalf ? h->prm.alpha_F : h->prm.alpha_W);
    a.beta = (float)(fhalf ? h->prm.beta_F : h->prm.beta_W);
    a.eps_log = (float)h->prm.eps_log;
    a.eps_g = (float)h->prm.eps_g;
    a.eps_x = (float)h->prm.eps_x;
    a.t_max = h->prm.t_max;
    a.j_max = h->prm.j_max;
    a.literal_break = h->prm.literal_break;
    a.guard = h->prm.guard;
    a.tile_bf16 = h->prm.tile_bf16;
    a.model_from_tiles = h->prm.tile_bf16 || h->prm.out_of_core;
    a.Apc = h->long_half[fhalf ? 0 : 1] ? h->Apc : nullptr;
    a.Prows = fhalf ? pr.n : pr.m;
    return a;
}

// The handle's argument entries: each half reading the model values in either storage order
// (through the position map when they are in the other half's order).
void make_args(nmfkl_handle* h, SweepArgs (&args)[kNumArgs]) {
    for (int k = 0; k < kNumArgs; ++k) {
        const bool fhalf = k == kArgFfromCsr || k == kArgFfromCsc;
        args[k] = sweep_args(h, fhalf);
    }
    args[kArgFfromCsr].Min = h->Mcsr; args[kArgFfromCsr].Mmap = h->csc2csr; args[kArgFfromCsr].Mout = h->Mcsc;
    // in-place read/write of Mcsc is safe: each entry is read and written by one lane
    args[kArgFfromCsc].Min = h->Mcsc; args[kArgFfromCsc].Mmap = nullptr; args[kArgFfromCsc].Mout = h->Mcsc;
    args[kArgWfromCsc].Min = h->Mcsc; args[kArgWfromCsc].Mmap = h->csr2csc; args[kArgWfromCsc].Mout = h->Mcsr;
    args[kArgWfromCsr].Min = h->Mcsr; args[kArgWfromCsr].Mmap = nullptr; args[kArgWfromCsr].Mout = h->Mcsr;
    // bf16 tiles: every segment computes its model values from the rounded tiles, so none are
    // carried (the objective then evaluates eq. 1 from W and F)
    if (h->prm.tile_bf16)
        for (auto& a : args) a.Mout = nullptr;
}

// Permute jobs of the handle: the two halves' fixed factors in the order of (seed, t), and W
// and F in their natural order for the objective.
void make_jobs(nmfkl_handle* h, PermJob (&jobs)[kNumJobs]) {
    const nmfkl_problem& pr = h->prob;
    for (int k = 0; k < kNumJobs; ++k) {
        PermJob j{};
        const bool onW = k == kJobF || k == kJobSumW;
        j.A = onW ? pr.W : pr.F;
        j.P = onW ? pr.n : pr.m;
        j.rpb = (j.P + h->sum_blocks - 1) / h->sum_blocks;
        j.partials = h->partials;
        j.seed = h->prm.seed;
        j.stream = 0;
        j.r = pr.r;
        j.Sp = h->Sp;
        j.first_block = 0;
        j.nblocks = h->sum_blocks;
        j.first_sum = 0;
        if (k == kJobF || k == kJobW) {
            j.Ap = h->Ap;
            j.Apc = h->long_half[k == kJobF ? 0 : 1] ? h->Apc : nullptr;
            j.sums = h->sumA;
            j.ids = h->ids;
            j.identity = 0;
            j.bf16 = h->prm.tile_bf16;
        } else {
            // the objective's two jobs run in one launch: SumF after SumW, with partials of its own
            j.Ap = nullptr;
            j.sums = h->sums2 + (k == kJobSumW ? 0 : pr.r);
            j.ids = nullptr;
            j.identity = 1;
            if (k == kJobSumF) {
                j.first_block = h->sum_blocks;
                j.first_sum = pr.r;
                j.partials = h->partials + (size_t)h->sum_blocks * pr.r;
            }
        }
        jobs[k] = j;
    }
}

// Model values at the nonzeros in CSC order from scratch (the objective's SDDMM pass).
int refresh_model(nmfkl_handle* h) {
    const nmfkl_problem& pr = h->prob;
    const int tm = timer_begin(h, NMFKL_T_MODEL);
    HIP_TRY(h, launch_model_objective(pr.csc_ptr, pr.csc_idx, pr.csc_val, pr.m, pr.W, pr.F, pr.r,
                                      h->Mcsc, h->obj_partials, h->obj_blocks, h->stream));
    timer_end(h, tm);
    h->model = kModelCscFresh;
    return NMFKL_OK;
}

// Enqueues one half-sweep's sweep launches (cooperative long segments, then fused)
// over the plan, with the argument table tab; timed: bracket them with the handle's timers.
// stats: some entry of tab collects statistics.
hipError_t enqueue_plan(const BinPlan& plan, const SweepArgs* tab, unsigned long long* coop_words,
                        unsigned* dev_err, bool cooperative, bool lookahead, bool stats, hipStream_t s,
                        nmfkl_handle* timed, int long_kind, int fused_kind, int open_timer = -1) {
    hipError_t e;
    const bool any_long = !plan.rounds.empty();
    // timed groups follow each other: each one's start event ends the group before it
    // (open_timer: a group the caller started just before)
    int prev = open_timer;
    const int tl = (timed && any_long) ? timer_switch(timed, prev, long_kind) : -1;
    if (tl >= 0) prev = tl;
    for (const auto& rd : plan.rounds)
        if ((e = launch_sweep_long(tab, plan.long_work + rd.first, rd.nblocks, rd.grid, coop_words, rd.ngroups,
                                   dev_err, rd.pmax, cooperative, rd.wide, s)) != hipSuccess)
            return e;
    const int tf = (timed && plan.nblocks) ? timer_switch(timed, prev, fused_kind) : -1;
    if (tf >= 0) prev = tf;
    if ((e = launch_sweep_fused(tab, plan.work, plan.segs, plan.nblocks, lookahead, stats, s)) != hipSuccess) return e;
    if (timed) timer_end(timed, prev);
    return hipSuccess;
}

// Out-of-core V: stage chunk c of half `half` into buffer c % 2 on the copy stream, once the
// kernels that last used that buffer are done, and make the handle's stream wait for it.
hipError_t ooc_stage(nmfkl_handle* h, int half, size_t c) {
    const auto& ch = h->chunks[half][c];
    const nmfkl_problem& pr = h->prob;
    const int b = (int)(c & 1);
    const int32_t* idx = half == 0 ? pr.csc_idx : pr.csr_idx;
    const float* val = half == 0 ? pr.csc_val : pr.csr_val;
    const int64_t nseg = ch.seg1 - ch.seg0, nnz = ch.nnz1 - ch.nnz0;
    hipError_t e;
    if (h->used_recorded[b] && (e = hipStreamWaitEvent(h->copy_stream, h->ev_used[b], 0)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(h->d_ptr[b], h->h_lptr + ch.lptr, (size_t)(nseg + 1) * sizeof(int64_t),
                            hipMemcpyHostToDevice, h->copy_stream)) != hipSuccess)
        return e;
    if (nnz > 0) {
        if ((e = hipMemcpyAsync(h->d_idx[b], idx + ch.nnz0, (size_t)nnz * sizeof(int32_t), hipMemcpyHostToDevice,
                                h->copy_stream)) != hipSuccess)
            return e;
        if ((e = hipMemcpyAsync(h->d_val[b], val + ch.nnz0, (size_t)nnz * sizeof(float), hipMemcpyHostToDevice,
                                h->copy_stream)) != hipSuccess)
            return e;
    }
    if ((e = hipEventRecord(h->ev_copied[b], h->copy_stream)) != hipSuccess) return e;
    h->staged_bytes += (nseg + 1) * 8 + nnz * 8;
    return hipStreamWaitEvent(h->stream, h->ev_copied[b], 0);
}

hipError_t ooc_release(nmfkl_handle* h, size_t c) {
    const int b = (int)(c & 1);
    h->used_recorded[b] = true;
    return hipEventRecord(h->ev_used[b], h->stream);
}

int half_sweep_ooc(nmfkl_handle* h, int32_t t, bool fhalf) {
    const nmfkl_problem& pr = h->prob;
    const int half = fhalf ? 0 : 1;
    const int ts = timer_begin(h, fhalf ? NMFKL_T_SUMS_F : NMFKL_T_SUMS_W);
    const PermJob* job = h->jobtab + (fhalf ? kJobF : kJobW);
    HIP_TRY(h, launch_permute_jobs(job, 1, h->sum_blocks, t, nullptr, h->stream));
    HIP_TRY(h, launch_finalize_jobs(job, 1, pr.r, h->stream));
    timer_end(h, ts);
    const size_t first = fhalf ? 0 : h->chunks[0].size();
    for (size_t c = 0; c < h->chunks[half].size(); ++c) {
        HIP_TRY(h, ooc_stage(h, half, c));
        HIP_TRY(h, enqueue_plan(h->chunks[half][c].plan, h->ooc_args + first + c, h->coop_words, h->dev_err, true,
                                (h->prm.tuning & 1) != 0, h->prm.collect_stats != 0, h->stream, h, fhalf ? NMFKL_T_LONG_F : NMFKL_T_LONG_W,
                                fhalf ? NMFKL_T_FUSED_F : NMFKL_T_FUSED_W));
        HIP_TRY(h, ooc_release(h, c));
    }
    h->model = kModelNone;
    return NMFKL_OK;
}

int half_sweep(nmfkl_handle* h, int32_t t, bool fhalf) {
    if (!h) return fail(nullptr, NMFKL_E_INVAL, "null handle");
    if (t < 0) return fail(h, NMFKL_E_INVAL, "t must be >= 0");
    if (h->ooc) return half_sweep_ooc(h, t, fhalf);
    const nmfkl_problem& pr = h->prob;
    const BinPlan& plan = fhalf ? h->binF : h->binW;
    if (h->prm.tile_bf16) {
        // the sweep computes the model values from the rounded tiles itself
    } else if (fhalf) {
        const bool fresh_needed = h->model == kModelNone || (h->prm.refresh_model && h->model != kModelCscFresh);
        if (fresh_needed) {
            const int rc = refresh_model(h);
            if (rc) return rc;
        }
    } else if (h->model == kModelNone) {
        const int rc = refresh_model(h);
        if (rc) return rc;
    }
    const int ts = timer_begin(h, fhalf ? NMFKL_T_SUMS_F : NMFKL_T_SUMS_W);
    const PermJob* job = h->jobtab + (fhalf ? kJobF : kJobW);
    HIP_TRY(h, launch_permute_jobs(job, 1, h->sum_blocks, t, nullptr, h->stream));
    HIP_TRY(h, launch_finalize_jobs(job, 1, pr.r, h->stream));
    int ai;
    if (fhalf) ai = (h->model == kModelCsc || h->model == kModelCscFresh) ? kArgFfromCsc : kArgFfromCsr;
    else ai = h->model == kModelCsr ? kArgWfromCsr : kArgWfromCsc;
    HIP_TRY(h, enqueue_plan(plan, h->argtab + ai, h->coop_words, h->dev_err, true,
                            (h->prm.tuning & 1) != 0, h->prm.collect_stats != 0, h->stream, h,
                            fhalf ? NMFKL_T_LONG_F : NMFKL_T_LONG_W, fhalf ? NMFKL_T_FUSED_F : NMFKL_T_FUSED_W, ts));
    h->model = h->prm.tile_bf16 ? kModelNone : (fhalf ? kModelCsc : kModelCsr);
    return NMFKL_OK;
}

}  // namespace

extern "C" {

int nmfkl_params_default(nmfkl_params* p) {
    if (!p) return NMFKL_E_INVAL;
    std::memset(p, 0, sizeof(*p));
    p->eps_log = 1e-10;
    p->eps_g = 1e-5;
    p->eps_x = 0.1;
    p->t_max = 16;
    p->j_max = 8;
    p->literal_break = 0;
    p->guard = 1;
    p->seed = 0;
    p->foldin_max_passes = 200;
    p->foldin_tol = 1e-5;
    p->refresh_model = 0;
    p->collect_stats = 0;
    p->collect_timings = 0;
    p->tuning = 0;
    p->bin_shift = 0;
    p->tile_bf16 = 0;
    return NMFKL_OK;
}

int nmfkl_permutation(uint64_t seed, uint64_t t, uint64_t stream, int32_t r, int32_t* ids) {
    if (!ids || r < 1 || r > NMFKL_R_MAX) return NMFKL_E_INVAL;
    coordinate_order(seed, t, stream, r, ids);
    return NMFKL_OK;
}

const char* nmfkl_last_error(const nmfkl_handle* h) {
    return h ? h->err.c_str() : g_create_error.c_str();
}

}  // extern "C"

namespace {

// Host-side validation of V for the out-of-core mode: pointer arrays, index ranges and
// strict order, values; the CSR copy is the transpose of the CSC copy if every row count
// agrees and an order-independent checksum of the (row, column, value) entries agrees.
std::string validate_host_v(const nmfkl_problem& pr) {
    auto check_ptr = [](const int64_t* ptr, int64_t Q, int64_t nnz) {
        if (ptr[0] != 0 || ptr[Q] != nnz) return false;
        for (int64_t q = 0; q < Q; ++q)
            if (ptr[q + 1] < ptr[q]) return false;
        return true;
    };
    if (!check_ptr(pr.csc_ptr, pr.m, pr.nnz) || !check_ptr(pr.csr_ptr, pr.n, pr.nnz))
        return "pointer array not monotone / wrong ends";
    auto mix = [](uint64_t x) {
        x ^= x >> 33; x *= 0xFF51AFD7ED558CCDull; x ^= x >> 33; x *= 0xC4CEB9FE1A85EC53ull; x ^= x >> 33;
        return x;
    };
    std::vector<int64_t> rowcount((size_t)pr.n, 0);
    uint64_t sum_csc = 0, sum_csr = 0;
    for (int64_t j = 0; j < pr.m; ++j)
        for (int64_t q = pr.csc_ptr[j]; q < pr.csc_ptr[j + 1]; ++q) {
            const int32_t i = pr.csc_idx[q];
            const float v = pr.csc_val[q];
            if (i < 0 || i >= pr.n) return "index out of range";
            if (q > pr.csc_ptr[j] && i <= pr.csc_idx[q - 1]) return "indices not strictly increasing within a column";
            if (!(v >= 0.0f) || !std::isfinite(v)) return "value negative or not finite";
            rowcount[(size_t)i] += 1;
            uint32_t vb;
            std::memcpy(&vb, &v, 4);
            sum_csc += mix(((uint64_t)i << 32 | (uint64_t)j) ^ mix(vb));
        }
    for (int64_t i = 0; i < pr.n; ++i) {
        if (pr.csr_ptr[i + 1] - pr.csr_ptr[i] != rowcount[(size_t)i]) return "CSR is not the transpose of CSC";
        for (int64_t q = pr.csr_ptr[i]; q < pr.csr_ptr[i + 1]; ++q) {
            const int32_t j = pr.csr_idx[q];
            const float v = pr.csr_val[q];
            if (j < 0 || j >= pr.m) return "index out of range";
            if (q > pr.csr_ptr[i] && j <= pr.csr_idx[q - 1]) return "indices not strictly increasing within a row";
            uint32_t vb;
            std::memcpy(&vb, &v, 4);
            sum_csr += mix(((uint64_t)i << 32 | (uint64_t)j) ^ mix(vb));
        }
    }
    if (sum_csc != sum_csr) return "CSR is not the transpose of CSC";
    return "";
}

// Chunks of whole segments of at most `budget` nonzeros (a longer segment gets a chunk of its
// own), with their pointers rebased into `lptr`.
void make_chunks(const int64_t* ptr, int64_t Q, int64_t budget, std::vector<nmfkl_handle::Chunk>* out,
                 std::vector<int64_t>* lptr, int64_t* max_nnz, int64_t* max_segs) {
    int64_t q = 0;
    while (q < Q) {
        nmfkl_handle::Chunk c{};
        c.seg0 = q;
        c.nnz0 = ptr[q];
        int64_t q1 = q + 1;
        while (q1 < Q && ptr[q1 + 1] - c.nnz0 <= budget) ++q1;
        c.seg1 = q1;
        c.nnz1 = ptr[q1];
        c.lptr = (int64_t)lptr->size();
        for (int64_t k = q; k <= q1; ++k) lptr->push_back(ptr[k] - c.nnz0);
        *max_nnz = std::max(*max_nnz, c.nnz1 - c.nnz0);
        *max_segs = std::max(*max_segs, c.seg1 - c.seg0);
        out->push_back(c);
        q = q1;
    }
}

// True if p is device memory of the current device (or managed memory).
bool is_device_memory(const void* p) {
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();   // unregistered host memory
        return false;
    }
    return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

int create_ooc(const nmfkl_problem& pr, const nmfkl_params& prm, void* hip_stream, nmfkl_handle** out) {
    for (const void* q : {(const void*)pr.csc_ptr, (const void*)pr.csc_idx, (const void*)pr.csc_val,
                          (const void*)pr.csr_ptr, (const void*)pr.csr_idx, (const void*)pr.csr_val})
        if (q && is_device_memory(q))
            return fail(nullptr, NMFKL_E_INVAL, "out_of_core: V's arrays must be host memory");
    if (!is_device_memory(pr.W) || !is_device_memory(pr.F))
        return fail(nullptr, NMFKL_E_INVAL, "W and F must be device memory");
    std::string why = validate_host_v(pr);
    if (!why.empty()) return fail(nullptr, NMFKL_E_INVAL, "invalid input: " + why);
    nmfkl_handle* h = new (std::nothrow) nmfkl_handle();
    if (!h) return fail(nullptr, NMFKL_E_NOMEM, "host allocation failed");
    h->prob = pr;
    h->prm = prm;
    h->ooc = true;
    h->stream = reinterpret_cast<hipStream_t>(hip_stream);
    auto bail = [&](int code) {
        g_create_error = h->err;
        if (h->stream) (void)hipStreamSynchronize(h->stream);
        if (h->copy_stream) (void)hipStreamSynchronize(h->copy_stream);
        release(h);
        delete h;
        return code;
    };
#define OOC_HIP(expr)                                            \
    do {                                                         \
        hipError_t e_ = (expr);                                  \
        if (e_ != hipSuccess) return bail(hip_fail(h, e_, #expr)); \
    } while (0)
    OOC_HIP(hipGetDevice(&h->device));
    h->Sp = (pr.r + kChunk - 1) / kChunk * kChunk;
    const int64_t Pmax = std::max<int64_t>(pr.n, pr.m);
    unsigned* flags = nullptr;
    OOC_HIP(dalloc(&flags, 1));
    OOC_HIP(hipMemsetAsync(flags, 0, sizeof(unsigned), h->stream));
    OOC_HIP(launch_validate_factor(pr.W, (int64_t)pr.n * pr.r, flags, kBadW, h->stream));
    OOC_HIP(launch_validate_factor(pr.F, (int64_t)pr.m * pr.r, flags, kBadF, h->stream));
    unsigned hf = 0;
    OOC_HIP(hipMemcpyAsync(&hf, flags, sizeof(unsigned), hipMemcpyDeviceToHost, h->stream));
    OOC_HIP(hipStreamSynchronize(h->stream));
    (void)hipFree(flags);
    if (hf) {
        fail(h, NMFKL_E_INVAL, std::string("invalid input:") + ((hf & kBadW) ? " W negative or not finite;" : "") +
                                   ((hf & kBadF) ? " F negative or not finite;" : ""));
        return bail(NMFKL_E_INVAL);
    }
    OOC_HIP(dalloc(&h->Ap, (size_t)Pmax * h->Sp));
    OOC_HIP(dalloc(&h->sumA, NMFKL_R_MAX));
    h->sum_blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, Pmax / 64));
    OOC_HIP(dalloc(&h->partials, 2 * (size_t)h->sum_blocks * pr.r));
    OOC_HIP(dalloc(&h->ids, NMFKL_R_MAX));
    h->obj_blocks = 4096;
    OOC_HIP(dalloc(&h->obj_partials, h->obj_blocks));
    OOC_HIP(alloc_results(h));
    OOC_HIP(dalloc(&h->stats, 8));
    OOC_HIP(hipMemsetAsync(h->stats, 0, 8 * sizeof(unsigned long long), h->stream));
    OOC_HIP(hipMemsetAsync(h->dev_err, 0, sizeof(unsigned), h->stream));
    int ncu = 0;
    OOC_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device));
    h->long_capacity = long_kernel_blocks_per_cu() * ncu;
    h->wide_capacity = wide_kernel_blocks_per_cu() * ncu;
    if (h->long_capacity <= 0 || h->wide_capacity <= 0) {
        fail(h, NMFKL_E_DEVICE, "occupancy query of the long-segment kernel failed");
        return bail(NMFKL_E_DEVICE);
    }
    // chunks and their bins
    const int64_t budget = prm.ooc_chunk_nnz > 0 ? prm.ooc_chunk_nnz : ((int64_t)1 << 25);
    std::vector<int64_t> lptr;
    int64_t max_nnz = 0, max_segs = 0;
    make_chunks(pr.csc_ptr, pr.m, budget, &h->chunks[0], &lptr, &max_nnz, &max_segs);
    make_chunks(pr.csr_ptr, pr.n, budget, &h->chunks[1], &lptr, &max_nnz, &max_segs);
    int groups = 1, pmax = 1;
    for (int half = 0; half < 2; ++half)
        for (auto& c : h->chunks[half]) {
            std::vector<int64_t> local(lptr.begin() + c.lptr, lptr.begin() + c.lptr + (c.seg1 - c.seg0) + 1);
            std::string why_plan;
            const int rc = plan_bins({SegSource{&local, pr.r, 0}}, h->long_capacity, h->wide_capacity, prm.bin_shift, false, &c.plan,
                                     &why_plan, (prm.tuning & 4) != 0);
            if (rc) {
                fail(h, rc, why_plan);
                return bail(rc);
            }
            groups = std::max(groups, c.plan.max_groups);
            pmax = std::max(pmax, c.plan.max_pmax);
            if (!c.plan.rounds.empty()) h->long_half[half] = true;
        }
    if (h->long_half[0] || h->long_half[1]) OOC_HIP(dalloc(&h->Apc, (size_t)Pmax * ((pr.r + 3) & ~3)));
    OOC_HIP(dalloc(&h->coop_words, (size_t)groups * 2 * pmax * kCoopValues + 1));
    OOC_HIP(hipHostMalloc(reinterpret_cast<void**>(&h->h_lptr), lptr.size() * sizeof(int64_t), hipHostMallocDefault));
    std::memcpy(h->h_lptr, lptr.data(), lptr.size() * sizeof(int64_t));
    for (int b = 0; b < 2; ++b) {
        OOC_HIP(dalloc(&h->d_ptr[b], (size_t)max_segs + 1));
        OOC_HIP(dalloc(&h->d_idx[b], (size_t)max_nnz));
        OOC_HIP(dalloc(&h->d_val[b], (size_t)max_nnz));
        OOC_HIP(hipEventCreateWithFlags(&h->ev_copied[b], hipEventDisableTiming));
        OOC_HIP(hipEventCreateWithFlags(&h->ev_used[b], hipEventDisableTiming));
    }
    OOC_HIP(hipStreamCreateWithFlags(&h->copy_stream, hipStreamNonBlocking));
    OOC_HIP(dalloc(&h->d_chunk_obj, h->chunks[0].size()));
    {
        std::vector<SweepArgs> args;
        for (int half = 0; half < 2; ++half)
            for (size_t c = 0; c < h->chunks[half].size(); ++c) {
                SweepArgs a = sweep_args(h, half == 0);
                const int b = (int)(c & 1);
                a.ptr = h->d_ptr[b];
                a.idx = h->d_idx[b];
                a.val = h->d_val[b];
                a.X = (half == 0 ? pr.F : pr.W) + h->chunks[half][c].seg0 * pr.r;
                a.Min = nullptr;
                a.Mmap = nullptr;
                a.Mout = nullptr;
                a.model_from_tiles = 1;
                args.push_back(a);
            }
        OOC_HIP(dalloc(&h->ooc_args, args.size()));
        OOC_HIP(hipMemcpy(h->ooc_args, args.data(), args.size() * sizeof(SweepArgs), hipMemcpyHostToDevice));
        PermJob jobs[kNumJobs];
        make_jobs(h, jobs);
        OOC_HIP(dalloc(&h->jobtab, kNumJobs));
        OOC_HIP(hipMemcpy(h->jobtab, jobs, sizeof(jobs), hipMemcpyHostToDevice));
    }
    OOC_HIP(hipStreamSynchronize(h->stream));
#undef OOC_HIP
    h->model = kModelNone;
    *out = h;
    return NMFKL_OK;
}

}  // namespace

extern "C" {

int nmfkl_create(const nmfkl_problem* prob, const nmfkl_params* p, void* hip_stream,
                 nmfkl_handle** out) {
    if (!out) return fail(nullptr, NMFKL_E_INVAL, "out is null");
    *out = nullptr;
    if (!prob) return fail(nullptr, NMFKL_E_INVAL, "problem is null");
    nmfkl_params prm;
    if (p) prm = *p;
    else nmfkl_params_default(&prm);
    std::string why;
    if (check_params(&prm, &why)) return fail(nullptr, NMFKL_E_INVAL, why);
    const nmfkl_problem& pr = *prob;
    if (pr.n < 1 || pr.m < 1) return fail(nullptr, NMFKL_E_INVAL, "n and m must be >= 1");
    if (pr.r < 1 || pr.r > NMFKL_R_MAX) return fail(nullptr, NMFKL_E_INVAL, "r must be in [1, NMFKL_R_MAX]");
    if (pr.nnz < 0) return fail(nullptr, NMFKL_E_INVAL, "nnz must be >= 0");
    if (pr.nnz > INT32_MAX) return fail(nullptr, NMFKL_E_UNSUPPORTED, "nnz above 2^31-1");
    if (!pr.csc_ptr || !pr.csr_ptr || !pr.W || !pr.F) return fail(nullptr, NMFKL_E_INVAL, "null pointer");
    if (pr.nnz > 0 && (!pr.csc_idx || !pr.csc_val || !pr.csr_idx || !pr.csr_val))
        return fail(nullptr, NMFKL_E_INVAL, "null index/value pointer");
    if ((int64_t)pr.n * pr.r > ((int64_t)1 << 40) || (int64_t)pr.m * pr.r > ((int64_t)1 << 40))
        return fail(nullptr, NMFKL_E_UNSUPPORTED, "factor too large");
    if (prm.out_of_core) return create_ooc(pr, prm, hip_stream, out);
    for (const void* q : {(const void*)pr.csc_ptr, (const void*)pr.csr_ptr, (const void*)pr.W, (const void*)pr.F})
        if (!is_device_memory(q)) return fail(nullptr, NMFKL_E_INVAL, "V's pointers and W, F must be device memory");
    if (pr.nnz > 0)
        for (const void* q : {(const void*)pr.csc_idx, (const void*)pr.csc_val, (const void*)pr.csr_idx,
                              (const void*)pr.csr_val})
            if (!is_device_memory(q)) return fail(nullptr, NMFKL_E_INVAL, "V's arrays must be device memory");

    nmfkl_handle* h = new (std::nothrow) nmfkl_handle();
    if (!h) return fail(nullptr, NMFKL_E_NOMEM, "host allocation failed");
    h->prob = pr;
    h->prm = prm;
    h->stream = reinterpret_cast<hipStream_t>(hip_stream);
    auto bail = [&](int code) {
        g_create_error = h->err;
        if (h->stream) (void)hipStreamSynchronize(h->stream);
        release(h);
        delete h;
        return code;
    };
#define CREATE_HIP(expr)                                         \
    do {                                                         \
        hipError_t e_ = (expr);                                  \
        if (e_ != hipSuccess) return bail(hip_fail(h, e_, #expr)); \
    } while (0)
    CREATE_HIP(hipGetDevice(&h->device));
    h->Sp = (pr.r + kChunk - 1) / kChunk * kChunk;
    const int64_t Pmax = std::max<int64_t>(pr.n, pr.m);
    const int64_t nnz = pr.nnz;
    unsigned* flags = nullptr;
    CREATE_HIP(dalloc(&flags, 1));
    CREATE_HIP(hipMemsetAsync(flags, 0, sizeof(unsigned), h->stream));
    CREATE_HIP(launch_validate_ptr(pr.csc_ptr, pr.m, nnz, flags, h->stream));
    CREATE_HIP(launch_validate_ptr(pr.csr_ptr, pr.n, nnz, flags, h->stream));
    CREATE_HIP(launch_validate_factor(pr.W, (int64_t)pr.n * pr.r, flags, kBadW, h->stream));
    CREATE_HIP(launch_validate_factor(pr.F, (int64_t)pr.m * pr.r, flags, kBadF, h->stream));
    unsigned hf = 0;
    CREATE_HIP(hipMemcpyAsync(&hf, flags, sizeof(unsigned), hipMemcpyDeviceToHost, h->stream));
    CREATE_HIP(hipStreamSynchronize(h->stream));
    if (hf == 0) {
        CREATE_HIP(launch_validate_entries(pr.csc_ptr, pr.csc_idx, pr.csc_val, pr.m, pr.n, nnz, flags, h->stream));
        CREATE_HIP(launch_validate_entries(pr.csr_ptr, pr.csr_idx, pr.csr_val, pr.n, pr.m, nnz, flags, h->stream));
        CREATE_HIP(hipMemcpyAsync(&hf, flags, sizeof(unsigned), hipMemcpyDeviceToHost, h->stream));
        CREATE_HIP(hipStreamSynchronize(h->stream));
    }
    if (hf == 0) {
        CREATE_HIP(dalloc(&h->csc2csr, nnz));
        CREATE_HIP(dalloc(&h->csr2csc, nnz));
        CREATE_HIP(launch_build_maps(pr.csr_ptr, pr.csr_idx, pr.csr_val, pr.csc_ptr, pr.csc_idx, pr.csc_val,
                                     pr.n, nnz, h->csr2csc, h->csc2csr, flags, h->stream));
        CREATE_HIP(hipMemcpyAsync(&hf, flags, sizeof(unsigned), hipMemcpyDeviceToHost, h->stream));
        CREATE_HIP(hipStreamSynchronize(h->stream));
    }
    (void)hipFree(flags);
    if (hf) {
        std::string m = "invalid input:";
        if (hf & kBadPtr) m += " pointer array not monotone / wrong ends;";
        if (hf & kBadIndex) m += " index out of range;";
        if (hf & kBadOrder) m += " indices not strictly increasing within a column/row;";
        if (hf & kBadValue) m += " value negative or not finite;";
        if (hf & kBadTranspose) m += " CSR is not the transpose of CSC;";
        if (hf & kBadW) m += " W negative or not finite;";
        if (hf & kBadF) m += " F negative or not finite;";
        fail(h, NMFKL_E_INVAL, m);
        return bail(NMFKL_E_INVAL);
    }
    CREATE_HIP(dalloc(&h->Ap, (size_t)Pmax * h->Sp));
    CREATE_HIP(dalloc(&h->sumA, NMFKL_R_MAX));
    h->sum_blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, Pmax / 64));
    CREATE_HIP(dalloc(&h->partials, 2 * (size_t)h->sum_blocks * pr.r));
    CREATE_HIP(dalloc(&h->ids, NMFKL_R_MAX));
    CREATE_HIP(dalloc(&h->Mcsc, nnz));
    CREATE_HIP(dalloc(&h->Mcsr, nnz));
    h->obj_blocks = (int)std::min<int64_t>(4096, std::max<int64_t>(1, pr.m / 8));
    CREATE_HIP(dalloc(&h->obj_partials, h->obj_blocks));
    CREATE_HIP(alloc_results(h));
    CREATE_HIP(dalloc(&h->stats, 8));
    CREATE_HIP(hipMemsetAsync(h->stats, 0, 8 * sizeof(unsigned long long), h->stream));
    {
        int ncu = 0;
        CREATE_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device));
        h->long_capacity = long_kernel_blocks_per_cu() * ncu;
        h->wide_capacity = wide_kernel_blocks_per_cu() * ncu;
        if (h->long_capacity <= 0 || h->wide_capacity <= 0) {
            fail(h, NMFKL_E_DEVICE, "occupancy query of the long-segment kernel failed");
            return bail(NMFKL_E_DEVICE);
        }
        h->hptr_csc.resize((size_t)pr.m + 1);
        h->hptr_csr.resize((size_t)pr.n + 1);
        CREATE_HIP(hipMemcpy(h->hptr_csc.data(), pr.csc_ptr, h->hptr_csc.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
        CREATE_HIP(hipMemcpy(h->hptr_csr.data(), pr.csr_ptr, h->hptr_csr.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
        std::string why_plan;
        int rc = plan_bins({SegSource{&h->hptr_csc, pr.r, 0}}, h->long_capacity, h->wide_capacity, prm.bin_shift, false, &h->binF,
                           &why_plan, (prm.tuning & 4) != 0);
        if (!rc)
            rc = plan_bins({SegSource{&h->hptr_csr, pr.r, 0}}, h->long_capacity, h->wide_capacity, prm.bin_shift, false, &h->binW,
                           &why_plan, (prm.tuning & 4) != 0);
        if (rc) {
            fail(h, rc, why_plan);
            return bail(rc);
        }
        h->long_half[0] = !h->binF.rounds.empty();
        h->long_half[1] = !h->binW.rounds.empty();
        if (h->long_half[0] || h->long_half[1])
            CREATE_HIP(dalloc(&h->Apc, (size_t)Pmax * ((pr.r + 3) & ~3)));
        const int groups = std::max(h->binF.max_groups, h->binW.max_groups);
        const int pmax = std::max(h->binF.max_pmax, h->binW.max_pmax);
        // the queue kernel addresses words + group * (2 * pmax * kCoopValues) + ..., then the
        // ticket counter after the last group
        CREATE_HIP(dalloc(&h->coop_words, (size_t)std::max(groups, 1) * 2 * std::max(pmax, 1) * kCoopValues + 1));
        CREATE_HIP(hipMemsetAsync(h->dev_err, 0, sizeof(unsigned), h->stream));
    }
    {
        SweepArgs args[kNumArgs];
        PermJob jobs[kNumJobs];
        make_args(h, args);
        make_jobs(h, jobs);
        CREATE_HIP(dalloc(&h->argtab, kNumArgs));
        CREATE_HIP(dalloc(&h->jobtab, kNumJobs));
        CREATE_HIP(hipMemcpy(h->argtab, args, sizeof(args), hipMemcpyHostToDevice));
        CREATE_HIP(hipMemcpy(h->jobtab, jobs, sizeof(jobs), hipMemcpyHostToDevice));
    }
    CREATE_HIP(hipStreamSynchronize(h->stream));
#undef CREATE_HIP
    {
        const double r = pr.r;
        auto& k = h->timings.k;
        k[NMFKL_T_FUSED_F].gather_bytes = h->binF.fused_bytes;
        k[NMFKL_T_FUSED_F].updates = h->binF.fused_updates;
        k[NMFKL_T_LONG_F].gather_bytes = h->binF.long_bytes;
        k[NMFKL_T_LONG_F].updates = h->binF.long_updates;
        k[NMFKL_T_FUSED_W].gather_bytes = h->binW.fused_bytes;
        k[NMFKL_T_FUSED_W].updates = h->binW.fused_updates;
        k[NMFKL_T_LONG_W].gather_bytes = h->binW.long_bytes;
        k[NMFKL_T_LONG_W].updates = h->binW.long_updates;
        k[NMFKL_T_SUMS_F].gather_bytes = (double)pr.n * r * 4.0 * 2.0;   // read W, write its copy
        k[NMFKL_T_SUMS_W].gather_bytes = (double)pr.m * r * 4.0 * 2.0;
        k[NMFKL_T_MODEL].gather_bytes = (double)nnz * (16.0 + 4.0 * r) + (double)pr.m * (8.0 + 4.0 * r);
        k[NMFKL_T_TERMS].gather_bytes = (double)nnz * 12.0;
    }
    h->model = kModelNone;
    *out = h;
    return NMFKL_OK;
}

int nmfkl_sweep_F(nmfkl_handle* h, int32_t t) { return half_sweep(h, t, true); }

int nmfkl_sweep_W(nmfkl_handle* h, int32_t t) { return half_sweep(h, t, false); }

int nmfkl_invalidate_model(nmfkl_handle* h) {
    if (!h) return fail(nullptr, NMFKL_E_INVAL, "null handle");
    h->model = kModelNone;
    return NMFKL_OK;
}

namespace {
int objective_impl(nmfkl_handle* h, double* D_out, bool carried);
int objective_enqueue(nmfkl_handle* h, bool carried);
int objective_finish(nmfkl_handle* h, double* D_out);
}

int nmfkl_objective(nmfkl_handle* h, double* D_out) { return objective_impl(h, D_out, false); }

int nmfkl_objective_carried(nmfkl_handle* h, double* D_out) { return objective_impl(h, D_out, true); }

int nmfkl_objective_enqueue(nmfkl_handle* h) {
    if (!h) return fail(nullptr, NMFKL_E_INVAL, "null handle");
    const int rc = objective_enqueue(h, true);
    if (rc) return rc;
    h->objective_pending = true;
    return NMFKL_OK;
}

int nmfkl_objective_read(nmfkl_handle* h, double* D_out) {
    if (!h) return fail(nullptr, NMFKL_E_INVAL, "null handle");
    if (!D_out) return fail(h, NMFKL_E_INVAL, "D_out is null");
    if (!h->objective_pending) return fail(h, NMFKL_E_INVAL, "no objective enqueued since the last read");
    h->objective_pending = false;
    return objective_finish(h, D_out);
}

namespace {
int objective_impl(nmfkl_handle* h, double* D_out, bool carried) {
    if (!h) return fail(nullptr, NMFKL_E_INVAL, "null handle");
    if (!D_out) return fail(h, NMFKL_E_INVAL, "D_out is null");
    const int rc = objective_enqueue(h, carried);
    if (rc) return rc;
    h->objective_pending = false;
    return objective_finish(h, D_out);
}

// eq. 1's kernels and the copy of the results block into pinned host memory (no wait).
int objective_enqueue(nmfkl_handle* h, bool carried) {
    const nmfkl_problem& pr = h->prob;
    // natural-order float64 column sums of W and F: sum over all cells of W^T F = sumW . sumF
    // both jobs (adjacent in the table) in one permute and one finalize launch
    HIP_TRY(h, launch_permute_jobs(h->jobtab + kJobSumW, 2, 2 * h->sum_blocks, 0, nullptr, h->stream));
    HIP_TRY(h, launch_finalize_jobs(h->jobtab + kJobSumW, 2, 2 * pr.r, h->stream));
    if (h->ooc) {
        // eq. 1 streamed: each column chunk's model values and terms (no model values kept)
        const int tm = timer_begin(h, NMFKL_T_MODEL);
        for (size_t c = 0; c < h->chunks[0].size(); ++c) {
            const auto& ch = h->chunks[0][c];
            const int b = (int)(c & 1);
            const int64_t nseg = ch.seg1 - ch.seg0;
            const int nb = (int)std::min<int64_t>(h->obj_blocks, std::max<int64_t>(1, nseg / 8));
            HIP_TRY(h, ooc_stage(h, 0, c));
            HIP_TRY(h, launch_model_objective(h->d_ptr[b], h->d_idx[b], h->d_val[b], (int)nseg, pr.W,
                                              pr.F + ch.seg0 * pr.r, pr.r, nullptr, h->obj_partials, nb, h->stream));
            HIP_TRY(h, launch_sum_f64(h->obj_partials, nb, h->d_chunk_obj + c, h->stream));
            HIP_TRY(h, ooc_release(h, c));
        }
        timer_end(h, tm);
        HIP_TRY(h, launch_sum_f64(h->d_chunk_obj, (int)h->chunks[0].size(), h->dscal, h->stream));
    } else if (carried && (h->model == kModelCsr || h->model == kModelCsc || h->model == kModelCscFresh)) {
        const bool csr = h->model == kModelCsr;
        const int tm = timer_begin(h, NMFKL_T_TERMS);
        HIP_TRY(h, launch_model_terms(csr ? h->Mcsr : h->Mcsc, csr ? pr.csr_val : pr.csc_val, pr.nnz,
                                      h->obj_partials, h->obj_blocks, h->stream));
        timer_end(h, tm);
    } else {
        const int rc = refresh_model(h);
        if (rc) return rc;
    }
    if (!h->ooc) HIP_TRY(h, launch_sum_f64(h->obj_partials, h->obj_blocks, h->dscal, h->stream));
    // one copy of [total, sums, error flags] into pinned memory
    HIP_TRY(h, hipMemcpyAsync(h->host_res, h->dres, results_words(pr.r) * sizeof(double), hipMemcpyDeviceToHost,
                              h->stream));
    return NMFKL_OK;
}

// Waits for the copy and forms D from the results block.
int objective_finish(nmfkl_handle* h, double* D_out) {
    const nmfkl_problem& pr = h->prob;
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    unsigned derr = 0;
    std::memcpy(&derr, h->host_res + 1 + 2 * (size_t)pr.r, sizeof(unsigned));
    if (derr) return fail(h, NMFKL_E_DEVICE, "a cross-block wait of a long segment timed out");
    const double part = h->host_res[0];
    const double* sums = h->host_res + 1;
    double total = 0.0;
    for (int k = 0; k < pr.r; ++k) {
        if (!std::isfinite(sums[k]) || !std::isfinite(sums[pr.r + k]))
            return fail(h, NMFKL_E_NONFINITE, "a factor holds NaN or Inf");
        total += sums[k] * sums[pr.r + k];
    }
    if (std::isnan(part)) return fail(h, NMFKL_E_NONFINITE, "objective is NaN");
    *D_out = part + total;
    return NMFKL_OK;
}
}  // namespace

int nmfkl_get_stats(nmfkl_handle* h, nmfkl_stats* out) {
    if (!h) return fail(nullptr, NMFKL_E_INVAL, "null handle");
    if (!out) return fail(h, NMFKL_E_INVAL, "out is null");
    // exact zeros of W and F now, counted into words 6 and 7 of the statistics buffer
    const nmfkl_problem& pr = h->prob;
    HIP_TRY(h, hipMemsetAsync(h->stats + 6, 0, 2 * sizeof(unsigned long long), h->stream));
    HIP_TRY(h, launch_count_zeros(pr.W, (int64_t)pr.n * pr.r, h->stats + 6, h->stream));
    HIP_TRY(h, launch_count_zeros(pr.F, (int64_t)pr.m * pr.r, h->stats + 7, h->stream));
    unsigned long long c[8];
    HIP_TRY(h, hipMemcpyAsync(c, h->stats, sizeof(c), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    out->coords = (int64_t)c[0];
    out->evals = (int64_t)c[1];
    out->steps = (int64_t)c[2];
    out->halvings = (int64_t)c[3];
    out->rejects = (int64_t)c[4];
    out->tmax_hits = (int64_t)c[5];
    out->zeros_W = (int64_t)c[6];
    out->zeros_F = (int64_t)c[7];
    return NMFKL_OK;
}

int nmfkl_get_timings(nmfkl_handle* h, nmfkl_timings* out) {
    if (!h) return fail(nullptr, NMFKL_E_INVAL, "null handle");
    if (!out) return fail(h, NMFKL_E_INVAL, "out is null");
    HIP_TRY(h, resolve_timings(h));
    *out = h->timings;
    return NMFKL_OK;
}

int nmfkl_reset_timings(nmfkl_handle* h) {
    if (!h) return fail(nullptr, NMFKL_E_INVAL, "null handle");
    HIP_TRY(h, resolve_timings(h));
    for (auto& k : h->timings.k) {
        k.ms_total = 0.0;
        k.launches = 0;
    }
    return NMFKL_OK;
}

int nmfkl_destroy(nmfkl_handle* h) {
    if (!h) return NMFKL_E_INVAL;
    hipError_t e = hipStreamSynchronize(h->stream);
    release(h);
    delete h;
    return e == hipSuccess ? NMFKL_OK : NMFKL_E_DEVICE;
}

}  // extern "C"

// ------------------------------------------------------------------ batched problems
struct nmfkl_batch {
    std::vector<nmfkl_handle*> hs;
    nmfkl_params prm{};
    hipStream_t stream = nullptr;     // the caller's stream
    hipStream_t cap = nullptr;        // capture stream (non-blocking, default priority)
    SweepArgs* argtab = nullptr;      // device: [2][nprob], F-half entries then W-half entries
    PermJob* jobtab = nullptr;        // device: [2][nprob]
    int perm_blocks[2] = {0, 0};
    int nsum[2] = {0, 0};
    BinPlan plan[2];
    unsigned long long* coop_words = nullptr;
    size_t coop_words_n = 0;
    unsigned* dev_err = nullptr;
    int64_t* t_dev = nullptr;
    int long_capacity = 0;
    int wide_capacity = 0;
    int graph_coop = -1;
    std::vector<std::pair<int, hipGraphExec_t>> graphs;
    std::string err;
};

namespace {

thread_local std::string g_batch_error;

int bfail(nmfkl_batch* b, int code, const std::string& msg) {
    if (b) b->err = msg;
    else g_batch_error = msg;
    return code;
}

#define BHIP(b, expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return bfail(b, NMFKL_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

void drop_graphs(nmfkl_batch* b) {
    for (auto& g : b->graphs) (void)hipGraphExecDestroy(g.second);
    b->graphs.clear();
}

void batch_release(nmfkl_batch* b) {
    drop_graphs(b);
    free_plan(&b->plan[0]);
    free_plan(&b->plan[1]);
    auto f = [](void* p) { if (p) (void)hipFree(p); };
    f(b->argtab); f(b->jobtab); f(b->coop_words); f(b->dev_err); f(b->t_dev);
    b->argtab = nullptr; b->jobtab = nullptr; b->coop_words = nullptr;
    b->dev_err = nullptr; b->t_dev = nullptr;
    if (b->cap) (void)hipStreamDestroy(b->cap);
    b->cap = nullptr;
    for (nmfkl_handle* h : b->hs) nmfkl_destroy(h);
    b->hs.clear();
}

// Bins of both halves over all problems under b->prm.bin_shift, and cross-block scratch for
// their cooperative launches.
int batch_plan(nmfkl_batch* b) {
    drop_graphs(b);
    free_plan(&b->plan[0]);
    free_plan(&b->plan[1]);
    std::vector<SegSource> srcF, srcW;
    for (size_t p = 0; p < b->hs.size(); ++p) {
        srcF.push_back(SegSource{&b->hs[p]->hptr_csc, b->hs[p]->prob.r, (int)p});
        srcW.push_back(SegSource{&b->hs[p]->hptr_csr, b->hs[p]->prob.r, (int)p});
    }
    std::string why;
    const bool pm = (b->prm.tuning & 2) != 0;
    const bool p2 = (b->prm.tuning & 4) != 0;
    int rc = plan_bins(srcF, b->long_capacity, b->wide_capacity, b->prm.bin_shift, pm, &b->plan[0], &why, p2);
    if (!rc) rc = plan_bins(srcW, b->long_capacity, b->wide_capacity, b->prm.bin_shift, pm, &b->plan[1], &why, p2);
    if (rc) return bfail(b, rc, why);
    const int groups = std::max(std::max(b->plan[0].max_groups, b->plan[1].max_groups), 1);
    const int pmax = std::max(std::max(b->plan[0].max_pmax, b->plan[1].max_pmax), 1);
    const size_t nw = (size_t)groups * 2 * pmax * kCoopValues + 1;
    if (nw > b->coop_words_n) {
        if (b->coop_words) (void)hipFree(b->coop_words);
        b->coop_words = nullptr;
        BHIP(b, dalloc(&b->coop_words, nw));
        b->coop_words_n = nw;
    }
    return NMFKL_OK;
}

// Every problem's model values in CSR order (the order the graph's F-half reads): computed
// from W and F if none are carried, converted if they are in CSC order.
int batch_models(nmfkl_batch* b) {
    for (nmfkl_handle* h : b->hs) {
        if (h->model == kModelNone) {
            const int rc = refresh_model(h);
            if (rc) return bfail(b, rc, h->err);
        }
        if (h->model == kModelCsc || h->model == kModelCscFresh) {
            BHIP(b, launch_gather_f64(h->Mcsc, h->csr2csc, h->prob.nnz, h->Mcsr, b->stream));
            h->model = kModelCsr;
        }
    }
    return NMFKL_OK;
}

// nsweeps outer iterations, t = *t_dev + k, on stream s.
hipError_t batch_enqueue(nmfkl_batch* b, hipStream_t s, int nsweeps, bool cooperative) {
    const int np = (int)b->hs.size();
    const bool la = (b->prm.tuning & 1) != 0;
    hipError_t e;
    for (int k = 0; k < nsweeps; ++k)
        for (int half = 0; half < 2; ++half) {
            const PermJob* jobs = b->jobtab + (size_t)half * np;
            if ((e = launch_permute_jobs(jobs, np, b->perm_blocks[half], k, b->t_dev, s)) != hipSuccess) return e;
            if ((e = launch_finalize_jobs(jobs, np, b->nsum[half], s)) != hipSuccess) return e;
            if ((e = enqueue_plan(b->plan[half], b->argtab + (size_t)half * np, b->coop_words,
                                  b->dev_err, cooperative, la, b->prm.collect_stats != 0, s, nullptr, 0, 0)) != hipSuccess)
                return e;
        }
    return hipSuccess;
}

hipError_t batch_capture(nmfkl_batch* b, int nsweeps, bool cooperative, hipGraphExec_t* exec) {
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t ee = batch_enqueue(b, b->cap, nsweeps, cooperative);
    e = hipStreamEndCapture(b->cap, &g);
    if (ee != hipSuccess || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return ee != hipSuccess ? ee : e;
    }
    e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    return e;
}

}  // namespace

extern "C" {

const char* nmfkl_batch_last_error(const nmfkl_batch* b) { return b ? b->err.c_str() : g_batch_error.c_str(); }

int nmfkl_batch_create(int32_t nprob, const nmfkl_problem* probs, const nmfkl_params* p, void* hip_stream,
                       nmfkl_batch** out) {
    if (!out) return bfail(nullptr, NMFKL_E_INVAL, "out is null");
    *out = nullptr;
    if (nprob < 1 || nprob > 65536) return bfail(nullptr, NMFKL_E_INVAL, "nprob must be in [1, 65536]");
    if (!probs) return bfail(nullptr, NMFKL_E_INVAL, "probs is null");
    nmfkl_params prm;
    if (p) prm = *p;
    else nmfkl_params_default(&prm);
    std::string why;
    if (check_params(&prm, &why)) return bfail(nullptr, NMFKL_E_INVAL, why);
    if (prm.out_of_core) return bfail(nullptr, NMFKL_E_UNSUPPORTED, "batches keep V in device memory");
    nmfkl_batch* b = new (std::nothrow) nmfkl_batch();
    if (!b) return bfail(nullptr, NMFKL_E_NOMEM, "host allocation failed");
    b->prm = prm;
    b->prm.collect_timings = 0;
    b->stream = reinterpret_cast<hipStream_t>(hip_stream);
    auto bail = [&](int code) {
        g_batch_error = b->err;
        if (b->stream) (void)hipStreamSynchronize(b->stream);
        batch_release(b);
        delete b;
        return code;
    };
    for (int32_t q = 0; q < nprob; ++q) {
        nmfkl_handle* h = nullptr;
        const int rc = nmfkl_create(&probs[q], &b->prm, hip_stream, &h);
        if (rc) {
            bfail(b, rc, "problem " + std::to_string(q) + ": " + nmfkl_last_error(nullptr));
            return bail(rc);
        }
        b->hs.push_back(h);
    }
    b->long_capacity = b->hs[0]->long_capacity;
    b->wide_capacity = b->hs[0]->wide_capacity;
    std::vector<SweepArgs> args(2 * (size_t)nprob);
    std::vector<PermJob> jobs(2 * (size_t)nprob);
    for (int half = 0; half < 2; ++half) {
        int first_block = 0, first_sum = 0;
        for (int32_t q = 0; q < nprob; ++q) {
            nmfkl_handle* h = b->hs[q];
            SweepArgs a[kNumArgs];
            PermJob j[kNumJobs];
            make_args(h, a);
            make_jobs(h, j);
            args[(size_t)half * nprob + q] = a[half == 0 ? kArgFfromCsr : kArgWfromCsc];
            PermJob jb = j[half == 0 ? kJobF : kJobW];
            jb.first_block = first_block;
            jb.first_sum = first_sum;
            first_block += jb.nblocks;
            first_sum += jb.r;
            jobs[(size_t)half * nprob + q] = jb;
        }
        b->perm_blocks[half] = first_block;
        b->nsum[half] = first_sum;
    }
    auto dev = [&](hipError_t e, const char* what) {
        bfail(b, NMFKL_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
        return bail(NMFKL_E_DEVICE);
    };
    hipError_t e;
    if ((e = dalloc(&b->argtab, args.size())) != hipSuccess) return dev(e, "allocation");
    if ((e = dalloc(&b->jobtab, jobs.size())) != hipSuccess) return dev(e, "allocation");
    if ((e = hipMemcpy(b->argtab, args.data(), args.size() * sizeof(SweepArgs), hipMemcpyHostToDevice)) != hipSuccess)
        return dev(e, "table upload");
    if ((e = hipMemcpy(b->jobtab, jobs.data(), jobs.size() * sizeof(PermJob), hipMemcpyHostToDevice)) != hipSuccess)
        return dev(e, "table upload");
    if ((e = dalloc(&b->dev_err, 1)) != hipSuccess) return dev(e, "allocation");
    if ((e = dalloc(&b->t_dev, 1)) != hipSuccess) return dev(e, "allocation");
    if ((e = hipMemsetAsync(b->dev_err, 0, sizeof(unsigned), b->stream)) != hipSuccess) return dev(e, "memset");
    if ((e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking)) != hipSuccess) return dev(e, "stream");
    const int rc = batch_plan(b);
    if (rc) return bail(rc);
    if ((e = hipStreamSynchronize(b->stream)) != hipSuccess) return dev(e, "synchronize");
    *out = b;
    return NMFKL_OK;
}

int nmfkl_batch_run(nmfkl_batch* b, int32_t t0, int32_t nsweeps) {
    if (!b) return bfail(nullptr, NMFKL_E_INVAL, "null batch");
    if (t0 < 0) return bfail(b, NMFKL_E_INVAL, "t0 must be >= 0");
    if (nsweeps < 1 || nsweeps > 100000) return bfail(b, NMFKL_E_INVAL, "nsweeps must be in [1, 100000]");
    int rc = batch_models(b);
    if (rc) return rc;
    hipGraphExec_t exec = nullptr;
    for (auto& g : b->graphs)
        if (g.first == nsweeps) exec = g.second;
    if (!exec) {
        // the capture stream must see the model work already enqueued on the caller's stream
        // only through the graph launch's stream order, so nothing else is needed here
        hipError_t e = hipErrorUnknown;
        if (b->graph_coop != 0) {
            e = batch_capture(b, nsweeps, true, &exec);
            if (e == hipSuccess) b->graph_coop = 1;
        }
        if (e != hipSuccess) {
            exec = nullptr;
            e = batch_capture(b, nsweeps, false, &exec);
            if (e != hipSuccess) return bfail(b, NMFKL_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
            b->graph_coop = 0;
        }
        b->graphs.emplace_back(nsweeps, exec);
    }
    BHIP(b, launch_set_i64(b->t_dev, t0, b->stream));
    BHIP(b, hipGraphLaunch(exec, b->stream));
    for (nmfkl_handle* h : b->hs) h->model = h->prm.tile_bf16 ? kModelNone : kModelCsr;
    return NMFKL_OK;
}

int nmfkl_batch_objective(nmfkl_batch* b, double* D_out) {
    if (!b) return bfail(nullptr, NMFKL_E_INVAL, "null batch");
    if (!D_out) return bfail(b, NMFKL_E_INVAL, "D_out is null");
    unsigned derr = 0;
    BHIP(b, hipMemcpyAsync(&derr, b->dev_err, sizeof(unsigned), hipMemcpyDeviceToHost, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    if (derr) return bfail(b, NMFKL_E_DEVICE, "a cross-block wait of a long segment timed out");
    for (size_t q = 0; q < b->hs.size(); ++q) {
        const int rc = objective_impl(b->hs[q], D_out + q, true);
        if (rc) return bfail(b, rc, "problem " + std::to_string(q) + ": " + b->hs[q]->err);
    }
    return NMFKL_OK;
}

int nmfkl_batch_tune(nmfkl_batch* b, int32_t t, nmfkl_params* chosen) {
    if (!b) return bfail(nullptr, NMFKL_E_INVAL, "null batch");
    if (t < 0) return bfail(b, NMFKL_E_INVAL, "t must be >= 0");
    int rc = batch_models(b);
    if (rc) return rc;
    // saved state: W, F and the CSR-order model values of every problem
    struct Saved { float* W = nullptr; float* F = nullptr; double* M = nullptr; };
    std::vector<Saved> sv(b->hs.size());
    auto free_saved = [&]() {
        for (auto& x : sv) {
            if (x.W) (void)hipFree(x.W);
            if (x.F) (void)hipFree(x.F);
            if (x.M) (void)hipFree(x.M);
            x = Saved{};
        }
    };
    auto copy_all = [&](bool save) -> hipError_t {
        hipError_t e;
        for (size_t q = 0; q < b->hs.size(); ++q) {
            const nmfkl_problem& pr = b->hs[q]->prob;
            const size_t nw = (size_t)pr.n * pr.r * sizeof(float), nf = (size_t)pr.m * pr.r * sizeof(float);
            const size_t nm = (size_t)pr.nnz * sizeof(double);
            if (save) {
                if ((e = hipMemcpyAsync(sv[q].W, pr.W, nw, hipMemcpyDeviceToDevice, b->stream)) != hipSuccess) return e;
                if ((e = hipMemcpyAsync(sv[q].F, pr.F, nf, hipMemcpyDeviceToDevice, b->stream)) != hipSuccess) return e;
                if (nm && (e = hipMemcpyAsync(sv[q].M, b->hs[q]->Mcsr, nm, hipMemcpyDeviceToDevice, b->stream)) != hipSuccess)
                    return e;
            } else {
                if ((e = hipMemcpyAsync(pr.W, sv[q].W, nw, hipMemcpyDeviceToDevice, b->stream)) != hipSuccess) return e;
                if ((e = hipMemcpyAsync(pr.F, sv[q].F, nf, hipMemcpyDeviceToDevice, b->stream)) != hipSuccess) return e;
                if (nm && (e = hipMemcpyAsync(b->hs[q]->Mcsr, sv[q].M, nm, hipMemcpyDeviceToDevice, b->stream)) != hipSuccess)
                    return e;
            }
        }
        return hipSuccess;
    };
    for (size_t q = 0; q < b->hs.size(); ++q) {
        const nmfkl_problem& pr = b->hs[q]->prob;
        hipError_t e = dalloc(&sv[q].W, (size_t)pr.n * pr.r);
        if (e == hipSuccess) e = dalloc(&sv[q].F, (size_t)pr.m * pr.r);
        if (e == hipSuccess) e = dalloc(&sv[q].M, (size_t)pr.nnz);
        if (e != hipSuccess) {
            free_saved();
            return bfail(b, NMFKL_E_NOMEM, "no device memory for the tuner's saved state");
        }
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const nmfkl_params orig = b->prm;
    int best_shift = orig.bin_shift, best_tuning = orig.tuning;
    float best_ms = 0.0f;
    bool have = false;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = copy_all(true);
    for (int shift = 0; shift <= 2 && e == hipSuccess && rc == NMFKL_OK; ++shift)
        for (int bits = 0; bits <= 7 && e == hipSuccess && rc == NMFKL_OK; ++bits) {
            b->prm.bin_shift = shift;
            b->prm.tuning = (orig.tuning & ~7) | bits;
            rc = batch_plan(b);
            if (rc) break;
            float ms = 0.0f;
            for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {  // the first run warms caches up
                if ((e = launch_set_i64(b->t_dev, t, b->stream)) != hipSuccess) break;
                if ((e = hipEventRecord(e0, b->stream)) != hipSuccess) break;
                if ((e = batch_enqueue(b, b->stream, 1, true)) != hipSuccess) break;
                if ((e = hipEventRecord(e1, b->stream)) != hipSuccess) break;
                if ((e = copy_all(false)) != hipSuccess) break;
                if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
                if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
            }
            if (e == hipSuccess && (!have || ms < best_ms)) {
                have = true;
                best_ms = ms;
                best_shift = shift;
                best_tuning = b->prm.tuning;
            }
        }
    hipError_t es = hipStreamSynchronize(b->stream);
    if (e == hipSuccess) e = es;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    free_saved();
    b->prm.bin_shift = have ? best_shift : orig.bin_shift;
    b->prm.tuning = have ? best_tuning : orig.tuning;
    const int rc2 = batch_plan(b);
    if (e != hipSuccess) return bfail(b, NMFKL_E_DEVICE, std::string("tuner: ") + hipGetErrorString(e));
    if (rc) return rc;
    if (rc2) return rc2;
    unsigned derr = 0;
    BHIP(b, hipMemcpy(&derr, b->dev_err, sizeof(unsigned), hipMemcpyDeviceToHost));
    if (derr) return bfail(b, NMFKL_E_DEVICE, "a cross-block wait of a long segment timed out");
    if (chosen) *chosen = b->prm;
    return NMFKL_OK;
}

int nmfkl_batch_get_info(nmfkl_batch* b, nmfkl_batch_info* out) {
    if (!b) return bfail(nullptr, NMFKL_E_INVAL, "null batch");
    if (!out) return bfail(b, NMFKL_E_INVAL, "out is null");
    std::memset(out, 0, sizeof(*out));
    out->nprob = (int32_t)b->hs.size();
    out->bin_shift = b->prm.bin_shift;
    out->tuning = b->prm.tuning;
    out->graph_cooperative = b->graph_coop;
    for (int half = 0; half < 2; ++half) {
        out->fused_blocks[half] = b->plan[half].nblocks;
        out->long_parts[half] = b->plan[half].rounds.empty() ? 0 : b->plan[half].rounds[0].nblocks;
        out->long_rounds[half] = (int32_t)b->plan[half].rounds.size();
    }
    for (nmfkl_handle* h : b->hs) out->nnz_total += h->prob.nnz;
    return NMFKL_OK;
}

int nmfkl_batch_destroy(nmfkl_batch* b) {
    if (!b) return NMFKL_E_INVAL;
    const hipError_t e = hipStreamSynchronize(b->stream);
    batch_release(b);
    delete b;
    return e == hipSuccess ? NMFKL_OK : NMFKL_E_DEVICE;
}

}  // extern "C"
