// C ABI of the NMF-KL coordinate-descent library: handle life cycle, validation, nnz
// binning, and the enqueue sequence of each half-sweep and of the objective.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
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
    // long segments: those fitting one block in an ordinary launch (single_blocks entries at
    // the start of long_work), the others in cooperative launches ("rounds"), each within
    // the co-residency capacity
    LongWork* long_work = nullptr;  // device: single-block entries, then all rounds
    int single_blocks = 0;
    struct Round { int first, nblocks, ngroups, pmax; };
    std::vector<Round> rounds;
    int max_groups = 0, max_pmax = 0;
    // algorithmic (gather-model) bytes and updates of the fused and of the long launches
    double fused_bytes = 0, fused_updates = 0, long_bytes = 0, long_updates = 0;
};

}  // namespace

struct nmfkl_handle {
    nmfkl_problem prob{};
    nmfkl_params prm{};
    hipStream_t stream = nullptr;
    int device = 0;
    int Sp = 0;
    // scratch
    float* Ap = nullptr;          // permuted padded copy of the fixed factor
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
    double* sums2 = nullptr;      // 2 x r natural-order sums (objective)
    double* dscal = nullptr;      // device scalar (objective total)
    double* host_scal = nullptr;  // pinned host scalar
    unsigned long long* stats = nullptr;
    double* coop_partials = nullptr;   // cross-block partial sums of long segments
    unsigned* coop_counters = nullptr; // their arrival flags (one line per block)
    unsigned* dev_err = nullptr;       // device-side error flags (bounded waits)
    int long_capacity = 0;             // co-resident long-segment blocks
    BinPlan binF, binW;
    // timing (params.collect_timings): event pairs per launch group, resolved on demand
    struct Pending { int kind; hipEvent_t a, b; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> event_pool;
    nmfkl_timings timings{};
    int model = kModelNone;
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
hipError_t take_event(nmfkl_handle* h, hipEvent_t* ev) {
    if (!h->event_pool.empty()) {
        *ev = h->event_pool.back();
        h->event_pool.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(ev);
}

// Starts a timed launch group; returns the index of the pending record or -1 when off.
int timer_begin(nmfkl_handle* h, int kind) {
    if (!h->prm.collect_timings) return -1;
    nmfkl_handle::Pending p{kind, nullptr, nullptr};
    if (take_event(h, &p.a) != hipSuccess || take_event(h, &p.b) != hipSuccess) return -1;
    if (hipEventRecord(p.a, h->stream) != hipSuccess) return -1;
    h->pending.push_back(p);
    return (int)h->pending.size() - 1;
}

void timer_end(nmfkl_handle* h, int idx) {
    if (idx < 0) return;
    (void)hipEventRecord(h->pending[idx].b, h->stream);
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
        h->event_pool.push_back(p.a);
        h->event_pool.push_back(p.b);
    }
    h->pending.clear();
    return hipSuccess;
}

void release(nmfkl_handle* h) {
    for (auto& p : h->pending) { h->event_pool.push_back(p.a); h->event_pool.push_back(p.b); }
    h->pending.clear();
    for (hipEvent_t ev : h->event_pool) (void)hipEventDestroy(ev);
    h->event_pool.clear();
    auto f = [](void* p) { if (p) (void)hipFree(p); };
    f(h->Ap); f(h->sumA); f(h->partials); f(h->ids); f(h->Mcsc); f(h->Mcsr);
    f(h->csc2csr); f(h->csr2csc); f(h->obj_partials); f(h->sums2); f(h->dscal); f(h->stats);
    f(h->binF.work); f(h->binF.segs); f(h->binW.work); f(h->binW.segs);
    f(h->binF.long_work); f(h->binW.long_work);
    f(h->coop_partials); f(h->coop_counters); f(h->dev_err);
    if (h->host_scal) (void)hipHostFree(h->host_scal);
}

// Variant for a segment of length L in the fused launch (-1: too long).
int variant_for(int64_t L) {
    for (int v = 0; v < kNumVariants; ++v)
        if (L <= (int64_t)kVariants[v].G * kVariants[v].E) return v;
    return -1;
}

// Segments up to kMaxFusedLength: grouped by variant (longest variants first, so that long
// blocks start early) and cut into blocks of kFusedThreads / G segments.  Longer segments:
// B = ceil(L / kLongCapacity) blocks each, packed longest first into cooperative rounds of at
// most long_capacity blocks.
int plan_bins(nmfkl_handle* h, const int64_t* dptr, int64_t Q, BinPlan* plan) {
    std::vector<int64_t> ptr(Q + 1);
    HIP_TRY(h, hipMemcpy(ptr.data(), dptr, (Q + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
    auto len = [&](int32_t q) { return ptr[q + 1] - ptr[q]; };
    std::vector<std::vector<int32_t>> groups(kNumVariants);
    std::vector<int32_t> longs;
    for (int64_t q = 0; q < Q; ++q) {
        const int v = variant_for(len((int32_t)q));
        if (v < 0) longs.push_back((int32_t)q);
        else groups[v].push_back((int32_t)q);
    }
    const double r = h->prob.r;
    auto seg_bytes = [&](int32_t q) { return (double)len(q) * (8.0 + 4.0 * r) + 8.0 + 8.0 * r; };
    for (int v = 0; v < kNumVariants; ++v)
        for (int32_t q : groups[v]) { plan->fused_bytes += seg_bytes(q); plan->fused_updates += (double)len(q) * r; }
    for (int32_t q : longs) { plan->long_bytes += seg_bytes(q); plan->long_updates += (double)len(q) * r; }
    std::vector<int32_t> segs;
    std::vector<BlockWork> work;
    for (int v = kNumVariants - 1; v >= 0; --v) {
        const int spb = kFusedThreads / kVariants[v].G;
        auto& g = groups[v];
        std::stable_sort(g.begin(), g.end(), [&](int32_t a, int32_t b) { return len(a) > len(b); });
        for (size_t i = 0; i < g.size(); i += spb) {
            BlockWork w;
            w.variant = v;
            w.first = (int32_t)segs.size();
            w.count = (int32_t)std::min<size_t>(spb, g.size() - i);
            w.pad = 0;
            for (int k = 0; k < w.count; ++k) segs.push_back(g[i + k]);
            work.push_back(w);
        }
    }
    plan->nblocks = (int)work.size();
    HIP_TRY(h, dalloc(&plan->work, work.size()));
    HIP_TRY(h, dalloc(&plan->segs, segs.size()));
    if (!work.empty())
        HIP_TRY(h, hipMemcpy(plan->work, work.data(), work.size() * sizeof(BlockWork), hipMemcpyHostToDevice));
    if (!segs.empty())
        HIP_TRY(h, hipMemcpy(plan->segs, segs.data(), segs.size() * sizeof(int32_t), hipMemcpyHostToDevice));

    std::stable_sort(longs.begin(), longs.end(), [&](int32_t a, int32_t b) { return len(a) > len(b); });
    std::vector<LongWork> lw;
    for (int32_t q : longs)
        if (len(q) <= kLongCapacity) lw.push_back(LongWork{q, 0, 1, 0});
    plan->single_blocks = (int)lw.size();
    BinPlan::Round cur{(int)lw.size(), 0, 0, 0};
    for (int32_t q : longs) {
        const int B = (int)((len(q) + kLongCapacity - 1) / kLongCapacity);
        if (B == 1) continue;
        if (B > h->long_capacity)
            return fail(h, NMFKL_E_UNSUPPORTED,
                        "a segment of " + std::to_string(len(q)) + " nonzeros needs " + std::to_string(B) +
                            " co-resident blocks; this device holds " + std::to_string(h->long_capacity));
        if (cur.nblocks + B > h->long_capacity) {
            plan->rounds.push_back(cur);
            cur = BinPlan::Round{(int)lw.size(), 0, 0, 0};
        }
        for (int p = 0; p < B; ++p) lw.push_back(LongWork{q, p, B, cur.ngroups});
        cur.nblocks += B;
        cur.ngroups += 1;
        cur.pmax = std::max(cur.pmax, B);
    }
    if (cur.nblocks > 0) plan->rounds.push_back(cur);
    for (const auto& r : plan->rounds) {
        plan->max_groups = std::max(plan->max_groups, r.ngroups);
        plan->max_pmax = std::max(plan->max_pmax, r.pmax);
    }
    if (!lw.empty()) {
        HIP_TRY(h, dalloc(&plan->long_work, lw.size()));
        HIP_TRY(h, hipMemcpy(plan->long_work, lw.data(), lw.size() * sizeof(LongWork), hipMemcpyHostToDevice));
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
    return a;
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

int half_sweep(nmfkl_handle* h, int32_t t, bool fhalf) {
    if (!h) return fail(nullptr, NMFKL_E_INVAL, "null handle");
    if (t < 0) return fail(h, NMFKL_E_INVAL, "t must be >= 0");
    const nmfkl_problem& pr = h->prob;
    const BinPlan& plan = fhalf ? h->binF : h->binW;
    if (fhalf) {
        const bool fresh_needed = h->model == kModelNone || (h->prm.refresh_model && h->model != kModelCscFresh);
        if (fresh_needed) {
            const int rc = refresh_model(h);
            if (rc) return rc;
        }
    } else if (h->model == kModelNone) {
        const int rc = refresh_model(h);
        if (rc) return rc;
    }
    const float* A = fhalf ? pr.W : pr.F;
    const int64_t P = fhalf ? pr.n : pr.m;
    const int ts = timer_begin(h, fhalf ? NMFKL_T_SUMS_F : NMFKL_T_SUMS_W);
    OrderArg order{};
    coordinate_order(h->prm.seed, (uint64_t)t, 0, pr.r, order.ids);
    HIP_TRY(h, launch_permute_colsum(A, P, pr.r, h->Sp, order, h->ids, h->Ap, h->partials, h->sum_blocks, h->stream));
    HIP_TRY(h, launch_finalize_sums(h->partials, h->sum_blocks, pr.r, h->sumA, h->stream));
    timer_end(h, ts);
    SweepArgs a = sweep_args(h, fhalf);
    if (fhalf) {
        const bool from_csc = h->model == kModelCsc || h->model == kModelCscFresh;
        a.Min = from_csc ? h->Mcsc : h->Mcsr;
        a.Mmap = from_csc ? nullptr : h->csc2csr;
        a.Mout = h->Mcsc;
        // in-place read/write of Mcsc is safe: each entry is read and written by one lane
    } else {
        const bool from_csr = h->model == kModelCsr;
        a.Min = from_csr ? h->Mcsr : h->Mcsc;
        a.Mmap = from_csr ? nullptr : h->csr2csc;
        a.Mout = h->Mcsr;
    }
    const bool any_long = plan.single_blocks > 0 || !plan.rounds.empty();
    const int tl = any_long ? timer_begin(h, fhalf ? NMFKL_T_LONG_F : NMFKL_T_LONG_W) : -1;
    HIP_TRY(h, launch_sweep_long_single(a, plan.long_work, plan.single_blocks, h->stream));
    for (const auto& rd : plan.rounds)
        HIP_TRY(h, launch_sweep_long(a, plan.long_work + rd.first, rd.nblocks, h->coop_partials,
                                     h->coop_counters, rd.ngroups, h->dev_err, rd.pmax, h->stream));
    timer_end(h, tl);
    const int tf = plan.nblocks ? timer_begin(h, fhalf ? NMFKL_T_FUSED_F : NMFKL_T_FUSED_W) : -1;
    HIP_TRY(h, launch_sweep_fused(a, plan.work, plan.segs, plan.nblocks, (h->prm.tuning & 1) != 0, h->stream));
    timer_end(h, tf);
    h->model = fhalf ? kModelCsc : kModelCsr;
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
    CREATE_HIP(dalloc(&h->partials, (size_t)h->sum_blocks * pr.r));
    CREATE_HIP(dalloc(&h->ids, NMFKL_R_MAX));
    CREATE_HIP(dalloc(&h->Mcsc, nnz));
    CREATE_HIP(dalloc(&h->Mcsr, nnz));
    h->obj_blocks = (int)std::min<int64_t>(4096, std::max<int64_t>(1, pr.m / 8));
    CREATE_HIP(dalloc(&h->obj_partials, h->obj_blocks));
    CREATE_HIP(dalloc(&h->sums2, 2 * (size_t)pr.r));
    CREATE_HIP(dalloc(&h->dscal, 1));
    CREATE_HIP(dalloc(&h->stats, 6));
    CREATE_HIP(hipMemsetAsync(h->stats, 0, 6 * sizeof(unsigned long long), h->stream));
    CREATE_HIP(hipHostMalloc(reinterpret_cast<void**>(&h->host_scal), sizeof(double), hipHostMallocDefault));
    {
        int ncu = 0;
        CREATE_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device));
        h->long_capacity = long_kernel_blocks_per_cu() * ncu;
        if (h->long_capacity <= 0) {
            fail(h, NMFKL_E_DEVICE, "occupancy query of the long-segment kernel failed");
            return bail(NMFKL_E_DEVICE);
        }
        int rc = plan_bins(h, pr.csc_ptr, pr.m, &h->binF);
        if (rc) return bail(rc);
        rc = plan_bins(h, pr.csr_ptr, pr.n, &h->binW);
        if (rc) return bail(rc);
        const int groups = std::max(h->binF.max_groups, h->binW.max_groups);
        const int pmax = std::max(h->binF.max_pmax, h->binW.max_pmax);
        // k_sweep_long<true> addresses partials + group * (2 * pmax * kCoopValues) + ...
        CREATE_HIP(dalloc(&h->coop_partials, (size_t)std::max(groups, 1) * 2 * std::max(pmax, 1) * kCoopValues));
        // ... and flags + group * (pmax * kFlagStride) + part * kFlagStride
        CREATE_HIP(dalloc(&h->coop_counters, (size_t)std::max(groups, 1) * std::max(pmax, 1) * kFlagStride));
        CREATE_HIP(dalloc(&h->dev_err, 1));
        CREATE_HIP(hipMemsetAsync(h->dev_err, 0, sizeof(unsigned), h->stream));
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
}

int nmfkl_objective(nmfkl_handle* h, double* D_out) { return objective_impl(h, D_out, false); }

int nmfkl_objective_carried(nmfkl_handle* h, double* D_out) { return objective_impl(h, D_out, true); }

namespace {
int objective_impl(nmfkl_handle* h, double* D_out, bool carried) {
    if (!h) return fail(nullptr, NMFKL_E_INVAL, "null handle");
    if (!D_out) return fail(h, NMFKL_E_INVAL, "D_out is null");
    const nmfkl_problem& pr = h->prob;
    unsigned* flags = nullptr;
    // natural-order float64 column sums of W and F: sum over all cells of W^T F = sumW . sumF
    OrderArg identity{};
    for (int k = 0; k < pr.r; ++k) identity.ids[k] = k;
    HIP_TRY(h, launch_permute_colsum(pr.W, pr.n, pr.r, h->Sp, identity, nullptr, nullptr, h->partials, h->sum_blocks, h->stream));
    HIP_TRY(h, launch_finalize_sums(h->partials, h->sum_blocks, pr.r, h->sums2, h->stream));
    HIP_TRY(h, launch_permute_colsum(pr.F, pr.m, pr.r, h->Sp, identity, nullptr, nullptr, h->partials, h->sum_blocks, h->stream));
    HIP_TRY(h, launch_finalize_sums(h->partials, h->sum_blocks, pr.r, h->sums2 + pr.r, h->stream));
    if (carried && (h->model == kModelCsr || h->model == kModelCsc || h->model == kModelCscFresh)) {
        const bool csr = h->model == kModelCsr;
        const int tm = timer_begin(h, NMFKL_T_MODEL);
        HIP_TRY(h, launch_model_terms(csr ? h->Mcsr : h->Mcsc, csr ? pr.csr_val : pr.csc_val, pr.nnz,
                                      h->obj_partials, h->obj_blocks, h->stream));
        timer_end(h, tm);
    } else {
        const int rc = refresh_model(h);
        if (rc) return rc;
    }
    HIP_TRY(h, launch_sum_f64(h->obj_partials, h->obj_blocks, h->dscal, h->stream));
    double part = 0.0;
    std::vector<double> sums(2 * (size_t)pr.r);
    HIP_TRY(h, hipMemcpyAsync(h->host_scal, h->dscal, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipMemcpyAsync(sums.data(), h->sums2, sums.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    unsigned derr = 0;
    HIP_TRY(h, hipMemcpyAsync(&derr, h->dev_err, sizeof(unsigned), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    if (derr) return fail(h, NMFKL_E_DEVICE, "a cross-block wait of a long segment timed out");
    part = *h->host_scal;
    double total = 0.0;
    for (int k = 0; k < pr.r; ++k) {
        if (!std::isfinite(sums[k]) || !std::isfinite(sums[pr.r + k]))
            return fail(h, NMFKL_E_NONFINITE, "a factor holds NaN or Inf");
        total += sums[k] * sums[pr.r + k];
    }
    (void)flags;
    if (std::isnan(part)) return fail(h, NMFKL_E_NONFINITE, "objective is NaN");
    *D_out = part + total;
    return NMFKL_OK;
}
}  // namespace

int nmfkl_get_stats(nmfkl_handle* h, nmfkl_stats* out) {
    if (!h) return fail(nullptr, NMFKL_E_INVAL, "null handle");
    if (!out) return fail(h, NMFKL_E_INVAL, "out is null");
    unsigned long long c[6];
    HIP_TRY(h, hipMemcpyAsync(c, h->stats, sizeof(c), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    out->coords = (int64_t)c[0];
    out->evals = (int64_t)c[1];
    out->steps = (int64_t)c[2];
    out->halvings = (int64_t)c[3];
    out->rejects = (int64_t)c[4];
    out->tmax_hits = (int64_t)c[5];
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
