// C ABI of fold-in (W fixed) and of the continuously batched fold-in server.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "nmfkl_internal.hpp"

using namespace nmfkl;

namespace {
thread_local std::string g_model_error;

double now_seconds() {
    using clk = std::chrono::steady_clock;
    return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}
}  // namespace

struct nmfkl_model {
    int32_t n = 0, r = 0;
    const float* W = nullptr;
    nmfkl_params prm{};
    hipStream_t stream = nullptr;
    double* sumW = nullptr;
    double* rowsumW = nullptr;
    double totW = 0.0;
    int32_t* perm = nullptr;  // [foldin_max_passes][r]
    unsigned long long* stats = nullptr;
    // plain fold-in scratch
    int32_t* docs = nullptr;
    size_t docs_cap = 0;
    std::string err;
};

namespace {

int mfail(nmfkl_model* m, int code, const std::string& msg) {
    if (m) m->err = msg;
    else g_model_error = msg;
    return code;
}

#define MHIP(m, expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) return mfail(m, NMFKL_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

SweepArgs foldin_sweep_args(const nmfkl_model* m) {
    SweepArgs a{};
    a.r = m->r;
    a.alpha = (float)m->prm.alpha_F;
    a.beta = (float)m->prm.beta_F;
    a.eps_log = (float)m->prm.eps_log;
    a.eps_g = (float)m->prm.eps_g;
    a.eps_x = (float)m->prm.eps_x;
    a.t_max = m->prm.t_max;
    a.j_max = m->prm.j_max;
    a.literal_break = m->prm.literal_break;
    a.guard = m->prm.guard;
    a.sumA = m->sumW;
    a.stats = m->prm.collect_stats ? m->stats : nullptr;
    return a;
}

FoldinArgs foldin_args(const nmfkl_model* m, const int64_t* ptr, const int32_t* idx, const float* val,
                       float* F, int32_t* passes, double* kl) {
    FoldinArgs f{};
    f.ptr = ptr;
    f.idx = idx;
    f.val = val;
    f.W = m->W;
    f.sumW = m->sumW;
    f.rowsumW = m->rowsumW;
    f.totW = m->totW;
    f.perm = m->perm;
    f.F = F;
    f.passes = passes;
    f.kl = kl;
    f.r = m->r;
    f.max_passes = m->prm.foldin_max_passes;
    f.tol = m->prm.foldin_tol;
    return f;
}

int variant_of_length(int64_t L) {
    for (int v = 0; v < kFoldinVariants; ++v)
        if (L <= kFoldinCapacity[v]) return v;
    return -1;
}

// Documents grouped by variant; returns NMFKL_E_UNSUPPORTED for a document above the largest
// capacity.  lists[v] holds document indices.
int group_docs(nmfkl_model* m, const std::vector<int64_t>& len, std::vector<int32_t> lists[kFoldinVariants]) {
    for (size_t d = 0; d < len.size(); ++d) {
        const int v = variant_of_length(len[d]);
        if (v < 0)
            return mfail(m, NMFKL_E_UNSUPPORTED, "a document has " + std::to_string(len[d]) +
                                                     " distinct words; fold-in supports up to " +
                                                     std::to_string(kFoldinCapacity[kFoldinVariants - 1]));
        lists[v].push_back((int32_t)d);
    }
    return NMFKL_OK;
}

// Launch the variants for grouped documents whose lists were uploaded to dev_docs (variant v
// at offset off[v]), shortest documents first: the launches of a stream run one after the
// other, so the many short documents of a batch finish (and, in the server, come back) before
// the few long ones have started.
int launch_grouped(nmfkl_model* m, const FoldinArgs& f, const int32_t* dev_docs, const int off[kFoldinVariants],
                   const int cnt[kFoldinVariants], hipStream_t stream) {
    const SweepArgs a = foldin_sweep_args(m);
    for (int v = 0; v < kFoldinVariants; ++v)
        MHIP(m, launch_foldin(f, a, v, dev_docs + off[v], cnt[v], stream));
    return NMFKL_OK;
}

}  // namespace

// ----------------------------------------------------------------------------- server
// Each lane is a stream that runs one batch of documents at a time.  Documents are returned
// one by one as they finish: the fold-in kernels write every document's result straight into
// host-coherent pinned memory and then set the document's completion word to the batch tag,
// which the host polls.  A lane takes a new batch once every document of the current one has
// been returned and the lane's stream is idle.
struct nmfkl_server {
    nmfkl_model* model = nullptr;
    int64_t budget_words = 0;     // device words (index + count) that may be in flight
    int32_t max_docs = 0;         // documents per lane batch
    int64_t lane_words = 0;       // words per lane batch
    int32_t max_queued = 0;       // documents that may wait for a lane (0: no limit)
    struct Req {
        uint64_t id;
        int32_t L;
        double t_submit;
        double expires;            // steady-clock seconds after which it is not launched (0: never)
        std::vector<int32_t> idx;  // host copy of the document (taken at submit)
        std::vector<float> val;
    };
    struct Lane {
        hipStream_t stream = nullptr;
        hipEvent_t done = nullptr;
        bool busy = false;
        unsigned tag = 0;           // batch tag written into h_flag by the kernels
        int64_t* d_ptr = nullptr;
        int32_t* d_idx = nullptr;
        float* d_val = nullptr;
        int32_t* d_docs = nullptr;
        int64_t* h_ptr = nullptr;   // pinned staging of the batch
        int32_t* h_idx = nullptr;
        float* h_val = nullptr;
        int32_t* h_docs = nullptr;
        float* h_F = nullptr;       // host-coherent outputs, written by the kernels
        int32_t* h_passes = nullptr;
        double* h_kl = nullptr;
        unsigned* h_flag = nullptr;
        float* k_F = nullptr;       // the same outputs as device addresses
        int32_t* k_passes = nullptr;
        double* k_kl = nullptr;
        unsigned* k_flag = nullptr;
        std::vector<Req> reqs;
        std::vector<char> returned;
        int32_t nreturned = 0;
        int64_t words = 0;
    };
    std::vector<Lane> lanes;
    std::deque<Req> pending;
    int64_t timed_pending = 0;       // waiting documents that have a time limit
    int64_t words_in_flight = 0;     // pending + launched
    struct Done {
        uint64_t id;
        int32_t passes, status;
        double kl, t_submit, t_done;
        std::vector<float> f;
    };
    std::deque<Done> done;
    std::string err;
};

namespace {

int sfail(nmfkl_server* s, int code, const std::string& msg) {
    if (s) s->err = msg;
    else g_model_error = msg;
    return code;
}

#define SHIP(s, expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) return sfail(s, NMFKL_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

void release_lane(nmfkl_server::Lane& L) {
    auto df = [](void* p) { if (p) (void)hipFree(p); };
    auto hf = [](void* p) { if (p) (void)hipHostFree(p); };
    df(L.d_ptr); df(L.d_idx); df(L.d_val); df(L.d_docs);
    hf(L.h_ptr); hf(L.h_idx); hf(L.h_val); hf(L.h_docs); hf(L.h_F); hf(L.h_passes); hf(L.h_kl); hf(L.h_flag);
    if (L.done) (void)hipEventDestroy(L.done);
    if (L.stream) (void)hipStreamDestroy(L.stream);
}

void finish_unlaunched(nmfkl_server* s, nmfkl_server::Req&& q, int status, double t) {
    if (q.expires > 0.0) --s->timed_pending;
    nmfkl_server::Done d;
    d.id = q.id;
    d.passes = 0;
    d.status = status;
    d.kl = 0.0;
    d.t_submit = q.t_submit;
    d.t_done = t;
    d.f.assign((size_t)s->model->r, 0.0f);
    s->words_in_flight -= q.L;
    s->done.push_back(std::move(d));
}

// Return the finished documents of every busy lane; free a lane whose documents are all back.
int collect(nmfkl_server* s) {
    const int r = s->model->r;
    for (auto& L : s->lanes) {
        if (!L.busy) continue;
        const int nd = (int)L.reqs.size();
        double t = 0.0;
        for (int i = 0; i < nd; ++i) {
            if (L.returned[i]) continue;
            if (__atomic_load_n(L.h_flag + i, __ATOMIC_ACQUIRE) != L.tag) continue;
            if (t == 0.0) t = now_seconds();
            nmfkl_server::Done d;
            d.id = L.reqs[i].id;
            d.passes = L.h_passes[i];
            d.status = NMFKL_OK;
            d.kl = L.h_kl[i];
            d.t_submit = L.reqs[i].t_submit;
            d.t_done = t;
            d.f.assign(L.h_F + (size_t)i * r, L.h_F + (size_t)(i + 1) * r);
            s->done.push_back(std::move(d));
            L.returned[i] = 1;
            ++L.nreturned;
        }
        if (L.nreturned < nd) {
            // a device error would leave documents unfinished: surface it
            const hipError_t q = hipEventQuery(L.done);
            if (q != hipSuccess && q != hipErrorNotReady)
                return sfail(s, NMFKL_E_DEVICE, std::string("lane: ") + hipGetErrorString(q));
            if (q == hipSuccess) {
                // the kernels have ended: every completion word must be set
                for (int i = 0; i < nd; ++i)
                    if (!L.returned[i] && __atomic_load_n(L.h_flag + i, __ATOMIC_ACQUIRE) != L.tag)
                        return sfail(s, NMFKL_E_DEVICE, "lane ended with an unfinished document");
            }
            continue;
        }
        const hipError_t q = hipEventQuery(L.done);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return sfail(s, NMFKL_E_DEVICE, std::string("lane: ") + hipGetErrorString(q));
        s->words_in_flight -= L.words;
        L.reqs.clear();
        L.words = 0;
        L.busy = false;
    }
    return NMFKL_OK;
}

// Return every waiting document whose time limit has passed (only while some have one), so
// that a caller learns of it while the lanes are still busy.
void expire_pending(nmfkl_server* s) {
    if (s->timed_pending == 0) return;
    const double t = now_seconds();
    for (auto it = s->pending.begin(); it != s->pending.end();) {
        if (it->expires > 0.0 && t > it->expires) {
            nmfkl_server::Req q = std::move(*it);
            it = s->pending.erase(it);
            finish_unlaunched(s, std::move(q), NMFKL_RESULT_EXPIRED, t);
        } else {
            ++it;
        }
    }
}

// Form a batch for every idle lane from the waiting documents (FIFO; those past their time
// limit are returned as expired instead) and launch it.
int dispatch(nmfkl_server* s) {
    nmfkl_model* m = s->model;
    double t = 0.0;
    for (auto& L : s->lanes) {
        if (L.busy || s->pending.empty()) continue;
        int nd = 0;
        int64_t w = 0;
        L.h_ptr[0] = 0;
        while (!s->pending.empty() && nd < s->max_docs && w + s->pending.front().L <= s->lane_words) {
            nmfkl_server::Req q = std::move(s->pending.front());
            s->pending.pop_front();
            if (q.expires > 0.0) {
                if (t == 0.0) t = now_seconds();
                if (t > q.expires) {
                    finish_unlaunched(s, std::move(q), NMFKL_RESULT_EXPIRED, t);
                    continue;
                }
            }
            if (q.expires > 0.0) --s->timed_pending;
            std::memcpy(L.h_idx + w, q.idx.data(), (size_t)q.L * sizeof(int32_t));
            std::memcpy(L.h_val + w, q.val.data(), (size_t)q.L * sizeof(float));
            w += q.L;
            L.h_ptr[nd + 1] = w;
            q.idx.clear();
            q.val.clear();
            L.reqs.push_back(std::move(q));
            ++nd;
        }
        if (nd == 0) continue;
        // group by variant
        std::vector<int32_t> lists[kFoldinVariants];
        for (int d = 0; d < nd; ++d) lists[variant_of_length(L.h_ptr[d + 1] - L.h_ptr[d])].push_back(d);
        int off[kFoldinVariants], cnt[kFoldinVariants], pos = 0;
        for (int v = 0; v < kFoldinVariants; ++v) {
            off[v] = pos;
            cnt[v] = (int)lists[v].size();
            std::memcpy(L.h_docs + pos, lists[v].data(), lists[v].size() * sizeof(int32_t));
            pos += cnt[v];
        }
        L.tag += 1u;
        if (L.tag == 0u) L.tag = 1u;   // 0 is the words' initial value
        SHIP(s, hipMemcpyAsync(L.d_ptr, L.h_ptr, (size_t)(nd + 1) * sizeof(int64_t), hipMemcpyHostToDevice, L.stream));
        SHIP(s, hipMemcpyAsync(L.d_idx, L.h_idx, (size_t)w * sizeof(int32_t), hipMemcpyHostToDevice, L.stream));
        SHIP(s, hipMemcpyAsync(L.d_val, L.h_val, (size_t)w * sizeof(float), hipMemcpyHostToDevice, L.stream));
        SHIP(s, hipMemcpyAsync(L.d_docs, L.h_docs, (size_t)pos * sizeof(int32_t), hipMemcpyHostToDevice, L.stream));
        FoldinArgs f = foldin_args(m, L.d_ptr, L.d_idx, L.d_val, L.k_F, L.k_passes, L.k_kl);
        f.done = L.k_flag;
        f.done_tag = L.tag;
        const int rc = launch_grouped(m, f, L.d_docs, off, cnt, L.stream);
        if (rc) return sfail(s, rc, m->err);
        SHIP(s, hipEventRecord(L.done, L.stream));
        L.returned.assign((size_t)nd, 0);
        L.nreturned = 0;
        L.words = w;
        L.busy = true;
    }
    return NMFKL_OK;
}

}  // namespace

extern "C" {

const char* nmfkl_model_last_error(const nmfkl_model* m) { return m ? m->err.c_str() : g_model_error.c_str(); }

int nmfkl_model_create(const float* W, int32_t n, int32_t r, const nmfkl_params* p, void* hip_stream,
                       nmfkl_model** out) {
    if (!out) return mfail(nullptr, NMFKL_E_INVAL, "out is null");
    *out = nullptr;
    if (!W) return mfail(nullptr, NMFKL_E_INVAL, "W is null");
    if (n < 1) return mfail(nullptr, NMFKL_E_INVAL, "n must be >= 1");
    if (r < 1 || r > NMFKL_R_MAX) return mfail(nullptr, NMFKL_E_INVAL, "r must be in [1, NMFKL_R_MAX]");
    nmfkl_params prm;
    if (p) prm = *p;
    else nmfkl_params_default(&prm);
    if (prm.foldin_max_passes < 1 || prm.foldin_max_passes > 100000 || !(prm.foldin_tol >= 0) || prm.t_max < 1 ||
        prm.j_max < 0 || !(prm.eps_log >= 0) || !(prm.eps_g >= 0) || !(prm.eps_x >= 0) || !(prm.alpha_F >= 0) ||
        !(prm.beta_F >= 0))
        return mfail(nullptr, NMFKL_E_INVAL, "invalid parameters");
    nmfkl_model* m = new (std::nothrow) nmfkl_model();
    if (!m) return mfail(nullptr, NMFKL_E_NOMEM, "host allocation failed");
    m->n = n;
    m->r = r;
    m->W = W;
    m->prm = prm;
    m->stream = reinterpret_cast<hipStream_t>(hip_stream);
    auto bail = [&](int code) {
        g_model_error = m->err;
        nmfkl_model_destroy(m);
        return code;
    };
#define CM(expr)                                                                            \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) { mfail(m, NMFKL_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); return bail(NMFKL_E_DEVICE); } \
    } while (0)
    unsigned* flags = nullptr;
    CM(hipMalloc(reinterpret_cast<void**>(&flags), sizeof(unsigned)));
    CM(hipMemsetAsync(flags, 0, sizeof(unsigned), m->stream));
    CM(launch_validate_factor(W, (int64_t)n * r, flags, kBadW, m->stream));
    unsigned hf = 0;
    CM(hipMemcpyAsync(&hf, flags, sizeof(unsigned), hipMemcpyDeviceToHost, m->stream));
    CM(hipStreamSynchronize(m->stream));
    (void)hipFree(flags);
    if (hf) {
        mfail(m, NMFKL_E_INVAL, "W negative or not finite");
        return bail(NMFKL_E_INVAL);
    }
    CM(hipMalloc(reinterpret_cast<void**>(&m->sumW), sizeof(double) * NMFKL_R_MAX));
    CM(hipMalloc(reinterpret_cast<void**>(&m->rowsumW), sizeof(double) * n));
    const int blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, n / 64));
    double* partials = nullptr;
    CM(hipMalloc(reinterpret_cast<void**>(&partials), sizeof(double) * blocks * r));
    PermJob job{};
    job.A = W;
    job.partials = partials;
    job.sums = m->sumW;
    job.P = n;
    job.rpb = (n + blocks - 1) / blocks;
    job.r = r;
    job.Sp = r;
    job.nblocks = blocks;
    job.identity = 1;
    PermJob* djob = nullptr;
    CM(hipMalloc(reinterpret_cast<void**>(&djob), sizeof(PermJob)));
    CM(hipMemcpyAsync(djob, &job, sizeof(PermJob), hipMemcpyHostToDevice, m->stream));
    CM(launch_permute_jobs(djob, 1, blocks, 0, nullptr, m->stream));
    CM(launch_finalize_jobs(djob, 1, r, m->stream));
    CM(launch_row_sums(W, n, r, m->rowsumW, m->stream));
    std::vector<double> sw(r);
    CM(hipMemcpyAsync(sw.data(), m->sumW, sizeof(double) * r, hipMemcpyDeviceToHost, m->stream));
    const int P = prm.foldin_max_passes;
    std::vector<int32_t> perm((size_t)P * r);
    for (int q = 0; q < P; ++q) coordinate_order(prm.seed, (uint64_t)q, 1, r, perm.data() + (size_t)q * r);
    CM(hipMalloc(reinterpret_cast<void**>(&m->perm), sizeof(int32_t) * perm.size()));
    CM(hipMemcpyAsync(m->perm, perm.data(), sizeof(int32_t) * perm.size(), hipMemcpyHostToDevice, m->stream));
    CM(hipMalloc(reinterpret_cast<void**>(&m->stats), sizeof(unsigned long long) * 6));
    CM(hipMemsetAsync(m->stats, 0, sizeof(unsigned long long) * 6, m->stream));
    CM(hipStreamSynchronize(m->stream));
    (void)hipFree(partials);
    (void)hipFree(djob);
    m->totW = 0.0;
    for (int k = 0; k < r; ++k) m->totW += sw[k];
#undef CM
    *out = m;
    return NMFKL_OK;
}

int nmfkl_foldin(nmfkl_model* m, int32_t ndocs, const int64_t* doc_ptr, const int32_t* word_idx,
                 const float* counts, float* F_out, int32_t* passes_out, double* kl_out) {
    if (!m) return mfail(nullptr, NMFKL_E_INVAL, "null model");
    if (ndocs < 0) return mfail(m, NMFKL_E_INVAL, "ndocs must be >= 0");
    if (ndocs == 0) return NMFKL_OK;
    if (!doc_ptr || !F_out || !passes_out || !kl_out) return mfail(m, NMFKL_E_INVAL, "null pointer");
    std::vector<int64_t> ptr(ndocs + 1);
    MHIP(m, hipMemcpyAsync(ptr.data(), doc_ptr, sizeof(int64_t) * (ndocs + 1), hipMemcpyDeviceToHost, m->stream));
    MHIP(m, hipStreamSynchronize(m->stream));
    if (ptr[0] != 0) return mfail(m, NMFKL_E_INVAL, "doc_ptr[0] must be 0");
    std::vector<int64_t> len(ndocs);
    for (int d = 0; d < ndocs; ++d) {
        len[d] = ptr[d + 1] - ptr[d];
        if (len[d] < 0) return mfail(m, NMFKL_E_INVAL, "doc_ptr not monotone");
    }
    const int64_t nnz = ptr[ndocs];
    if (nnz > INT32_MAX) return mfail(m, NMFKL_E_UNSUPPORTED, "more than 2^31-1 words in one call");
    if (nnz > 0 && (!word_idx || !counts)) return mfail(m, NMFKL_E_INVAL, "null word/count pointer");
    unsigned* flags = nullptr;
    MHIP(m, hipMalloc(reinterpret_cast<void**>(&flags), sizeof(unsigned)));
    MHIP(m, hipMemsetAsync(flags, 0, sizeof(unsigned), m->stream));
    MHIP(m, launch_validate_entries(doc_ptr, word_idx, counts, ndocs, m->n, nnz, flags, m->stream));
    unsigned hf = 0;
    MHIP(m, hipMemcpyAsync(&hf, flags, sizeof(unsigned), hipMemcpyDeviceToHost, m->stream));
    MHIP(m, hipStreamSynchronize(m->stream));
    (void)hipFree(flags);
    if (hf) return mfail(m, NMFKL_E_INVAL, "invalid documents: word id out of range, ids not increasing, or count negative / not finite");
    std::vector<int32_t> lists[kFoldinVariants];
    int rc = group_docs(m, len, lists);
    if (rc) return rc;
    if ((size_t)ndocs > m->docs_cap) {
        if (m->docs) (void)hipFree(m->docs);
        m->docs = nullptr;
        MHIP(m, hipMalloc(reinterpret_cast<void**>(&m->docs), sizeof(int32_t) * ndocs));
        m->docs_cap = ndocs;
    }
    std::vector<int32_t> all;
    int off[kFoldinVariants], cnt[kFoldinVariants];
    for (int v = 0; v < kFoldinVariants; ++v) {
        off[v] = (int)all.size();
        cnt[v] = (int)lists[v].size();
        all.insert(all.end(), lists[v].begin(), lists[v].end());
    }
    MHIP(m, hipMemcpyAsync(m->docs, all.data(), sizeof(int32_t) * all.size(), hipMemcpyHostToDevice, m->stream));
    const FoldinArgs f = foldin_args(m, doc_ptr, word_idx, counts, F_out, passes_out, kl_out);
    rc = launch_grouped(m, f, m->docs, off, cnt, m->stream);
    if (rc) return rc;
    // the list buffer is reused by the next call: keep the host copy alive until it is read
    MHIP(m, hipStreamSynchronize(m->stream));
    return NMFKL_OK;
}

int nmfkl_model_get_stats(nmfkl_model* m, nmfkl_stats* out) {
    if (!m || !out) return mfail(m, NMFKL_E_INVAL, "null argument");
    unsigned long long c[6];
    MHIP(m, hipMemcpyAsync(c, m->stats, sizeof(c), hipMemcpyDeviceToHost, m->stream));
    MHIP(m, hipStreamSynchronize(m->stream));
    out->coords = (int64_t)c[0];
    out->evals = (int64_t)c[1];
    out->steps = (int64_t)c[2];
    out->halvings = (int64_t)c[3];
    out->rejects = (int64_t)c[4];
    out->tmax_hits = (int64_t)c[5];
    out->zeros_W = -1;   // a model holds no factors being fitted
    out->zeros_F = -1;
    return NMFKL_OK;
}

int nmfkl_model_destroy(nmfkl_model* m) {
    if (!m) return NMFKL_E_INVAL;
    if (m->stream) (void)hipStreamSynchronize(m->stream);
    auto f = [](void* p) { if (p) (void)hipFree(p); };
    f(m->sumW); f(m->rowsumW); f(m->perm); f(m->stats); f(m->docs);
    delete m;
    return NMFKL_OK;
}

// ---------------------------------------------------------------------------- server
int nmfkl_server_create(nmfkl_model* m, int64_t mem_budget_bytes, int32_t lanes, int32_t lane_docs,
                        int32_t max_queued, nmfkl_server** out) {
    if (!out) return sfail(nullptr, NMFKL_E_INVAL, "out is null");
    *out = nullptr;
    if (!m) return sfail(nullptr, NMFKL_E_INVAL, "null model");
    if (lanes < 1 || lanes > 64) return sfail(nullptr, NMFKL_E_INVAL, "lanes must be in [1, 64]");
    if (lane_docs < 1) return sfail(nullptr, NMFKL_E_INVAL, "lane_docs must be >= 1");
    if (max_queued < 0) return sfail(nullptr, NMFKL_E_INVAL, "max_queued must be >= 0");
    const int64_t bytes_per_word = (int64_t)(sizeof(int32_t) + sizeof(float));
    const int64_t max_doc_words = kFoldinCapacity[kFoldinVariants - 1];
    if (mem_budget_bytes < max_doc_words * bytes_per_word)
        return sfail(nullptr, NMFKL_E_INVAL, "memory budget below one largest document");
    nmfkl_server* s = new (std::nothrow) nmfkl_server();
    if (!s) return sfail(nullptr, NMFKL_E_NOMEM, "host allocation failed");
    s->model = m;
    s->budget_words = mem_budget_bytes / bytes_per_word;
    s->max_docs = lane_docs;
    s->max_queued = max_queued;
    s->lane_words = std::max<int64_t>(max_doc_words, s->budget_words / lanes);
    s->lanes.resize(lanes);
    const int r = m->r;
    for (auto& L : s->lanes) {
        auto fail_out = [&](hipError_t e) {
            sfail(nullptr, NMFKL_E_DEVICE, std::string("server lane: ") + hipGetErrorString(e));
            for (auto& K : s->lanes) release_lane(K);
            delete s;
            return NMFKL_E_DEVICE;
        };
        hipError_t e;
        if ((e = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking)) != hipSuccess) return fail_out(e);
        if ((e = hipEventCreateWithFlags(&L.done, hipEventDisableTiming)) != hipSuccess) return fail_out(e);
        const size_t nd = (size_t)lane_docs, nw = (size_t)s->lane_words;
        // outputs and completion words: host-coherent pinned memory that the kernels write
        const unsigned coh = hipHostMallocCoherent | hipHostMallocMapped;
        if ((e = hipMalloc(reinterpret_cast<void**>(&L.d_ptr), (nd + 1) * sizeof(int64_t))) != hipSuccess ||
            (e = hipMalloc(reinterpret_cast<void**>(&L.d_idx), nw * sizeof(int32_t))) != hipSuccess ||
            (e = hipMalloc(reinterpret_cast<void**>(&L.d_val), nw * sizeof(float))) != hipSuccess ||
            (e = hipMalloc(reinterpret_cast<void**>(&L.d_docs), nd * sizeof(int32_t))) != hipSuccess ||
            (e = hipHostMalloc(reinterpret_cast<void**>(&L.h_ptr), (nd + 1) * sizeof(int64_t), hipHostMallocDefault)) != hipSuccess ||
            (e = hipHostMalloc(reinterpret_cast<void**>(&L.h_idx), nw * sizeof(int32_t), hipHostMallocDefault)) != hipSuccess ||
            (e = hipHostMalloc(reinterpret_cast<void**>(&L.h_val), nw * sizeof(float), hipHostMallocDefault)) != hipSuccess ||
            (e = hipHostMalloc(reinterpret_cast<void**>(&L.h_docs), nd * sizeof(int32_t), hipHostMallocDefault)) != hipSuccess ||
            (e = hipHostMalloc(reinterpret_cast<void**>(&L.h_F), nd * r * sizeof(float), coh)) != hipSuccess ||
            (e = hipHostMalloc(reinterpret_cast<void**>(&L.h_passes), nd * sizeof(int32_t), coh)) != hipSuccess ||
            (e = hipHostMalloc(reinterpret_cast<void**>(&L.h_kl), nd * sizeof(double), coh)) != hipSuccess ||
            (e = hipHostMalloc(reinterpret_cast<void**>(&L.h_flag), nd * sizeof(unsigned), coh)) != hipSuccess)
            return fail_out(e);
        std::memset(L.h_flag, 0, nd * sizeof(unsigned));
        if ((e = hipHostGetDevicePointer(reinterpret_cast<void**>(&L.k_F), L.h_F, 0)) != hipSuccess ||
            (e = hipHostGetDevicePointer(reinterpret_cast<void**>(&L.k_passes), L.h_passes, 0)) != hipSuccess ||
            (e = hipHostGetDevicePointer(reinterpret_cast<void**>(&L.k_kl), L.h_kl, 0)) != hipSuccess ||
            (e = hipHostGetDevicePointer(reinterpret_cast<void**>(&L.k_flag), L.h_flag, 0)) != hipSuccess)
            return fail_out(e);
    }
    *out = s;
    return NMFKL_OK;
}

int nmfkl_server_submit(nmfkl_server* s, uint64_t req_id, int32_t L, const int32_t* word_idx, const float* counts,
                        double timeout_s) {
    if (!s) return sfail(nullptr, NMFKL_E_INVAL, "null server");
    if (L < 0 || (L > 0 && (!word_idx || !counts))) return sfail(s, NMFKL_E_INVAL, "bad document");
    if (!(timeout_s == timeout_s)) return sfail(s, NMFKL_E_INVAL, "timeout is NaN");
    if (variant_of_length(L) < 0) return sfail(s, NMFKL_E_UNSUPPORTED, "document too long for fold-in");
    const int32_t n = s->model->n;
    for (int32_t l = 0; l < L; ++l) {
        if (word_idx[l] < 0 || word_idx[l] >= n || (l > 0 && word_idx[l] <= word_idx[l - 1]))
            return sfail(s, NMFKL_E_INVAL, "word ids must be in range and strictly increasing");
        if (!(counts[l] >= 0.0f) || !std::isfinite(counts[l]))
            return sfail(s, NMFKL_E_INVAL, "counts must be finite and >= 0");
    }
    if (s->max_queued > 0 && (int64_t)s->pending.size() >= s->max_queued)
        return sfail(s, NMFKL_E_BUSY, "every waiting slot is taken");
    if (s->words_in_flight + L > s->budget_words) return sfail(s, NMFKL_E_NOMEM, "memory budget exhausted");
    nmfkl_server::Req q;
    q.id = req_id;
    q.L = L;
    q.t_submit = now_seconds();
    q.expires = timeout_s > 0.0 ? q.t_submit + timeout_s : 0.0;
    q.idx.assign(word_idx, word_idx + L);
    q.val.assign(counts, counts + L);
    if (q.expires > 0.0) ++s->timed_pending;
    s->pending.push_back(std::move(q));
    s->words_in_flight += L;
    return NMFKL_OK;
}

int nmfkl_server_cancel(nmfkl_server* s, uint64_t req_id) {
    if (!s) return sfail(nullptr, NMFKL_E_INVAL, "null server");
    for (auto it = s->pending.begin(); it != s->pending.end(); ++it) {
        if (it->id != req_id) continue;
        nmfkl_server::Req q = std::move(*it);
        s->pending.erase(it);
        finish_unlaunched(s, std::move(q), NMFKL_RESULT_CANCELLED, now_seconds());
        return NMFKL_OK;
    }
    return sfail(s, NMFKL_E_INVAL, "no waiting document has this id (launched, finished or unknown)");
}

int nmfkl_server_poll(nmfkl_server* s, int32_t max_results, nmfkl_result* out, float* f_out, int32_t* n_out) {
    if (!s || !n_out || (max_results > 0 && (!out || !f_out))) return sfail(s, NMFKL_E_INVAL, "null argument");
    int rc = collect(s);
    if (rc) return rc;
    expire_pending(s);
    rc = dispatch(s);
    if (rc) return rc;
    const int r = s->model->r;
    int k = 0;
    while (k < max_results && !s->done.empty()) {
        const auto& d = s->done.front();
        out[k].req_id = d.id;
        out[k].passes = d.passes;
        out[k].status = d.status;
        out[k].kl = d.kl;
        out[k].t_submit = d.t_submit;
        out[k].t_done = d.t_done;
        std::memcpy(f_out + (size_t)k * r, d.f.data(), (size_t)r * sizeof(float));
        s->done.pop_front();
        ++k;
    }
    *n_out = k;
    return NMFKL_OK;
}

int nmfkl_server_pending(nmfkl_server* s, int64_t* queued, int64_t* in_flight_words) {
    if (!s) return sfail(nullptr, NMFKL_E_INVAL, "null server");
    int64_t busy = 0;
    for (auto& L : s->lanes) busy += L.busy ? (int64_t)(L.reqs.size() - L.nreturned) : 0;
    if (queued) *queued = (int64_t)s->pending.size() + busy + (int64_t)s->done.size();
    if (in_flight_words) *in_flight_words = s->words_in_flight;
    return NMFKL_OK;
}

int nmfkl_server_now(double* t_out) {
    if (!t_out) return NMFKL_E_INVAL;
    *t_out = now_seconds();
    return NMFKL_OK;
}

const char* nmfkl_server_last_error(const nmfkl_server* s) { return s ? s->err.c_str() : g_model_error.c_str(); }

int nmfkl_server_destroy(nmfkl_server* s) {
    if (!s) return NMFKL_E_INVAL;
    for (auto& L : s->lanes) {
        if (L.stream) (void)hipStreamSynchronize(L.stream);
        release_lane(L);
    }
    delete s;
    return NMFKL_OK;
}

}  // extern "C"

// ------------------------------------------------------- fold-in without allocation
// nmfkl_foldin_noalloc: the scratch of nmfkl_foldin (validation flags and the documents
// grouped by kernel variant) lives in one file-scope device array instead of hipMalloc'd
// buffers, and the document pointers are checked and grouped on the device, so the call
// allocates nothing on the device or the host heap.  Each device holds its own copy of the
// array; the host takes its address once per device with hipGetSymbolAddress and passes
// that address to the kernels (the array's name is not a device address in host code).
namespace {

constexpr int kNoAllocMaxDocs = 16384;
constexpr int kNoAllocDocsOffset = 256;   // bytes: the header, then the grouped document list
constexpr size_t kNoAllocBytes = kNoAllocDocsOffset + sizeof(int32_t) * (size_t)kNoAllocMaxDocs;
constexpr int kMaxDevices = 64;

// Flag bits of the header beyond the shared validation bits.
constexpr unsigned kTooLong = 1u << 8;      // a document above the largest fold-in variant
constexpr unsigned kTooManyWords = 1u << 9; // more than 2^31 - 1 words
constexpr unsigned kNullWords = 1u << 10;   // words present but a null index or count array

struct NoAllocHeader {
    unsigned flags;                  // validation bits (kBad*, kTooLong, ...)
    int32_t count[kFoldinVariants];  // documents per variant
    int64_t nnz;                     // doc_ptr[ndocs] (valid when kBadPtr is clear)
};
static_assert(sizeof(NoAllocHeader) <= kNoAllocDocsOffset, "header must fit before the list");

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_scratch_mutex;
unsigned char* g_scratch_addr[kMaxDevices] = {};

// The device address of `scratch` on device dev (current), looked up once per device.
hipError_t scratch_address(int dev, unsigned char** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_scratch_addr[dev];
    return hipSuccess;
}

__device__ __forceinline__ int foldin_variant(int64_t L) {
    for (int v = 0; v < kFoldinVariants; ++v)
        if (L <= kFoldinCapacity[v]) return v;
    return -1;
}

// One block: checks the document pointers (doc_ptr[0] = 0, monotone, lengths within the
// largest variant, total below 2^31), counts the documents per variant and writes their
// indices grouped by variant, in document order inside each group, after the header.  Every
// header field is written here, so nothing in the scratch needs clearing first.
constexpr int kGroupThreads = 1024;
__global__ void __launch_bounds__(kGroupThreads)
k_group_docs_noalloc(const int64_t* __restrict__ ptr, int ndocs, const int32_t* idx, const float* val,
                     unsigned char* base) {
    __shared__ unsigned s_flags;
    __shared__ int s_count[kFoldinVariants];
    __shared__ int s_wave[kGroupThreads / 64][kFoldinVariants];
    __shared__ int s_run[kFoldinVariants];
    NoAllocHeader* hdr = reinterpret_cast<NoAllocHeader*>(base);
    int32_t* list = reinterpret_cast<int32_t*>(base + kNoAllocDocsOffset);
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    if (tid == 0) s_flags = 0u;
    if (tid < kFoldinVariants) { s_count[tid] = 0; s_run[tid] = 0; }
    __syncthreads();
    unsigned bad = 0u;
    int cnt[kFoldinVariants] = {0, 0, 0, 0, 0};
    for (int d = tid; d < ndocs; d += kGroupThreads) {
        const int64_t p0 = ptr[d], p1 = ptr[d + 1];
        if (d == 0 && p0 != 0) bad |= kBadPtr;
        if (p1 < p0) { bad |= kBadPtr; continue; }
        const int v = foldin_variant(p1 - p0);
        if (v < 0) bad |= kTooLong;
        else cnt[v] += 1;
    }
    if (bad) atomicOr(&s_flags, bad);
#pragma unroll
    for (int v = 0; v < kFoldinVariants; ++v)
        if (cnt[v]) atomicAdd(&s_count[v], cnt[v]);
    __syncthreads();
    int off[kFoldinVariants];
    int acc = 0;
#pragma unroll
    for (int v = 0; v < kFoldinVariants; ++v) { off[v] = acc; acc += s_count[v]; }
    // stable grouping, one chunk of kGroupThreads documents at a time
    for (int c0 = 0; c0 < ndocs; c0 += kGroupThreads) {
        const int d = c0 + tid;
        int v = -1;
        if (d < ndocs) {
            const int64_t p0 = ptr[d], p1 = ptr[d + 1];
            if (p1 >= p0) v = foldin_variant(p1 - p0);
        }
        int before[kFoldinVariants];
#pragma unroll
        for (int k = 0; k < kFoldinVariants; ++k) {
            const unsigned long long mask = __ballot(v == k);
            before[k] = __popcll(mask & ((1ull << lane) - 1ull));
            if (lane == 0) s_wave[wave][k] = __popcll(mask);
        }
        __syncthreads();
        if (v >= 0) {
            int pos = off[v] + s_run[v] + before[v];
            for (int q = 0; q < wave; ++q) pos += s_wave[q][v];
            list[pos] = d;
        }
        __syncthreads();
        if (tid < kFoldinVariants) {
            int t = 0;
            for (int q = 0; q < kGroupThreads / 64; ++q) t += s_wave[q][tid];
            s_run[tid] += t;
        }
        __syncthreads();
    }
    if (tid == 0) {
        unsigned f = s_flags;
        int64_t nnz = 0;
        if (!(f & kBadPtr)) {
            nnz = ndocs > 0 ? ptr[ndocs] : 0;
            if (nnz > (int64_t)INT32_MAX) f |= kTooManyWords;
            if (nnz > 0 && (!idx || !val)) f |= kNullWords;
        }
        hdr->flags = f;
        for (int v = 0; v < kFoldinVariants; ++v) hdr->count[v] = s_count[v];
        hdr->nnz = nnz;
    }
}

// Word ids in [0, n) and strictly increasing per document, counts finite and >= 0: block b
// checks documents b, b + gridDim.x, ...  Runs only over pointers the grouping accepted.
__global__ void __launch_bounds__(256)
k_validate_docs_noalloc(const int64_t* __restrict__ ptr, const int32_t* __restrict__ idx,
                        const float* __restrict__ val, int ndocs, int n, unsigned char* base) {
    NoAllocHeader* hdr = reinterpret_cast<NoAllocHeader*>(base);
    if (hdr->flags & (kBadPtr | kTooManyWords | kNullWords)) return;
    unsigned bad = 0u;
    for (int d = blockIdx.x; d < ndocs; d += gridDim.x) {
        const int64_t p0 = ptr[d], p1 = ptr[d + 1];
        for (int64_t q = p0 + threadIdx.x; q < p1; q += blockDim.x) {
            const int32_t i = idx[q];
            if (i < 0 || i >= n) bad |= kBadIndex;
            if (q > p0 && idx[q - 1] >= i) bad |= kBadOrder;
            const float v = val[q];
            if (!(v >= 0.0f) || !isfinite(v)) bad |= kBadValue;
        }
    }
    if (bad) atomicOr(&hdr->flags, bad);
}

}  // namespace

extern "C" int nmfkl_foldin_noalloc(nmfkl_model* m, int32_t ndocs, const int64_t* doc_ptr, const int32_t* word_idx,
                                    const float* counts, float* F_out, int32_t* passes_out, double* kl_out) {
    if (!m) return mfail(nullptr, NMFKL_E_INVAL, "null model");
    if (ndocs < 0) return mfail(m, NMFKL_E_INVAL, "ndocs must be >= 0");
    if (ndocs > kNoAllocMaxDocs)
        return mfail(m, NMFKL_E_UNSUPPORTED, "nmfkl_foldin_noalloc takes at most 16384 documents per call");
    if (ndocs == 0) return NMFKL_OK;
    if (!doc_ptr || !F_out || !passes_out || !kl_out) return mfail(m, NMFKL_E_INVAL, "null pointer");
    int dev = -1;
    MHIP(m, hipGetDevice(&dev));
    if (m->stream) {
        int sdev = -1;
        MHIP(m, hipStreamGetDevice(m->stream, &sdev));
        if (sdev != dev) return mfail(m, NMFKL_E_INVAL, "the model's stream belongs to another device than the current one");
    }
    if (dev < 0 || dev >= kMaxDevices) return mfail(m, NMFKL_E_UNSUPPORTED, "device ordinal beyond 63");
    unsigned char* base = nullptr;
    MHIP(m, scratch_address(dev, &base));
    hipLaunchKernelGGL(k_group_docs_noalloc, dim3(1), dim3(kGroupThreads), 0, m->stream, doc_ptr, ndocs, word_idx,
                       counts, base);
    MHIP(m, hipGetLastError());
    const int vblocks = std::min(ndocs, 2048);
    hipLaunchKernelGGL(k_validate_docs_noalloc, dim3(vblocks), dim3(256), 0, m->stream, doc_ptr, word_idx, counts,
                       ndocs, m->n, base);
    MHIP(m, hipGetLastError());
    NoAllocHeader hdr;
    MHIP(m, hipMemcpyAsync(&hdr, base, sizeof(hdr), hipMemcpyDeviceToHost, m->stream));
    MHIP(m, hipStreamSynchronize(m->stream));
    if (hdr.flags & kBadPtr) return mfail(m, NMFKL_E_INVAL, "doc_ptr[0] must be 0 and doc_ptr monotone");
    if (hdr.flags & kNullWords) return mfail(m, NMFKL_E_INVAL, "null word/count pointer");
    if (hdr.flags & kTooManyWords) return mfail(m, NMFKL_E_UNSUPPORTED, "more than 2^31-1 words in one call");
    if (hdr.flags & kTooLong)
        return mfail(m, NMFKL_E_UNSUPPORTED, "a document has more distinct words than fold-in supports (5120)");
    if (hdr.flags)
        return mfail(m, NMFKL_E_INVAL, "invalid documents: word id out of range, ids not increasing, or count negative / not finite");
    int off[kFoldinVariants], cnt[kFoldinVariants], pos = 0;
    for (int v = 0; v < kFoldinVariants; ++v) {
        off[v] = pos;
        cnt[v] = hdr.count[v];
        pos += cnt[v];
    }
    const int32_t* list = reinterpret_cast<const int32_t*>(base + kNoAllocDocsOffset);
    const FoldinArgs f = foldin_args(m, doc_ptr, word_idx, counts, F_out, passes_out, kl_out);
    const int rc = launch_grouped(m, f, list, off, cnt, m->stream);
    if (rc) return rc;
    // the grouped list is read by the kernels: the next call may rewrite it only after they end
    MHIP(m, hipStreamSynchronize(m->stream));
    return NMFKL_OK;
}
