// Device kernels of the NMF-KL randomized coordinate-descent sweep for gfx950 (wave64).
//
// Half-sweep (Alg. 1's F-half or W-half): every segment (a column of V for the F-half, a row
// for the W-half) runs Alg. 2 on its own r-vector x.  The fixed factor A has been copied with
// its columns permuted into this outer iteration's coordinate order (so coordinate step s
// always reads permuted column s) and padded to a row stride Sp that is a multiple of the
// chunk width.  A segment is handled by G lanes; lane g holds the nonzeros l = g + G*e,
// e < E, in registers: the count v_l, the model Ax_l (float64), w_l = v_l/(Ax_l+eps) and
// u_l = w_l/(Ax_l+eps) (float32), so that eq. 6's sums are
//     S1 = sum_l v_l A_lk/(Ax_l+eps) = sum_l A_lk w_l,   S2 = sum_l A_lk^2 u_l,
// and streams the fixed-factor values of its nonzeros through registers one chunk of CW
// coordinates at a time (8 in the binned register variants, 4 in the LDS-form variants and
// the long-segment kernels; the kernels are latency-bound at their occupancy, where a
// prefetched second chunk would spill).  S1 and S2 are all-reduced over the G lanes with DPP
// row operations (and LDS, or a cross-block exchange, for multi-wave segments), so every lane
// of a segment takes the same Newton decisions.
//
// Precision: the derivative sums are float32 (all terms are positive).  The model values
// are float64 because a coordinate step can remove most of a nonzero's model value (for
// example when the other coordinates of a one-nonzero column drop to zero): in float32 the
// rounding error of the starting value would then become a large relative error of the
// small remainder, and with it of the derivatives.
#include <algorithm>

#include "nmfkl_internal.hpp"

namespace nmfkl {

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ float dpp_quad_xor1(float v) {
    return __builtin_amdgcn_update_dpp(0.0f, v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
}
__device__ __forceinline__ float dpp_quad_xor2(float v) {
    return __builtin_amdgcn_update_dpp(0.0f, v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
}
__device__ __forceinline__ float dpp_half_mirror(float v) {
    return __builtin_amdgcn_update_dpp(0.0f, v, 0x141, 0xF, 0xF, false);  // row_half_mirror
}
__device__ __forceinline__ float dpp_mirror(float v) {
    return __builtin_amdgcn_update_dpp(0.0f, v, 0x140, 0xF, 0xF, false);  // row_mirror
}

// Sum of the lane's value and that of lane ^ 16 (ROWS = 16) or lane ^ 32 (ROWS = 32): the
// gfx950 row-swap permutes exchange whole 16-lane rows (odd rows of the first operand with
// even rows of the second; the upper half of the first with the lower half of the second),
// so adding the two results gives both partners the same sum, in registers only.
template <int ROWS>
__device__ __forceinline__ float row_swap_sum(float v) {
    const unsigned u = __float_as_uint(v);
    if constexpr (ROWS == 16) {
        const auto p = __builtin_amdgcn_permlane16_swap(u, u, false, false);
        return __uint_as_float(p[0]) + __uint_as_float(p[1]);
    } else {
        const auto p = __builtin_amdgcn_permlane32_swap(u, u, false, false);
        return __uint_as_float(p[0]) + __uint_as_float(p[1]);
    }
}

// All-reduce over aligned groups of G lanes (G a power of two, G <= 64).  After the two quad
// steps every lane holds its quad's sum; the half-row mirror pairs quad q with the other quad
// of its 8-lane half, the row mirror pairs the two halves of a 16-lane row, and the row swaps
// pair rows.  Each step adds the same two partial sums on both partners, so all lanes of a
// group end bit-identical.
template <int G>
__device__ __forceinline__ float group_sum(float v) {
    if constexpr (G >= 2) v += dpp_quad_xor1(v);
    if constexpr (G >= 4) v += dpp_quad_xor2(v);
    if constexpr (G >= 8) v += dpp_half_mirror(v);
    if constexpr (G >= 16) v += dpp_mirror(v);
    if constexpr (G >= 32) v = row_swap_sum<16>(v);
    if constexpr (G >= 64) v = row_swap_sum<32>(v);
    return v;
}

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// ------------------------------------------------- permuted copy + float64 column sums
// bfloat16 of a finite float: round to nearest, ties to even (the upper 16 bits after adding
// 0x7FFF plus the lowest kept bit).
__device__ __forceinline__ uint16_t bf16_rne(float x) {
    const unsigned u = __float_as_uint(x);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_float(uint16_t q) { return __uint_as_float((unsigned)q << 16); }

// Job of a block: the last job whose first index is <= b (jobs in increasing order).
template <class Key>
__device__ __forceinline__ int find_job(const PermJob* jobs, int njobs, int b, Key key) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (key(jobs[mid]) <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The job's coordinate order into sid[0..NMFKL_R_MAX) (-1 beyond r): the Fisher-Yates
// shuffle of coordinate_order, with its Philox blocks computed by parallel threads (block q
// gives words 4q..4q+3; step i = r-1, ..., 1 uses word r-1-i) and the swaps by thread 0.
__device__ void job_order(const PermJob& jb, int64_t t, int32_t* sid, uint64_t* words) {
    const int r = jb.r;
    if (jb.identity) {
        for (int s = threadIdx.x; s < NMFKL_R_MAX; s += blockDim.x) sid[s] = s < r ? s : -1;
        __syncthreads();
        return;
    }
    const int nblk = (r - 1 + 3) / 4;
    for (int q = threadIdx.x; q < nblk; q += blockDim.x) {
        const uint64_t ctr[4] = {(uint64_t)q, (uint64_t)t, jb.stream, 0};
        const uint64_t key[2] = {jb.seed, 0};
        uint64_t out[4];
        philox4x64_10(ctr, key, out);
        for (int k = 0; k < 4; ++k) words[4 * q + k] = out[k];
    }
    for (int s = threadIdx.x; s < NMFKL_R_MAX; s += blockDim.x) sid[s] = s < r ? s : -1;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = r - 1; i >= 1; --i) {
            const int j = (int)__umul64hi(words[r - 1 - i], (uint64_t)(i + 1));
            const int32_t tmp = sid[i];
            sid[i] = sid[j];
            sid[j] = tmp;
        }
    }
    __syncthreads();
}

// Block b of job j covers rows [lb*rpb, (lb+1)*rpb), lb = b - first_block.  Thread (ry, cx)
// walks rows ry, ry+4, ... for permuted column s = s0 + cx, reading A[p][ids[s]] and
// writing Ap[p][s] (zero in the padding), and the chunk-major copy when the job has one.  Per-block float64 partial sums go to
// partials[lb*r + s]; k_finalize_jobs adds them in a fixed order, so the result is
// deterministic.  The job's first block also stores the order for the sweep kernels.
__global__ void __launch_bounds__(256) k_permute_jobs(const PermJob* __restrict__ jobs, int njobs,
                                                      int64_t t_arg, const int64_t* __restrict__ t_dev) {
    __shared__ int32_t sid[NMFKL_R_MAX];
    __shared__ uint64_t words[NMFKL_R_MAX];
    __shared__ double red[4][64];
    const int jj = find_job(jobs, njobs, (int)blockIdx.x, [](const PermJob& q) { return q.first_block; });
    const PermJob jb = jobs[jj];
    const int64_t lb = (int64_t)blockIdx.x - jb.first_block;
    const int64_t t = t_arg + (t_dev ? *t_dev : 0);
    job_order(jb, t, sid, words);
    const int r = jb.r, Sp = jb.Sp, Sc = (r + 3) & ~3;
    if (jb.ids && lb == 0)
        for (int s = threadIdx.x; s < r; s += 256) jb.ids[s] = sid[s];
    const int cx = threadIdx.x & 63, ry = threadIdx.x >> 6;
    const int64_t p0 = lb * jb.rpb;
    const int64_t p1 = p0 + jb.rpb < jb.P ? p0 + jb.rpb : jb.P;
    for (int s0 = 0; s0 < Sp; s0 += 64) {
        const int s = s0 + cx;
        const int k = s < Sp ? sid[s] : -1;
        double acc = 0.0;
        if (s < Sp) {
            // rows ry, ry + 4, ...: U loads issued before their stores (the copy may not alias
            // the factor), then added in row order
            constexpr int U = 4;
            const float* __restrict__ A = jb.A;
            for (int64_t pb = p0 + ry; pb < p1; pb += 4 * U) {
                float a[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t p = pb + 4 * u;
                    a[u] = (k >= 0 && p < p1) ? A[p * r + k] : 0.0f;
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t p = pb + 4 * u;
                    if (p >= p1) break;
                    if (jb.bf16) {
                        const uint16_t q = bf16_rne(a[u]);
                        a[u] = bf16_to_float(q);
                        if (jb.Ap) reinterpret_cast<uint16_t*>(jb.Ap)[p * Sp + s] = q;
                    } else if (jb.Ap) {
                        jb.Ap[p * Sp + s] = a[u];
                    }
                    acc += (double)a[u];
                }
            }
        }
        red[ry][cx] = acc;
        __syncthreads();
        if (ry == 0 && s < r)
            jb.partials[lb * r + s] = ((red[0][cx] + red[1][cx]) + red[2][cx]) + red[3][cx];
        __syncthreads();
    }
    if (jb.Apc) {
        // the chunk-major copy: thread (row group, component q) writes 256 / kChunkMajorW
        // consecutive rows' chunk entries per block pass, so the stores are contiguous
        constexpr int W = kChunkMajorW;
        const int q = threadIdx.x % W;
        const float* __restrict__ A = jb.A;
        for (int c = 0; c < Sc / W; ++c) {
            const int k = sid[W * c + q];
            for (int64_t p = p0 + (threadIdx.x / W); p < p1; p += 256 / W) {
                const float a = k >= 0 ? A[p * r + k] : 0.0f;
                const int64_t pc = ((int64_t)c * jb.P + p) * W + q;
                if (jb.bf16) reinterpret_cast<uint16_t*>(jb.Apc)[pc] = bf16_rne(a);
                else jb.Apc[pc] = a;
            }
        }
    }
}

hipError_t launch_permute_jobs(const PermJob* jobs, int njobs, int nblocks, int64_t t_arg,
                               const int64_t* t_dev, hipStream_t stream) {
    if (njobs <= 0 || nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_permute_jobs, dim3(nblocks), dim3(256), 0, stream, jobs, njobs, t_arg, t_dev);
    return hipGetLastError();
}

// Block b = (job j, column s = b - first_sum): the block's threads add the job's per-block
// partials q = t, t+256, ... and a fixed tree combines them.
__global__ void __launch_bounds__(256) k_finalize_jobs(const PermJob* __restrict__ jobs, int njobs) {
    __shared__ double red[256];
    const int jj = find_job(jobs, njobs, (int)blockIdx.x, [](const PermJob& q) { return q.first_sum; });
    const PermJob& jb = jobs[jj];
    const int s = (int)blockIdx.x - jb.first_sum;
    double acc = 0.0;
    for (int b = threadIdx.x; b < jb.nblocks; b += 256) acc += jb.partials[(int64_t)b * jb.r + s];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) jb.sums[s] = red[0];
}

hipError_t launch_finalize_jobs(const PermJob* jobs, int njobs, int nsum, hipStream_t stream) {
    if (njobs <= 0 || nsum <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize_jobs, dim3(nsum), dim3(256), 0, stream, jobs, njobs);
    return hipGetLastError();
}

// --------------------------------------------------------------- the sweep
// Per-nonzero state of a lane's E nonzeros: the model ax (float64, registers) and the
// count v, w = v/(ax+eps), u = w/(ax+eps) and the point id, either in registers
// (RegElems) or in LDS slots e*STRIDE + lane of the block (LdsElems: the fold-in's block
// kernel; LdsElemsNoWU, below, without w and u: the LDS-form binned variants and the
// long-segment kernels, whose register budget holds the tile and the model of more
// nonzeros that way).
template <int E>
struct RegElems {
    static constexpr int kE = E;
    static constexpr bool kStoresWU = true;
    double ax[E];
    int32_t id_[E];
    float v_[E], w_[E], u_[E];
    __device__ __forceinline__ int32_t& id(int e) { return id_[e]; }
    __device__ __forceinline__ float& v(int e) { return v_[e]; }
    __device__ __forceinline__ void wu(int e, float eps, float& w, float& u) { w = w_[e]; u = u_[e]; }
    __device__ __forceinline__ void set_wu(int e, float w, float u) { w_[e] = w; u_[e] = u; }
};

template <int E, int STRIDE>
struct LdsElems {
    static constexpr int kE = E;
    static constexpr bool kStoresWU = true;
    double ax[E];
    int32_t* idp;
    float *vp, *wp, *up;
    __device__ __forceinline__ int32_t& id(int e) { return idp[e * STRIDE]; }
    __device__ __forceinline__ float& v(int e) { return vp[e * STRIDE]; }
    __device__ __forceinline__ void wu(int e, float eps, float& w, float& u) { w = wp[e * STRIDE]; u = up[e * STRIDE]; }
    __device__ __forceinline__ void set_wu(int e, float w, float u) { wp[e * STRIDE] = w; up[e * STRIDE] = u; }
};

// Counts and ids in LDS, the model in registers; w and u are recomputed from the model when
// needed (by the same formula that produces them on the other paths, so the values agree).
template <int E, int STRIDE>
struct LdsElemsNoWU {
    static constexpr int kE = E;
    static constexpr bool kStoresWU = false;
    double ax[E];
    int32_t* idp;
    float* vp;
    __device__ __forceinline__ int32_t& id(int e) { return idp[e * STRIDE]; }
    __device__ __forceinline__ float& v(int e) { return vp[e * STRIDE]; }
    __device__ __forceinline__ void wu(int e, float eps, float& w, float& u) {
        const float ri = __builtin_amdgcn_rcpf((float)ax[e] + eps);
        w = vp[e * STRIDE] * ri;
        u = w * ri;
    }
    __device__ __forceinline__ void set_wu(int, float, float) {}
};

// ---- segment-wide all-reduce of NV partial sums ----------------------------------------
// sum(v, lo) all-reduces v[lo..NV) over the lanes of a segment.  Every lane of a segment
// receives bit-identical sums, so every lane takes the same Newton decisions.  lo is a
// compile-time constant after unrolling at every call site.

// Segments of G <= 64 lanes inside one wave: DPP / lane shuffles only.
__device__ __forceinline__ double shfl_xor_f64(double v, int m) {
    int2 p = *reinterpret_cast<int2*>(&v);
    p.x = __shfl_xor(p.x, m);
    p.y = __shfl_xor(p.y, m);
    return *reinterpret_cast<double*>(&p);
}

// Values that every lane of a segment holds bit for bit (the reduced sums, x_k, the column
// sum) are wave-uniform when a wave holds lanes of one segment only (G >= 64): moved into
// scalar registers with readfirstlane, the Newton logic's branches on them are uniform
// branches instead of exec-mask sequences.
template <bool UNI>
__device__ __forceinline__ float seg_uniform(float v) {
    if constexpr (UNI) return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
    else return v;
}
template <bool UNI>
__device__ __forceinline__ double seg_uniform(double v) {
    if constexpr (UNI) {
        const long long b = __double_as_longlong(v);
        const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xFFFFFFFFll));
        const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
        return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
    } else {
        return v;
    }
}

template <int G>
struct WaveReducer {
    static constexpr bool kUniform = G == 64;
    // float64 all-reduce over the segment's lanes (butterfly: identical on every lane)
    __device__ __forceinline__ double sum_f64(double v) {
#pragma unroll
        for (int m = 1; m < G; m <<= 1) v += shfl_xor_f64(v, m);
        return v;
    }
    template <int NV>
    __device__ __forceinline__ void sum(float (&v)[NV], int lo) {
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (i >= lo) v[i] = group_sum<G>(v[i]);
    }
};

// One segment per block of NT threads: wave sums, then the NT/64 wave sums through LDS in
// wave order (double-buffered by parity: one barrier per reduction).  red holds
// 2 * (NT/64) * kMaxRed floats.
constexpr int kMaxRed = kCoopValues;

template <int NT>
struct BlockReducer {
    static constexpr bool kUniform = true;
    float* red;
    int parity;
    double* red64;  // LDS, 2 * NT/64 doubles (float64 sums; optional)
    __device__ __forceinline__ double sum_f64(double v) {
        constexpr int W = NT / 64;
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) v += shfl_xor_f64(v, m);
        const int wv = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) red64[parity * W + wv] = v;
        __syncthreads();
        double t = red64[parity * W];
#pragma unroll
        for (int q = 1; q < W; ++q) t += red64[parity * W + q];
        parity ^= 1;
        return t;
    }
    template <int NV>
    __device__ __forceinline__ void sum(float (&v)[NV], int lo) {
        constexpr int W = NT / 64;
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (i >= lo) v[i] = group_sum<64>(v[i]);
        const int wv = threadIdx.x >> 6;
        float* mine = red + (parity * W + wv) * kMaxRed;
        if ((threadIdx.x & 63) == 0) {
#pragma unroll
            for (int i = 0; i < NV; ++i)
                if (i >= lo) mine[i] = v[i];
        }
        __syncthreads();
        const float* base = red + parity * W * kMaxRed;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            if (i >= lo) {
                float t = base[i];
#pragma unroll
                for (int q = 1; q < W; ++q) t += base[q * kMaxRed + i];
                v[i] = t;
            }
        }
        parity ^= 1;
    }
};

// A long segment split over B co-resident blocks (cooperative launch).  Each reduction:
// block sum (float32, exactly representable in float64); lanes i < NV publish partial i as
// one 64-bit word (round tag << 32 | float bits) into slot `round & 1` of the group's
// partials with a coherent atomic store.  Readers poll the data words themselves: thread
// (i, j) loads word i of blocks j, j+16, ... (up to kInFlight loads in flight) until every
// tag equals this round's, adding the values in float64 in block order; thread i < NV then
// adds the 16 results in order, so every block obtains the same totals.  One round trip per
// exchange: no separate arrival flag and no wait for the stores to be performed.  The
// slot of round k is rewritten at round k + 2 only after every block has published round
// k + 1, which each does after reading round k.  Every shared access is an atomic performed
// at the device coherence point.  The waits are bounded: after kSpinLimit polls, or once any
// block has recorded an error, the block records an error and continues (the host reports it
// at the next synchronising call).  The words are zeroed before each launch.
constexpr unsigned kSpinLimit = 1u << 20;

template <int NT>
struct CoopReducer {
    static constexpr bool kUniform = true;
    static constexpr int J = NT / kMaxRed;   // block groups per value
    static constexpr int kInFlight = 4;
    BlockReducer<NT> blk;
    double* tmp;                 // LDS, J * kMaxRed doubles
    double* bcast;               // LDS, kMaxRed doubles
    unsigned long long* words;   // global: [2][B][kMaxRed] tagged partials of this group
    unsigned* err;               // global error flags
    int B, part;
    unsigned round;
    template <int NV>
    __device__ __forceinline__ void sum(float (&v)[NV], int lo) {
        static_assert(NV <= kMaxRed, "at most kMaxRed values per exchange");
        blk.sum(v, lo);
        if (B == 1) return;
        const unsigned tag = round + 1u;
        unsigned long long* slot = words + (size_t)(round & 1u) * B * kMaxRed;
        const int tid = threadIdx.x;
        if (tid >= lo && tid < NV) {
            float mine = 0.0f;
#pragma unroll
            for (int i = 0; i < NV; ++i)
                if (i == tid) mine = v[i];
            __hip_atomic_store(slot + (size_t)part * kMaxRed + tid,
                               ((unsigned long long)tag << 32) | __float_as_uint(mine), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        const int i = tid % kMaxRed, j = tid / kMaxRed;
        double acc = 0.0;
        if (i >= lo && i < NV) {
            for (int b0 = j; b0 < B; b0 += J * kInFlight) {
                unsigned long long w[kInFlight];
                unsigned spins = 0;
                for (;;) {
                    bool ok = true;
#pragma unroll
                    for (int q = 0; q < kInFlight; ++q) {
                        const int b = b0 + q * J;
                        w[q] = b < B ? __hip_atomic_load(slot + (size_t)b * kMaxRed + i, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT)
                                     : ((unsigned long long)tag << 32);
                        ok &= (unsigned)(w[q] >> 32) == tag;
                    }
                    if (ok) break;
                    __builtin_amdgcn_s_sleep(1);
                    if (++spins > kSpinLimit ||
                        __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                        atomicOr(err, 1u);
                        break;
                    }
                }
#pragma unroll
                for (int q = 0; q < kInFlight; ++q)
                    acc += (double)__uint_as_float((unsigned)(w[q] & 0xFFFFFFFFull));
            }
        }
        tmp[j * kMaxRed + i] = acc;
        __syncthreads();
        if (tid >= lo && tid < NV) {
            double t = 0.0;
            for (int q = 0; q < J; ++q) t += tmp[q * kMaxRed + tid];
            bcast[tid] = t;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NV; ++q)
            if (q >= lo) v[q] = (float)bcast[q];
        ++round;
    }
};

// Elements handled by this lane: l = lo + lane + STRIDE * e, e < E, restricted to l < L.
// A tile chunk holds CW consecutive permuted coordinates (CW = 2: the first two components
// of one float4 per nonzero; CW a multiple of 4: CW / 4 float4 per nonzero).  Chunks of 4
// come from the chunk-major copy when there is one: the 16 bytes of every row for chunk c
// then lie in one compact slice, which stays in L2 while the blocks of a long-segment launch
// work through chunk c, where rows of the row-major copy are evicted between chunks.
template <int CW>
constexpr int kQuads = (CW + 3) / 4;

template <int E, int STRIDE, int CW, class St>
__device__ __forceinline__ void load_chunk(const SweepArgs& a, St& st, int L, int lo,
                                           int lane, int c, float4 (&t)[E][kQuads<CW>]) {
    // (row p, chunk c) starts at element p * rs + c * cs of the copy (uniform strides)
    const bool cm = CW == kChunkMajorW && a.Apc != nullptr;
    const float* base = cm ? a.Apc : a.Ap;
    const int64_t cs = cm ? a.Prows * kChunkMajorW : (int64_t)CW;
    const int64_t rs = cm ? kChunkMajorW : (int64_t)a.Sp;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (lo + lane + STRIDE * e < L) {
            const int64_t off = (int64_t)st.id(e) * rs + c * cs;
            if (a.tile_bf16) {
                // CW bfloat16 values: one 4- or 8-byte load (CW = 2, 4) or CW / 8 16-byte loads
                const uint16_t* p = reinterpret_cast<const uint16_t*>(base) + off;
                if constexpr (CW == 2) {
                    const unsigned w = *reinterpret_cast<const unsigned*>(p);
                    t[e][0] = make_float4(__uint_as_float(w << 16), __uint_as_float(w & 0xFFFF0000u), 0.f, 0.f);
                } else if constexpr (CW == 4) {
                    const uint2 w = *reinterpret_cast<const uint2*>(p);
                    t[e][0] = make_float4(__uint_as_float(w.x << 16), __uint_as_float(w.x & 0xFFFF0000u),
                                          __uint_as_float(w.y << 16), __uint_as_float(w.y & 0xFFFF0000u));
                } else {
#pragma unroll
                    for (int q = 0; q < CW / 8; ++q) {
                        const uint4 w = reinterpret_cast<const uint4*>(p)[q];
                        t[e][2 * q] = make_float4(__uint_as_float(w.x << 16), __uint_as_float(w.x & 0xFFFF0000u),
                                                  __uint_as_float(w.y << 16), __uint_as_float(w.y & 0xFFFF0000u));
                        t[e][2 * q + 1] = make_float4(__uint_as_float(w.z << 16), __uint_as_float(w.z & 0xFFFF0000u),
                                                      __uint_as_float(w.w << 16), __uint_as_float(w.w & 0xFFFF0000u));
                    }
                }
            } else if constexpr (CW == 2) {
                const float2 w = *reinterpret_cast<const float2*>(base + off);
                t[e][0] = make_float4(w.x, w.y, 0.f, 0.f);
            } else {
                const float4* p = reinterpret_cast<const float4*>(base + off);
#pragma unroll
                for (int q = 0; q < CW / 4; ++q) t[e][q] = p[q];
            }
        } else {
#pragma unroll
            for (int q = 0; q < kQuads<CW>; ++q) t[e][q] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
}

template <int E, int CW>
__device__ __forceinline__ float comp(const float4 (&t)[E][kQuads<CW>], int e, int cc) {
    const float4 q = t[e][cc >> 2];
    switch (cc & 3) {
        case 0: return q.x;
        case 1: return q.y;
        case 2: return q.z;
        default: return q.w;
    }
}

// Alg. 2's inner loop for coordinate s of one segment, given the lane's fixed-factor values
// Per-lane statistics (coordinates, evaluations, accepted steps, halvings, rejections,
// step-limit exits).  Counters<false> compiles them away for launches that do not collect
// them: six registers fewer in a kernel bounded by 128.
template <bool ON>
struct Counters {
    unsigned c[6] = {0, 0, 0, 0, 0, 0};
    __device__ __forceinline__ void add(int q) { c[q] += 1; }
};
template <>
struct Counters<false> {
    __device__ __forceinline__ void add(int) {}
};

// tk[e] for this coordinate and eq. 6's sums S1, S2 at the current model.  A trial keeps NACC
// float sums with the coordinate's own S1, S2 at acc[OFF], acc[OFF + 1]; later(e, ww, uu, acc)
// adds further sums per element (the lookahead form adds those of the chunk's later
// coordinates) and red.sum(acc, OFF) all-reduces acc[OFF..NACC); commit(acc) runs when a
// trial is accepted.
template <int E, int NACC, int OFF, class Later, class Commit, class Red, class St, class Cnt>
__device__ __forceinline__ void newton_coordinate(const SweepArgs& a, int s, const float (&tk)[E], float S1,
                                                  float S2, Later&& later, Commit&& commit, St& st, float* xs,
                                                  Red& red, Cnt& cnt) {
    constexpr bool UNI = Red::kUniform;
    float xk = seg_uniform<UNI>(xs[s]);
    const double sA = seg_uniform<UNI>(a.sumA[s]);
    S1 = seg_uniform<UNI>(S1);
    S2 = seg_uniform<UNI>(S2);
    double P = sA + (double)a.alpha * xk + (double)a.beta;
    double g = P - (double)S1;
    float h = S2 + a.alpha;
    cnt.add(0);
    int steps = 0;
    while ((g < -(double)a.eps_g * P) || (g > (double)a.eps_g * P && xk > 0.0f)) {
        float d;
        if (h <= 0.0f) {
            if (g > 0.0) d = -xk;
            else break;
        } else {
            // g / h by the reciprocal and one Newton-Raphson correction (within an ulp or two of
            // the quotient; the IEEE division's scale/fixup sequence is on every step's chain)
            const float gf = (float)g;
            const float rh = fast_rcp(h);
            float q = gf * rh;
            q = fmaf(fmaf(-h, q, gf), rh, q);
            const float xn = xk - q;
            d = fmaxf(xn, 0.0f) - xk;
        }
        const float dN = d;  // Alg. 2's projected Newton step (the break test uses it)
        // the trials write the lane state in place; the model before the step is kept for
        // a halved retry and for the restore after a rejection
        double axo[E];
#pragma unroll
        for (int e = 0; e < E; ++e) axo[e] = st.ax[e];
        float acc[NACC];
        double gn, Pn;
        float hn;
        int j = 0;
        bool rejected = false;
        for (;;) {
#pragma unroll
            for (int i = 0; i < NACC; ++i) acc[i] = 0.0f;
            // the trial coordinate as it will be stored (float32), and the model moved by the
            // stored increment (exact in float64), so that the model values stay those of the
            // factors as stored: carried from one half-sweep to the next, they then equal
            // recomputed ones up to float64 rounding
            const float xt = xk + d;
            const double dd = (double)xt - (double)xk;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const double m = fmax(fma(dd, (double)tk[e], axo[e]), 0.0);
                const float ri = fast_rcp((float)m + a.eps_log);
                const float ww = st.v(e) * ri;
                const float uu = ww * ri;
                st.ax[e] = m;
                st.set_wu(e, ww, uu);
                acc[OFF] = fmaf(tk[e], ww, acc[OFF]);
                acc[OFF + 1] = fmaf(tk[e], tk[e] * uu, acc[OFF + 1]);
                later(e, ww, uu, acc);
            }
            red.sum(acc, OFF);
            cnt.add(1);
            Pn = sA + (double)a.alpha * xt + (double)a.beta;
            gn = Pn - (double)seg_uniform<UNI>(acc[OFF]);
            hn = seg_uniform<UNI>(acc[OFF + 1]) + a.alpha;
            if (!(a.guard && d < 0.0f && g + gn < 0.0)) break;
            if (j == a.j_max) { rejected = true; break; }
            d *= 0.5f;
            ++j;
            cnt.add(3);
        }
        if (rejected) {
            // back to the model before the step; w and u by the formula that made them
#pragma unroll
            for (int e = 0; e < E; ++e) {
                st.ax[e] = axo[e];
                const float ri = fast_rcp((float)axo[e] + a.eps_log);
                const float ww = st.v(e) * ri;
                st.set_wu(e, ww, ww * ri);
            }
            cnt.add(4);
            break;
        }
        commit(acc);
        const float xprev = xk;
        xk = xk + d;
        g = gn;
        h = hn;
        P = Pn;
        ++steps;
        cnt.add(2);
        const bool stop = a.literal_break ? (dN < a.eps_x * xprev) : (fabsf(dN) < a.eps_x * xprev);
        if (stop) break;
        if (steps >= a.t_max) { cnt.add(5); break; }
    }
    xs[s] = xk;
}

// eq. 6's sums of one coordinate at the current model, all-reduced over the segment.
template <int E, class Red, class St, class Cnt>
__device__ __forceinline__ void coordinate_sums(const SweepArgs& a, const float (&tk)[E], St& st, Red& red,
                                                float& S1, float& S2, Cnt& cnt) {
    float acc[2] = {0.0f, 0.0f};
#pragma unroll
    for (int e = 0; e < E; ++e) {
        float we, ue;
        st.wu(e, a.eps_log, we, ue);
        acc[0] = fmaf(tk[e], we, acc[0]);
        acc[1] = fmaf(tk[e], tk[e] * ue, acc[1]);
    }
    red.sum(acc, 0);
    S1 = acc[0];
    S2 = acc[1];
    cnt.add(1);
}

// Coordinate s = c*CW + cc with the chunk's tile values in registers.  LA (lookahead):
// LS[2k], LS[2k+1] hold eq. 6's sums S1, S2 of chunk coordinate k >= cc at the current model;
// every trial evaluation also computes the sums of the chunk coordinates after cc at the
// trial model, so that an accepted step leaves LS valid.  The sums are the same numbers the
// sequential order would compute later from the same model.  Without LA, the coordinate's
// own sums are evaluated here.
template <int cc, int E, bool LA, int CW, class Red, class St, class Cnt>
__device__ __forceinline__ void coordinate_step(const SweepArgs& a, int s,
                                                const float4 (&t)[E][kQuads<CW>], St& st, float* xs,
                                                Red& red, float (&LS)[2 * CW], Cnt& cnt) {
    float tk[E];
#pragma unroll
    for (int e = 0; e < E; ++e) tk[e] = comp<E, CW>(t, e, cc);
    if constexpr (LA) {
        auto later = [&](int e, float ww, float uu, float (&acc)[2 * CW]) {
#pragma unroll
            for (int k = cc + 1; k < CW; ++k) {
                const float tq = comp<E, CW>(t, e, k);
                acc[2 * k] = fmaf(tq, ww, acc[2 * k]);
                acc[2 * k + 1] = fmaf(tq, tq * uu, acc[2 * k + 1]);
            }
        };
        auto commit = [&](const float (&acc)[2 * CW]) {
#pragma unroll
            for (int k = cc + 1; k < CW; ++k) {
                LS[2 * k] = acc[2 * k];
                LS[2 * k + 1] = acc[2 * k + 1];
            }
        };
        newton_coordinate<E, 2 * CW, 2 * cc>(a, s, tk, LS[2 * cc], LS[2 * cc + 1], later, commit, st, xs, red, cnt);
    } else {
        float S1, S2;
        coordinate_sums(a, tk, st, red, S1, S2, cnt);
        newton_coordinate<E, 2, 0>(a, s, tk, S1, S2, [](int, float, float, float (&)[2]) {},
                                   [](const float (&)[2]) {}, st, xs, red, cnt);
    }
}

// The coordinates of chunk c in order (template recursion: each coordinate index is a
// compile-time constant, so every register array is indexed statically).
// cmap (fold-in): x and sumA are kept in the original coordinate order and step s of the
// pass visits coordinate cmap[s]; null: they are already in the sweep's order.
template <int CC, int E, bool LA, int CW, class Red, class St, class Cnt>
__device__ __forceinline__ void chunk_steps(const SweepArgs& a, int c, const float4 (&t)[E][kQuads<CW>],
                                            St& st, float* xs, Red& red, float (&LS)[2 * CW],
                                            Cnt& cnt, const int32_t* cmap = nullptr) {
    if constexpr (CC < CW) {
        const int s = c * CW + CC;
        if (s < a.r) {
            coordinate_step<CC, E, LA, CW>(a, cmap ? cmap[s] : s, t, st, xs, red, LS, cnt);
            chunk_steps<CC + 1, E, LA, CW>(a, c, t, st, xs, red, LS, cnt, cmap);
        }
    }
}

// Alg. 2 on one segment (or on this block's part [lo, lo + STRIDE*E) of a long segment).
// PREFETCH keeps the next tile chunk in flight while the current one is processed; CW is
// the tile chunk width (coordinates per chunk).
template <int STRIDE, bool PREFETCH, bool LA, int CW, bool STATS = true, class Red, class St>
__device__ __forceinline__ void sweep_segment(const SweepArgs& a, int seg, bool active, int lane,
                                              int lo, bool count_stats, float* xs, Red& red, St& st) {
    constexpr int E = St::kE;
    static_assert(LA || St::kStoresWU, "the per-coordinate evaluation reads stored w and u");
    int64_t base = 0;
    int L = 0;
    if (active) {
        base = a.ptr[seg];
        L = (int)(a.ptr[seg + 1] - base);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int l = lo + lane + STRIDE * e;
        float v = 0.0f;
        if (l < L) {
            const int64_t q = base + l;
            st.id(e) = a.idx[q];
            v = a.val[q];
            st.ax[e] = a.model_from_tiles ? 0.0 : (a.Mmap ? a.Min[a.Mmap[q]] : a.Min[q]);
        } else {
            st.id(e) = 0;
            st.ax[e] = 0.0;
        }
        st.v(e) = v;
    }
    if (!active) return;
    const int nchunks = (a.r + CW - 1) / CW;
    float4 cur[E][kQuads<CW>];
    if (a.model_from_tiles) {
        // Alg. 2's first step: Ax at the segment's nonzeros from the tiles and x (float64 sums
        // of exact float32 products), so that the model and the tiles define one subproblem
        // (bf16-rounded tiles; V streamed from host memory with no model values kept)
        for (int c = 0; c < nchunks; ++c) {
            load_chunk<E, STRIDE, CW>(a, st, L, lo, lane, c, cur);
#pragma unroll
            for (int cc = 0; cc < CW; ++cc) {
                const int sc = c * CW + cc;
                const double xv = sc < a.r ? (double)xs[sc] : 0.0;
#pragma unroll
                for (int e = 0; e < E; ++e) st.ax[e] = fma((double)comp<E, CW>(cur, e, cc), xv, st.ax[e]);
            }
        }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const float ri = fast_rcp((float)st.ax[e] + a.eps_log);
        st.set_wu(e, st.v(e) * ri, st.v(e) * ri * ri);
    }
    Counters<STATS> cnt;
    load_chunk<E, STRIDE, CW>(a, st, L, lo, lane, 0, cur);
    for (int c = 0; c < nchunks; ++c) {
        float4 nxt[E][kQuads<CW>];
        if (PREFETCH && c + 1 < nchunks) load_chunk<E, STRIDE, CW>(a, st, L, lo, lane, c + 1, nxt);
        float LS[2 * CW];
        if constexpr (LA) {
            // eq. 6's sums of every coordinate of the chunk at the current model
#pragma unroll
            for (int i = 0; i < 2 * CW; ++i) LS[i] = 0.0f;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                float we, ue;
                st.wu(e, a.eps_log, we, ue);
#pragma unroll
                for (int k = 0; k < CW; ++k) {
                    const float tq = comp<E, CW>(cur, e, k);
                    LS[2 * k] = fmaf(tq, we, LS[2 * k]);
                    LS[2 * k + 1] = fmaf(tq, tq * ue, LS[2 * k + 1]);
                }
            }
            red.sum(LS, 0);
            cnt.add(1);
        }
        chunk_steps<0, E, LA, CW>(a, c, cur, st, xs, red, LS, cnt);
        if (PREFETCH) {
#pragma unroll
            for (int e = 0; e < E; ++e)
#pragma unroll
                for (int q = 0; q < kQuads<CW>; ++q) cur[e][q] = nxt[e][q];
        } else if (c + 1 < nchunks) {
            load_chunk<E, STRIDE, CW>(a, st, L, lo, lane, c + 1, cur);
        }
    }
    // write back the model at the nonzeros (this segment order)
    if (a.Mout) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int l = lo + lane + STRIDE * e;
            if (l < L) a.Mout[base + l] = st.ax[e];
        }
    }
    if constexpr (STATS) {
        if (a.stats && count_stats && lane == 0) {
#pragma unroll
            for (int q = 0; q < 6; ++q) atomicAdd(&a.stats[q], (unsigned long long)cnt.c[q]);
        }
    }
}

// Tile chunk width of the fused launch (8 coordinates: half the chunk loads of 4, whose
// latency is exposed without prefetching).
constexpr int kFusedCW = 8;

template <int G, int E, bool LA, int CW = kFusedCW, bool STATS = true>
__device__ __forceinline__ void sweep_block(const SweepArgs& ag, const BlockWork& wk, const int32_t* segs,
                                            float* xs_all, float* red_lds, double* sA_lds) {
    const int slot = threadIdx.x / G;
    const int lane = threadIdx.x % G;
    const bool active = slot < wk.count;
    const int seg = active ? segs[wk.first + slot] : 0;
    float* xs = xs_all + slot * NMFKL_R_MAX;
    // x of the segment, permuted into this sweep's order; the column sums in LDS (every
    // coordinate step reads one, and the block's segments share them)
    if (active)
        for (int s = lane; s < ag.r; s += G) xs[s] = ag.X[(int64_t)seg * ag.r + ag.ids[s]];
    for (int s = threadIdx.x; s < ag.r; s += kFusedThreads) sA_lds[s] = ag.sumA[s];
    SweepArgs a = ag;
    a.sumA = sA_lds;
    __syncthreads();
    RegElems<E> st;
    if constexpr (G <= 64) {
        WaveReducer<G> red;
        sweep_segment<G, false, LA, CW, STATS>(a, seg, active, lane, 0, true, xs, red, st);
    } else {
        BlockReducer<G> red{red_lds, 0, nullptr};
        sweep_segment<G, false, LA, CW, STATS>(a, seg, active, lane, 0, true, xs, red, st);
        __syncthreads();
    }
    if (active)
        for (int s = lane; s < a.r; s += G) a.X[(int64_t)seg * a.r + a.ids[s]] = xs[s];
}

template <int G, int E, int CW, bool STATS = true>
__device__ __forceinline__ void sweep_block_lds(const SweepArgs& ag, const BlockWork& wk, const int32_t* segs,
                                                float* xs_all, double* sA_lds, int32_t* s_id, float* s_v,
                                                float* red_lds) {
    const int slot = threadIdx.x / G;
    const int lane = threadIdx.x % G;
    const bool active = slot < wk.count;
    const int seg = active ? segs[wk.first + slot] : 0;
    float* xs = xs_all + slot * NMFKL_R_MAX;
    if (active)
        for (int s = lane; s < ag.r; s += G) xs[s] = ag.X[(int64_t)seg * ag.r + ag.ids[s]];
    for (int s = threadIdx.x; s < ag.r; s += kFusedThreads) sA_lds[s] = ag.sumA[s];
    SweepArgs a = ag;
    a.sumA = sA_lds;
    __syncthreads();
    LdsElemsNoWU<E, G> st;
    st.idp = s_id + slot * G * E + lane;
    st.vp = s_v + slot * G * E + lane;
    if constexpr (G <= 64) {
        WaveReducer<G> red;
        sweep_segment<G, false, true, CW, STATS>(a, seg, active, lane, 0, true, xs, red, st);
    } else {
        BlockReducer<G> red{red_lds, 0, nullptr};
        sweep_segment<G, false, true, CW, STATS>(a, seg, active, lane, 0, true, xs, red, st);
        __syncthreads();
    }
    if (active)
        for (int s = lane; s < a.r; s += G) a.X[(int64_t)seg * a.r + a.ids[s]] = xs[s];
}

// The fused binned launch: each block picks its (G, E) variant from the work table.
// LA256 selects the lookahead form for the 256-lane variant.  The kernel is latency-bound
// (each coordinate is a dependent chain of sums, a reduction and Newton logic), so it runs
// at 4 waves per SIMD (at most 128 registers) without a prefetched second tile chunk.
template <bool LA256, bool STATS>
__global__ void __launch_bounds__(kFusedThreads, LA256 ? 2 : 4)
k_sweep_fused(const SweepArgs* __restrict__ tab, const BlockWork* __restrict__ work,
              const int32_t* __restrict__ segs) {
    __shared__ float xs_all[(kFusedThreads / 8) * NMFKL_R_MAX];
    __shared__ float red[2 * (kFusedThreads / 64) * kMaxRed];
    __shared__ double sA_lds[NMFKL_R_MAX];
    __shared__ int32_t s_id[kFusedThreads * 8];
    __shared__ float s_v[kFusedThreads * 8];
    const BlockWork wk = work[blockIdx.x];
    const SweepArgs a = tab[wk.prob];
    // the variants of kVariants, in its order (E = 3 between the E = 4 ones: lanes hold a
    // segment more tightly, so fewer lanes idle in its per-coordinate work)
    switch (wk.variant) {
        case 0: sweep_block<8, 3, false, kFusedCW, STATS>(a, wk, segs, xs_all, red, sA_lds); break;
        case 1: sweep_block<8, 4, false, kFusedCW, STATS>(a, wk, segs, xs_all, red, sA_lds); break;
        case 2: sweep_block<16, 3, false, kFusedCW, STATS>(a, wk, segs, xs_all, red, sA_lds); break;
        case 3: sweep_block<16, 4, false, kFusedCW, STATS>(a, wk, segs, xs_all, red, sA_lds); break;
        case 4: sweep_block<32, 3, false, kFusedCW, STATS>(a, wk, segs, xs_all, red, sA_lds); break;
        case 5: sweep_block<32, 4, false, kFusedCW, STATS>(a, wk, segs, xs_all, red, sA_lds); break;
        case 6: sweep_block<64, 3, false, kFusedCW, STATS>(a, wk, segs, xs_all, red, sA_lds); break;
        case 7: sweep_block<64, 4, false, kFusedCW, STATS>(a, wk, segs, xs_all, red, sA_lds); break;
        case 8: sweep_block<64, 5, false, kFusedCW, STATS>(a, wk, segs, xs_all, red, sA_lds); break;
        case 9: sweep_block_lds<64, 6, 4, STATS>(a, wk, segs, xs_all, sA_lds, s_id, s_v, red); break;
        case 10: sweep_block_lds<64, 8, 4, STATS>(a, wk, segs, xs_all, sA_lds, s_id, s_v, red); break;
        case 11: sweep_block<256, 3, LA256, kFusedCW, STATS>(a, wk, segs, xs_all, red, sA_lds); break;
        case 12: sweep_block<256, 4, LA256, kFusedCW, STATS>(a, wk, segs, xs_all, red, sA_lds); break;
        default: sweep_block_lds<256, 8, 4, STATS>(a, wk, segs, xs_all, sA_lds, s_id, s_v, red); break;
    }
}

hipError_t launch_sweep_fused(const SweepArgs* tab, const BlockWork* work, const int32_t* segs,
                              int nblocks, bool lookahead, bool stats, hipStream_t stream) {
    if (nblocks <= 0) return hipSuccess;
    const dim3 grid(nblocks), block(kFusedThreads);
    if (lookahead && stats)
        hipLaunchKernelGGL((k_sweep_fused<true, true>), grid, block, 0, stream, tab, work, segs);
    else if (lookahead)
        hipLaunchKernelGGL((k_sweep_fused<true, false>), grid, block, 0, stream, tab, work, segs);
    else if (stats)
        hipLaunchKernelGGL((k_sweep_fused<false, true>), grid, block, 0, stream, tab, work, segs);
    else
        hipLaunchKernelGGL((k_sweep_fused<false, false>), grid, block, 0, stream, tab, work, segs);
    return hipGetLastError();
}

// Long segments (more than kMaxFusedLength nonzeros), lookahead form: B = ceil(L /
// kCoopCapacity) blocks of kCoopThreads threads x kCoopE nonzeros (256 x 20 at 2 blocks per
// compute unit, 10240 nonzeros per unit; or the wide form, 512 x 20 at one block per unit)
// cooperate through CoopReducer; all blocks of such a launch are co-resident (cooperative
// launch), so every wait ends.  Counts and ids live in LDS, the model values in registers, w
// and u are recomputed from the model at each chunk start, and tile chunks are 4 coordinates
// wide.
constexpr int kCoopCW = kChunkMajorW;

// One block's part of a long segment (NT threads): the segment's x and column sums into LDS,
// the sweep with the segment's other blocks (through CoopReducer), and x back (part 0).
template <int E, int NT>
__device__ __forceinline__ void long_part(const SweepArgs* __restrict__ tab, const LongWork& wk,
                                          unsigned long long* words, unsigned* err, int pmax, float* xs,
                                          float* red_lds, double* tmp, double* bcast, int32_t* s_id, float* s_v,
                                          double* sA_lds) {
    constexpr int CAP = NT * E;
    SweepArgs a = tab[wk.prob];
    const int lane = threadIdx.x;
    LdsElemsNoWU<E, NT> st;
    st.idp = s_id + lane;
    st.vp = s_v + lane;
    for (int s = lane; s < a.r; s += NT) {
        xs[s] = a.X[(int64_t)wk.seg * a.r + a.ids[s]];
        sA_lds[s] = a.sumA[s];
    }
    a.sumA = sA_lds;
    __syncthreads();
    CoopReducer<NT> red;
    red.blk.red = red_lds;
    red.blk.parity = 0;
    red.tmp = tmp;
    red.bcast = bcast;
    red.words = words + (size_t)wk.group * 2 * pmax * kMaxRed;
    red.err = err;
    red.B = wk.B;
    red.part = wk.part;
    red.round = 0;
    sweep_segment<NT, false, true, kCoopCW>(a, wk.seg, true, lane, wk.part * CAP, wk.part == 0, xs, red, st);
    __syncthreads();
    if (wk.part == 0)
        for (int s = lane; s < a.r; s += NT) a.X[(int64_t)wk.seg * a.r + a.ids[s]] = xs[s];
}

// Long segments whose parts all fit the co-resident capacity: one part per block of NT
// threads (kCoopThreads, or kWideThreads).
template <int E, int NT, int BPC>
__global__ void __launch_bounds__(NT, BPC)
k_sweep_long_flat(const SweepArgs* __restrict__ tab, const LongWork* __restrict__ work,
                  unsigned long long* __restrict__ words, unsigned* __restrict__ err, int pmax) {
    __shared__ float xs[NMFKL_R_MAX];
    __shared__ float red_lds[2 * (NT / 64) * kMaxRed];
    __shared__ double tmp[CoopReducer<NT>::J * kMaxRed];
    __shared__ double bcast[kMaxRed];
    __shared__ int32_t s_id[NT * E];
    __shared__ float s_v[NT * E];
    __shared__ double sA_lds[NMFKL_R_MAX];
    long_part<E, NT>(tab, work[blockIdx.x], words, err, pmax, xs, red_lds, tmp, bcast, s_id, s_v, sA_lds);
}

// Every long segment of a launch in one cooperative launch of at most the co-resident
// capacity: the blocks take parts from the work list in order through a ticket counter.  The
// parts of a segment are consecutive, so the blocks that take them work on it together.  A
// block waits for its partners only once every earlier part has been taken by a running
// block; the blocks holding parts of earlier segments finish without waiting on later
// parts, and each block takes a new ticket as soon as it is free, so every wait ends (given
// B <= the grid, which the planner checks).  The list holds the largest B first.
template <int E, int NT, int BPC>
__global__ void __launch_bounds__(NT, BPC)
k_sweep_long_queue(const SweepArgs* __restrict__ tab, const LongWork* __restrict__ work, int nparts,
                   unsigned long long* __restrict__ words, unsigned long long* __restrict__ ticket,
                   unsigned* __restrict__ err, int pmax) {
    __shared__ float xs[NMFKL_R_MAX];
    __shared__ float red_lds[2 * (NT / 64) * kMaxRed];
    __shared__ double tmp[CoopReducer<NT>::J * kMaxRed];
    __shared__ double bcast[kMaxRed];
    __shared__ int32_t s_id[NT * E];
    __shared__ float s_v[NT * E];
    __shared__ double sA_lds[NMFKL_R_MAX];
    __shared__ int s_ticket;
    for (;;) {
        if (threadIdx.x == 0) s_ticket = (int)atomicAdd(ticket, 1ull);
        __syncthreads();
        // uniform: keeps the work entry and everything derived from it in scalar registers
        const int t = __builtin_amdgcn_readfirstlane(s_ticket);
        __syncthreads();
        if (t >= nparts) break;
        long_part<E, NT>(tab, work[t], words, err, pmax, xs, red_lds, tmp, bcast, s_id, s_v, sA_lds);
    }
}

__global__ void k_zero_u64(unsigned long long* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

hipError_t launch_sweep_long(const SweepArgs* tab, const LongWork* work, int nparts, int grid,
                             unsigned long long* words, int ngroups, unsigned* err, int pmax, bool cooperative,
                             bool wide, hipStream_t stream) {
    if (nparts <= 0 || grid <= 0) return hipSuccess;
    // the groups' words, then the ticket counter
    const int64_t nwords = (int64_t)ngroups * 2 * pmax * kCoopValues;
    unsigned long long* ticket = words + nwords;
    hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)((nwords + 1 + 255) / 256)), dim3(256), 0, stream, words,
                       nwords + 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // one part per block when every part has a block of its own, else the ticket queue; wide:
    // blocks of kWideThreads (the parts were cut at kWideCapacity)
    const bool flat = grid == nparts;
    const void* fn;
    if (wide)
        fn = flat ? reinterpret_cast<const void*>(k_sweep_long_flat<kCoopE, kWideThreads, kWideBlocksPerCU>)
                  : reinterpret_cast<const void*>(k_sweep_long_queue<kCoopE, kWideThreads, kWideBlocksPerCU>);
    else
        fn = flat ? reinterpret_cast<const void*>(k_sweep_long_flat<kCoopE, kCoopThreads, kCoopBlocksPerCU>)
                  : reinterpret_cast<const void*>(k_sweep_long_queue<kCoopE, kCoopThreads, kCoopBlocksPerCU>);
    const dim3 block(wide ? kWideThreads : kCoopThreads);
    void* fargs[] = {&tab, &work, &words, &err, &pmax};
    void* qargs[] = {&tab, &work, &nparts, &words, &ticket, &err, &pmax};
    // cooperative = false (inside a captured graph): an ordinary launch of the same grid
    if (cooperative) return hipLaunchCooperativeKernel(fn, dim3(grid), block, flat ? fargs : qargs, 0, stream);
    return hipLaunchKernel(fn, dim3(grid), block, flat ? fargs : qargs, 0, stream);
}

int wide_kernel_blocks_per_cu() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void*>(k_sweep_long_queue<kCoopE, kWideThreads, kWideBlocksPerCU>), kWideThreads,
            0) != hipSuccess)
        return 0;
    return nb;
}

int long_kernel_blocks_per_cu() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(
                                                              k_sweep_long_queue<kCoopE, kCoopThreads, kCoopBlocksPerCU>),
                                                     kCoopThreads, 0) != hipSuccess)
        return 0;
    return nb;
}

// ------------------------------------------------------------------------ fold-in
// Documents folded in with W fixed (Alg. 1's F-half applied to new columns): each document
// starts from the mass-matched constant x0 = sum(v) / sum(sumW) (model x0 * rowsum(W) at
// its nonzeros) and runs Alg. 2 passes; pass p visits the coordinates in the order
// perm[p] (Philox stream 1) and gathers W[i][perm[p][s]] for the lane's nonzeros.  After
// every pass the document's KL (eq. 1 restricted to the column, float64) is all-reduced;
// the document stops after the first pass whose KL decrease is <= tol * KL, or after
// max_passes passes.  The documents of a launch are independent: a document's result does
// not depend on which others share the launch.
template <int E, int STRIDE, class St>
__device__ __forceinline__ void load_chunk_gather(const FoldinArgs& f, St& st, int L, int lane, int c,
                                                  const int32_t* perm, float4 (&t)[E][2]) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
        float q[kChunk];
        const bool ok = lane + STRIDE * e < L;
        const float* row = f.W + (int64_t)st.id(e) * f.r;
#pragma unroll
        for (int cc = 0; cc < kChunk; ++cc) {
            const int s = c * kChunk + cc;
            q[cc] = (ok && s < f.r) ? row[perm[s]] : 0.0f;
        }
        t[e][0] = make_float4(q[0], q[1], q[2], q[3]);
        t[e][1] = make_float4(q[4], q[5], q[6], q[7]);
    }
}

// The document's KL at the current model and x: sum_l (v log(v/ax) - v) + sum_k sumW_k x_k.
template <int G, int E, class Red, class St>
__device__ __forceinline__ double doc_kl(const FoldinArgs& f, St& st, int lane, const float* xs, Red& red) {
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const double v = (double)st.v(e);
        if (v != 0.0) acc += v * log(v / st.ax[e]) - v;
    }
    for (int k = lane; k < f.r; k += G) acc += f.sumW[k] * (double)xs[k];
    return red.sum_f64(acc);
}

template <int G, bool LA, class Red, class St>
__device__ __forceinline__ void foldin_segment(const FoldinArgs& f, const SweepArgs& a, int d, bool active,
                                               int lane, float* xs, int32_t* perm_lds, Red& red, St& st) {
    constexpr int E = St::kE;
    int64_t base = 0;
    int L = 0;
    if (active) {
        base = f.ptr[d];
        L = (int)(f.ptr[d + 1] - base);
    }
    double mass = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int l = lane + G * e;
        float v = 0.0f;
        st.id(e) = 0;
        if (l < L) {
            st.id(e) = f.idx[base + l];
            v = f.val[base + l];
        }
        st.v(e) = v;
        mass += (double)v;
    }
    if (!active) return;
    mass = red.sum_f64(mass);
    const double x0 = mass / f.totW;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        st.ax[e] = (lane + G * e < L) ? x0 * f.rowsumW[st.id(e)] : 0.0;
        const float ri = fast_rcp((float)st.ax[e] + a.eps_log);
        st.set_wu(e, st.v(e) * ri, st.v(e) * ri * ri);
    }
    for (int k = lane; k < f.r; k += G) xs[k] = (float)x0;
    if constexpr (G > 64) __syncthreads();
    double kl_prev = doc_kl<G, E>(f, st, lane, xs, red);
    double kl = kl_prev;
    Counters<true> cnt;
    const int nchunks = (f.r + kChunk - 1) / kChunk;
    int p = 0;
    while (p < f.max_passes) {
        for (int s = lane; s < f.r; s += G) perm_lds[s] = f.perm[(int64_t)p * f.r + s];
        if constexpr (G > 64) __syncthreads();
        for (int c = 0; c < nchunks; ++c) {
            float4 cur[E][2];
            load_chunk_gather<E, G>(f, st, L, lane, c, perm_lds, cur);
            float LS[2 * kChunk];
            if constexpr (LA) {
#pragma unroll
                for (int i = 0; i < 2 * kChunk; ++i) LS[i] = 0.0f;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    float we, ue;
                    st.wu(e, a.eps_log, we, ue);
#pragma unroll
                    for (int k = 0; k < kChunk; ++k) {
                        const float tq = comp<E, kChunk>(cur, e, k);
                        LS[2 * k] = fmaf(tq, we, LS[2 * k]);
                        LS[2 * k + 1] = fmaf(tq, tq * ue, LS[2 * k + 1]);
                    }
                }
                red.sum(LS, 0);
                cnt.add(1);
            }
            chunk_steps<0, E, LA, kChunk>(a, c, cur, st, xs, red, LS, cnt, perm_lds);
        }
        if constexpr (G > 64) __syncthreads();
        ++p;
        kl = doc_kl<G, E>(f, st, lane, xs, red);
        if (kl_prev - kl <= f.tol * kl) break;
        kl_prev = kl;
    }
    for (int k = lane; k < f.r; k += G) f.F[(int64_t)d * f.r + k] = xs[k];
    if (lane == 0) {
        f.passes[d] = p;
        f.kl[d] = kl;
    }
    if (f.done) {
        // the document's outputs are visible system-wide before its completion word: every
        // lane orders its own stores (a wave waits for all of its lanes'), and a multi-wave
        // document's waves meet at a barrier (the whole block works on that one document)
        __threadfence_system();
        if constexpr (G > 64) __syncthreads();
        if (lane == 0) __hip_atomic_store(f.done + d, f.done_tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    if (a.stats && lane == 0) {
#pragma unroll
        for (int q = 0; q < 6; ++q) atomicAdd(&a.stats[q], (unsigned long long)cnt.c[q]);
    }
}

template <int G, int E>
__global__ void __launch_bounds__(kFusedThreads, 2)
k_foldin(FoldinArgs f, SweepArgs a, const int32_t* __restrict__ docs, int ndocs) {
    constexpr int SPB = kFusedThreads / G;
    __shared__ float xs_all[SPB * NMFKL_R_MAX];
    __shared__ int32_t perm_all[SPB * NMFKL_R_MAX];
    __shared__ float red[2 * (kFusedThreads / 64) * kMaxRed];
    __shared__ double red64[2 * (kFusedThreads / 64)];
    __shared__ double sA_lds[NMFKL_R_MAX];
    const int slot = threadIdx.x / G, lane = threadIdx.x % G;
    const int di = blockIdx.x * SPB + slot;
    const bool active = di < ndocs;
    const int d = active ? docs[di] : 0;
    for (int k = threadIdx.x; k < a.r; k += kFusedThreads) sA_lds[k] = a.sumA[k];
    __syncthreads();
    a.sumA = sA_lds;
    RegElems<E> st;
    if constexpr (G <= 64) {
        WaveReducer<G> rd;
        foldin_segment<G, true>(f, a, d, active, lane, xs_all + slot * NMFKL_R_MAX,
                                perm_all + slot * NMFKL_R_MAX, rd, st);
    } else {
        BlockReducer<G> rd{red, 0, red64};
        foldin_segment<G, true>(f, a, d, active, lane, xs_all, perm_all, rd, st);
    }
}

// One document per block of G threads (the longest documents): counts, w, u and word ids in
// LDS, the model values and the tile chunk in registers.  LA = false evaluates each
// coordinate's sums on their own (fewer registers; the same sums in the same order).
template <int G, int E, bool LA>
__global__ void __launch_bounds__(G)
k_foldin_block(FoldinArgs f, SweepArgs a, const int32_t* __restrict__ docs, int ndocs) {
    __shared__ float xs[NMFKL_R_MAX];
    __shared__ int32_t perm[NMFKL_R_MAX];
    __shared__ float red[2 * (G / 64) * kMaxRed];
    __shared__ double red64[2 * (G / 64)];
    __shared__ int32_t s_id[G * E];
    __shared__ float s_v[G * E], s_w[G * E], s_u[G * E];
    __shared__ double sA_lds[NMFKL_R_MAX];
    const bool active = (int)blockIdx.x < ndocs;
    const int d = active ? docs[blockIdx.x] : 0;
    const int lane = threadIdx.x;
    for (int k = lane; k < a.r; k += G) sA_lds[k] = a.sumA[k];
    __syncthreads();
    a.sumA = sA_lds;
    BlockReducer<G> rd{red, 0, red64};
    LdsElems<E, G> st;
    st.idp = s_id + lane;
    st.vp = s_v + lane;
    st.wp = s_w + lane;
    st.up = s_u + lane;
    foldin_segment<G, LA>(f, a, d, active, lane, xs, perm, rd, st);
}

hipError_t launch_foldin(const FoldinArgs& f, const SweepArgs& a, int variant, const int32_t* docs,
                         int ndocs, hipStream_t stream) {
    if (ndocs <= 0) return hipSuccess;
    switch (variant) {
        case 0:
            hipLaunchKernelGGL((k_foldin<16, 4>), dim3((ndocs + 15) / 16), dim3(kFusedThreads), 0, stream, f, a, docs, ndocs);
            break;
        case 1:
            hipLaunchKernelGGL((k_foldin<64, 4>), dim3((ndocs + 3) / 4), dim3(kFusedThreads), 0, stream, f, a, docs, ndocs);
            break;
        case 2:
            hipLaunchKernelGGL((k_foldin<256, 4>), dim3(ndocs), dim3(kFusedThreads), 0, stream, f, a, docs, ndocs);
            break;
        case 3:
            hipLaunchKernelGGL((k_foldin_block<256, 8, true>), dim3(ndocs), dim3(256), 0, stream, f, a, docs, ndocs);
            break;
        default:
            hipLaunchKernelGGL((k_foldin_block<512, 10, false>), dim3(ndocs), dim3(512), 0, stream, f, a, docs, ndocs);
            break;
    }
    return hipGetLastError();
}

// Row sums of W in float64 (one thread per row).
__global__ void k_row_sums(const float* __restrict__ W, int64_t n, int r, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int k = 0; k < r; ++k) acc += (double)W[i * r + k];
    out[i] = acc;
}

// Exact zeros of a factor (the sparsity the paper reports for its solutions, Table 2): each
// block counts its grid-stride share in a register, then one atomic add per wave.
__global__ void __launch_bounds__(256) k_count_zeros(const float* __restrict__ A, int64_t count,
                                                    unsigned long long* __restrict__ out) {
    unsigned long long c = 0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count; q += (int64_t)gridDim.x * blockDim.x)
        c += A[q] == 0.0f ? 1ull : 0ull;
    for (int m = 32; m >= 1; m >>= 1) c += __shfl_xor(c, m);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}

hipError_t launch_count_zeros(const float* A, int64_t count, unsigned long long* out, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>(2048, (count + 255) / 256);
    hipLaunchKernelGGL(k_count_zeros, dim3((unsigned)blocks), dim3(256), 0, stream, A, count, out);
    return hipGetLastError();
}

hipError_t launch_row_sums(const float* W, int64_t n, int r, double* out, hipStream_t stream) {
    hipLaunchKernelGGL(k_row_sums, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, W, n, r, out);
    return hipGetLastError();
}

// ------------------------------------------------- model at the nonzeros + objective
// One column per 64-lane wave (4 per block).  The wave stages F_j in LDS; lane g takes the
// nonzeros g, g+64, ...: M = W_i . F_j accumulated in float64 (products of float32 values
// are exact in float64), written to Mcsc, and the eq. 1 term v log(v/M) - v accumulated in
// float64.  Block partials go to partials[blockIdx].
__global__ void __launch_bounds__(256) k_model_objective(const int64_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ idx,
                                                         const float* __restrict__ val, int m,
                                                         const float* __restrict__ W,
                                                         const float* __restrict__ F, int r,
                                                         double* __restrict__ Mcsc,
                                                         double* __restrict__ partials,
                                                         int cols_per_block) {
    __shared__ float fj[4][NMFKL_R_MAX];
    __shared__ double red[256];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double acc = 0.0;
    const int j0 = blockIdx.x * cols_per_block;
    for (int jj = wv; jj < cols_per_block; jj += 4) {
        const int j = j0 + jj;
        if (j >= m) break;
        for (int k = lane; k < r; k += 64) fj[wv][k] = F[(int64_t)j * r + k];
        __builtin_amdgcn_wave_barrier();
        const int64_t b = ptr[j], e = ptr[j + 1];
        for (int64_t q = b + lane; q < e; q += 64) {
            const float* wi = W + (int64_t)idx[q] * r;
            double M = 0.0;
            for (int k = 0; k < r; ++k) M = fma((double)wi[k], (double)fj[wv][k], M);
            if (Mcsc) Mcsc[q] = M;
            const float v = val[q];
            if (v != 0.0f) acc += (double)v * log((double)v / M) - (double)v;
        }
        __builtin_amdgcn_wave_barrier();
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

hipError_t launch_model_objective(const int64_t* csc_ptr, const int32_t* csc_idx,
                                  const float* csc_val, int m, const float* W, const float* F, int r,
                                  double* Mcsc, double* partials, int nblocks, hipStream_t stream) {
    const int cpb = (m + nblocks - 1) / nblocks;
    hipLaunchKernelGGL(k_model_objective, dim3(nblocks), dim3(256), 0, stream, csc_ptr, csc_idx,
                       csc_val, m, W, F, r, Mcsc, partials, cpb);
    return hipGetLastError();
}

// eq. 1's per-nonzero terms v log(v/M) - v from model values already at hand (float64),
// block partials to partials[blockIdx].
__global__ void __launch_bounds__(256) k_model_terms(const double* __restrict__ M,
                                                     const float* __restrict__ val, int64_t nnz,
                                                     double* __restrict__ partials) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < nnz; q += (int64_t)gridDim.x * 256) {
        const float v = val[q];
        if (v != 0.0f) acc += (double)v * log((double)v / M[q]) - (double)v;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

hipError_t launch_model_terms(const double* M, const float* val, int64_t nnz, double* partials,
                              int nblocks, hipStream_t stream) {
    hipLaunchKernelGGL(k_model_terms, dim3(nblocks), dim3(256), 0, stream, M, val, nnz, partials);
    return hipGetLastError();
}

// dst[q] = src[map[q]]: the model values of one storage order in the other.
__global__ void __launch_bounds__(256) k_gather_f64(const double* __restrict__ src,
                                                    const int32_t* __restrict__ map, int64_t count,
                                                    double* __restrict__ dst) {
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < count; q += (int64_t)gridDim.x * 256)
        dst[q] = src[map[q]];
}

hipError_t launch_gather_f64(const double* src, const int32_t* map, int64_t count, double* dst,
                             hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    const int64_t nb = std::min<int64_t>((count + 255) / 256, 8192);
    hipLaunchKernelGGL(k_gather_f64, dim3((unsigned)nb), dim3(256), 0, stream, src, map, count, dst);
    return hipGetLastError();
}

__global__ void k_set_i64(int64_t* p, int64_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t stream) {
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(64), 0, stream, p, v);
    return hipGetLastError();
}

__global__ void k_sum_f64(const double* __restrict__ in, int count, double* __restrict__ out) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < count; i += 256) acc += in[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

hipError_t launch_sum_f64(const double* in, int count, double* out, hipStream_t stream) {
    hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(256), 0, stream, in, count, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- validation
__global__ void k_validate_ptr(const int64_t* __restrict__ ptr, int64_t Q, int64_t nnz,
                               unsigned* flags) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q > Q) return;
    const int64_t v = ptr[q];
    bool bad = v < 0 || v > nnz;
    if (q == 0) bad |= v != 0;
    if (q == Q) bad |= v != nnz;
    if (q < Q) bad |= ptr[q + 1] < v;
    if (bad) atomicOr(flags, kBadPtr);
}

hipError_t launch_validate_ptr(const int64_t* ptr, int64_t Q, int64_t nnz, unsigned* flags,
                               hipStream_t stream) {
    const int64_t n = Q + 1;
    hipLaunchKernelGGL(k_validate_ptr, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, ptr, Q,
                       nnz, flags);
    return hipGetLastError();
}

// Segment of entry q by binary search over ptr (valid pointers assumed: run after
// k_validate_ptr reported success).
__device__ __forceinline__ int64_t segment_of(const int64_t* ptr, int64_t Q, int64_t q) {
    int64_t lo = 0, hi = Q;  // ptr[lo] <= q < ptr[hi]
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (ptr[mid] <= q) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ void k_validate_entries(const int64_t* __restrict__ ptr, const int32_t* __restrict__ idx,
                                   const float* __restrict__ val, int64_t Q, int64_t P, int64_t nnz,
                                   unsigned* flags) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nnz) return;
    unsigned bad = 0;
    const int32_t i = idx[q];
    if (i < 0 || (int64_t)i >= P) bad |= kBadIndex;
    const float v = val[q];
    if (!(v >= 0.0f) || !isfinite(v)) bad |= kBadValue;
    const int64_t seg = segment_of(ptr, Q, q);
    if (q > ptr[seg] && idx[q - 1] >= i) bad |= kBadOrder;
    if (bad) atomicOr(flags, bad);
}

hipError_t launch_validate_entries(const int64_t* ptr, const int32_t* idx, const float* val,
                                   int64_t Q, int64_t P, int64_t nnz, unsigned* flags,
                                   hipStream_t stream) {
    if (nnz == 0) return hipSuccess;
    hipLaunchKernelGGL(k_validate_entries, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, stream,
                       ptr, idx, val, Q, P, nnz, flags);
    return hipGetLastError();
}

__global__ void k_validate_factor(const float* __restrict__ A, int64_t count, unsigned* flags,
                                  unsigned bit) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float v = A[i];
    if (!(v >= 0.0f) || !isfinite(v)) atomicOr(flags, bit);
}

hipError_t launch_validate_factor(const float* A, int64_t count, unsigned* flags, unsigned bit,
                                  hipStream_t stream) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_validate_factor, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream,
                       A, count, flags, bit);
    return hipGetLastError();
}

// For every CSR entry p = (row i, column j): find j's CSC entry holding row i by binary
// search; record both directions of the position map and check the values agree.  With
// equal nnz and strictly increasing indices this proves CSR == transpose(CSC).
__global__ void k_build_maps(const int64_t* __restrict__ csr_ptr, const int32_t* __restrict__ csr_idx,
                             const float* __restrict__ csr_val, const int64_t* __restrict__ csc_ptr,
                             const int32_t* __restrict__ csc_idx, const float* __restrict__ csc_val,
                             int64_t n, int64_t nnz, int32_t* __restrict__ csr2csc,
                             int32_t* __restrict__ csc2csr, unsigned* flags) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnz) return;
    const int32_t i = (int32_t)segment_of(csr_ptr, n, p);
    const int32_t j = csr_idx[p];
    int64_t lo = csc_ptr[j], hi = csc_ptr[j + 1];
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (csc_idx[mid] < i) lo = mid + 1;
        else hi = mid;
    }
    if (lo >= csc_ptr[j + 1] || csc_idx[lo] != i || csc_val[lo] != csr_val[p]) {
        atomicOr(flags, kBadTranspose);
        return;
    }
    csr2csc[p] = (int32_t)lo;
    csc2csr[lo] = (int32_t)p;
}

hipError_t launch_build_maps(const int64_t* csr_ptr, const int32_t* csr_idx, const float* csr_val,
                             const int64_t* csc_ptr, const int32_t* csc_idx, const float* csc_val,
                             int64_t n, int64_t nnz, int32_t* csr2csc, int32_t* csc2csr,
                             unsigned* flags, hipStream_t stream) {
    if (nnz == 0) return hipSuccess;
    hipLaunchKernelGGL(k_build_maps, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, stream, csr_ptr,
                       csr_idx, csr_val, csc_ptr, csc_idx, csc_val, n, nnz, csr2csc, csc2csr, flags);
    return hipGetLastError();
}

}  // namespace nmfkl
