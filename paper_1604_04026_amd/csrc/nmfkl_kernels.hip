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
// and streams the fixed-factor values of its nonzeros through registers one chunk of
// kChunk coordinates at a time (two float4 loads per nonzero per chunk, next chunk
// prefetched while the current one is processed).  S1 and S2 are all-reduced over the G
// lanes with DPP row operations (and LDS for multi-wave segments), so every lane of a
// segment takes the same Newton decisions.
//
// Precision: the derivative sums are float32 (all terms are positive).  The model values
// are float64 because a coordinate step can remove most of a nonzero's model value (for
// example when the other coordinates of a one-nonzero column drop to zero): in float32 the
// rounding error of the starting value would then become a large relative error of the
// small remainder, and with it of the derivatives.
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

// All-reduce over aligned groups of G lanes (G a power of two, G <= 64).  After the two quad
// steps every lane holds its quad's sum; the half-row mirror pairs quad q with the other quad
// of its 8-lane half, the row mirror pairs the two halves of a 16-lane row.  Each step adds
// the same two partial sums on both partners, so all lanes of a group end bit-identical.
template <int G>
__device__ __forceinline__ float group_sum(float v) {
    if constexpr (G >= 2) v += dpp_quad_xor1(v);
    if constexpr (G >= 4) v += dpp_quad_xor2(v);
    if constexpr (G >= 8) v += dpp_half_mirror(v);
    if constexpr (G >= 16) v += dpp_mirror(v);
    if constexpr (G >= 32) v += __shfl_xor(v, 16);
    if constexpr (G >= 64) v += __shfl_xor(v, 32);
    return v;
}

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// ---------------------------------------------------------------- permutation
__global__ void k_make_order(uint64_t seed, uint64_t t, uint64_t stream_id, int r, int32_t* ids) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int32_t tmp[NMFKL_R_MAX];
        coordinate_order(seed, t, stream_id, r, tmp);
        for (int i = 0; i < r; ++i) ids[i] = tmp[i];
    }
}

hipError_t launch_make_order(uint64_t seed, uint64_t t, uint64_t stream_id, int r, int32_t* ids,
                             hipStream_t stream) {
    hipLaunchKernelGGL(k_make_order, dim3(1), dim3(64), 0, stream, seed, t, stream_id, r, ids);
    return hipGetLastError();
}

// ------------------------------------------------- permuted copy + float64 column sums
// Block b covers rows [b*rpb, (b+1)*rpb).  Thread (ry, cx) walks rows ry, ry+4, ... of the
// block for permuted column s = s0 + cx, reading A[p][ids[s]] and writing Ap[p][s] (zero in
// the padding).  Per-block float64 partial sums go to partials[b*r + s]; the final sum over
// blocks is taken in block order by k_finalize_sums, so the result is deterministic.
__global__ void __launch_bounds__(256) k_permute_colsum(const float* __restrict__ A, int64_t P,
                                                        int r, int Sp,
                                                        const int32_t* __restrict__ ids,
                                                        float* __restrict__ Ap,
                                                        double* __restrict__ partials,
                                                        int64_t rpb) {
    __shared__ int32_t sid[NMFKL_R_MAX];
    __shared__ double red[4][64];
    for (int s = threadIdx.x; s < NMFKL_R_MAX; s += 256) sid[s] = s < r ? (ids ? ids[s] : s) : -1;
    __syncthreads();
    const int cx = threadIdx.x & 63, ry = threadIdx.x >> 6;
    const int64_t p0 = (int64_t)blockIdx.x * rpb;
    const int64_t p1 = p0 + rpb < P ? p0 + rpb : P;
    for (int s0 = 0; s0 < Sp; s0 += 64) {
        const int s = s0 + cx;
        const int k = s < Sp ? sid[s] : -1;
        double acc = 0.0;
        if (s < Sp) {
            for (int64_t p = p0 + ry; p < p1; p += 4) {
                const float a = k >= 0 ? A[p * r + k] : 0.0f;
                if (Ap) Ap[p * Sp + s] = a;
                acc += (double)a;
            }
        }
        red[ry][cx] = acc;
        __syncthreads();
        if (ry == 0 && s < r)
            partials[(int64_t)blockIdx.x * r + s] = ((red[0][cx] + red[1][cx]) + red[2][cx]) + red[3][cx];
        __syncthreads();
    }
}

hipError_t launch_permute_colsum(const float* A, int64_t P, int r, int Sp, const int32_t* ids,
                                 float* Ap, double* partials, int nblocks, hipStream_t stream) {
    const int64_t rpb = (P + nblocks - 1) / nblocks;
    hipLaunchKernelGGL(k_permute_colsum, dim3(nblocks), dim3(256), 0, stream, A, P, r, Sp, ids, Ap,
                       partials, rpb);
    return hipGetLastError();
}

__global__ void k_finalize_sums(const double* __restrict__ partials, int nblocks, int r,
                                double* __restrict__ out) {
    const int s = threadIdx.x;
    if (s < r) {
        double acc = 0.0;
        for (int b = 0; b < nblocks; ++b) acc += partials[(int64_t)b * r + s];
        out[s] = acc;
    }
}

hipError_t launch_finalize_sums(const double* partials, int nblocks, int r, double* out,
                                hipStream_t stream) {
    hipLaunchKernelGGL(k_finalize_sums, dim3(1), dim3(NMFKL_R_MAX), 0, stream, partials, nblocks, r,
                       out);
    return hipGetLastError();
}

// --------------------------------------------------------------- the sweep
// Per-segment element state held in registers.
template <int E>
struct Elems {
    int32_t id[E];
    double ax[E];
    float v[E], w[E], u[E];
};

// ---- segment-wide all-reduce of (S1, S2): three reducers with one interface -----------
// Every lane of a segment receives bit-identical sums, so every lane takes the same Newton
// decisions.

// Segments of G <= 64 lanes inside one wave: DPP / lane shuffles only.
template <int G>
struct WaveReducer {
    __device__ __forceinline__ float2 sum(float2 s) {
        s.x = group_sum<G>(s.x);
        s.y = group_sum<G>(s.y);
        return s;
    }
};

// One segment per block of NT threads: wave sums, then the NT/64 wave sums through LDS in
// wave order (double-buffered by parity, one barrier per reduction).
template <int NT>
struct BlockReducer {
    float2* red;  // LDS, 2 * NT/64 entries
    int parity;
    __device__ __forceinline__ float2 sum(float2 s) {
        s.x = group_sum<64>(s.x);
        s.y = group_sum<64>(s.y);
        constexpr int W = NT / 64;
        const int wv = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) red[parity * W + wv] = s;
        __syncthreads();
        float2 t = red[parity * W];
#pragma unroll
        for (int q = 1; q < W; ++q) {
            t.x += red[parity * W + q].x;
            t.y += red[parity * W + q].y;
        }
        parity ^= 1;
        return t;
    }
};

// A long segment split over B co-resident blocks (cooperative launch).  Each reduction:
// block sum; thread 0 publishes it (float64) in slot parity of the group's partials and
// arrives on the group's counter with release semantics, then waits (acquire) until all B
// blocks arrived; wave 0 reads the B partials, lane b holding partials b, b+64, ..., and
// all-reduces them with a fixed butterfly, so every block obtains the same total.  The wait
// is bounded: after kSpinLimit polls, or as soon as any block has recorded an error, the
// block records an error and continues (the host reports it at the next synchronising call).
constexpr unsigned kSpinLimit = 1u << 20;

__device__ __forceinline__ double shfl_xor_f64(double v, int m) {
    int2 p = *reinterpret_cast<int2*>(&v);
    p.x = __shfl_xor(p.x, m);
    p.y = __shfl_xor(p.y, m);
    return *reinterpret_cast<double*>(&p);
}

template <int NT>
struct CoopReducer {
    BlockReducer<NT> blk;
    double* bcast;      // LDS, 2 doubles
    double* partials;   // global: [2][B][2] for this group
    unsigned* counter;  // global: arrivals of this group
    unsigned* err;      // global error flags
    int B, part;
    unsigned round;
    __device__ __forceinline__ float2 sum(float2 s) {
        const float2 b = blk.sum(s);
        if (B == 1) return b;
        const unsigned slot = round & 1u;
        if (threadIdx.x == 0) {
            double* p = partials + ((size_t)slot * B + part) * 2;
            __hip_atomic_store(p, (double)b.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(p + 1, (double)b.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned target = (round + 1u) * (unsigned)B;
            unsigned spins = 0;
            while (__hip_atomic_load(counter, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
                __builtin_amdgcn_s_sleep(1);
                // give up on a timeout, or at once once any block has given up
                if (++spins > kSpinLimit ||
                    __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                    atomicOr(err, 1u);
                    break;
                }
            }
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            double sx = 0.0, sy = 0.0;
            for (int q = threadIdx.x; q < B; q += 64) {
                const double* p = partials + ((size_t)slot * B + q) * 2;
                sx += __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                sy += __hip_atomic_load(p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
#pragma unroll
            for (int m = 1; m < 64; m <<= 1) {
                sx += shfl_xor_f64(sx, m);
                sy += shfl_xor_f64(sy, m);
            }
            if (threadIdx.x == 0) {
                bcast[0] = sx;
                bcast[1] = sy;
            }
        }
        __syncthreads();
        ++round;
        return make_float2((float)bcast[0], (float)bcast[1]);
    }
};

// Alg. 2's inner loop for one coordinate s of one segment.  tk[e] holds A[i_l][s] for the
// lane's nonzeros.  xs points at the segment's x in LDS (permuted order).
template <int E, class Red>
__device__ __forceinline__ void coordinate_step(const SweepArgs& a, int s, const float (&tk)[E],
                                                Elems<E>& st, float* xs, Red& red,
                                                unsigned (&cnt)[6]) {
    float xk = xs[s];
    const double sA = a.sumA[s];
    float2 acc = make_float2(0.0f, 0.0f);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        acc.x = fmaf(tk[e], st.w[e], acc.x);
        acc.y = fmaf(tk[e] * tk[e], st.u[e], acc.y);
    }
    acc = red.sum(acc);
    double P = sA + (double)a.alpha * xk + (double)a.beta;
    double g = P - (double)acc.x;
    float h = acc.y + a.alpha;
    cnt[0] += 1;
    cnt[1] += 1;
    int steps = 0;
    while ((g < -(double)a.eps_g * P) || (g > (double)a.eps_g * P && xk > 0.0f)) {
        float d;
        if (h <= 0.0f) {
            if (g > 0.0) d = -xk;
            else break;
        } else {
            const float xn = xk - (float)g / h;
            d = fmaxf(xn, 0.0f) - xk;
        }
        const float dN = d;  // Alg. 2's projected Newton step (the break test uses it)
        double mm[E];
        float wn[E], un[E];
        double gn, Pn;
        float hn;
        int j = 0;
        bool rejected = false;
        for (;;) {
            float2 t2 = make_float2(0.0f, 0.0f);
            const double dd = (double)d;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const double m = fmax(fma(dd, (double)tk[e], st.ax[e]), 0.0);
                const float ri = fast_rcp((float)m + a.eps_log);
                const float ww = st.v[e] * ri;
                mm[e] = m;
                wn[e] = ww;
                un[e] = ww * ri;
                t2.x = fmaf(tk[e], ww, t2.x);
                t2.y = fmaf(tk[e] * tk[e], un[e], t2.y);
            }
            t2 = red.sum(t2);
            cnt[1] += 1;
            const float xt = xk + d;
            Pn = sA + (double)a.alpha * xt + (double)a.beta;
            gn = Pn - (double)t2.x;
            hn = t2.y + a.alpha;
            if (!(a.guard && d < 0.0f && g + gn < 0.0)) break;
            if (j == a.j_max) { rejected = true; break; }
            d *= 0.5f;
            ++j;
            cnt[3] += 1;
        }
        if (rejected) { cnt[4] += 1; break; }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            st.ax[e] = mm[e];
            st.w[e] = wn[e];
            st.u[e] = un[e];
        }
        const float xprev = xk;
        xk = xk + d;
        g = gn;
        h = hn;
        P = Pn;
        ++steps;
        cnt[2] += 1;
        const bool stop = a.literal_break ? (dN < a.eps_x * xprev) : (fabsf(dN) < a.eps_x * xprev);
        if (stop) break;
        if (steps >= a.t_max) { cnt[5] += 1; break; }
    }
    xs[s] = xk;
}

// Elements handled by this lane: l = lo + lane + STRIDE * e, e < E, restricted to l < L.
template <int E, int STRIDE>
__device__ __forceinline__ void load_chunk(const SweepArgs& a, const Elems<E>& st, int L, int lo,
                                           int lane, int c, float4 (&t)[E][2]) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (lo + lane + STRIDE * e < L) {
            const float4* p = reinterpret_cast<const float4*>(a.Ap + (int64_t)st.id[e] * a.Sp + c * kChunk);
            t[e][0] = p[0];
            t[e][1] = p[1];
        } else {
            t[e][0] = make_float4(0.f, 0.f, 0.f, 0.f);
            t[e][1] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
}

template <int E>
__device__ __forceinline__ float comp(const float4 (&t)[E][2], int e, int cc) {
    const float4 q = t[e][cc >> 2];
    switch (cc & 3) {
        case 0: return q.x;
        case 1: return q.y;
        case 2: return q.z;
        default: return q.w;
    }
}

// Alg. 2 on one segment (or on this block's part [lo, lo + STRIDE*E) of a long segment).
// PREFETCH: keep the next tile chunk in flight while the current one is processed.
template <int STRIDE, int E, bool PREFETCH, class Red>
__device__ __forceinline__ void sweep_segment(const SweepArgs& a, int seg, bool active, int lane,
                                              int lo, bool count_stats, float* xs, Red& red) {
    int64_t base = 0;
    int L = 0;
    if (active) {
        base = a.ptr[seg];
        L = (int)(a.ptr[seg + 1] - base);
    }
    Elems<E> st;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int l = lo + lane + STRIDE * e;
        if (l < L) {
            const int64_t q = base + l;
            st.id[e] = a.idx[q];
            st.v[e] = a.val[q];
            st.ax[e] = a.Mmap ? a.Min[a.Mmap[q]] : a.Min[q];
        } else {
            st.id[e] = 0;
            st.v[e] = 0.0f;
            st.ax[e] = 0.0;
        }
        const float ri = fast_rcp((float)st.ax[e] + a.eps_log);
        st.w[e] = st.v[e] * ri;
        st.u[e] = st.w[e] * ri;
    }
    if (!active) return;
    unsigned cnt[6] = {0, 0, 0, 0, 0, 0};
    const int nchunks = (a.r + kChunk - 1) / kChunk;
    float4 cur[E][2];
    load_chunk<E, STRIDE>(a, st, L, lo, lane, 0, cur);
    for (int c = 0; c < nchunks; ++c) {
        float4 nxt[E][2];
        if (PREFETCH && c + 1 < nchunks) load_chunk<E, STRIDE>(a, st, L, lo, lane, c + 1, nxt);
#pragma unroll
        for (int cc = 0; cc < kChunk; ++cc) {
            const int s = c * kChunk + cc;
            if (s < a.r) {
                float tk[E];
#pragma unroll
                for (int e = 0; e < E; ++e) tk[e] = comp<E>(cur, e, cc);
                coordinate_step<E>(a, s, tk, st, xs, red, cnt);
            }
        }
        if (PREFETCH) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                cur[e][0] = nxt[e][0];
                cur[e][1] = nxt[e][1];
            }
        } else if (c + 1 < nchunks) {
            load_chunk<E, STRIDE>(a, st, L, lo, lane, c + 1, cur);
        }
    }
    // write back the model at the nonzeros (this segment order)
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int l = lo + lane + STRIDE * e;
        if (l < L) a.Mout[base + l] = st.ax[e];
    }
    if (a.stats && count_stats && lane == 0) {
#pragma unroll
        for (int q = 0; q < 6; ++q) atomicAdd(&a.stats[q], (unsigned long long)cnt[q]);
    }
}

template <int G, int E>
__device__ __forceinline__ void sweep_block(const SweepArgs& a, const BlockWork& wk, const int32_t* segs,
                                            float* xs_all, float2* red_lds) {
    const int slot = threadIdx.x / G;
    const int lane = threadIdx.x % G;
    const bool active = slot < wk.count;
    const int seg = active ? segs[wk.first + slot] : 0;
    float* xs = xs_all + slot * NMFKL_R_MAX;
    // x of the segment, permuted into this sweep's order
    if (active)
        for (int s = lane; s < a.r; s += G) xs[s] = a.X[(int64_t)seg * a.r + a.ids[s]];
    __syncthreads();
    if constexpr (G <= 64) {
        WaveReducer<G> red;
        sweep_segment<G, E, true>(a, seg, active, lane, 0, true, xs, red);
    } else {
        BlockReducer<G> red{red_lds, 0};
        sweep_segment<G, E, true>(a, seg, active, lane, 0, true, xs, red);
        __syncthreads();
    }
    if (active)
        for (int s = lane; s < a.r; s += G) a.X[(int64_t)seg * a.r + a.ids[s]] = xs[s];
}

// The fused binned launch: each block picks its (G, E) variant from the work table.
__global__ void __launch_bounds__(kFusedThreads, 2)
k_sweep_fused(SweepArgs a, const BlockWork* __restrict__ work, const int32_t* __restrict__ segs) {
    __shared__ float xs_all[(kFusedThreads / 8) * NMFKL_R_MAX];
    __shared__ float2 red[2 * (kFusedThreads / 64)];
    const BlockWork wk = work[blockIdx.x];
    switch (wk.variant) {
        case 0: sweep_block<8, 4>(a, wk, segs, xs_all, red); break;
        case 1: sweep_block<16, 4>(a, wk, segs, xs_all, red); break;
        case 2: sweep_block<32, 4>(a, wk, segs, xs_all, red); break;
        case 3: sweep_block<64, 4>(a, wk, segs, xs_all, red); break;
        default: sweep_block<256, 4>(a, wk, segs, xs_all, red); break;
    }
}

hipError_t launch_sweep_fused(const SweepArgs& a, const BlockWork* work, const int32_t* segs,
                              int nblocks, hipStream_t stream) {
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sweep_fused, dim3(nblocks), dim3(kFusedThreads), 0, stream, a, work, segs);
    return hipGetLastError();
}

// Long segments: kLongThreads threads x kLongE elements per block; a segment of L nonzeros
// takes B = ceil(L / (kLongThreads*kLongE)) blocks that cooperate through CoopReducer.  All
// blocks of one launch are co-resident (cooperative launch), so every wait ends.
__global__ void __launch_bounds__(kLongThreads)
k_sweep_long(SweepArgs a, const LongWork* __restrict__ work, double* __restrict__ partials,
             unsigned* __restrict__ counters, unsigned* __restrict__ err, int pmax) {
    __shared__ float xs[NMFKL_R_MAX];
    __shared__ float2 red_lds[2 * (kLongThreads / 64)];
    __shared__ double bcast[2];
    const LongWork wk = work[blockIdx.x];
    const int lane = threadIdx.x;
    for (int s = lane; s < a.r; s += kLongThreads) xs[s] = a.X[(int64_t)wk.seg * a.r + a.ids[s]];
    __syncthreads();
    CoopReducer<kLongThreads> red;
    red.blk.red = red_lds;
    red.blk.parity = 0;
    red.bcast = bcast;
    red.partials = partials + (size_t)wk.group * 2 * 2 * pmax;
    red.counter = counters + wk.group;
    red.err = err;
    red.B = wk.B;
    red.part = wk.part;
    red.round = 0;
    sweep_segment<kLongThreads, kLongE, false>(a, wk.seg, true, lane, wk.part * kLongThreads * kLongE,
                                               wk.part == 0, xs, red);
    __syncthreads();
    if (wk.part == 0)
        for (int s = lane; s < a.r; s += kLongThreads) a.X[(int64_t)wk.seg * a.r + a.ids[s]] = xs[s];
}

__global__ void k_zero_u32(unsigned* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

hipError_t launch_sweep_long(const SweepArgs& a, const LongWork* work, int nblocks, double* partials,
                             unsigned* counters, int ngroups, unsigned* err, int pmax,
                             hipStream_t stream) {
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u32, dim3((ngroups + 255) / 256), dim3(256), 0, stream, counters, ngroups);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    SweepArgs aa = a;
    void* args[] = {&aa, &work, &partials, &counters, &err, &pmax};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_sweep_long), dim3(nblocks),
                                      dim3(kLongThreads), args, 0, stream);
}

int long_kernel_blocks_per_cu() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(k_sweep_long),
                                                     kLongThreads, 0) != hipSuccess)
        return 0;
    return nb;
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
            Mcsc[q] = M;
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
