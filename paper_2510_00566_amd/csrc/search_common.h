// Device-side helpers shared by the search kernels: the canonical distance
// recipe, the certified pruning threshold, wave/block scans and bitonic sorts.
#pragma once

#include "internal.h"

namespace pano {

constexpr int NT = 256;         // threads per workgroup (4 wavefronts)
constexpr int MERGE_LDS_KEYS = 2048;  // entries the merge sorts in LDS
constexpr int GMAX = 16;        // max queries per scan work item
constexpr int SB_MAX = 512;     // per-wave sort buffer (entries)
constexpr int WALK_CHUNKS = 8;  // four-float chunks of a level the per-pair walk requests at once
constexpr uint64_t KEY_MAX = ~0ull;
constexpr int FLAG_OVERFLOW = 1;

// Wave-uniform reads of query slices go through the constant address space so
// that they become scalar loads into SGPRs (a free broadcast to all lanes).
struct UniformF4 {
    const float *p;
    __device__ inline float4 operator[](int i) const
    {
#if defined(__HIP_DEVICE_COMPILE__)
        typedef __attribute__((address_space(4))) const float cfloat;
        cfloat *q = (cfloat *)p;
        return make_float4(q[4 * i], q[4 * i + 1], q[4 * i + 2], q[4 * i + 3]);
#else
        return make_float4(p[4 * i], p[4 * i + 1], p[4 * i + 2], p[4 * i + 3]);
#endif
    }
};
__device__ inline UniformF4 uniform_f4(const float *p) { return UniformF4{p}; }

// Scalars of one search, passed by value.
struct SearchConsts {
    int k;
    int kc;            // local top-k capacity per query (power of two >= k)
    int G;             // queries per work item
    int bpi;           // blocks per work item
    int item_cap;      // items per query group and list at most (0 = no cap)
    int capq;          // per-query result buffer capacity
    int nlist;
    int ceil8;         // ceil(nlist / 8)
    int prune;         // 1 = pruned scan, 0 = brute force
    int dense_min;     // refine a level densely while at least this many pairs survive
    int walk_lanes;    // lanes per pair in the per-pair walk (0 = by the number of pairs)
    int bf16;          // 1: read level tiles in bfloat16 (certified margin, FP32 rescoring)
    float ub;          // bfloat16 unit roundoff 2^-8, rounded up (covers the stored-norm rounding)
    float bfdelta;     // bfloat16 scan: u_b max ||x|| (0 for the FP32 scan)
    float eps;
    float one_m_eps2;  // 2 (1 - eps)
    Margins mg;
    LevelGeom g;
};

// Canonical distance: sequential FP64 sum of ((double)q_j - (double)x_j)^2,
// every operation rounded separately, then rounded to float32.
__device__ inline float canon_dist(const float *__restrict__ q, const float *__restrict__ x, int d)
{
#pragma clang fp contract(off)
    double s = 0.0;
    for (int j = 0; j < d; ++j) {
        double t = (double)q[j] - (double)x[j];
        double t2 = t * t;
        s = s + t2;
    }
    return (float)s;
}

// The same value with x read from global memory in 32-float chunks, the next
// chunk requested while the current one is summed (identical arithmetic,
// identical order; q in LDS).
__device__ inline float canon_dist_stream(const float *q_lds, const float *__restrict__ x, int d)
{
#pragma clang fp contract(off)
    double s = 0.0;
    int j = 0;
    if ((d & 3) == 0 && d >= 32) {
        // rows of a multiple of 4 floats start 16-byte aligned
        const float4 *x4 = reinterpret_cast<const float4 *>(x);
        float4 cur[8], nxt[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) cur[u] = x4[u];
        const int n32 = d >> 5;
        for (int c = 0; c < n32; ++c) {
            if (c + 1 < n32) {
#pragma unroll
                for (int u = 0; u < 8; ++u) nxt[u] = x4[(c + 1) * 8 + u];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const float xv[4] = {cur[u].x, cur[u].y, cur[u].z, cur[u].w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    double t = (double)q_lds[c * 32 + u * 4 + e] - (double)xv[e];
                    double t2 = t * t;
                    s = s + t2;
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) cur[u] = nxt[u];
        }
        j = n32 << 5;
    }
    for (; j < d; ++j) {
        double t = (double)q_lds[j] - (double)x[j];
        double t2 = t * t;
        s = s + t2;
    }
    return (float)s;
}

// Bounds for bfloat16 tiles.  With x~ the bfloat16 rounding of the stored
// FP32 row x, ||x_h - x~_h|| <= delta = u_b ||x|| (plus a subnormal term), so
// by the triangle inequality a certified bracket [s_lo, s_hi] of
// ||q_h - x~_h||^2 gives one of ||q_h - x_h||^2.  The factors cover the FP32
// square root and square.
__device__ inline float bf_head_lower(float s_lo, float delta)
{
    const float r = fmaxf(__builtin_sqrtf(fmaxf(s_lo, 0.f)) * (1.f - 1e-6f) - delta, 0.f);
    return r * r * (1.f - 1e-6f);
}
__device__ inline float bf_head_upper(float s_hi, float delta)
{
    const float r = __builtin_sqrtf(fmaxf(s_hi, 0.f)) * (1.f + 1e-6f) + delta;
    return r * r * (1.f + 1e-6f);
}

// Error model of a computed stored-frame distance Dt of a query with absolute
// margin A (dot-product form): the exact value lies in
// [(Dt - A)(1 - c_final), (Dt + A)(1 + c_final)].  A distance computed from
// bfloat16 rows (dl > 0, dl >= u_b max ||x||) is to the rounded row; the
// triangle inequality widens the bracket by dl on the square root.
__device__ inline float dist_upper(float Dt, float A, const Margins &mg, float dl = 0.f)
{
    const float u = (Dt + A) * (1.f + mg.c_final) * (1.f + 1e-6f);
    return dl == 0.f ? u : bf_head_upper(u, dl);
}
__device__ inline float dist_lower(float Dt, float A, const Margins &mg, float dl = 0.f)
{
    const float l = (Dt - A) * (1.f - mg.c_final);
    return dl == 0.f ? l : bf_head_lower(l, dl);
}

// Pruning threshold tau^2 from the k-th best computed distance Dk: with
// E = e_q + e_max (transform error) and rho the conditioning of the FP32
// transform, tau = E + rho (sqrt(upper(Dk)) + E).  A candidate whose lower
// bound exceeds tau^2 has a canonical distance above that of k committed
// candidates.  Slack covers the FP32 evaluation of the formula itself.
__device__ inline float prune_threshold(float Dk, float E, float A, const Margins &mg, float dl = 0.f)
{
    if (!(Dk < INFINITY)) return INFINITY;
    float r = __builtin_sqrtf(dist_upper(Dk, A, mg, dl));
    float tau = E + mg.rho * (r + E);
    return tau * tau * (1.f + 1e-6f);
}

__device__ inline uint64_t make_key(float dist, int32_t id)
{
    return ((uint64_t)__float_as_uint(dist) << 32) | (uint32_t)id;
}
__device__ inline float key_dist(uint64_t k) { return __uint_as_float((uint32_t)(k >> 32)); }
__device__ inline int32_t key_id(uint64_t k) { return (int32_t)(uint32_t)(k & 0xffffffffu); }

__device__ inline void atomic_min_nonneg(float *addr, float v)
{
    atomicMin(reinterpret_cast<int *>(addr), __float_as_int(v));
}

// Bitonic sort (ascending) of buf[0..n), n a power of two, by one wavefront.
// LDS traffic from one wavefront is processed in order; the wave barrier
// keeps the compiler from moving accesses across stages.
__device__ inline void wave_bitonic_sort(volatile uint64_t *buf, int n, int lane)
{
    for (int kk = 2; kk <= n; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int i = lane; i < n; i += 64) {
                int ixj = i ^ j;
                if (ixj > i) {
                    uint64_t a = buf[i], b = buf[ixj];
                    bool up = (i & kk) == 0;
                    if ((a > b) == up) {
                        buf[i] = b;
                        buf[ixj] = a;
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
}

// Bitonic sort of buf[0..n) by the whole workgroup (n a power of two).
__device__ inline void block_bitonic_sort(uint64_t *buf, int n)
{
    for (int kk = 2; kk <= n; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                int ixj = i ^ j;
                if (ixj > i) {
                    uint64_t a = buf[i], b = buf[ixj];
                    bool up = (i & kk) == 0;
                    if ((a > b) == up) {
                        buf[i] = b;
                        buf[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
}

__device__ inline uint16_t bf16_bits_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Blocks per work item of a list: bpi, raised for long lists so that a query
// group meets at most `cap` items per list (0 = no cap).  Fewer, longer items
// on long lists keep the number of per-item publications per query bounded.
__host__ __device__ inline int list_bpi(int bpi, int64_t nblk, int cap)
{
    if (cap <= 0) return bpi;
    const int64_t need = (nblk + cap - 1) / cap;
    return need > bpi ? (int)need : bpi;
}

__host__ __device__ inline int next_pow2(int v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// p-th smallest (1-based) of n non-negative floats V[0..n) by one wavefront:
// an MSB-first radix select over the IEEE bit patterns (monotone for
// non-negative values), 8 bits per round, with a 256-bin LDS histogram.
__device__ inline float wave_select_nonneg(const float *V, int n, int p, int *hist, int lane)
{
    uint32_t prefix = 0, mask = 0;
    int need = p;
    for (int shift = 24; shift >= 0; shift -= 8) {
        for (int i = lane; i < 256; i += 64) hist[i] = 0;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        for (int i = lane; i < n; i += 64) {
            const uint32_t u = __float_as_uint(V[i]);
            if ((u & mask) == prefix) atomicAdd(&hist[(u >> shift) & 255u], 1);
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        // lane owns bins 4*lane .. 4*lane+3
        int h[4], sum = 0;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            h[t] = hist[lane * 4 + t];
            sum += h[t];
        }
        int incl = sum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            int v = __shfl_up(incl, o, 64);
            if (lane >= o) incl += v;
        }
        const int excl = incl - sum;
        // the lane whose range holds the need-th element
        const bool mine = excl < need && need <= incl;
        const uint64_t bal = __ballot(mine);
        const int owner = (int)__ffsll((unsigned long long)bal) - 1;
        int digit = 0, before = 0;
        if (lane == owner) {
            int run = excl;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (run + h[t] >= need) {
                    digit = lane * 4 + t;
                    before = run;
                    break;
                }
                run += h[t];
            }
        }
        digit = __shfl(digit, owner, 64);
        before = __shfl(before, owner, 64);
        prefix |= (uint32_t)digit << shift;
        mask |= 255u << shift;
        need -= before;
        __builtin_amdgcn_wave_barrier();
    }
    return __uint_as_float(prefix);
}

// Exclusive prefix sum of one int per thread over the workgroup; returns the
// thread's offset and writes the total to *total (all threads).  Uses
// wave_tmp[4] in LDS.
__device__ inline int block_exclusive_scan(int v, int *wave_tmp, int *total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) wave_tmp[w] = incl;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) {
        int s = wave_tmp[i];
        if (i < w) base += s;
        tot += s;
    }
    *total = tot;
    __syncthreads();
    return base + incl - v;
}

}  // namespace pano
