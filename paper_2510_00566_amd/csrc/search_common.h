// Device-side helpers shared by the search kernels: the canonical distance
// recipe, the certified pruning threshold, wave/block scans and bitonic sorts.
#pragma once

#include "internal.h"

namespace pano {

constexpr int NT = 256;         // threads per workgroup (4 wavefronts)
constexpr int GMAX = 16;        // max queries per scan work item
constexpr int SB_MAX = 512;     // per-wave sort buffer (entries)
constexpr uint64_t KEY_MAX = ~0ull;
constexpr int FLAG_OVERFLOW = 1;

// Scalars of one search, passed by value.
struct SearchConsts {
    int k;
    int kc;            // local top-k capacity per query (power of two >= k)
    int G;             // queries per work item
    int bpi;           // blocks per work item
    int capq;          // per-query result buffer capacity
    int nlist;
    int ceil8;         // ceil(nlist / 8)
    int prune;         // 1 = pruned scan, 0 = brute force
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

// Pruning threshold tau^2 from the k-th best computed distance Dk (see the
// error model: tau = E + rho (sqrt(Dk (1 + c_final)) + E)), with slack for
// the FP32 evaluation of this formula itself.
__device__ inline float prune_threshold(float Dk, float E, const Margins &mg)
{
    if (!(Dk < INFINITY)) return INFINITY;
    float r = __builtin_sqrtf(Dk * (1.f + mg.c_final));
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

__host__ __device__ inline int next_pow2(int v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
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
