// Device-side helpers shared by the search kernels: the canonical distance
// recipe, the certified pruning threshold, wave/block scans and bitonic sorts.
#pragma once

#include "internal.h"

namespace pano {

constexpr int NT = 256;         // threads per workgroup (4 wavefronts)
constexpr int MERGE_LDS_KEYS = 2048;  // entries the merge sorts in LDS
constexpr int IOFF_LDS = 1032;  // item offsets a scan workgroup keeps in LDS (lists up to 1024)
constexpr int GMAX = 16;        // max queries per scan work item
constexpr int SB_MAX = 512;     // per-wave sort buffer (entries)
constexpr int WALK_CHUNKS = 8;  // four-float chunks of a level the per-pair walk requests at once
constexpr uint64_t KEY_MAX = ~0ull;
constexpr int FLAG_OVERFLOW = 1;
constexpr int FLAG_NONFINITE = 2;  // host flag word only: the query has a non-finite value
constexpr int FLAG_BADID = 4;      // refine: a candidate id outside [-1, n)
constexpr int FLAG_SEEDED = 8;     // the seeding committed the query's first k buffer entries

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

constexpr int WAVE_PAIRS = 512;  // pair list of one wavefront in the per-wave scan

// LDS of one wavefront of the per-wave scan: byte offsets of its arrays.
struct WaveLds {
    int qid, thr, A, E, kc;  // [16] each: query ids, thresholds, margins, k-best counts
    int qtl;                 // [16][L] query tail norms
    int kb;                  // [16][k] the k best committed distances per query
    int sb;                  // [next_pow2(k + 64)] sort buffer
    int code, pS;            // [WAVE_PAIRS] pair codes (query << 8 | slot), partial distances
    int q1;                  // [16][w_1] the group's level-1 query slices
    int rq, a1;              // [16] level-1 head energy a_0^2 - a_1^2 and tail a_1 per query
    int bytes;
};
__host__ __device__ inline int wl_take(int &o, int b)
{
    const int r = o;
    o += (b + 15) & ~15;
    return r;
}
__host__ __device__ inline WaveLds wave_lds_layout(int L, int k, int w1)
{
    WaveLds w{};
    int o = 0;
    w.qid = wl_take(o, 64);
    w.thr = wl_take(o, 64);
    w.A = wl_take(o, 64);
    w.E = wl_take(o, 64);
    w.kc = wl_take(o, 64);
    w.qtl = wl_take(o, 16 * L * 4);
    w.kb = wl_take(o, 16 * k * 4);
    int p = 1;
    while (p < k + 64) p <<= 1;
    w.sb = wl_take(o, p * 4);
    w.code = wl_take(o, WAVE_PAIRS * 2);
    w.pS = wl_take(o, WAVE_PAIRS * 4);
    // (the pruned scan's per-item staging; none for the brute-force scan, whose
    // occupancy the extra bytes could cost a workgroup per compute unit)
    w.q1 = wl_take(o, 16 * w1 * 4);
    w.rq = wl_take(o, w1 > 0 ? 64 : 0);
    w.a1 = wl_take(o, w1 > 0 ? 64 : 0);
    w.bytes = o;
    return w;
}

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
    int walk2;         // 1: with four lanes per pair the walk reads two levels per step
    int bf16;          // 1: read level tiles in bfloat16 (certified margin, FP32 rescoring)
    float ub;          // bfloat16 unit roundoff 2^-8, rounded up (covers the stored-norm rounding)
    float bfdelta;     // bfloat16 scan: u_b max ||x|| (0 for the FP32 scan)
    float eps;
    float one_m_eps2;  // 2 (1 - eps)
    Margins mg;
    LevelGeom g;
    WaveLds wl;        // per-wave scan: LDS layout of one wavefront
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

// The canonical distance computed by a whole wavefront (all 64 lanes call it
// with the same arguments and get the same value).  The per-element terms are
// those of the canonical recipe, t = (double)q_j - (double)x_j and t * t, each
// rounded; only their summation order differs: lane partial sums, then a
// butterfly.  Any order of a sum of n non-negative terms lies within
// gamma(n - 1) S of the exact sum S, so the sequential sum lies within
// 2 gamma(n - 1) S / (1 - gamma(n - 1)) of this one; when both ends of that
// interval round to the same float, that float is the canonical value.
// Otherwise (an interval straddling a float rounding boundary, or a
// non-finite value) the sequential recipe itself is evaluated.
// The certified rounding of a parallel FP64 sum s of the d squared
// differences: any summation order of d non-negative terms lies within
// gamma_53(d - 1) s of the exact sum, so the sequential sum lies within
// del of s; when both ends of [s - del, s + del] round to the same float,
// that float is the canonical value, otherwise the sequential recipe runs
// (every lane computes it).
__device__ inline float canon_finish(double s, const float *q, const float *__restrict__ x, int d)
{
#pragma clang fp contract(off)
    const double gm = (double)d * 0x1p-53;
    const double gam = gm / (1.0 - gm);
    const double del = 2.0 * gam * s / (1.0 - gam) * 1.01 + 0x1p-1074;
    const float lo = (float)(s - del), hi = (float)(s + del);
    if (lo == hi) return lo;
    double r = 0.0;
    for (int j = 0; j < d; ++j) {
        const double t = (double)q[j] - (double)x[j];
        const double t2 = t * t;
        r = r + t2;
    }
    return (float)r;
}

__device__ inline float wave_canon_dist(const float *q, const float *__restrict__ x, int d, int lane)
{
#pragma clang fp contract(off)
    double s = 0.0;
    for (int j0 = 0; j0 < d; j0 += 64 * 8) {
        float xv[8], qv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int j = min(j0 + u * 64 + lane, d - 1);  // clamped: no branch around the loads
            xv[u] = x[j];
            qv[u] = q[j];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (j0 + u * 64 + lane < d) {
                const double t = (double)qv[u] - (double)xv[u];
                const double t2 = t * t;
                s = s + t2;
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s = s + __shfl_xor(s, o, 64);
    return canon_finish(s, q, x, d);
}

// Two rows at a time, for callers with several rows per wavefront: both
// rows' loads in flight together, sixteen per lane (a row of up to 1024
// values takes one round trip); each sum is certified by canon_finish.
__device__ inline void wave_canon_dist2(const float *q, const float *__restrict__ x0, const float *__restrict__ x1,
                                        int d, int lane, float &r0, float &r1)
{
#pragma clang fp contract(off)
    double s0 = 0.0, s1 = 0.0;
    for (int j0 = 0; j0 < d; j0 += 64 * 16) {
        float a[16], b[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int j = min(j0 + u * 64 + lane, d - 1);  // clamped: no branch around the loads
            a[u] = x0[j];
            b[u] = x1[j];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int j = j0 + u * 64 + lane;
            if (j < d) {
                const double qd = (double)q[j];
                const double t0 = qd - (double)a[u];
                const double t1 = qd - (double)b[u];
                const double p0 = t0 * t0, p1 = t1 * t1;
                s0 = s0 + p0;
                s1 = s1 + p1;
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        s0 = s0 + __shfl_xor(s0, o, 64);
        s1 = s1 + __shfl_xor(s1, o, 64);
    }
    r0 = canon_finish(s0, q, x0, d);
    r1 = canon_finish(s1, q, x1, d);
}

// Bounds for bfloat16 tiles.  With x~ the bfloat16 rounding of the stored
// FP32 row x, ||x_h - x~_h|| <= delta = u_b ||x|| (plus a subnormal term), so
// by the triangle inequality a certified bracket [s_lo, s_hi] of
// ||q_h - x~_h||^2 gives one of ||q_h - x_h||^2.  The factors cover the FP32
// square root and square.
// Certified upper bound on the norm of a stored row's head (the coordinates
// before the tail whose norm is bl) from its stored norm b0 and tail norm bl,
// each within a relative 2^-24 of the exact value: the slack 8u on both
// squares covers those and the FP32 products and difference (u = 2^-24).
// With bfloat16 tiles, ||x_h - x~_h|| <= u_b ||x_h|| (elementwise rounding),
// so the bracket of a head distance widens by u_b times this, not by u_b ||x||.
__device__ inline float head_norm_upper(float b0, float bl)
{
    const float h2 = b0 * b0 * (1.f + 4.8e-7f) - bl * bl * (1.f - 4.8e-7f);
    return __builtin_sqrtf(fmaxf(h2, 0.f)) * (1.f + 2.4e-7f);
}

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

// Cross-lane sums of 16-bit masks by one ballot per bit: scalar popcounts
// and lane-prefix counts, with no shuffle through LDS.
// The set bits of every lane's m, summed over the wavefront.
__device__ inline int wave_count16(uint32_t m)
{
    int n = 0;
#pragma unroll
    for (int b = 0; b < 16; ++b) n += __popcll(__ballot((m >> b) & 1u));
    return n;
}
// The same sum over the lanes below this one (an exclusive prefix); total
// receives the sum over all lanes.
__device__ inline int wave_prefix16(uint32_t m, int &total)
{
    int off = 0, n = 0;
#pragma unroll
    for (int b = 0; b < 16; ++b) {
        const uint64_t bb = __ballot((m >> b) & 1u);
        off += (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bb, 0u));
        n += __popcll(bb);
    }
    total = n;
    return off;
}
// The OR of every lane's m.
__device__ inline uint32_t wave_or16(uint32_t m)
{
    uint32_t r = 0;
#pragma unroll
    for (int b = 0; b < 16; ++b) r |= (__ballot((m >> b) & 1u) != 0ull ? 1u : 0u) << b;
    return r;
}

// The certified bounds of one (query, row) pair after a level, in the
// stored frame (Eq. 3 at eps = 1, Eq. 4 below it, with the margins of the
// soundness analysis): sh = the computed head distance over the levels read,
// a, b = the query's and the row's tail norms after the level, err = the
// head's absolute error bound, ct = the tail term's (c_tail (a + b)^2),
// ome2 = 2 (1 - eps).  The lower bound is what the scans compare with the
// pruning threshold; the upper bound (the Cauchy-Schwarz bound with the sum
// of the tails) holds after every level and for every eps.
// RELAX = false: eps = 1 known at compile time, the 2 (1 - eps) a b term is
// dropped (it is an exact +0 there, so the value is the same).
template <bool RELAX = true>
__device__ __forceinline__ float pair_lower(float sh, float a, float b, float err, float ct, float ome2)
{
    const float dt = a - b;
    return RELAX ? (sh + dt * dt + ome2 * a * b) - (err + ct) : (sh + dt * dt) - (err + ct);
}
__device__ __forceinline__ float pair_upper(float sh, float a, float b, float err, float ct)
{
    return sh + err + (a + b) * (a + b) + ct;
}
// bfloat16 rows: sh is the head distance to the rounded row, and delta
// (u_b times a bound on the head's norm) widens its square root.
template <bool RELAX = true>
__device__ __forceinline__ float pair_lower_bf(float sh, float a, float b, float err, float ct, float ome2,
                                               float delta)
{
    const float dt = a - b;
    return RELAX ? bf_head_lower(sh - err, delta) + dt * dt + ome2 * a * b - ct
                 : bf_head_lower(sh - err, delta) + dt * dt - ct;
}
__device__ __forceinline__ float pair_upper_bf(float sh, float a, float b, float err, float ct, float delta)
{
    return bf_head_upper(sh + err, delta) + (a + b) * (a + b) + ct;
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

// The same for non-negative floats (and +inf), compared as bit patterns.
__device__ inline void wave_bitonic_sort_f(volatile float *buf, int n, int lane)
{
    volatile uint32_t *u = reinterpret_cast<volatile uint32_t *>(buf);
    for (int kk = 2; kk <= n; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int i = lane; i < n; i += 64) {
                int ixj = i ^ j;
                if (ixj > i) {
                    uint32_t a = u[i], b = u[ixj];
                    bool up = (i & kk) == 0;
                    if ((a > b) == up) {
                        u[i] = b;
                        u[ixj] = a;
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

// The p-th smallest (1-based) of the valid values among u[0..VPL) of every
// lane of one wavefront (n valid in total, 1 <= p <= n), as float bit
// patterns of non-negative floats (their unsigned order is the float order):
// a bitwise radix select.  Bits common to every value come from the AND / OR
// of all values; each remaining bit costs one pass that counts, with ballots,
// the candidates still matching the prefix whose bit is 0.  It stops as soon
// as one candidate is left.  No LDS atomics: values that share their leading
// bits (the usual case) cost nothing extra.
template <int VPL>
__device__ inline uint32_t wave_select_core(const uint32_t (&u)[VPL], const bool (&ok)[VPL], int n, int p)
{
    uint32_t vor = 0u, vand = ~0u;
#pragma unroll
    for (int j = 0; j < VPL; ++j) {
        vor |= ok[j] ? u[j] : 0u;
        vand &= ok[j] ? u[j] : ~0u;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        vor |= (uint32_t)__shfl_xor((int)vor, o, 64);
        vand &= (uint32_t)__shfl_xor((int)vand, o, 64);
    }
    const uint32_t diff = vor ^ vand;
    if (diff == 0u) return vand;  // all values equal
    const int top = 31 - __builtin_clz(diff);
    uint32_t mask = top >= 31 ? 0u : ~((2u << top) - 1u);
    uint32_t prefix = vand & mask;
    int need = p, left = n;  // rank sought among the `left` candidates matching prefix
    for (int b = top; b >= 0; --b) {
        const uint32_t bit = 1u << b;
        int c0 = 0;
#pragma unroll
        for (int j = 0; j < VPL; ++j) c0 += __popcll(__ballot(ok[j] && (u[j] & (mask | bit)) == prefix));
        mask |= bit;
        if (need <= c0) {
            left = c0;
        } else {
            need -= c0;
            left -= c0;
            prefix |= bit;
        }
        if (left == 1) {
            // the one candidate left: its bits complete the prefix
            uint32_t found = 0u;
#pragma unroll
            for (int j = 0; j < VPL; ++j) {
                const uint64_t m = __ballot(ok[j] && (u[j] & mask) == prefix);
                if (m) found = (uint32_t)__shfl((int)u[j], (int)__builtin_ctzll(m), 64);
            }
            return found;
        }
    }
    return prefix;
}

// The p-th smallest of n <= 64 * VPL non-negative floats V[0..n) in LDS.
template <int VPL>
__device__ inline float wave_select_regs(const float *V, int n, int p, int lane)
{
    uint32_t u[VPL];
    bool ok[VPL];
#pragma unroll
    for (int j = 0; j < VPL; ++j) {
        const int i = j * 64 + lane;
        ok[j] = i < n;
        u[j] = ok[j] ? __float_as_uint(V[i]) : 0u;
    }
    return __uint_as_float(wave_select_core<VPL>(u, ok, n, p));
}

// The same for n <= 64 * VPL and p <= 64, first narrowing the candidates:
// the p-th smallest of the 64 per-lane minima bounds the answer from above
// (those p minima are p of the values), so only values at or below it are
// copied to C (LDS, n entries) and selected among.
template <int VPL>
__device__ inline float wave_select_small_p(const float *V, int n, int p, float *C, int lane)
{
    uint32_t u[VPL];
    bool ok[VPL];
    uint32_t mn = ~0u;
#pragma unroll
    for (int j = 0; j < VPL; ++j) {
        const int i = j * 64 + lane;
        ok[j] = i < n;
        u[j] = ok[j] ? __float_as_uint(V[i]) : 0u;
        mn = ok[j] ? min(mn, u[j]) : mn;
    }
    // every lane holds a value when n >= 64
    const uint32_t m1[1] = {mn};
    const bool o1[1] = {true};
    const uint32_t bound = wave_select_core<1>(m1, o1, 64, p);
    int cnt = 0;
#pragma unroll
    for (int j = 0; j < VPL; ++j) {
        const bool c = ok[j] && u[j] <= bound;
        const uint64_t bal = __ballot(c);
        if (c) C[cnt + __popcll(bal & ((1ull << lane) - 1ull))] = __uint_as_float(u[j]);
        cnt += __popcll(bal);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (cnt <= 64) return wave_select_regs<1>(C, cnt, p, lane);
    if (cnt <= 256) return wave_select_regs<4>(C, cnt, p, lane);
    return __uint_as_float(wave_select_core<VPL>(u, ok, n, p));
}

// The p-th smallest of any n >= 1 non-negative floats V[0..n) in LDS:
// values in registers up to 4096 (narrowed through C, n floats of LDS, when
// p <= 64), else an MSB-first radix select, 8 bits per round, with a 256-bin
// LDS histogram (hist[256]).
// NMAX: the largest n of the caller; only the register-resident forms that n
// can reach are compiled (their register needs grow with the values per
// lane), so a caller with few lists keeps a small register footprint.
template <int NMAX>
__device__ inline float wave_select_nonneg(const float *V, int n, int p, int *hist, float *C, int lane)
{
    if (n <= 256) return wave_select_regs<4>(V, n, p, lane);
    if (NMAX > 256 && n <= 1024)
        return p <= 64 ? wave_select_small_p<16>(V, n, p, C, lane) : wave_select_regs<16>(V, n, p, lane);
    if (NMAX > 1024 && n <= 4096)
        return p <= 64 ? wave_select_small_p<64>(V, n, p, C, lane) : wave_select_regs<64>(V, n, p, lane);
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

// The k smallest (k <= 128) of `total` distinct 64-bit keys (KEY_MAX pads
// empty slots), by one workgroup of NT threads:
// radix select of the k-th key over the 64 bits, 8 per pass, with a 256-bin
// histogram in LDS, then the keys up to it are gathered and sorted.
__device__ __forceinline__ void fallback_select_block(const uint64_t *__restrict__ keys, int64_t total, int k,
                                                      int64_t *__restrict__ out_ids, float *__restrict__ out_d)
{
    __shared__ int hist[256];
    __shared__ int sel[2];
    __shared__ int nsel;
    __shared__ uint64_t best[128];
    const int kk = (int)min<int64_t>(k, total);
    uint64_t prefix = 0, mask = 0;
    int rank = kk;
    for (int shift = 56; shift >= 0 && kk > 0; shift -= 8) {
        for (int i = threadIdx.x; i < 256; i += NT) hist[i] = 0;
        __syncthreads();
        for (int64_t i = threadIdx.x; i < total; i += NT) {
            const uint64_t v = keys[i];
            if ((v & mask) == prefix) atomicAdd(&hist[(int)((v >> shift) & 255u)], 1);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int acc = 0, dg = 0;
            while (dg < 255 && acc + hist[dg] < rank) acc += hist[dg++];
            sel[0] = dg;
            sel[1] = rank - acc;
        }
        __syncthreads();
        prefix |= (uint64_t)sel[0] << shift;
        mask |= (uint64_t)255u << shift;
        rank = sel[1];
        __syncthreads();
    }
    // prefix is now the kk-th smallest key.  Real keys are distinct, so fewer
    // than kk keys lie below it; it is added once unless it is the padding
    if (threadIdx.x == 0) nsel = 0;
    for (int i = threadIdx.x; i < 128; i += NT) best[i] = KEY_MAX;
    __syncthreads();
    if (kk > 0) {
        for (int64_t i = threadIdx.x; i < total; i += NT) {
            const uint64_t v = keys[i];
            if (v < prefix) {
                const int pos = atomicAdd(&nsel, 1);
                if (pos < 128) best[pos] = v;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0 && prefix != KEY_MAX && nsel < 128) best[nsel] = prefix;
    }
    __syncthreads();
    block_bitonic_sort(best, 128);
    for (int r = threadIdx.x; r < k; r += NT) {
        const uint64_t b = r < kk ? best[r] : KEY_MAX;
        if (b == KEY_MAX) {
            out_ids[r] = -1;
            out_d[r] = INFINITY;
        } else {
            out_ids[r] = key_id(b);
            out_d[r] = key_dist(b);
        }
    }
}

}  // namespace pano
