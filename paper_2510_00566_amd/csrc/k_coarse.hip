// Coarse probing: the nprobe nearest lists of every query, in the exact
// (D, list) order of the canonical distance (the IVF stage ahead of
// Algorithm 1: Section 6.1's index scans the nprobe nearest clusters of a
// query).
//
// One wavefront per query.  Approximate distances to every centroid come from
// the dense product S = q . c (chunked FP32 on the matrix cores), with a
// certified absolute error bound c_co (||q||^2 + ||c||^2).  A list is
// certainly in the probe set if its upper bound is below the (p+1)-th smallest
// lower bound; the uncertain lists of the band are rescored with the canonical
// recipe and ordered by (D, l).
//
// Up to 4096 lists, the bounds stay in registers (nlist / 64 per lane) and the
// band is ordered in a small LDS buffer, so a compute unit holds many
// queries at once.  A query whose band outgrows that buffer is marked and
// finished by the LDS instance, which keeps every bound in LDS and has no
// band limit; beyond 4096 lists that instance serves every query.
#include "search_common.h"

namespace pano {

// Band members the register-resident instance orders per wavefront.
constexpr int COARSE_BAND = 256;

// ||q||^2 in FP32: per lane its values in increasing column order (fused
// multiply-add), then a butterfly -- the order the bound c_co counts.  The row
// is loaded in rounds of eight loads per lane, all in flight together; with
// qrow, it is also copied there.
__device__ inline float coarse_qnorm(const float *__restrict__ qr, int d, int lane, float *qrow)
{
    float qq = 0.f;
    for (int j0 = 0; j0 < d; j0 += 512) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int j = j0 + u * 64 + lane;
            v[u] = qr[min(j, d - 1)];  // clamped: no branch around the load
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int j = j0 + u * 64 + lane;
            if (j < d) {
                if (qrow) qrow[j] = v[u];
                qq = __builtin_fmaf(v[u], v[u], qq);
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) qq += __shfl_xor(qq, o, 64);
    return qq;
}

// The certified interval [lo, up] of one list's squared distance from the
// product s = q . c, the norms and c_co (non-negative; widened by a relative
// 1.2e-7 for the rounding of the bound arithmetic itself).
__device__ inline void coarse_bounds(float qq, float cv, float sv, float c_co, float &lo, float &up)
{
    const float a = qq + cv - 2.f * sv;
    const float del = c_co * (qq + cv);
    lo = fmaxf(a - del, 0.f) * (1.0f - 1.2e-7f);
    up = fmaxf(a + del, 0.f) * (1.0f + 1.2e-7f);
}

__device__ inline int coarse_nprobe(const int32_t *nprobe_dev, int nprobe_all, int64_t qi, int nlist, int np_max)
{
    int p = nprobe_dev ? nprobe_dev[qi] : nprobe_all;
    p = p < 1 ? 1 : (p > nlist ? nlist : p);
    return p > np_max ? np_max : p;
}

__host__ __device__ inline size_t coarse_lds_per_wave(int nlist, int d)
{
    // keys [next_pow2(nlist)] (the band's sort pads to a power of two), LO,
    // UP, list ids [nlist], query row [d], select histogram [256]
    return (((size_t)next_pow2(nlist) * 8 + (size_t)nlist * 12 + (size_t)d * 4 + 1024 + 64) + 15) & ~(size_t)15;
}

// One query by one wavefront with every bound in LDS (base: its
// coarse_lds_per_wave bytes).
template <int NMAX>
__device__ void coarse_query_lds(int64_t qi, char *base, const float *__restrict__ S, const float *__restrict__ cn2,
                                 const float *__restrict__ q, const float *__restrict__ cent, int d, int nlist,
                                 const int32_t *__restrict__ nprobe_dev, int nprobe_all, float c_co, int np_max,
                                 int32_t *__restrict__ probes, int32_t *__restrict__ np_out,
                                 int32_t *__restrict__ list_cnt, float *__restrict__ qn2, int lane)
{
    uint64_t *keys = reinterpret_cast<uint64_t *>(base);            // [next_pow2(nlist)]
    float *LO = reinterpret_cast<float *>(keys + next_pow2(nlist));  // [nlist]
    float *UP = LO + nlist;                                          // [nlist]
    int32_t *lst = reinterpret_cast<int32_t *>(UP + nlist);          // [nlist]
    float *qrow = reinterpret_cast<float *>(lst + nlist);            // [d]
    int *hist = reinterpret_cast<int *>(qrow + d);                   // [256] (nlist > 4096)
    const int p = coarse_nprobe(nprobe_dev, nprobe_all, qi, nlist, np_max);
    const float qq = coarse_qnorm(q + qi * d, d, lane, qrow);
    if (qn2 != nullptr && lane == 0) qn2[qi] = qq;
    for (int l0 = 0; l0 < nlist; l0 += 512) {
        float cv[8], sv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int l = l0 + u * 64 + lane;
            const int lc = min(l, nlist - 1);  // clamped: no branch around the loads
            cv[u] = cn2[lc];
            sv[u] = S[qi * nlist + lc];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int l = l0 + u * 64 + lane;
            if (l < nlist) coarse_bounds(qq, cv[u], sv[u], c_co, LO[l], UP[l]);
        }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    // (the key buffer, not in use yet, holds the selects' candidates)
    float *cand = reinterpret_cast<float *>(keys);
    const float Up = wave_select_nonneg<NMAX>(UP, nlist, p, hist, cand, lane);
    const float Lp1 = p < nlist ? wave_select_nonneg<NMAX>(LO, nlist, p + 1, hist, cand, lane) : INFINITY;
    // certain lists go to the output; uncertain band members are collected
    int ncert = 0, nunc = 0;
    for (int b0 = 0; b0 < nlist; b0 += 64) {
        const int l = b0 + lane;
        const bool inb = l < nlist && LO[l] <= Up;
        const bool cert = inb && UP[l] < Lp1;
        const bool unc = inb && !cert;
        const uint64_t bc = __ballot(cert), bu = __ballot(unc);
        const uint64_t below = (1ull << lane) - 1ull;
        if (cert) {
            const int pos = ncert + __popcll(bc & below);
            if (pos < p) {
                probes[qi * np_max + pos] = l;
                atomicAdd(&list_cnt[l], 1);  // queries per list, for the work lists
            }
        }
        if (unc) lst[nunc + __popcll(bu & below)] = l;
        ncert += __popcll(bc);
        nunc += __popcll(bu);
    }
    if (ncert > p) ncert = p;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const int need = p - ncert;
    if (need > 0) {
        const int PU = next_pow2(nunc);
        // one band member at a time, each by the whole wavefront
        for (int i = 0; i < nunc; ++i) {
            const int l = lst[i];
            const float dv = wave_canon_dist(qrow, cent + (int64_t)l * d, d, lane);
            if (lane == 0) keys[i] = make_key(dv, l);
        }
        for (int i = nunc + lane; i < PU; i += 64) keys[i] = KEY_MAX;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        wave_bitonic_sort(keys, PU, lane);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        for (int i = lane; i < need; i += 64) {
            const int l = key_id(keys[i]);
            probes[qi * np_max + ncert + i] = l;
            atomicAdd(&list_cnt[l], 1);
        }
    }
    for (int i = p + lane; i < np_max; i += 64) probes[qi * np_max + i] = -1;
    if (lane == 0) np_out[qi] = p;
}

// The LDS instance, one wavefront per query (any number of lists).
template <int NMAX>
__global__ __launch_bounds__(NT) void k_coarse_lds(const float *__restrict__ S, const float *__restrict__ cn2,
                                                   const float *__restrict__ q, const float *__restrict__ cent, int d,
                                                   int nlist, int64_t nq, const int32_t *__restrict__ nprobe_dev,
                                                   int nprobe_all, float c_co, int np_max, int32_t *__restrict__ probes,
                                                   int32_t *__restrict__ np_out, int32_t *__restrict__ list_cnt,
                                                   float *__restrict__ qn2)
{
    extern __shared__ char smc[];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t qi = (int64_t)blockIdx.x * (blockDim.x >> 6) + w;
    if (qi >= nq) return;
    coarse_query_lds<NMAX>(qi, smc + coarse_lds_per_wave(nlist, d) * w, S, cn2, q, cent, d, nlist, nprobe_dev,
                           nprobe_all, c_co, np_max, probes, np_out, list_cnt, qn2, lane);
}

// The queries the register-resident instance left (np_out < 0), by the LDS
// instance: one wavefront per workgroup walks the flags 64 at a time.
template <int NMAX>
__global__ __launch_bounds__(64) void k_coarse_finish(const float *__restrict__ S, const float *__restrict__ cn2,
                                                      const float *__restrict__ q, const float *__restrict__ cent,
                                                      int d, int nlist, int64_t nq,
                                                      const int32_t *__restrict__ nprobe_dev, int nprobe_all,
                                                      float c_co, int np_max, int32_t *__restrict__ probes,
                                                      int32_t *__restrict__ np_out, int32_t *__restrict__ list_cnt,
                                                      float *__restrict__ qn2)
{
    extern __shared__ char smc[];
    const int lane = threadIdx.x;
    for (int64_t b = (int64_t)blockIdx.x * 64; b < nq; b += (int64_t)gridDim.x * 64) {
        const bool left = b + lane < nq && np_out[b + lane] < 0;
        uint64_t m = __ballot(left);
        while (m) {
            const int i = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            coarse_query_lds<NMAX>(b + i, smc, S, cn2, q, cent, d, nlist, nprobe_dev, nprobe_all, c_co, np_max,
                                   probes, np_out, list_cnt, qn2, lane);
        }
    }
}

// The p-th smallest (1-based, p <= 64 * VPL) of the values u[0..VPL) of every
// lane (float bit patterns of non-negative floats, or all-ones), by bits from
// the most significant one in which the values differ: each bit counts, per
// lane and then over the wavefront, the values that match the prefix found so
// far with this bit 0, and takes 0 or 1 accordingly; once a single value
// matches the prefix, that value is the answer.  Counts stay in vector
// registers, so the values are the only large live set.
template <int VPL>
__device__ inline uint32_t coarse_kth(const uint32_t (&u)[VPL], int p)
{
    uint32_t vor = 0u, vand = ~0u;
#pragma unroll
    for (int j = 0; j < VPL; ++j) {
        vor |= u[j];
        vand &= u[j];
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
    int need = p, left = 64 * VPL;
    for (int b = top; b >= 0; --b) {
        const uint32_t m2 = mask | (1u << b);
        int c = 0;
#pragma unroll
        for (int j = 0; j < VPL; ++j) c += (u[j] & m2) == prefix;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
        mask = m2;
        if (need <= c) {
            left = c;
        } else {
            need -= c;
            left -= c;
            prefix |= 1u << b;
        }
        if (left == 1) {
            uint32_t f = 0u;
#pragma unroll
            for (int j = 0; j < VPL; ++j) f = (u[j] & mask) == prefix ? u[j] : f;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) f = max(f, (uint32_t)__shfl_xor((int)f, o, 64));
            return f;
        }
    }
    return prefix;
}

// A raw buffer resource over n floats at p: loads past the end read 0
// instead of faulting, and each load needs one offset register per lane
// (the per-round offsets are scalars).
__device__ inline __amdgpu_buffer_rsrc_t coarse_rsrc(const float *p, int n)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(p), (short)0, n * 4, 0x00020000);
}

// One bound per list of a query into registers, v[u] for list u * 64 + lane
// (UPPER: the upper bound, else the lower), as float bit patterns; lists past
// nlist get all-ones.  rs: the query's row of products, rc: the centroid
// norms; vo: the lane's byte offset (4 * lane).  Loads go 16 per lane at a
// time.
template <int VPL, bool UPPER>
__device__ inline void coarse_bound_regs(__amdgpu_buffer_rsrc_t rs, __amdgpu_buffer_rsrc_t rc, int nlist, float qq,
                                         float c_co, int lane, int vo, uint32_t (&v)[VPL])
{
    constexpr int R = VPL < 16 ? VPL : 16;
#pragma unroll
    for (int u0 = 0; u0 < VPL; u0 += R) {
        float cv[R], sv[R];
#pragma unroll
        for (int u = 0; u < R; ++u) {
            cv[u] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rc, vo, (u0 + u) * 256, 0));
            sv[u] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, vo, (u0 + u) * 256, 0));
        }
#pragma unroll
        for (int u = 0; u < R; ++u) {
            float lo, up;
            coarse_bounds(qq, cv[u], sv[u], c_co, lo, up);
            v[u0 + u] = (u0 + u) * 64 + lane < nlist ? __float_as_uint(UPPER ? up : lo) : ~0u;
        }
    }
}

// The register-resident instance for nlist <= 64 * VPL: lane t holds the
// bounds of lists j * 64 + t (as float bit patterns; absent lists carry
// all-ones, above every bound, so the p-th smallest of all values is the p-th
// smallest bound).  The band goes to LDS; a query whose band exceeds
// COARSE_BAND while it still needs band members writes np_out = -1 and
// nothing else.
template <int VPL>
__global__ __launch_bounds__(NT) void k_coarse_regs(const float *__restrict__ S, const float *__restrict__ cn2,
                                                    const float *__restrict__ q, const float *__restrict__ cent, int d,
                                                    int nlist, int64_t nq, const int32_t *__restrict__ nprobe_dev,
                                                    int nprobe_all, float c_co, int np_max,
                                                    int32_t *__restrict__ probes, int32_t *__restrict__ np_out,
                                                    int32_t *__restrict__ list_cnt, float *__restrict__ qn2)
{
    __shared__ uint64_t band_s[NT / 64][COARSE_BAND];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t qi = (int64_t)blockIdx.x * (NT / 64) + w;
    if (qi >= nq) return;
    volatile uint64_t *band = band_s[w];
    const int p = coarse_nprobe(nprobe_dev, nprobe_all, qi, nlist, np_max);
    const float *qr = q + qi * d;
    const float qq = coarse_qnorm(qr, d, lane, nullptr);
    if (qn2 != nullptr && lane == 0) qn2[qi] = qq;
    // three passes over the query's products (the later ones from the
    // caches), so that one bound per list is live at a time: the upper
    // bounds give U_p, the lower bounds L_(p+1) and the lists in reach
    // (lo <= U_p), the upper bounds again the certain ones (up < L_(p+1));
    // membership is kept as per-lane bit masks (bit u: list u * 64 + lane)
    uint32_t v[VPL];
    // (each pass's offset depends on the previous select's result, which is
    // non-negative, so its sign bit is 0: the loads cannot be issued ahead
    // of the select, which would hold all three passes in registers)
    const __amdgpu_buffer_rsrc_t rs = coarse_rsrc(S + qi * nlist, nlist), rc = coarse_rsrc(cn2, nlist);
    int vo = lane * 4;
    coarse_bound_regs<VPL, true>(rs, rc, nlist, qq, c_co, lane, vo, v);
    const float Up = __uint_as_float(coarse_kth<VPL>(v, p));
    vo += (int)(__float_as_uint(Up) >> 31);
    coarse_bound_regs<VPL, false>(rs, rc, nlist, qq, c_co, lane, vo, v);
    const float Lp1 = p < nlist ? __uint_as_float(coarse_kth<VPL>(v, p + 1)) : INFINITY;
    uint64_t inbm = 0;
#pragma unroll
    for (int u = 0; u < VPL; ++u) inbm |= (uint64_t)(__uint_as_float(v[u]) <= Up) << u;  // all-ones (NaN): false
    vo += (int)(__float_as_uint(Lp1) >> 31);
    coarse_bound_regs<VPL, true>(rs, rc, nlist, qq, c_co, lane, vo, v);
    uint64_t certm = 0;
#pragma unroll
    for (int u = 0; u < VPL; ++u) certm |= (uint64_t)(__uint_as_float(v[u]) < Lp1) << u;
    certm &= inbm;
    uint64_t uncm = inbm & ~certm;
    // the counts first: a band that outgrows the buffer leaves the whole
    // query to the LDS instance before anything is written
    int ncert = __popcll(certm), nunc = __popcll(uncm);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        ncert += __shfl_xor(ncert, o, 64);
        nunc += __shfl_xor(nunc, o, 64);
    }
    const int need = p - (ncert < p ? ncert : p);
    if (need > 0 && nunc > COARSE_BAND) {
        if (lane == 0) np_out[qi] = -1;
        return;
    }
    if (need == 0) uncm = 0;
    const uint64_t below = (1ull << lane) - 1ull;
    int nc = 0, nb = 0;
    for (int u = 0; u < VPL; ++u) {
        const int l = u * 64 + lane;
        const bool cert = (certm >> u) & 1ull, unc = (uncm >> u) & 1ull;
        const uint64_t bc = __ballot(cert), bu = __ballot(unc);
        if (cert) {
            const int pos = nc + __popcll(bc & below);
            if (pos < p) {
                probes[qi * np_max + pos] = l;
                atomicAdd(&list_cnt[l], 1);  // queries per list, for the work lists
            }
        }
        if (unc) band[nb + __popcll(bu & below)] = (uint64_t)l;
        nc += __popcll(bc);
        nb += __popcll(bu);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (need > 0) {
        const int first = p - need;
        const int PU = next_pow2(nb);
        // one band member at a time, each by the whole wavefront; its slot
        // then takes its (D, l) key
        for (int i = 0; i < nb; ++i) {
            const int l = (int)band[i];
            const float dv = wave_canon_dist(qr, cent + (int64_t)l * d, d, lane);
            __builtin_amdgcn_wave_barrier();
            if (lane == 0) band[i] = make_key(dv, l);
        }
        for (int i = nb + lane; i < PU; i += 64) band[i] = KEY_MAX;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        wave_bitonic_sort(band, PU, lane);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        for (int i = lane; i < need; i += 64) {
            const int l = key_id(band[i]);
            probes[qi * np_max + first + i] = l;
            atomicAdd(&list_cnt[l], 1);
        }
    }
    for (int i = p + lane; i < np_max; i += 64) probes[qi * np_max + i] = -1;
    if (lane == 0) np_out[qi] = p;
}

__global__ void k_single_list(int64_t nq, int np_max, int32_t *__restrict__ probes, int32_t *__restrict__ np_out,
                              int32_t *__restrict__ list_cnt)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    atomicAdd(&list_cnt[0], 1);
    probes[i * np_max] = 0;
    for (int r = 1; r < np_max; ++r) probes[i * np_max + r] = -1;
    np_out[i] = 1;
}

float coarse_error_bound(int d)
{
    const double u_ = std::ldexp(1.0, -24);
    auto gam = [&](double nn) { return nn * u_ / (1.0 - nn * u_); };
    return (float)((gam(d / 64.0 + 8) + gam(2.0 * (32.0 + (d + 31) / 32 + 2)) + 4 * u_) * 1.1);
}

typedef void (*CoarseKernel)(const float *, const float *, const float *, const float *, int, int, int64_t,
                             const int32_t *, int, float, int, int32_t *, int32_t *, int32_t *, float *);

CoarsePlan coarse_prepare(int nlist, int d)
{
    CoarsePlan cp;
    cp.nlist = nlist;
    cp.d = d;
    cp.c_co = coarse_error_bound(d);
    if (nlist <= 1) return cp;
    cp.lds_wave = coarse_lds_per_wave(nlist, d);
    PANO_REQUIRE(cp.lds_wave <= 160 * 1024, "nlist too large for the coarse step");
    if (nlist <= 4096) {
        CoarseKernel fin = nlist <= 256 ? k_coarse_finish<256> : (nlist <= 1024 ? k_coarse_finish<1024> : k_coarse_finish<4096>);
        PANO_HIP(hipFuncSetAttribute((const void *)fin, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cp.lds_wave));
        cp.finish = (const void *)fin;
        cp.regs = (const void *)(nlist <= 256 ? k_coarse_regs<4> : (nlist <= 1024 ? k_coarse_regs<16> : k_coarse_regs<64>));
    } else {
        cp.wpb = (int)std::max<size_t>(1, std::min<size_t>(4, (64 * 1024) / cp.lds_wave));
        CoarseKernel k = k_coarse_lds<(1 << 30)>;
        PANO_HIP(hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)(cp.lds_wave * cp.wpb)));
        cp.lds = (const void *)k;
    }
    return cp;
}

void coarse_enqueue(const CoarsePlan &cp, const float *S, const float *cn2, const float *q, const float *cent, int64_t nq,
                    const int32_t *nprobe_dev, int nprobe_all, int np_max, int32_t *probes, int32_t *npq,
                    int32_t *list_cnt, float *qn2, hipStream_t s)
{
    if (nq == 0) return;
    const int nlist = cp.nlist, d = cp.d;
    if (nlist <= 1) {
        hipLaunchKernelGGL(k_single_list, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, s, nq, np_max, probes, npq,
                           list_cnt);
        PANO_HIP(hipGetLastError());
        return;
    }
    if (cp.regs) {
        hipLaunchKernelGGL((CoarseKernel)cp.regs, dim3((unsigned)((nq + 3) / 4)), dim3(NT), 0, s, S, cn2, q, cent, d,
                           nlist, nq, nprobe_dev, nprobe_all, cp.c_co, np_max, probes, npq, list_cnt, qn2);
        PANO_HIP(hipGetLastError());
        const unsigned g = (unsigned)std::min<int64_t>(256, (nq + 63) / 64);
        hipLaunchKernelGGL((CoarseKernel)cp.finish, dim3(g), dim3(64), cp.lds_wave, s, S, cn2, q, cent, d, nlist, nq,
                           nprobe_dev, nprobe_all, cp.c_co, np_max, probes, npq, list_cnt, qn2);
    } else {
        hipLaunchKernelGGL((CoarseKernel)cp.lds, dim3((unsigned)((nq + cp.wpb - 1) / cp.wpb)), dim3(64 * cp.wpb),
                           cp.lds_wave * cp.wpb, s, S, cn2, q, cent, d, nlist, nq, nprobe_dev, nprobe_all, cp.c_co,
                           np_max, probes, npq, list_cnt, qn2);
    }
    PANO_HIP(hipGetLastError());
}

void launch_coarse_probes(const float *S, const float *cn2, const float *q, const float *cent, int d, int nlist,
                          int64_t nq, const int32_t *nprobe_dev, int nprobe_all, int np_max, int32_t *probes,
                          int32_t *npq, int32_t *list_cnt, float *qn2, hipStream_t s)
{
    coarse_enqueue(coarse_prepare(nlist, d), S, cn2, q, cent, nq, nprobe_dev, nprobe_all, np_max, probes, npq,
                   list_cnt, qn2, s);
}

}  // namespace pano
