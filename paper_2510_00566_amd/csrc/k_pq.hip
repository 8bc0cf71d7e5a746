// The IVFPQ form of the pruned scan for gfx950 (Section 4.2 spectrum shaping,
// Section 6.2 the PQ scan): PQ training and encoding, the sub-quantizer-major
// block layout, and the search: coarse probing, the query in the shaped
// frame, per-query look-up tables in LDS and a level-by-level scan whose
// candidates are dropped once the bound of Eq. 3/4 (with the table partial
// sums as head term) exceeds the running k-th distance.
//
// Distances: a table entry is float32 of the sequential FP64 sum over its
// sub-vector of (y_j - c_j)^2, y the query in the shaped frame (a sequential
// FP64 product); the canonical distance of a candidate is float32 of the
// sequential FP64 sum of its M entries.  The scan sums entries in FP32 (the
// same order) with certified margins, and every candidate that can reach the
// answer is rescored canonically before the top k are taken by
// (distance, id).
#include "internal.h"
#include "search_common.h"

#include <algorithm>
#include <cmath>

namespace pano {

constexpr int PQ_B = 256;      // slots per block (the scan encodes a slot in 8 bits)
constexpr int PQ_MAXM = 128;   // sub-quantizers: the table of M KB lives in LDS
constexpr int PQ_MAXL = 64;
constexpr int PQ_MAXNP = 1024; // probed lists per query
constexpr int PQ_LDS = 160 * 1024;

struct PqGeom {
    int M, dsub, L, d;
    int ml, mw;                // sub-quantizers per level; 32-bit words per slot and level (ml <= 4 mw)
    int sub_off[PQ_MAXL + 1];  // level cuts in sub-quantizers
    int cut[PQ_MAXL + 1];      // level cuts in coordinates
};

// ---------------------------------------------------------------- query in the shaped frame
// y_i = sum_j T_ij (q_j - mu_j), sequential in j in FP64, every product and
// sum rounded separately.  Tt is the transposed transform (Tt[j][i] =
// T[i][j]).  A workgroup takes 64 output coordinates (one per lane) for 64
// queries (16 per wavefront); the centred query values of a 64-coordinate
// chunk are staged in LDS.  A query with a non-finite y gets FLAG_NONFINITE.
__global__ __launch_bounds__(256) void k_pq_yseq(const float *__restrict__ q, int64_t nq, int d,
                                                 const double *__restrict__ Tt, const double *__restrict__ mu,
                                                 double *__restrict__ y, int32_t *__restrict__ qflags)
{
#pragma clang fp contract(off)
    __shared__ double qc[64][65];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane;
    const int64_t qb = (int64_t)blockIdx.y * 64;
    double acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.0;
    for (int j0 = 0; j0 < d; j0 += 64) {
        __syncthreads();
        for (int e = threadIdx.x; e < 64 * 64; e += 256) {
            const int qq = e >> 6, jj = e & 63;
            const int64_t qr = qb + qq;
            const int j = j0 + jj;
            qc[qq][jj] = (qr < nq && j < d) ? (double)q[qr * d + j] - mu[j] : 0.0;
        }
        __syncthreads();
        const int jn = min(64, d - j0);
        if (i < d) {
            for (int jj = 0; jj < jn; ++jj) {
                const double t = Tt[(size_t)(j0 + jj) * d + i];
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const double pr = t * qc[w * 16 + u][jj];
                    acc[u] = acc[u] + pr;
                }
            }
        }
    }
    if (i < d) {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int64_t qr = qb + w * 16 + u;
            if (qr < nq) {
                y[qr * d + i] = acc[u];
                if (!isfinite(acc[u])) atomicOr(&qflags[qr], FLAG_NONFINITE);
            }
        }
    }
}

// ---------------------------------------------------------------- training and encoding
// codes[r][m] = the codeword of sub-quantizer m nearest to row r's sub-vector
// (FP32 squared distance, ties to the smaller code).  Grid (rows / 256, M).
template <int DS>
__global__ __launch_bounds__(256) void k_pq_assign_sub(const float *__restrict__ Y, int64_t n, int ldy, int M,
                                                       const float *__restrict__ cb, uint8_t *__restrict__ codes)
{
    __shared__ float cw[256 * DS];
    const int m = blockIdx.y;
    for (int e = threadIdx.x; e < 256 * DS; e += 256) cw[e] = cb[(size_t)m * 256 * DS + e];
    __syncthreads();
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= n) return;
    float v[DS];
#pragma unroll
    for (int j = 0; j < DS; ++j) v[j] = Y[r * ldy + m * DS + j];
    float best = INFINITY;
    int bc = 0;
    for (int c = 0; c < 256; ++c) {
        float s = 0.f;
#pragma unroll
        for (int j = 0; j < DS; ++j) {
            const float t = v[j] - cw[c * DS + j];
            s = __builtin_fmaf(t, t, s);
        }
        if (s < best) {
            best = s;
            bc = c;
        }
    }
    codes[r * M + m] = (uint8_t)bc;
}

static void launch_assign_sub(const float *Y, int64_t n, int ldy, int M, int dsub, const float *cb, uint8_t *codes,
                              hipStream_t s)
{
    if (n == 0) return;
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)M);
    switch (dsub) {
    case 1: hipLaunchKernelGGL(k_pq_assign_sub<1>, grid, dim3(256), 0, s, Y, n, ldy, M, cb, codes); break;
    case 2: hipLaunchKernelGGL(k_pq_assign_sub<2>, grid, dim3(256), 0, s, Y, n, ldy, M, cb, codes); break;
    case 4: hipLaunchKernelGGL(k_pq_assign_sub<4>, grid, dim3(256), 0, s, Y, n, ldy, M, cb, codes); break;
    case 8: hipLaunchKernelGGL(k_pq_assign_sub<8>, grid, dim3(256), 0, s, Y, n, ldy, M, cb, codes); break;
    case 16: hipLaunchKernelGGL(k_pq_assign_sub<16>, grid, dim3(256), 0, s, Y, n, ldy, M, cb, codes); break;
    default: throw Error{PANO_EINVAL, "dsub must be 1, 2, 4, 8 or 16"};
    }
    PANO_HIP(hipGetLastError());
}

// Y[r] -= yc[assign[r]] for r < n (the residual of each row in the shaped
// frame, FP32).
__global__ __launch_bounds__(256) void k_pq_residual(float *__restrict__ Y, int64_t n, int d,
                                                     const int32_t *__restrict__ assign, const float *__restrict__ yc)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n * d) return;
    const int64_t r = t / d;
    const int j = (int)(t - r * d);
    Y[t] -= yc[(int64_t)assign[r] * d + j];
}

// One thread per slot: the sub-quantizer-major codes of its block, the norms
// of its reconstruction beyond levels 1..L-1 (FP64 sums of the codeword
// energies cwe [M][256]), its id.
__global__ __launch_bounds__(256) void k_pq_pack(PqGeom g, const uint8_t *__restrict__ codes_row,
                                                 const double *__restrict__ cwe, const int64_t *__restrict__ perm,
                                                 const int64_t *__restrict__ start, const int64_t *__restrict__ list_blk,
                                                 const int32_t *__restrict__ block_list, int64_t nblocks,
                                                 uint8_t *__restrict__ codes, float *__restrict__ tails,
                                                 int32_t *__restrict__ ids, int32_t *__restrict__ blk_cnt,
                                                 float *__restrict__ list_b0max, const double *__restrict__ yc,
                                                 const float *__restrict__ cbook, float *__restrict__ sx)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= nblocks * PQ_B) return;
    const int64_t b = t / PQ_B;
    const int sl = (int)(t % PQ_B);
    const int l = block_list[b];
    const int64_t pos = (b - list_blk[l]) * PQ_B + sl;
    const int64_t len = start[l + 1] - start[l];
    const int M = g.M, L = g.L;
    const int ml = g.ml, wb = 4 * g.mw;  // a slot's codes of one level: wb bytes (ml used)
    uint8_t *cb = codes + (size_t)b * L * PQ_B * wb + (size_t)sl * wb;
    float *tb = tails + (size_t)b * (L - 1) * PQ_B + sl;
    float *sbp = sx + (size_t)b * L * PQ_B + sl;
    if (sl == 0) blk_cnt[b] = (int32_t)min<int64_t>(PQ_B, len - (b - list_blk[l]) * PQ_B);
    if (pos >= len) {
        for (int lv = 0; lv < L; ++lv)
            for (int j = 0; j < wb; ++j) cb[(size_t)lv * PQ_B * wb + j] = 0;
        for (int lv = 0; lv + 1 < L; ++lv) tb[(size_t)lv * PQ_B] = 0.f;
        for (int lv = 0; lv < L; ++lv) sbp[(size_t)lv * PQ_B] = 0.f;
        ids[b * PQ_B + sl] = -1;
        return;
    }
    const int64_t row = perm[start[l] + pos];
    const uint8_t *cr = codes_row + row * M;
    double suffix = 0.0;
    for (int lv = L - 1; lv >= 1; --lv) {
        double e = 0.0;
        for (int m = g.sub_off[lv]; m < g.sub_off[lv + 1]; ++m) e += cwe[m * 256 + cr[m]];
        suffix += e;
        tb[(size_t)(lv - 1) * PQ_B] = (float)sqrt(suffix);
    }
    for (int m = g.sub_off[0]; m < g.sub_off[1]; ++m) suffix += cwe[m * 256 + cr[m]];
    // the largest reconstruction norm of the list, rounded up (non-negative
    // floats order as their bit patterns)
    atomicMax(reinterpret_cast<int *>(list_b0max + l), __float_as_int((float)sqrt(suffix) * (1.f + 0x1p-20f)));
    for (int lv = 0; lv < L; ++lv)
        for (int j = 0; j < wb; ++j) cb[(size_t)lv * PQ_B * wb + j] = j < ml ? cr[lv * ml + j] : 0;
    // per level: the sum over its codes of ||C||^2 + 2 <y_c, C> (FP64, one rounding)
    const int dsub = g.dsub;
    const double *yl = yc + (int64_t)l * g.d;
    for (int lv = 0; lv < L; ++lv) {
        double acc = 0.0;
        for (int m = lv * ml; m < (lv + 1) * ml; ++m) {
            const float *cw = cbook + ((size_t)m * 256 + cr[m]) * dsub;
            for (int j = 0; j < dsub; ++j) acc += (double)cw[j] * ((double)cw[j] + 2.0 * yl[m * dsub + j]);
        }
        sbp[(size_t)lv * PQ_B] = (float)acc;
    }
    (void)M;
    ids[b * PQ_B + sl] = (int32_t)row;
}

// ---------------------------------------------------------------- the scan
// A table entry splits as ||z_m - C||^2 = ||z_m||^2 + (||C||^2 + 2 <y_c, C>)
// - 2 <y_m, C> with z = y - y_c(list).  The middle term, summed over a
// level's sub-quantizers, depends on the stored vector alone and is kept per
// slot and level (sx); the last is the query's table, built once per query
// in LDS; the first is the residual's energy per level.  A level's
// contribution is zl + sx + the level's table look-ups.
struct PqScan {
    PqGeom g;
    int64_t nq;
    int k, np_max, cap, waves, nlr;  // nlr: probed lists whose constants share LDS in one round
    float eps;
    float g_part;  // relative error of an FP32 partial sum of table entries
    float g_adc;   // |canonical - FP32 sum| <= g_adc * FP32 sum
    const double *y;   // [nq][d] the queries in the shaped frame
    const double *yc;  // [nlist][d] the list centroids in the shaped frame
    const float *sx;   // [nblocks][L][256] per slot and level: sum of ||C||^2 + 2 <y_c, C> over its codes
    const float *ycn;  // [nlist] ||y_c(l)||
    const float *b0max;  // [nlist] the largest reconstruction norm of each list
    const float *codebooks;
    const int32_t *probes, *npq;
    const int64_t *list_blk;
    const int32_t *blk_cnt;
    const int32_t *block_list;
    const uint8_t *codes;
    const float *tails;
    const int32_t *ids;
    int32_t *qflags;
    int64_t *out_ids;
    float *out_d;
    unsigned long long *stats;  // [0] look-ups, [1] candidates, [2] overflowed queries, [3] bytes of codes and tails read
};

// Table entry (m, c) of the residual query z = y - y_c(list): float32 of the
// sequential FP64 sum over the sub-vector of (z_j - C[m][c][j])^2.
__device__ __forceinline__ float pq_entry(const double *__restrict__ yq, const double *__restrict__ yl,
                                          const float *__restrict__ cw, int m, int dsub)
{
#pragma clang fp contract(off)
    double s = 0.0;
    for (int j = 0; j < dsub; ++j) {
        const double z = yq[m * dsub + j] - yl[m * dsub + j];
        const double t = z - (double)cw[j];
        const double t2 = t * t;
        s = s + t2;
    }
    return (float)s;
}

// The canonical distance of the candidate in `slot` (its list's table
// entries recomputed, summed in FP64 in sub-quantizer order, then rounded).
__device__ __forceinline__ float pq_canonical(const PqScan &a, const double *yq, int64_t slot)
{
#pragma clang fp contract(off)
    const int M = a.g.M, dsub = a.g.dsub, d = a.g.d;
    const int64_t b = slot / PQ_B;
    const double *yl = a.yc + (int64_t)a.block_list[b] * d;
    const int ml = a.g.ml, wb = 4 * a.g.mw;
    const uint8_t *cs = a.codes + (size_t)b * a.g.L * PQ_B * wb + (size_t)(slot % PQ_B) * wb;
    double s = 0.0;
    for (int m = 0; m < M; ++m) {
        const int lv = m / ml;
        const int c = cs[(size_t)lv * PQ_B * wb + (m - lv * ml)];
        s = s + (double)pq_entry(yq, yl, a.codebooks + ((size_t)m * 256 + c) * dsub, m, dsub);
    }
    return (float)s;
}

// The same canonical distance computed by a whole wavefront (every lane gets
// it): lane t takes sub-quantizers t and t + 64 (their entries by the same
// recipe, four coordinates' loads issued together), then the entries are
// added in sub-quantizer order in FP64 through lane broadcasts.
__device__ __forceinline__ float pq_canonical_wave(const PqScan &a, const double *yq, int64_t slot, int lane)
{
#pragma clang fp contract(off)
    const int M = a.g.M, d = a.g.d, ml = a.g.ml, wb = 4 * a.g.mw, dsub = a.g.dsub;
    const int64_t b = slot / PQ_B;
    const double *yl = a.yc + (int64_t)a.block_list[b] * d;
    const uint8_t *cs = a.codes + (size_t)b * a.g.L * PQ_B * wb + (size_t)(slot % PQ_B) * wb;
    auto entry = [&](int m) -> float {
        if (m >= M) return 0.f;
        const int lv = m / ml;
        const int c = cs[(size_t)lv * PQ_B * wb + (m - lv * ml)];
        const float *cw = a.codebooks + ((size_t)m * 256 + c) * dsub;
        double s = 0.0;
        for (int j0 = 0; j0 < dsub; j0 += 4) {
            double yv[4], lv2[4];
            float cv[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int jj = min(j0 + j, dsub - 1);
                yv[j] = yq[m * dsub + jj];
                lv2[j] = yl[m * dsub + jj];
                cv[j] = cw[jj];
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (j0 + j < dsub) {
                    const double z = yv[j] - lv2[j];
                    const double t = z - (double)cv[j];
                    const double t2 = t * t;
                    s = s + t2;
                }
            }
        }
        return (float)s;
    };
    const float e0 = entry(lane);
    const float e1 = entry(lane + 64);
    double s = 0.0;
    for (int m = 0; m < M; ++m) s = s + (double)__shfl(m < 64 ? e0 : e1, m & 63, 64);
    return (float)s;
}

// A certified lower bound on the canonical distance from the FP32 partial sum
// p of the levels read and the tail norms a (query residual) and b
// (reconstruction): P + (a - b)^2 of Eq. 3 (plus 2 (1 - eps) a b, Eq. 4),
// with room for the rounding of p, a, b, the split table entries (dl, the
// list's bound on their summed error) and the final float32 rounding.
__device__ __forceinline__ float pq_lower_bound(float p, float a, float b, float eps, float g_part, float dl)
{
    const float dab = fabsf(a - b) - 0x1p-22f * (a + b);
    const float t = dab > 0.f ? dab * dab : 0.f;
    return (p * (1.f - g_part) - dl + t * (1.f - 0x1p-22f) + 2.f * (1.f - eps) * a * b) * (1.f - 0x1p-21f);
}

// Sort the wavefront's buffer (keys: upper bounds on the canonical
// distances) and keep the k smallest plus every entry that may still reach
// the answer: T, the k-th upper bound, bounds the query's canonical k-th
// distance from above, and an entry's lower bound is at least its upper bound
// minus 2 (g up + dm).  T goes to the shared threshold.  Returns the new count.
__device__ __noinline__ int pq_wave_trim(uint64_t *wb, int wc, int cap, int k, float g, float dm, unsigned *thr,
                                         int lane)
{
    for (int i = wc + lane; i < cap; i += 64) wb[i] = KEY_MAX;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    wave_bitonic_sort(wb, cap, lane);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (wc < k) return wc;
    const float T = key_dist(wb[k - 1]);
    int keep = k;
    for (int i0 = k; i0 < wc; i0 += 64) {
        const int i = i0 + lane;
        const float up = i < wc ? key_dist(wb[i]) : 0.f;
        const bool in = i < wc && up - 2.f * (g * up + dm) <= T;
        const uint64_t bm = __ballot(in);
        keep += __popcll(bm);
        if (bm != (i0 + 64 <= wc ? ~0ull : ((1ull << (wc - i0)) - 1ull))) break;
    }
    if (lane == 0) atomicMin(thr, __float_as_uint(T));
    return keep;
}

// One workgroup per query.  Its table (-2 <y_m, C_mc>, FP64 then rounded) is
// built once in LDS; the probed lists are taken nlr at a time: their
// residual energies per level, tail norms and error bounds go to LDS, then
// the wavefronts take quarter blocks (64 slots, one per lane) of those lists
// from a shared counter and run the level loop: a level's terms are summed in
// FP32, the bound is checked against the shared threshold, and a wavefront
// stops once no slot is alive.  Survivors that may reach the answer go to the
// wavefront's LDS buffer.  At the end every buffered entry that may reach
// the answer is rescored canonically and the k smallest (distance, id) keys
// are written.
// The query's table -2 <y_m, C_mc> (FP64 dots, rounded once) in LDS: each
// thread keeps one sub-vector y_m in registers and takes a run of codewords,
// four at a time with their loads issued together.
template <int DS>
__device__ void pq_query_table(float *__restrict__ lut, const double *__restrict__ yq,
                               const float *__restrict__ cb, int M, int tid, int nt)
{
    const int tpm = max(1, nt / M);  // threads per sub-quantizer
    const int per = (256 + tpm - 1) / tpm;
    for (int slot = tid; slot < M * tpm; slot += nt) {
        const int m = slot / tpm, c0 = (slot - m * tpm) * per, c1 = min(256, c0 + per);
        double y[DS];
#pragma unroll
        for (int j = 0; j < DS; ++j) y[j] = yq[m * DS + j];
        for (int c = c0; c < c1; c += 4) {
            float w[4][DS];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int cc = min(c + u, c1 - 1);
#pragma unroll
                for (int j = 0; j < DS; ++j) w[u][j] = cb[((size_t)m * 256 + cc) * DS + j];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                double dot = 0.0;
#pragma unroll
                for (int j = 0; j < DS; ++j) dot += y[j] * (double)w[u][j];
                if (c + u < c1) lut[m * 256 + c + u] = (float)(-2.0 * dot);
            }
        }
    }
}

// One level's look-ups of a slot: the codes of its ml sub-quantizers packed
// in MW 32-bit words, against the level's slice of the table.
template <int MW>
__device__ __forceinline__ float pq_level_sum(const float *__restrict__ lm, const uint32_t (&wv)[MW], int ml, float p)
{
#pragma unroll
    for (int u = 0; u < MW; ++u) {
        const uint32_t x = wv[u];
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (4 * u + e < ml) p += lm[(4 * u + e) * 256 + ((x >> (8 * e)) & 255u)];
    }
    return p;
}

template <bool PRUNE, int MW>
__global__ __launch_bounds__(1024) void k_pq_scan(PqScan a)
{
    extern __shared__ __align__(16) char sm[];
    const int M = a.g.M, L = a.g.L, d = a.g.d, dsub = a.g.dsub, nlr = a.nlr;
    float *lut = reinterpret_cast<float *>(sm);                                   // [M][256]
    uint64_t *wbuf = reinterpret_cast<uint64_t *>(lut + (size_t)M * 256);         // [waves][cap]
    double *e2 = reinterpret_cast<double *>(wbuf + (size_t)a.waves * a.cap);     // [nlr][L]
    int64_t *rb0 = reinterpret_cast<int64_t *>(e2 + (size_t)nlr * L);            // [nlr]
    float *zl = reinterpret_cast<float *>(rb0 + nlr);                            // [nlr][L]
    float *qa = zl + (size_t)nlr * L;                                            // [nlr][L]
    float *dl = qa + (size_t)nlr * L;                                            // [nlr]
    int32_t *rpref = reinterpret_cast<int32_t *>(dl + nlr);                     // [nlr + 1]
    int32_t *rnb = rpref + nlr + 1;                                              // [nlr]
    __shared__ unsigned thr, dmax;
    __shared__ float ynorm;
    __shared__ double ysq[16];
    __shared__ int task, ovf;
    __shared__ int wcount[16];
    const int64_t qi = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nt = blockDim.x;
    const int k = a.k;
    int64_t *oi = a.out_ids + qi * k;
    float *od = a.out_d + qi * k;
    if (a.qflags[qi] & FLAG_NONFINITE) {
        for (int r = tid; r < k; r += nt) {
            oi[r] = -1;
            od[r] = INFINITY;
        }
        return;
    }
    const int np = a.npq[qi];
    const double *yq = a.y + qi * d;
    if (tid == 0) {
        thr = 0x7f800000u;  // +inf
        dmax = 0u;
        ovf = 0;
    }
    {
        // the query's table, and ||y|| (for the error bound)
        switch (dsub) {
        case 1: pq_query_table<1>(lut, yq, a.codebooks, M, tid, nt); break;
        case 2: pq_query_table<2>(lut, yq, a.codebooks, M, tid, nt); break;
        case 4: pq_query_table<4>(lut, yq, a.codebooks, M, tid, nt); break;
        case 8: pq_query_table<8>(lut, yq, a.codebooks, M, tid, nt); break;
        default: pq_query_table<16>(lut, yq, a.codebooks, M, tid, nt); break;
        }
        double s = 0.0;
        for (int j = tid; j < d; j += nt) s += yq[j] * yq[j];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (lane == 0) ysq[w] = s;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int i = 0; i < (nt >> 6); ++i) t += ysq[i];
            ynorm = (float)(sqrt(t) * (1.0 + 1e-6));
        }
    }
    const int cap = a.cap;
    uint64_t *wb = wbuf + (size_t)w * cap;
    int wc = 0;
    unsigned long long looks = 0, cands = 0, bytes = 0;
    const float g_adc = a.g_adc;
    const int ml = a.g.ml;
    for (int r0 = 0; r0 < np; r0 += nlr) {
        const int nl = min(nlr, np - r0);
        __syncthreads();  // the previous round's constants are no longer read
        if (tid == 0) task = 0;
        // the residual z = y - y_c(list): its energy per level, in FP64
        for (int e = tid; e < nl * L; e += nt) {
            const int li = e / L, lv = e - li * L;
            const double *yl = a.yc + (int64_t)a.probes[qi * a.np_max + r0 + li] * d;
            double s = 0.0;
            for (int j = a.g.cut[lv]; j < a.g.cut[lv + 1]; ++j) {
                const double z = yq[j] - yl[j];
                s += z * z;
            }
            e2[e] = s;
            zl[e] = (float)s;
        }
        if (tid < nl) {
            const int l = a.probes[qi * a.np_max + r0 + tid];
            rb0[tid] = a.list_blk[l];
            rnb[tid] = (int)(a.list_blk[l + 1] - a.list_blk[l]);
        }
        __syncthreads();
        if (tid < nl) {
            // the residual's norm beyond level l, l = 1..L-1
            double acc = 0.0;
            for (int lv = L - 1; lv >= 1; --lv) {
                acc += e2[tid * L + lv];
                qa[tid * L + lv - 1] = (float)sqrt(acc);
            }
            acc += e2[tid * L];
            // the error of a distance summed from the split terms: each term is
            // an FP64 value rounded once and the FP32 sum runs over M + 2 L
            // terms; the terms' magnitudes sum to at most ||z||^2 + b^2 +
            // 2 (||y_c|| + ||y||) b (Cauchy-Schwarz), b the reconstruction norm
            const int l = a.probes[qi * a.np_max + r0 + tid];
            const double b = a.b0max[l];
            const double S = acc + b * b + 2.0 * ((double)a.ycn[l] + ynorm) * b;
            const float dlv = (float)((M + 2 * L + 8) * 1.1 * 0x1p-24 * S);
            dl[tid] = dlv;
            atomicMax(&dmax, __float_as_uint(dlv));
        }
        if (tid == 0) {
            // quarter blocks of the round's lists, as an exclusive prefix
            int run = 0;
            for (int li = 0; li < nl; ++li) {
                rpref[li] = run;
                run += 4 * rnb[li];
            }
            rpref[nl] = run;
        }
        __syncthreads();
        const int ntask = rpref[nl];
        for (;;) {
            int t = 0;
            if (lane == 0) t = atomicAdd(&task, 1);
            t = __shfl(t, 0, 64);
            if (t >= ntask) break;
            int li = 0;
            while (li + 1 < nl && rpref[li + 1] <= t) ++li;
            const int64_t b = rb0[li] + (t - rpref[li]) / 4;
            const int slot = ((t - rpref[li]) & 3) * 64 + lane;
            bool alive = a.ids[b * PQ_B + slot] >= 0;  // empty slots hold id -1
            cands += alive ? 1ull : 0ull;
            float p = 0.f;
            const float *qal = qa + li * L;
            const float *zll = zl + li * L;
            const float dlv = dl[li];
            // this slot's codes, level by level (MW words each), its level terms
            // and tail norms: those of CH levels are requested together
            constexpr int CH = MW == 1 ? 8 : 12 / MW;
            const uint32_t *cw = reinterpret_cast<const uint32_t *>(a.codes) + ((size_t)b * L * PQ_B + slot) * MW;
            const float *tb = a.tails + (size_t)b * (L - 1) * PQ_B + slot;
            const float *sb = a.sx + (size_t)b * L * PQ_B + slot;
            for (int l0 = 0; l0 < L; l0 += CH) {
                if (PRUNE && __ballot(alive) == 0) break;
                uint32_t cv[CH][MW];
                float tv[CH], sv[CH];
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    const int lv = l0 + c;
#pragma unroll
                    for (int u = 0; u < MW; ++u) cv[c][u] = lv < L ? cw[(size_t)lv * PQ_B * MW + u] : 0u;
                    sv[c] = lv < L ? sb[(size_t)lv * PQ_B] : 0.f;
                    tv[c] = (PRUNE && lv + 1 < L) ? tb[(size_t)lv * PQ_B] : 0.f;
                }
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    const int lv = l0 + c;
                    if (lv < L && alive) {
                        looks += (unsigned long long)ml;
                        p += zll[lv];
                        p += sv[c];
                        p = pq_level_sum<MW>(lut + (size_t)lv * ml * 256, cv[c], ml, p);
                        if (PRUNE && lv + 1 < L) {
                            const float T = __uint_as_float(__hip_atomic_load(&thr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
                            if (pq_lower_bound(p, qal[lv], tv[c], a.eps, a.g_part, dlv) > T) alive = false;
                        }
                    }
                }
                if (lane == 0) {
                    const int nlv = min(CH, L - l0);
                    bytes += (unsigned long long)(nlv * 64 * (4 * MW + 4) + (PRUNE ? 256 * min(nlv, L - 1 - l0) : 0));
                }
            }
            // commit a candidate that may reach the answer; its key is an
            // upper bound on its canonical distance
            const float T = __uint_as_float(__hip_atomic_load(&thr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
            const float up = p * (1.f + g_adc) + dlv;
            const float dm = __uint_as_float(__hip_atomic_load(&dmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
            const bool has = alive && up - 2.f * (g_adc * up + dm) <= T;
            const uint64_t bm = __ballot(has);
            if (bm == 0) continue;
            const int nn = __popcll(bm);
            if (wc + nn > cap) {
                wc = pq_wave_trim(wb, wc, cap, k, g_adc, dm, &thr, lane);
                if (wc + nn > cap) {
                    if (lane == 0) ovf = 1;
                    continue;
                }
            }
            if (has) wb[wc + __popcll(bm & ((1ull << lane) - 1ull))] = make_key(up, (int32_t)(b * PQ_B + slot));
            wc += nn;
        }
    }
    const float dmf = __uint_as_float(__hip_atomic_load(&dmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
    wc = pq_wave_trim(wb, wc, cap, k, g_adc, dmf, &thr, lane);
    if (lane == 0) wcount[w] = wc;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        looks += __shfl_xor(looks, o, 64);
        cands += __shfl_xor(cands, o, 64);
        bytes += __shfl_xor(bytes, o, 64);
    }
    if (lane == 0 && a.stats) {
        atomicAdd(&a.stats[0], looks);
        atomicAdd(&a.stats[1], cands);
        atomicAdd(&a.stats[3], bytes);
    }
    __syncthreads();
    if (ovf) {
        if (tid == 0) {
            atomicOr(&a.qflags[qi], FLAG_OVERFLOW);
            if (a.stats) atomicAdd(&a.stats[2], 1ull);
        }
        return;
    }
    // canonical distances of every entry that may reach the answer: each
    // wavefront rescores its own buffer, one entry at a time (the buffer is
    // sorted, so the entries that qualify come first)
    const float T = __uint_as_float(thr);
    const int tot = a.waves * cap;
    {
        const int n_w = wcount[w];
        for (int r = 0; r < cap; ++r) {
            uint64_t key = KEY_MAX;
            if (r < n_w) {
                const uint64_t e = wb[r];
                const float up = key_dist(e);
                if (up - 2.f * (g_adc * up + dmf) <= T) {
                    const int32_t slot = key_id(e);
                    key = make_key(pq_canonical_wave(a, yq, slot, lane), a.ids[slot]);
                }
            }
            __builtin_amdgcn_wave_barrier();
            if (lane == 0) wb[r] = key;
            __builtin_amdgcn_wave_barrier();
            if (r >= n_w) {
                for (int i = r + lane; i < cap; i += 64) wb[i] = KEY_MAX;
                break;
            }
        }
    }
    __syncthreads();
    block_bitonic_sort(wbuf, tot);
    for (int r = tid; r < k; r += nt) {
        const uint64_t e = wbuf[r];
        if (e == KEY_MAX) {
            oi[r] = -1;
            od[r] = INFINITY;
        } else {
            oi[r] = key_id(e);
            od[r] = key_dist(e);
        }
    }
}

// The exact answer of each query whose buffers overflowed (a band of equal
// or nearly equal distances wider than the buffers): one workgroup takes the
// canonical distance of every probed candidate into `keys` and selects the k
// smallest (distance, id) keys.  The flags are checked NT queries at a time;
// overflow is rare, so the queries that need it are handled one after another.
__global__ __launch_bounds__(NT) void k_pq_fallback(PqScan a, uint64_t *__restrict__ keys)
{
    __shared__ int32_t todo[NT];
    __shared__ int ntodo;
    const int d = a.g.d;
    for (int64_t q0 = 0; q0 < a.nq; q0 += NT) {
        if (threadIdx.x == 0) ntodo = 0;
        __syncthreads();
        {
            const int64_t qq = q0 + threadIdx.x;
            if (qq < a.nq && (a.qflags[qq] & FLAG_OVERFLOW) && !(a.qflags[qq] & FLAG_NONFINITE))
                todo[atomicAdd(&ntodo, 1)] = (int32_t)threadIdx.x;
        }
        __syncthreads();
        const int nt = ntodo;
        for (int jt = 0; jt < nt; ++jt) {
            const int64_t qi = q0 + todo[jt];
            const double *yq = a.y + qi * d;
            const int np = a.npq[qi];
            int64_t total = 0;
            for (int li = 0; li < np; ++li) {
                const int l = a.probes[qi * a.np_max + li];
                const int64_t nslots = (a.list_blk[l + 1] - a.list_blk[l]) * PQ_B;
                for (int64_t t = threadIdx.x; t < nslots; t += NT) {
                    const int64_t slot = a.list_blk[l] * PQ_B + t;
                    const int32_t id = a.ids[slot];
                    keys[total + t] = id >= 0 ? make_key(pq_canonical(a, yq, slot), id) : KEY_MAX;
                }
                total += nslots;
            }
            __syncthreads();
            fallback_select_block(keys, total, a.k, a.out_ids + qi * a.k, a.out_d + qi * a.k);
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------- host: build
static PqGeom geom_of(const pano_pq_index *ix)
{
    PqGeom g{};
    g.M = ix->M;
    g.dsub = ix->dsub;
    g.L = ix->L;
    g.d = ix->d;
    g.ml = ix->M / ix->L;
    g.mw = (g.ml + 3) / 4;
    for (int l = 0; l <= ix->L; ++l) {
        g.sub_off[l] = ix->sub_off[l];
        g.cut[l] = ix->cuts[l];
    }
    return g;
}

void run_pq_build(pano_ctx *ctx, pano_pq_index *ix, const pano_transform *tf, const float *x_dev,
                  const float *centroids_dev, const int32_t *assign_dev, int iters, int64_t sample, uint64_t seed,
                  hipStream_t s)
{
    const int64_t n = ix->n;
    const int d = ix->d, M = ix->M, dsub = ix->dsub, L = ix->L, nlist = ix->nlist;
    (void)ctx;
    // the transform: FP32 row-major for the encoding, FP64 transposed for the queries
    std::vector<float> T32((size_t)d * d), mu32(d);
    std::vector<double> Tt((size_t)d * d);
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            T32[(size_t)i * d + j] = (float)tf->T[(size_t)i * d + j];
            Tt[(size_t)j * d + i] = tf->T[(size_t)i * d + j];
        }
    for (int j = 0; j < d; ++j) mu32[j] = (float)tf->mu[j];
    DevMem T32d, mu32d, padcol_d;
    T32d.alloc(sizeof(float) * T32.size());
    mu32d.alloc(sizeof(float) * d);
    ix->Tt64.alloc(sizeof(double) * Tt.size());
    ix->mu64.alloc(sizeof(double) * d);
    std::vector<int32_t> padcol(d);
    for (int j = 0; j < d; ++j) padcol[j] = j;
    padcol_d.alloc(sizeof(int32_t) * d);
    PANO_HIP(hipMemcpyAsync(T32d.p, T32.data(), sizeof(float) * T32.size(), hipMemcpyHostToDevice, s));
    PANO_HIP(hipMemcpyAsync(mu32d.p, mu32.data(), sizeof(float) * d, hipMemcpyHostToDevice, s));
    PANO_HIP(hipMemcpyAsync(ix->Tt64.p, Tt.data(), sizeof(double) * Tt.size(), hipMemcpyHostToDevice, s));
    PANO_HIP(hipMemcpyAsync(ix->mu64.p, tf->mu.data(), sizeof(double) * d, hipMemcpyHostToDevice, s));
    PANO_HIP(hipMemcpyAsync(padcol_d.p, padcol.data(), sizeof(int32_t) * d, hipMemcpyHostToDevice, s));

    // the list centroids in the shaped frame: FP64, each coordinate a sequential
    // sum over j (the recipe of the queries' coordinates)
    std::vector<float> ch_cent((size_t)nlist * d);
    PANO_HIP(hipMemcpyAsync(ch_cent.data(), centroids_dev, sizeof(float) * ch_cent.size(), hipMemcpyDeviceToHost, s));
    std::vector<int32_t> asg(n);
    PANO_HIP(hipMemcpyAsync(asg.data(), assign_dev, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
    PANO_HIP(hipStreamSynchronize(s));
    for (int64_t i = 0; i < n; ++i) PANO_REQUIRE(asg[i] >= 0 && asg[i] < nlist, "assignment out of range");
    std::vector<double> yc((size_t)nlist * d);
    std::vector<float> yc32((size_t)nlist * d);
    parallel_for(nlist, 1, [&](int64_t l0, int64_t l1) {
#pragma clang fp contract(off)
        std::vector<double> cc(d);
        for (int64_t l = l0; l < l1; ++l) {
            for (int j = 0; j < d; ++j) cc[j] = (double)ch_cent[(size_t)l * d + j] - tf->mu[j];
            for (int i = 0; i < d; ++i) {
                double acc = 0.0;
                for (int j = 0; j < d; ++j) {
                    const double pr = tf->T[(size_t)i * d + j] * cc[j];
                    acc = acc + pr;
                }
                yc[(size_t)l * d + i] = acc;
                yc32[(size_t)l * d + i] = (float)acc;
            }
        }
    });
    ix->yc64.alloc(sizeof(double) * yc.size());
    PANO_HIP(hipMemcpyAsync(ix->yc64.p, yc.data(), sizeof(double) * yc.size(), hipMemcpyHostToDevice, s));
    {
        std::vector<float> ycn(nlist);
        for (int l = 0; l < nlist; ++l) {
            double acc = 0.0;
            for (int i = 0; i < d; ++i) acc += yc[(size_t)l * d + i] * yc[(size_t)l * d + i];
            ycn[l] = (float)(std::sqrt(acc) * (1.0 + 1e-6));
        }
        ix->ycn.alloc(sizeof(float) * nlist);
        PANO_HIP(hipMemcpyAsync(ix->ycn.p, ycn.data(), sizeof(float) * nlist, hipMemcpyHostToDevice, s));
        PANO_HIP(hipStreamSynchronize(s));
    }
    DevMem yc32d;
    yc32d.alloc(sizeof(float) * yc32.size());
    PANO_HIP(hipMemcpyAsync(yc32d.p, yc32.data(), sizeof(float) * yc32.size(), hipMemcpyHostToDevice, s));
    // training sample: residuals in the shaped frame
    const int64_t ns = std::min<int64_t>(n, std::max<int64_t>(256, sample));
    std::vector<int64_t> rows = seeded_sample(n, ns, seed ^ 0x2545F4914F6CDD1Dull);
    DevMem rows_d, xs, Ys, codes_s, cb;
    rows_d.alloc(sizeof(int64_t) * ns);
    xs.alloc(sizeof(float) * (size_t)ns * d);
    Ys.alloc(sizeof(float) * (size_t)ns * d);
    codes_s.alloc((size_t)ns * M);
    PANO_HIP(hipMemcpyAsync(rows_d.p, rows.data(), sizeof(int64_t) * ns, hipMemcpyHostToDevice, s));
    launch_gather_rows(x_dev, rows_d.as<int64_t>(), ns, d, xs.as<float>(), s);
    launch_transform(xs.as<float>(), ns, d, T32d.as<float>(), mu32d.as<float>(), padcol_d.as<int32_t>(),
                     Ys.as<float>(), d, s);
    std::vector<float> Yh((size_t)ns * d);
    PANO_HIP(hipMemcpyAsync(Yh.data(), Ys.p, sizeof(float) * Yh.size(), hipMemcpyDeviceToHost, s));
    PANO_HIP(hipStreamSynchronize(s));
    for (float v : Yh) PANO_REQUIRE(std::isfinite(v), "x has a non-finite value");
    for (int64_t r = 0; r < ns; ++r) {
        const float *c = yc32.data() + (size_t)asg[rows[r]] * d;
        for (int j = 0; j < d; ++j) Yh[(size_t)r * d + j] -= c[j];
    }
    PANO_HIP(hipMemcpyAsync(Ys.p, Yh.data(), sizeof(float) * Yh.size(), hipMemcpyHostToDevice, s));
    // initial codewords: 256 sample rows spread over the sample
    std::vector<float> C((size_t)M * 256 * dsub);
    for (int c = 0; c < 256; ++c) {
        const int64_t r = (int64_t)c * ns / 256;
        for (int m = 0; m < M; ++m)
            for (int j = 0; j < dsub; ++j)
                C[((size_t)m * 256 + c) * dsub + j] = Yh[(size_t)r * d + m * dsub + j];
    }
    cb.alloc(sizeof(float) * C.size());
    std::vector<uint8_t> ch((size_t)ns * M);
    for (int it = 0; it < iters; ++it) {
        PANO_HIP(hipMemcpyAsync(cb.p, C.data(), sizeof(float) * C.size(), hipMemcpyHostToDevice, s));
        launch_assign_sub(Ys.as<float>(), ns, d, M, dsub, cb.as<float>(), codes_s.as<uint8_t>(), s);
        PANO_HIP(hipMemcpyAsync(ch.data(), codes_s.p, ch.size(), hipMemcpyDeviceToHost, s));
        PANO_HIP(hipStreamSynchronize(s));
        // means in FP64 over the sample in row order; an empty cell keeps its codeword
        parallel_for(M, 1, [&](int64_t m0, int64_t m1) {
            std::vector<double> sum((size_t)256 * dsub);
            std::vector<int64_t> cnt(256);
            for (int64_t m = m0; m < m1; ++m) {
                std::fill(sum.begin(), sum.end(), 0.0);
                std::fill(cnt.begin(), cnt.end(), 0);
                for (int64_t r = 0; r < ns; ++r) {
                    const int c = ch[(size_t)r * M + m];
                    cnt[c]++;
                    for (int j = 0; j < dsub; ++j) sum[(size_t)c * dsub + j] += Yh[(size_t)r * d + m * dsub + j];
                }
                for (int c = 0; c < 256; ++c)
                    if (cnt[c] > 0)
                        for (int j = 0; j < dsub; ++j)
                            C[((size_t)m * 256 + c) * dsub + j] = (float)(sum[(size_t)c * dsub + j] / cnt[c]);
            }
        });
    }
    ix->codebooks.alloc(sizeof(float) * C.size());
    PANO_HIP(hipMemcpyAsync(ix->codebooks.p, C.data(), sizeof(float) * C.size(), hipMemcpyHostToDevice, s));

    // encode every row, in chunks
    ix->codes_row.alloc((size_t)n * M);
    {
        const int64_t chunk = std::min<int64_t>(n, std::max<int64_t>(4096, ((int64_t)1 << 28) / (4 * d)));
        DevMem Yc;
        Yc.alloc(sizeof(float) * (size_t)chunk * d);
        for (int64_t r0 = 0; r0 < n; r0 += chunk) {
            const int64_t rn = std::min(chunk, n - r0);
            launch_transform(x_dev + r0 * d, rn, d, T32d.as<float>(), mu32d.as<float>(), padcol_d.as<int32_t>(),
                             Yc.as<float>(), d, s);
            hipLaunchKernelGGL(k_pq_residual, dim3((unsigned)((rn * d + 255) / 256)), dim3(256), 0, s, Yc.as<float>(),
                               rn, d, assign_dev + r0, yc32d.as<float>());
            PANO_HIP(hipGetLastError());
            launch_assign_sub(Yc.as<float>(), rn, d, M, dsub, ix->codebooks.as<float>(),
                              ix->codes_row.as<uint8_t>() + r0 * M, s);
        }
        PANO_HIP(hipStreamSynchronize(s));
    }
    // codeword energies in FP64
    std::vector<double> cwe((size_t)M * 256);
    for (size_t e = 0; e < cwe.size(); ++e) {
        double acc = 0.0;
        for (int j = 0; j < dsub; ++j) acc += (double)C[e * dsub + j] * (double)C[e * dsub + j];
        cwe[e] = acc;
    }
    // lists: stable counting sort by assignment, blocks of 256 slots
    ix->list_len.assign(nlist, 0);
    for (int64_t i = 0; i < n; ++i) ix->list_len[asg[i]]++;
    std::vector<int64_t> start(nlist + 1, 0);
    for (int l = 0; l < nlist; ++l) start[l + 1] = start[l] + ix->list_len[l];
    std::vector<int64_t> perm(n);
    {
        std::vector<int64_t> fill(start.begin(), start.end() - 1);
        for (int64_t i = 0; i < n; ++i) perm[fill[asg[i]]++] = i;
    }
    ix->list_blk.assign(nlist + 1, 0);
    for (int l = 0; l < nlist; ++l) ix->list_blk[l + 1] = ix->list_blk[l] + (ix->list_len[l] + PQ_B - 1) / PQ_B;
    ix->nblocks = ix->list_blk[nlist];
    {
        std::vector<int64_t> nb(nlist);
        for (int l = 0; l < nlist; ++l) nb[l] = ix->list_blk[l + 1] - ix->list_blk[l];
        std::sort(nb.begin(), nb.end(), std::greater<int64_t>());
        ix->top_blk_prefix.assign(nlist + 1, 0);
        for (int l = 0; l < nlist; ++l) ix->top_blk_prefix[l + 1] = ix->top_blk_prefix[l] + nb[l];
    }
    PANO_REQUIRE(ix->nblocks * PQ_B < ((int64_t)1 << 31), "too many slots for 32-bit slot numbers");
    std::vector<int32_t> block_list(std::max<int64_t>(1, ix->nblocks));
    for (int l = 0; l < nlist; ++l)
        for (int64_t b = ix->list_blk[l]; b < ix->list_blk[l + 1]; ++b) block_list[b] = l;
    DevMem perm_d, start_d, cwe_d;
    DevMem &block_list_d = ix->block_list;
    perm_d.alloc(sizeof(int64_t) * n);
    start_d.alloc(sizeof(int64_t) * (nlist + 1));
    block_list_d.alloc(sizeof(int32_t) * block_list.size());
    cwe_d.alloc(sizeof(double) * cwe.size());
    ix->list_blk_d.alloc(sizeof(int64_t) * (nlist + 1));
    PANO_HIP(hipMemcpyAsync(perm_d.p, perm.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, s));
    PANO_HIP(hipMemcpyAsync(start_d.p, start.data(), sizeof(int64_t) * (nlist + 1), hipMemcpyHostToDevice, s));
    PANO_HIP(hipMemcpyAsync(block_list_d.p, block_list.data(), sizeof(int32_t) * block_list.size(),
                            hipMemcpyHostToDevice, s));
    PANO_HIP(hipMemcpyAsync(cwe_d.p, cwe.data(), sizeof(double) * cwe.size(), hipMemcpyHostToDevice, s));
    PANO_HIP(hipMemcpyAsync(ix->list_blk_d.p, ix->list_blk.data(), sizeof(int64_t) * (nlist + 1),
                            hipMemcpyHostToDevice, s));
    const size_t slots = (size_t)std::max<int64_t>(1, ix->nblocks) * PQ_B;
    ix->codes.alloc(slots * L * 4 * ((M / L + 3) / 4));
    ix->tails.alloc(sizeof(float) * slots * std::max(1, L - 1));
    ix->ids.alloc(sizeof(int32_t) * slots);
    ix->blk_cnt.alloc(sizeof(int32_t) * std::max<int64_t>(1, ix->nblocks));
    ix->b0max.alloc(sizeof(float) * nlist);
    ix->sx.alloc(sizeof(float) * slots * L);
    PANO_HIP(hipMemsetAsync(ix->b0max.p, 0, sizeof(float) * nlist, s));
    if (ix->nblocks > 0) {
        hipLaunchKernelGGL(k_pq_pack, dim3((unsigned)((ix->nblocks * PQ_B + 255) / 256)), dim3(256), 0, s, geom_of(ix),
                           ix->codes_row.as<uint8_t>(), cwe_d.as<double>(), perm_d.as<int64_t>(),
                           start_d.as<int64_t>(), ix->list_blk_d.as<int64_t>(), block_list_d.as<int32_t>(),
                           ix->nblocks, ix->codes.as<uint8_t>(), ix->tails.as<float>(), ix->ids.as<int32_t>(),
                           ix->blk_cnt.as<int32_t>(), ix->b0max.as<float>(), ix->yc64.as<double>(),
                           ix->codebooks.as<float>(), ix->sx.as<float>());
        PANO_HIP(hipGetLastError());
    }
    ix->cent.alloc(sizeof(float) * ((size_t)nlist * d + nlist));
    PANO_HIP(hipMemcpyAsync(ix->cent.p, centroids_dev, sizeof(float) * (size_t)nlist * d, hipMemcpyDeviceToDevice, s));
    launch_sqnorms(ix->cent.as<float>(), nlist, d, ix->cent.as<float>() + (size_t)nlist * d, s);
    PANO_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------- host: search
static size_t aup(size_t b) { return (b + 255) & ~(size_t)255; }

// consecutive 256-byte aligned sub-buffers of one allocation
struct PqCarver {
    char *base;
    size_t off = 0;
    explicit PqCarver(void *b) : base((char *)b) {}
    template <class T> T *take(size_t count)
    {
        T *p = reinterpret_cast<T *>(base + off);
        off += aup(sizeof(T) * std::max<size_t>(count, 1));
        return p;
    }
};

void run_pq_search(pano_ctx *ctx, pano_pq_index *ix, const float *q, int64_t nq, int k, const int32_t *nprobe_dev,
                   int nprobe_all, float eps, int64_t *ids, float *dists, uint32_t flags, hipStream_t s)
{
    const int d = ix->d, M = ix->M, L = ix->L, nlist = ix->nlist;
    PANO_REQUIRE(k >= 1 && k <= 128, "the PQ search supports 1 <= k <= 128");
    const int np_max = nprobe_dev ? (nprobe_all > 0 ? std::min(nprobe_all, nlist) : nlist) : std::min(nprobe_all, nlist);
    PANO_REQUIRE(np_max >= 1 && np_max <= PQ_MAXNP, "the PQ search probes at most 1024 lists per query");
    const bool brute = (flags & PANO_PQ_BRUTE) != 0;
    const bool want_stats = (flags & PANO_SEARCH_STATS) != 0;
    ctx->quiesce();
    // scan geometry: per-wave buffers of cap keys, then as many lists' tables
    // (with their tail norms) as fit
    int cap = 1;
    while (cap < k + 96) cap <<= 1;
    const size_t per_list = (size_t)L * 16 + 24;
    const size_t budget = (size_t)PQ_LDS - 2048 - 64 - (size_t)M * 256 * 4;
    int waves = 16;
    while (waves > 2 && (size_t)waves * cap * 8 + per_list > budget) waves >>= 1;
    PANO_REQUIRE((size_t)waves * cap * 8 + per_list <= budget, "k and M too large for the PQ scan's LDS");
    const int nlr = (int)std::min<size_t>({(budget - (size_t)waves * cap * 8) / per_list, (size_t)np_max, (size_t)128});
    const size_t scan_shm = (size_t)M * 256 * 4 + (size_t)waves * cap * 8 + (size_t)nlr * per_list + 64;
    // scratch
    const size_t nS = nlist > 1 ? aup(sizeof(float) * nq * nlist) : 256;
    const size_t nP = aup(sizeof(int32_t) * nq * np_max) + aup(sizeof(int32_t) * nq) + aup(sizeof(int32_t) * nlist) +
                      aup(sizeof(float) * nq) + aup(sizeof(int32_t) * nq) + aup(sizeof(unsigned long long) * 4);
    const size_t nY = aup(sizeof(double) * nq * d);
    const int64_t s_np = ix->top_blk_prefix[std::min<int64_t>(np_max, nlist)];
    const size_t nK = aup(sizeof(uint64_t) * std::max<int64_t>(1, s_np * PQ_B));
    ctx->scratch[5].ensure(nS);
    ctx->scratch[6].ensure(nP);
    ctx->scratch[7].ensure(nY);
    ctx->scratch[8].ensure(nK);
    float *S = ctx->scratch[5].as<float>();
    PqCarver cp(ctx->scratch[6].p);
    int32_t *probes = cp.take<int32_t>(nq * np_max);
    int32_t *npq = cp.take<int32_t>(nq);
    int32_t *list_cnt = cp.take<int32_t>(nlist);
    float *qn2 = cp.take<float>(nq);
    int32_t *qflags = cp.take<int32_t>(nq);
    unsigned long long *stats = cp.take<unsigned long long>(4);
    double *y = ctx->scratch[7].as<double>();
    uint64_t *keys = ctx->scratch[8].as<uint64_t>();
    hipStream_t ws = ctx->work_stream();
    PANO_HIP(hipEventRecord(ctx->ev_in, s));
    PANO_HIP(hipStreamWaitEvent(ws, ctx->ev_in, 0));
    PANO_HIP(hipMemsetAsync(list_cnt, 0, sizeof(int32_t) * nlist, ws));
    PANO_HIP(hipMemsetAsync(qflags, 0, sizeof(int32_t) * nq, ws));
    PANO_HIP(hipMemsetAsync(stats, 0, sizeof(unsigned long long) * 4, ws));
    if (nlist > 1) launch_gemm_nt(q, nq, d, ix->cent.as<float>(), nlist, S, ws);
    launch_coarse_probes(S, ix->cent.as<float>() + (size_t)nlist * d, q, ix->cent.as<float>(), d, nlist, nq, nprobe_dev,
                         nprobe_all, np_max, probes, npq, list_cnt, qn2, ws);
    hipLaunchKernelGGL(k_pq_yseq, dim3((unsigned)((d + 63) / 64), (unsigned)((nq + 63) / 64)), dim3(256), 0, ws, q, nq,
                       d, ix->Tt64.as<double>(), ix->mu64.as<double>(), y, qflags);
    PANO_HIP(hipGetLastError());
    PqScan a{};
    a.g = geom_of(ix);
    a.nq = nq;
    a.k = k;
    a.np_max = np_max;
    a.cap = cap;
    a.waves = waves;
    a.nlr = nlr;
    a.eps = eps;
    const double u = std::ldexp(1.0, -24);
    a.g_part = (float)(2.0 * (M + 2) * u);
    a.g_adc = (float)((4.0 * (M + 2) + 2.0) * u);
    a.y = y;
    a.yc = ix->yc64.as<double>();
    a.sx = ix->sx.as<float>();
    a.ycn = ix->ycn.as<float>();
    a.b0max = ix->b0max.as<float>();
    a.block_list = ix->block_list.as<int32_t>();
    a.codebooks = ix->codebooks.as<float>();
    a.probes = probes;
    a.npq = npq;
    a.list_blk = ix->list_blk_d.as<int64_t>();
    a.blk_cnt = ix->blk_cnt.as<int32_t>();
    a.codes = ix->codes.as<uint8_t>();
    a.tails = ix->tails.as<float>();
    a.ids = ix->ids.as<int32_t>();
    a.qflags = qflags;
    a.out_ids = ids;
    a.out_d = dists;
    a.stats = want_stats ? stats : nullptr;
    typedef void (*PqKern)(PqScan);
    const int mw = (M / L + 3) / 4;
    static const PqKern kp[4] = {k_pq_scan<true, 1>, k_pq_scan<true, 2>, k_pq_scan<true, 3>, k_pq_scan<true, 4>};
    static const PqKern kb[4] = {k_pq_scan<false, 1>, k_pq_scan<false, 2>, k_pq_scan<false, 3>, k_pq_scan<false, 4>};
    PANO_REQUIRE(mw >= 1 && mw <= 4, "at most 16 sub-quantizers per level");
    const PqKern kern = brute ? kb[mw - 1] : kp[mw - 1];
    PANO_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)scan_shm));
    if (want_stats) PANO_HIP(hipEventRecord(ctx->ev[1], ws));
    hipLaunchKernelGGL(kern, dim3((unsigned)nq), dim3(64 * waves), scan_shm, ws, a);
    PANO_HIP(hipGetLastError());
    if (want_stats) PANO_HIP(hipEventRecord(ctx->ev[2], ws));
    hipLaunchKernelGGL(k_pq_fallback, dim3(1), dim3(NT), 0, ws, a, keys);
    PANO_HIP(hipGetLastError());
    std::vector<int32_t> hf(nq);
    PANO_HIP(hipMemcpyAsync(hf.data(), qflags, sizeof(int32_t) * nq, hipMemcpyDeviceToHost, ws));
    unsigned long long hs[4] = {0, 0, 0, 0};
    if (want_stats) PANO_HIP(hipMemcpyAsync(hs, stats, sizeof(hs), hipMemcpyDeviceToHost, ws));
    PANO_HIP(hipEventRecord(ctx->ev_in, ws));
    PANO_HIP(hipStreamWaitEvent(s, ctx->ev_in, 0));
    PANO_HIP(hipStreamSynchronize(ws));
    for (int64_t i = 0; i < nq; ++i) PANO_REQUIRE(!(hf[i] & FLAG_NONFINITE), "a query has a non-finite value");
    if (want_stats) {
        float ms = 0.f;
        PANO_HIP(hipEventElapsedTime(&ms, ctx->ev[1], ctx->ev[2]));
        ix->last_ms_scan = ms;
        ix->last_stats[0] = (int64_t)hs[0];
        ix->last_stats[1] = (int64_t)hs[1] * M;
        ix->last_stats[2] = (int64_t)hs[2];
        ix->last_stats[3] = (int64_t)hs[1];
        ix->last_stats[4] = (int64_t)hs[3];
    }
}

}  // namespace pano
