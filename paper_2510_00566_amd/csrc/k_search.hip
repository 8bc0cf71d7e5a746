// Search kernels for gfx950: coarse probing, work decomposition, threshold
// seeding, the persistent pruned scan (Algorithm 1 with the Compute / Update /
// Consolidate phases of Section 6.1 fused per level), the per-query merge with
// canonical rescoring of the boundary band, and the exact fallback.
#include "search_common.h"

#include <algorithm>
#include <cstring>
#include <mutex>

namespace pano {

// ================================================================ work list
// One workgroup: per-list query offsets (to list_qoff in global memory and/or
// qoff_lds, 32-bit, in LDS) and, when item_off is given, the item offsets of
// the eight XCD queues (lists are ordered by (l mod 8, l div 8)).
__device__ inline void wl_offsets_block(int nlist, int ceil8, int G, int bpi, int item_cap,
                                        const int32_t *__restrict__ list_cnt, const int64_t *__restrict__ list_blk,
                                        int64_t *__restrict__ list_qoff, int32_t *qoff_lds,
                                        int64_t *__restrict__ item_off, int *wave_tmp)
{
    int64_t run = 0;
    for (int base = 0; base < nlist; base += NT) {
        int l = base + threadIdx.x;
        int c = l < nlist ? list_cnt[l] : 0;
        int tot;
        int o = block_exclusive_scan(c, wave_tmp, &tot);
        if (l < nlist) {
            if (list_qoff) list_qoff[l] = run + o;
            if (qoff_lds) qoff_lds[l] = (int32_t)(run + o);
        }
        run += tot;
    }
    if (threadIdx.x == 0) {
        if (list_qoff) list_qoff[nlist] = run;
        if (qoff_lds) qoff_lds[nlist] = (int32_t)run;
    }
    if (item_off == nullptr) return;
    __syncthreads();
    const int npos = 8 * ceil8;
    int64_t irun = 0;
    for (int base = 0; base < npos; base += NT) {
        int pos = base + threadIdx.x;
        int items = 0;
        if (pos < npos) {
            int l = (pos % ceil8) * 8 + pos / ceil8;
            if (l < nlist) {
                int c = list_cnt[l];
                int64_t nb = list_blk[l + 1] - list_blk[l];
                const int b = list_bpi(bpi, nb, item_cap);
                if (c > 0 && nb > 0) items = ((c + G - 1) / G) * (int)((nb + b - 1) / b);
            }
        }
        int tot;
        int o = block_exclusive_scan(items, wave_tmp, &tot);
        if (pos < npos) item_off[pos] = irun + o;
        irun += tot;
    }
    if (threadIdx.x == 0) item_off[npos] = irun;
}

__global__ __launch_bounds__(NT) void k_wl_offsets(int nlist, int ceil8, int G, int bpi, int item_cap,
                                                   const int32_t *__restrict__ list_cnt,
                                                   const int64_t *__restrict__ list_blk,
                                                   int64_t *__restrict__ list_qoff,
                                                   int64_t *__restrict__ item_off)
{
    __shared__ int wave_tmp[NT / 64];
    wl_offsets_block(nlist, ceil8, G, bpi, item_cap, list_cnt, list_blk, list_qoff, nullptr, item_off, wave_tmp);
}

// The per-list query arrays in one launch (up to WL_FUSED_LISTS lists): every
// workgroup derives the per-list query offsets from the counts in its LDS
// (workgroup 0 also publishes them and the item offsets for the scan), then
// places its share of the (query, probe) pairs.
constexpr int WL_FUSED_LISTS = 8192;
__global__ __launch_bounds__(NT) void k_wl_fill_fused(int64_t nq, int np_max, const int32_t *__restrict__ probes,
                                                      const int32_t *__restrict__ np, int nlist, int ceil8, int G,
                                                      int bpi, int item_cap, const int32_t *__restrict__ list_cnt,
                                                      const int64_t *__restrict__ list_blk,
                                                      int64_t *__restrict__ list_qoff, int64_t *__restrict__ item_off,
                                                      int32_t *__restrict__ list_fill, int32_t *__restrict__ list_q)
{
    extern __shared__ int32_t qoff_s[];  // [nlist + 1]
    __shared__ int wave_tmp[NT / 64];
    const bool first = blockIdx.x == 0;
    wl_offsets_block(nlist, ceil8, G, bpi, item_cap, list_cnt, list_blk, first ? list_qoff : nullptr, qoff_s,
                     first ? item_off : nullptr, wave_tmp);
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nq * np_max) return;
    const int64_t i = t / np_max;
    const int r = (int)(t % np_max);
    if (r < np[i]) {
        const int l = probes[t];
        const int pos = atomicAdd(&list_fill[l], 1);
        list_q[qoff_s[l] + pos] = (int32_t)i;
    }
}

__global__ void k_wl_fill(int64_t nq, int np_max, const int32_t *__restrict__ probes,
                          const int32_t *__restrict__ np, const int64_t *__restrict__ list_qoff,
                          int32_t *__restrict__ list_fill, int32_t *__restrict__ list_q)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nq * np_max) return;
    const int64_t i = t / np_max;
    const int r = (int)(t % np_max);
    if (r < np[i]) {
        const int l = probes[t];
        const int pos = atomicAdd(&list_fill[l], 1);
        list_q[list_qoff[l] + pos] = (int32_t)i;
    }
}

// Orders each list's queries by their approximate distance to the list's
// centroid (from the coarse products), so that a query group holds queries
// at similar distance: the queries of the list's own cluster come first and
// the far ones, whose candidates fail the level-1 bound, share groups of
// their own.  A pure reordering of the work; the answer does not change.
// A list is ordered in chunks of WL_SORT_CHUNK queries, one workgroup per
// chunk (blockIdx.y), so that long lists do not serialise on one workgroup:
// each chunk spans the list's distance range in order, so its groups still
// hold queries of similar distance.
constexpr int WL_SORT_CHUNK = 1024;
__global__ __launch_bounds__(NT) void k_wl_sort(int nlist, const int32_t *__restrict__ list_cnt,
                                                const int64_t *__restrict__ list_qoff, int32_t *__restrict__ list_q,
                                                const float *__restrict__ S, const float *__restrict__ qn2,
                                                const float *__restrict__ cn2)
{
    __shared__ uint64_t Kq[WL_SORT_CHUNK];
    const int l = blockIdx.x;
    const int c0 = blockIdx.y * WL_SORT_CHUNK;
    const int cnt = min(list_cnt[l] - c0, WL_SORT_CHUNK);
    if (cnt < 2) return;
    const int64_t off = list_qoff[l] + c0;
    const int P = next_pow2(cnt);
    const float c2 = cn2[l];
    for (int i = threadIdx.x; i < P; i += NT) {
        if (i < cnt) {
            const int32_t qq = list_q[off + i];
            const float dv = fmaxf(qn2[qq] + c2 - 2.f * S[(int64_t)qq * nlist + l], 0.f);
            Kq[i] = make_key(dv, qq);
        } else {
            Kq[i] = KEY_MAX;
        }
    }
    __syncthreads();
    block_bitonic_sort(Kq, P);
    for (int i = threadIdx.x; i < cnt; i += NT) list_q[off + i] = key_id(Kq[i]);
}


// ================================================================ index views
struct IndexView {
    const float *levels;
    const uint16_t *levels16;  // bfloat16 copy of the level tiles (same layout) or null
    const float *tails;   // [block][level][B]
    const int32_t *ids;   // [block][B]
    const int32_t *blk_cnt;
    const int64_t *list_blk;
    const float *raw;     // [n][d]
};

struct QueryView {
    const float *qy;      // [nq][d_pad]
    const float *qtail;   // [nq][L]
    const float *qE;      // [nq]
    const float *qA;      // [nq]
    const float *qraw;    // [nq][d]
};

// ================================================================ seeding
__host__ __device__ inline size_t seed_key_bytes(int pool) { return ((size_t)8 * next_pow2(pool) + 15) / 16 * 16; }
__host__ __device__ inline size_t seed_lds_bytes(int pool, int d_pad)
{
    return seed_key_bytes(pool) + (size_t)(d_pad >> 2) * (16 + 8);
}
// One workgroup per query: rank the first `pool` candidates of the query's
// nearest list by their level-1 lower bound, compute the full distance of the
// `cnt` most promising ones and start d_k from their k-th best (Algorithm 1
// seeds its heap with exact distances before the first batch).  The kernel
// needs only the transformed queries and the coarse products: the query's
// norms and its constants E_q, A_q (the formulas of the row-norms kernel,
// with FP64 sums in another order, far inside their 1e-6 rounding slack) are
// computed here, so it runs beside the row norms and the coarse step.
// qa_cabs, qa_b0max2: the A_q constants of the scan that uses the threshold.
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_seed(SearchConsts c, IndexView ix, QueryView qv,
                                             const float *__restrict__ S_, const float *__restrict__ cn2,
                                             int d, int nlist, const int32_t *__restrict__ nprobe_dev,
                                             int nprobe_all, int np_max, float c_co,
                                             const int64_t *__restrict__ list_len, int pool, int cnt,
                                             const float *__restrict__ mu, float qa_cabs, float qa_b0max2,
                                             float *__restrict__ thr, uint64_t *__restrict__ buf,
                                             int32_t *__restrict__ buf_cnt, int capq, int32_t *__restrict__ flags)
{
    // dynamic LDS (seed_lds_bytes): keys [next_pow2(pool)], the rotated
    // query [d_pad / 4] float4, chunk offsets and widths [d_pad / 4] each;
    // sized to the workload so that the coarse step's waves fit beside it
    extern __shared__ __align__(16) char seed_sm[];
    uint64_t *K = reinterpret_cast<uint64_t *>(seed_sm);
    float4 *qs_l = reinterpret_cast<float4 *>(seed_sm + seed_key_bytes(pool));
    int *chunk_off = reinterpret_cast<int *>(qs_l + (c.g.d_pad >> 2));
    int *chunk_w = chunk_off + (c.g.d_pad >> 2);
    __shared__ float Ds[256];
    __shared__ int Ps[256];  // pool position of the i-th most promising candidate
    __shared__ float red_f[NT / 64];
    __shared__ int red_i[NT / 64];
    const int64_t q = blockIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // The list to seed from: the centroid nearest by the approximate
    // distances of the coarse products, taken only when it is certainly in
    // the probe set, i.e. fewer than p other lists have a lower bound at or
    // below its upper bound (the bounds are those of the coarse step).  This
    // needs no result of the coarse step, so the two run side by side.
    int l0 = 0;
    if (nlist > 1) {
        int p = nprobe_dev ? nprobe_dev[q] : nprobe_all;
        p = p < 1 ? 1 : (p > nlist ? nlist : p);
        if (p > np_max) p = np_max;
        // ||q||^2 in the coarse step's FP32 order (per lane, columns in
        // increasing order, then a butterfly)
        // (eight loads per lane in flight together, clamped so that no
        // branch surrounds them; the summation order is unchanged)
        float qq = 0.f;
        for (int j0 = 0; j0 < d; j0 += 512) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = qv.qraw[q * d + min(j0 + u * 64 + lane, d - 1)];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (j0 + u * 64 + lane < d) qq = __builtin_fmaf(v[u], v[u], qq);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) qq += __shfl_xor(qq, o, 64);
        const float *Sq = S_ + q * nlist;
        float bu = INFINITY;
        int bl = 0x7fffffff;
        for (int l0 = 0; l0 < nlist; l0 += 8 * NT) {
            float cv[8], sv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int lc = min(l0 + u * NT + (int)threadIdx.x, nlist - 1);
                cv[u] = cn2[lc];
                sv[u] = Sq[lc];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int l = l0 + u * NT + (int)threadIdx.x;
                if (l < nlist) {
                    const float a = qq + cv[u] - 2.f * sv[u];
                    const float del = c_co * (qq + cv[u]);
                    const float up = fmaxf(a + del, 0.f) * (1.0f + 1.2e-7f);
                    if (up < bu) {
                        bu = up;
                        bl = l;
                    }
                }
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const float ou = __shfl_xor(bu, o, 64);
            const int ol = __shfl_xor(bl, o, 64);
            if (ou < bu || (ou == bu && ol < bl)) {
                bu = ou;
                bl = ol;
            }
        }
        if (lane == 0) {
            red_f[wv] = bu;
            red_i[wv] = bl;
        }
        __syncthreads();
        bu = red_f[0];
        bl = red_i[0];
        for (int w = 1; w < NT / 64; ++w)
            if (red_f[w] < bu || (red_f[w] == bu && red_i[w] < bl)) {
                bu = red_f[w];
                bl = red_i[w];
            }
        int before = 0;
        for (int l0 = 0; l0 < nlist; l0 += 8 * NT) {
            float cv[8], sv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int lc = min(l0 + u * NT + (int)threadIdx.x, nlist - 1);
                cv[u] = cn2[lc];
                sv[u] = Sq[lc];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int l = l0 + u * NT + (int)threadIdx.x;
                const float a = qq + cv[u] - 2.f * sv[u];
                const float del = c_co * (qq + cv[u]);
                const float lo = fmaxf(a - del, 0.f) * (1.0f - 1.2e-7f);
                before += (l < nlist && l != bl && lo <= bu) ? 1 : 0;
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) before += __shfl_xor(before, o, 64);
        __syncthreads();
        if (lane == 0) red_i[wv] = before;
        __syncthreads();
        int tot = 0;
        for (int w = 0; w < NT / 64; ++w) tot += red_i[w];
        if (tot >= p) return;  // not certain to be probed: no seed for this query
        l0 = bl;
    }
    const int64_t len = list_len[l0];
    const int P = (int)min<int64_t>(pool, len);
    const int S = min(cnt, P);
    if (S < c.k) return;
    const LevelGeom &g = c.g;
    const int64_t b0 = ix.list_blk[l0];
    const float *qy = qv.qy + q * g.d_pad;
    const int w0 = g.wp[0], w04 = w0 >> 2;
    const int nch = g.d_pad >> 2;
    // ||q'||^2 and the energy after level 1 from the rotated query, and
    // ||fl(q - mu)||^2 from the raw one, in FP64 (per thread, then per wave,
    // then over the four waves)
    double e0 = 0.0, e1 = 0.0, ev = 0.0;
    for (int ch = threadIdx.x; ch < nch; ch += NT) {
        const float4 v = *reinterpret_cast<const float4 *>(qy + ch * 4);
        qs_l[ch] = v;
        const double s2 = (double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z + (double)v.w * v.w;
        e0 += s2;
        if (4 * ch >= g.mp[1]) e1 += s2;  // never for a single level (mp[1] = d_pad)
    }
    for (int j0 = 0; j0 < d; j0 += 4 * NT) {
        float xv[4], mv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = min(j0 + u * NT + (int)threadIdx.x, d - 1);  // clamped: no branch
            xv[u] = qv.qraw[q * d + j];
            mv[u] = mu[j];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (j0 + u * NT + (int)threadIdx.x < d) {
                const double t = (double)(xv[u] - mv[u]);
                ev += t * t;
            }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        e0 += __shfl_xor(e0, o, 64);
        e1 += __shfl_xor(e1, o, 64);
        ev += __shfl_xor(ev, o, 64);
    }
    __shared__ double red_d[3][NT / 64];
    if (lane == 0) {
        red_d[0][wv] = e0;
        red_d[1][wv] = e1;
        red_d[2][wv] = ev;
    }
    for (int ch = threadIdx.x; ch < nch; ch += NT) {
        int lv = 0;
        while (4 * ch >= g.mp[lv + 1]) ++lv;
        if (lv == 0) {
            chunk_off[ch] = 4 * ch * g.B;
            chunk_w[ch] = 4;
        } else {
            chunk_off[ch] = g.B * g.mp[lv] + (4 * ch - g.mp[lv]);
            chunk_w[ch] = g.wp[lv];
        }
    }
    __syncthreads();
    e0 = e1 = ev = 0.0;
    for (int w = 0; w < NT / 64; ++w) {
        e0 += red_d[0][w];
        e1 += red_d[1][w];
        ev += red_d[2][w];
    }
    const float a0 = (float)sqrt(e0);  // the tail norm after level 0, rounded to FP32
    const float a1 = (float)sqrt(e1);
    const float qE_s = (float)((double)c.mg.kappa * sqrt(ev) * (1.0 + 1e-6)) + c.mg.e_max;
    const float qA_s =
        (float)((double)qa_cabs * ((double)a0 * (double)a0 * (1.0 + 1e-6) + (double)qa_b0max2) * (1.0 + 1e-6));
    if (!isfinite(qE_s) || !isfinite(qA_s)) return;  // a non-finite query: no seed
    // level-1 lower bound of every pool candidate (the level-1 slice is at
    // most 16 chunks, all loads in flight together; clamped addresses, so no
    // branch surrounds them)
    const int PP = next_pow2(P);
    for (int p = threadIdx.x; p < PP; p += NT) {
        // (the query chunks are read from LDS in each iteration: kept in
        // registers across iterations they would push the kernel past the
        // register budget of four workgroups per compute unit)
        asm volatile("" ::: "memory");
        const int pc = min(p, P - 1);
        const int64_t gb = b0 + pc / g.B;
        const int s = pc % g.B;
        const float *x = ix.levels + gb * (int64_t)g.B * g.d_pad + (int64_t)s * 4;
        const float b1 = g.L > 1 ? ix.tails[gb * (int64_t)g.B * g.L + g.B + s] : 0.f;
        float4 xs[16];
#pragma unroll
        for (int j = 0; j < 16; ++j)
            xs[j] = *reinterpret_cast<const float4 *>(x + (int64_t)min(j, w04 - 1) * 4 * g.B);
        float sh = 0.f;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            if (j < w04) {
                const float4 q4 = qs_l[j];
                float t0 = q4.x - xs[j].x, t1 = q4.y - xs[j].y, t2 = q4.z - xs[j].z, t3 = q4.w - xs[j].w;
                sh = __builtin_fmaf(t0, t0, sh);
                sh = __builtin_fmaf(t1, t1, sh);
                sh = __builtin_fmaf(t2, t2, sh);
                sh = __builtin_fmaf(t3, t3, sh);
            }
        }
        const float tt = a1 - b1;
        K[p] = p < P ? make_key(sh + tt * tt, p) : KEY_MAX;
    }
    __syncthreads();
    block_bitonic_sort(K, PP);
    // full distance of the S most promising candidates: 8 lanes per
    // candidate, 32 candidates per round, each lane's chunks in groups of
    // sixteen loads in flight together (clamped to a valid chunk)
    const int team = threadIdx.x >> 3, tl = threadIdx.x & 7;
    for (int base = 0; base < S; base += NT / 8) {
        const int si = base + team;
        float part = 0.f;
        if (si < S) {
            const int p = key_id(K[si]);
            if (tl == 0) Ps[si] = p;
            const int64_t gb = b0 + p / g.B;
            const int s = p % g.B;
            const float *blk = ix.levels + gb * (int64_t)g.B * g.d_pad;
            for (int ch0 = tl; ch0 < nch; ch0 += 8 * 16) {
                float4 xs[16];
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const int ch = min(ch0 + 8 * j, nch - 1);
                    xs[j] = *reinterpret_cast<const float4 *>(blk + chunk_off[ch] + (int64_t)s * chunk_w[ch]);
                }
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    if (ch0 + 8 * j < nch) {
                        const float4 q4 = qs_l[ch0 + 8 * j];
                        float t0 = q4.x - xs[j].x, t1 = q4.y - xs[j].y, t2 = q4.z - xs[j].z,
                              t3 = q4.w - xs[j].w;
                        part = __builtin_fmaf(t0, t0, part);
                        part = __builtin_fmaf(t1, t1, part);
                        part = __builtin_fmaf(t2, t2, part);
                        part = __builtin_fmaf(t3, t3, part);
                    }
                }
            }
        }
#pragma unroll
        for (int o = 4; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
        if (si < S && tl == 0) Ds[si] = part;
    }
    __syncthreads();
    const int PS = next_pow2(S);
    for (int i = threadIdx.x; i < PS; i += NT) K[i] = i < S ? make_key(Ds[i], i) : KEY_MAX;
    __syncthreads();
    block_bitonic_sort(K, PS);
    // the k best seeds go to the query's result buffer, so the threshold
    // stands on committed candidates even if a relaxed bound (eps < 1)
    // prunes them when the scan meets them (the merge keeps one copy of a
    // candidate committed twice)
    // (the seeding runs before the scan on an empty buffer, so bpos is 0 and
    // k <= 128 keys fit)
    __shared__ int bpos_s;
    if (threadIdx.x == 0) {
        bpos_s = atomicAdd(&buf_cnt[q], c.k);
        atomicOr(&flags[q], FLAG_SEEDED);
    }
    __syncthreads();
    {
        const int bpos = bpos_s;
        for (int i = threadIdx.x; i < c.k; i += NT) {
            const int p = Ps[key_id(K[i])];
            const int64_t gb = b0 + p / g.B;
            if (bpos + i < capq) buf[q * capq + bpos + i] = make_key(key_dist(K[i]), ix.ids[gb * g.B + p % g.B]);
        }
    }
    if (threadIdx.x == 0) {
        float t = prune_threshold(key_dist(K[c.k - 1]), qE_s, qA_s, c.mg);
        atomic_min_nonneg(&thr[q], t);
    }
}

// ================================================================ scan
struct WorkView {
    const int32_t *list_cnt;
    const int64_t *list_qoff;
    const int32_t *list_q;
    const int64_t *item_off;
    int32_t *heads;        // [8] queue heads
    float *thr;            // [nq]
    uint64_t *buf;         // [nq][capq]
    int32_t *buf_cnt;      // [nq]
    int32_t *flags;        // [nq]
    unsigned long long *stats;  // optional counters
};

// Counters layout (unsigned long long): [0] items, [1] committed, [2] bytes,
// [8 + l] pairs reading level l.
constexpr int ST_ITEMS = 0, ST_COMMIT = 1, ST_BYTES = 2, ST_LEVEL = 8, ST_CYCLES = 80;

typedef float floatx4_t __attribute__((ext_vector_type(4)));

// Dot products of the (up to 16) queries of the group with 64 slots of the
// block (this wavefront's share) over one level of at most 64 dimensions
// (kg_count <= 16 groups of four), on the matrix cores: v_mfma_f32_16x16x4f32
// with queries as rows and slots as columns.  The reduction index is permuted
// so that each lane feeds four consecutive dimensions from one 16-byte load:
// in step t, lane (r, q) supplies dimensions 16t + 4q .. 16t + 4q + 3 of query
// r (from LDS) and of slot r (from the level tile: [group][slot][4] for level
// 1, slot-major rows of row_w floats for later levels).  qload(kg) returns
// the four query values of group kg for this lane's query row.  The loads of
// step t + 2 are issued before the products of step t, so two steps are
// always in flight; a lane past the last group reads a valid group and feeds
// zeros.  The level is summed in fresh accumulators and then added to acc
// (chunked accumulation, as the error bound assumes); FRESH: acc is
// overwritten.
template <bool FRESH = false, typename QLoad>
__device__ inline void level_dots(const float *__restrict__ tile, int B, int kg_count, QLoad qload, int wave_slot0,
                                  int lane, floatx4_t acc[4], int row_w = 0)
{
    const int r16 = lane & 15, kq = lane >> 4;
    const int T = (kg_count + 3) >> 2;
    auto fetch = [&](int t, float4 xa[4], float4 &qa) {
        const int kg = 4 * t + kq;
        const bool ok = kg < kg_count;
        const int kgc = ok ? kg : kg_count - 1;
        const float4 qv4 = qload(kgc);
        qa = ok ? qv4 : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            // 32-bit offsets from the uniform tile base (a level tile is far
            // below 4 GiB), so the loads can use scalar-base addressing
            const uint32_t slot = (uint32_t)(wave_slot0 + nt * 16 + r16);
            const uint32_t off = row_w ? slot * (uint32_t)row_w + (uint32_t)kgc * 4u
                                       : ((uint32_t)kgc * (uint32_t)B + slot) * 4u;
            // read unconditionally (a valid group of the same slot): the
            // query side is zero for a lane past the last group, so its
            // products vanish
            xa[nt] = *reinterpret_cast<const float4 *>(tile + off);
        }
    };
    floatx4_t part[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) part[nt] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    auto products = [&](const float4 xa[4], const float4 &qa) {
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            part[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa.x, xa[nt].x, part[nt], 0, 0, 0);
            part[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa.y, xa[nt].y, part[nt], 0, 0, 0);
            part[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa.z, xa[nt].z, part[nt], 0, 0, 0);
            part[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa.w, xa[nt].w, part[nt], 0, 0, 0);
        }
    };
    float4 xa0[4], xa1[4], qa0, qa1;
    fetch(0, xa0, qa0);
    if (T > 1) fetch(1, xa1, qa1);
    products(xa0, qa0);
    if (T > 2) fetch(2, xa0, qa0);
    if (T > 1) products(xa1, qa1);
    if (T > 3) fetch(3, xa1, qa1);
    if (T > 2) products(xa0, qa0);
    if (T > 3) products(xa1, qa1);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = FRESH ? part[nt] : acc[nt] + part[nt];
}

// The same dot products from the bfloat16 copy x~ of the tiles on
// v_mfma_f32_16x16x16bf16_1k (one step covers 16 dimensions).  Lane (r, q)
// feeds dimensions 16t + 4q .. +3 of query r and of slot r.  The FP32 query
// is split into q_hi + q_lo, both bfloat16 (|q - q_hi - q_lo| <= u_b^2 |q|),
// so the products are those with x~ up to a u_b^2 relative term.  Each lane
// also sums the squares of the x~ values it feeds; ex[nt] ends as
// ||x~_level||^2 of slot nt*16 + r16 (summed over the four lanes that share
// r16).  Loads run two steps ahead as in level_dots; acc is overwritten.
typedef short shortx4_t __attribute__((ext_vector_type(4)));
template <typename QLoad>
__device__ inline void level_dots_bf16(const uint16_t *__restrict__ tile, int B, int kg_count, QLoad qload,
                                       int wave_slot0, int lane, floatx4_t acc[4], float ex[4], int row_w = 0)
{
    const int r16 = lane & 15, kq = lane >> 4;
    const int T = (kg_count + 3) >> 2;
    auto fetch = [&](int t, uint2 xr[4], float4 &qf, bool &okf) {
        const int kg = 4 * t + kq;
        const bool ok = kg < kg_count;
        const int kgc = ok ? kg : kg_count - 1;
        const float4 qv4 = qload(kgc);
        qf = ok ? qv4 : make_float4(0.f, 0.f, 0.f, 0.f);
        okf = ok;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const uint32_t slot = (uint32_t)(wave_slot0 + nt * 16 + r16);
            const uint32_t off = row_w ? slot * (uint32_t)row_w + (uint32_t)kgc * 4u
                                       : ((uint32_t)kgc * (uint32_t)B + slot) * 4u;
            // read unconditionally (a valid group of the same slot); a lane
            // past the last group feeds a zero query and adds nothing to ex
            xr[nt] = *reinterpret_cast<const uint2 *>(tile + off);
        }
    };
    floatx4_t part[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        part[nt] = floatx4_t{0.f, 0.f, 0.f, 0.f};
        ex[nt] = 0.f;
    }
    auto products = [&](const uint2 xr[4], const float4 &qf, bool okf) {
        shortx4_t qh, ql;
        const float qv[4] = {qf.x, qf.y, qf.z, qf.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint16_t h = bf16_bits_rne(qv[e]);
            qh[e] = (short)h;
            ql[e] = (short)bf16_bits_rne(qv[e] - bf16_to_f32(h));
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            shortx4_t xa;
            xa[0] = (short)(xr[nt].x & 0xffffu);
            xa[1] = (short)(xr[nt].x >> 16);
            xa[2] = (short)(xr[nt].y & 0xffffu);
            xa[3] = (short)(xr[nt].y >> 16);
            part[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(qh, xa, part[nt], 0, 0, 0);
            part[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ql, xa, part[nt], 0, 0, 0);
            const float x0 = __uint_as_float(xr[nt].x << 16), x1 = __uint_as_float(xr[nt].x & 0xffff0000u);
            const float x2 = __uint_as_float(xr[nt].y << 16), x3 = __uint_as_float(xr[nt].y & 0xffff0000u);
            float e = ex[nt];
            e = __builtin_fmaf(x0, x0, e);
            e = __builtin_fmaf(x1, x1, e);
            e = __builtin_fmaf(x2, x2, e);
            e = __builtin_fmaf(x3, x3, e);
            ex[nt] = okf ? e : ex[nt];
        }
    };
    uint2 xr0[4], xr1[4];
    float4 qf0, qf1;
    bool ok0 = false, ok1 = false;
    fetch(0, xr0, qf0, ok0);
    if (T > 1) fetch(1, xr1, qf1, ok1);
    products(xr0, qf0, ok0);
    if (T > 2) fetch(2, xr0, qf0, ok0);
    if (T > 1) products(xr1, qf1, ok1);
    if (T > 3) fetch(3, xr1, qf1, ok1);
    if (T > 2) products(xr0, qf0, ok0);
    if (T > 3) products(xr1, qf1, ok1);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        acc[nt] = part[nt];
        ex[nt] += __shfl_xor(ex[nt], 16, 64);
        ex[nt] += __shfl_xor(ex[nt], 32, 64);
    }
}

// Refine one (query, candidate) pair level by level from lv_start (Algorithm 1
// per candidate, Eq. 3 / Eq. 4 bounds with the certified margin), stopping
// when its lower bound exceeds th.  sh enters as the head distance of levels
// before lv_start and leaves as the head distance of the levels read; lv_end
// is one past the last level read.  Returns true if the pair survives; then
// `accepted` tells that its upper bound proved it a survivor before the last
// level, and the levels from lv_end on are left to the caller to add.
template <bool BF>
__device__ __forceinline__ bool walk_pair(const SearchConsts &c, const float *__restrict__ blk,
                                          const uint16_t *__restrict__ blk16, const float *__restrict__ tl, int ss,
                                          const float *__restrict__ qrow, const float *qt, float th, float Aq,
                                          int lv_start, float &sh, int &lv_end, bool &accepted, int sub = 0,
                                          int lpp = 1)
{
    accepted = false;
    const LevelGeom &g = c.g;
    // four coordinates of level lv of slot ss (FP32 tile, or the bfloat16
    // copy widened to FP32)
    auto ld4 = [&](int lv, int c4) -> float4 {
        const int64_t o = (int64_t)g.B * g.mp[lv] + (int64_t)ss * g.wp[lv] + c4 * 4;
        if (BF) {
            const uint2 xr = *reinterpret_cast<const uint2 *>(blk16 + o);
            return make_float4(__uint_as_float(xr.x << 16), __uint_as_float(xr.x & 0xffff0000u),
                               __uint_as_float(xr.y << 16), __uint_as_float(xr.y & 0xffff0000u));
        }
        return *reinterpret_cast<const float4 *>(blk + o);
    };
    auto level_part = [&](int lv) -> float {
        const int w4 = g.wp[lv] >> 2;
        const float *qq4 = qrow + g.mp[lv];
        float part = 0.f;
        // lpp lanes (1, 2 or 4, neighbours in the wavefront) share the pair:
        // lane sub takes chunks sub, sub + lpp, ...  Each lane requests up to
        // WALK_CHUNKS chunks at once (one memory round trip per group), sums
        // them in order, and the lanes' partial sums are added.
        for (int c0 = sub; c0 < w4; c0 += WALK_CHUNKS * lpp) {
            float4 xs[WALK_CHUNKS], qs[WALK_CHUNKS];
#pragma unroll
            for (int j = 0; j < WALK_CHUNKS; ++j) {
                const int c4 = c0 + j * lpp;
                if (c4 < w4) {
                    xs[j] = ld4(lv, c4);
                    qs[j] = *reinterpret_cast<const float4 *>(qq4 + c4 * 4);
                }
            }
#pragma unroll
            for (int j = 0; j < WALK_CHUNKS; ++j) {
                if (c0 + j * lpp < w4) {
                    float t0 = qs[j].x - xs[j].x, t1 = qs[j].y - xs[j].y, t2 = qs[j].z - xs[j].z,
                          t3 = qs[j].w - xs[j].w;
                    part = __builtin_fmaf(t0, t0, part);
                    part = __builtin_fmaf(t1, t1, part);
                    part = __builtin_fmaf(t2, t2, part);
                    part = __builtin_fmaf(t3, t3, part);
                }
            }
        }
        if (lpp >= 2) part += __shfl_xor(part, 1, 64);
        if (lpp >= 4) part += __shfl_xor(part, 2, 64);
        return part;
    };
    // bfloat16 rows: ||x_h - x~_h|| <= u_b ||x_h|| for the head read so far
    const float b0row = BF ? tl[ss] : 0.f;
    // the bound of a pair whose head distance sh covers the levels up to lv:
    // 1 = pruned, 2 = accepted (its upper bound is under the threshold; the
    // other side of Cauchy-Schwarz, UB = ||q_h - x_h||^2 + (||q_t|| +
    // ||x_t||)^2, never grows with the level and every later bound, any eps,
    // stays below it, so the remaining levels need no further tests), 0 = go on
    auto test = [&](int lv, float b) -> int {
        const bool last = (lv + 1 == g.L);
        const float a = last ? 0.f : qt[lv + 1];
        const float dt = a - b;
        const float err = c.mg.c_level[lv + 1] * fmaxf(sh, 0.f) + Aq;
        const float ct = c.mg.c_tail * (a + b) * (a + b);
        const float delta = BF ? c.ub * head_norm_upper(b0row, b) + 1e-37f : 0.f;
        const bool pruned = BF ? pair_lower_bf(sh, a, b, err, ct, c.one_m_eps2, delta) > th
                               : pair_lower(sh, a, b, err, ct, c.one_m_eps2) > th;
        if (pruned) return 1;
        const float ub = BF ? pair_upper_bf(sh, a, b, err, ct, delta) : pair_upper(sh, a, b, err, ct);
        if (!last && ub <= th) return 2;
        return 0;
    };
    int lv = lv_start;
    if (lpp == 4 && c.walk2) {
        // two levels per memory round trip: with four lanes per pair and
        // levels of at most 64 dimensions, a lane's share of two levels is at
        // most eight chunks, all requested together; the second level's
        // reads are wasted when the first one prunes the pair
        while (lv < g.L) {
            const bool has2 = lv + 1 < g.L;
            float4 xs[8], qs[8];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int l2 = min(lv + h, g.L - 1);
                const int w4 = g.wp[l2] >> 2;
                const float *qq4 = qrow + g.mp[l2];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int c4 = sub + 4 * j;
                    if (c4 < w4 && (h == 0 || has2)) {
                        xs[h * 4 + j] = ld4(l2, c4);
                        qs[h * 4 + j] = *reinterpret_cast<const float4 *>(qq4 + c4 * 4);
                    }
                }
            }
            const float b0 = lv + 1 < g.L ? tl[(int64_t)(lv + 1) * g.B + ss] : 0.f;
            const float b1 = lv + 2 < g.L ? tl[(int64_t)(lv + 2) * g.B + ss] : 0.f;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (h == 1 && !has2) break;
                const int w4 = g.wp[lv + h] >> 2;
                float part = 0.f;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (sub + 4 * j < w4) {
                        const float4 x4 = xs[h * 4 + j], q4 = qs[h * 4 + j];
                        float t0 = q4.x - x4.x, t1 = q4.y - x4.y, t2 = q4.z - x4.z, t3 = q4.w - x4.w;
                        part = __builtin_fmaf(t0, t0, part);
                        part = __builtin_fmaf(t1, t1, part);
                        part = __builtin_fmaf(t2, t2, part);
                        part = __builtin_fmaf(t3, t3, part);
                    }
                }
                part += __shfl_xor(part, 1, 64);
                part += __shfl_xor(part, 2, 64);
                sh += part;
                const int r = test(lv + h, h == 0 ? b0 : b1);
                if (r) {
                    lv_end = lv + h + 1;
                    accepted = r == 2;
                    return r == 2;
                }
            }
            lv += has2 ? 2 : 1;
        }
        lv_end = g.L;
        return true;
    }
    for (; lv < g.L; ++lv) {
        const bool last = (lv + 1 == g.L);
        const float b = last ? 0.f : tl[(int64_t)(lv + 1) * g.B + ss];
        sh += level_part(lv);
        const int r = test(lv, b);
        if (r) {
            lv_end = lv + 1;
            accepted = r == 2;
            return r == 2;
        }
    }
    lv_end = lv;
    return true;
}

template <bool PRUNE, bool BF, bool STATS>
__device__ __forceinline__ void scan_body(const SearchConsts &c, const IndexView &ix, const QueryView &qv,
                                          const WorkView &wk)
{
    __shared__ uint16_t pr[GMAX * 256];  // (query in group) << 8 | slot
    __shared__ float pS[GMAX * 256];
    // dynamic LDS: [per-wave sort buffers: 4 x sbw][local top-kc: G x kc]; the
    // walk's keep flags alias the sort buffers (never live at the same time)
    extern __shared__ uint64_t dyn[];
    const int sbw = next_pow2(c.kc + 64);
    uint64_t *topk = dyn + 4 * sbw;
    uint8_t *keep = reinterpret_cast<uint8_t *>(dyn);
    __shared__ int wave_tmp[NT / 64];
    __shared__ int qid_s[GMAX], tcnt[GMAX], ncand[GMAX];
    __shared__ float thr_s[GMAX], E_s[GMAX], A_s[GMAX], rqh_s[GMAX];
    __shared__ int item_s, npairs_s;
    __shared__ float qtl_s[GMAX][64];
    __shared__ unsigned long long my_lv[64];
    __shared__ unsigned long long sparse_bytes_s;
    // query rows for the matrix-core dot products: level-1 slices (pruned
    // scan) or one level at a time (brute force), [query][group of 4]
    __shared__ float4 qrow_s[GMAX][16];
    // the queue-ordered item offsets (up to 1024 lists), copied once per
    // workgroup so that pulling and decoding an item costs LDS reads, not a
    // chain of dependent global loads; item numbers fit in 32 bits
    __shared__ int32_t ioff_s[IOFF_LDS];

    const LevelGeom &g = c.g;
    const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n_ioff = 8 * c.ceil8 + 1;
    const bool ioff_in_lds = n_ioff <= IOFF_LDS;
    if (ioff_in_lds)
        for (int i = tid; i < n_ioff; i += NT) ioff_s[i] = (int32_t)wk.item_off[i];
    auto ioff = [&](int i) -> int64_t { return ioff_in_lds ? (int64_t)ioff_s[i] : wk.item_off[i]; };
    const int r16 = lane & 15, kq = lane >> 4;
    // matrix-core operand of this lane's query row, from the staged slices
    auto q_lds = [&](int kg) -> float4 { return qrow_s[r16][kg]; };
    int queue = blockIdx.x & 7;
    int tried = 0;
    unsigned long long my_items = 0, my_bytes = 0;
    const int Lc = g.L < 64 ? g.L : 64;
    for (int i = tid; i < 64; i += NT) my_lv[i] = 0;
    if (tid == 0) sparse_bytes_s = 0;
    // phase cycle counters (thread 0, stats runs only) live in LDS so they
    // hold no registers in the hot loops
    __shared__ unsigned long long cyc[7];
    if (tid == 0) {
        for (int i = 0; i < 6; ++i) cyc[i] = 0;
        cyc[6] = __builtin_readcyclecounter();
    }
#define PANO_PHASE(i)                                                  \
    do {                                                               \
        if (STATS && wk.stats && tid == 0) {                                    \
            unsigned long long now_ = __builtin_readcyclecounter();    \
            cyc[i] += now_ - cyc[6];                                   \
            cyc[6] = now_;                                             \
        }                                                              \
    } while (0)

    __syncthreads();
    while (true) {
        // ---- pull the next item from this workgroup's XCD queue, then steal
        if (tid == 0) {
            int it = -1;
            while (tried < 8) {
                const int64_t qb = ioff(queue * c.ceil8), qe = ioff((queue + 1) * c.ceil8);
                if (qe > qb) {
                    int v = atomicAdd(&wk.heads[queue], 1);
                    if (qb + v < qe) {
                        it = (int)(qb + v);
                        break;
                    }
                }
                queue = (queue + 1) & 7;
                ++tried;
            }
            item_s = it;
        }
        __syncthreads();
        // uniform over the workgroup: kept in scalar registers
        const int item = __builtin_amdgcn_readfirstlane(item_s);
        PANO_PHASE(0);
        if (item < 0) break;
        // ---- decode: binary search the queue-ordered item offsets
        int lo = 0, hi = 8 * c.ceil8;
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (ioff(mid) <= item) lo = mid;
            else hi = mid;
        }
        const int pos = lo;
        const int l = (pos % c.ceil8) * 8 + pos / c.ceil8;
        const int local = (int)(item - ioff(pos));
        const int qcnt = wk.list_cnt[l];
        const int groups = (qcnt + c.G - 1) / c.G;
        const int gi = local % groups, ri = local / groups;
        const int ng = min(c.G, qcnt - gi * c.G);
        const int64_t lb0 = ix.list_blk[l], nblk = ix.list_blk[l + 1] - lb0;
        const int bpl = list_bpi(c.bpi, nblk, c.item_cap);
        const int bstart = ri * bpl;
        const int bend = (int)min<int64_t>(nblk, (int64_t)(ri + 1) * bpl);
        if (tid < ng) {
            const int qq = wk.list_q[wk.list_qoff[l] + gi * c.G + tid];
            qid_s[tid] = qq;
            tcnt[tid] = 0;
            thr_s[tid] = INFINITY;
            E_s[tid] = qv.qE[qq];
            A_s[tid] = qv.qA[qq];
        }
        if (STATS) ++my_items;
        __syncthreads();
        for (int e = tid; e < ng * 64; e += NT) {
            const int gq = e >> 6, lv = e & 63;
            qtl_s[gq][lv] = lv < g.L ? qv.qtail[(int64_t)qid_s[gq] * g.L + lv] : 0.f;
        }
        __syncthreads();
        if (tid < ng) {
            // head energy of level 1: ||q_h||^2 = a_0^2 - a_1^2
            const float a0 = qtl_s[tid][0], a1 = g.L > 1 ? qtl_s[tid][1] : 0.f;
            rqh_s[tid] = a0 * a0 - a1 * a1;
        }
        __syncthreads();

        for (int bb = bstart; bb < bend; ++bb) {
            // the thread index, opaque to the compiler at every block: values
            // derived from it are recomputed here instead of being computed
            // once and spilled to memory
            int tid_o = threadIdx.x;
            asm volatile("" : "+v"(tid_o));
            const int tid = tid_o, lane = tid_o & 63, r16 = lane & 15, kq = lane >> 4;
            const int wv = __builtin_amdgcn_readfirstlane(tid_o >> 6);
            auto q_lds = [&](int kg) -> float4 { return qrow_s[r16][kg]; };
            const int64_t gb = lb0 + bb;
            const int cnt = ix.blk_cnt[gb];
            const float *blk = ix.levels + gb * (int64_t)g.B * g.d_pad;
            const uint16_t *blk16 = BF ? ix.levels16 + gb * (int64_t)g.B * g.d_pad : nullptr;
            const float *tl = ix.tails + gb * (int64_t)g.B * g.L;
            if (tid < ng) {
                float t = __hip_atomic_load(&wk.thr[qid_s[tid]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                thr_s[tid] = fminf(thr_s[tid], t);
                ncand[tid] = 0;
            }
            if (PRUNE) {
                // level-1 query slices (the dense refinement of the previous
                // block may have left another level's slices here)
                const int kg0 = g.wp[0] >> 2;
                for (int e = tid; e < GMAX * 16; e += NT) {
                    const int gq = e >> 4, c4 = e & 15;
                    qrow_s[gq][c4] = (gq < ng && c4 < kg0)
                                         ? *reinterpret_cast<const float4 *>(qv.qy + (int64_t)qid_s[gq] * g.d_pad + c4 * 4)
                                         : make_float4(0.f, 0.f, 0.f, 0.f);
                }
            }
            __syncthreads();
            // ---- dense phase on the matrix cores.  Lane (r16, kq) of wave wv
            // ends with the dot products of queries 4 kq + v (v = 0..3) with
            // slots wv*64 + nt*16 + r16 (nt = 0..3).
            floatx4_t acc[4];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) acc[nt] = floatx4_t{0.f, 0.f, 0.f, 0.f};
            // opaque to the optimiser, so the tile addresses derived from it are
            // recomputed per block instead of being held in registers
            int slot0 = wv * 64;
            asm volatile("" : "+v"(slot0));
            const bool wave_live = slot0 < cnt;
            uint32_t mask = 0;  // bit nt*4 + v: pair (query 4kq+v, slot slot0+nt*16+r16) kept
            float sval[16];
            int lv_start = 1;  // first level left to the per-pair walk
            // tail norms of this lane's slots, requested before the products so
            // that both loads are in flight together (every slot of a block has
            // tails, 0 for an empty slot)
            float tb0[4], tb1[4];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const int sc = min(slot0 + nt * 16 + r16, g.B - 1);
                tb0[nt] = tl[sc];
                tb1[nt] = g.L > 1 ? tl[g.B + sc] : 0.f;
            }
            // this lane's four queries (4 kq + v): tail after level 1, head
            // energy of level 1, margin and threshold (the entries past the
            // group are never used)
            float qa1[4], qrq[4], qAq[4], qth[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gq = 4 * kq + v;
                qa1[v] = g.L > 1 ? qtl_s[gq][1] : 0.f;
                qrq[v] = rqh_s[gq];
                qAq[v] = A_s[gq];
                qth[v] = thr_s[gq];
            }
            if (PRUNE && BF) {
                // level 1 from the bfloat16 tile: the dot-product form gives
                // ||q_h - x~_h||^2 within A; the triangle inequality moves the
                // bound to x
                float ex[4] = {0.f, 0.f, 0.f, 0.f};
                if (wave_live) level_dots_bf16(blk16, g.B, g.wp[0] >> 2, q_lds, slot0, lane, acc, ex);
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    const int s = slot0 + nt * 16 + r16;
                    const bool valid = s < cnt;
                    const float b0 = valid ? tb0[nt] : 0.f;
                    const float b1 = valid ? tb1[nt] : 0.f;
                    const float delta = c.ub * head_norm_upper(b0, b1) + 1e-37f;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const bool on = valid && 4 * kq + v < ng;
                        const float a1 = qa1[v];
                        const float sh = qrq[v] + ex[nt] - 2.f * acc[nt][v];
                        const float lb = pair_lower_bf(sh, a1, b1, qAq[v], c.mg.c_tail * (a1 + b1) * (a1 + b1),
                                                       c.one_m_eps2, delta);
                        const bool sv = on & (lb <= qth[v]);  // both sides evaluated: no branch per pair
                        mask |= (uint32_t)sv << (nt * 4 + v);
                        sval[nt * 4 + v] = sh;
                    }
                }
                if (STATS && tid == 0) {
                    my_bytes += (unsigned long long)cnt * (g.wp[0] * 2 + (g.L > 1 ? 8 : 4) + 4);
                    if (Lc > 0) my_lv[0] += (unsigned long long)cnt * ng;
                }
            } else if (PRUNE) {
                if (wave_live) level_dots<true>(blk, g.B, g.wp[0] >> 2, q_lds, slot0, lane, acc);
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    const int s = slot0 + nt * 16 + r16;
                    const bool valid = s < cnt;
                    const float b0 = valid ? tb0[nt] : 0.f;
                    const float b1 = valid ? tb1[nt] : 0.f;
                    const float rxh = b0 * b0 - b1 * b1;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const bool on = valid && 4 * kq + v < ng;
                        const float a1 = qa1[v];
                        const float sh = qrq[v] + rxh - 2.f * acc[nt][v];
                        const float lb = pair_lower(sh, a1, b1, qAq[v], c.mg.c_tail * (a1 + b1) * (a1 + b1),
                                                    c.one_m_eps2);
                        const bool sv = on & (lb <= qth[v]);  // both sides evaluated: no branch per pair
                        mask |= (uint32_t)sv << (nt * 4 + v);
                        sval[nt * 4 + v] = sh;
                    }
                }
                if (STATS && tid == 0) {
                    my_bytes += (unsigned long long)cnt * (g.wp[0] * 4 + (g.L > 1 ? 8 : 4) + 4);
                    if (Lc > 0) my_lv[0] += (unsigned long long)cnt * ng;
                }
            }
            PANO_PHASE(1);
            if (PRUNE) {
                // While the survivors stay dense (typically the candidates of a
                // query's own cluster), keep refining whole levels on the matrix
                // cores: one coalesced pass over the level tile serves all of
                // them, instead of one gather per pair.
                while (lv_start < g.L) {
                    int alive_tot;
                    (void)block_exclusive_scan(__popc(mask), wave_tmp, &alive_tot);
                    alive_tot = __builtin_amdgcn_readfirstlane(alive_tot);
                    if (alive_tot == 0 || alive_tot < c.dense_min || alive_tot * 4 < cnt) break;
                    const int lv = lv_start;
                    const int kgc = g.wp[lv] >> 2;
                    if (kgc > 16) break;
                    for (int e = tid; e < GMAX * 16; e += NT) {
                        const int gq = e >> 4, c4 = e & 15;
                        qrow_s[gq][c4] = (gq < ng && c4 < kgc)
                                             ? *reinterpret_cast<const float4 *>(qv.qy + (int64_t)qid_s[gq] * g.d_pad +
                                                                                 g.mp[lv] + c4 * 4)
                                             : make_float4(0.f, 0.f, 0.f, 0.f);
                    }
                    __syncthreads();
                    floatx4_t acc2[4];
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt) acc2[nt] = floatx4_t{0.f, 0.f, 0.f, 0.f};
                    float ex2[4] = {0.f, 0.f, 0.f, 0.f};
                    const bool last = lv + 1 == g.L;
                    // tails of this level and the next, requested before the products
                    float tbl[4], tbn[4];
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt) {
                        const int sc = min(slot0 + nt * 16 + r16, g.B - 1);
                        tbl[nt] = tl[(int64_t)lv * g.B + sc];
                        tbn[nt] = last ? 0.f : tl[(int64_t)(lv + 1) * g.B + sc];
                    }
                    if (wave_live) {
                        if (BF)
                            level_dots_bf16(blk16 + (int64_t)g.B * g.mp[lv], g.B, kgc, q_lds, slot0, lane, acc2, ex2,
                                            g.wp[lv]);
                        else
                            level_dots<true>(blk + (int64_t)g.B * g.mp[lv], g.B, kgc, q_lds, slot0, lane, acc2, g.wp[lv]);
                    }
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt) {
                        const int s = slot0 + nt * 16 + r16;
                        const bool valid = s < cnt;
                        const float bl = valid ? tbl[nt] : 0.f;
                        const float bn = valid ? tbn[nt] : 0.f;
                        const float rxl = BF ? ex2[nt] : bl * bl - bn * bn;
                        const float delta = BF ? c.ub * head_norm_upper(valid ? tb0[nt] : 0.f, bn) + 1e-37f : 0.f;
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int b = nt * 4 + v;
                            if (!(mask & (1u << b))) continue;
                            const int gq = 4 * kq + v;
                            const float al = qtl_s[gq][lv], an = last ? 0.f : qtl_s[gq][lv + 1];
                            const float sh = sval[b] + (al * al - an * an) + rxl - 2.f * acc2[nt][v];
                            sval[b] = sh;
                            const float err = c.mg.c_level[lv + 1] * fmaxf(sh, 0.f) + A_s[gq];
                            const float ct = c.mg.c_tail * (an + bn) * (an + bn);
                            const float lb = BF ? pair_lower_bf(sh, an, bn, err, ct, c.one_m_eps2, delta)
                                                : pair_lower(sh, an, bn, err, ct, c.one_m_eps2);
                            if (lb > thr_s[gq]) mask &= ~(1u << b);
                        }
                    }
                    if (STATS && tid == 0) {
                        my_bytes += (unsigned long long)cnt * (g.wp[lv] * (BF ? 2 : 4) + 8);
                        if (lv < 64) my_lv[lv] += (unsigned long long)alive_tot;
                    }
                    ++lv_start;
                    __syncthreads();
                }
            } else {
                // brute force: every level, query rows staged per level
                for (int lv = 0; lv < g.L; ++lv) {
                    const int kgc = g.wp[lv] >> 2;
                    for (int base = 0; base < kgc; base += 16) {
                        const int kgn = min(16, kgc - base);
                        __syncthreads();
                        for (int e = tid; e < GMAX * 16; e += NT) {
                            const int gq = e >> 4, c4 = e & 15;
                            qrow_s[gq][c4] = (gq < ng && c4 < kgn)
                                                 ? *reinterpret_cast<const float4 *>(qv.qy + (int64_t)qid_s[gq] * g.d_pad +
                                                                                     g.mp[lv] + (base + c4) * 4)
                                                 : make_float4(0.f, 0.f, 0.f, 0.f);
                        }
                        __syncthreads();
                        if (wave_live) {
                            if (lv == 0)
                                level_dots(blk + (int64_t)base * 4 * g.B, g.B, kgn, q_lds, slot0, lane, acc);
                            else
                                level_dots(blk + (int64_t)g.B * g.mp[lv] + base * 4, g.B, kgn, q_lds, slot0,
                                           lane, acc, g.wp[lv]);
                        }
                    }
                }
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    const int s = slot0 + nt * 16 + r16;
                    const bool valid = s < cnt;
                    const float b0 = valid ? tl[s] : 0.f;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int gq = 4 * kq + v;
                        const bool on = valid && gq < ng;
                        const float a0 = on ? qtl_s[gq][0] : 0.f;
                        const float dd = a0 * a0 + b0 * b0 - 2.f * acc[nt][v];
                        const bool sv = on && dist_lower(dd, A_s[gq], c.mg) <= thr_s[gq];
                        mask |= (uint32_t)sv << (nt * 4 + v);
                        sval[nt * 4 + v] = dd;
                    }
                }
                if (STATS && tid == 0) {
                    my_bytes += (unsigned long long)cnt * (g.d_pad * 4 + 4 + 4);
                    for (int lv = 0; lv < Lc; ++lv) my_lv[lv] += (unsigned long long)cnt * ng;
                }
            }
            PANO_PHASE(5);
            // ---- consolidate: survivors into the (query, slot) pair list
            {
                int tot;
                int off = block_exclusive_scan(__popc(mask), wave_tmp, &tot);
#pragma unroll
                for (int b = 0; b < 16; ++b) {
                    if (mask & (1u << b)) {
                        const int nt = b >> 2, v = b & 3;
                        pr[off] = (uint16_t)(((4 * kq + v) << 8) | (slot0 + nt * 16 + r16));
                        pS[off] = sval[b];
                        ++off;
                    }
                }
                if (tid == 0) npairs_s = tot;
                __syncthreads();
            }
            // ---- later levels: each surviving pair is refined by one lane, level
            // after level, until its bound exceeds the threshold or the last
            // level is read (no barrier between levels; the Update and
            // Consolidate phases of Section 6.1 run once, after the walk)
            if (PRUNE && lv_start < g.L) {
                const int np_ = __builtin_amdgcn_readfirstlane(npairs_s);
                unsigned long long my_dims = 0;
                // few pairs: several lanes per pair, so that each lane's
                // share of a level is one memory round trip and the pairs
                // spread over all four wavefronts
                const int lpp = c.walk_lanes ? c.walk_lanes : (np_ <= NT / 4 ? 4 : (np_ <= NT / 2 ? 2 : 1));
                const int sub = tid & (lpp - 1);
                for (int p = tid / lpp; p < np_; p += NT / lpp) {
                    const uint32_t pv = pr[p];
                    const int gq = (int)(pv >> 8), ss = (int)(pv & 255u);
                    const int qq = qid_s[gq];
                    float sh = pS[p];
                    int lv;
                    bool acc;
                    const bool alive = walk_pair<BF>(c, blk, blk16, tl, ss, qv.qy + (int64_t)qq * g.d_pad, &qtl_s[gq][0],
                                                     thr_s[gq], A_s[gq], lv_start, sh, lv, acc, sub, lpp);
                    // 0 pruned, 1 complete, 2 + l: accepted, levels from l left
                    // (the lanes of a pair hold the same values)
                    keep[p] = !alive ? 0 : (acc ? (uint8_t)(2 + lv) : 1);
                    pS[p] = sh;
                    if (STATS && wk.stats && sub == 0) {
                        const int lr = acc ? g.L : lv;
                        for (int v = lv_start; v < lr && v < 64; ++v) atomicAdd(&my_lv[v], 1ull);
                        my_dims += (unsigned long long)(g.mp[lr < g.L ? lr : g.L] - g.mp[lv_start]);
                    }
                }
                if (STATS && wk.stats && my_dims) atomicAdd(&sparse_bytes_s, my_dims * (BF ? 2ull : 4ull));
                __syncthreads();
                // Accepted pairs need their remaining levels summed, no more
                // tests: a whole wavefront reads them for one pair at a time
                // (64 lanes over the pair's remaining four-dimension chunks),
                // so one long read does not hold back the workgroup.
                for (int base = wv * 64; base < np_; base += NT) {
                    const int i = base + lane;
                    const uint64_t bal = __ballot(i < np_ && keep[i] >= 2);
                    uint64_t todo = bal;
                    while (todo) {
                        const int j = base + (int)__builtin_ctzll(todo);
                        todo &= todo - 1ull;
                        const uint32_t pv = pr[j];
                        const int gq = (int)(pv >> 8), ss = (int)(pv & 255u);
                        const int l0 = keep[j] - 2;
                        const float *qrow = qv.qy + (int64_t)qid_s[gq] * g.d_pad;
                        const int f0 = g.mp[l0] >> 2, f1 = g.mp[g.L] >> 2;  // chunk range left
                        float part = 0.f;
                        int l = l0;
#pragma unroll 4
                        for (int f = f0 + lane; f < f1; f += 64) {
                            while (4 * f >= g.mp[l + 1]) ++l;
                            const int64_t o = (int64_t)g.B * g.mp[l] + (int64_t)ss * g.wp[l] + (4 * f - g.mp[l]);
                            float4 x4;
                            if (BF) {
                                const uint2 xr = *reinterpret_cast<const uint2 *>(blk16 + o);
                                x4 = make_float4(__uint_as_float(xr.x << 16), __uint_as_float(xr.x & 0xffff0000u),
                                                 __uint_as_float(xr.y << 16), __uint_as_float(xr.y & 0xffff0000u));
                            } else {
                                x4 = *reinterpret_cast<const float4 *>(blk + o);
                            }
                            const float4 q4 = *reinterpret_cast<const float4 *>(qrow + 4 * f);
                            float t0 = q4.x - x4.x, t1 = q4.y - x4.y, t2 = q4.z - x4.z, t3 = q4.w - x4.w;
                            part = __builtin_fmaf(t0, t0, part);
                            part = __builtin_fmaf(t1, t1, part);
                            part = __builtin_fmaf(t2, t2, part);
                            part = __builtin_fmaf(t3, t3, part);
                        }
#pragma unroll
                        for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
                        if (lane == 0) {
                            pS[j] += part;
                            keep[j] = 1;
                        }
                    }
                }
                __syncthreads();
                // one stable compaction of the pairs that survived every level
                int kept = 0;
                for (int base = 0; base < np_; base += NT) {
                    const int i = base + tid;
                    const bool f = i < np_ && keep[i];
                    const uint32_t pv = f ? pr[i] : 0u;
                    const float sv = f ? pS[i] : 0.f;
                    int tot;
                    int off = block_exclusive_scan(f ? 1 : 0, wave_tmp, &tot);
                    if (f) {
                        pr[kept + off] = (uint16_t)pv;
                        pS[kept + off] = sv;
                    }
                    kept += tot;
                    __syncthreads();
                }
                if (tid == 0) npairs_s = kept;
                __syncthreads();
            }
            PANO_PHASE(2);
            // ---- commit: merge each query's survivors into its local top-kc
            const int np_ = __builtin_amdgcn_readfirstlane(npairs_s);
            if (np_ > 0) {
                for (int i = tid; i < np_; i += NT) atomicAdd(&ncand[pr[i] >> 8], 1);
                __syncthreads();
                volatile uint64_t *SB = dyn + wv * sbw;
                for (int gq = wv; gq < ng; gq += NT / 64) {
                    if (ncand[gq] == 0) continue;
                    int cntk = tcnt[gq];
                    uint64_t *tk = &topk[gq * c.kc];
                    for (int i = lane; i < cntk; i += 64) SB[i] = tk[i];
                    int napp = 0;
                    float tnew = thr_s[gq];
                    bool ovf = false;
                    // sort what is buffered, keep the best kc, refresh d_k
                    auto flush = [&]() {
                        const int tot = cntk + napp;
                        const int n2 = next_pow2(tot);
                        for (int i = tot + lane; i < n2; i += 64) SB[i] = KEY_MAX;
                        __builtin_amdgcn_wave_barrier();
                        wave_bitonic_sort(SB, n2, lane);
                        const int keepn = min(c.kc, tot);
                        if (keepn >= c.k)
                            tnew = fminf(tnew, prune_threshold(key_dist(SB[c.k - 1]), E_s[gq], A_s[gq], c.mg,
                                                               c.bfdelta));
                        for (int i = c.kc + lane; i < tot; i += 64)
                            if (dist_lower(key_dist(SB[i]), A_s[gq], c.mg, c.bfdelta) <= tnew) ovf = true;
                        cntk = keepn;
                        napp = 0;
                        __builtin_amdgcn_wave_barrier();
                    };
                    for (int base = 0; base < np_; base += 64) {
                        if (cntk + napp + 64 > sbw) flush();
                        const int i = base + lane;
                        bool f = false;
                        uint64_t key = 0;
                        if (i < np_) {
                            const uint32_t pv = pr[i];
                            if ((int)(pv >> 8) == gq) {
                                f = true;
                                key = make_key(fmaxf(pS[i], 0.f), ix.ids[gb * g.B + (pv & 255u)]);
                            }
                        }
                        const uint64_t bal = __ballot(f);
                        const int rk = __popcll(bal & ((1ull << lane) - 1ull));
                        if (f) SB[cntk + napp + rk] = key;
                        napp += __popcll(bal);
                    }
                    flush();
                    for (int i = lane; i < cntk; i += 64) tk[i] = SB[i];
                    const bool anyovf = __ballot(ovf) != 0ull;
                    if (lane == 0) {
                        tcnt[gq] = cntk;
                        thr_s[gq] = tnew;
                        if (tnew < INFINITY) atomic_min_nonneg(&wk.thr[qid_s[gq]], tnew);
                        if (anyovf) atomicOr(&wk.flags[qid_s[gq]], FLAG_OVERFLOW);
                    }
                    __builtin_amdgcn_wave_barrier();
                }
            }
            __syncthreads();
            PANO_PHASE(3);
        }
        // ---- item end: publish each query's local top-kc entries that can
        // still reach its final band
        for (int gq = wv; gq < ng; gq += NT / 64) {
            const int qq = qid_s[gq];
            const float t = fminf(thr_s[gq], __hip_atomic_load(&wk.thr[qq], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            const float Aq = A_s[gq];
            const int cntk = tcnt[gq];
            int nout = 0;
            for (int base = 0; base < cntk; base += 64) {
                const int i = base + lane;
                const bool f = i < cntk && dist_lower(key_dist(topk[gq * c.kc + i]), Aq, c.mg, c.bfdelta) <= t;
                nout += __popcll(__ballot(f));
            }
            int basepos = 0;
            if (lane == 0 && nout > 0) basepos = atomicAdd(&wk.buf_cnt[qq], nout);
            basepos = __shfl(basepos, 0, 64);
            int w = 0;
            for (int base = 0; base < cntk; base += 64) {
                const int i = base + lane;
                const uint64_t key = i < cntk ? topk[gq * c.kc + i] : KEY_MAX;
                const bool f = i < cntk && dist_lower(key_dist(key), Aq, c.mg, c.bfdelta) <= t;
                const uint64_t bal = __ballot(f);
                const int rk = __popcll(bal & ((1ull << lane) - 1ull));
                if (f) {
                    const int dst = basepos + w + rk;
                    if (dst < c.capq) wk.buf[(int64_t)qq * c.capq + dst] = key;
                    else atomicOr(&wk.flags[qq], FLAG_OVERFLOW);
                }
                w += __popcll(bal);
            }
        }
        __syncthreads();
        PANO_PHASE(4);
    }
#undef PANO_PHASE
    if (STATS && wk.stats && tid == 0) {
        for (int i = 0; i < 6; ++i) atomicAdd(&wk.stats[ST_CYCLES + i], cyc[i]);
        atomicAdd(&wk.stats[ST_ITEMS], my_items);
        atomicAdd(&wk.stats[ST_BYTES], my_bytes + sparse_bytes_s);
        for (int lv = 0; lv < Lc; ++lv)
            if (my_lv[lv]) atomicAdd(&wk.stats[ST_LEVEL + lv], my_lv[lv]);
    }
}

// The pruned scan is tuned for three workgroups per CU (its time goes to the
// latency of the per-pair level walks); the brute-force scan keeps its
// registers (its time goes to the dense matrix-core phase).
// The searches themselves run the instances without counters; a search
// asked for counters runs the *_stats instances (same arithmetic).
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_scan_pruned(SearchConsts c,
                                                                                            IndexView ix,
                                                                                            QueryView qv,
                                                                                            WorkView wk)
{
    scan_body<true, false, false>(c, ix, qv, wk);
}

__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_scan_pruned_stats(
    SearchConsts c, IndexView ix, QueryView qv, WorkView wk)
{
    scan_body<true, false, true>(c, ix, qv, wk);
}

__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_scan_pruned_bf16(
    SearchConsts c, IndexView ix, QueryView qv, WorkView wk)
{
    scan_body<true, true, false>(c, ix, qv, wk);
}

__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_scan_pruned_bf16_stats(
    SearchConsts c, IndexView ix, QueryView qv, WorkView wk)
{
    scan_body<true, true, true>(c, ix, qv, wk);
}

__global__ __launch_bounds__(NT) void k_scan_brute(SearchConsts c, IndexView ix, QueryView qv, WorkView wk)
{
    scan_body<false, false, false>(c, ix, qv, wk);
}

__global__ __launch_bounds__(NT) void k_scan_brute_stats(SearchConsts c, IndexView ix, QueryView qv, WorkView wk)
{
    scan_body<false, false, true>(c, ix, qv, wk);
}

// ================================================================ per-wave scan
// Every wavefront is its own worker: it pulls work items (list, group of up to
// 16 queries, block range) from the XCD queues and walks each block in steps
// of 64 slots, with no barrier shared with the other wavefronts of its
// workgroup.  One step is Algorithm 1 for a batch of 16 x 64 (query, slot)
// pairs:
//  * Compute / Update for level 1 on the matrix cores (the dot-product form of
//    the Eq. 3 bound with its certified margin), the query slices staged in
//    LDS for the whole item;
//  * Consolidate: the surviving pairs are compacted by ballots (per-bit lane counts)
//    into the wave's pair list in LDS;
//  * the later levels level-synchronously over that list: each pass reads one
//    level of every live pair (one, two or four lanes per pair by the level
//    width), adds its exact partial distance, tests the bound and compacts
//    the list in place;
//  * commit: a pair that survives the last level has its FP32 distance; it is
//    appended to its query's result buffer if it can still reach the final
//    band, and the k best distances the wave has committed for the query give
//    its threshold (published with atomicMin).
// The brute-force instance reads every level of every pair on the matrix
// cores and commits the pairs within the threshold.
#ifndef WAVE_SCAN_WPE
#define WAVE_SCAN_WPE 3  // wavefronts per SIMD the per-wave scan is compiled for
#endif
template <bool BF>
__device__ __forceinline__ float4 wave_ld4(const float *__restrict__ blk, const uint16_t *__restrict__ blk16,
                                           int64_t o)
{
    if (BF) {
        const uint2 xr = *reinterpret_cast<const uint2 *>(blk16 + o);
        return make_float4(__uint_as_float(xr.x << 16), __uint_as_float(xr.x & 0xffff0000u),
                           __uint_as_float(xr.y << 16), __uint_as_float(xr.y & 0xffff0000u));
    }
    return *reinterpret_cast<const float4 *>(blk + o);
}

template <bool PRUNE, bool BF, bool STATS, bool RELAX = true>
__device__ __forceinline__ void wave_scan_body(const SearchConsts &c, const IndexView &ix, const QueryView &qv,
                                               const WorkView &wk)
{
    extern __shared__ __align__(16) char wdyn[];
    __shared__ int32_t ioff_s[IOFF_LDS];
    __shared__ unsigned long long st_lv[64];
    __shared__ unsigned long long st_misc[2];  // items, bytes
    const LevelGeom &g = c.g;
    // (the wave index through readfirstlane: the compiler then keeps it and
    // every per-wave LDS address in scalar registers)
    const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n_ioff = 8 * c.ceil8 + 1;
    const bool ioff_in_lds = n_ioff <= IOFF_LDS;
    if (ioff_in_lds)
        for (int i = tid; i < n_ioff; i += NT) ioff_s[i] = (int32_t)wk.item_off[i];
    if (STATS) {
        for (int i = tid; i < 64; i += NT) st_lv[i] = 0;
        if (tid < 2) st_misc[tid] = 0;
    }
    // the only workgroup barrier before the end: the waves run independently
    __syncthreads();
    auto ioff = [&](int i) -> int64_t { return ioff_in_lds ? (int64_t)ioff_s[i] : wk.item_off[i]; };
    const WaveLds &lay = c.wl;
    char *wb = wdyn + (size_t)wv * lay.bytes;
    int *qid_w = reinterpret_cast<int *>(wb + lay.qid);
    float *thr_w = reinterpret_cast<float *>(wb + lay.thr);
    float *A_w = reinterpret_cast<float *>(wb + lay.A);
    float *E_w = reinterpret_cast<float *>(wb + lay.E);
    int *kc_w = reinterpret_cast<int *>(wb + lay.kc);
    float *qtl = reinterpret_cast<float *>(wb + lay.qtl);  // [16][L]
    float *kb = reinterpret_cast<float *>(wb + lay.kb);    // [16][k]
    float *sb = reinterpret_cast<float *>(wb + lay.sb);
    uint16_t *pcode = reinterpret_cast<uint16_t *>(wb + lay.code);
    float *pS = reinterpret_cast<float *>(wb + lay.pS);
    float4 *q1s = reinterpret_cast<float4 *>(wb + lay.q1);  // [16][kg0]
    float *rq_w = reinterpret_cast<float *>(wb + lay.rq);
    float *a1_w = reinterpret_cast<float *>(wb + lay.a1);
    const int r16 = lane & 15, kq = lane >> 4;
    const int L = g.L;
    const int kg0 = g.wp[0] >> 2;  // four-dimension chunks of level 1 (at most 16)
    const int T0 = (kg0 + 3) >> 2;
    const uint64_t below = (1ull << lane) - 1ull;
    auto wave_sync = [&]() {
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    };
    int queue = blockIdx.x & 7;
    int tried = 0;
    while (true) {
        // ---- pull an item from this workgroup's XCD queue, then steal
        int it = -1;
        if (lane == 0) {
            while (tried < 8) {
                const int64_t qb = ioff(queue * c.ceil8), qe = ioff((queue + 1) * c.ceil8);
                if (qe > qb) {
                    const int v = atomicAdd(&wk.heads[queue], 1);
                    if (qb + v < qe) {
                        it = (int)(qb + v);
                        break;
                    }
                }
                queue = (queue + 1) & 7;
                ++tried;
            }
        }
        const int item = __builtin_amdgcn_readfirstlane(__shfl(it, 0, 64));
        if (item < 0) break;
        // ---- decode: binary search of the queue-ordered item offsets
        int lo = 0, hi = 8 * c.ceil8;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (ioff(mid) <= item) lo = mid;
            else hi = mid;
        }
        const int l = (lo % c.ceil8) * 8 + lo / c.ceil8;
        const int local = (int)(item - ioff(lo));
        const int qcnt = wk.list_cnt[l];
        const int groups = (qcnt + c.G - 1) / c.G;
        const int gi = local % groups, ri = local / groups;
        const int ng = min(c.G, qcnt - gi * c.G);
        const int64_t lb0 = ix.list_blk[l], nblk = ix.list_blk[l + 1] - lb0;
        const int bpl = list_bpi(c.bpi, nblk, c.item_cap);
        const int bstart = ri * bpl;
        const int bend = (int)min<int64_t>(nblk, (int64_t)(ri + 1) * bpl);
        // ---- the item's queries
        if (lane < 16) {
            const bool on = lane < ng;
            const int qq = on ? wk.list_q[wk.list_qoff[l] + (int64_t)gi * c.G + lane] : 0;
            qid_w[lane] = on ? qq : -1;
            thr_w[lane] = INFINITY;
            A_w[lane] = on ? qv.qA[qq] : 0.f;
            E_w[lane] = on ? qv.qE[qq] : 0.f;
            kc_w[lane] = 0;
        }
        wave_sync();
        for (int e = lane; e < 16 * L; e += 64) {
            const int gq = e / L, lv = e - gq * L;
            qtl[e] = gq < ng ? qv.qtail[(int64_t)qid_w[gq] * L + lv] : 0.f;
        }
        // the group's level-1 query slices, read at every step of the item
        // from LDS (one address register instead of a global pointer per
        // chunk)
        // (the brute-force instances have no room for them and do not use them)
        if (PRUNE)
            for (int e = lane; e < ng * kg0; e += 64) {
                const int gq = e / kg0, kg = e - gq * kg0;
                q1s[e] = *reinterpret_cast<const float4 *>(qv.qy + (int64_t)qid_w[gq] * g.d_pad + kg * 4);
            }
        // per query: head energy of level 1, ||q_h||^2 = a_0^2 - a_1^2, and
        // the tail a_1 (zero past the group; pruned scan only)
        if (PRUNE && lane < 16) {
            const bool on = lane < ng;
            const float a0 = on ? qtl[lane * L] : 0.f;
            const float a1 = (on && L > 1) ? qtl[lane * L + 1] : 0.f;
            rq_w[lane] = a0 * a0 - a1 * a1;
            a1_w[lane] = a1;
        }
        wave_sync();
        if (STATS && lane == 0) atomicAdd(&st_misc[0], 1ull);

        for (int bb = bstart; bb < bend; ++bb) {
            const int64_t gb = lb0 + bb;
            const int cnt = ix.blk_cnt[gb];
            const float *blk = ix.levels + gb * (int64_t)g.B * g.d_pad;
            const uint16_t *blk16 = BF ? ix.levels16 + gb * (int64_t)g.B * g.d_pad : nullptr;
            const float *tl = ix.tails + gb * (int64_t)g.B * L;
            for (int slot0 = 0; slot0 < cnt; slot0 += 64) {
                // the lane index, opaque to the compiler at every step: values
                // derived from it are recomputed here (a few instructions)
                // instead of being computed once and spilled to memory
                // (the brute-force instances keep their hoisted values: they
                // have the registers for them)
                int lane_o = lane;
                if (PRUNE) asm volatile("" : "+v"(lane_o));
                const int lane = lane_o, r16 = lane_o & 15, kq = lane_o >> 4;
                const uint64_t below = (1ull << lane_o) - 1ull;
                // ---- thresholds: the queries' current d_k, requested now and
                // published to the wave's copy once the step's level-1 products
                // are done (the load overlaps the tile loads)
                const float thr_new =
                    lane < ng ? __hip_atomic_load(&wk.thr[qid_w[lane]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                              : INFINITY;
                float tb0[4], tb1[4];
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    const int sc = min(slot0 + nt * 16 + r16, g.B - 1);
                    tb0[nt] = tl[sc];
                    tb1[nt] = L > 1 ? tl[g.B + sc] : 0.f;
                }
                floatx4_t acc[4];
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) acc[nt] = floatx4_t{0.f, 0.f, 0.f, 0.f};
                float ex[4] = {0.f, 0.f, 0.f, 0.f};
                uint32_t mask = 0;
                float sval[16];
                if (PRUNE) {
                    // query operand: chunks 4 t + kq of query r16, zero past
                    // the group or the level
                    float4 qa[4];
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int kg = 4 * t + kq;
                        qa[t] = (t < T0 && r16 < ng && kg < kg0) ? q1s[r16 * kg0 + kg] : make_float4(0.f, 0.f, 0.f, 0.f);
                    }
                    // level 1 of the 64 slots against the group, on the matrix cores
                    if (BF) {
                        // bfloat16 tiles on v_mfma_f32_16x16x16bf16_1k (16
                        // dimensions per step); the FP32 query is split into
                        // two bfloat16 terms, and each lane also sums the
                        // squares of the tile values it feeds (||x~_h||^2)
                        uint2 xr[4][4];
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            if (t < T0) {
                                const int kgc = min(4 * t + kq, kg0 - 1);
#pragma unroll
                                for (int nt = 0; nt < 4; ++nt) {
                                    const uint32_t slot = (uint32_t)(slot0 + nt * 16 + r16);
                                    xr[t][nt] = *reinterpret_cast<const uint2 *>(
                                        blk16 + ((uint32_t)kgc * (uint32_t)g.B + slot) * 4u);
                                }
                            }
                        }
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            if (t < T0) {
                                const bool okq = 4 * t + kq < kg0;
                                shortx4_t qh, ql;
                                const float qv4[4] = {qa[t].x, qa[t].y, qa[t].z, qa[t].w};
#pragma unroll
                                for (int e = 0; e < 4; ++e) {
                                    const uint16_t h = bf16_bits_rne(qv4[e]);
                                    qh[e] = (short)h;
                                    ql[e] = (short)bf16_bits_rne(qv4[e] - bf16_to_f32(h));
                                }
#pragma unroll
                                for (int nt = 0; nt < 4; ++nt) {
                                    shortx4_t xa;
                                    xa[0] = (short)(xr[t][nt].x & 0xffffu);
                                    xa[1] = (short)(xr[t][nt].x >> 16);
                                    xa[2] = (short)(xr[t][nt].y & 0xffffu);
                                    xa[3] = (short)(xr[t][nt].y >> 16);
                                    acc[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(qh, xa, acc[nt], 0, 0, 0);
                                    acc[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ql, xa, acc[nt], 0, 0, 0);
                                    const float x0 = __uint_as_float(xr[t][nt].x << 16);
                                    const float x1 = __uint_as_float(xr[t][nt].x & 0xffff0000u);
                                    const float x2 = __uint_as_float(xr[t][nt].y << 16);
                                    const float x3 = __uint_as_float(xr[t][nt].y & 0xffff0000u);
                                    float e2 = ex[nt];
                                    e2 = __builtin_fmaf(x0, x0, e2);
                                    e2 = __builtin_fmaf(x1, x1, e2);
                                    e2 = __builtin_fmaf(x2, x2, e2);
                                    e2 = __builtin_fmaf(x3, x3, e2);
                                    ex[nt] = okq ? e2 : ex[nt];
                                }
                            }
                        }
#pragma unroll
                        for (int nt = 0; nt < 4; ++nt) {
                            ex[nt] += __shfl_xor(ex[nt], 16, 64);
                            ex[nt] += __shfl_xor(ex[nt], 32, 64);
                        }
                    } else {
                        const int T = T0;
                        auto fetch = [&](int t, float4 xa[4]) {
                            const int kgc = min(4 * t + kq, kg0 - 1);
#pragma unroll
                            for (int nt = 0; nt < 4; ++nt) {
                                const uint32_t slot = (uint32_t)(slot0 + nt * 16 + r16);
                                xa[nt] = *reinterpret_cast<const float4 *>(blk + ((uint32_t)kgc * (uint32_t)g.B + slot) * 4u);
                            }
                        };
                        auto products = [&](const float4 xa[4], const float4 &q4) {
#pragma unroll
                            for (int nt = 0; nt < 4; ++nt) {
                                acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(q4.x, xa[nt].x, acc[nt], 0, 0, 0);
                                acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(q4.y, xa[nt].y, acc[nt], 0, 0, 0);
                                acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(q4.z, xa[nt].z, acc[nt], 0, 0, 0);
                                acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(q4.w, xa[nt].w, acc[nt], 0, 0, 0);
                            }
                        };
                        float4 xa0[4], xa1[4];
                        fetch(0, xa0);
                        if (T > 1) fetch(1, xa1);
                        products(xa0, qa[0]);
                        if (T > 2) fetch(2, xa0);
                        if (T > 1) products(xa1, qa[1]);
                        if (T > 3) fetch(3, xa1);
                        if (T > 2) products(xa0, qa[2]);
                        if (T > 3) products(xa1, qa[3]);
                    }
                    if (lane < ng) thr_w[lane] = fminf(thr_w[lane], thr_new);
                    wave_sync();
                    // this lane's queries 4 kq + v: threshold, level-1 head
                    // energy, tail after level 1, margin
                    // (four consecutive queries: one LDS read per array; the
                    // entries past the group are zero, and masked below)
                    const float4 th4 = *reinterpret_cast<const float4 *>(thr_w + 4 * kq);
                    const float4 rq4 = *reinterpret_cast<const float4 *>(rq_w + 4 * kq);
                    const float4 a14 = *reinterpret_cast<const float4 *>(a1_w + 4 * kq);
                    const float4 A4 = *reinterpret_cast<const float4 *>(A_w + 4 * kq);
                    const float th[4] = {th4.x, th4.y, th4.z, th4.w};
                    const float rqh[4] = {rq4.x, rq4.y, rq4.z, rq4.w};
                    const float a1q[4] = {a14.x, a14.y, a14.z, a14.w};
                    const float Aq[4] = {A4.x, A4.y, A4.z, A4.w};
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt) {
                        const int s = slot0 + nt * 16 + r16;
                        const bool valid = s < cnt;
                        const float b0 = valid ? tb0[nt] : 0.f;
                        const float b1 = valid ? tb1[nt] : 0.f;
                        const float rxh = b0 * b0 - b1 * b1;
                        const float delta = BF ? c.ub * head_norm_upper(b0, b1) + 1e-37f : 0.f;
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int gq = 4 * kq + v;
                            const bool on = valid && gq < ng;
                            const float a1 = a1q[v];
                            const float sh = rqh[v] + (BF ? ex[nt] : rxh) - 2.f * acc[nt][v];
                            const float ct = c.mg.c_tail * (a1 + b1) * (a1 + b1);
                            const float lb = BF ? pair_lower_bf<RELAX>(sh, a1, b1, Aq[v], ct, c.one_m_eps2, delta)
                                                : pair_lower<RELAX>(sh, a1, b1, Aq[v], ct, c.one_m_eps2);
                            // (both sides evaluated: no branch per pair)
                            const bool sv = on & (lb <= th[v]);
                            mask |= (uint32_t)sv << (nt * 4 + v);
                            sval[nt * 4 + v] = sh;
                        }
                    }
                    if (STATS && lane == 0) {
                        const int cs = min(64, cnt - slot0);
                        atomicAdd(&st_lv[0], (unsigned long long)cs * ng);
                        atomicAdd(&st_misc[1], (unsigned long long)cs * (g.wp[0] * (BF ? 2 : 4) + (L > 1 ? 8 : 4)));
                    }
                } else {
                    // brute force: every level on the matrix cores, the query
                    // operand loaded per level; from bfloat16 tiles, the
                    // distance is to the rounded row (its squared norm summed
                    // from the values fed) and carries the bfloat16 bracket
                    const int qq = r16 < ng ? qid_w[r16] : 0;
                    for (int lv = 0; lv < L; ++lv) {
                        const int kgc = g.wp[lv] >> 2;
                        for (int base = 0; base < kgc; base += 16) {
                            const int kgn = min(16, kgc - base);
                            const float *qrow = qv.qy + (int64_t)qq * g.d_pad + g.mp[lv] + base * 4;
                            auto qload = [&](int kg) -> float4 {
                                return r16 < ng ? *reinterpret_cast<const float4 *>(qrow + kg * 4)
                                                : make_float4(0.f, 0.f, 0.f, 0.f);
                            };
                            if (BF) {
                                floatx4_t part[4];
                                float ex2[4];
                                if (lv == 0)
                                    level_dots_bf16(blk16 + (int64_t)base * 4 * g.B, g.B, kgn, qload, slot0, lane, part, ex2);
                                else
                                    level_dots_bf16(blk16 + (int64_t)g.B * g.mp[lv] + base * 4, g.B, kgn, qload, slot0,
                                                    lane, part, ex2, g.wp[lv]);
#pragma unroll
                                for (int nt = 0; nt < 4; ++nt) {
                                    acc[nt] += part[nt];
                                    ex[nt] += ex2[nt];
                                }
                            } else if (lv == 0) {
                                level_dots(blk + (int64_t)base * 4 * g.B, g.B, kgn, qload, slot0, lane, acc);
                            } else {
                                level_dots(blk + (int64_t)g.B * g.mp[lv] + base * 4, g.B, kgn, qload, slot0, lane, acc,
                                           g.wp[lv]);
                            }
                        }
                    }
                    if (lane < ng) thr_w[lane] = fminf(thr_w[lane], thr_new);
                    wave_sync();
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt) {
                        const int s = slot0 + nt * 16 + r16;
                        const bool valid = s < cnt;
                        const float b0 = valid ? tb0[nt] : 0.f;
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int gq = 4 * kq + v;
                            const bool on = valid && gq < ng;
                            const float a0 = qtl[gq * L];  // zero past the group
                            const float dd = a0 * a0 + (BF ? ex[nt] : b0 * b0) - 2.f * acc[nt][v];
                            const bool sv = on & (dist_lower(dd, A_w[gq], c.mg, c.bfdelta) <= thr_w[gq]);
                            mask |= (uint32_t)sv << (nt * 4 + v);
                            sval[nt * 4 + v] = dd;
                        }
                    }
                    if (STATS && lane == 0) {
                        const int cs = min(64, cnt - slot0);
                        for (int lv = 0; lv < L && lv < 64; ++lv) atomicAdd(&st_lv[lv], (unsigned long long)cs * ng);
                        atomicAdd(&st_misc[1], (unsigned long long)cs * (g.d_pad * (BF ? 2 : 4) + 4 + 4));
                    }
                }
                // ---- while many pairs of the step are alive, refine the next
                // level densely on the matrix cores (one pass over the 64
                // slots' level tile serves all of them; the dot-product form
                // with the margins of level 1)
                int lv_first = 1;  // first level left to the sparse passes
                if (PRUNE) {
                    int alive = wave_count16(mask);
                    while (lv_first < L && alive >= c.dense_min && g.wp[lv_first] <= 64) {
                        const int lv = lv_first;
                        const bool last = lv + 1 == L;
                        const int kgc = g.wp[lv] >> 2;
                        const float *qrow = qv.qy + (int64_t)(r16 < ng ? qid_w[r16] : 0) * g.d_pad + g.mp[lv];
                        float tbl[4], tbn[4];
#pragma unroll
                        for (int nt = 0; nt < 4; ++nt) {
                            const int sc = min(slot0 + nt * 16 + r16, g.B - 1);
                            tbl[nt] = tl[(int64_t)lv * g.B + sc];
                            tbn[nt] = last ? 0.f : tl[(int64_t)(lv + 1) * g.B + sc];
                        }
                        floatx4_t acc2[4];
                        float ex2[4] = {0.f, 0.f, 0.f, 0.f};
                        auto qload = [&](int kg) -> float4 {
                            return r16 < ng ? *reinterpret_cast<const float4 *>(qrow + kg * 4)
                                            : make_float4(0.f, 0.f, 0.f, 0.f);
                        };
                        if (BF)
                            level_dots_bf16(blk16 + (int64_t)g.B * g.mp[lv], g.B, kgc, qload, slot0, lane, acc2, ex2,
                                            g.wp[lv]);
                        else
                            level_dots<true>(blk + (int64_t)g.B * g.mp[lv], g.B, kgc, qload, slot0, lane, acc2, g.wp[lv]);
                        // this lane's four queries at this level: head energy
                        // a_l^2 - a_(l+1)^2, tail a_(l+1), margin, threshold
                        // (for pairs that are not alive the values do not matter)
                        float rql[4], anq[4];
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int gq = 4 * kq + v;
                            const float al = qtl[gq * L + lv];
                            const float an = last ? 0.f : qtl[gq * L + lv + 1];
                            rql[v] = al * al - an * an;
                            anq[v] = an;
                        }
                        const float4 A4 = *reinterpret_cast<const float4 *>(A_w + 4 * kq);
                        const float4 th4 = *reinterpret_cast<const float4 *>(thr_w + 4 * kq);
                        const float Agq[4] = {A4.x, A4.y, A4.z, A4.w};
                        const float thq[4] = {th4.x, th4.y, th4.z, th4.w};
#pragma unroll
                        for (int nt = 0; nt < 4; ++nt) {
                            const int sidx = slot0 + nt * 16 + r16;
                            const bool valid = sidx < cnt;
                            const float bl = valid ? tbl[nt] : 0.f;
                            const float bn = valid ? tbn[nt] : 0.f;
                            const float rxl = BF ? ex2[nt] : bl * bl - bn * bn;
                            const float delta = BF ? c.ub * head_norm_upper(valid ? tb0[nt] : 0.f, bn) + 1e-37f : 0.f;
#pragma unroll
                            for (int v = 0; v < 4; ++v) {
                                const int b = nt * 4 + v;
                                const float an = anq[v];
                                const float sh = sval[b] + rql[v] + rxl - 2.f * acc2[nt][v];
                                const float Ag = Agq[v];
                                const float th = thq[v];
                                const float err = c.mg.c_level[lv + 1] * fmaxf(sh, 0.f) + Ag;
                                const float ct = c.mg.c_tail * (an + bn) * (an + bn);
                                const bool pruned = (BF ? pair_lower_bf<RELAX>(sh, an, bn, err, ct, c.one_m_eps2, delta)
                                                        : pair_lower<RELAX>(sh, an, bn, err, ct, c.one_m_eps2)) > th;
                                sval[b] = sh;
                                // (a pair that is not alive has its bit clear already)
                                mask &= pruned ? ~(1u << b) : ~0u;
                            }
                        }
                        if (STATS && lane == 0) {
                            const int cs = min(64, cnt - slot0);
                            atomicAdd(&st_lv[lv < 64 ? lv : 63], (unsigned long long)alive);
                            atomicAdd(&st_misc[1], (unsigned long long)cs * (g.wp[lv] * (BF ? 2 : 4) + 8));
                        }
                        ++lv_first;
                        alive = wave_count16(mask);
                    }
                }
                // ---- consolidate into the pair list, refine the later levels,
                // commit; in two halves (slots 0-31, 32-63) when more pairs
                // survive than the list holds
                const int tot = wave_count16(mask);
                const int halves = tot > WAVE_PAIRS ? 2 : 1;
                for (int hf = 0; hf < halves; ++hf) {
                    const uint32_t m = halves == 1 ? mask : (mask & (hf == 0 ? 0x00ffu : 0xff00u));
                    int n = 0;
                    int off = wave_prefix16(m, n);
                    if (n == 0) continue;
#pragma unroll
                    for (int b = 0; b < 16; ++b) {
                        if (m & (1u << b)) {
                            const int nt = b >> 2, v = b & 3;
                            pcode[off] = (uint16_t)(((4 * kq + v) << 8) | (slot0 + nt * 16 + r16));
                            pS[off] = sval[b];
                            ++off;
                        }
                    }
                    wave_sync();
                    // ---- later levels, one pass per level over the live pairs
                    for (int lv = lv_first; PRUNE && lv < L && n > 0; ++lv) {
                        const bool last = lv + 1 == L;
                        const int w4 = g.wp[lv] >> 2;
                        const int lpp = (w4 <= 4 && n > 16) ? 1 : ((w4 <= 8 && n > 16) ? 2 : 4);
                        const int sub = lane & (lpp - 1);
                        const int ppi = 64 / lpp;
                        const float *lvbase = blk + (int64_t)g.B * g.mp[lv];
                        const uint16_t *lvbase16 = BF ? blk16 + (int64_t)g.B * g.mp[lv] : nullptr;
                        int nout = 0;
                        if (STATS && lane == 0) {
                            atomicAdd(&st_lv[lv < 64 ? lv : 63], (unsigned long long)n);
                            atomicAdd(&st_misc[1], (unsigned long long)n * (g.wp[lv] * (BF ? 2 : 4) + 4));
                        }
                        for (int base = 0; base < n; base += ppi) {
                            const int i = base + lane / lpp;
                            const bool act = i < n;
                            const int ic = act ? i : n - 1;
                            const uint32_t pc = pcode[ic];
                            float sh = pS[ic];
                            const int gq = (int)(pc >> 8), ss = (int)(pc & 255u);
                            const float *qrow = qv.qy + (int64_t)qid_w[gq] * g.d_pad + g.mp[lv];
                            const float b = last ? 0.f : tl[(int64_t)(lv + 1) * g.B + ss];
                            float part = 0.f;
                            for (int c0 = sub; c0 < w4; c0 += 4 * lpp) {
                                float4 xs[4], qs4[4];
#pragma unroll
                                for (int j = 0; j < 4; ++j) {
                                    const int cc = min(c0 + j * lpp, w4 - 1);
                                    xs[j] = wave_ld4<BF>(lvbase, lvbase16, (int64_t)ss * g.wp[lv] + cc * 4);
                                    qs4[j] = *reinterpret_cast<const float4 *>(qrow + cc * 4);
                                }
#pragma unroll
                                for (int j = 0; j < 4; ++j) {
                                    if (c0 + j * lpp < w4) {
                                        const float t0 = qs4[j].x - xs[j].x, t1 = qs4[j].y - xs[j].y,
                                                    t2 = qs4[j].z - xs[j].z, t3 = qs4[j].w - xs[j].w;
                                        part = __builtin_fmaf(t0, t0, part);
                                        part = __builtin_fmaf(t1, t1, part);
                                        part = __builtin_fmaf(t2, t2, part);
                                        part = __builtin_fmaf(t3, t3, part);
                                    }
                                }
                            }
                            if (lpp >= 2) part += __shfl_xor(part, 1, 64);
                            if (lpp >= 4) part += __shfl_xor(part, 2, 64);
                            sh += part;
                            // the bound after this level (Eq. 3 / Eq. 4 with the
                            // certified margin)
                            const float a = last ? 0.f : qtl[gq * L + lv + 1];
                            const float err = c.mg.c_level[lv + 1] * fmaxf(sh, 0.f) + A_w[gq];
                            const float ct = c.mg.c_tail * (a + b) * (a + b);
                            const float th = thr_w[gq];
                            const bool pruned =
                                (BF ? pair_lower_bf<RELAX>(sh, a, b, err, ct, c.one_m_eps2,
                                                    c.ub * head_norm_upper(tl[ss], b) + 1e-37f)
                                    : pair_lower<RELAX>(sh, a, b, err, ct, c.one_m_eps2)) > th;
                            const bool keep = act && !pruned && sub == 0;
                            const uint64_t bal = __ballot(keep);
                            if (keep) {
                                const int pos = nout + __popcll(bal & below);
                                pcode[pos] = (uint16_t)pc;
                                pS[pos] = sh;
                            }
                            nout += __popcll(bal);
                        }
                        n = nout;
                        wave_sync();
                    }
                    if (n == 0) continue;
                    // ---- commit the survivors, 64 pairs at a time: those that
                    // can reach the final band go to their query's result buffer
                    // (one atomic per query of the chunk, all issued together),
                    // then each query's k best distances and threshold are
                    // updated
                    for (int base = 0; base < n; base += 64) {
                        const int i = base + lane;
                        const bool act = i < n;
                        const uint32_t pc = act ? pcode[i] : 0u;
                        const int gq = act ? (int)(pc >> 8) : 0;
                        const float D = act ? fmaxf(pS[i], 0.f) : 0.f;
                        const bool keep = act && dist_lower(D, A_w[gq], c.mg, c.bfdelta) <= thr_w[gq];
                        uint32_t qm = wave_or16(keep ? 1u << gq : 0u);
                        // per query of the chunk: its count (to lane gq) and each
                        // kept pair's rank among the query's kept pairs
                        int cnt_l = 0, rk = 0;
                        for (uint32_t m2 = qm; m2; m2 &= m2 - 1u) {
                            const int g2 = __builtin_ctz(m2);
                            const uint64_t bal = __ballot(keep && gq == g2);
                            if (lane == g2) cnt_l = __popcll(bal);
                            if (keep && gq == g2) rk = __popcll(bal & below);
                        }
                        int bpos = 0;
                        if (cnt_l > 0) bpos = atomicAdd(&wk.buf_cnt[qid_w[lane]], cnt_l);
                        bpos = __shfl(bpos, gq, 64);
                        if (keep) {
                            const int dst = bpos + rk;
                            const int qq = qid_w[gq];
                            const int32_t id = ix.ids[gb * g.B + (pc & 255u)];
                            if (dst < c.capq) wk.buf[(int64_t)qq * c.capq + dst] = make_key(D, id);
                            else atomicOr(&wk.flags[qq], FLAG_OVERFLOW);
                        }
                        // the k best distances so far and the threshold, one
                        // query at a time
                        while (qm) {
                            const int g2 = __builtin_ctz(qm);
                            qm &= qm - 1u;
                            const bool mine = keep && gq == g2;
                            const uint64_t mbal = __ballot(mine);
                            const int nk = __popcll(mbal);
                            int cntk = kc_w[g2];
                            const int tn = cntk + nk;
                            if (c.k <= 64) {
                                // merge by ranks: lane j < cntk holds the j-th best
                                // so far; each value's place in the union is its
                                // rank (kept values before new equal ones, new
                                // ones in lane order), found with one broadcast
                                // per value, with no sort
                                // (a lane may hold both a kept value and a new one)
                                const float kv = lane < cntk ? kb[g2 * c.k + lane] : INFINITY;
                                int posk = lane, posn = 0;
                                for (uint64_t mb = mbal; mb; mb &= mb - 1ull) {
                                    const int src = __builtin_ctzll(mb);
                                    const float v = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__float_as_int(D), src));
                                    const int r = __popcll(mbal & ((1ull << src) - 1ull));
                                    posk += v < kv;
                                    posn += v < D || (v == D && r < rk);
                                }
                                for (int j = 0; j < cntk; ++j) {
                                    const float v = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__float_as_int(kv), j));
                                    posn += v <= D;
                                }
                                wave_sync();
                                if (lane < cntk && posk < c.k) kb[g2 * c.k + posk] = kv;
                                if (mine && posn < c.k) kb[g2 * c.k + posn] = D;
                                wave_sync();
                                cntk = min(c.k, tn);
                                if (lane == 0 && cntk == c.k) sb[c.k - 1] = kb[g2 * c.k + c.k - 1];
                            } else {
                                for (int j = lane; j < cntk; j += 64) sb[j] = kb[g2 * c.k + j];
                                if (mine) sb[cntk + rk] = D;
                                const int P2 = next_pow2(tn);
                                for (int j = tn + lane; j < P2; j += 64) sb[j] = INFINITY;
                                wave_sync();
                                wave_bitonic_sort_f(sb, P2, lane);
                                wave_sync();
                                cntk = min(c.k, tn);
                                for (int j = lane; j < cntk; j += 64) kb[g2 * c.k + j] = sb[j];
                            }
                            if (lane == 0) {
                                kc_w[g2] = cntk;
                                if (cntk == c.k) {
                                    const float th = fminf(thr_w[g2], prune_threshold(sb[c.k - 1], E_w[g2], A_w[g2],
                                                                                      c.mg, c.bfdelta));
                                    thr_w[g2] = th;
                                    atomic_min_nonneg(&wk.thr[qid_w[g2]], th);
                                }
                            }
                            wave_sync();
                        }
                    }
                }
            }
        }
    }
    if (STATS && wk.stats) {
        __syncthreads();
        for (int i = tid; i < 64; i += NT)
            if (st_lv[i]) atomicAdd(&wk.stats[ST_LEVEL + i], st_lv[i]);
        if (tid == 0) {
            atomicAdd(&wk.stats[ST_ITEMS], st_misc[0]);
            atomicAdd(&wk.stats[ST_BYTES], st_misc[1]);
        }
    }
}

__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WAVE_SCAN_WPE, WAVE_SCAN_WPE))) void k_scan_wave(SearchConsts c, IndexView ix,
                                                                                            QueryView qv, WorkView wk)
{
    wave_scan_body<true, false, false, false>(c, ix, qv, wk);
}
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WAVE_SCAN_WPE, WAVE_SCAN_WPE))) void k_scan_wave_stats(SearchConsts c,
                                                                                                  IndexView ix,
                                                                                                  QueryView qv,
                                                                                                  WorkView wk)
{
    wave_scan_body<true, false, true, false>(c, ix, qv, wk);
}
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WAVE_SCAN_WPE, WAVE_SCAN_WPE))) void k_scan_wave_bf16(SearchConsts c,
                                                                                                 IndexView ix,
                                                                                                 QueryView qv,
                                                                                                 WorkView wk)
{
    wave_scan_body<true, true, false, false>(c, ix, qv, wk);
}
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WAVE_SCAN_WPE, WAVE_SCAN_WPE))) void k_scan_wave_bf16_stats(
    SearchConsts c, IndexView ix, QueryView qv, WorkView wk)
{
    wave_scan_body<true, true, true, false>(c, ix, qv, wk);
}
// The same pruned scans for eps < 1 (the relaxed bound of Eq. 4); the
// instances above are those of eps = 1, which drop its 2 (1 - eps) a b term.
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WAVE_SCAN_WPE, WAVE_SCAN_WPE))) void k_scan_wave_relaxed(SearchConsts c, IndexView ix, QueryView qv, WorkView wk)
{
    wave_scan_body<true, false, false, true>(c, ix, qv, wk);
}
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WAVE_SCAN_WPE, WAVE_SCAN_WPE))) void k_scan_wave_relaxed_stats(SearchConsts c, IndexView ix, QueryView qv, WorkView wk)
{
    wave_scan_body<true, false, true, true>(c, ix, qv, wk);
}
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WAVE_SCAN_WPE, WAVE_SCAN_WPE))) void k_scan_wave_bf16_relaxed(SearchConsts c, IndexView ix, QueryView qv, WorkView wk)
{
    wave_scan_body<true, true, false, true>(c, ix, qv, wk);
}
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WAVE_SCAN_WPE, WAVE_SCAN_WPE))) void k_scan_wave_bf16_relaxed_stats(SearchConsts c, IndexView ix, QueryView qv, WorkView wk)
{
    wave_scan_body<true, true, true, true>(c, ix, qv, wk);
}
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WAVE_SCAN_WPE, WAVE_SCAN_WPE))) void k_scan_wave_brute(SearchConsts c,
                                                                                                  IndexView ix,
                                                                                                  QueryView qv,
                                                                                                  WorkView wk)
{
    wave_scan_body<false, false, false>(c, ix, qv, wk);
}
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WAVE_SCAN_WPE, WAVE_SCAN_WPE))) void k_scan_wave_brute_stats(
    SearchConsts c, IndexView ix, QueryView qv, WorkView wk)
{
    wave_scan_body<false, false, true>(c, ix, qv, wk);
}
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WAVE_SCAN_WPE, WAVE_SCAN_WPE))) void k_scan_wave_brute_bf16(
    SearchConsts c, IndexView ix, QueryView qv, WorkView wk)
{
    wave_scan_body<false, true, false>(c, ix, qv, wk);
}
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WAVE_SCAN_WPE, WAVE_SCAN_WPE))) void k_scan_wave_brute_bf16_stats(
    SearchConsts c, IndexView ix, QueryView qv, WorkView wk)
{
    wave_scan_body<false, true, true>(c, ix, qv, wk);
}


// ================================================================ merge
// Distance bits of the k-th smallest of n keys in global memory: radix
// select over the 32 bits of the (non-negative) distance, 8 bits per pass,
// with a 256-bin histogram in LDS.
__device__ uint32_t block_kth_dist_bits(const uint64_t *__restrict__ keys, int n, int k, int *hist, int *sel)
{
    uint32_t prefix = 0, mask = 0;
    int rank = k;
    for (int shift = 24; shift >= 0; shift -= 8) {
        for (int i = threadIdx.x; i < 256; i += NT) hist[i] = 0;
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += NT) {
            const uint32_t b = (uint32_t)(keys[i] >> 32);
            if ((b & mask) == prefix) atomicAdd(&hist[(b >> shift) & 255u], 1);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int acc = 0, dg = 0;
            while (dg < 255 && acc + hist[dg] < rank) acc += hist[dg++];
            sel[0] = dg;
            sel[1] = rank - acc;
        }
        __syncthreads();
        prefix |= (uint32_t)sel[0] << shift;
        mask |= 255u << shift;
        rank = sel[1];
        __syncthreads();
    }
    return prefix;
}

// One workgroup per query: sort the committed entries, find the k-th best
// computed distance, rescore every entry of the boundary band with the
// canonical recipe and emit the first k by (D, id).  A buffer longer than the
// LDS sort holds is first cut to the entries that can reach the band: the k-th
// smallest distance is found by radix select in global memory.  Every return
// is taken by the whole workgroup, and only thread 0 changes flags[q].
__device__ __forceinline__ void merge_query(const SearchConsts &c, uint64_t *__restrict__ buf,
                                            const int32_t *__restrict__ buf_cnt, int32_t *__restrict__ flags,
                                            const float *__restrict__ qE, const float *__restrict__ qA,
                                            const float *__restrict__ qraw, const float *__restrict__ raw, int d,
                                            int64_t *__restrict__ out_ids, float *__restrict__ out_d,
                                            unsigned long long *stats)
{
    // dynamic LDS: [MERGE_LDS_KEYS keys][d floats of the raw query]
    extern __shared__ uint64_t K[];
    __shared__ int nb_s;
    __shared__ int hist[256], sel[2];
    float *qrow = reinterpret_cast<float *>(K + MERGE_LDS_KEYS);
    const int64_t q = blockIdx.x;
    for (int j = threadIdx.x; j < d; j += NT) qrow[j] = qraw[q * d + j];
    const int n_all = buf_cnt[q];
    if ((flags[q] & FLAG_OVERFLOW) || n_all > c.capq) {
        if (threadIdx.x == 0) atomicOr(&flags[q], FLAG_OVERFLOW);
        return;
    }
    uint64_t *bq = buf + q * c.capq;
    int n = n_all;
    if ((flags[q] & FLAG_SEEDED) && n > c.k) {
        // the first k entries are the seeding's; the scan may have committed
        // the same candidates again (with another FP32 rounding of their
        // distance): drop those copies, in place, so that every candidate
        // counts once when the k-th distance and the band are taken
        __shared__ int32_t sid[128];
        __shared__ int wtmp[NT / 64];
        for (int i = threadIdx.x; i < c.k; i += NT) sid[i] = key_id(bq[i]);
        __syncthreads();
        int kept = c.k;
        for (int base = c.k; base < n; base += NT) {
            const int i = base + threadIdx.x;
            const uint64_t v = i < n ? bq[i] : KEY_MAX;
            bool keep = i < n;
            if (keep) {
                const int32_t id = key_id(v);
                for (int j = 0; j < c.k; ++j) keep = keep && sid[j] != id;
            }
            int tot;
            const int off = block_exclusive_scan(keep ? 1 : 0, wtmp, &tot);
            if (keep) bq[kept + off] = v;
            kept += tot;
            __syncthreads();
        }
        n = kept;
    }
    if (n > MERGE_LDS_KEYS) {
        const float dk = __uint_as_float(block_kth_dist_bits(bq, n, c.k, hist, sel));
        const float cut = prune_threshold(dk, qE[q], qA[q], c.mg, c.bfdelta);
        if (threadIdx.x == 0) nb_s = 0;
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += NT) {
            const uint64_t key = bq[i];
            if (dist_lower(key_dist(key), qA[q], c.mg, c.bfdelta) <= cut) {
                const int pos = atomicAdd(&nb_s, 1);
                if (pos < MERGE_LDS_KEYS) K[pos] = key;
            }
        }
        __syncthreads();
        n = nb_s;
        __syncthreads();
        if (n > MERGE_LDS_KEYS) {
            if (threadIdx.x == 0) atomicOr(&flags[q], FLAG_OVERFLOW);
            return;
        }
        const int P = next_pow2(n > 0 ? n : 1);
        for (int i = n + threadIdx.x; i < P; i += NT) K[i] = KEY_MAX;
        __syncthreads();
    } else {
        const int P = next_pow2(n > 0 ? n : 1);
        for (int i = threadIdx.x; i < P; i += NT) K[i] = i < n ? bq[i] : KEY_MAX;
        __syncthreads();
    }
    const int P = next_pow2(n > 0 ? n : 1);
    block_bitonic_sort(K, P);
    const float Aq = qA[q];
    const float thr = n >= c.k ? prune_threshold(key_dist(K[c.k - 1]), qE[q], Aq, c.mg, c.bfdelta) : INFINITY;
    if (threadIdx.x == 0) nb_s = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += NT)
        if (dist_lower(key_dist(K[i]), Aq, c.mg, c.bfdelta) <= thr) atomicMax(&nb_s, i + 1);
    __syncthreads();
    const int nb = nb_s;
    if (nb > MERGE_LDS_KEYS) {
        if (threadIdx.x == 0) atomicOr(&flags[q], FLAG_OVERFLOW);
        return;
    }
    // canonical rescoring of the band (the band is a prefix of the sort):
    // two rows per wavefront at a time (the last one alone)
    {
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        for (int i = 2 * wv; i < nb; i += 2 * (NT / 64)) {
            const int32_t id0 = key_id(K[i]);
            if (i + 1 < nb) {
                const int32_t id1 = key_id(K[i + 1]);
                float d0, d1;
                wave_canon_dist2(qrow, raw + (int64_t)id0 * d, raw + (int64_t)id1 * d, d, lane, d0, d1);
                if (lane == 0) {
                    K[i] = make_key(d0, id0);
                    K[i + 1] = make_key(d1, id1);
                }
            } else {
                const float dv = wave_canon_dist(qrow, raw + (int64_t)id0 * d, d, lane);
                if (lane == 0) K[i] = make_key(dv, id0);
            }
        }
    }
    const int PB = next_pow2(nb > 0 ? nb : 1);
    for (int i = nb + threadIdx.x; i < PB; i += NT) K[i] = KEY_MAX;
    __syncthreads();
    block_bitonic_sort(K, PB);
    // a candidate committed twice (by the seeding and by the scan) has the
    // same canonical key twice, next to each other: keep one
    if (threadIdx.x == 0) {
        int r = 0;
        for (int i = 0; i < nb && r < c.k; ++i) {
            if (i > 0 && K[i] == K[i - 1]) continue;
            out_ids[q * c.k + r] = key_id(K[i]);
            out_d[q * c.k + r] = key_dist(K[i]);
            ++r;
        }
        for (; r < c.k; ++r) {
            out_ids[q * c.k + r] = -1;
            out_d[q * c.k + r] = INFINITY;
        }
    }
    if (stats && threadIdx.x == 0) {
        atomicAdd(&stats[ST_COMMIT], (unsigned long long)n_all);
        atomicAdd(&stats[3], (unsigned long long)nb);
    }
}

// The merge kernel: one workgroup per query.  When hflags (pinned host memory
// of nq words) is given, each query's final flag word, with FLAG_NONFINITE
// set for a query that has a non-finite value, goes to hflags[q], so the
// host reads them after the stream completes without copies of its own.
__global__ __launch_bounds__(NT) void k_merge(SearchConsts c, uint64_t *__restrict__ buf,
                                              const int32_t *__restrict__ buf_cnt,
                                              int32_t *__restrict__ flags, const float *__restrict__ qE,
                                              const float *__restrict__ qA,
                                              const float *__restrict__ qraw, const float *__restrict__ raw,
                                              int d, int64_t *__restrict__ out_ids, float *__restrict__ out_d,
                                              unsigned long long *stats, int32_t *hflags,
                                              const int32_t *__restrict__ qbad)
{
    merge_query(c, buf, buf_cnt, flags, qE, qA, qraw, raw, d, out_ids, out_d, stats);
    if (hflags != nullptr && threadIdx.x == 0)
        hflags[blockIdx.x] = flags[blockIdx.x] | (qbad[blockIdx.x] ? FLAG_NONFINITE : 0);
}

// ================================================================ fallback
// Exact answer for one query by brute force with the canonical recipe:
// keys of every candidate of the probed lists, then k rounds of a
// workgroup-wide minimum above the previous key.
__global__ __launch_bounds__(NT) void k_fallback_keys(const float *__restrict__ q, int d,
                                                      const int32_t *__restrict__ lists, int nl,
                                                      const int64_t *__restrict__ list_blk, int B,
                                                      const int32_t *__restrict__ ids,
                                                      const int32_t *__restrict__ blk_cnt,
                                                      const float *__restrict__ raw, int64_t total,
                                                      uint64_t *__restrict__ keys)
{
    // grid-stride over the probed lists' blocks' slots
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = idx; t < total; t += stride) {
        // locate (list, slot): lists are visited in order; total counts slots
        int64_t rem = t;
        int li = 0;
        int64_t nslots = 0;
        for (; li < nl; ++li) {
            nslots = (list_blk[lists[li] + 1] - list_blk[lists[li]]) * B;
            if (rem < nslots) break;
            rem -= nslots;
        }
        const int64_t gb = list_blk[lists[li]] + rem / B;
        const int s = (int)(rem % B);
        if (s < blk_cnt[gb]) {
            const int32_t id = ids[gb * B + s];
            keys[t] = make_key(canon_dist(q, raw + (int64_t)id * d, d), id);
        } else {
            keys[t] = KEY_MAX;
        }
    }
}

__global__ __launch_bounds__(NT) void k_fallback_select(const uint64_t *__restrict__ keys, int64_t total, int k,
                                                        int64_t *__restrict__ out_ids, float *__restrict__ out_d)
{
    fallback_select_block(keys, total, k, out_ids, out_d);
}

// The exact fallback on the device, for searches that do not wait on the
// host: one workgroup checks the queries NT at a time; a query with a
// non-finite value gets (-1, +inf) and is counted in nonfinite[0]; a query
// whose result buffer overflowed gets the canonical distances of all its
// probed candidates (keys in `keys`, room for the largest probe set) and the
// k smallest of them.  Overflow is rare, so the queries that need it are
// handled one after another.
__global__ __launch_bounds__(NT) void k_fallback_device(int64_t nq, int k, int d, int np_max,
                                                        const int32_t *__restrict__ qflags,
                                                        const int32_t *__restrict__ qbad,
                                                        const int32_t *__restrict__ probes,
                                                        const int32_t *__restrict__ npq, const float *__restrict__ q,
                                                        const int64_t *__restrict__ list_blk, int B,
                                                        const int32_t *__restrict__ ids,
                                                        const int32_t *__restrict__ blk_cnt,
                                                        const float *__restrict__ raw, uint64_t *__restrict__ keys,
                                                        int64_t *__restrict__ out_ids, float *__restrict__ out_d,
                                                        unsigned long long *__restrict__ nonfinite)
{
    __shared__ int32_t todo[NT];
    __shared__ int ntodo;
    for (int64_t q0 = 0; q0 < nq; q0 += NT) {
        if (threadIdx.x == 0) ntodo = 0;
        __syncthreads();
        const int64_t qi = q0 + threadIdx.x;
        if (qi < nq) {
            if (qbad[qi]) {
                for (int r = 0; r < k; ++r) {
                    out_ids[qi * k + r] = -1;
                    out_d[qi * k + r] = INFINITY;
                }
                atomicAdd(nonfinite, 1ull);
            } else if (qflags[qi] & FLAG_OVERFLOW) {
                todo[atomicAdd(&ntodo, 1)] = (int32_t)threadIdx.x;
            }
        }
        __syncthreads();
        const int nt = ntodo;
        for (int j = 0; j < nt; ++j) {
            const int64_t qj = q0 + todo[j];
            const int npv = npq[qj];
            const int32_t *lists = probes + qj * np_max;
            int64_t total = 0;
            for (int li = 0; li < npv; ++li) {
                const int l = lists[li];
                const int64_t nslots = (list_blk[l + 1] - list_blk[l]) * B;
                for (int64_t t = threadIdx.x; t < nslots; t += NT) {
                    const int64_t gb = list_blk[l] + t / B;
                    const int sl = (int)(t % B);
                    uint64_t key = KEY_MAX;
                    if (sl < blk_cnt[gb]) {
                        const int32_t id = ids[gb * B + sl];
                        key = make_key(canon_dist(q + qj * d, raw + (int64_t)id * d, d), id);
                    }
                    keys[total + t] = key;
                }
                total += nslots;
            }
            __syncthreads();
            fallback_select_block(keys, total, k, out_ids + qj * k, out_d + qj * k);
            __syncthreads();
        }
    }
}


// Slots of a query's probe set (the exact fallback's key count), for callers
// that keep the probe list on the device.
__global__ void k_probe_slots(const int32_t *__restrict__ lists, int nl, const int64_t *__restrict__ list_blk, int B,
                              int64_t *__restrict__ total)
{
    __shared__ int64_t part[NT];
    int64_t t = 0;
    for (int i = threadIdx.x; i < nl; i += NT) t += (list_blk[lists[i] + 1] - list_blk[lists[i]]) * B;
    part[threadIdx.x] = t;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = part[0];
}

// ================================================================ refine
// Position of every row in the level-major blocks (block * B + slot), so that
// a scattered candidate id finds its level slices and tails.
__global__ void k_build_idpos(const int32_t *__restrict__ ids, const int32_t *__restrict__ blk_cnt, int64_t nblocks,
                              int B, int64_t *__restrict__ idpos)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nblocks * B) return;
    const int64_t gb = t / B;
    const int s = (int)(t % B);
    if (s < blk_cnt[gb]) idpos[ids[t]] = t;
}

// The point-centric form of Algorithm 1 (B = 1 in the paper's table of its
// two modes; Section 6.4, Refine): each query's own candidate ids, scattered
// over the index, taken in groups of 64 (one lane per candidate, the group's
// ids read in one sweep), each candidate refined level by level and dropped
// at its first level whose bound (Eq. 3 / Eq. 4 with the certified margin)
// exceeds the query's d_k; the survivors of a group update d_k before the
// next group (the first group runs without a threshold and seeds it, as the
// first k candidates seed the heap).  One wavefront per query.  Survivors
// that can still reach the final band are appended to the query's result
// buffer for the merge's canonical rescoring.
__global__ __launch_bounds__(NT) void k_refine(SearchConsts c, IndexView ix, QueryView qv, WorkView wk,
                                               const int64_t *__restrict__ cand, int kprime, int64_t nq,
                                               const int64_t *__restrict__ idpos, int64_t n)
{
    extern __shared__ __align__(16) float rdyn[];  // per wave: k best [k], sort buffer [next_pow2(k + 64)]
    const LevelGeom &g = c.g;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t qi = (int64_t)blockIdx.x * (NT / 64) + wv;
    if (qi >= nq) return;
    const int sbn = next_pow2(c.k + 64);
    float *kb = rdyn + (size_t)wv * (c.k + sbn);
    float *sb = kb + c.k;
    const int L = g.L;
    const float *qrow = qv.qy + qi * g.d_pad;
    const float *qt = qv.qtail + qi * L;
    const float Aq = qv.qA[qi], Eq = qv.qE[qi];
    const uint64_t below = (1ull << lane) - 1ull;
    float th = INFINITY;
    int cntk = 0;
    bool bad = false;
    for (int base = 0; base < kprime; base += 64) {
        const int ci = base + lane;
        const int64_t id = ci < kprime ? cand[qi * kprime + ci] : -1;
        bad |= id < -1 || id >= n;
        bool act = id >= 0 && id < n;
        const int64_t pos = act ? idpos[id] : 0;
        const int64_t gb = pos / g.B;
        const int ss = (int)(pos - gb * g.B);
        const float *blk = ix.levels + gb * (int64_t)g.B * g.d_pad;
        const float *tl = ix.tails + gb * (int64_t)g.B * L;
        float sh = 0.f;
        for (int lv = 0; lv < L; ++lv) {
            if (__ballot(act) == 0ull) break;
            const bool last = lv + 1 == L;
            const int w4 = g.wp[lv] >> 2;
            const float b = (act && !last) ? tl[(int64_t)(lv + 1) * g.B + ss] : 0.f;
            float part = 0.f;
            if (act) {
                for (int c0 = 0; c0 < w4; c0 += 4) {
                    float4 xs[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int cc = min(c0 + j, w4 - 1);
                        // level 1 is interleaved by groups of four dimensions,
                        // later levels are slot-contiguous
                        const int64_t o = lv == 0 ? ((int64_t)cc * g.B + ss) * 4
                                                  : (int64_t)g.B * g.mp[lv] + (int64_t)ss * g.wp[lv] + cc * 4;
                        xs[j] = *reinterpret_cast<const float4 *>(blk + o);
                    }
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        if (c0 + j < w4) {
                            const float4 q4 = *reinterpret_cast<const float4 *>(qrow + g.mp[lv] + (c0 + j) * 4);
                            const float t0 = q4.x - xs[j].x, t1 = q4.y - xs[j].y, t2 = q4.z - xs[j].z,
                                        t3 = q4.w - xs[j].w;
                            part = __builtin_fmaf(t0, t0, part);
                            part = __builtin_fmaf(t1, t1, part);
                            part = __builtin_fmaf(t2, t2, part);
                            part = __builtin_fmaf(t3, t3, part);
                        }
                    }
                }
            }
            sh += part;
            const float a = last ? 0.f : qt[lv + 1];
            const float err = c.mg.c_level[lv + 1] * fmaxf(sh, 0.f) + Aq;
            const float ct = c.mg.c_tail * (a + b) * (a + b);
            const bool pruned = pair_lower(sh, a, b, err, ct, c.one_m_eps2) > th;
            act = act && !pruned;
        }
        // commit the group's survivors: append those that can reach the final
        // band, keep the k best distances, refresh d_k
        const float D = act ? fmaxf(sh, 0.f) : 0.f;
        const bool keep = act && dist_lower(D, Aq, c.mg) <= th;
        const uint64_t bal = __ballot(keep);
        const int nk = __popcll(bal);
        if (nk == 0) continue;
        int bpos = 0;
        if (lane == 0) bpos = atomicAdd(&wk.buf_cnt[qi], nk);
        bpos = __shfl(bpos, 0, 64);
        const int rk = __popcll(bal & below);
        if (keep) {
            const int dst = bpos + rk;
            const int32_t rid = ix.ids[gb * g.B + ss];
            if (dst < c.capq) wk.buf[qi * c.capq + dst] = make_key(D, rid);
            else atomicOr(&wk.flags[qi], FLAG_OVERFLOW);
        }
        for (int j = lane; j < cntk; j += 64) sb[j] = kb[j];
        if (keep) sb[cntk + rk] = D;
        const int tn = cntk + nk;
        const int P2 = next_pow2(tn);
        for (int j = tn + lane; j < P2; j += 64) sb[j] = INFINITY;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        wave_bitonic_sort_f(sb, P2, lane);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        cntk = min(c.k, tn);
        for (int j = lane; j < cntk; j += 64) kb[j] = sb[j];
        if (cntk == c.k) th = fminf(th, prune_threshold(sb[c.k - 1], Eq, Aq, c.mg));
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
    if (__ballot(bad) != 0ull && lane == 0) atomicOr(&wk.flags[qi], FLAG_BADID);
}

// ================================================================ fixed scratch
// Device scratch of the allocation-free search: one array per GPU, in the
// code object, held until the process ends.  Host code never uses its name
// as an address: fixed_scratch() returns the device address that
// hipGetSymbolAddress reports for the current device.
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

// ================================================================ buffer clearing
__global__ void k_fill_multi(FillList f)
{
    for (int sgm = 0; sgm < f.m; ++sgm) {
        uint32_t *p = reinterpret_cast<uint32_t *>(f.p[sgm]);
        const uint32_t v = f.v[sgm];
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < f.n[sgm]; i += (int64_t)gridDim.x * blockDim.x)
            p[i] = v;
    }
}

}  // namespace pano

// ================================================================ host side
namespace pano {

static size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// Workgroups of NT threads that fit on one compute unit for this kernel and
// dynamic LDS (at least 1), cached per kernel and size.
static std::mutex g_occ_mu;
static int resident_blocks(const void *kern, size_t shm)
{
    static std::vector<std::pair<std::pair<const void *, size_t>, int>> cache;
    std::lock_guard<std::mutex> lk(g_occ_mu);
    for (auto &e : cache)
        if (e.first.first == kern && e.first.second == shm) return e.second;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, NT, shm) != hipSuccess || nb < 1) nb = 1;
    cache.push_back({{kern, shm}, nb});
    return nb;
}

static std::mutex g_fixed_mu;
static void *g_fixed_ptr[MAX_DEVICES];

void *fixed_scratch(int device)
{
    PANO_REQUIRE(device >= 0 && device < MAX_DEVICES, "device index out of range");
    std::lock_guard<std::mutex> lk(g_fixed_mu);
    if (!g_fixed_ptr[device]) {
        // the address of this device's copy of the array (the caller has
        // made `device` current)
        void *p = nullptr;
        PANO_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        PANO_REQUIRE(p != nullptr, "no device address for the fixed scratch");
        g_fixed_ptr[device] = p;
    }
    return g_fixed_ptr[device];
}

// Carves consecutive sub-buffers out of one device allocation.
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base((char *)b) {}
    template <class T> T *take(size_t count)
    {
        T *p = reinterpret_cast<T *>(base + off);
        off += align_up(sizeof(T) * std::max<size_t>(count, 1));
        return p;
    }
};

// Launch constants and scratch sizes of one search (no device work).
struct SearchPlan {
    size_t need[7];     // bytes of scratch slots 0..3 (4, 5 unused) and the bound on the exact
                        // fallback's key buffer (one query)
    bool wave;          // per-wave scan (every wavefront its own worker)
};

// Probe slots per query: nprobe_all (at most nlist) for a common probe count;
// for per-query counts, nprobe_all when positive (an upper bound the kernels
// clamp to), else nlist.
static int probe_cap(bool per_query_np, int nprobe_all, int nlist)
{
    if (per_query_np) return nprobe_all > 0 ? std::min(nprobe_all, nlist) : nlist;
    return std::min(nprobe_all, nlist);
}

static void plan_search(const pano_index *ix, int64_t nq, int k, bool per_query_np, int nprobe_all, float eps,
                        const pano_search_params *prm, bool brute, SearchConsts &c, SearchPlan &pl)
{
    // scan mode 3: every candidate's full distance, no pruning (the brute-force
    // scan), chosen by the tuner where the bounds prune too little to pay
    if (prm && prm->reserved[1] == 3) brute = true;
    PANO_REQUIRE(!prm || (prm->reserved[1] >= 0 && prm->reserved[1] <= 4 && prm->reserved[1] != 2),
                 "scan mode must be 0, 1, 3 or 4");
    PANO_REQUIRE(k <= 128, "k up to 128 is supported");
    const int d = ix->d, L = ix->L, nlist = ix->nlist;
    size_t *need = pl.need;
    c = SearchConsts{};
    c.k = k;
    // local top-k per query of a work item: its k best and their margin
    // band; the bfloat16 scan's wider bracket makes the band longer, so
    // it keeps at least 64
    const bool bf16_req = prm && prm->use_bf16;
    c.kc = next_pow2(std::max(2 * k, bf16_req ? 64 : 16));
    int G = 16;
    while (G > 1 && G * c.kc > 2048) G >>= 1;
    if (prm && prm->group > 0) G = std::min(prm->group, G);
    c.G = G;
    // scan mode: 0 or 1 = the workgroup scan (dense levels, per-pair walk
    // and local top-k per work item), 4 = the per-wave scan (every wavefront
    // its own worker, survivors appended to the result buffers)
    const int mode_req = prm ? prm->reserved[1] : 0;
    // the brute-force scan of bfloat16 tiles is an instance of the per-wave scan
    pl.wave = mode_req == 4 || (brute && bf16_req);
    // (the level-1 query slices are staged only by the pruned scan: the
    // brute-force instances keep the smaller layout and their occupancy)
    c.wl = wave_lds_layout(L, k, brute ? 0 : ix->wp[0]);
    // a query group meets at most 32 work items per list
    c.bpi = (prm && prm->blocks_per_item > 0) ? prm->blocks_per_item : 1;
    c.item_cap = 32;
    // Per-query result buffer: a work item of the workgroup scan publishes
    // about k entries (its local best k and their margin band), and a query
    // meets about nprobe * ceil(mean blocks per list / bpi) work items (at
    // most 32 per list); the per-wave scan appends its surviving pairs.
    // Twice the estimate, within [2048, 65536] and 4 GiB over the batch; a
    // query that still overflows takes the exact fallback.
    {
        const int np_est = per_query_np ? std::min(nlist, 128) : std::min(nprobe_all, nlist);
        const double mean_blk = (double)ix->list_blk.back() / std::max(1, nlist);
        const double items = (double)np_est * (std::min(32.0, std::ceil(mean_blk / c.bpi)) + 1.0);
        const double want = 2.0 * items * (k + 8);
        int64_t cap = 2048;
        while (cap < want && cap < 65536) cap <<= 1;
        while (cap > 2048 && (double)cap * 8.0 * (double)nq > 4.0 * 1073741824.0) cap >>= 1;
        c.capq = (int)cap;
    }
    c.nlist = nlist;
    c.ceil8 = (nlist + 7) / 8;
    c.prune = brute ? 0 : 1;
    c.dense_min = (prm && prm->reserved[0] > 0) ? prm->reserved[0] : 64;
    c.walk_lanes = prm ? prm->reserved[2] : 0;
    {
        // two levels per step of the walk (four lanes per pair) when every
        // level has at most 64 dimensions, unless one level per step is asked
        int wmax = 0;
        for (int l = 0; l < L; ++l) wmax = std::max(wmax, ix->wp[l]);
        const int step = prm ? prm->reserved[3] : 0;
        PANO_REQUIRE(step >= 0 && step <= 2, "walk levels per step must be 0, 1 or 2");
        c.walk2 = (wmax <= 64 && step != 1) ? 1 : 0;
    }
    PANO_REQUIRE(c.walk_lanes == 0 || c.walk_lanes == 1 || c.walk_lanes == 2 || c.walk_lanes == 4,
                 "walk lanes per pair must be 0, 1, 2 or 4");
    c.eps = eps;
    c.one_m_eps2 = 2.f * (1.f - eps);
    c.mg = ix->mg;
    const bool use_bf16 = prm && prm->use_bf16;
    PANO_REQUIRE(!use_bf16 || ix->has_bf16, "bfloat16 search needs an index built with PANO_BF16");
    c.bf16 = use_bf16 ? 1 : 0;
    c.ub = (float)(std::ldexp(1.0, -8) * (1.0 + 1e-6));
    // committed distances of the bfloat16 scan are to the rounded rows; their
    // bracket widens by u_b max ||x|| on the square root
    c.bfdelta = use_bf16 ? (float)((double)c.ub * std::sqrt((double)ix->mg.b0max2) * (1.0 + 1e-6) + 1e-37) : 0.f;
    c.g = LevelGeom{};
    c.g.L = L;
    c.g.d = d;
    c.g.d_pad = ix->d_pad;
    c.g.B = ix->B;
    for (int l = 0; l <= L; ++l) c.g.mp[l] = ix->mp[l];
    for (int l = 0; l < L; ++l) c.g.wp[l] = ix->wp[l];
    const int np_max = probe_cap(per_query_np, nprobe_all, nlist);
    need[0] = align_up(sizeof(float) * nq * ix->d_pad) + align_up(sizeof(float) * nq * L) +
              3 * align_up(sizeof(float) * nq) + align_up(sizeof(double) * nq);
    need[1] = nlist > 1 ? align_up(sizeof(float) * nq * nlist) : 256;
    need[2] = align_up(sizeof(int32_t) * nq * np_max) * 2 + align_up(sizeof(int32_t) * nq) +
              2 * align_up(sizeof(int32_t) * nlist) + align_up(sizeof(int32_t) * 8) +
              align_up(sizeof(int64_t) * (nlist + 1)) + align_up(sizeof(int64_t) * (8 * c.ceil8 + 1));
    need[3] = 4 * align_up(sizeof(float) * nq) + align_up(sizeof(uint64_t) * nq * c.capq) +
              align_up(sizeof(unsigned long long) * 128);
    need[4] = need[5] = 0;
    {
        // the exact fallback of one query: its probed list ids and one 64-bit
        // key per slot of its probe set, at most the np_max largest lists
        const int64_t s_np = ix->top_blk_prefix[std::min<int64_t>(np_max, nlist)];
        need[6] = align_up(sizeof(int32_t) * (size_t)std::max(1, np_max)) +
                  align_up(sizeof(uint64_t) * (size_t)std::max<int64_t>(1, s_np * ix->B));
    }
}

size_t search_scratch_bytes(const pano_index *ix, int64_t nq, int k, bool per_query_np, int nprobe_all,
                            const pano_search_params *prm, bool brute)
{
    SearchConsts c;
    SearchPlan pl;
    plan_search(ix, nq, k, per_query_np, nprobe_all, 1.f, prm, brute, c, pl);
    size_t t = 0;
    for (int i = 0; i < 7; ++i) t += pl.need[i];
    return t;
}

size_t search_fixed_bytes(const pano_index *ix, int64_t nq, int k, bool per_query_np, int nprobe_all,
                          const pano_search_params *prm)
{
    SearchConsts c;
    SearchPlan pl;
    plan_search(ix, nq, k, per_query_np, nprobe_all, 1.f, prm, false, c, pl);
    size_t t = align_up(sizeof(int32_t) * (size_t)std::max<int64_t>(1, nq)) + align_up(sizeof(int64_t));
    for (int i = 0; i < 7; ++i) t += pl.need[i];
    return t;
}

// The allocation-free search after planning: every kernel on the caller's
// stream s, then the per-query flag words read back through a buffer on the
// stack, and the exact fallback for flagged queries with its keys in the
// fixed scratch (fb_keys, fb_bytes) and its probe list read on the device.
template <class Enqueue>
static void run_fixed_tail(pano_index *ix, const float *q, int64_t nq, int k, int d, int np_max, int64_t *ids,
                           float *dists, const int32_t *probes, const int32_t *npq, const int32_t *flags_dev,
                           int64_t *fb_total, void *fb_keys, size_t fb_bytes, hipStream_t s, Enqueue enqueue)
{
    enqueue(s);
    PANO_HIP(hipGetLastError());
    constexpr int CH = 1024;
    int32_t hf[CH];
    for (int64_t c0 = 0; c0 < nq; c0 += CH) {
        const int64_t cn = std::min<int64_t>(CH, nq - c0);
        PANO_HIP(hipMemcpyAsync(hf, flags_dev + c0, sizeof(int32_t) * cn, hipMemcpyDeviceToHost, s));
        PANO_HIP(hipStreamSynchronize(s));
        for (int64_t i = 0; i < cn; ++i) PANO_REQUIRE(!(hf[i] & FLAG_NONFINITE), "a query has a non-finite value");
        for (int64_t i = 0; i < cn; ++i) {
            if (!(hf[i] & FLAG_OVERFLOW)) continue;
            const int64_t qi = c0 + i;
            int32_t npv = 0;
            PANO_HIP(hipMemcpyAsync(&npv, npq + qi, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            PANO_HIP(hipStreamSynchronize(s));
            const int32_t *lists = probes + qi * np_max;
            hipLaunchKernelGGL(k_probe_slots, dim3(1), dim3(NT), 0, s, lists, npv, ix->list_blk_d.as<int64_t>(),
                               ix->B, fb_total);
            int64_t total = 0;
            PANO_HIP(hipMemcpyAsync(&total, fb_total, sizeof(int64_t), hipMemcpyDeviceToHost, s));
            PANO_HIP(hipStreamSynchronize(s));
            PANO_REQUIRE((size_t)std::max<int64_t>(1, total) * sizeof(uint64_t) <= fb_bytes,
                         "fallback keys exceed the fixed scratch");
            uint64_t *keys = reinterpret_cast<uint64_t *>(fb_keys);
            unsigned gr = (unsigned)std::min<int64_t>(4096, std::max<int64_t>(1, (total + NT - 1) / NT));
            hipLaunchKernelGGL(k_fallback_keys, dim3(gr), dim3(NT), 0, s, q + qi * d, d, lists, npv,
                               ix->list_blk_d.as<int64_t>(), ix->B, ix->ids.as<int32_t>(), ix->blk_cnt.as<int32_t>(),
                               ix->raw.as<float>(), total, keys);
            hipLaunchKernelGGL(k_fallback_select, dim3(1), dim3(NT), 0, s, keys, total, k, ids + qi * k,
                               dists + qi * k);
            PANO_HIP(hipGetLastError());
            PANO_HIP(hipStreamSynchronize(s));
        }
    }
}

void run_search(pano_ctx *ctx, pano_index *ix, const float *q, int64_t nq, int k, const int32_t *nprobe_dev,
                int nprobe_all, float eps, int64_t *ids, float *dists, const pano_search_params *prm,
                uint32_t flags, bool brute, hipStream_t s, void *fixed, size_t fixed_bytes)
{
    PANO_REQUIRE(ctx->device == ix->ctx->device, "context and index are on different devices");
    PANO_HIP(hipSetDevice(ctx->device));
    if (prm && prm->reserved[1] == 3) brute = true;  // scan mode 3: no pruning
    const bool wave = (prm && prm->reserved[1] == 4) || (brute && prm && prm->use_bf16);
    const int d = ix->d, L = ix->L, nlist = ix->nlist;
    SearchConsts c;
    SearchPlan pl;
    plan_search(ix, nq, k, nprobe_dev != nullptr, nprobe_all, eps, prm, brute, c, pl);
    const size_t *need = pl.need;
    const bool use_bf16 = c.bf16 != 0;
    // Absolute margin of the dot-product form: the bfloat16 scan splits each
    // query value into two bfloat16 terms and reads rows of norm up to
    // (1 + u_b) ||x||, which its own constant covers.
    Margins mq = ix->mg;
    if (use_bf16) {
        mq.c_abs = ix->c_abs_bf;
        mq.b0max2 = (float)((double)ix->mg.b0max2 * (1.0 + std::ldexp(1.0, -8)) * (1.0 + std::ldexp(1.0, -8)) *
                            (1.0 + 1e-6));
    }
    const int seed_pool = std::min(1024, (prm && prm->seed_pool > 0) ? prm->seed_pool : 512);
    const int seed_cnt = std::min(256, std::max(k, (prm && prm->seed_count > 0) ? prm->seed_count : std::max(2 * k, 32)));
    const int grid = (prm && prm->grid > 0) ? prm->grid : ctx->num_cu * (brute ? 2 : 3);
    const int np_max = probe_cap(nprobe_dev != nullptr, nprobe_all, nlist);
    const bool want_stats = (flags & PANO_SEARCH_STATS) != 0;
    const bool want_timing = !want_stats && (flags & PANO_SEARCH_TIMING) != 0;
    // a search that does not wait: the exact fallback runs on the device and
    // non-finite queries are counted for pano_ctx_status
    const bool async_mode = (flags & PANO_SEARCH_ASYNC) != 0;
    PANO_REQUIRE(!async_mode || (!want_stats && !want_timing && !fixed),
                 "an asynchronous search takes no stats or timing flags");
    // the seeding starts every scan's threshold, the brute-force scan's too
    // (it then commits fewer candidates; every distance is still computed),
    // and at eps < 1 as well: its k best are committed, so the threshold
    // stands on candidates of the answer set even if the relaxed bound
    // prunes them in the scan
    const bool seed_on = true;
    // ---- scratch: the context's buffers (grown on demand), or consecutive
    // regions of the caller's fixed memory
    const size_t need0 = need[0], need1 = need[1], need2 = need[2], need3 = need[3];
    void *sp[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    int32_t *flags_dev = nullptr;
    int64_t *fb_total = nullptr;
    if (fixed) {
        PANO_REQUIRE((flags & (PANO_SEARCH_STATS | PANO_SEARCH_TIMING)) == 0,
                     "the allocation-free search takes no stats or timing flags");
        const size_t want = search_fixed_bytes(ix, nq, k, nprobe_dev != nullptr, nprobe_all, prm);
        if (want > fixed_bytes)
            throw Error{PANO_EINVAL, "this search needs " + std::to_string(want) +
                                         " bytes of scratch; the allocation-free search has " +
                                         std::to_string(fixed_bytes) + " (fewer queries per call fit)"};
        Carver cf(fixed);
        sp[0] = cf.take<char>(need0);
        sp[1] = cf.take<char>(need1);
        sp[2] = cf.take<char>(need2);
        sp[3] = cf.take<char>(need3);
        sp[4] = cf.take<char>(need[6]);
        flags_dev = cf.take<int32_t>(nq);
        fb_total = cf.take<int64_t>(1);
    } else {
        // a search is ordered after the context's last asynchronous one (they
        // share its scratch), and buffers that must grow wait for it to end
        if (ctx->async_pending) {
            PANO_HIP(hipStreamWaitEvent(s, ctx->ev_async, 0));
            if (need0 > ctx->scratch[0].bytes || need1 > ctx->scratch[1].bytes || need2 > ctx->scratch[2].bytes ||
                need3 > ctx->scratch[3].bytes || (async_mode && need[6] > ctx->scratch[4].bytes) ||
                sizeof(int32_t) * (size_t)nq > ctx->pinned_bytes)
                ctx->quiesce();
        }
        ctx->scratch[0].ensure(need0);
        ctx->scratch[1].ensure(need1);
        ctx->scratch[2].ensure(need2);
        ctx->scratch[3].ensure(need3);
        for (int i = 0; i < 4; ++i) sp[i] = ctx->scratch[i].p;
        if (async_mode) {
            ctx->scratch[4].ensure(need[6]);
            sp[4] = ctx->scratch[4].p;
            ctx->status_ensure();
        }
    }
    Carver c0(sp[0]), c2(sp[2]), c3(sp[3]);
    float *qy = c0.take<float>(nq * ix->d_pad);
    float *qtail = c0.take<float>(nq * L);
    float *qE = c0.take<float>(nq);
    float *qA = c0.take<float>(nq);
    int32_t *qbad = c3.take<int32_t>(nq);
    double *vnorm = c0.take<double>(nq);
    float *qn2 = c0.take<float>(nq);
    float *Sco = reinterpret_cast<float *>(sp[1]);
    int32_t *probes = c2.take<int32_t>(nq * np_max);
    int32_t *list_q = c2.take<int32_t>(nq * np_max);
    int32_t *npq = c2.take<int32_t>(nq);
    int32_t *list_cnt = c2.take<int32_t>(nlist);
    int32_t *list_fill = c2.take<int32_t>(nlist);
    int32_t *heads = c2.take<int32_t>(8);
    int64_t *list_qoff = c2.take<int64_t>(nlist + 1);
    int64_t *item_off = c2.take<int64_t>(8 * c.ceil8 + 1);
    float *thr = c3.take<float>(nq);
    int32_t *buf_cnt = c3.take<int32_t>(nq);
    int32_t *qflags = c3.take<int32_t>(nq);
    uint64_t *buf = c3.take<uint64_t>(nq * c.capq);
    unsigned long long *stats = c3.take<unsigned long long>(128);

    // ---- launch geometry that does not depend on the stream
    const CoarsePlan coarse = coarse_prepare(nlist, d);
    const float c_co = coarse.c_co;
    const size_t merge_shm = sizeof(uint64_t) * MERGE_LDS_KEYS + sizeof(float) * (size_t)d;
    const size_t scan_shm = wave ? (size_t)(NT / 64) * c.wl.bytes
                                 : sizeof(uint64_t) * (4 * (size_t)next_pow2(c.kc + 64) + (size_t)c.G * c.kc);
    PANO_HIP(hipFuncSetAttribute((const void *)k_merge, hipFuncAttributeMaxDynamicSharedMemorySize, (int)merge_shm));
    // query groups ordered by distance to the list (reserved[4] = 1 keeps the
    // arrival order), in chunks of WL_SORT_CHUNK queries
    const bool sort_groups = nlist > 1 && !(prm && prm->reserved[4] == 1) && nq > c.G;
    const int sort_chunks = (int)std::min<int64_t>((nq + WL_SORT_CHUNK - 1) / WL_SORT_CHUNK, 65535);
    // the per-wave scan instance of this search (and its counting twin)
    typedef void (*ScanKernel)(SearchConsts, IndexView, QueryView, WorkView);
    const bool relaxed = eps < 1.f;
    const ScanKernel wave_kern =
        brute ? (use_bf16 ? k_scan_wave_brute_bf16 : k_scan_wave_brute)
              : (use_bf16 ? (relaxed ? k_scan_wave_bf16_relaxed : k_scan_wave_bf16)
                          : (relaxed ? k_scan_wave_relaxed : k_scan_wave));
    const ScanKernel wave_kern_stats =
        brute ? (use_bf16 ? k_scan_wave_brute_bf16_stats : k_scan_wave_brute_stats)
              : (use_bf16 ? (relaxed ? k_scan_wave_bf16_relaxed_stats : k_scan_wave_bf16_stats)
                          : (relaxed ? k_scan_wave_relaxed_stats : k_scan_wave_stats));
    if (wave) {
        PANO_REQUIRE(scan_shm <= 160 * 1024, "k and L too large for the per-wave scan's LDS");
        PANO_HIP(hipFuncSetAttribute((const void *)wave_kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)scan_shm));
        PANO_HIP(hipFuncSetAttribute((const void *)wave_kern_stats, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)scan_shm));
    }
    // per-query flag words written by the merge: pinned host memory, or the
    // fixed scratch (read back in chunks)
    int32_t *h_flags = flags_dev;
    if (!fixed) {
        ctx->pinned_ensure(sizeof(int32_t) * nq);
        h_flags = reinterpret_cast<int32_t *>(ctx->pinned);
    }
    IndexView iv{ix->levels.as<float>(), ix->has_bf16 ? ix->levels_bf16.as<uint16_t>() : nullptr, ix->tails.as<float>(), ix->ids.as<int32_t>(), ix->blk_cnt.as<int32_t>(),
                 ix->list_blk_d.as<int64_t>(), ix->raw.as<float>()};
    QueryView qv{qy, qtail, qE, qA, q};
    WorkView wk{list_cnt, list_qoff, list_q, item_off, heads, thr, buf, buf_cnt, qflags, nullptr};

    // Every device step of one search, on stream st (and, with seeding, two
    // more branches).  No memset nodes: buffers are cleared by kernels so the
    // sequence can be captured into a graph.  The products kernel clears the
    // counters, thresholds and flags in a prologue (every later kernel may
    // use them); the transformed queries are cleared beforehand only when the
    // levels have padding columns, which the transform does not write.
    //
    // After the products the search forks three ways: the coarse probing and
    // the work decomposition on st, the threshold seeding on the context's
    // second stream and the row norms (tails, E_q, A_q, needed from the scan
    // on) on its third; both side branches join st before the scan.  Seeding
    // runs only for the exact bound: a seed's own relaxed bound (eps < 1) may
    // exceed its distance, so the scan could prune the very candidates that
    // set d_k and return fewer than k; without seeding, every d_k comes from
    // committed candidates.
    auto enqueue = [&](hipStream_t st, bool stats_on, bool events_on) {
        FillList fl{};
        fl.add(list_cnt, nlist, 0u);
        fl.add(list_fill, nlist, 0u);
        fl.add(heads, 8, 0u);
        fl.add(thr, nq, 0x7f800000u);
        fl.add(buf_cnt, nq, 0u);
        fl.add(qflags, nq, 0u);
        if (stats_on) fl.add(stats, 256, 0u);
        if (ix->d_pad != ix->d) {
            FillList fq{};
            fq.add(qy, nq * (int64_t)ix->d_pad, 0u);
            hipLaunchKernelGGL(k_fill_multi, dim3(256), dim3(256), 0, st, fq);
        }
        // query transform and query x centroid products in one launch (their
        // tiles run side by side)
        {
            const GemmJob jt = transform_job(q, nq, d, ix->T32.as<float>(), ix->mu32.as<float>(),
                                             ix->meta.as<int32_t>(), qy, ix->d_pad);
            if (nlist > 1) {
                const GemmJob jc = product_job(q, nq, d, ix->cent.as<float>(), nlist, Sco);
                launch_gemm_jobs(jt, &jc, st, &fl);
            } else {
                launch_gemm_jobs(jt, nullptr, st, &fl);
            }
        }
        // the transformed queries' tails and error bounds
        auto row_norms = [&](hipStream_t rs_) {
            QueryConstsOut qc;
            qc.mg = mq;
            qc.qE = qE;
            qc.qA = qA;
            qc.badq = qbad;
            launch_row_norms(qy, nq, c.g, q, ix->mu32.as<float>(), qtail, vnorm, rs_, &qc);
        };
        // the allocation-free search runs every kernel on st, in order
        const bool fork = seed_on && !fixed;
        hipStream_t sa = fork ? ctx->aux : st, sb = fork ? ctx->aux2 : st;
        if (fork) {
            PANO_HIP(hipEventRecord(ctx->ev_fork, st));
        } else {
            row_norms(st);
        }
        // the seeding, the longest branch, is launched first so that its waves
        // are dispatched first
        if (seed_on) {
            if (fork) PANO_HIP(hipStreamWaitEvent(sa, ctx->ev_fork, 0));
            hipLaunchKernelGGL(k_seed, dim3((unsigned)nq), dim3(NT), seed_lds_bytes(seed_pool, c.g.d_pad), sa, c, iv,
                               qv, Sco, ix->cent.as<float>() + (size_t)nlist * d, d, nlist, nprobe_dev, nprobe_all,
                               np_max, c_co, ix->list_len_d.as<int64_t>(), seed_pool, seed_cnt,
                               ix->mu32.as<float>(), mq.c_abs, mq.b0max2, thr, buf, buf_cnt, c.capq, qflags);
            if (fork) PANO_HIP(hipEventRecord(ctx->ev_join, sa));
        }
        // coarse probing (and the number of queries per list)
        coarse_enqueue(coarse, Sco, ix->cent.as<float>() + (size_t)nlist * d, q, ix->cent.as<float>(), nq, nprobe_dev,
                       nprobe_all, np_max, probes, npq, list_cnt, qn2, st);
        if (fork) {
            PANO_HIP(hipStreamWaitEvent(sb, ctx->ev_fork, 0));
            row_norms(sb);
            PANO_HIP(hipEventRecord(ctx->ev_join2, sb));
        }
        // work decomposition
        // one launch when the fill grid is small (every fill workgroup derives
        // the offsets itself); else the offsets once, then the fill
        const unsigned wl_grid = (unsigned)((nq * np_max + 255) / 256);
        if (nlist <= WL_FUSED_LISTS && (int64_t)wl_grid * nlist <= (int64_t)1 << 21) {
            hipLaunchKernelGGL(k_wl_fill_fused, dim3(wl_grid), dim3(NT), sizeof(int32_t) * (size_t)(nlist + 1), st, nq,
                               np_max, probes, npq, nlist, c.ceil8, c.G, c.bpi, c.item_cap, list_cnt,
                               ix->list_blk_d.as<int64_t>(), list_qoff, item_off, list_fill, list_q);
        } else {
            hipLaunchKernelGGL(k_wl_offsets, dim3(1), dim3(NT), 0, st, nlist, c.ceil8, c.G, c.bpi, c.item_cap,
                               list_cnt, ix->list_blk_d.as<int64_t>(), list_qoff, item_off);
            hipLaunchKernelGGL(k_wl_fill, dim3(wl_grid), dim3(256), 0, st, nq, np_max, probes, npq, list_qoff,
                               list_fill, list_q);
        }
        if (sort_groups)
            hipLaunchKernelGGL(k_wl_sort, dim3((unsigned)nlist, (unsigned)sort_chunks), dim3(NT), 0, st, nlist,
                               list_cnt, list_qoff, list_q, Sco, qn2, ix->cent.as<float>() + (size_t)nlist * d);
        if (fork) {
            PANO_HIP(hipStreamWaitEvent(st, ctx->ev_join, 0));
            PANO_HIP(hipStreamWaitEvent(st, ctx->ev_join2, 0));
        }
        if (events_on) PANO_HIP(hipEventRecord(ctx->ev[1], st));
        WorkView w2 = wk;
        w2.stats = stats_on ? stats : nullptr;
        if (wave) {
            auto kern = stats_on ? wave_kern_stats : wave_kern;
            const int wgrid = (prm && prm->grid > 0) ? prm->grid : ctx->num_cu * resident_blocks((const void *)kern, scan_shm);
            hipLaunchKernelGGL(kern, dim3(wgrid), dim3(NT), scan_shm, st, c, iv, qv, w2);
        } else if (brute) {
            if (stats_on)
                hipLaunchKernelGGL(k_scan_brute_stats, dim3(grid), dim3(NT), scan_shm, st, c, iv, qv, w2);
            else
                hipLaunchKernelGGL(k_scan_brute, dim3(grid), dim3(NT), scan_shm, st, c, iv, qv, w2);
        } else if (use_bf16) {
            if (stats_on)
                hipLaunchKernelGGL(k_scan_pruned_bf16_stats, dim3(grid), dim3(NT), scan_shm, st, c, iv, qv, w2);
            else
                hipLaunchKernelGGL(k_scan_pruned_bf16, dim3(grid), dim3(NT), scan_shm, st, c, iv, qv, w2);
        } else {
            if (stats_on)
                hipLaunchKernelGGL(k_scan_pruned_stats, dim3(grid), dim3(NT), scan_shm, st, c, iv, qv, w2);
            else
                hipLaunchKernelGGL(k_scan_pruned, dim3(grid), dim3(NT), scan_shm, st, c, iv, qv, w2);
        }
        if (events_on) PANO_HIP(hipEventRecord(ctx->ev[2], st));
        hipLaunchKernelGGL(k_merge, dim3((unsigned)nq), dim3(NT), merge_shm, st, c, buf, buf_cnt, qflags, qE, qA, q,
                           ix->raw.as<float>(), d, ids, dists, stats_on ? stats : nullptr, async_mode ? nullptr : h_flags,
                           qbad);
        if (async_mode) {
            Carver c4(sp[4]);
            (void)c4.take<int32_t>(std::max(1, np_max));
            hipLaunchKernelGGL(k_fallback_device, dim3(1), dim3(NT), 0, st, nq, k, d, np_max, qflags, qbad, probes, npq,
                               q, ix->list_blk_d.as<int64_t>(), ix->B, ix->ids.as<int32_t>(), ix->blk_cnt.as<int32_t>(),
                               ix->raw.as<float>(), c4.take<uint64_t>(1), ids, dists,
                               reinterpret_cast<unsigned long long *>(ctx->status.p));
        }
        if (events_on) PANO_HIP(hipEventRecord(ctx->ev[3], st));
        PANO_HIP(hipGetLastError());
    };

    // A graph is captured on the context's own stream (the caller's may be
    // the null stream, which cannot be captured) and launched on the
    // caller's stream, so it is ordered after the caller's work without an
    // event.  Eager searches run on the context's stream, ordered after the
    // caller's by an event.
    if (fixed) {
        run_fixed_tail(ix, q, nq, k, d, np_max, ids, dists, probes, npq, h_flags, fb_total, sp[4], need[6], s,
                       [&](hipStream_t st) { enqueue(st, false, false); });
        return;
    }
    hipStream_t ws = ctx->work_stream();
    hipStream_t rs = ws;  // the stream the search ran on
    const bool use_graph = !want_stats && !want_timing && !(flags & PANO_SEARCH_EAGER);
    if (!use_graph) {
        PANO_HIP(hipEventRecord(ctx->ev_in, s));
        PANO_HIP(hipStreamWaitEvent(ws, ctx->ev_in, 0));
    }
    if (want_stats || want_timing) {
        PANO_HIP(hipEventRecord(ctx->ev[0], ws));
        enqueue(ws, want_stats, true);
    } else if (use_graph) {
        GraphKey key{ix->serial, q, nq, k, nprobe_dev, nprobe_all, eps, brute, ids, dists, c.G, c.bpi, seed_pool, seed_cnt, grid,
                     c.dense_min, c.bf16, (wave ? 2 : 0) | (sort_groups ? 4 : 0) | (async_mode ? 8 : 0), c.walk_lanes, c.walk2, ctx->scratch[0].p, ctx->scratch[1].p, ctx->scratch[2].p, ctx->scratch[3].p,
                     async_mode ? sp[4] : nullptr, async_mode ? ctx->status.p : nullptr, ctx->pinned};
        if (!ctx->graph_exec || !(ctx->graph_key == key)) {
            ctx->drop_graph();
            hipGraph_t graph;
            PANO_HIP(hipStreamBeginCapture(ws, hipStreamCaptureModeThreadLocal));
            try {
                enqueue(ws, false, false);
            } catch (...) {
                hipGraph_t dummy;
                (void)hipStreamEndCapture(ws, &dummy);
                throw;
            }
            PANO_HIP(hipStreamEndCapture(ws, &graph));
            hipError_t ie = hipGraphInstantiate(&ctx->graph_exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            PANO_HIP(ie);
            ctx->graph_key = key;
        }
        PANO_HIP(hipGraphLaunch(ctx->graph_exec, s));
        rs = s;
    } else {
        enqueue(ws, false, false);
    }
    if (async_mode) {
        // ordered on the caller's stream (graph) or after it (eager); results
        // are complete in stream order, nothing waits here
        if (!use_graph) {
            PANO_HIP(hipEventRecord(ctx->ev_in, ws));
            PANO_HIP(hipStreamWaitEvent(s, ctx->ev_in, 0));
        }
        PANO_HIP(hipEventRecord(ctx->ev_async, s));
        ctx->async_pending = true;
        return;
    }
    PANO_HIP(hipStreamSynchronize(rs));
    std::vector<int32_t> hflags(h_flags, h_flags + nq);
    for (int64_t qi = 0; qi < nq; ++qi)
        PANO_REQUIRE(!(hflags[qi] & FLAG_NONFINITE), "a query has a non-finite value");
    s = ws;
    // ---- exact fallback for queries whose bounded buffers overflowed

    int64_t nfall = 0;
    for (int64_t qi = 0; qi < nq; ++qi) {
        if (!(hflags[qi] & FLAG_OVERFLOW)) continue;
        ++nfall;
        std::vector<int32_t> pr(np_max);
        int32_t npv = 0;
        PANO_HIP(hipMemcpyAsync(pr.data(), probes + qi * np_max, sizeof(int32_t) * np_max, hipMemcpyDeviceToHost, s));
        PANO_HIP(hipMemcpyAsync(&npv, npq + qi, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        PANO_HIP(hipStreamSynchronize(s));
        int64_t total = 0;
        for (int r = 0; r < npv; ++r) total += (ix->list_blk[pr[r] + 1] - ix->list_blk[pr[r]]) * ix->B;
        ctx->scratch[4].ensure(align_up(sizeof(int32_t) * std::max(1, npv)) + align_up(sizeof(uint64_t) * std::max<int64_t>(1, total)));
        Carver c4(ctx->scratch[4].p);
        int32_t *lists_d = c4.take<int32_t>(std::max(1, npv));
        uint64_t *keys = c4.take<uint64_t>(std::max<int64_t>(1, total));
        PANO_HIP(hipMemcpyAsync(lists_d, pr.data(), sizeof(int32_t) * npv, hipMemcpyHostToDevice, s));
        unsigned gr = (unsigned)std::min<int64_t>(4096, std::max<int64_t>(1, (total + NT - 1) / NT));
        hipLaunchKernelGGL(k_fallback_keys, dim3(gr), dim3(NT), 0, s, q + qi * d, d, lists_d, npv,
                           ix->list_blk_d.as<int64_t>(), ix->B, ix->ids.as<int32_t>(), ix->blk_cnt.as<int32_t>(),
                           ix->raw.as<float>(), total, keys);
        hipLaunchKernelGGL(k_fallback_select, dim3(1), dim3(NT), 0, s, keys, total, k, ids + qi * k, dists + qi * k);
        PANO_HIP(hipGetLastError());
        PANO_HIP(hipStreamSynchronize(s));
    }
    if (want_timing) {
        PANO_HIP(hipEventRecord(ctx->ev[4], s));
        PANO_HIP(hipEventSynchronize(ctx->ev[4]));
        pano_stats_t &st = ix->stats;
        float t;
        PANO_HIP(hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[4]));
        st.ms_total = t;
        PANO_HIP(hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[1]));
        st.ms_prep = t;
        PANO_HIP(hipEventElapsedTime(&t, ctx->ev[1], ctx->ev[2]));
        st.ms_scan = t;
        PANO_HIP(hipEventElapsedTime(&t, ctx->ev[2], ctx->ev[3]));
        st.ms_merge = t;
    }
    if (want_stats) {
        PANO_HIP(hipEventRecord(ctx->ev[4], s));
        PANO_HIP(hipEventSynchronize(ctx->ev[4]));
        std::vector<unsigned long long> hs(128);
        PANO_HIP(hipMemcpy(hs.data(), stats, sizeof(unsigned long long) * 128, hipMemcpyDeviceToHost));
        pano_stats_t &st = ix->stats;
        std::memset(&st, 0, sizeof(st));
        st.nq = nq;
        st.items = (int64_t)hs[ST_ITEMS];
        st.committed = (int64_t)hs[ST_COMMIT];
        st.band = (int64_t)hs[3];
        st.scan_bytes = (int64_t)hs[ST_BYTES];
        st.fallback_queries = nfall;
        int64_t dims = 0;
        for (int l = 0; l < L && l < 64; ++l) {
            st.level_reads[l] = (int64_t)hs[ST_LEVEL + l];
            dims += st.level_reads[l] * (int64_t)(ix->m[l + 1] - ix->m[l]);
        }
        st.candidates = st.level_reads[0];
        st.dims_read = dims;
        float t;
        PANO_HIP(hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[4]));
        st.ms_total = t;
        PANO_HIP(hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[1]));
        st.ms_prep = t;
        PANO_HIP(hipEventElapsedTime(&t, ctx->ev[1], ctx->ev[2]));
        st.ms_scan = t;
        PANO_HIP(hipEventElapsedTime(&t, ctx->ev[2], ctx->ev[3]));
        st.ms_merge = t;
        for (int i = 0; i < 6; ++i) st.scan_cycles[i] = (int64_t)hs[ST_CYCLES + i];
    }
}


// Refine (the point-centric scan of given candidate ids): query transform
// and constants, k_refine, and the merge's canonical rescoring, on the
// context's stream; the caller's stream is ordered before by an event.
// ================================================================ bound audit
// The certified bounds of sampled (query, row) pairs after every level, from
// the index's own tiles and tails and the query constants of a search, with
// the bound functions the scans use (eps = 1).  One thread per pair; the head
// sums are sequential fused multiply-adds over the level's coordinates (an
// order the margins cover, as they cover the matrix cores' chunked sums).
// out [npairs][L][4]: lower, upper bound with the head from coordinate
// differences; lower, upper bound in the dot-product form.  rows (optional)
// [npairs][2][d_pad]: the transformed query and the FP32 stored row.
__global__ void k_audit_bounds(SearchConsts c, IndexView ix, QueryView qv, const uint16_t *__restrict__ lv16,
                               int64_t nq, int64_t n, const int32_t *__restrict__ pair_q,
                               const int64_t *__restrict__ pair_row, const int64_t *__restrict__ idpos,
                               int64_t npairs, int bf, float *__restrict__ out, float *__restrict__ rows,
                               int32_t *__restrict__ bad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npairs) return;
    const LevelGeom &g = c.g;
    const int L = g.L;
    const int32_t qi = pair_q[i];
    const int64_t r = pair_row[i];
    if (qi < 0 || qi >= nq || r < 0 || r >= n) {
        atomicOr(bad, 1);
        for (int e = 0; e < 4 * L; ++e) out[i * 4 * L + e] = NAN;
        return;
    }
    const int64_t pos = idpos[r];
    const int64_t blk = pos / g.B;
    const int ss = (int)(pos % g.B);
    const float *X = ix.levels + blk * (int64_t)g.B * g.d_pad;
    const uint16_t *X16 = bf ? lv16 + blk * (int64_t)g.B * g.d_pad : nullptr;
    const float *tl = ix.tails + blk * (int64_t)L * g.B;
    const float *qr = qv.qy + (int64_t)qi * g.d_pad;
    const float *qt = qv.qtail + (int64_t)qi * L;
    const float A = qv.qA[qi];
    const float b0 = tl[ss];
    float shd = 0.f, shp = 0.f;
    for (int lv = 0; lv < L; ++lv) {
        const bool last = lv + 1 == L;
        const float al = qt[lv], an = last ? 0.f : qt[lv + 1];
        const float bl = tl[(int64_t)lv * g.B + ss], bn = last ? 0.f : tl[(int64_t)(lv + 1) * g.B + ss];
        float part = 0.f, dot = 0.f, ex = 0.f;
        for (int j = 0; j < g.wp[lv]; ++j) {
            // level 1: groups of four coordinates stored for all B slots; later
            // levels: each slot's slice contiguous
            const int64_t o = lv == 0 ? (int64_t)(j >> 2) * 4 * g.B + (int64_t)ss * 4 + (j & 3)
                                      : (int64_t)g.B * g.mp[lv] + (int64_t)ss * g.wp[lv] + j;
            const float x = bf ? __uint_as_float((uint32_t)X16[o] << 16) : X[o];
            const float y = qr[g.mp[lv] + j];
            const float t = y - x;
            part = __builtin_fmaf(t, t, part);
            dot = __builtin_fmaf(y, x, dot);
            ex = __builtin_fmaf(x, x, ex);
            if (rows) {
                rows[(i * 2) * g.d_pad + g.mp[lv] + j] = y;
                rows[(i * 2 + 1) * g.d_pad + g.mp[lv] + j] = X[o];
            }
        }
        shd += part;
        const float rxl = bf ? ex : bl * bl - bn * bn;
        shp = (lv == 0 ? (al * al - an * an) : shp + (al * al - an * an)) + rxl - 2.f * dot;
        const float ct = c.mg.c_tail * (an + bn) * (an + bn);
        const float errd = c.mg.c_level[lv + 1] * fmaxf(shd, 0.f) + A;
        const float errp = lv == 0 ? A : c.mg.c_level[lv + 1] * fmaxf(shp, 0.f) + A;
        float *o4 = out + (i * L + lv) * 4;
        if (bf) {
            const float delta = c.ub * head_norm_upper(b0, bn) + 1e-37f;
            o4[0] = pair_lower_bf<false>(shd, an, bn, errd, ct, 0.f, delta);
            o4[1] = pair_upper_bf(shd, an, bn, errd, ct, delta);
            o4[2] = pair_lower_bf<false>(shp, an, bn, errp, ct, 0.f, delta);
            o4[3] = pair_upper_bf(shp, an, bn, errp, ct, delta);
        } else {
            o4[0] = pair_lower<false>(shd, an, bn, errd, ct, 0.f);
            o4[1] = pair_upper(shd, an, bn, errd, ct);
            o4[2] = pair_lower<false>(shp, an, bn, errp, ct, 0.f);
            o4[3] = pair_upper(shp, an, bn, errp, ct);
        }
    }
}

void run_audit_bounds(pano_ctx *ctx, pano_index *ix, const float *q, int64_t nq, const int32_t *pair_q,
                      const int64_t *pair_row, int64_t npairs, bool bf, float *out, float *rows, hipStream_t s)
{
    PANO_HIP(hipSetDevice(ctx->device));
    PANO_REQUIRE(!bf || ix->has_bf16, "the index has no bfloat16 tiles");
    const int d = ix->d, L = ix->L;
    SearchConsts c{};
    c.k = 1;
    c.nlist = ix->nlist;
    c.eps = 1.f;
    c.one_m_eps2 = 0.f;
    c.bf16 = bf ? 1 : 0;
    c.ub = (float)(std::ldexp(1.0, -8) * (1.0 + 1e-6));
    c.mg = ix->mg;
    c.g = LevelGeom{};
    c.g.L = L;
    c.g.d = d;
    c.g.d_pad = ix->d_pad;
    c.g.B = ix->B;
    for (int l = 0; l <= L; ++l) c.g.mp[l] = ix->mp[l];
    for (int l = 0; l < L; ++l) c.g.wp[l] = ix->wp[l];
    // the query constants of a search that reads these tiles
    Margins mq = ix->mg;
    if (bf) {
        mq.c_abs = ix->c_abs_bf;
        mq.b0max2 = (float)((double)ix->mg.b0max2 * (1.0 + std::ldexp(1.0, -8)) * (1.0 + std::ldexp(1.0, -8)) *
                            (1.0 + 1e-6));
    }
    if (!ix->idpos.p) {
        ix->idpos.alloc(sizeof(int64_t) * (size_t)ix->n);
        const int64_t slots = ix->nblocks * ix->B;
        hipLaunchKernelGGL(k_build_idpos, dim3((unsigned)((slots + 255) / 256)), dim3(256), 0, ctx->work_stream(),
                           ix->ids.as<int32_t>(), ix->blk_cnt.as<int32_t>(), ix->nblocks, ix->B,
                           ix->idpos.as<int64_t>());
        PANO_HIP(hipGetLastError());
    }
    const size_t need0 = align_up(sizeof(float) * nq * ix->d_pad) + align_up(sizeof(float) * nq * L) +
                         3 * align_up(sizeof(float) * nq) + align_up(sizeof(double) * nq);
    const size_t need3 = align_up(sizeof(int32_t) * nq) + align_up(sizeof(int32_t));
    ctx->quiesce();
    ctx->scratch[0].ensure(need0);
    ctx->scratch[3].ensure(need3);
    Carver c0(ctx->scratch[0].p), c3(ctx->scratch[3].p);
    float *qy = c0.take<float>(nq * ix->d_pad);
    float *qtail = c0.take<float>(nq * L);
    float *qE = c0.take<float>(nq);
    float *qA = c0.take<float>(nq);
    double *vnorm = c0.take<double>(nq);
    int32_t *qbad = c3.take<int32_t>(nq);
    int32_t *bad = c3.take<int32_t>(1);
    hipStream_t ws = ctx->work_stream();
    PANO_HIP(hipEventRecord(ctx->ev_in, s));
    PANO_HIP(hipStreamWaitEvent(ws, ctx->ev_in, 0));
    FillList fl{};
    fl.add(bad, 1, 0u);
    if (rows) fl.add(rows, npairs * 2 * (int64_t)ix->d_pad, 0u);
    if (ix->d_pad != ix->d) fl.add(qy, nq * (int64_t)ix->d_pad, 0u);
    hipLaunchKernelGGL(k_fill_multi, dim3(256), dim3(256), 0, ws, fl);
    const GemmJob jt = transform_job(q, nq, d, ix->T32.as<float>(), ix->mu32.as<float>(), ix->meta.as<int32_t>(), qy,
                                     ix->d_pad);
    launch_gemm_jobs(jt, nullptr, ws, nullptr);
    QueryConstsOut qc;
    qc.mg = mq;
    qc.qE = qE;
    qc.qA = qA;
    qc.badq = qbad;
    launch_row_norms(qy, nq, c.g, q, ix->mu32.as<float>(), qtail, vnorm, ws, &qc);
    IndexView iv{ix->levels.as<float>(), nullptr, ix->tails.as<float>(), ix->ids.as<int32_t>(),
                 ix->blk_cnt.as<int32_t>(), ix->list_blk_d.as<int64_t>(), ix->raw.as<float>()};
    QueryView qv{qy, qtail, qE, qA, q};
    if (npairs > 0)
        hipLaunchKernelGGL(k_audit_bounds, dim3((unsigned)((npairs + 255) / 256)), dim3(256), 0, ws, c, iv, qv,
                           bf ? ix->levels_bf16.as<uint16_t>() : nullptr, nq, ix->n, pair_q, pair_row,
                           ix->idpos.as<int64_t>(), npairs, bf ? 1 : 0, out, rows, bad);
    PANO_HIP(hipGetLastError());
    int32_t hbad = 0;
    PANO_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, ws));
    PANO_HIP(hipStreamSynchronize(ws));
    PANO_REQUIRE(hbad == 0, "a pair's query or row index is out of range");
}

void run_refine(pano_ctx *ctx, pano_index *ix, const float *q, int64_t nq, int k, const int64_t *cand, int kprime,
                float eps, int64_t *ids, float *dists, hipStream_t s)
{
    PANO_HIP(hipSetDevice(ctx->device));
    PANO_REQUIRE(k <= 128, "k up to 128 is supported");
    const int d = ix->d, L = ix->L;
    SearchConsts c{};
    c.k = k;
    c.kc = next_pow2(std::max(2 * k, 16));
    // every candidate is appended at most once: the buffer cannot overflow
    c.capq = next_pow2(std::max(kprime, 64));
    c.nlist = ix->nlist;
    c.prune = 1;
    c.eps = eps;
    c.one_m_eps2 = 2.f * (1.f - eps);
    c.mg = ix->mg;
    c.g = LevelGeom{};
    c.g.L = L;
    c.g.d = d;
    c.g.d_pad = ix->d_pad;
    c.g.B = ix->B;
    for (int l = 0; l <= L; ++l) c.g.mp[l] = ix->mp[l];
    for (int l = 0; l < L; ++l) c.g.wp[l] = ix->wp[l];
    c.wl = wave_lds_layout(L, k, ix->wp[0]);
    if (!ix->idpos.p) {
        ix->idpos.alloc(sizeof(int64_t) * (size_t)ix->n);
        const int64_t slots = ix->nblocks * ix->B;
        hipLaunchKernelGGL(k_build_idpos, dim3((unsigned)((slots + 255) / 256)), dim3(256), 0, ctx->work_stream(),
                           ix->ids.as<int32_t>(), ix->blk_cnt.as<int32_t>(), ix->nblocks, ix->B,
                           ix->idpos.as<int64_t>());
        PANO_HIP(hipGetLastError());
    }
    const size_t need0 = align_up(sizeof(float) * nq * ix->d_pad) + align_up(sizeof(float) * nq * L) +
                         3 * align_up(sizeof(float) * nq) + align_up(sizeof(double) * nq);
    const size_t need3 = 4 * align_up(sizeof(float) * nq) + align_up(sizeof(uint64_t) * nq * c.capq) +
                         align_up(sizeof(unsigned long long) * 128);
    ctx->quiesce();  // the scratch is the one an asynchronous search may still use
    ctx->scratch[0].ensure(need0);
    ctx->scratch[3].ensure(need3);
    Carver c0(ctx->scratch[0].p), c3(ctx->scratch[3].p);
    float *qy = c0.take<float>(nq * ix->d_pad);
    float *qtail = c0.take<float>(nq * L);
    float *qE = c0.take<float>(nq);
    float *qA = c0.take<float>(nq);
    double *vnorm = c0.take<double>(nq);
    int32_t *qbad = c3.take<int32_t>(nq);
    float *thr = c3.take<float>(nq);
    int32_t *buf_cnt = c3.take<int32_t>(nq);
    int32_t *qflags = c3.take<int32_t>(nq);
    uint64_t *buf = c3.take<uint64_t>(nq * c.capq);
    (void)thr;
    ctx->pinned_ensure(sizeof(int32_t) * nq);
    int32_t *h_flags = reinterpret_cast<int32_t *>(ctx->pinned);
    const size_t merge_shm = sizeof(uint64_t) * MERGE_LDS_KEYS + sizeof(float) * (size_t)d;
    PANO_HIP(hipFuncSetAttribute((const void *)k_merge, hipFuncAttributeMaxDynamicSharedMemorySize, (int)merge_shm));
    hipStream_t ws = ctx->work_stream();
    PANO_HIP(hipEventRecord(ctx->ev_in, s));
    PANO_HIP(hipStreamWaitEvent(ws, ctx->ev_in, 0));
    FillList fl{};
    fl.add(buf_cnt, nq, 0u);
    fl.add(qflags, nq, 0u);
    if (ix->d_pad != ix->d) {
        FillList fq{};
        fq.add(qy, nq * (int64_t)ix->d_pad, 0u);
        hipLaunchKernelGGL(k_fill_multi, dim3(256), dim3(256), 0, ws, fq);
    }
    const GemmJob jt = transform_job(q, nq, d, ix->T32.as<float>(), ix->mu32.as<float>(), ix->meta.as<int32_t>(), qy,
                                     ix->d_pad);
    launch_gemm_jobs(jt, nullptr, ws, &fl);
    QueryConstsOut qc;
    qc.mg = ix->mg;
    qc.qE = qE;
    qc.qA = qA;
    qc.badq = qbad;
    launch_row_norms(qy, nq, c.g, q, ix->mu32.as<float>(), qtail, vnorm, ws, &qc);
    IndexView iv{ix->levels.as<float>(), nullptr, ix->tails.as<float>(), ix->ids.as<int32_t>(),
                 ix->blk_cnt.as<int32_t>(), ix->list_blk_d.as<int64_t>(), ix->raw.as<float>()};
    QueryView qv{qy, qtail, qE, qA, q};
    WorkView wk{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, buf, buf_cnt, qflags, nullptr};
    const size_t rshm = sizeof(float) * (size_t)(NT / 64) * (k + next_pow2(k + 64));
    hipLaunchKernelGGL(k_refine, dim3((unsigned)((nq + NT / 64 - 1) / (NT / 64))), dim3(NT), rshm, ws, c, iv, qv, wk,
                       cand, kprime, nq, ix->idpos.as<int64_t>(), ix->n);
    hipLaunchKernelGGL(k_merge, dim3((unsigned)nq), dim3(NT), merge_shm, ws, c, buf, buf_cnt, qflags, qE, qA, q,
                       ix->raw.as<float>(), d, ids, dists, nullptr, h_flags, qbad);
    PANO_HIP(hipGetLastError());
    PANO_HIP(hipStreamSynchronize(ws));
    for (int64_t qi = 0; qi < nq; ++qi) {
        PANO_REQUIRE(!(h_flags[qi] & FLAG_NONFINITE), "a query has a non-finite value");
        PANO_REQUIRE(!(h_flags[qi] & FLAG_BADID), "a candidate id is outside [-1, n)");
        PANO_REQUIRE(!(h_flags[qi] & FLAG_OVERFLOW), "refine result buffer overflow");
    }
}

}  // namespace pano
