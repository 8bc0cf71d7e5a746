// Build-side kernels for gfx950: the FP32 transform of rows into the
// rotated frame (Section 4.1, applied as T (v - mu)), k-means assignment and
// update (the IVF coarse quantiser of Section 6.1), per-row tail norms
// (Section 6.5) and the level-major packing of Section 6.1.
#include "internal.h"
#include "search_common.h"

#include <algorithm>
#include <cmath>

namespace pano {

// ---------------------------------------------------------------- tiled product
// Dense products Out = (A - mu) B^t on the matrix cores: one workgroup per
// 64 x 64 output tile, each wavefront a 32 x 32 sub-tile made of four
// v_mfma_f32_16x16x4f32 accumulators.  The reduction dimension is consumed in
// chunks of 32: each chunk is summed in fresh accumulators and then added to
// the running total, so every output carries a rounding error of at most
// gamma(32 + ceil(K/32) + 1) times the sum of the absolute products (the
// bound the pruning margins are built on).
constexpr int TM = 64, TN = 64, TK = 32, TLD = 36;
constexpr int RF = TM / 32;  // 16-row fragments per wavefront (waves in a 2 x 2 grid)
typedef float floatx4_t __attribute__((ext_vector_type(4)));

// One launch may carry two independent products (jobs): the workgroups with
// blockIdx.y < y0 take job j0, the others job j1 (column tile blockIdx.y - y0).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_tile_nt(GemmJob j0, GemmJob j1,
                                                                                           int y0, FillList clear)
{
    for (int sgm = 0; sgm < clear.m; ++sgm) {
        uint32_t *p = reinterpret_cast<uint32_t *>(clear.p[sgm]);
        const uint32_t v = clear.v[sgm];
        const int64_t nthr = (int64_t)gridDim.x * gridDim.y * blockDim.x;
        for (int64_t i = ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x; i < clear.n[sgm];
             i += nthr)
            p[i] = v;
    }
    const bool first = (int)blockIdx.y < y0;
    const float *__restrict__ A = first ? j0.A : j1.A;
    const int64_t n = first ? j0.n : j1.n;
    const int K = first ? j0.K : j1.K;
    const float *__restrict__ Bm = first ? j0.Bm : j1.Bm;
    const int nb = first ? j0.nb : j1.nb;
    const float *__restrict__ mu = first ? j0.mu : j1.mu;
    const int32_t *__restrict__ outcol = first ? j0.outcol : j1.outcol;
    float *__restrict__ Out = first ? j0.Out : j1.Out;
    const int ld_out = first ? j0.ld_out : j1.ld_out;
    // two LDS stages: the next chunk is fetched into registers while the
    // current one feeds the matrix cores
    __shared__ float As[2][TM][TLD];
    __shared__ float Bs[2][TN][TLD];
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int r16 = lane & 15, kq = lane >> 4;
    const int wr = (w >> 1) * (TM / 2), wc = (w & 1) * 32;
    const int64_t r0 = (int64_t)blockIdx.x * TM;
    const int c0 = (first ? (int)blockIdx.y : (int)blockIdx.y - y0) * TN;
    constexpr int NA = (TM * TK) / 256, NB = (TN * TK) / 256;
    // a register set holds one fetched chunk as loaded (this thread's share
    // of A and B, and the one mu value of its column: e % TK is tid % TK for
    // every element e of the thread) and the chunk's start; the out-of-range
    // values are replaced and mu subtracted only when the chunk is stored to
    // LDS, so nothing waits for the loads before then
    static_assert(256 % TK == 0, "a thread keeps one column of each chunk");
    struct RegSet {
        float a[NA], b[NB], m;
        int k0;
    };
    const bool sub_mu = mu != nullptr;
    const float *__restrict__ mu_ld = sub_mu ? mu : A;  // any valid row when unused
    // every load is issued from a clamped (valid) index, so no branch
    // separates the loads of a chunk and they are all in flight together
    auto fetch = [&](int k0, RegSet &R) {
        R.k0 = k0;
        R.m = mu_ld[min(k0 + tid % TK, K - 1)];
#pragma unroll
        for (int t = 0; t < NA; ++t) {
            const int e = tid + t * 256;
            const int64_t r = min(r0 + e / TK, n - 1);
            const int kx = min(k0 + e % TK, K - 1);
            R.a[t] = A[r * K + kx];
        }
#pragma unroll
        for (int t = 0; t < NB; ++t) {
            const int e = tid + t * 256;
            const int c = min(c0 + e / TK, nb - 1);
            const int kx = min(k0 + e % TK, K - 1);
            R.b[t] = Bm[(int64_t)c * K + kx];
        }
    };
    auto stash = [&](int buf, const RegSet &R) {
#pragma unroll
        for (int t = 0; t < NA; ++t) {
            const int e = tid + t * 256;
            const bool ok = r0 + e / TK < n && R.k0 + e % TK < K;
            As[buf][e / TK][e % TK] = ok ? (sub_mu ? R.a[t] - R.m : R.a[t]) : 0.f;
        }
#pragma unroll
        for (int t = 0; t < NB; ++t) {
            const int e = tid + t * 256;
            const bool ok = c0 + e / TK < nb && R.k0 + e % TK < K;
            Bs[buf][e / TK][e % TK] = ok ? R.b[t] : 0.f;
        }
    };
    floatx4_t tot[RF][2];
#pragma unroll
    for (int i = 0; i < RF; ++i) tot[i][0] = tot[i][1] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    const int nchunks = (K + TK - 1) / TK;
    auto compute = [&](int buf) {
        floatx4_t acc[RF][2];
#pragma unroll
        for (int i = 0; i < RF; ++i) acc[i][0] = acc[i][1] = floatx4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < TK / 4; ++ks) {
            float a[RF], b[2];
#pragma unroll
            for (int i = 0; i < RF; ++i) a[i] = As[buf][wr + i * 16 + r16][ks * 4 + kq];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[buf][wc + j * 16 + r16][ks * 4 + kq];
#pragma unroll
            for (int i = 0; i < RF; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < RF; ++i) {
            tot[i][0] += acc[i][0];
            tot[i][1] += acc[i][1];
        }
    };
    // Four chunks in flight.  Register set R[j] receives chunks j, j + 4, ...;
    // step ch computes LDS stage ch & 1, stores chunk ch + 1 into the other
    // stage and requests chunk ch + 4 into the set chunk ch left free.  Full
    // groups of four steps run without branches (requests past the last
    // chunk re-read it and are never used), so the waits for each set stay
    // exact; the last steps follow with their guards.
    RegSet R[4];
    fetch(0, R[0]);
    stash(0, R[0]);
    fetch(min(1, nchunks - 1) * TK, R[1]);
    fetch(min(2, nchunks - 1) * TK, R[2]);
    fetch(min(3, nchunks - 1) * TK, R[3]);
    __syncthreads();
    int base = 0;
    for (; base + 4 <= nchunks; base += 4) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int ch = base + j;
            compute(j & 1);
            stash((j + 1) & 1, R[(j + 1) & 3]);
            fetch(min(ch + 4, nchunks - 1) * TK, R[j]);
            __syncthreads();
        }
    }
    // (unrolled with constant set indices, so the sets stay in registers)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int ch = base + j;
        if (ch < nchunks) {
            compute(j & 1);
            if (ch + 1 < nchunks) stash((j + 1) & 1, R[(j + 1) & 3]);
            __syncthreads();
        }
    }
    // lane holds rows 4*(lane/16) + v of column lane%16 of each 16 x 16 tile
#pragma unroll
    for (int i = 0; i < RF; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t r = r0 + wr + i * 16 + 4 * kq + v;
                const int c = c0 + wc + j * 16 + r16;
                if (r < n && c < nb) {
                    const int oc = outcol ? outcol[c] : c;
                    Out[r * ld_out + oc] = tot[i][j][v];
                }
            }
}

GemmJob transform_job(const float *X, int64_t n, int d, const float *T, const float *mu, const int32_t *padcol,
                      float *Y, int ld_y)
{
    return GemmJob{X, n, d, T, d, mu, padcol, Y, ld_y};
}

GemmJob product_job(const float *A, int64_t n, int d, const float *Bm, int nb, float *S)
{
    return GemmJob{A, n, d, Bm, nb, nullptr, nullptr, S, nb};
}

void launch_gemm_jobs(const GemmJob &j0, const GemmJob *j1, hipStream_t s, const FillList *clear)
{
    const int64_t n = j1 ? std::max(j0.n, j1->n) : j0.n;
    if (n == 0) return;
    const int y0 = (j0.nb + TN - 1) / TN;
    const int y1 = j1 ? (j1->nb + TN - 1) / TN : 0;
    dim3 grid((unsigned)((n + TM - 1) / TM), (unsigned)(y0 + y1));
    FillList none{};
    hipLaunchKernelGGL(k_tile_nt, grid, dim3(256), 0, s, j0, j1 ? *j1 : j0, y0, clear ? *clear : none);
    PANO_HIP(hipGetLastError());
}

void launch_transform(const float *X, int64_t n, int d, const float *T, const float *mu,
                      const int32_t *padcol, float *Y, int ld_y, hipStream_t s)
{
    launch_gemm_jobs(transform_job(X, n, d, T, mu, padcol, Y, ld_y), nullptr, s);
}

void launch_gemm_nt(const float *A, int64_t n, int d, const float *Bm, int nb, float *S, hipStream_t s)
{
    launch_gemm_jobs(product_job(A, n, d, Bm, nb, S), nullptr, s);
}

// ---------------------------------------------------------------- row norms
// One wavefront per row.  Level energies are summed in FP64, the tail norm
// after level l is the square root of the suffix sum, rounded to FP32.
__device__ inline double wave_sum_f64(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Rows of up to 64 * VPL padded values are read into registers at once
// (every load in flight together); wider rows loop over the level slices.
// Both give the same sums in the same order: per lane, its values of the
// level in increasing column order, then the butterfly of wave_sum_f64.
template <int VPL>
__global__ __launch_bounds__(256) void k_row_norms(const float *__restrict__ Y, int64_t n, LevelGeom g,
                                                   const float *__restrict__ X,
                                                   const float *__restrict__ mu,
                                                   float *__restrict__ tails, double *__restrict__ vnorm,
                                                   QueryConstsOut qc)
{
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= n) return;
    const float *y = Y + r * g.d_pad;
    double suffix = 0.0;
    float tail0 = 0.f;  // the tail norm after level 0 (the row's norm), last one computed
    if (VPL > 0) {
        float v[VPL > 0 ? VPL : 1];
#pragma unroll
        for (int j = 0; j < VPL; ++j) v[j] = y[min(j * 64 + lane, g.d_pad - 1)];  // clamped: no branch
        for (int l = g.L - 1; l >= 0; --l) {
            const int lo = g.mp[l], hi = g.mp[l + 1];
            double e = 0.0;
#pragma unroll
            for (int j = 0; j < VPL; ++j) {
                const int c = j * 64 + lane;
                if (c >= lo && c < hi) {
                    const double t = (double)v[j];
                    e += t * t;
                }
            }
            e = wave_sum_f64(e);
            suffix += e;
            const float tv = (float)sqrt(suffix);
            if (lane == 0) tails[r * g.L + l] = tv;
            tail0 = tv;
        }
    } else {
        for (int l = g.L - 1; l >= 0; --l) {
            double e = 0.0;
            for (int c = g.mp[l] + lane; c < g.mp[l + 1]; c += 64) {
                double v = (double)y[c];
                e += v * v;
            }
            e = wave_sum_f64(e);
            suffix += e;
            const float tv = (float)sqrt(suffix);
            if (lane == 0) tails[r * g.L + l] = tv;
            tail0 = tv;
        }
    }
    if (vnorm) {
        const float *x = X + r * g.d;
        double e = 0.0;
        for (int c0 = 0; c0 < g.d; c0 += 64 * 8) {
            float xv[8], mv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int c = min(c0 + u * 64 + lane, g.d - 1);  // clamped: no branch
                xv[u] = x[c];
                mv[u] = mu[c];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (c0 + u * 64 + lane < g.d) {
                    const double t = (double)(xv[u] - mv[u]);
                    e += t * t;
                }
            }
        }
        e = wave_sum_f64(e);
        const double vn = sqrt(e);
        if (lane == 0) vnorm[r] = vn;
        if (qc.qE && lane == 0) {
            // the query's error bound E_q = kappa ||fl(q - mu)|| + e_max and
            // absolute margin A_q = c_abs (a_0^2 + b0max2), each rounded up
            // by a relative 1e-6 to cover the FP32 rounding
            if (qc.badq) qc.badq[r] = isfinite(vn) ? 0 : 1;
            qc.qE[r] = (float)((double)qc.mg.kappa * vn * (1.0 + 1e-6)) + qc.mg.e_max;
            const double a0 = (double)tail0;
            qc.qA[r] = (float)((double)qc.mg.c_abs * (a0 * a0 * (1.0 + 1e-6) + (double)qc.mg.b0max2) * (1.0 + 1e-6));
        }
    }
}

void launch_row_norms(const float *Y, int64_t n, const LevelGeom &g, const float *X, const float *mu,
                      float *tails_rowmajor, double *vnorm, hipStream_t s, const QueryConstsOut *qc)
{
    if (n == 0) return;
    dim3 grid((unsigned)((n + 3) / 4));
    QueryConstsOut q{};
    if (qc) q = *qc;
    if (g.d_pad <= 256)
        hipLaunchKernelGGL(k_row_norms<4>, grid, dim3(256), 0, s, Y, n, g, X, mu, tails_rowmajor, vnorm, q);
    else if (g.d_pad <= 1024)
        hipLaunchKernelGGL(k_row_norms<16>, grid, dim3(256), 0, s, Y, n, g, X, mu, tails_rowmajor, vnorm, q);
    else
        hipLaunchKernelGGL(k_row_norms<0>, grid, dim3(256), 0, s, Y, n, g, X, mu, tails_rowmajor, vnorm, q);
    PANO_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- k-means
__global__ __launch_bounds__(256) void k_sqnorms(const float *__restrict__ X, int64_t n, int d,
                                                 float *__restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= n) return;
    float e = 0.f;
    for (int c = lane; c < d; c += 64) e = __builtin_fmaf(X[r * d + c], X[r * d + c], e);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o, 64);
    if (lane == 0) out[r] = e;
}

void launch_sqnorms(const float *X, int64_t n, int d, float *out, hipStream_t s)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_sqnorms, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, X, n, d, out);
    PANO_HIP(hipGetLastError());
}

// assign[r] = argmin_c (||c||^2 - 2 <x_r, c>), ties to the smaller c.
__global__ __launch_bounds__(256) void k_argmin_rows(const float *__restrict__ S, int64_t n, int nb,
                                                     const float *__restrict__ cnorm,
                                                     int32_t *__restrict__ assign)
{
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= n) return;
    float best = INFINITY;
    int bi = 0x7fffffff;
    for (int c = lane; c < nb; c += 64) {
        float v = cnorm[c] - 2.f * S[r * nb + c];
        if (v < best || (v == best && c < bi)) {
            best = v;
            bi = c;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        float ov = __shfl_xor(best, o, 64);
        int oi = __shfl_xor(bi, o, 64);
        if (ov < best || (ov == best && oi < bi)) {
            best = ov;
            bi = oi;
        }
    }
    if (lane == 0) assign[r] = bi;
}

void launch_argmin_rows(const float *S, int64_t n, int nb, const float *cnorm, int32_t *assign,
                        hipStream_t s)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_argmin_rows, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, S, n, nb, cnorm, assign);
    PANO_HIP(hipGetLastError());
}

// The final assignment by the canonical (D, l) rule, D the canonical distance
// (sequential FP64 over the raw rows, rounded to FP32), ties to the smaller
// list.  One wavefront per row.  The FP32 score a_l = ||c_l||^2 - 2 <x, c_l>
// lies within del_l = c_as (||x||^2 + ||c_l||^2) + 2^-22 |a_l| of its exact
// value (c_as covers the rounding of the norms and of the tiled products);
// with U the smallest a_l + del_l, widened by 2^-20 (||x||^2 + |U|) for the
// FP32 rounding of D, only lists with a_l - del_l <= U can hold the smallest
// key.  A single such list is the answer; several are rescored with the
// canonical distance.  Rows without any (a non-finite value) keep the FP32
// argmin.
__global__ __launch_bounds__(256) void k_assign_canon(const float *__restrict__ S, int64_t n, int nb,
                                                      const float *__restrict__ cnorm, const float *__restrict__ X,
                                                      const float *__restrict__ cent, int d, float c_as,
                                                      int32_t *__restrict__ assign)
{
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= n) return;
    const float *x = X + r * d;
    float xx = 0.f;
    for (int j = lane; j < d; j += 64) xx = __builtin_fmaf(x[j], x[j], xx);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) xx += __shfl_xor(xx, o, 64);
    const float *srow = S + r * nb;
    float ub = INFINITY, best = INFINITY;
    int bi = 0x7fffffff;
    for (int c = lane; c < nb; c += 64) {
        const float a = cnorm[c] - 2.f * srow[c];
        const float del = c_as * (xx + cnorm[c]) + 0x1p-22f * fabsf(a);
        ub = fminf(ub, a + del);
        if (a < best || (a == best && c < bi)) {
            best = a;
            bi = c;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        ub = fminf(ub, __shfl_xor(ub, o, 64));
        const float ov = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ov < best || (ov == best && oi < bi)) {
            best = ov;
            bi = oi;
        }
    }
    const float U = ub + 0x1p-20f * (xx + fabsf(ub));
    // the lists that can hold the smallest key: count them, keep one
    int cnt = 0, one = -1;
    for (int c0 = 0; c0 < nb; c0 += 64) {
        const int c = c0 + lane;
        bool mem = false;
        if (c < nb) {
            const float a = cnorm[c] - 2.f * srow[c];
            const float del = c_as * (xx + cnorm[c]) + 0x1p-22f * fabsf(a);
            mem = a - del <= U;
        }
        const uint64_t bm = __ballot(mem);
        if (bm != 0 && one < 0) one = c0 + __ffsll((long long)bm) - 1;
        cnt += __popcll(bm);
    }
    int ans = bi;
    if (cnt == 1) {
        ans = one;
    } else if (cnt > 1) {
        uint64_t key = KEY_MAX;
        for (int c0 = 0; c0 < nb; c0 += 64) {
            const int c = c0 + lane;
            if (c < nb) {
                const float a = cnorm[c] - 2.f * srow[c];
                const float del = c_as * (xx + cnorm[c]) + 0x1p-22f * fabsf(a);
                if (a - del <= U) {
                    const uint64_t kc = make_key(canon_dist(x, cent + (int64_t)c * d, d), c);
                    key = kc < key ? kc : key;
                }
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const uint32_t lo = __shfl_xor((uint32_t)key, o, 64), hi = __shfl_xor((uint32_t)(key >> 32), o, 64);
            const uint64_t ok = ((uint64_t)hi << 32) | lo;
            key = ok < key ? ok : key;
        }
        if (key != KEY_MAX) ans = key_id(key);
    }
    if (lane == 0) assign[r] = ans;
}

void launch_assign_canon(const float *S, int64_t n, int nb, const float *cnorm, const float *X, const float *cent,
                         int d, int32_t *assign, hipStream_t s)
{
    if (n == 0) return;
    // rounding of ||c||^2 (per-lane FMA chains over d / 64 terms, then six
    // additions) and of the tiled product (gamma(32 + ceil(d / 32) + 1) of the
    // absolute products, which sum to at most (||x||^2 + ||c||^2) / 2, twice)
    const double u = std::ldexp(1.0, -24);
    auto gam = [&](double m) { return m * u / (1.0 - m * u); };
    const float c_as = (float)(1.25 * (gam(d / 64.0 + 8) + gam(33.0 + (d + 31) / 32) + 2 * u));
    hipLaunchKernelGGL(k_assign_canon, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, S, n, nb, cnorm, X, cent, d,
                       c_as, assign);
    PANO_HIP(hipGetLastError());
}

// One workgroup per cluster: mean of its members (FP64 sums over members in
// ascending row order).  Empty clusters keep their centroid.
__global__ __launch_bounds__(256) void k_centroid_update(const float *__restrict__ X, int d,
                                                         const int64_t *__restrict__ perm,
                                                         const int64_t *__restrict__ off,
                                                         float *__restrict__ cent)
{
    const int c = blockIdx.x;
    const int64_t b = off[c], e = off[c + 1];
    if (e <= b) return;
    for (int j = threadIdx.x; j < d; j += blockDim.x) {
        double s = 0.0;
        for (int64_t t = b; t < e; ++t) s += (double)X[perm[t] * d + j];
        cent[(int64_t)c * d + j] = (float)(s / (double)(e - b));
    }
}

void launch_centroid_update(const float *X, int d, const int64_t *perm, const int64_t *off, int nlist,
                            float *cent, hipStream_t s)
{
    hipLaunchKernelGGL(k_centroid_update, dim3(nlist), dim3(256), 0, s, X, d, perm, off, cent);
    PANO_HIP(hipGetLastError());
}

// k-means++ seeding (D^2 sampling): keep, for every sampled row, the squared
// distance to its nearest chosen centroid.
__global__ __launch_bounds__(256) void k_update_mind(const float *__restrict__ X, int64_t n, int d,
                                                     const float *__restrict__ c, float *__restrict__ mind)
{
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= n) return;
    float e = 0.f;
    for (int j = lane; j < d; j += 64) {
        float t = X[r * d + j] - c[j];
        e = __builtin_fmaf(t, t, e);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o, 64);
    if (lane == 0) mind[r] = fminf(mind[r], e);
}

// Greedy k-means++: for each of nc candidate centres, the potential
// sum_i min(mind_i, ||x_i - cand||^2) over the sampled rows.
__global__ __launch_bounds__(256) void k_cand_potential(const float *__restrict__ X, int64_t n, int d,
                                                        const float *__restrict__ cand, int nc,
                                                        const float *__restrict__ mind, double *__restrict__ pot)
{
    constexpr int NCMAX = 16;
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    double acc[NCMAX];
#pragma unroll
    for (int c = 0; c < NCMAX; ++c) acc[c] = 0.0;
    for (int64_t r = wave; r < n; r += nwaves) {
        const float m = mind[r];
#pragma unroll
        for (int c = 0; c < NCMAX; ++c) {
            if (c >= nc) break;
            float e = 0.f;
            for (int j = lane; j < d; j += 64) {
                float t = X[r * d + j] - cand[(int64_t)c * d + j];
                e = __builtin_fmaf(t, t, e);
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o, 64);
            acc[c] += (double)fminf(m, e);
        }
    }
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < NCMAX; ++c)
            if (c < nc) atomicAdd(&pot[c], acc[c]);
}

void launch_cand_potential(const float *X, int64_t n, int d, const float *cand, int nc, const float *mind,
                           double *pot, hipStream_t s)
{
    if (n == 0) return;
    unsigned grid = (unsigned)std::min<int64_t>(1024, (n + 3) / 4);
    hipLaunchKernelGGL(k_cand_potential, dim3(grid), dim3(256), 0, s, X, n, d, cand, std::min(nc, 16), mind, pot);
    PANO_HIP(hipGetLastError());
}

void launch_update_mind(const float *X, int64_t n, int d, const float *c, float *mind, hipStream_t s)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_update_mind, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, X, n, d, c, mind);
    PANO_HIP(hipGetLastError());
}

__global__ __launch_bounds__(256) void k_gather_rows(const float *__restrict__ X, const int64_t *__restrict__ rows,
                                                     int64_t n, int d, float *__restrict__ out)
{
    const int64_t r = blockIdx.x;
    if (r >= n) return;
    const int64_t src = rows[r];
    for (int j = threadIdx.x; j < d; j += blockDim.x) out[r * d + j] = X[src * d + j];
}

void launch_gather_rows(const float *X, const int64_t *rows, int64_t n, int d, float *out, hipStream_t s)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)n), dim3(256), 0, s, X, rows, n, d, out);
    PANO_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- packing
__device__ inline uint16_t f32_to_bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    return (uint16_t)(u >> 16);
}

// One workgroup per block of B slots.  Level-major within the block: all B
// slices of level 0, then all B slices of level 1, ...  Inside a level the
// level-1 slices are interleaved by groups of four dimensions
// ([group][slot][4]) so that one 16-byte load per lane reads consecutive slots;
// the slices of later levels are stored slot after slot.
__global__ __launch_bounds__(256) void k_pack(const float *__restrict__ Y, const float *__restrict__ tails_row,
                                              const int64_t *__restrict__ perm,
                                              const int64_t *__restrict__ list_start,
                                              const int64_t *__restrict__ list_blk,
                                              const int32_t *__restrict__ block_list, LevelGeom g,
                                              float *__restrict__ levels, uint16_t *__restrict__ levels_bf16,
                                              float *__restrict__ tails, int32_t *__restrict__ ids,
                                              int32_t *__restrict__ blk_cnt)
{
    __shared__ int lvl_of[4096];
    __shared__ int64_t rows[1024];
    const int64_t gb = blockIdx.x;
    const int l = block_list[gb];
    const int64_t first = (gb - list_blk[l]) * g.B;
    const int64_t len = list_start[l + 1] - list_start[l];
    const int cnt = (int)min<int64_t>(g.B, len - first);
    for (int c = threadIdx.x; c < g.d_pad; c += blockDim.x) {
        int lv = 0;
        while (c >= g.mp[lv + 1]) ++lv;
        lvl_of[c] = lv;
    }
    for (int s = threadIdx.x; s < g.B; s += blockDim.x)
        rows[s] = s < cnt ? perm[list_start[l] + first + s] : -1;
    __syncthreads();
    if (threadIdx.x == 0) blk_cnt[gb] = cnt;
    float *dst = levels + gb * (int64_t)g.B * g.d_pad;
    uint16_t *dstb = levels_bf16 ? levels_bf16 + gb * (int64_t)g.B * g.d_pad : nullptr;
    const int64_t tot = (int64_t)g.B * g.d_pad;
    for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) {
        int s = (int)(e / g.d_pad), c = (int)(e % g.d_pad);
        int lv = lvl_of[c];
        int64_t r = rows[s];
        float v = r >= 0 ? Y[r * g.d_pad + c] : 0.f;
        // level 1 (read densely by every query of a group): groups of 4
        // consecutive dimensions, each group stored for all B slots (float4 per
        // slot); later levels (read per surviving candidate): each slot's slice
        // contiguous
        const int j = c - g.mp[lv];
        int64_t o = lv == 0 ? (int64_t)(j >> 2) * 4 * g.B + (int64_t)s * 4 + (j & 3)
                            : (int64_t)g.B * g.mp[lv] + (int64_t)s * g.wp[lv] + j;
        dst[o] = v;
        if (dstb) dstb[o] = f32_to_bf16_rne(v);
    }
    for (int e = threadIdx.x; e < g.B * g.L; e += blockDim.x) {
        int lv = e / g.B, s = e % g.B;
        int64_t r = rows[s];
        tails[gb * (int64_t)g.B * g.L + e] = r >= 0 ? tails_row[r * g.L + lv] : 0.f;
    }
    for (int s = threadIdx.x; s < g.B; s += blockDim.x) ids[gb * g.B + s] = (int32_t)rows[s];
}

void launch_pack(const float *Y, const float *tails_row, const int64_t *perm, const int64_t *list_start,
                 const int64_t *list_blk, const int32_t *block_list, int64_t nblocks, const LevelGeom &g,
                 float *levels, uint16_t *levels_bf16, float *tails, int32_t *ids, int32_t *blk_cnt,
                 hipStream_t s)
{
    if (nblocks == 0) return;
    hipLaunchKernelGGL(k_pack, dim3((unsigned)nblocks), dim3(256), 0, s, Y, tails_row, perm, list_start,
                       list_blk, block_list, g, levels, levels_bf16, tails, ids, blk_cnt);
    PANO_HIP(hipGetLastError());
}

}  // namespace pano
