// Internal declarations of the pruned-scan library: handle layouts, error
// helpers and the host-side launchers of the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/panorama.h"

namespace pano {

// Size of the fixed device scratch array of the allocation-free search (per
// GPU), and the devices it is set up for.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
constexpr int MAX_DEVICES = 64;

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
struct Error {
    pano_status st;
    std::string msg;
};
#define PANO_HIP(call)                                                                          \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            throw ::pano::Error{PANO_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)
#define PANO_REQUIRE(cond, msg)                                  \
    do {                                                         \
        if (!(cond)) throw ::pano::Error{PANO_EINVAL, (msg)};    \
    } while (0)

// ---------------------------------------------------------------- host linalg
void parallel_for(int64_t n, int64_t min_chunk, const std::function<void(int64_t, int64_t)> &fn);
std::vector<int64_t> seeded_sample(int64_t n, int64_t count, uint64_t seed);
void mean_cov_fp64(const float *x, int64_t n, int d, const std::vector<int64_t> &rows,
                   std::vector<double> &mu, std::vector<double> &cov);
bool symmetric_eigen(const std::vector<double> &sym, int n, std::vector<double> &evals,
                     std::vector<double> &evecs_rows);

// ---------------------------------------------------------------- device memory
struct DevMem {
    void *p = nullptr;
    size_t bytes = 0;
    DevMem() = default;
    DevMem(const DevMem &) = delete;
    DevMem &operator=(const DevMem &) = delete;
    ~DevMem() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    void alloc(size_t b)
    {
        release();
        if (b == 0) b = 256;
        if (hipMalloc(&p, b) != hipSuccess) {
            p = nullptr;
            throw Error{PANO_ENOMEM, "hipMalloc of " + std::to_string(b) + " bytes failed"};
        }
        bytes = b;
    }
    void ensure(size_t b)
    {
        if (b > bytes) alloc(b + b / 4);
    }
    template <class T> T *as() const { return reinterpret_cast<T *>(p); }
};

// ---------------------------------------------------------------- error model
// Constants of the certified floating-point margins.  u = 2^-24 (FP32 unit
// roundoff); gamma(n) = n u / (1 - n u).
struct Margins {
    float c_level[65];  // coefficient on the head distance after level l (l = 1..L)
    float c_tail;       // coefficient on (a + b)^2 for the tail term
    float e_max;        // max over stored rows of the transform error bound
    float kappa;        // per-unit-norm transform error bound (queries use kappa*||v||)
    float rho;          // sigma_max/sigma_min of the FP32 transform times (1+u')/(1-u') root
    float c_final;      // coefficient on D~ for the error of the full distance
    float c_abs;        // per-query absolute margin A_q = c_abs (a_0^2 + b0max2) for the
                        // dot-product form (matrix-core level 1 and brute force)
    float b0max2;       // bound on the largest stored squared norm
};

// Up to MAXSEG buffers cleared (or set to a 32-bit pattern) by one kernel.
struct FillList {
    static constexpr int MAXSEG = 14;
    void *p[MAXSEG];
    int64_t n[MAXSEG];  // counts of 32-bit words
    uint32_t v[MAXSEG];
    int m;
    void add(void *ptr, int64_t count, uint32_t val)
    {
        if (m >= MAXSEG) throw Error{PANO_EUNSUPPORTED, "too many buffers to clear"};
        p[m] = ptr;
        n[m] = count;
        v[m] = val;
        ++m;
    }
};

// Identity of a captured search graph: every value baked into its nodes.
struct GraphKey {
    uint64_t ix_serial;  // unique per index built, so a freed index's address cannot match
    const void *q;
    int64_t nq;
    int k;
    const void *npd;
    int np_all;
    float eps;
    bool brute;
    const void *ids, *dists;
    int G, bpi, seed_pool, seed_cnt, grid, dense_min, bf16, split, walk_lanes, walk2;
    const void *s0, *s1, *s2, *s3, *s5, *s6, *pinned;
    bool operator==(const GraphKey &o) const
    {
        return ix_serial == o.ix_serial && q == o.q && nq == o.nq && k == o.k && npd == o.npd && np_all == o.np_all &&
               eps == o.eps && brute == o.brute && ids == o.ids && dists == o.dists && G == o.G && bpi == o.bpi &&
               seed_pool == o.seed_pool && seed_cnt == o.seed_cnt && grid == o.grid && dense_min == o.dense_min &&
               bf16 == o.bf16 && split == o.split && walk_lanes == o.walk_lanes && walk2 == o.walk2 && s0 == o.s0 && s1 == o.s1 &&
               s2 == o.s2 && s3 == o.s3 && s5 == o.s5 && s6 == o.s6 && pinned == o.pinned;
    }
};

}  // namespace pano

// ---------------------------------------------------------------- handles
struct pano_ctx {
    int device = 0;
    int num_cu = 256;
    pano::DevMem scratch[12];
    // the context's own stream (default priority), events and graph cache
    hipStream_t stream = nullptr, aux = nullptr, aux2 = nullptr;
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_join2 = nullptr;
    hipEvent_t ev_in = nullptr;
    // the end of the last asynchronous search, while it may still run: the
    // next search is ordered after it, and nothing it uses is freed before it
    hipEvent_t ev_async = nullptr;
    bool async_pending = false;
    hipGraphExec_t graph_exec = nullptr;
    pano::GraphKey graph_key{};
    void *pinned = nullptr;
    size_t pinned_bytes = 0;
    pano::DevMem status;  // asynchronous searches: count of non-finite queries since the last status call

    void status_ensure()
    {
        if (status.p) return;
        status.alloc(256);
        if (hipMemset(status.p, 0, 256) != hipSuccess) throw pano::Error{PANO_EDEVICE, "hipMemset failed"};
    }

    hipStream_t work_stream()
    {
        if (!stream) {
            if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess)
                throw pano::Error{PANO_EDEVICE, "hipStreamCreate failed"};
            for (auto &e : ev)
                if (hipEventCreate(&e) != hipSuccess) throw pano::Error{PANO_EDEVICE, "hipEventCreate failed"};
            if (hipEventCreateWithFlags(&ev_in, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&ev_join, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&ev_join2, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&ev_async, hipEventDisableTiming) != hipSuccess)
                throw pano::Error{PANO_EDEVICE, "hipEventCreate failed"};
            if (hipStreamCreateWithFlags(&aux, hipStreamNonBlocking) != hipSuccess ||
                hipStreamCreateWithFlags(&aux2, hipStreamNonBlocking) != hipSuccess)
                throw pano::Error{PANO_EDEVICE, "hipStreamCreate failed"};
        }
        return stream;
    }
    void pinned_ensure(size_t b)
    {
        if (b <= pinned_bytes) return;
        drop_graph();
        if (pinned) (void)hipHostFree(pinned);
        pinned = nullptr;
        pinned_bytes = 0;
        size_t nb = b + b / 4 + 256;
        if (hipHostMalloc(&pinned, nb, hipHostMallocDefault) != hipSuccess)
            throw pano::Error{PANO_ENOMEM, "hipHostMalloc failed"};
        pinned_bytes = nb;
    }
    // wait for the last asynchronous search (before its memory or graph goes)
    void quiesce()
    {
        if (!async_pending) return;
        async_pending = false;
        if (hipEventSynchronize(ev_async) != hipSuccess) throw pano::Error{PANO_EDEVICE, "hipEventSynchronize failed"};
    }
    void drop_graph()
    {
        quiesce();
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        graph_exec = nullptr;
    }
    ~pano_ctx()
    {
        if (async_pending) (void)hipEventSynchronize(ev_async);
        async_pending = false;
        drop_graph();
        if (pinned) (void)hipHostFree(pinned);
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        if (ev_join2) (void)hipEventDestroy(ev_join2);
        if (ev_async) (void)hipEventDestroy(ev_async);
        if (aux) (void)hipStreamDestroy(aux);
        if (aux2) (void)hipStreamDestroy(aux2);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

// the IVFPQ index: shaped transform, PQ codebooks and the sub-quantizer-major
// block layout of the codes
struct pano_pq_index {
    pano_ctx *ctx = nullptr;
    int64_t n = 0;
    int d = 0, nlist = 0, L = 0, M = 0, dsub = 0;
    std::vector<int> cuts;     // level cuts in coordinates
    std::vector<int> sub_off;  // level cuts in sub-quantizers
    std::vector<int64_t> list_blk, list_len, top_blk_prefix;
    int64_t nblocks = 0;
    pano::DevMem Tt64, mu64;  // shaped transform in FP64, transposed (Tt[j][i] = T[i][j]), and the mean
    pano::DevMem codebooks;   // [M][256][dsub] FP32
    pano::DevMem codes_row;   // [n][M] codes of the residuals T (x - c) in row order
    pano::DevMem codes;       // [nblocks][M][256]
    pano::DevMem tails;       // [nblocks][L - 1][256] norms of xhat beyond levels 1..L-1
    pano::DevMem ids;         // [nblocks][256], -1 for empty slots
    pano::DevMem blk_cnt;     // [nblocks]
    pano::DevMem list_blk_d;  // [nlist + 1]
    pano::DevMem cent;        // [nlist][d] raw-space centroids, then their squared norms
    pano::DevMem yc64;        // [nlist][d] the centroids in the shaped frame, FP64
    pano::DevMem sx;          // [nblocks][L][256] per slot and level: sum of ||C||^2 + 2 <y_c, C> over its codes
    pano::DevMem ycn;         // [nlist] norms of the shaped centroids (rounded up)
    pano::DevMem b0max;       // [nlist] the largest reconstruction norm of each list (rounded up)
    pano::DevMem block_list;  // [nblocks] the list of each block
    int64_t last_stats[5] = {0, 0, 0, 0, 0};
    double last_ms_scan = 0.0;
};

struct pano_transform {
    int d = 0;
    std::vector<double> mu, T, lambda;
    double alpha = 0.0;
};

struct pano_index {
    pano_ctx *ctx = nullptr;
    uint64_t serial = 0;  // process-wide build counter
    int64_t n = 0;
    int d = 0, d_pad = 0, nlist = 0, L = 0, B = 256;
    bool has_bf16 = false;
    std::vector<int32_t> m, mp, wp;          // cuts, padded cuts, padded widths
    std::vector<int64_t> list_len, list_blk; // list lengths, block offsets (nlist+1)
    std::vector<int64_t> top_blk_prefix;     // [i]: blocks of the i largest lists together (nlist+1)
    int64_t nblocks = 0, max_list_len = 0, max_list_blocks = 0;
    pano::DevMem mu32, T32, cent, raw, levels, levels_bf16, tails, ids, blk_cnt, list_blk_d,
        list_len_d, meta;
    pano::DevMem idpos;  // row id -> block * B + slot (built on the first refine)
    pano::Margins mg{};
    double transform_err_max = 0.0, sigma_ratio = 1.0;
    float c_abs_bf = 0.f;  // c_abs of the bfloat16 scan (two query terms per product, u_b^2 split error)
    pano_stats_t stats{};
};

namespace pano {

// ---------------------------------------------------------------- device launchers
// Level geometry passed to kernels by value.
struct LevelGeom {
    int L;
    int d;
    int d_pad;
    int B;
    int mp[65];  // padded cuts
    int wp[64];  // padded widths
};

// One dense product Out[r][outcol ? outcol[c] : c] = sum_k (A[r][k] - mu[k])
// Bm[c][k] (mu may be null) for r < n, c < nb, K = reduction length, with the
// chunked FP32 accumulation of launch_transform.
struct GemmJob {
    const float *A;
    int64_t n;
    int K;
    const float *Bm;
    int nb;
    const float *mu;
    const int32_t *outcol;
    float *Out;
    int ld_out;
};
GemmJob transform_job(const float *X, int64_t n, int d, const float *T, const float *mu, const int32_t *padcol,
                      float *Y, int ld_y);
GemmJob product_job(const float *A, int64_t n, int d, const float *Bm, int nb, float *S);
// Both jobs (j1 may be null) in one launch: their tiles run side by side.
// clear: buffers the kernel fills in a prologue (none of them is read by it)
void launch_gemm_jobs(const GemmJob &j0, const GemmJob *j1, hipStream_t s, const FillList *clear = nullptr);

// Y[r][padcol[j]] = sum_j T[i][j] * (X[r][j] - mu[j]) with chunked FP32
// accumulation; Y has ld_y columns (padding columns are left untouched).
void launch_transform(const float *X, int64_t n, int d, const float *T, const float *mu,
                      const int32_t *padcol, float *Y, int ld_y, hipStream_t s);
// Dense product S[r][c] = sum_j A[r][j] * Bm[c][j] (FP32), for k-means and the
// coarse step.
void launch_gemm_nt(const float *A, int64_t n, int d, const float *Bm, int nb, float *S,
                    hipStream_t s);
// Optional per-query outputs of launch_row_norms: the error bound E_q, the
// absolute margin A_q of the dot-product form, and a flag set when a query
// has a non-finite value.
struct QueryConstsOut {
    Margins mg;
    float *qE = nullptr;
    float *qA = nullptr;
    int32_t *badq = nullptr;  // per row: 1 if the row has a non-finite value, else 0
};
// Per row: tail norms sqrt(sum_{j >= mp_l} y_j^2) for l = 0..L-1 (FP64 sums),
// and ||fl(x - mu)|| in FP64 (vnorm); with qc, the query constants too.
void launch_row_norms(const float *Y, int64_t n, const LevelGeom &g, const float *X, const float *mu,
                      float *tails_rowmajor, double *vnorm, hipStream_t s, const QueryConstsOut *qc = nullptr);
void launch_argmin_rows(const float *S, int64_t n, int nb, const float *cnorm, int32_t *assign,
                        hipStream_t s);
void launch_assign_canon(const float *S, int64_t n, int nb, const float *cnorm, const float *X, const float *cent,
                         int d, int32_t *assign, hipStream_t s);
void launch_centroid_update(const float *X, int d, const int64_t *perm, const int64_t *off, int nlist,
                            float *cent, hipStream_t s);
void launch_sqnorms(const float *X, int64_t n, int d, float *out, hipStream_t s);
void launch_update_mind(const float *X, int64_t n, int d, const float *c, float *mind, hipStream_t s);
void launch_cand_potential(const float *X, int64_t n, int d, const float *cand, int nc, const float *mind,
                           double *pot, hipStream_t s);
std::vector<std::pair<int, int>> shape_plan(const std::vector<double> &lam, const std::vector<int> &cuts, double kappa,
                                            std::vector<double> *v_out);
void haar_rotation(int n, uint64_t seed, uint64_t stream, std::vector<double> &Q);
std::vector<double> shape_transform(std::vector<double> &T, int d, const std::vector<double> &lam,
                                    const std::vector<int> &cuts, double kappa, bool isotropize, uint64_t seed);
// The coarse step: every query's p = min(nprobe, nlist, np_max) nearest lists
// by (canonical D, list id), written to probes[q][0..p) (the rest -1) and
// npq[q] = p, with list_cnt[l] += queries probing l (list_cnt must be zero
// before).  S [nq][nlist] = q c^T from the tiled FP32 product (launch_gemm_nt
// or the search's product job), cn2 the centroids' squared norms, qn2 (may be
// null) receives ||q||^2.  nlist = 1 puts every query on list 0.
// coarse_prepare picks the kernels for (nlist, d) and sets their attributes
// (call it outside graph capture); coarse_enqueue only launches.
struct CoarsePlan {
    int nlist = 1, d = 0;
    float c_co = 0.f;         // relative error bound of the product-form distances
    size_t lds_wave = 0;      // LDS bytes per wavefront of the LDS instance
    int wpb = 1;              // wavefronts per workgroup of the LDS instance
    const void *regs = nullptr, *finish = nullptr, *lds = nullptr;
};
float coarse_error_bound(int d);
CoarsePlan coarse_prepare(int nlist, int d);
void coarse_enqueue(const CoarsePlan &cp, const float *S, const float *cn2, const float *q, const float *cent, int64_t nq,
                    const int32_t *nprobe_dev, int nprobe_all, int np_max, int32_t *probes, int32_t *npq,
                    int32_t *list_cnt, float *qn2, hipStream_t s);
void launch_coarse_probes(const float *S, const float *cn2, const float *q, const float *cent, int d, int nlist,
                          int64_t nq, const int32_t *nprobe_dev, int nprobe_all, int np_max, int32_t *probes,
                          int32_t *npq, int32_t *list_cnt, float *qn2, hipStream_t s);
void run_pq_build(pano_ctx *ctx, pano_pq_index *ix, const pano_transform *tf, const float *x_dev,
                  const float *centroids_dev, const int32_t *assign_dev, int iters, int64_t sample, uint64_t seed,
                  hipStream_t s);
void run_pq_search(pano_ctx *ctx, pano_pq_index *ix, const float *q, int64_t nq, int k, const int32_t *nprobe_dev,
                   int nprobe_all, float eps, int64_t *ids, float *dists, uint32_t flags, hipStream_t s);
void launch_gather_rows(const float *X, const int64_t *rows, int64_t n, int d, float *out, hipStream_t s);
void launch_pack(const float *Y, const float *tails_row, const int64_t *perm, const int64_t *list_start,
                 const int64_t *list_blk, const int32_t *block_list, int64_t nblocks, const LevelGeom &g,
                 float *levels, uint16_t *levels_bf16, float *tails, int32_t *ids, int32_t *blk_cnt,
                 hipStream_t s);

// fixed: when not null, every scratch buffer of the search is carved from
// this device memory of fixed_bytes (the allocation-free entry point): no
// allocation, no graph, every kernel on stream s.
void run_search(pano_ctx *ctx, pano_index *idx, const float *q, int64_t nq, int k, const int32_t *nprobe_dev,
                int nprobe_all, float eps, int64_t *ids, float *dists, const pano_search_params *prm,
                uint32_t flags, bool brute, hipStream_t s, void *fixed = nullptr, size_t fixed_bytes = 0);
// The point-centric refine of given candidate ids (synchronous).
void run_audit_bounds(pano_ctx *ctx, pano_index *ix, const float *q, int64_t nq, const int32_t *pair_q,
                      const int64_t *pair_row, int64_t npairs, bool bf, float *out, float *rows, hipStream_t s);
void run_refine(pano_ctx *ctx, pano_index *ix, const float *q, int64_t nq, int k, const int64_t *cand, int kprime,
                float eps, int64_t *ids, float *dists, hipStream_t s);
// Bytes of fixed scratch a search needs (the allocation-free entry point).
size_t search_fixed_bytes(const pano_index *ix, int64_t nq, int k, bool per_query_np, int nprobe_all,
                          const pano_search_params *prm);
// Device address of this device's fixed scratch array (set up on first use
// with the device current).
void *fixed_scratch(int device);
size_t search_scratch_bytes(const pano_index *ix, int64_t nq, int k, bool per_query_np, int nprobe_all,
                            const pano_search_params *prm, bool brute);

}  // namespace pano
