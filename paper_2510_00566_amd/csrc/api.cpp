// C ABI of the pruned k-NN scan: argument checking, handle management, the
// index build (transform, tails, level-major packing) and the search
// orchestration.  Every exported function catches all exceptions and maps
// them to a pano_status with a thread-local message.
#include "internal.h"
#include "search_common.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <memory>

namespace pano {

static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }

template <class F> static pano_status guarded(F &&f)
{
    try {
        g_last_error.clear();
        f();
        return PANO_OK;
    } catch (const Error &e) {
        g_last_error = e.msg;
        return e.st;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return PANO_ENOMEM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return PANO_EDEVICE;
    } catch (...) {
        g_last_error = "unknown failure";
        return PANO_EDEVICE;
    }
}

static double gamma_n(double nn)
{
    const double u = std::ldexp(1.0, -24);
    return nn * u / (1.0 - nn * u);
}

// Certified error constants of the FP32 path (see the design notes):
//  * transform outputs carry |err| <= kappa ||fl(v - mu)||, kappa from the
//    chunked accumulation bound and the row/column sums of |T32|;
//  * the FP32 matrix has singular values in [sqrt(1 - delta), sqrt(1 + delta)]
//    with delta = ||T32 T32^t - I||_F;
//  * a head distance over m coordinates has relative error <= gamma(m + L + 24).
static void compute_margins(pano_index *ix, const std::vector<float> &T32)
{
    const int d = ix->d;
    const double u = std::ldexp(1.0, -24);
    std::vector<double> rs(d, 0.0), cs(d, 0.0);
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            double a = std::fabs((double)T32[(size_t)i * d + j]);
            rs[i] += a;
            cs[j] += a;
        }
    const double nabs = std::sqrt(*std::max_element(rs.begin(), rs.end()) * *std::max_element(cs.begin(), cs.end()));
    std::vector<double> part(d, 0.0);
    parallel_for(d, 8, [&](int64_t ib, int64_t ie) {
        for (int64_t i = ib; i < ie; ++i) {
            double acc = 0.0;
            for (int j = 0; j < d; ++j) {
                double s = 0.0;
                for (int t = 0; t < d; ++t) s += (double)T32[(size_t)i * d + t] * (double)T32[(size_t)j * d + t];
                double e = s - (i == j ? 1.0 : 0.0);
                acc += e * e;
            }
            part[i] = acc;
        }
    });
    double fro2 = 0.0;
    for (double v : part) fro2 += v;
    const double delta = std::sqrt(fro2) * (1.0 + 1e-6) + 1e-15 * d * d;
    if (delta >= 0.5) throw Error{PANO_EINVAL, "transform is not orthonormal in FP32"};
    const double smax = std::sqrt(1.0 + delta), smin = std::sqrt(1.0 - delta);
    const int tk = 32;
    // counts doubled: the bound must hold if the matrix cores' adders truncate
    const double gT = gamma_n(2.0 * ((double)tk + (d + tk - 1) / tk + 2));
    const double kappa = (gT * nabs * (1.0 + u) + smax * u * (1.0 + u)) * (1.0 + 1e-6);
    const double up = u * (1.0 + 1e-5);
    const double rho = (smax / smin) * std::sqrt((1.0 + up) / (1.0 - up)) * (1.0 + 1e-7);
    Margins &mg = ix->mg;
    std::memset(&mg, 0, sizeof(mg));
    for (int l = 1; l <= ix->L; ++l) mg.c_level[l] = (float)(gamma_n((double)ix->mp[l] + ix->L + 24) * 1.01);
    mg.c_final = mg.c_level[ix->L];
    mg.c_tail = (float)(12.0 * u);
    mg.kappa = (float)kappa;
    mg.rho = (float)rho;
    ix->sigma_ratio = smax / smin;
}

static std::atomic<uint64_t> g_index_serial{0};

static LevelGeom geom_of(const pano_index *ix)
{
    LevelGeom g{};
    g.L = ix->L;
    g.d = ix->d;
    g.d_pad = ix->d_pad;
    g.B = ix->B;
    for (int l = 0; l <= ix->L; ++l) g.mp[l] = ix->mp[l];
    for (int l = 0; l < ix->L; ++l) g.wp[l] = ix->wp[l];
    return g;
}

static bool all_finite(const float *x, int64_t count)
{
    for (int64_t i = 0; i < count; ++i)
        if (!std::isfinite(x[i])) return false;
    return true;
}

}  // namespace pano

using namespace pano;

extern "C" {

const char *pano_last_error(void) { return g_last_error.c_str(); }
const char *pano_version(void) { return "panorama-mi355x 0.1"; }

pano_status pano_ctx_create(int device, pano_ctx **out)
{
    return guarded([&] {
        PANO_REQUIRE(out != nullptr, "out is NULL");
        int count = 0;
        PANO_HIP(hipGetDeviceCount(&count));
        PANO_REQUIRE(device >= 0 && device < count, "device index out of range");
        PANO_HIP(hipSetDevice(device));
        // set up this device's fixed scratch of the allocation-free search
        // while the device is current
        (void)fixed_scratch(device);
        auto *c = new pano_ctx();
        c->device = device;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->num_cu = prop.multiProcessorCount;
        *out = c;
    });
}

void pano_ctx_destroy(pano_ctx *ctx) { delete ctx; }

pano_status pano_ctx_scratch_bytes(const pano_ctx *ctx, int64_t *bytes)
{
    return guarded([&] {
        PANO_REQUIRE(ctx && bytes, "null argument");
        int64_t t = 0;
        for (const auto &m : ctx->scratch) t += (int64_t)m.bytes;
        *bytes = t;
    });
}

pano_status pano_ctx_status(pano_ctx *ctx, int64_t *nonfinite_queries)
{
    return guarded([&] {
        PANO_REQUIRE(ctx && nonfinite_queries, "null argument");
        PANO_HIP(hipSetDevice(ctx->device));
        PANO_HIP(hipDeviceSynchronize());
        unsigned long long v = 0;
        if (ctx->status.p) {
            PANO_HIP(hipMemcpy(&v, ctx->status.p, sizeof(v), hipMemcpyDeviceToHost));
            PANO_HIP(hipMemset(ctx->status.p, 0, sizeof(v)));
        }
        *nonfinite_queries = (int64_t)v;
        PANO_REQUIRE(v == 0, "asynchronous searches met queries with a non-finite value");
    });
}

pano_status pano_ctx_trim(pano_ctx *ctx)
{
    return guarded([&] {
        PANO_REQUIRE(ctx, "null argument");
        PANO_HIP(hipSetDevice(ctx->device));
        if (ctx->stream) PANO_HIP(hipStreamSynchronize(ctx->stream));
        ctx->drop_graph();
        for (auto &m : ctx->scratch) m.release();
    });
}

pano_status pano_build_transform(const float *x_host, int64_t n, int32_t d, int64_t fit_sample, uint64_t seed,
                                 pano_transform **out)
{
    return guarded([&] {
        PANO_REQUIRE(out != nullptr && x_host != nullptr, "null argument");
        PANO_REQUIRE(n >= 2 && d >= 1, "need n >= 2 rows and d >= 1");
        std::vector<int64_t> rows = seeded_sample(n, fit_sample, seed);
        for (int64_t r : rows)
            PANO_REQUIRE(all_finite(x_host + r * (int64_t)d, d), "x has a non-finite value");
        auto tf = std::make_unique<pano_transform>();
        tf->d = d;
        std::vector<double> cov;
        mean_cov_fp64(x_host, n, d, rows, tf->mu, cov);
        if (!symmetric_eigen(cov, d, tf->lambda, tf->T))
            throw Error{PANO_EDEVICE, "eigensolver did not converge"};
        // alpha: least-squares fit of log E(m) ~ -alpha m / d where E(m) >= 1e-3
        std::vector<double> tail(d + 1, 0.0);
        for (int j = d - 1; j >= 0; --j) tail[j] = tail[j + 1] + std::max(tf->lambda[j], 0.0);
        double sxx = 0.0, sxy = 0.0;
        for (int m = 0; m < d; ++m) {
            double e = tail[0] > 0 ? tail[m] / tail[0] : 0.0;
            if (e < 1e-3) continue;
            double xm = (double)m / d;
            sxx += xm * xm;
            sxy += xm * std::log(e);
        }
        tf->alpha = sxx > 0 ? -sxy / sxx : 0.0;
        *out = tf.release();
    });
}

pano_status pano_transform_identity(int32_t d, pano_transform **out)
{
    return guarded([&] {
        PANO_REQUIRE(out != nullptr && d >= 1, "bad arguments");
        auto tf = std::make_unique<pano_transform>();
        tf->d = d;
        tf->mu.assign(d, 0.0);
        tf->T.assign((size_t)d * d, 0.0);
        for (int i = 0; i < d; ++i) tf->T[(size_t)i * d + i] = 1.0;
        tf->lambda.assign(d, 0.0);
        *out = tf.release();
    });
}

pano_status pano_transform_from(int32_t d, const double *mu_host, const double *T_host, pano_transform **out)
{
    return guarded([&] {
        PANO_REQUIRE(out != nullptr && mu_host != nullptr && T_host != nullptr && d >= 1, "bad arguments");
        double worst = 0.0;
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) {
                double s = 0.0;
                for (int t = 0; t < d; ++t) s += T_host[(size_t)i * d + t] * T_host[(size_t)j * d + t];
                worst = std::max(worst, std::fabs(s - (i == j ? 1.0 : 0.0)));
            }
        PANO_REQUIRE(worst <= 1e-9, "T is not orthonormal to 1e-9");
        auto tf = std::make_unique<pano_transform>();
        tf->d = d;
        tf->mu.assign(mu_host, mu_host + d);
        tf->T.assign(T_host, T_host + (size_t)d * d);
        tf->lambda.assign(d, 0.0);
        *out = tf.release();
    });
}

pano_status pano_transform_get(const pano_transform *tf, int32_t *d, double *mu_host, double *T_host,
                               double *lambda_host, double *alpha)
{
    return guarded([&] {
        PANO_REQUIRE(tf != nullptr, "transform is NULL");
        if (d) *d = tf->d;
        if (mu_host) std::copy(tf->mu.begin(), tf->mu.end(), mu_host);
        if (T_host) std::copy(tf->T.begin(), tf->T.end(), T_host);
        if (lambda_host) std::copy(tf->lambda.begin(), tf->lambda.end(), lambda_host);
        if (alpha) *alpha = tf->alpha;
    });
}

void pano_transform_free(pano_transform *tf) { delete tf; }

pano_status pano_ivf_assign(pano_ctx *ctx, const float *x_dev, int64_t n, int32_t d, int32_t nlist, int32_t iters,
                            uint64_t seed, float *centroids_dev, int32_t *assign_dev, void *stream)
{
    return guarded([&] {
        PANO_REQUIRE(ctx && x_dev && centroids_dev && assign_dev, "null argument");
        PANO_REQUIRE(n >= 1 && d >= 1 && nlist >= 1 && nlist <= n, "need 1 <= nlist <= n");
        PANO_REQUIRE(iters >= 0, "iters must be >= 0");
        PANO_HIP(hipSetDevice(ctx->device));
        hipStream_t s = (hipStream_t)stream;
        // initial centroids: k-means++ (D^2 sampling, Arthur & Vassilvitskii 2007)
        // over a seeded sample of rows
        {
            const int64_t ns = std::min<int64_t>(n, std::max<int64_t>(65536, std::min<int64_t>(262144, 64LL * nlist)));
            std::vector<int64_t> samp = seeded_sample(n, ns, seed ^ 0x5bd1e995ull);
            DevMem rows_d, xs, mind;
            rows_d.alloc(sizeof(int64_t) * ns);
            xs.alloc(sizeof(float) * (size_t)ns * d);
            mind.alloc(sizeof(float) * ns);
            PANO_HIP(hipMemcpyAsync(rows_d.p, samp.data(), sizeof(int64_t) * ns, hipMemcpyHostToDevice, s));
            launch_gather_rows(x_dev, rows_d.as<int64_t>(), ns, d, xs.as<float>(), s);
            PANO_HIP(hipMemsetD32Async((hipDeviceptr_t)mind.p, 0x7f800000, ns, s));
            uint64_t st = seed * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
            auto next_u01 = [&st]() {
                uint64_t z = (st += 0x9E3779B97F4A7C15ull);
                z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
                z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
                z ^= z >> 31;
                return (double)(z >> 11) * (1.0 / 9007199254740992.0);
            };
            // greedy variant: each step draws several candidates by D^2 and keeps
            // the one that lowers the potential most
            const int ncand = std::min(16, 2 + (int)std::log((double)nlist));
            DevMem cand_d, pot_d;
            cand_d.alloc(sizeof(float) * (size_t)ncand * d);
            pot_d.alloc(sizeof(double) * ncand);
            std::vector<float> hm(ns);
            std::vector<double> pot(ncand);
            std::vector<int64_t> picks(ncand);
            int64_t pick = (int64_t)(next_u01() * ns) % ns;
            for (int c = 0; c < nlist; ++c) {
                PANO_HIP(hipMemcpyAsync(centroids_dev + (int64_t)c * d, xs.as<float>() + pick * d, sizeof(float) * d,
                                        hipMemcpyDeviceToDevice, s));
                if (c + 1 == nlist) break;
                launch_update_mind(xs.as<float>(), ns, d, centroids_dev + (int64_t)c * d, mind.as<float>(), s);
                PANO_HIP(hipMemcpyAsync(hm.data(), mind.p, sizeof(float) * ns, hipMemcpyDeviceToHost, s));
                PANO_HIP(hipStreamSynchronize(s));
                std::vector<double> cum(ns);
                double tot = 0.0;
                for (int64_t i = 0; i < ns; ++i) {
                    tot += (double)hm[i];
                    cum[i] = tot;
                }
                if (!(tot > 0.0)) {
                    pick = (int64_t)(next_u01() * ns) % ns;
                    continue;
                }
                for (int t = 0; t < ncand; ++t) {
                    double r = next_u01() * tot;
                    int64_t i = std::upper_bound(cum.begin(), cum.end(), r) - cum.begin();
                    picks[t] = std::min<int64_t>(i, ns - 1);
                    PANO_HIP(hipMemcpyAsync(cand_d.as<float>() + (size_t)t * d, xs.as<float>() + picks[t] * d,
                                            sizeof(float) * d, hipMemcpyDeviceToDevice, s));
                }
                PANO_HIP(hipMemsetAsync(pot_d.p, 0, sizeof(double) * ncand, s));
                launch_cand_potential(xs.as<float>(), ns, d, cand_d.as<float>(), ncand, mind.as<float>(),
                                      pot_d.as<double>(), s);
                PANO_HIP(hipMemcpyAsync(pot.data(), pot_d.p, sizeof(double) * ncand, hipMemcpyDeviceToHost, s));
                PANO_HIP(hipStreamSynchronize(s));
                int best = 0;
                for (int t = 1; t < ncand; ++t)
                    if (pot[t] < pot[best]) best = t;
                pick = picks[best];
            }
        }
        DevMem S, cn, perm_d, off_d;
        const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(n, (int64_t)(1ll << 28) / std::max(1, nlist)));
        S.alloc(sizeof(float) * chunk * nlist);
        cn.alloc(sizeof(float) * nlist);
        perm_d.alloc(sizeof(int64_t) * n);
        off_d.alloc(sizeof(int64_t) * (nlist + 1));
        std::vector<int32_t> asg(n);
        std::vector<int64_t> perm(n), off(nlist + 1);
        // the iterations assign by the FP32 score; the final pass by the
        // canonical (D, l) key
        auto assign_pass = [&](bool canonical) {
            launch_sqnorms(centroids_dev, nlist, d, cn.as<float>(), s);
            for (int64_t r0 = 0; r0 < n; r0 += chunk) {
                int64_t rn = std::min(chunk, n - r0);
                launch_gemm_nt(x_dev + r0 * d, rn, d, centroids_dev, nlist, S.as<float>(), s);
                if (canonical)
                    launch_assign_canon(S.as<float>(), rn, nlist, cn.as<float>(), x_dev + r0 * d, centroids_dev, d,
                                        assign_dev + r0, s);
                else
                    launch_argmin_rows(S.as<float>(), rn, nlist, cn.as<float>(), assign_dev + r0, s);
            }
        };
        for (int it = 0; it < iters; ++it) {
            assign_pass(false);
            PANO_HIP(hipMemcpyAsync(asg.data(), assign_dev, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
            PANO_HIP(hipStreamSynchronize(s));
            std::fill(off.begin(), off.end(), 0);
            for (int64_t i = 0; i < n; ++i) off[asg[i] + 1]++;
            for (int c = 0; c < nlist; ++c) off[c + 1] += off[c];
            std::vector<int64_t> fill(off.begin(), off.end() - 1);
            for (int64_t i = 0; i < n; ++i) perm[fill[asg[i]]++] = i;
            PANO_HIP(hipMemcpyAsync(perm_d.p, perm.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, s));
            PANO_HIP(hipMemcpyAsync(off_d.p, off.data(), sizeof(int64_t) * (nlist + 1), hipMemcpyHostToDevice, s));
            launch_centroid_update(x_dev, d, perm_d.as<int64_t>(), off_d.as<int64_t>(), nlist, centroids_dev, s);
            PANO_HIP(hipStreamSynchronize(s));
        }
        assign_pass(true);
        PANO_HIP(hipStreamSynchronize(s));
    });
}

pano_status pano_build_levels(pano_ctx *ctx, const pano_transform *tf, const float *x_dev, int64_t n, int32_t d,
                              const float *centroids_dev, const int32_t *assign_dev, int32_t nlist,
                              const int32_t *m_host, int32_t L, int32_t block, pano_dtype store, pano_index **out,
                              void *stream)
{
    return guarded([&] {
        // argument values first, so that they are reported even for null handles
        if (block == 0) block = 256;
        PANO_REQUIRE(block == 64 || block == 128 || block == 256, "block must be 64, 128 or 256");
        PANO_REQUIRE(store == PANO_F32 || store == PANO_BF16, "unknown storage dtype");
        PANO_REQUIRE(n >= 1 && d >= 1 && nlist >= 1, "bad sizes");
        PANO_REQUIRE(L >= 1 && L <= 64, "L must be in [1, 64]");
        PANO_REQUIRE(m_host != nullptr, "null argument");
        PANO_REQUIRE(m_host[0] == 0 && m_host[L] == d, "level cuts must start at 0 and end at d");
        for (int l = 0; l < L; ++l) PANO_REQUIRE(m_host[l] < m_host[l + 1], "level cuts must increase");
        {
            int w0 = (m_host[1] + 3) / 4 * 4, dp = 0;
            for (int l = 0; l < L; ++l) dp += (m_host[l + 1] - m_host[l] + 3) / 4 * 4;
            PANO_REQUIRE(w0 <= 64, "the first level may hold at most 64 dimensions");
            PANO_REQUIRE(dp <= 4096, "d up to 4096 is supported");
        }
        PANO_REQUIRE(ctx && tf && x_dev && centroids_dev && assign_dev && out, "null argument");
        PANO_REQUIRE(tf->d == d, "transform dimension does not match d");
        PANO_HIP(hipSetDevice(ctx->device));
        hipStream_t s = (hipStream_t)stream;
        auto ix = std::make_unique<pano_index>();
        ix->ctx = ctx;
        ix->serial = ++g_index_serial;
        ix->n = n;
        ix->d = d;
        ix->nlist = nlist;
        ix->L = L;
        ix->B = block;
        ix->m.assign(m_host, m_host + L + 1);
        ix->mp.assign(L + 1, 0);
        ix->wp.assign(L, 0);
        for (int l = 0; l < L; ++l) {
            ix->wp[l] = ((m_host[l + 1] - m_host[l]) + 3) / 4 * 4;
            ix->mp[l + 1] = ix->mp[l] + ix->wp[l];
        }
        ix->d_pad = ix->mp[L];
        PANO_REQUIRE(ix->wp[0] <= 64, "the first level may hold at most 64 dimensions");
        PANO_REQUIRE(ix->d_pad <= 4096, "d up to 4096 is supported");
        ix->has_bf16 = store == PANO_BF16;
        // transform in FP32
        std::vector<float> T32((size_t)d * d), mu32(d);
        for (size_t i = 0; i < T32.size(); ++i) T32[i] = (float)tf->T[i];
        for (int j = 0; j < d; ++j) mu32[j] = (float)tf->mu[j];
        compute_margins(ix.get(), T32);
        ix->T32.alloc(sizeof(float) * T32.size());
        ix->mu32.alloc(sizeof(float) * d);
        PANO_HIP(hipMemcpyAsync(ix->T32.p, T32.data(), sizeof(float) * T32.size(), hipMemcpyHostToDevice, s));
        PANO_HIP(hipMemcpyAsync(ix->mu32.p, mu32.data(), sizeof(float) * d, hipMemcpyHostToDevice, s));
        std::vector<int32_t> padcol(d);
        for (int l = 0; l < L; ++l)
            for (int j = m_host[l]; j < m_host[l + 1]; ++j) padcol[j] = ix->mp[l] + (j - m_host[l]);
        DevMem padcol_d, Y, tails_row, vnorm;
        padcol_d.alloc(sizeof(int32_t) * d);
        PANO_HIP(hipMemcpyAsync(padcol_d.p, padcol.data(), sizeof(int32_t) * d, hipMemcpyHostToDevice, s));
        ix->meta.alloc(sizeof(int32_t) * d);
        PANO_HIP(hipMemcpyAsync(ix->meta.p, padcol.data(), sizeof(int32_t) * d, hipMemcpyHostToDevice, s));
        Y.alloc(sizeof(float) * (size_t)n * ix->d_pad);
        PANO_HIP(hipMemsetAsync(Y.p, 0, Y.bytes, s));
        launch_transform(x_dev, n, d, ix->T32.as<float>(), ix->mu32.as<float>(), padcol_d.as<int32_t>(), Y.as<float>(),
                         ix->d_pad, s);
        tails_row.alloc(sizeof(float) * (size_t)n * L);
        vnorm.alloc(sizeof(double) * n);
        LevelGeom g = geom_of(ix.get());
        launch_row_norms(Y.as<float>(), n, g, x_dev, ix->mu32.as<float>(), tails_row.as<float>(), vnorm.as<double>(), s);
        std::vector<double> vn(n);
        PANO_HIP(hipMemcpyAsync(vn.data(), vnorm.p, sizeof(double) * n, hipMemcpyDeviceToHost, s));
        std::vector<int32_t> asg(n);
        PANO_HIP(hipMemcpyAsync(asg.data(), assign_dev, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
        PANO_HIP(hipStreamSynchronize(s));
        double vmax = 0.0;
        for (double v : vn) vmax = std::max(vmax, v);
        ix->transform_err_max = (double)ix->mg.kappa * vmax * (1.0 + 1e-6);
        ix->mg.e_max = (float)(ix->transform_err_max * (1.0 + 1e-6));
        {
            // ||y|| <= sigma_max ||v|| + kappa ||v|| for every stored row
            const double smax = std::sqrt(1.0 + (ix->sigma_ratio * ix->sigma_ratio - 1.0));
            const double b0 = (smax + (double)ix->mg.kappa) * vmax * (1.0 + 1e-6);
            ix->mg.b0max2 = (float)(b0 * b0 * (1.0 + 1e-6));
            int wmax = 0;
            for (int l = 0; l < L; ++l) wmax = std::max(wmax, ix->wp[l]);
            // covers the dot-product form of any number of levels: per level
            // gamma(w + 2)(R_q + R_x) for the product plus 4u (a_l^2 + b_l^2) for
            // the level energies taken as differences of squared tails.  The
            // counts are doubled so that the bound also holds if the matrix
            // cores' adders truncate instead of rounding to nearest.
            ix->mg.c_abs = (float)((gamma_n(2.0 * (wmax + 4.0 * L + 16)) + 6.0 * std::ldexp(1.0, -24)) * 1.01);
            // bfloat16 scan: 2w products per level (q = q_hi + q_lo), the level
            // energies of the rounded rows summed in FP32, and the split error
            // 2 u_b^2 |<q, x~>| <= u_b^2 (R_q + R_x~)
            const double ub = std::ldexp(1.0, -8);
            ix->c_abs_bf = (float)((gamma_n(2.0 * (2.0 * wmax + 4.0 * L + 16)) + 6.0 * std::ldexp(1.0, -24) +
                                    ub * ub * (1.0 + ub)) *
                                   1.01);
        }
        // lists: stable counting sort by assignment
        ix->list_len.assign(nlist, 0);
        for (int64_t i = 0; i < n; ++i) {
            PANO_REQUIRE(asg[i] >= 0 && asg[i] < nlist, "assignment out of range");
            ix->list_len[asg[i]]++;
        }
        std::vector<int64_t> start(nlist + 1, 0);
        for (int l = 0; l < nlist; ++l) start[l + 1] = start[l] + ix->list_len[l];
        std::vector<int64_t> perm(n);
        {
            std::vector<int64_t> fill(start.begin(), start.end() - 1);
            for (int64_t i = 0; i < n; ++i) perm[fill[asg[i]]++] = i;
        }
        ix->list_blk.assign(nlist + 1, 0);
        for (int l = 0; l < nlist; ++l) {
            int64_t nb = (ix->list_len[l] + block - 1) / block;
            ix->list_blk[l + 1] = ix->list_blk[l] + nb;
            ix->max_list_len = std::max(ix->max_list_len, ix->list_len[l]);
            ix->max_list_blocks = std::max(ix->max_list_blocks, nb);
        }
        ix->nblocks = ix->list_blk[nlist];
        {
            std::vector<int64_t> nb(nlist);
            for (int l = 0; l < nlist; ++l) nb[l] = ix->list_blk[l + 1] - ix->list_blk[l];
            std::sort(nb.begin(), nb.end(), std::greater<int64_t>());
            ix->top_blk_prefix.assign(nlist + 1, 0);
            for (int l = 0; l < nlist; ++l) ix->top_blk_prefix[l + 1] = ix->top_blk_prefix[l] + nb[l];
        }
        std::vector<int32_t> block_list(std::max<int64_t>(1, ix->nblocks));
        for (int l = 0; l < nlist; ++l)
            for (int64_t b = ix->list_blk[l]; b < ix->list_blk[l + 1]; ++b) block_list[b] = l;
        DevMem perm_d, start_d, block_list_d;
        perm_d.alloc(sizeof(int64_t) * n);
        start_d.alloc(sizeof(int64_t) * (nlist + 1));
        block_list_d.alloc(sizeof(int32_t) * block_list.size());
        ix->list_blk_d.alloc(sizeof(int64_t) * (nlist + 1));
        ix->list_len_d.alloc(sizeof(int64_t) * nlist);
        PANO_HIP(hipMemcpyAsync(perm_d.p, perm.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, s));
        PANO_HIP(hipMemcpyAsync(start_d.p, start.data(), sizeof(int64_t) * (nlist + 1), hipMemcpyHostToDevice, s));
        PANO_HIP(hipMemcpyAsync(block_list_d.p, block_list.data(), sizeof(int32_t) * block_list.size(),
                                hipMemcpyHostToDevice, s));
        PANO_HIP(hipMemcpyAsync(ix->list_blk_d.p, ix->list_blk.data(), sizeof(int64_t) * (nlist + 1),
                                hipMemcpyHostToDevice, s));
        PANO_HIP(hipMemcpyAsync(ix->list_len_d.p, ix->list_len.data(), sizeof(int64_t) * nlist, hipMemcpyHostToDevice, s));
        const size_t slots = (size_t)ix->nblocks * block;
        ix->levels.alloc(sizeof(float) * slots * ix->d_pad);
        if (ix->has_bf16) ix->levels_bf16.alloc(sizeof(uint16_t) * slots * ix->d_pad);
        ix->tails.alloc(sizeof(float) * slots * L);
        ix->ids.alloc(sizeof(int32_t) * slots);
        ix->blk_cnt.alloc(sizeof(int32_t) * std::max<int64_t>(1, ix->nblocks));
        launch_pack(Y.as<float>(), tails_row.as<float>(), perm_d.as<int64_t>(), start_d.as<int64_t>(),
                    ix->list_blk_d.as<int64_t>(), block_list_d.as<int32_t>(), ix->nblocks, g, ix->levels.as<float>(),
                    ix->has_bf16 ? ix->levels_bf16.as<uint16_t>() : nullptr, ix->tails.as<float>(),
                    ix->ids.as<int32_t>(), ix->blk_cnt.as<int32_t>(), s);
        ix->raw.alloc(sizeof(float) * (size_t)n * d);
        PANO_HIP(hipMemcpyAsync(ix->raw.p, x_dev, sizeof(float) * (size_t)n * d, hipMemcpyDeviceToDevice, s));
        ix->cent.alloc(sizeof(float) * ((size_t)nlist * d + nlist));
        PANO_HIP(hipMemcpyAsync(ix->cent.p, centroids_dev, sizeof(float) * (size_t)nlist * d, hipMemcpyDeviceToDevice, s));
        launch_sqnorms(ix->cent.as<float>(), nlist, d, ix->cent.as<float>() + (size_t)nlist * d, s);
        PANO_HIP(hipStreamSynchronize(s));
        *out = ix.release();
    });
}

pano_status pano_search_ctx(pano_ctx *ctx, pano_index *idx, const float *q_dev, int64_t nq, int32_t k,
                            const int32_t *nprobe_dev, int32_t nprobe_all, float eps, int64_t *ids_dev,
                            float *dists_dev, const pano_search_params *params, uint32_t flags, void *stream)
{
    return guarded([&] {
        PANO_REQUIRE(ctx && idx && (nq == 0 || (q_dev && ids_dev && dists_dev)), "null argument");
        PANO_REQUIRE(k >= 1 && nq >= 0, "need k >= 1 and nq >= 0");
        PANO_REQUIRE(eps >= 0.f && eps <= 1.f, "eps must be in [0, 1]");
        PANO_REQUIRE(nprobe_dev != nullptr || nprobe_all >= 1, "nprobe_all must be >= 1");
        if (nq == 0) return;
        run_search(ctx, idx, q_dev, nq, k, nprobe_dev, nprobe_all, eps, ids_dev, dists_dev, params, flags, false,
                   (hipStream_t)stream);
    });
}

pano_status pano_search(pano_index *idx, const float *q_dev, int64_t nq, int32_t k, const int32_t *nprobe_dev,
                        int32_t nprobe_all, float eps, int64_t *ids_dev, float *dists_dev,
                        const pano_search_params *params, uint32_t flags, void *stream)
{
    if (!idx) {
        set_error("null argument");
        return PANO_EINVAL;
    }
    return pano_search_ctx(idx->ctx, idx, q_dev, nq, k, nprobe_dev, nprobe_all, eps, ids_dev, dists_dev, params,
                           flags, stream);
}

pano_status pano_search_noalloc(pano_index *idx, const float *q_dev, int64_t nq, int32_t k,
                                const int32_t *nprobe_dev, int32_t nprobe_all, float eps, int64_t *ids_dev,
                                float *dists_dev, const pano_search_params *params, void *stream)
{
    return guarded([&] {
        PANO_REQUIRE(idx && (nq == 0 || (q_dev && ids_dev && dists_dev)), "null argument");
        PANO_REQUIRE(k >= 1 && nq >= 0, "need k >= 1 and nq >= 0");
        PANO_REQUIRE(eps >= 0.f && eps <= 1.f, "eps must be in [0, 1]");
        PANO_REQUIRE(nprobe_dev != nullptr || nprobe_all >= 1, "nprobe_all must be >= 1");
        if (nq == 0) return;
        PANO_HIP(hipSetDevice(idx->ctx->device));
        void *fx = fixed_scratch(idx->ctx->device);
        run_search(idx->ctx, idx, q_dev, nq, k, nprobe_dev, nprobe_all, eps, ids_dev, dists_dev, params, 0u, false,
                   (hipStream_t)stream, fx, NOALLOC_SCRATCH_BYTES);
    });
}

pano_status pano_refine(pano_index *idx, const float *q_dev, int64_t nq, int32_t k, const int64_t *cand_dev,
                        int32_t kprime, float eps, int64_t *ids_dev, float *dists_dev, void *stream)
{
    return guarded([&] {
        PANO_REQUIRE(idx && (nq == 0 || (q_dev && cand_dev && ids_dev && dists_dev)), "null argument");
        PANO_REQUIRE(k >= 1 && nq >= 0 && kprime >= 1, "need k >= 1, kprime >= 1 and nq >= 0");
        PANO_REQUIRE(eps >= 0.f && eps <= 1.f, "eps must be in [0, 1]");
        if (nq == 0) return;
        run_refine(idx->ctx, idx, q_dev, nq, k, cand_dev, kprime, eps, ids_dev, dists_dev, (hipStream_t)stream);
    });
}

pano_status pano_audit_bounds(pano_index *idx, const float *q_dev, int64_t nq, const int32_t *pair_q_dev,
                              const int64_t *pair_row_dev, int64_t npairs, int32_t bf16, float *bounds_dev,
                              float *rows_dev, void *stream)
{
    return guarded([&] {
        PANO_REQUIRE(idx && (npairs == 0 || (q_dev && pair_q_dev && pair_row_dev && bounds_dev)), "null argument");
        PANO_REQUIRE(nq >= 1 && npairs >= 0, "need nq >= 1 and npairs >= 0");
        run_audit_bounds(idx->ctx, idx, q_dev, nq, pair_q_dev, pair_row_dev, npairs, bf16 != 0, bounds_dev, rows_dev,
                         (hipStream_t)stream);
    });
}

pano_status pano_search_scratch_bytes(const pano_index *idx, int64_t nq, int32_t k, int32_t per_query_nprobe,
                                      int32_t nprobe_all, const pano_search_params *params, int64_t *bytes)
{
    return guarded([&] {
        PANO_REQUIRE(idx && bytes, "null argument");
        PANO_REQUIRE(k >= 1 && nq >= 0, "need k >= 1 and nq >= 0");
        PANO_REQUIRE(per_query_nprobe || nprobe_all >= 1, "nprobe_all must be >= 1");
        *bytes = (int64_t)search_scratch_bytes(idx, nq, k, per_query_nprobe != 0, nprobe_all, params, false);
    });
}

pano_status pano_search_bruteforce(pano_index *idx, const float *q_dev, int64_t nq, int32_t k,
                                   const int32_t *nprobe_dev, int32_t nprobe_all, int64_t *ids_dev, float *dists_dev,
                                   const pano_search_params *params, uint32_t flags, void *stream)
{
    return guarded([&] {
        PANO_REQUIRE(idx && (nq == 0 || (q_dev && ids_dev && dists_dev)), "null argument");
        PANO_REQUIRE(k >= 1 && nq >= 0, "need k >= 1 and nq >= 0");
        PANO_REQUIRE(nprobe_dev != nullptr || nprobe_all >= 1, "nprobe_all must be >= 1");
        if (nq == 0) return;
        run_search(idx->ctx, idx, q_dev, nq, k, nprobe_dev, nprobe_all, 1.f, ids_dev, dists_dev, params, flags,
                   true, (hipStream_t)stream);
    });
}

pano_status pano_index_info(const pano_index *idx, pano_index_info_t *out)
{
    return guarded([&] {
        PANO_REQUIRE(idx && out, "null argument");
        std::memset(out, 0, sizeof(*out));
        out->n = idx->n;
        out->d = idx->d;
        out->d_pad = idx->d_pad;
        out->nlist = idx->nlist;
        out->L = idx->L;
        out->block = idx->B;
        out->has_bf16 = idx->has_bf16;
        out->nblocks = idx->nblocks;
        out->max_list_len = idx->max_list_len;
        const int64_t slots = idx->nblocks * idx->B;
        out->bytes_levels = slots * idx->d_pad * 4;
        out->bytes_levels_bf16 = idx->has_bf16 ? slots * idx->d_pad * 2 : 0;
        out->bytes_tails = slots * idx->L * 4;
        out->bytes_ids = slots * 4;
        out->bytes_raw = idx->n * idx->d * 4;
        out->transform_err_max = idx->transform_err_max;
        out->sigma_ratio = idx->sigma_ratio;
    });
}

pano_status pano_index_layout(const pano_index *idx, int32_t *m_host, int64_t *list_len_host)
{
    return guarded([&] {
        PANO_REQUIRE(idx, "null index");
        if (m_host) std::copy(idx->m.begin(), idx->m.end(), m_host);
        if (list_len_host) std::copy(idx->list_len.begin(), idx->list_len.end(), list_len_host);
    });
}

pano_status pano_stats_get(const pano_index *idx, pano_stats_t *out)
{
    return guarded([&] {
        PANO_REQUIRE(idx && out, "null argument");
        *out = idx->stats;
    });
}

void pano_index_free(pano_index *idx)
{
    if (!idx) return;
    // the context's captured search graph may point into this index's memory
    if (idx->ctx && idx->ctx->graph_exec && idx->ctx->graph_key.ix_serial == idx->serial) idx->ctx->drop_graph();
    delete idx;
}

// ---------------------------------------------------------------- IVFPQ
static std::vector<int> checked_cuts(const int32_t *m_host, int32_t L, int32_t d)
{
    PANO_REQUIRE(m_host != nullptr, "null argument");
    PANO_REQUIRE(L >= 1 && L <= 64, "L must be in [1, 64]");
    PANO_REQUIRE(m_host[0] == 0 && m_host[L] == d, "level cuts must start at 0 and end at d");
    for (int l = 0; l < L; ++l) PANO_REQUIRE(m_host[l] < m_host[l + 1], "level cuts must increase");
    return std::vector<int>(m_host, m_host + L + 1);
}

pano_status pano_shape_plan(const double *lambda_host, int32_t d, const int32_t *m_host, int32_t L, double kappa,
                            int32_t *blocks_host, int32_t cap, int32_t *nblocks)
{
    return guarded([&] {
        PANO_REQUIRE(lambda_host && nblocks && (cap == 0 || blocks_host), "null argument");
        PANO_REQUIRE(d >= 1, "d must be >= 1");
        PANO_REQUIRE(kappa >= 1.0, "kappa must be >= 1");
        const std::vector<int> cuts = checked_cuts(m_host, L, d);
        const auto blocks = shape_plan(std::vector<double>(lambda_host, lambda_host + d), cuts, kappa, nullptr);
        *nblocks = (int32_t)blocks.size();
        PANO_REQUIRE((int32_t)blocks.size() <= cap, "the plan has more blocks than cap");
        for (size_t i = 0; i < blocks.size(); ++i) {
            blocks_host[2 * i] = blocks[i].first;
            blocks_host[2 * i + 1] = blocks[i].second;
        }
    });
}

pano_status pano_transform_shape(const pano_transform *pca, const int32_t *m_host, int32_t L, double kappa,
                                 int32_t isotropize, uint64_t seed, pano_transform **out)
{
    return guarded([&] {
        PANO_REQUIRE(pca && out, "null argument");
        PANO_REQUIRE(kappa >= 1.0, "kappa must be >= 1");
        const std::vector<int> cuts = checked_cuts(m_host, L, pca->d);
        auto tf = std::make_unique<pano_transform>();
        tf->d = pca->d;
        tf->mu = pca->mu;
        tf->T = pca->T;
        tf->alpha = pca->alpha;
        std::vector<double> lam = pca->lambda;
        if (lam.size() != (size_t)pca->d) lam.assign(pca->d, 0.0);
        tf->lambda = shape_transform(tf->T, pca->d, lam, cuts, kappa, isotropize != 0, seed);
        *out = tf.release();
    });
}

pano_status pano_pq_build(pano_ctx *ctx, const pano_transform *tf, const float *x_dev, int64_t n, int32_t d,
                          const float *centroids_dev, const int32_t *assign_dev, int32_t nlist, const int32_t *m_host,
                          int32_t L, int32_t dsub, int32_t iters, int64_t sample, uint64_t seed, pano_pq_index **out,
                          void *stream)
{
    return guarded([&] {
        PANO_REQUIRE(n >= 256 && d >= 1 && nlist >= 1 && nlist <= n, "need n >= 256 and 1 <= nlist <= n");
        PANO_REQUIRE(dsub == 1 || dsub == 2 || dsub == 4 || dsub == 8 || dsub == 16, "dsub must be 1, 2, 4, 8 or 16");
        PANO_REQUIRE(d % dsub == 0 && d / dsub <= 128, "need d divisible by dsub and M = d / dsub <= 128");
        PANO_REQUIRE(iters >= 0, "iters must be >= 0");
        const std::vector<int> cuts = checked_cuts(m_host, L, d);
        for (int l = 0; l <= L; ++l) PANO_REQUIRE(cuts[l] % dsub == 0, "level cuts must fall on sub-vector boundaries");
        for (int l = 0; l < L; ++l)
            PANO_REQUIRE(cuts[l + 1] - cuts[l] == d / L, "the PQ index takes levels of equal width");
        PANO_REQUIRE(d / dsub / L <= 16, "at most 16 sub-quantizers per level");
        PANO_REQUIRE(ctx && tf && x_dev && centroids_dev && assign_dev && out, "null argument");
        PANO_REQUIRE(tf->d == d, "transform dimension does not match d");
        PANO_HIP(hipSetDevice(ctx->device));
        auto ix = std::make_unique<pano_pq_index>();
        ix->ctx = ctx;
        ix->n = n;
        ix->d = d;
        ix->nlist = nlist;
        ix->L = L;
        ix->dsub = dsub;
        ix->M = d / dsub;
        ix->cuts = cuts;
        ix->sub_off.resize(L + 1);
        for (int l = 0; l <= L; ++l) ix->sub_off[l] = cuts[l] / dsub;
        run_pq_build(ctx, ix.get(), tf, x_dev, centroids_dev, assign_dev, iters, sample, seed, (hipStream_t)stream);
        *out = ix.release();
    });
}

pano_status pano_pq_search(pano_ctx *ctx, pano_pq_index *idx, const float *q_dev, int64_t nq, int32_t k,
                           const int32_t *nprobe_dev, int32_t nprobe_all, float eps, int64_t *ids_dev,
                           float *dists_dev, uint32_t flags, void *stream)
{
    return guarded([&] {
        PANO_REQUIRE(ctx && idx && (nq == 0 || (q_dev && ids_dev && dists_dev)), "null argument");
        PANO_REQUIRE(k >= 1 && k <= 128 && nq >= 0, "need 1 <= k <= 128 and nq >= 0");
        PANO_REQUIRE(eps >= 0.f && eps <= 1.f, "eps must be in [0, 1]");
        PANO_REQUIRE(nprobe_dev != nullptr || nprobe_all >= 1, "nprobe_all must be >= 1");
        PANO_REQUIRE((flags & ~(PANO_PQ_BRUTE | PANO_SEARCH_STATS)) == 0, "unsupported flags");
        if (nq == 0) return;
        PANO_HIP(hipSetDevice(ctx->device));
        run_pq_search(ctx, idx, q_dev, nq, k, nprobe_dev, nprobe_all, eps, ids_dev, dists_dev, flags,
                      (hipStream_t)stream);
    });
}

pano_status pano_pq_stats(const pano_pq_index *idx, int64_t *out5, double *ms_scan)
{
    return guarded([&] {
        PANO_REQUIRE(idx && out5, "null argument");
        for (int i = 0; i < 5; ++i) out5[i] = idx->last_stats[i];
        if (ms_scan) *ms_scan = idx->last_ms_scan;
    });
}

pano_status pano_pq_export(const pano_pq_index *idx, float *codebooks_host, uint8_t *codes_host, int32_t *M_out,
                           int32_t *dsub_out)
{
    return guarded([&] {
        PANO_REQUIRE(idx, "null argument");
        if (M_out) *M_out = idx->M;
        if (dsub_out) *dsub_out = idx->dsub;
        if (!codebooks_host && !codes_host) return;
        PANO_HIP(hipSetDevice(idx->ctx->device));
        if (codebooks_host)
            PANO_HIP(hipMemcpy(codebooks_host, idx->codebooks.p, sizeof(float) * (size_t)idx->M * 256 * idx->dsub,
                               hipMemcpyDeviceToHost));
        if (codes_host)
            PANO_HIP(hipMemcpy(codes_host, idx->codes_row.p, (size_t)idx->n * idx->M, hipMemcpyDeviceToHost));
    });
}

void pano_pq_free(pano_pq_index *idx)
{
    if (!idx) return;
    if (idx->ctx) idx->ctx->quiesce();
    delete idx;
}

}  // extern "C"
