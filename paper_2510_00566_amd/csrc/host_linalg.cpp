// Host-side FP64 linear algebra for the PCA fit (Section 4.1): mean and
// covariance accumulation over a seeded sample of rows, and a symmetric
// eigensolver (Householder reduction to tridiagonal form followed by the
// implicit symmetric QR iteration with Wilkinson shifts, as described in
// Golub & Van Loan, "Matrix Computations", Sections 8.3.1 and 8.3.3).
// Independent rows of the eigenvector matrix are updated on several threads.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <functional>
#include <thread>
#include <vector>

namespace pano {

static int host_threads()
{
    unsigned h = std::thread::hardware_concurrency();
    if (h == 0) h = 4;
    return (int)std::min<unsigned>(h, 32);
}

void parallel_for(int64_t n, int64_t min_chunk, const std::function<void(int64_t, int64_t)> &fn)
{
    int t = host_threads();
    int64_t chunks = std::max<int64_t>(1, std::min<int64_t>(t, n / std::max<int64_t>(1, min_chunk)));
    if (chunks <= 1) {
        fn(0, n);
        return;
    }
    std::vector<std::thread> th;
    int64_t per = (n + chunks - 1) / chunks;
    for (int64_t c = 0; c < chunks; ++c) {
        int64_t b = c * per, e = std::min(n, b + per);
        if (b >= e) break;
        th.emplace_back(fn, b, e);
    }
    for (auto &x : th) x.join();
}

static uint64_t splitmix64(uint64_t &s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

std::vector<int64_t> seeded_sample(int64_t n, int64_t count, uint64_t seed)
{
    std::vector<int64_t> out;
    if (count <= 0 || count >= n) {
        out.resize(n);
        for (int64_t i = 0; i < n; ++i) out[i] = i;
        return out;
    }
    // Partial Fisher-Yates over an index array.
    std::vector<int64_t> idx(n);
    for (int64_t i = 0; i < n; ++i) idx[i] = i;
    uint64_t s = seed;
    for (int64_t i = 0; i < count; ++i) {
        uint64_t r = splitmix64(s) % (uint64_t)(n - i);
        std::swap(idx[i], idx[i + (int64_t)r]);
    }
    out.assign(idx.begin(), idx.begin() + count);
    std::sort(out.begin(), out.end());
    return out;
}

void mean_cov_fp64(const float *x, int64_t n, int d, const std::vector<int64_t> &rows,
                   std::vector<double> &mu, std::vector<double> &cov)
{
    const int64_t s = (int64_t)rows.size();
    mu.assign(d, 0.0);
    {
        int t = host_threads();
        std::vector<std::vector<double>> part(t, std::vector<double>(d, 0.0));
        int64_t per = (s + t - 1) / t;
        std::vector<std::thread> th;
        for (int c = 0; c < t; ++c) {
            th.emplace_back([&, c]() {
                int64_t b = c * per, e = std::min(s, b + per);
                for (int64_t r = b; r < e; ++r) {
                    const float *row = x + rows[r] * (int64_t)d;
                    for (int j = 0; j < d; ++j) part[c][j] += (double)row[j];
                }
            });
        }
        for (auto &z : th) z.join();
        for (int c = 0; c < t; ++c)
            for (int j = 0; j < d; ++j) mu[j] += part[c][j];
        for (int j = 0; j < d; ++j) mu[j] /= (double)s;
    }
    // Centred rows in chunks, transposed so the inner product over the chunk
    // is unit stride; each thread owns a set of output rows of the covariance.
    cov.assign((size_t)d * d, 0.0);
    const int CH = 128;
    std::vector<double> xt((size_t)d * CH);
    for (int64_t r0 = 0; r0 < s; r0 += CH) {
        int cn = (int)std::min<int64_t>(CH, s - r0);
        for (int c = 0; c < cn; ++c) {
            const float *row = x + rows[r0 + c] * (int64_t)d;
            for (int j = 0; j < d; ++j) xt[(size_t)j * CH + c] = (double)row[j] - mu[j];
        }
        for (int c = cn; c < CH; ++c)
            for (int j = 0; j < d; ++j) xt[(size_t)j * CH + c] = 0.0;
        parallel_for(d, 8, [&](int64_t ib, int64_t ie) {
            for (int64_t i = ib; i < ie; ++i) {
                const double *xi = &xt[(size_t)i * CH];
                double *ci = &cov[(size_t)i * d];
                for (int64_t j = i; j < d; ++j) {
                    const double *xj = &xt[(size_t)j * CH];
                    double acc = 0.0;
                    for (int c = 0; c < CH; ++c) acc += xi[c] * xj[c];
                    ci[j] += acc;
                }
            }
        });
    }
    for (int i = 0; i < d; ++i)
        for (int j = i; j < d; ++j) {
            double v = cov[(size_t)i * d + j] / (double)s;
            cov[(size_t)i * d + j] = v;
            cov[(size_t)j * d + i] = v;
        }
}

// Householder reduction of the symmetric matrix a (n x n, row-major, destroyed)
// to tridiagonal form: a = Q T Q^t.  diag/off receive T, q receives Q.
static void tridiagonalize(std::vector<double> &a, int n, std::vector<double> &diag,
                           std::vector<double> &off, std::vector<double> &q)
{
    std::vector<std::vector<double>> vs(std::max(0, n - 2));
    std::vector<double> betas(std::max(0, n - 2), 0.0);
    std::vector<double> p(n), w(n);
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;  // length of the column below the diagonal
        std::vector<double> &v = vs[k];
        v.assign(m, 0.0);
        double norm2 = 0.0;
        for (int i = 0; i < m; ++i) {
            v[i] = a[(size_t)(k + 1 + i) * n + k];
            norm2 += v[i] * v[i];
        }
        double nrm = std::sqrt(norm2);
        if (nrm == 0.0) {
            betas[k] = 0.0;
            continue;
        }
        double alpha = v[0] > 0 ? -nrm : nrm;
        v[0] -= alpha;
        double vv = 0.0;
        for (int i = 0; i < m; ++i) vv += v[i] * v[i];
        if (vv == 0.0) {
            betas[k] = 0.0;
            continue;
        }
        double beta = 2.0 / vv;
        betas[k] = beta;
        // p = beta * S v on the trailing block S = a[k+1:, k+1:]
        parallel_for(m, 32, [&](int64_t ib, int64_t ie) {
            for (int64_t i = ib; i < ie; ++i) {
                const double *row = &a[(size_t)(k + 1 + i) * n + (k + 1)];
                double acc = 0.0;
                for (int j = 0; j < m; ++j) acc += row[j] * v[j];
                p[i] = beta * acc;
            }
        });
        double pv = 0.0;
        for (int i = 0; i < m; ++i) pv += p[i] * v[i];
        double kk = 0.5 * beta * pv;
        for (int i = 0; i < m; ++i) w[i] = p[i] - kk * v[i];
        parallel_for(m, 32, [&](int64_t ib, int64_t ie) {
            for (int64_t i = ib; i < ie; ++i) {
                double *row = &a[(size_t)(k + 1 + i) * n + (k + 1)];
                const double vi = v[i], wi = w[i];
                for (int j = 0; j < m; ++j) row[j] -= vi * w[j] + wi * v[j];
            }
        });
        a[(size_t)(k + 1) * n + k] = alpha;
        a[(size_t)k * n + (k + 1)] = alpha;
        for (int i = 1; i < m; ++i) {
            a[(size_t)(k + 1 + i) * n + k] = 0.0;
            a[(size_t)k * n + (k + 1 + i)] = 0.0;
        }
    }
    diag.assign(n, 0.0);
    off.assign(std::max(0, n - 1), 0.0);
    for (int i = 0; i < n; ++i) diag[i] = a[(size_t)i * n + i];
    for (int i = 0; i + 1 < n; ++i) off[i] = a[(size_t)(i + 1) * n + i];
    // Q = H_0 H_1 ... H_{n-3}, accumulated from the right end.
    q.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) q[(size_t)i * n + i] = 1.0;
    std::vector<double> wt(n);
    for (int k = n - 3; k >= 0; --k) {
        if (betas[k] == 0.0) continue;
        const std::vector<double> &v = vs[k];
        const int m = n - k - 1;
        const int o = k + 1;
        // wt = v^t Q[o:, o:]
        std::fill(wt.begin(), wt.end(), 0.0);
        for (int i = 0; i < m; ++i) {
            const double vi = v[i];
            const double *row = &q[(size_t)(o + i) * n + o];
            for (int j = 0; j < m; ++j) wt[j] += vi * row[j];
        }
        const double beta = betas[k];
        parallel_for(m, 32, [&](int64_t ib, int64_t ie) {
            for (int64_t i = ib; i < ie; ++i) {
                double *row = &q[(size_t)(o + i) * n + o];
                const double s = beta * v[i];
                for (int j = 0; j < m; ++j) row[j] -= s * wt[j];
            }
        });
    }
}

// Implicit symmetric QR steps with Wilkinson shift on the tridiagonal
// (diag, off); the rotations are applied to the columns of z.
static bool tridiagonal_qr(std::vector<double> &diag, std::vector<double> &off, std::vector<double> &z,
                           int n)
{
    const double eps = std::ldexp(1.0, -52);
    std::vector<double> cs(n), sn(n);
    int64_t guard = 0;
    const int64_t max_steps = 60LL * n + 100;
    int hi = n - 1;
    while (hi > 0) {
        // deflate negligible off-diagonal entries
        for (int i = 0; i < hi; ++i)
            if (std::fabs(off[i]) <= eps * (std::fabs(diag[i]) + std::fabs(diag[i + 1]))) off[i] = 0.0;
        while (hi > 0 && off[hi - 1] == 0.0) --hi;
        if (hi == 0) break;
        int lo = hi - 1;
        while (lo > 0 && off[lo - 1] != 0.0) --lo;
        if (++guard > max_steps) return false;
        // Wilkinson shift from the trailing 2x2 block of the active window.
        double dl = 0.5 * (diag[hi - 1] - diag[hi]);
        double bb = off[hi - 1] * off[hi - 1];
        double den = dl + std::copysign(std::sqrt(dl * dl + bb), dl);
        double mu = diag[hi] - (den != 0.0 ? bb / den : 0.0);
        double x = diag[lo] - mu, zb = off[lo];
        double bulge = 0.0;
        int nrot = 0;
        for (int k = lo; k < hi; ++k) {
            if (k > lo) {
                x = off[k - 1];
                zb = bulge;
            }
            double r = std::hypot(x, zb);
            double c = 1.0, s = 0.0;
            if (r != 0.0) {
                c = x / r;
                s = zb / r;
            }
            if (k > lo) off[k - 1] = r;
            double ak = diag[k], ak1 = diag[k + 1], bk = off[k];
            diag[k] = c * c * ak + 2.0 * c * s * bk + s * s * ak1;
            diag[k + 1] = s * s * ak - 2.0 * c * s * bk + c * c * ak1;
            off[k] = c * s * (ak1 - ak) + (c * c - s * s) * bk;
            if (k + 1 < hi) {
                bulge = s * off[k + 1];
                off[k + 1] = c * off[k + 1];
            }
            cs[nrot] = c;
            sn[nrot] = s;
            ++nrot;
        }
        // z <- z G_lo ... G_{hi-1}; rows are independent.
        parallel_for(n, 64, [&](int64_t rb, int64_t re) {
            for (int64_t r = rb; r < re; ++r) {
                double *row = &z[(size_t)r * n];
                for (int t = 0; t < nrot; ++t) {
                    const int k = lo + t;
                    const double a0 = row[k], a1 = row[k + 1];
                    row[k] = cs[t] * a0 + sn[t] * a1;
                    row[k + 1] = -sn[t] * a0 + cs[t] * a1;
                }
            }
        });
    }
    return true;
}

bool symmetric_eigen(const std::vector<double> &sym, int n, std::vector<double> &evals,
                     std::vector<double> &evecs_rows)
{
    std::vector<double> a = sym, diag, off, z;
    if (n == 1) {
        evals.assign(1, sym[0]);
        evecs_rows.assign(1, 1.0);
        return true;
    }
    tridiagonalize(a, n, diag, off, z);
    if (!tridiagonal_qr(diag, off, z, n)) return false;
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int i, int j) { return diag[i] > diag[j]; });
    evals.resize(n);
    evecs_rows.assign((size_t)n * n, 0.0);
    for (int r = 0; r < n; ++r) {
        const int c = order[r];
        evals[r] = diag[c];
        // canonical sign: largest-magnitude entry positive
        int piv = 0;
        double best = -1.0;
        for (int i = 0; i < n; ++i) {
            double v = std::fabs(z[(size_t)i * n + c]);
            if (v > best) {
                best = v;
                piv = i;
            }
        }
        double sgn = z[(size_t)piv * n + c] < 0 ? -1.0 : 1.0;
        for (int i = 0; i < n; ++i) evecs_rows[(size_t)r * n + i] = sgn * z[(size_t)i * n + c];
    }
    return true;
}

}  // namespace pano
