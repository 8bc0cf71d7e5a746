/*
 * Plain C oracle for the pruned k-NN scan: the same definitions as the numpy
 * oracle (oracle/brute.py, oracle/panorama.py), written as simple loops with
 * OpenMP over queries.  TEST INFRASTRUCTURE ONLY: it is built and called only
 * by the test suite and the benchmark's CPU-baseline leg, and shares no code
 * with the HIP library.
 *
 * Compile with -ffp-contract=off: the canonical distance is a sequential FP64
 * sum in which every product and every sum is rounded separately.
 *
 * Definitions followed:
 *   Problem 1 (Section 3): the k candidates nearest to q, ties at equal
 *     canonical distance D broken by the smaller id.
 *   Problem 2 (Section 3) with IVF probing: the candidate set is every vector of
 *     the nprobe lists nearest to q by (D(q, c_l), l).
 *   Eq. 2-4 and Algorithm 1: a heap seeded with the exact distances of the
 *     first k candidates; batches of B candidates with the threshold frozen per
 *     batch; prune when LB_eps^l > d_k (+ a slack for FP64 and FP32 rounding);
 *     survivors' exact distances pushed to the heap, which is cropped to k.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Canonical distance: sum over j in order of ((double)q_j - (double)x_j)^2. */
static float canon(const float *q, const float *x, int d)
{
    double s = 0.0;
    for (int j = 0; j < d; ++j) {
        double t = (double)q[j] - (double)x[j];
        double t2 = t * t;
        s = s + t2;
    }
    return (float)s;
}

float orc_canonical_dist(const float *q, const float *x, int d) { return canon(q, x, d); }

/* (dist, id) strict order. */
static int key_less(float da, int64_t ia, float db, int64_t ib)
{
    return (da < db) || (da == db && ia < ib);
}

/* Keep the k best (dist, id) pairs of a small sorted array; insert one. */
static void heap_insert(float *hd, int64_t *hi, int *cnt, int k, float dv, int64_t iv)
{
    int c = *cnt;
    if (c == k && !key_less(dv, iv, hd[k - 1], hi[k - 1]))
        return;
    int pos = (c < k) ? c : k - 1;
    while (pos > 0 && key_less(dv, iv, hd[pos - 1], hi[pos - 1])) {
        hd[pos] = hd[pos - 1];
        hi[pos] = hi[pos - 1];
        --pos;
    }
    hd[pos] = dv;
    hi[pos] = iv;
    if (c < k)
        *cnt = c + 1;
}

static void set_threads(int threads)
{
#ifdef _OPENMP
    if (threads > 0)
        omp_set_num_threads(threads);
#else
    (void)threads;
#endif
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* O2 probe sets: the first nprobe[q] lists by (D(q, c_l), l); probes is
 * [nq][maxp], unused slots -1. */
void orc_probe(const float *qs, int64_t nq, const float *cent, int nlist, int d,
               const int32_t *nprobe, int maxp, int32_t *probes, int threads)
{
    set_threads(threads);
#pragma omp parallel
    {
        float *hd = (float *)malloc(sizeof(float) * (size_t)maxp);
        int64_t *hi = (int64_t *)malloc(sizeof(int64_t) * (size_t)maxp);
#pragma omp for schedule(dynamic, 1)
        for (int64_t qi = 0; qi < nq; ++qi) {
            int p = nprobe[qi];
            if (p < 1) p = 1;
            if (p > nlist) p = nlist;
            if (p > maxp) p = maxp;
            int cnt = 0;
            for (int l = 0; l < nlist; ++l)
                heap_insert(hd, hi, &cnt, p, canon(qs + qi * d, cent + (int64_t)l * d, d), l);
            for (int r = 0; r < maxp; ++r)
                probes[qi * maxp + r] = r < cnt ? (int32_t)hi[r] : -1;
        }
        free(hd);
        free(hi);
    }
}

/* O1/O2 brute force over an explicit candidate list per query (CSR:
 * cand_off[nq+1], cand_ids[]). */
void orc_knn_lists(const float *qs, int64_t nq, const float *xs, int d,
                   const int64_t *cand_off, const int64_t *cand_ids, int k,
                   int64_t *ids, float *dists, int threads)
{
    set_threads(threads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t qi = 0; qi < nq; ++qi) {
        float *hd = dists + qi * k;
        int64_t *hi = ids + qi * k;
        int cnt = 0;
        for (int64_t c = cand_off[qi]; c < cand_off[qi + 1]; ++c) {
            int64_t id = cand_ids[c];
            heap_insert(hd, hi, &cnt, k, canon(qs + qi * d, xs + id * d, d), id);
        }
        for (int r = cnt; r < k; ++r) {
            hd[r] = INFINITY;
            hi[r] = -1;
        }
    }
}

/* Section 4.1 transform applied in FP64: ys = T (x - mu), T row-major. */
void orc_transform(const double *mu, const double *T, const float *xs, int64_t n, int d,
                   double *ys, int threads)
{
    set_threads(threads);
#pragma omp parallel
    {
        double *v = (double *)malloc(sizeof(double) * (size_t)d);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            for (int j = 0; j < d; ++j)
                v[j] = (double)xs[i * d + j] - mu[j];
            for (int r = 0; r < d; ++r) {
                double s = 0.0;
                for (int j = 0; j < d; ++j)
                    s += T[(int64_t)r * d + j] * v[j];
                ys[i * d + r] = s;
            }
        }
        free(v);
    }
}

/* Eq. 2 tails: R[i][l] = sum_{j >= m[l]} ys[i][j]^2 for l = 0..L. */
void orc_tails(const double *ys, int64_t n, int d, const int32_t *m, int L, double *R, int threads)
{
    set_threads(threads);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        int l = L;
        R[i * (L + 1) + L] = 0.0;
        for (int j = d - 1; j >= 0; --j) {
            acc += ys[i * d + j] * ys[i * d + j];
            while (l > 0 && j == m[l - 1]) {
                --l;
                R[i * (L + 1) + l] = acc;
            }
        }
    }
}

/*
 * Algorithm 1 per query over its candidate list (CSR cand_off/cand_ids, in
 * probe-rank then list order), with the database already transformed (ys) and
 * its tails (R) precomputed; the query transform is done here (it is part of
 * the query's cost).  Returns ids/dists [nq][k] and the number of dimensions
 * read per query in dims_read.
 */
void orc_panorama(const float *qs, int64_t nq, const float *xs, const double *ys, const double *R,
                  int d, const double *mu, const double *T, const int32_t *m, int L,
                  const int64_t *cand_off, const int64_t *cand_ids, int k, int batch, double eps,
                  int64_t *ids, float *dists, int64_t *dims_read, int threads)
{
    set_threads(threads);
#pragma omp parallel
    {
        double *tq = (double *)malloc(sizeof(double) * (size_t)d);
        double *v = (double *)malloc(sizeof(double) * (size_t)d);
        double *rq = (double *)malloc(sizeof(double) * (size_t)(L + 1));
        double *p = (double *)malloc(sizeof(double) * (size_t)batch);
        char *alive = (char *)malloc((size_t)batch);
#pragma omp for schedule(dynamic, 1)
        for (int64_t qi = 0; qi < nq; ++qi) {
            const float *q = qs + qi * d;
            for (int j = 0; j < d; ++j)
                v[j] = (double)q[j] - mu[j];
            for (int r = 0; r < d; ++r) {
                double s = 0.0;
                for (int j = 0; j < d; ++j)
                    s += T[(int64_t)r * d + j] * v[j];
                tq[r] = s;
            }
            for (int l = 0; l <= L; ++l) {
                double s = 0.0;
                for (int j = m[l]; j < d; ++j)
                    s += tq[j] * tq[j];
                rq[l] = s;
            }
            float *hd = dists + qi * k;
            int64_t *hi = ids + qi * k;
            int cnt = 0;
            int64_t nread = 0;
            int64_t c0 = cand_off[qi], c1 = cand_off[qi + 1];
            int64_t seed_end = c0 + k < c1 ? c0 + k : c1;
            for (int64_t c = c0; c < seed_end; ++c) {
                int64_t id = cand_ids[c];
                heap_insert(hd, hi, &cnt, k, canon(q, xs + id * d, d), id);
                nread += d;
            }
            double dk = cnt == k ? (double)hd[k - 1] : INFINITY;
            for (int64_t b0 = seed_end; b0 < c1; b0 += batch) {
                int nb = (int)((c1 - b0) < batch ? (c1 - b0) : batch);
                for (int i = 0; i < nb; ++i) {
                    p[i] = 0.0;
                    alive[i] = 1;
                }
                for (int l = 1; l <= L; ++l) {
                    for (int i = 0; i < nb; ++i) {
                        if (!alive[i])
                            continue;
                        int64_t id = cand_ids[b0 + i];
                        const double *y = ys + id * d;
                        double s = 0.0;
                        for (int j = m[l - 1]; j < m[l]; ++j)
                            s += tq[j] * y[j];
                        p[i] += s;
                        double rx0 = R[id * (L + 1)];
                        double rxl = R[id * (L + 1) + l];
                        double lb = rq[0] + rx0 - 2.0 * (p[i] + eps * sqrt(rq[l] * rxl));
                        double slack = ldexp(dk, -22) + 1e-11 * (rq[0] + rx0);
                        if (lb > dk + slack) {
                            alive[i] = 0;
                            nread += m[l];
                        }
                    }
                }
                for (int i = 0; i < nb; ++i) {
                    if (!alive[i])
                        continue;
                    int64_t id = cand_ids[b0 + i];
                    nread += d;
                    heap_insert(hd, hi, &cnt, k, canon(q, xs + id * d, d), id);
                }
                dk = cnt == k ? (double)hd[k - 1] : INFINITY;
            }
            for (int r = cnt; r < k; ++r) {
                hd[r] = INFINITY;
                hi[r] = -1;
            }
            dims_read[qi] = nread;
        }
        free(tq);
        free(v);
        free(rq);
        free(p);
        free(alive);
    }
}
