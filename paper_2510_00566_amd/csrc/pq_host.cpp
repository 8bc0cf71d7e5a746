// Host-side parts of the spectrum shaping for product quantization
// (Section 4.2): the plan of Procedure 1 (which coordinate blocks the
// Robin Hood rotations act on), seeded Haar-random orthogonal matrices, and
// the composition U R T_PCA with Procedure 2's per-level rotations.
#include "internal.h"

#include <cmath>

namespace pano {

// Procedure 1 on expected variances: v starts as the PCA eigenvalues; level
// energies are sums of v over the levels and the cap is kappa times their
// mean.  A level above the cap is rotated with the fewest following
// coordinates s >= 1 whose Haar rotation brings the level's expected energy,
// b / (b + s) times the block total, to the cap or below (s stops at the
// last coordinate); the block's coordinates then carry its mean variance.
std::vector<std::pair<int, int>> shape_plan(const std::vector<double> &lam, const std::vector<int> &cuts, double kappa,
                                            std::vector<double> *v_out)
{
    std::vector<double> v(lam);
    const int L = (int)cuts.size() - 1;
    const int d = cuts[L];
    double tot = 0.0;
    for (double x : v) tot += x;
    // an energy within a relative 1e-9 of the cap counts as within it, so that
    // rounding alone never asks for a rotation
    const double tau = kappa * tot / L;
    const double cap = tau * (1.0 + 1e-9);
    std::vector<std::pair<int, int>> blocks;
    for (int l = 0; l < L; ++l) {
        const int lo = cuts[l], hi = cuts[l + 1], b = hi - lo;
        double e = 0.0;
        for (int j = lo; j < hi; ++j) e += v[j];
        if (e <= cap) continue;
        int s = 1;
        double blk = e + (hi < d ? v[hi] : 0.0);
        while (hi + s < d && (double)b / (b + s) * blk > cap) {
            blk += v[hi + s];
            ++s;
        }
        s = std::min(s, d - hi);
        if (s == 0) continue;
        double sum = 0.0;
        for (int j = lo; j < hi + s; ++j) sum += v[j];
        const double mean = sum / (b + s);
        for (int j = lo; j < hi + s; ++j) v[j] = mean;
        blocks.emplace_back(lo, b + s);
    }
    if (v_out) *v_out = v;
    return blocks;
}

// splitmix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", 2014) over a counter: one 64-bit output per index.
static uint64_t splitmix64(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// Standard normal draws by the Box-Muller transform of pairs of uniforms in
// (0, 1) (53-bit, offset by half a step so that 0 never occurs).
static void gaussians(uint64_t seed, uint64_t stream, size_t count, std::vector<double> &out)
{
    out.resize(count);
    const uint64_t base = splitmix64(seed ^ splitmix64(stream + 0x632BE59BD9B4E019ull));
    for (size_t i = 0; i < count; i += 2) {
        const double u1 = ((double)(splitmix64(base + 2 * i) >> 11) + 0.5) * 0x1p-53;
        const double u2 = ((double)(splitmix64(base + 2 * i + 1) >> 11) + 0.5) * 0x1p-53;
        const double r = std::sqrt(-2.0 * std::log(u1)), th = 2.0 * M_PI * u2;
        out[i] = r * std::cos(th);
        if (i + 1 < count) out[i + 1] = r * std::sin(th);
    }
}

// A Haar-distributed n x n orthogonal matrix (row-major): the Q factor of a
// Gaussian matrix by Householder QR, with each column's sign set so that R has
// a positive diagonal (Mezzadri, "How to generate random matrices from the
// classical compact groups", 2007).
void haar_rotation(int n, uint64_t seed, uint64_t stream, std::vector<double> &Q)
{
    std::vector<double> A;
    gaussians(seed, stream, (size_t)n * n, A);
    // Householder vectors stored below the diagonal of A; R on and above it
    std::vector<double> beta(n, 0.0), rdiag(n, 0.0);
    for (int k = 0; k < n; ++k) {
        double nrm = 0.0;
        for (int i = k; i < n; ++i) nrm += A[(size_t)i * n + k] * A[(size_t)i * n + k];
        nrm = std::sqrt(nrm);
        const double x0 = A[(size_t)k * n + k];
        const double alpha = x0 >= 0 ? -nrm : nrm;  // R_kk
        rdiag[k] = alpha;
        const double v0 = x0 - alpha;
        double vnorm2 = v0 * v0;
        for (int i = k + 1; i < n; ++i) vnorm2 += A[(size_t)i * n + k] * A[(size_t)i * n + k];
        A[(size_t)k * n + k] = v0;
        beta[k] = vnorm2 > 0 ? 2.0 / vnorm2 : 0.0;
        // apply H_k = I - beta v v^T to the remaining columns
        for (int j = k + 1; j < n; ++j) {
            double s = 0.0;
            for (int i = k; i < n; ++i) s += A[(size_t)i * n + k] * A[(size_t)i * n + j];
            s *= beta[k];
            for (int i = k; i < n; ++i) A[(size_t)i * n + j] -= s * A[(size_t)i * n + k];
        }
    }
    // Q = H_0 H_1 ... H_{n-1}, formed by applying the reflectors to I backwards
    Q.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
    for (int k = n - 1; k >= 0; --k) {
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int i = k; i < n; ++i) s += A[(size_t)i * n + k] * Q[(size_t)i * n + j];
            s *= beta[k];
            for (int i = k; i < n; ++i) Q[(size_t)i * n + j] -= s * A[(size_t)i * n + k];
        }
    }
    // column signs: Q diag(sign(R_kk))
    for (int k = 0; k < n; ++k)
        if (rdiag[k] < 0)
            for (int i = 0; i < n; ++i) Q[(size_t)i * n + k] = -Q[(size_t)i * n + k];
}

// Rows [s, s + n) of the row-major d x d matrix T replaced by Q times them.
static void rotate_rows(std::vector<double> &T, int d, int s, int n, const std::vector<double> &Q)
{
    std::vector<double> blk((size_t)n * d);
    parallel_for(n, 8, [&](int64_t r0, int64_t r1) {
        for (int64_t r = r0; r < r1; ++r)
            for (int c = 0; c < d; ++c) {
                double acc = 0.0;
                for (int i = 0; i < n; ++i) acc += Q[(size_t)r * n + i] * T[(size_t)(s + i) * d + c];
                blk[(size_t)r * d + c] = acc;
            }
    });
    std::copy(blk.begin(), blk.end(), T.begin() + (size_t)s * d);
}

// U R T_PCA: R applies one Haar rotation per plan block (in plan order, stream
// 1 + i for block i); U one per level (stream 1000003 + l) when isotropize.
// Returns the expected per-coordinate variances of the result (the plan's,
// evened out within each level by U).
std::vector<double> shape_transform(std::vector<double> &T, int d, const std::vector<double> &lam,
                                    const std::vector<int> &cuts, double kappa, bool isotropize, uint64_t seed)
{
    std::vector<double> v;
    const auto blocks = shape_plan(lam, cuts, kappa, &v);
    std::vector<double> Q;
    for (size_t i = 0; i < blocks.size(); ++i) {
        haar_rotation(blocks[i].second, seed, 1 + i, Q);
        rotate_rows(T, d, blocks[i].first, blocks[i].second, Q);
    }
    const int L = (int)cuts.size() - 1;
    if (isotropize) {
        for (int l = 0; l < L; ++l) {
            const int n = cuts[l + 1] - cuts[l];
            haar_rotation(n, seed, 1000003ull + l, Q);
            rotate_rows(T, d, cuts[l], n, Q);
            double e = 0.0;
            for (int j = cuts[l]; j < cuts[l + 1]; ++j) e += v[j];
            for (int j = cuts[l]; j < cuts[l + 1]; ++j) v[j] = e / n;
        }
    }
    return v;
}

}  // namespace pano
