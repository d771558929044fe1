// Atom decomposition by the modified recursive bisection along inertia-tensor
// principal axes (Sec. 3.1.2-3.1.5).  Host code: it orders the atoms so that
// each of `nparts` parts is a spatially compact, weight-balanced block, for
// distributing atoms over devices and for a locality-preserving atom order.
//
// A node of the binary tree owns a contiguous range of the order array and a
// number of parts n.  A node with n == 1 or no atoms is a leaf.  Otherwise:
//   C  = weighted centre of its atoms                       (Eq. (12))
//   T  = inertia tensor about C                             (Eq. (17), (18))
//   a  = the unit eigenvector of T whose projection maximises
//        F = sum_i w_i t_i^2 on |a| = 1                     (Eq. (14)-(16))
//   t_i = a . (x_i - C)                                     (Eq. (13))
// the atoms are sorted by t (ties by atom index), the first ceil(n/2) parts
// go to the lower-t child and the rest to the upper-t child, and the split
// index puts the cumulative weight as close as possible to the lower child's
// share of the node's weight (ties: one more atom to the lower child).
//
// Readings fixed here: the centre is normalised by the total weight (with unit
// weights this is the average position of Eq. (12)); the eigenvector's sign is
// chosen so that its largest-magnitude component is positive, which fixes the
// direction of the 1-D order.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <utility>
#include <vector>

#include "partition.hpp"

namespace hartree {
namespace {

// Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix.  On return
// the diagonal of `a` holds the eigenvalues and column k of `v` the unit
// eigenvector of eigenvalue a[k][k].
void jacobi3(double a[3][3], double v[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) v[i][j] = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 64; ++sweep) {
        const double off = std::fabs(a[0][1]) + std::fabs(a[0][2]) + std::fabs(a[1][2]);
        const double diag = std::fabs(a[0][0]) + std::fabs(a[1][1]) + std::fabs(a[2][2]);
        if (off == 0.0 || off <= 1e-300 || off < 1e-18 * diag) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                const double apq = a[p][q];
                if (apq == 0.0) continue;
                // rotation angle that zeroes a[p][q]: tan(2 phi) = 2 apq / (aqq - app)
                const double theta = (a[q][q] - a[p][p]) / (2.0 * apq);
                const double t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0);
                const double s = t * c;
                for (int k = 0; k < 3; ++k) {  // columns p, q of A
                    const double akp = a[k][p], akq = a[k][q];
                    a[k][p] = c * akp - s * akq;
                    a[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {  // rows p, q of A
                    const double apk = a[p][k], aqk = a[q][k];
                    a[p][k] = c * apk - s * aqk;
                    a[q][k] = s * apk + c * aqk;
                }
                a[p][q] = a[q][p] = 0.0;
                for (int k = 0; k < 3; ++k) {
                    const double vkp = v[k][p], vkq = v[k][q];
                    v[k][p] = c * vkp - s * vkq;
                    v[k][q] = s * vkp + c * vkq;
                }
            }
    }
}

struct Bisector {
    const double *pos;
    const double *w;  // nullptr: unit weights
    int32_t *order;
    int32_t *part_start;  // nparts + 1 entries
    std::vector<std::pair<double, int32_t>> keys;
    std::vector<double> cum;

    double weight(int32_t i) const { return w ? w[i] : 1.0; }

    // Principal axis of the atoms order[lo, hi): the eigenvector of the
    // inertia tensor that maximises sum w t^2, with its centre.
    void axis(int64_t lo, int64_t hi, double c[3], double ax[3]) const
    {
        double sw = 0.0, sx[3] = {0.0, 0.0, 0.0};
        for (int64_t j = lo; j < hi; ++j) {
            const int32_t i = order[j];
            const double wi = weight(i);
            sw += wi;
            for (int d = 0; d < 3; ++d) sx[d] += wi * pos[3 * i + d];
        }
        for (int d = 0; d < 3; ++d) c[d] = sx[d] / sw;
        // second moments M = sum w X X^T; T = tr(M) I - M is Eq. (17)
        double m[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
        for (int64_t j = lo; j < hi; ++j) {
            const int32_t i = order[j];
            const double wi = weight(i);
            const double X[3] = {pos[3 * i] - c[0], pos[3 * i + 1] - c[1], pos[3 * i + 2] - c[2]};
            for (int r = 0; r < 3; ++r)
                for (int s = r; s < 3; ++s) m[r][s] += wi * X[r] * X[s];
        }
        m[1][0] = m[0][1];
        m[2][0] = m[0][2];
        m[2][1] = m[1][2];
        const double tr = m[0][0] + m[1][1] + m[2][2];
        double T[3][3], V[3][3];
        for (int r = 0; r < 3; ++r)
            for (int s = 0; s < 3; ++s) T[r][s] = (r == s ? tr : 0.0) - m[r][s];
        jacobi3(T, V);
        // F at a unit eigenvector a equals a^T M a
        int best = 0;
        double fbest = -1.0;
        for (int k = 0; k < 3; ++k) {
            double f = 0.0;
            for (int r = 0; r < 3; ++r)
                for (int s = 0; s < 3; ++s) f += V[r][k] * m[r][s] * V[s][k];
            if (f > fbest) {
                fbest = f;
                best = k;
            }
        }
        double nrm = 0.0;
        int big = 0;
        for (int d = 0; d < 3; ++d) {
            ax[d] = V[d][best];
            nrm += ax[d] * ax[d];
            if (std::fabs(ax[d]) > std::fabs(ax[big])) big = d;
        }
        nrm = std::sqrt(nrm);
        const double sgn = ax[big] < 0.0 ? -1.0 : 1.0;
        for (int d = 0; d < 3; ++d) ax[d] = sgn * ax[d] / nrm;
    }

    void node(int64_t lo, int64_t hi, int32_t n, int32_t p0)
    {
        if (n == 1 || hi == lo) {
            // a leaf: parts p0 .. p0+n-1, all atoms of the range in part p0
            part_start[p0] = int32_t(lo);
            for (int32_t p = p0 + 1; p < p0 + n; ++p) part_start[p] = int32_t(hi);
            return;
        }
        double c[3], ax[3];
        axis(lo, hi, c, ax);
        const int64_t m = hi - lo;
        keys.resize(size_t(m));
        for (int64_t j = 0; j < m; ++j) {
            const int32_t i = order[lo + j];
            keys[size_t(j)] = {ax[0] * (pos[3 * i] - c[0]) + ax[1] * (pos[3 * i + 1] - c[1]) +
                                   ax[2] * (pos[3 * i + 2] - c[2]),
                               i};
        }
        std::sort(keys.begin(), keys.end());
        cum.resize(size_t(m) + 1);
        cum[0] = 0.0;
        for (int64_t j = 0; j < m; ++j) {
            order[lo + j] = keys[size_t(j)].second;
            cum[size_t(j) + 1] = cum[size_t(j)] + weight(keys[size_t(j)].second);
        }
        const int32_t nl = (n + 1) / 2;
        const double target = cum[size_t(m)] * double(nl) / double(n);
        // first k with cum[k] >= target, then the nearer of k-1 and k
        int64_t k = std::lower_bound(cum.begin(), cum.end(), target) - cum.begin();
        if (k > m) k = m;
        if (k > 0 && target - cum[size_t(k - 1)] < cum[size_t(k)] - target) --k;
        node(lo, lo + k, nl, p0);
        node(lo + k, hi, n - nl, p0 + nl);
    }
};

}  // namespace

const char *bisect_atoms(int32_t natoms, const double *pos, const double *weights, int32_t nparts, int32_t *order,
                         int32_t *part, int32_t *part_start)
{
    if (natoms < 0) return "natoms must be >= 0";
    if (nparts < 1) return "nparts must be >= 1";
    if (!order) return "order must not be NULL";
    if (natoms > 0 && !pos) return "pos must not be NULL";
    for (int64_t i = 0; i < 3 * int64_t(natoms); ++i)
        if (!std::isfinite(pos[i])) return "a position is not finite";
    if (weights)
        for (int32_t i = 0; i < natoms; ++i)
            if (!(weights[i] > 0.0) || !std::isfinite(weights[i])) return "weights must be finite and > 0";
    std::vector<int32_t> starts(size_t(nparts) + 1);
    Bisector b{pos, weights, order, starts.data(), {}, {}};
    for (int32_t i = 0; i < natoms; ++i) order[i] = i;
    b.node(0, natoms, nparts, 0);
    starts[size_t(nparts)] = natoms;
    if (part)
        for (int32_t p = 0; p < nparts; ++p)
            for (int32_t j = starts[size_t(p)]; j < starts[size_t(p) + 1]; ++j) part[order[j]] = p;
    if (part_start) std::copy(starts.begin(), starts.end(), part_start);
    return nullptr;
}

}  // namespace hartree
