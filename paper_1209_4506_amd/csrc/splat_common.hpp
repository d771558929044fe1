// Device helpers shared by the splat kernels (binning, VALU and MFMA forms).
#pragma once

#include "fft_core.hpp"
#include "kernels.hpp"

namespace hartree {

constexpr int kChunk = 32;  // atoms staged in LDS at a time

__device__ __forceinline__ int find_prob_atom(const SplatArgs &a, int atom)
{
    int p = 0;
    while (p + 1 < a.nprob && atom >= a.atom_off[p + 1]) ++p;
    return p;
}

__device__ __forceinline__ int wrapi(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

// bricks touched along one axis: circular range [start, start + count) mod nb
__device__ __forceinline__ void axis_bricks(int lo, int hi, int n, int bsz, int nb, int &start, int &count)
{
    if (hi < lo) {  // invalid atom: touches nothing
        start = 0;
        count = 0;
        return;
    }
    if (hi - lo + 1 >= n) {
        start = 0;
        count = nb;
        return;
    }
    const int s = wrapi(lo, n), e = wrapi(hi, n);
    const int bs = s / bsz, be = e / bsz;
    start = bs;
    if (s <= e)
        count = be - bs + 1;
    else
        count = (be >= bs) ? nb : (nb - bs) + be + 1;
}

__device__ __forceinline__ int brick_prob(const SplatArgs &a, int64_t b)
{
    int p = 0;
    while (p + 1 < a.nprob && b >= a.desc[p + 1].brick_off) ++p;
    return p;
}

template <typename T>
__device__ __forceinline__ T expT(T x);
template <>
__device__ __forceinline__ float expT<float>(float x) { return expf(x); }
template <>
__device__ __forceinline__ double expT<double>(double x) { return exp(x); }

// Per-atom 1-D factor tables, built once per binding by k_atom_tables: for
// atom a and axis x, row (a, x) holds (g, gd), the 1-D Gaussian factor and
// its displacement-weighted sum, at every grid index of the bricks the atom's
// window touches along x, brick by brick in touch order: entry
// u * bsz + q belongs to brick (st + u) mod nbricks, point q of it (zero past
// the end of the axis or outside the window).  A brick reads its bsz
// consecutive entries without index arithmetic per point.

// One atom of a group staged in LDS: its table row and touched brick ranges.
struct StagedAtom {
    int idx;           // atom index (table row)
    int st[3], ct[3];  // first touched brick and number of touched bricks per axis
    double w;          // Z (2 pi s^2)^(-3/2)
};

__device__ __forceinline__ void atom_bricks(const AtomInfo &in, const ProbDesc &d, int *st, int *ct)
{
    for (int x = 0; x < 3; ++x) axis_bricks(in.lo[x], in.hi[x], d.dims[x], d.bsz[x], d.nbricks[x], st[x], ct[x]);
}

// threads t < nc stage atoms list[c0 + t]
__device__ __forceinline__ void stage_atoms(StagedAtom *dst, const SplatArgs &a, const ProbDesc &d, int64_t off,
                                            int c0, int nc, int t)
{
    if (t < nc) {
        const int atom = a.list_sorted[off + c0 + t];
        const AtomInfo in = a.info[atom];
        StagedAtom s;
        s.idx = atom;
        atom_bricks(in, d, s.st, s.ct);
        s.w = in.w;
        dst[t] = s;
    }
}

// (g, gd) of a staged atom at point q of brick bidx along axis x, for an axis
// of nbx bricks of bsz points (passed by value: kernels keep them in
// registers rather than re-reading the problem descriptor).  The load is
// unconditional (from the row start when the entry lies outside the window)
// so that a thread's successive lookups need not wait for each other.
template <typename T>
__device__ __forceinline__ Cx<T> table_factor(const SplatArgs &a, int nbx, int bsz, int bidx, int q,
                                              const StagedAtom &at, int x, bool use = true)
{
    // select by value: indexing st[] / ct[] with a run-time axis would
    // put a copy of the struct in scratch memory
    const int m0 = -int(x == 0), m1 = -int(x == 1), m2 = -int(x == 2);
    const int st = (at.st[0] & m0) | (at.st[1] & m1) | (at.st[2] & m2);
    const int ct = (at.ct[0] & m0) | (at.ct[1] & m1) | (at.ct[2] & m2);
    int u = bidx - st;
    if (u < 0) u += nbx;
    const int e = u * bsz + q;
    const bool ok = use && u < ct && e < a.wcap;
    const Cx<T> *tab = reinterpret_cast<const Cx<T> *>(a.tab);
    const Cx<T> v = tab[(int64_t(at.idx) * 3 + x) * a.wcap + (ok ? e : 0)];
    return ok ? v : Cx<T>{T(0), T(0)};
}

}  // namespace hartree
