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

// 1-D periodic Gaussian factor along one axis at wrapped index ig:
// g = sum over unwrapped i' = ig (mod n) in [lo, hi] of exp(-(i' h - X)^2 / (2 s^2)),
// gd = the same sum weighted by the displacement (i' h - X).  The exponent is
// formed in double (positions near L lose digits in float) and evaluated in T.
template <typename T, bool WITH_D>
__device__ __forceinline__ void axis_factor_t(int ig, int n, double h, double X, int lo, int hi, double inv2s2, T &g,
                                              T &gd)
{
    g = T(0);
    gd = T(0);
    if (hi < lo || ig >= n) return;
    for (int ip = lo + wrapi(ig - lo, n); ip <= hi; ip += n) {
        const double dd = double(ip) * h - X;
        const T e = expT<T>(T(-dd * dd * inv2s2));
        g += e;
        if (WITH_D) gd += e * T(dd);
    }
}

// Per-atom 1-D factor tables, built once per call by k_atom_tables: for atom
// a and axis x, entry t of row (a, x) holds (g, gd), the 1-D Gaussian factor
// and its displacement-weighted sum,
//   window narrower than the axis (wl < n): the single image at unwrapped
//       index ip = lo + t, t < wl = hi - lo + 1;
//   window as wide as the axis: every image at wrapped index t < n.
// A brick reads the entries of its own index range from these rows.

// One atom of a group staged in LDS: its table row and window.
struct StagedAtom {
    int idx;                 // atom index (table row)
    int lo[3], low[3], wl[3];  // window start, start mod n, width (0: none)
    double w;                // Z (2 pi s^2)^(-3/2)
};

// threads t < nc stage atoms list[c0 + t]
__device__ __forceinline__ void stage_atoms(StagedAtom *dst, const SplatArgs &a, const ProbDesc &d, int64_t off,
                                            int c0, int nc, int t)
{
    if (t < nc) {
        const int atom = a.list_sorted[off + c0 + t];
        const AtomInfo in = a.info[atom];
        StagedAtom s;
        s.idx = atom;
        for (int x = 0; x < 3; ++x) {
            s.lo[x] = in.lo[x];
            s.low[x] = wrapi(in.lo[x], d.dims[x]);
            s.wl[x] = in.hi[x] >= in.lo[x] ? in.hi[x] - in.lo[x] + 1 : 0;
        }
        s.w = in.w;
        dst[t] = s;
    }
}

// (g, gd) of a staged atom at wrapped grid index ig along axis x
template <typename T>
__device__ __forceinline__ Cx<T> table_factor(const SplatArgs &a, int ig, int n, const StagedAtom &at, int x)
{
    const int wl = at.wl[x];
    if (wl <= 0 || ig >= n) return Cx<T>{T(0), T(0)};
    int t = ig;
    if (wl < n) {
        t = ig - at.low[x];
        if (t < 0) t += n;
        if (t >= wl) return Cx<T>{T(0), T(0)};
    }
    if (t >= a.wcap) return Cx<T>{T(0), T(0)};  // never for sigma <= max_sigma
    const Cx<T> *tab = reinterpret_cast<const Cx<T> *>(a.tab);
    return tab[(int64_t(at.idx) * 3 + x) * a.wcap + t];
}

}  // namespace hartree
