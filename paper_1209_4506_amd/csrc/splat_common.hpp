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

// One atom of a chunk staged in LDS for the table computations: the window
// start is also kept reduced into [0, n) so that a table entry needs no
// integer division.
struct StagedAtom {
    double X[3];
    double inv2s2;
    double w;
    int lo[3], low[3], hi[3];
    int pad;
};

// threads t < nc stage atoms list[c0 + t]
__device__ __forceinline__ void stage_atoms(StagedAtom *dst, const SplatArgs &a, const ProbDesc &d, int64_t off,
                                            int c0, int nc, int t)
{
    if (t < nc) {
        const AtomInfo in = a.info[a.list_sorted[off + c0 + t]];
        StagedAtom s;
        for (int x = 0; x < 3; ++x) {
            s.X[x] = in.X[x];
            s.lo[x] = in.lo[x];
            s.hi[x] = in.hi[x];
            s.low[x] = wrapi(in.lo[x], d.dims[x]);
        }
        s.inv2s2 = in.inv2s2;
        s.w = in.w;
        s.pad = 0;
        dst[t] = s;
    }
}

// axis_factor_t for a staged atom: the first unwrapped index congruent to ig
// is lo + ((ig - low) mod n), with ig and low both in [0, n)
template <typename T, bool WITH_D>
__device__ __forceinline__ void staged_factor(int ig, int n, double h, const StagedAtom &at, int x, T &g, T &gd)
{
    g = T(0);
    gd = T(0);
    const int lo = at.lo[x], hi = at.hi[x];
    if (hi < lo || ig >= n) return;
    int delta = ig - at.low[x];
    if (delta < 0) delta += n;
    for (int ip = lo + delta; ip <= hi; ip += n) {
        const double dd = double(ip) * h - at.X[x];
        const T dt = T(dd);
        const T e = expT<T>(-dt * dt * T(at.inv2s2));
        g += e;
        if (WITH_D) gd += e * dt;
    }
}

}  // namespace hartree
