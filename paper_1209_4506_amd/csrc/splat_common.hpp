// Device helpers shared by the splat kernels (binning, VALU and MFMA forms).
#pragma once

#include "fft_core.hpp"
#include "kernels.hpp"

namespace hartree {

// The last p < n whose start(p) is at or below v, for starts that do not
// decrease with p and start(0) <= v: the number of q in [1, n) with
// start(q) <= v.  v is the same in every lane and every lane is active:
// lane l compares start(q) for q = 1 + l, 65 + l, ..., so the lookup costs
// one load per 64 problems instead of a chain of dependent loads.
template <class Start>
__device__ __forceinline__ int wave_find(int n, int64_t v, Start start)
{
    const int lane = threadIdx.x & 63;
    int p = 0;
    for (int q0 = 1; q0 < n; q0 += 64) {
        const int q = q0 + lane;
        const bool le = q < n && start(q) <= v;
        p += __popcll(__ballot(le));
    }
    return __builtin_amdgcn_readfirstlane(p);
}

// the problem of an atom (atom_off ascending); callers hold the atom index
// in every lane with the whole wavefront active
__device__ __forceinline__ int find_prob_atom(const SplatArgs &a, int atom)
{
    return wave_find(a.nprob, atom, [&](int q) { return int64_t(a.atom_off[q]); });
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

// bricks touched by an atom along each axis
__device__ __forceinline__ void atom_bricks(const AtomInfo &in, const ProbDesc &d, int *st, int *ct)
{
    for (int x = 0; x < 3; ++x) axis_bricks(in.lo[x], in.hi[x], d.dims[x], d.bsz[x], d.nbricks[x], st[x], ct[x]);
}

// the problem of a brick (brick_off ascending), by bisection over the
// problems: a chain of scalar loads, which the scalar cache serves to every
// wavefront of the long splat kernels
__device__ __forceinline__ int brick_prob(const SplatArgs &a, int64_t b)
{
    int lo = 0, hi = a.nprob - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (b >= a.desc[mid].brick_off) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// the same by one vector load and a ballot, for the short binning kernels
// whose wavefronts are load chains; callers hold the brick index in every
// lane with the whole wavefront active
__device__ __forceinline__ int brick_prob_wave(const SplatArgs &a, int64_t b)
{
    return wave_find(a.nprob, b, [&](int q) { return a.desc[q].brick_off; });
}

// brick index of this workgroup: from the binning's work order where there
// is one (batched plans: bricks by descending atom count), else with
// consecutive bricks (which share cache lines at their edges along c) kept
// on one XCD
__device__ __forceinline__ int64_t brick_of_block(const SplatArgs &a)
{
    if (a.order) return a.order[blockIdx.x];
    return xcd_remap(blockIdx.x, gridDim.x);
}

// A brick's position (brick index per axis), kept in registers
struct BrickPos {
    int b0, b1, b2;
};

__device__ __forceinline__ BrickPos brick_pos(const ProbDesc &d, int64_t b)
{
    const int lb = int(b - d.brick_off);  // bricks of one problem fit 32 bits
    BrickPos p;
    p.b2 = lb % d.nbricks[2];
    const int bij = lb / d.nbricks[2];
    p.b1 = bij % d.nbricks[1];
    p.b0 = bij / d.nbricks[1];
    return p;
}

template <typename T>
__device__ __forceinline__ T expT(T x);
template <>
__device__ __forceinline__ float expT<float>(float x) { return expf(x); }
template <>
__device__ __forceinline__ double expT<double>(double x) { return exp(x); }

}  // namespace hartree
