// Gaussian atomic density on the grid (splat) and its adjoint (forces).
//
// The density of each atom is a product of three 1-D periodic Gaussians in
// an orthorhombic cell, so every contribution factorizes into per-axis
// factors.  The grid is cut into bricks of 16 x 16 x 32 points (8 x 8 x 32 in
// FP64 plans with a non-diagonal cell; the analogue of the paper's
// structure A / structure C idea, Sec. 3.2.2: the points touched by one
// atom's sphere, and a box around a group of atoms); each brick is one
// workgroup that gathers the atoms whose truncation window overlaps it.
//
// Binning is deterministic: every atom adds itself to the bricks its window
// touches (integer atomics), the per-brick lists are then sorted by atom
// index, and every sum below runs in a fixed order, so results do not depend
// on scheduling.
//
//   count   per atom: wrapped position, weight, window [lo, hi] per axis;
//           +1 on each touched brick
//   scan    per problem: Q = sum Z (fixed order), for the background
//           Q / Omega; exclusive prefix sum of the brick counts
//   fill    per atom: write its index into each touched brick's list
//   sort    per brick: order the list by atom index; clear the brick's
//           counters for the next binning
//   gather  per brick: rho = sum over its atoms of w gx(i) gy(j) gz(k) [- Q/Omega]
//   adjoint per brick: partial sum_r grad_rho(r) g(r) d(r) for each of its atoms
//   final   per atom: fixed-order sum of its partials over the touched bricks
#include <algorithm>

#include "splat_common.hpp"

namespace hartree {

// An atom's wrapped position, weight and window per axis; `report` sets
// the device status bits for an invalid atom (which then touches nothing).
__device__ __forceinline__ AtomInfo atom_prep(const SplatArgs &a, int atom, bool report)
{
    const int prob = find_prob_atom(a, atom);
    const ProbDesc &d = a.desc[prob];
    AtomInfo in;
    in.prob = prob;
    in.pad = 0;
    const double s = a.sigma[atom], z = a.Z[atom];
    bool ok = isfinite(s) && s > 0.0 && isfinite(z);
    for (int x = 0; x < 3; ++x) ok = ok && isfinite(a.pos[3 * atom + x]);
    if (ok && s > a.max_sigma) {
        if (report) atomicOr(&a.status->bits, 0x2u);
        ok = false;
    } else if (!ok) {
        if (report) atomicOr(&a.status->bits, 0x1u);
    }
    if (!ok) {
        for (int x = 0; x < 3; ++x) {
            in.X[x] = 0.0;
            in.lo[x] = 1;
            in.hi[x] = 0;
            in.st[x] = 0;
            in.ct[x] = 0;
        }
        in.w = 0.0;
        in.inv2s2 = 0.0;
        return in;
    }
    const double rc = a.cutoff * s;
    if (d.separable) {
        for (int x = 0; x < 3; ++x) {
            const double L = d.L[x];
            double X = a.pos[3 * atom + x];
            X -= floor(X / L) * L;
            if (X >= L) X -= L;
            if (X < 0.0) X = 0.0;
            const double h = d.h[x];
            in.X[x] = X;
            in.lo[x] = int(ceil((X - rc) / h));
            in.hi[x] = int(floor((X + rc) / h));
        }
    } else {
        // any cell: fractional coordinate f_x = R . b_x / (2 pi), wrapped
        // into [0, 1); the cutoff sphere spans f_x +- rc |b_x| / (2 pi)
        const double inv2pi = 0.15915494309189533576888376337251;
        double f[3];
        for (int x = 0; x < 3; ++x) {
            const double *bx = d.B + 3 * x;
            double fx = (a.pos[3 * atom] * bx[0] + a.pos[3 * atom + 1] * bx[1] + a.pos[3 * atom + 2] * bx[2]) * inv2pi;
            fx -= floor(fx);
            if (fx >= 1.0) fx -= 1.0;
            if (fx < 0.0) fx = 0.0;
            f[x] = fx;
            const double e = rc * sqrt(bx[0] * bx[0] + bx[1] * bx[1] + bx[2] * bx[2]) * inv2pi;
            in.lo[x] = int(ceil((fx - e) * d.dims[x]));
            in.hi[x] = int(floor((fx + e) * d.dims[x]));
        }
        for (int c = 0; c < 3; ++c) in.X[c] = f[0] * d.A[c] + f[1] * d.A[3 + c] + f[2] * d.A[6 + c];
    }
    const double s2 = 6.283185307179586476925286766559 * s * s;  // (2 pi s^2)^(-3/2) without pow
    in.w = z / (s2 * sqrt(s2));
    in.inv2s2 = 1.0 / (2.0 * s * s);
    atom_bricks(in, d, in.st, in.ct);
    return in;
}

// Bricks touched by one atom, enumerated t = 0 .. ntouch-1 in a fixed order:
// t = (u * ct[1] + v) * ct[2] + w over the circular ranges of the three axes.
struct Touch {
    int st[3], ct[3];
    __device__ int ntouch() const { return ct[0] * ct[1] * ct[2]; }
};

// (the ranges are formed once per atom by the count pass, in atom_prep)
__device__ __forceinline__ Touch atom_touch(const AtomInfo &in, const ProbDesc &)
{
    Touch t;
    for (int x = 0; x < 3; ++x) {
        t.st[x] = in.st[x];
        t.ct[x] = in.ct[x];
    }
    return t;
}

__device__ __forceinline__ int64_t touch_brick(const Touch &t, const ProbDesc &d, int i)
{
    const int w = i % t.ct[2];
    const int uv = i / t.ct[2];
    const int v = uv % t.ct[1], u = uv / t.ct[1];
    const int bi = (t.st[0] + u) % d.nbricks[0];
    const int bj = (t.st[1] + v) % d.nbricks[1];
    const int bk = (t.st[2] + w) % d.nbricks[2];
    return d.brick_off + (int64_t(bi) * d.nbricks[1] + bj) * d.nbricks[2] + bk;
}

// index t of the brick at per-axis position bc in the atom's enumeration
__device__ __forceinline__ int touch_index(const Touch &t, const ProbDesc &d, const int bc[3])
{
    const int u = (bc[0] - t.st[0] + d.nbricks[0]) % d.nbricks[0];
    const int v = (bc[1] - t.st[1] + d.nbricks[1]) % d.nbricks[1];
    const int w = (bc[2] - t.st[2] + d.nbricks[2]) % d.nbricks[2];
    return (u * t.ct[1] + v) * t.ct[2] + w;
}

// one wavefront per atom, lanes over the bricks it touches.  Wavefront w
// takes atom (w * visit_stride) mod natoms (a stride coprime to natoms), so
// that atoms adjacent in the input, which touch the same bricks, do not
// contend for the same counters at the same time.  The count pass also
// prepares the atom (every lane computes it, lane 0 stores it).
template <int MODE>  // 0: count, 1: fill
__global__ __launch_bounds__(256) void k_brick_visit(SplatArgs a)
{
    // the wavefront's index is uniform: kept in scalar registers, so that
    // the atom's and its problem's data come through scalar loads
    const int w = __builtin_amdgcn_readfirstlane(int(blockIdx.x * 4 + (threadIdx.x >> 6)));
    const int lane = threadIdx.x & 63;
    if (w >= a.natoms) return;
    const int atom = int((int64_t(w) * a.visit_stride) % a.natoms);
    AtomInfo in;
    if (MODE == 0) {
        in = atom_prep(a, atom, lane == 0);
        if (lane == 0) a.info[atom] = in;
    } else {
        in = a.info[atom];
    }
    const ProbDesc &d = a.desc[in.prob];
    const Touch t = atom_touch(in, d);
    const int nt = t.ntouch();
    for (int i = lane; i < nt; i += 64) {
        const int64_t b = touch_brick(t, d, i);
        if (MODE == 0) {
            atomicAdd(&a.counts[b], 1);
        } else {
            const int slot = atomicAdd(&a.cursor[b], 1);
            const int64_t idx = int64_t(a.offsets[b]) + slot;
            if (idx < a.capacity) a.list[idx] = atom;
        }
    }
}

// exclusive scan of counts[0..n) into offsets[0..n] by one workgroup, in
// chunks of kScanThreads * kScanPer entries: thread t loads the kScanPer
// consecutive counts at t * kScanPer of the chunk (four 16-byte loads), the
// workgroup scans the per-thread sums, and each thread writes its run
// (clamped to the capacity).  The same workgroup first sums each problem's
// charges Q = sum Z in a fixed order (for the background Q / Omega) and
// takes the largest weight |Z| (2 pi sigma^2)^(-3/2) of its valid atoms (the
// FP32 splat scales its 16-bit operands by it).
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 16;
// Work order of the bricks for the matrix-core kernels of batched plans
// (a.order, written by the same workgroup after the scan): a counting sort
// by descending number of 16-atom groups, so that the longest bricks start
// first and the short ones fill the tail.  The order within a group count is
// whatever the LDS atomics give: each brick writes only its own outputs, so
// results do not depend on it.
constexpr int kOrderKeys = 32;

// the weight |Z| (2 pi sigma^2)^(-3/2) of a valid atom in float (a bound
// for scaling: clamped to the float range), 0 for an invalid one
__device__ __forceinline__ float weight_bound(double z, double s, double max_sigma)
{
    const bool ok = isfinite(z) && s > 0.0 && s <= max_sigma;
    const float s2 = 6.2831855f * float(s) * float(s);
    const float wv = fabsf(float(z)) / (s2 * sqrtf(s2));
    return ok ? (wv < 3.0e38f ? wv : 3.0e38f) : 0.0f;
}

// Q += Z and wm = max(wm, weight) over the atoms i0, i0 + step, ... below
// i1, in that order; four atoms' loads are issued before their sums
__device__ __forceinline__ void charge_and_weight(const SplatArgs &a, int i0, int i1, int step, double &q, float &wm)
{
    int i = i0;
    for (; i + 3 * step < i1; i += 4 * step) {
        double z[4], sg[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            z[k] = a.Z[i + k * step];
            sg[k] = a.sigma[i + k * step];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            q += z[k];
            wm = fmaxf(wm, weight_bound(z[k], sg[k], a.max_sigma));
        }
    }
    for (; i < i1; i += step) {
        q += a.Z[i];
        wm = fmaxf(wm, weight_bound(a.Z[i], a.sigma[i], a.max_sigma));
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan(SplatArgs a)
{
    constexpr int NW = kScanThreads / 64;
    __shared__ int64_t wtot[NW];
    __shared__ double qw[NW];
    __shared__ float ww[NW];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t n = a.nbricks_total;
    constexpr int64_t CH = int64_t(kScanThreads) * kScanPer;
    // this thread's kScanPer consecutive counts from e0 (zeros past n)
    auto load_counts = [&](int64_t e0, int *v) {
        if (e0 + kScanPer <= n) {
            // the counts array is 256-byte aligned and e0 a multiple of 16
            const int4 *src = reinterpret_cast<const int4 *>(a.counts + e0);
#pragma unroll
            for (int k = 0; k < kScanPer / 4; ++k) {
                const int4 x = src[k];
                v[4 * k] = x.x;
                v[4 * k + 1] = x.y;
                v[4 * k + 2] = x.z;
                v[4 * k + 3] = x.w;
            }
        } else {
#pragma unroll
            for (int k = 0; k < kScanPer; ++k) v[k] = e0 + k < n ? a.counts[e0 + k] : 0;
        }
    };
    // the first chunk is loaded before the charge sums, so that its latency
    // overlaps them
    int v[kScanPer];
    load_counts(int64_t(t) * kScanPer, v);
    if (a.nprob <= 4) {
        // few problems: the whole workgroup sums each problem's charges,
        // thread t the atoms t, t + kScanThreads, ..., then fixed butterflies
        for (int p = 0; p < a.nprob; ++p) {
            double q = 0.0;
            float wm = 0.0f;
            charge_and_weight(a, a.atom_off[p] + t, a.atom_off[p + 1], kScanThreads, q, wm);
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                q += __shfl_xor(q, off, 64);
                wm = fmaxf(wm, __shfl_xor(wm, off, 64));
            }
            if (lane == 0) {
                qw[w] = q;
                ww[w] = wm;
            }
            __syncthreads();
            if (t == 0) {
                double tot = 0.0;
                float wmax = 0.0f;
                for (int k = 0; k < NW; ++k) {
                    tot += qw[k];
                    wmax = fmaxf(wmax, ww[k]);
                }
                a.qsum[p] = tot;
                a.qsum[a.nprob + p] = wmax;
            }
            __syncthreads();
        }
    } else {
        // many problems: wavefront w sums the charges of problems w, w + NW,
        // ...: lane l the atoms l, l + 64, ... of the problem, then a fixed
        // butterfly (no workgroup barrier per problem)
        for (int p = w; p < a.nprob; p += NW) {
            double q = 0.0;
            float wm = 0.0f;
            charge_and_weight(a, a.atom_off[p] + lane, a.atom_off[p + 1], 64, q, wm);
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                q += __shfl_xor(q, off, 64);
                wm = fmaxf(wm, __shfl_xor(wm, off, 64));
            }
            if (lane == 0) {
                a.qsum[p] = q;
                a.qsum[a.nprob + p] = wm;
            }
        }
    }
    int64_t carry = 0;  // total of the chunks before this one (the same in every thread)
    for (int64_t c0 = 0; c0 < n; c0 += CH) {
        const int64_t e0 = c0 + int64_t(t) * kScanPer;
        if (c0 > 0) load_counts(e0, v);
        int64_t s = 0;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) s += v[k];
        // inclusive scan of the thread sums within the wavefront, then across them
        int64_t x = s;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int64_t y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane == 63) wtot[w] = x;
        __syncthreads();
        int64_t before = 0, chunk = 0;
        for (int k = 0; k < NW; ++k) {
            if (k < w) before += wtot[k];
            chunk += wtot[k];
        }
        int64_t run = carry + before + x - s;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            if (e0 + k < n) a.offsets[e0 + k] = int32_t(run < a.capacity ? run : a.capacity);
            run += v[k];
        }
        carry += chunk;
        __syncthreads();  // wtot is rewritten by the next chunk
    }
    if (t == 0) {
        a.offsets[n] = int32_t(carry < a.capacity ? carry : a.capacity);
        if (carry > a.capacity) atomicOr(&a.status->bits, 0x4u);
    }
    if (a.order) {
        // bricks in strided order (thread t takes bricks t, t + kScanThreads,
        // ...), so that bricks next to each other in space stay next to each
        // other within a group count (the counts are read again, from cache:
        // the thread's registers hold a contiguous run instead)
        __shared__ int hist[kOrderKeys], next[kOrderKeys];
        auto key = [&](int64_t b) {
            const int k = (a.counts[b] + 15) >> 4;
            return k < kOrderKeys - 1 ? k : kOrderKeys - 1;
        };
        if (t < kOrderKeys) hist[t] = 0;
        __syncthreads();
        for (int64_t b = t; b < n; b += kScanThreads) atomicAdd(&hist[key(b)], 1);
        __syncthreads();
        if (t == 0) {
            int run = 0;
            for (int k = kOrderKeys - 1; k >= 0; --k) {
                next[k] = run;
                run += hist[k];
            }
        }
        __syncthreads();
        for (int64_t b = t; b < n; b += kScanThreads) a.order[atomicAdd(&next[key(b)], 1)] = int32_t(b);
    }
}

// one wavefront per brick: order the list by atom index, and record each
// entry's final slot under (atom, brick) for the adjoint's reduction.  A
// brick's atoms all belong to its problem, whose indices span
// [atom_off[p], atom_off[p + 1]).  The entries are distinct atom indices,
// and an entry's rank is the number of smaller ones: for lists of up to 64
// entries (the usual case) counted over the lanes' registers; for longer
// lists, when every problem's span fits rank_words 32-bit words
// (rank_words > 0), from an LDS bitmap of the span (each entry sets its bit;
// its rank is the number of set bits below it: prefix sums of the words'
// bit counts plus one popcount, O(cnt + span / 32) per brick); otherwise
// counted over the list in LDS (up to kSortLds entries) or in memory.
constexpr int kSortLds = 256;
constexpr int kRankWords = 1024;  // bitmap ranks for spans of up to 32,768 atoms

__global__ __launch_bounds__(256) void k_brick_sort(SplatArgs a, int rank_words)
{
    __shared__ int lst[4][kSortLds];
    extern __shared__ uint32_t rank_lds[];  // rank_words > 0: [4 waves][bitmap, word prefix][rank_words]
    const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    const int64_t b = int64_t(blockIdx.x) * 4 + w;  // uniform: scalar loads of its offsets and problem
    int64_t off = 0;
    int cnt = 0;
    if (b < a.nbricks_total) {
        off = a.offsets[b];
        cnt = int(a.offsets[b + 1] - off);
        // the next binning starts from zero counters (their last readers,
        // the scan and the fill, have finished)
        if (lane == 0) {
            a.counts[b] = 0;
            a.cursor[b] = 0;
        }
    }
    // the first 128 entries are loaded once, two per lane, and the first
    // entry's atom is fetched before the ranking so that its latency
    // overlaps the barriers
    const int v0 = lane < cnt ? a.list[off + lane] : 0;
    const int v1 = lane + 64 < cnt ? a.list[off + 64 + lane] : 0;
    AtomInfo in0;
    if (lane < cnt) in0 = a.info[v0];
    const int prob = cnt > 0 ? brick_prob_wave(a, b) : 0;
    const int a0 = a.atom_off[prob];
    const int span = a.atom_off[prob + 1] - a0;
    // ranks from the bitmap cost about span / 32 word operations per
    // wavefront plus a scan; counting smaller entries costs cnt per lane:
    // short lists over wide spans (many atoms per problem, few per brick)
    // are ranked by counting
    const int nw = (span + 31) >> 5;
    const bool small = cnt <= 64;
    const bool bitmap = !small && rank_words > 0 && !(cnt <= kSortLds && cnt <= nw / 32 + 16);
    uint32_t *bm = rank_lds + w * 2 * rank_words, *pre = bm + rank_words;
    const bool in_lds = !small && !bitmap && cnt <= kSortLds;
    auto entry = [&](int e) { return e < 64 ? v0 : (e < 128 ? v1 : a.list[off + e]); };
    // the barriers are reached by every wavefront whatever its brick's method
    if (bitmap)
        for (int i = lane; i < nw; i += 64) bm[i] = 0u;
    __syncthreads();
    if (bitmap) {
        for (int e = lane; e < cnt; e += 64) {
            const int r = entry(e) - a0;
            if (unsigned(r) < unsigned(span)) atomicOr(&bm[r >> 5], 1u << (r & 31));
        }
    } else if (in_lds) {
        for (int e = lane; e < cnt; e += 64) lst[w][e] = entry(e);
    }
    __syncthreads();
    if (bitmap) {
        // exclusive prefix of the words' bit counts: lane l takes a run of
        // consecutive words, a wavefront scan orders the runs
        const int wpl = (nw + 63) >> 6;
        const int w0 = lane * wpl < nw ? lane * wpl : nw, w1 = w0 + wpl < nw ? w0 + wpl : nw;
        int c = 0;
        for (int i = w0; i < w1; ++i) c += __popc(bm[i]);
        int x = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        int run = x - c;
        for (int i = w0; i < w1; ++i) {
            pre[i] = uint32_t(run);
            run += __popc(bm[i]);
        }
    }
    __syncthreads();
    if (cnt == 0) return;
    const ProbDesc &d = a.desc[prob];
    // the brick's position per axis (the bricks of one problem fit 32 bits)
    const int lb = int(b - d.brick_off);
    const int bc[3] = {lb / (d.nbricks[2] * d.nbricks[1]), (lb / d.nbricks[2]) % d.nbricks[1], lb % d.nbricks[2]};
    // the rank of entry v (-1: not an atom of this problem, never written)
    auto rank_of = [&](int v) {
        int rank = 0;
        if (small) {
            for (int j = 0; j < cnt; ++j) rank += __builtin_amdgcn_readlane(v0, j) < v ? 1 : 0;
        } else if (bitmap) {
            const int r = v - a0;
            if (unsigned(r) >= unsigned(span)) return -1;
            rank = int(pre[r >> 5]) + __popc(bm[r >> 5] & ((1u << (r & 31)) - 1u));
        } else if (in_lds) {
            for (int j = 0; j < cnt; ++j) rank += (lst[w][j] < v) ? 1 : 0;
        } else {
            for (int j = 0; j < cnt; ++j) rank += (a.list[off + j] < v) ? 1 : 0;
        }
        return rank;
    };
    auto emit = [&](int v, int rank, const AtomInfo &in) {
        a.list_sorted[off + rank] = v;
        const Touch t = atom_touch(in, d);
        const int ti = touch_index(t, d, bc);
        // with records, the adjoint writes its partials under (atom, touch)
        // directly; otherwise the slot map leads the reduction to them
        if (!a.rec && !a.rec64) a.slot_of[int64_t(v) * a.cap_pa + ti] = int32_t(off + rank);
        if (a.rec64) {
            // the atom relative to this brick, for the FP64 splat kernels
            SlotAtom64 r;
            for (int x = 0; x < 3; ++x) {
                r.X[x] = in.X[x];
                r.lo[x] = in.lo[x];
                r.r0[x] = wrapi(bc[x] * d.bsz[x] - in.lo[x], d.dims[x]);
                r.wl[x] = in.hi[x] >= in.lo[x] ? in.hi[x] - in.lo[x] + 1 : 0;
            }
            r.inv2s2 = in.inv2s2;
            r.w = in.w;
            r.atom = v;
            r.touch = ti;
            r.pad = 0;
            a.rec64[off + rank] = r;
        }
        if (a.rec) {
            // the atom relative to this brick, for the FP32 splat kernels
            SlotAtom r;
            for (int x = 0; x < 3; ++x) {
                const int n = d.dims[x];
                const double h = d.h[x];
                const double xb = in.X[x] - in.lo[x] * h;
                r.ax[x].xb = float(xb);
                r.ax[x].xbl = float(xb - double(r.ax[x].xb));
                r.ax[x].r0 = wrapi(bc[x] * d.bsz[x] - in.lo[x], n);
                r.ax[x].wl = in.hi[x] >= in.lo[x] ? in.hi[x] - in.lo[x] + 1 : 0;
            }
            r.c2 = float(1.4426950408889634073599246810019 * in.inv2s2);
            r.w = float(in.w);
            r.atom = v;
            r.touch = ti;
            a.rec[off + rank] = r;
        }
    };
    // the first entry of each lane with the atom fetched above, the rest
    // (lists longer than 64) with their own loads
    if (lane < cnt) {
        const int rank = rank_of(v0);
        if (rank >= 0) emit(v0, rank, in0);
    }
    for (int e = lane + 64; e < cnt; e += 64) {
        const int v = entry(e);
        const int rank = rank_of(v);
        if (rank >= 0) emit(v, rank, a.info[v]);
    }
}

// one wavefront per atom: lanes sum its per-brick partials (slots from the
// sort) in a fixed order, then a fixed butterfly combines the lanes
__global__ __launch_bounds__(256) void k_adjoint_final(SplatArgs a)
{
    const int atom = __builtin_amdgcn_readfirstlane(int(blockIdx.x * 4 + (threadIdx.x >> 6)));
    const int lane = threadIdx.x & 63;
    if (atom >= a.natoms) return;
    const AtomInfo in = a.info[atom];
    const ProbDesc &d = a.desc[in.prob];
    const Touch t = atom_touch(in, d);
    const int nt = t.ntouch();
    double f0 = 0.0, f1 = 0.0, f2 = 0.0;
    if (a.rec || a.rec64) {
        // partials stored per (atom, touched brick): one contiguous row
        const double *row = a.bpart + int64_t(atom) * a.cap_pa * 3;
        for (int i = lane; i < nt; i += 64) {
            f0 += row[i * 3 + 0];
            f1 += row[i * 3 + 1];
            f2 += row[i * 3 + 2];
        }
    } else {
        const int32_t *slots = a.slot_of + int64_t(atom) * a.cap_pa;
        for (int i = lane; i < nt; i += 64) {
            const int64_t s = slots[i];
            if (s >= 0 && s < a.capacity) {
                f0 += a.bpart[s * 3 + 0];
                f1 += a.bpart[s * 3 + 1];
                f2 += a.bpart[s * 3 + 2];
            }
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        f0 += __shfl_xor(f0, off, 64);
        f1 += __shfl_xor(f1, off, 64);
        f2 += __shfl_xor(f2, off, 64);
    }
    if (lane == 0) {
        const double scale = in.w * 2.0 * in.inv2s2;  // Z (2 pi s^2)^(-3/2) / s^2
        a.grad_pos[3 * atom + 0] = scale * f0;
        a.grad_pos[3 * atom + 1] = scale * f1;
        a.grad_pos[3 * atom + 2] = scale * f2;
    }
}

// ------------------------------------------------------------- host side

// The brick counters and cursors are zero on entry: the workspace binding
// clears them and every binning's sort pass leaves them cleared.
hipError_t run_bin(const SplatArgs &a, hipStream_t s)
{
    const int64_t nbt = a.nbricks_total;
    const int nw = int((a.natoms + 3) / 4);  // one wavefront per atom
    // the count pass prepares the atoms (AtomInfo): it runs first
    if (a.natoms > 0) hipLaunchKernelGGL(k_brick_visit<0>, dim3(nw), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, s, a);
    if (a.natoms > 0) hipLaunchKernelGGL(k_brick_visit<1>, dim3(nw), dim3(256), 0, s, a);
    int span = 0;
    for (int p = 0; p < a.nprob; ++p) span = std::max(span, a.atom_off[p + 1] - a.atom_off[p]);
    const int words = (span + 31) / 32;
    const int rank_words = words <= kRankWords ? words : 0;
    hipLaunchKernelGGL(k_brick_sort, dim3(int((nbt + 3) / 4)), dim3(256), size_t(rank_words) * 4 * 2 * 4, s, a,
                       rank_words);
    return hipGetLastError();
}

// diagonal cells run on the matrix cores (splat_mfma.hip: FP32,
// splat_mfma64.hip: FP64); any other cell evaluates the Gaussians point by
// point (splat_general.hip)
hipError_t run_gather(const SplatArgs &a, hipStream_t s)
{
    if (a.general) return run_gather_general(a, s);
    return a.fp64 ? run_gather_mfma64(a, s) : run_gather_mfma(a, s);
}

hipError_t run_adjoint(const SplatArgs &a, hipStream_t s)
{
    if (a.general) return run_adjoint_general(a, s);
    return a.fp64 ? run_adjoint_mfma64(a, s) : run_adjoint_mfma(a, s);
}

hipError_t run_adjoint_final(const SplatArgs &a, hipStream_t s)
{
    if (a.natoms > 0) hipLaunchKernelGGL(k_adjoint_final, dim3(int((a.natoms + 3) / 4)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace hartree
