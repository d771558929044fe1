// FP64 splat and splat adjoint on the matrix cores (v_mfma_f64_16x16x4f64).
//
// The same bricks (16 x 16 columns (i, j) by 32 points along c) and the same
// two contractions per brick as the FP32 kernels:
//
//   splat    rho[c][k]  = sum_a  W_a gx_a(i_c) gy_a(j_c)  *  gz_a(k)
//   adjoint  S[c][a, f] = sum_k  grho[c][k]  *  gz_a(k) (f = 0) or gdz_a(k) (f = 1),
//            F_a = sum_c [gdx gy S0, gx gdy S0, gx gy S1]
//
// here with FP64 operands, FP64 factors (displacements and exponentials in
// double) and FP64 accumulation.  The matrix cores run FP64 at the vector
// units' rate; what they add is the operand reuse of a dense product.
//
// Operand layout of v_mfma_f64_16x16x4f64 (D = A B + C, A 16x4, B 4x16):
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; after the call
// lane l holds D[4 r + l / 16][l % 16] in its accumulator element r = 0..3
// (rows interleaved across the lane groups, unlike the FP32 layouts).
// A 16-row tile is one i with its 16 j (row = j); wavefront w owns
// i = 4w .. 4w + 3.  Which reduction index sits in which K slot is free as
// long as A and B agree: the splat puts atom 4 m + l / 16 of a step in slot
// l / 16 of its product m; the adjoint puts point k = 8 (l / 16) + ks in slot
// l / 16 of its product ks, so that each lane's grad_rho values are runs of
// 8 consecutive points of one column.
#include "splat_common.hpp"

namespace hartree {

typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int kDThreads = 256;  // four wavefronts per brick
constexpr int kDStage = 128;    // records staged at once (whole lists, almost always)
constexpr int kDSub = 8;        // atoms per splat step: two K = 4 products per tile
constexpr int kDGroup = 8;      // atoms per adjoint group: 16 columns (g, gd)
static_assert(kDStage % kDSub == 0 && kDStage % kDGroup == 0 && kDStage <= kDThreads, "record staging");
static_assert(kMI + kMJ + kMK == 64, "one factor entry per lane");
static_assert(kMI == 16 && kMJ == 16 && kMK == 32, "the tiling below");

// What lane q (0 .. 63) of a wavefront evaluates for every atom: entry q of
// the atom's factor row over this brick (q < 16 along a, q < 32 along b, the
// rest along c): the axis, the point's offset within the brick, its grid
// index, the axis length and the spacing h.
struct LaneAxis64 {
    int x, qq, g, n;
    double h;
};

__device__ __forceinline__ LaneAxis64 lane_axis64(const ProbDesc &d, const BrickPos &p, int q)
{
    LaneAxis64 la;
    la.x = q < kMI ? 0 : (q < kMI + kMJ ? 1 : 2);
    la.qq = q - (la.x == 0 ? 0 : (la.x == 1 ? kMI : kMI + kMJ));
    const int b = la.x == 0 ? p.b0 * kMI : (la.x == 1 ? p.b1 * kMJ : p.b2 * kMK);
    la.g = b + la.qq;
    la.n = d.dims[la.x];
    la.h = d.h[la.x];
    return la;
}

struct Entry64 {
    double g, gd;  // factor and displacement-weighted factor
    bool more;     // the window holds further images of this point
};

// This lane's entry of one staged atom: the unwrapped offsets r, r + n, ...
// inside the window width wl have grid index lo + r and displacement
// d = (lo + r) h - X; g = sum of exp(-d^2 / (2 sigma^2)), gd = the same
// weighted by d.  entry64 takes the first image; more_images64 adds the
// others (windows wider than the cell only).
__device__ __forceinline__ Entry64 entry64(const LaneAxis64 &la, const SlotAtom64 &at, bool use)
{
    const double X = at.X[la.x];
    const int lo = at.lo[la.x], r0 = at.r0[la.x], wl = at.wl[la.x];
    const bool ok = use && la.g < la.n;
    int r = r0 + la.qq;
    r = r >= la.n ? r - la.n : r;
    const double d = double(lo + r) * la.h - X;
    double e = exp(-(d * d) * at.inv2s2);
    e = (ok && r < wl) ? e : 0.0;
    return Entry64{e, e * d, ok && r + la.n < wl};
}

__device__ __forceinline__ void more_images64(const LaneAxis64 &la, const SlotAtom64 &at, bool use, double &gs,
                                              double &gds)
{
    const double X = at.X[la.x];
    const int lo = at.lo[la.x], r0 = at.r0[la.x], wl = at.wl[la.x];
    if (!(use && la.g < la.n)) return;
    int r = r0 + la.qq;
    r = r >= la.n ? r - la.n : r;
    for (r += la.n; r < wl; r += la.n) {
        const double d = double(lo + r) * la.h - X;
        const double e = exp(-(d * d) * at.inv2s2);
        gs += e;
        gds += e * d;
    }
}

// threads t < nc copy the records of list entries c0 + t to LDS
__device__ __forceinline__ void stage64(SlotAtom64 *dst, const SplatArgs &a, int64_t off, int c0, int nc, int t)
{
    if (t < nc) dst[t] = a.rec64[off + c0 + t];
}

__device__ __forceinline__ bool brick_inside(const ProbDesc &d, const BrickPos &p)
{
    return (p.b0 + 1) * kMI <= d.dims[0] && (p.b1 + 1) * kMJ <= d.dims[1] && (p.b2 + 1) * kMK <= d.dims[2];
}

// ---------------------------------------------------------------- splat

// One step's factors: fxw[s][i] = W gx(i), fy[s][j] = gy(j), gz[s][k] of
// staged atom s of the step.
struct SplatBuf64 {
    double fxw[kDSub][kMI], fy[kDSub][kMJ], gz[kDSub][kMK];
};

// factors of staged atoms s0 .. s0 + kDSub - 1 into buf (zeros past nb):
// wavefront w evaluates atoms w and w + 4 of the step, lane q entry q
template <bool WIDE>
__device__ __forceinline__ void splat_factors64(SplatBuf64 &buf, const SlotAtom64 *recs, const LaneAxis64 &la,
                                                int s0, int nb, int wave, int lane)
{
    constexpr int R = kDSub / 4;
    double v[R];
    bool more = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int s = s0 + wave + 4 * r;
        const Entry64 e = entry64(la, recs[s < nb ? s : 0], s < nb);
        v[r] = e.g;
        more = more || e.more;
    }
    if constexpr (WIDE) {
        if (__any(more)) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int s = s0 + wave + 4 * r;
                double gd = 0.0;
                more_images64(la, recs[s < nb ? s : 0], s < nb, v[r], gd);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int st = wave + 4 * r;
        if (la.x == 0)
            buf.fxw[st][la.qq] = v[r] * recs[(s0 + st) < nb ? s0 + st : 0].w;
        else if (la.x == 1)
            buf.fy[st][la.qq] = v[r];
        else
            buf.gz[st][la.qq] = v[r];
    }
}

// products of one step: acc[u][c] is the tile of i = 4 wave + u and points
// k = 16 c .. 16 c + 15
__device__ __forceinline__ void splat_products64(const SplatBuf64 &buf, int wave, int lane, doublex4 (&acc)[4][2])
{
    const int jj = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int m = 0; m < kDSub / 4; ++m) {
        const int s = 4 * m + kq;
        const double y = buf.fy[s][jj];
        const double b0 = buf.gz[s][jj], b1 = buf.gz[s][16 + jj];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double av = buf.fxw[s][4 * wave + u] * y;
            acc[u][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b0, acc[u][0], 0, 0, 0);
            acc[u][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b1, acc[u][1], 0, 0, 0);
        }
    }
}

template <bool WIDE>
__global__ __launch_bounds__(kDThreads) void k_splat_mfma64(SplatArgs a)
{
    __shared__ SlotAtom64 recs[kDStage];
    __shared__ SplatBuf64 fac[2];  // double buffer of pipeline steps
    const int64_t b = brick_of_block(a);
    const int prob = brick_prob(a, b);
    const ProbDesc &d = a.desc[prob];
    const BrickPos p = brick_pos(d, b);
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    const int64_t off = a.offsets[b];
    const int cnt = int(a.offsets[b + 1] - off);
    const LaneAxis64 la = lane_axis64(d, p, lane);

    // the accumulators start at the background -Q / Omega
    const double bg = a.subtract_background ? a.qsum[prob] / (d.L[0] * d.L[1] * d.L[2]) : 0.0;
    doublex4 acc[4][2];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[u][c] = doublex4{-bg, -bg, -bg, -bg};

    for (int blk = 0; blk < cnt; blk += kDStage) {
        const int nb = (cnt - blk) < kDStage ? (cnt - blk) : kDStage;
        stage64(recs, a, off, blk, nb, t);
        __syncthreads();
        const int nsub = (nb + kDSub - 1) / kDSub;
        splat_factors64<WIDE>(fac[0], recs, la, 0, nb, wave, lane);
        __syncthreads();
        for (int c = 0; c + 1 < nsub; ++c) {
            splat_factors64<WIDE>(fac[(c + 1) & 1], recs, la, (c + 1) * kDSub, nb, wave, lane);
            splat_products64(fac[c & 1], wave, lane, acc);
            __syncthreads();
        }
        splat_products64(fac[(nsub - 1) & 1], wave, lane, acc);
        __syncthreads();  // recs and fac are reused by the next block
    }
    // lane l holds rows j = 4 r + l / 16 at point k = 16 c + l % 16
    double *out = reinterpret_cast<double *>(a.rho) + d.grid_off;
    const int64_t sb = d.dims[2], sa = int64_t(d.dims[1]) * d.dims[2];  // row strides along b and a
    const int kq = lane >> 4, kl = lane & 15;
    if (brick_inside(d, p)) {
        // a wavefront-uniform base plus a 32-bit lane offset
        const int w = __builtin_amdgcn_readfirstlane(wave);
        double *base = out + (int64_t(p.b0 * kMI + 4 * w) * d.dims[1] + p.b1 * kMJ) * sb + p.b2 * kMK;
        const uint32_t loff = uint32_t(kq * d.dims[2] + kl);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double *row = base + (u * sa + 4 * r * sb);
                row[loff] = acc[u][0][r];
                row[loff + 16] = acc[u][1][r];
            }
        return;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int ia = p.b0 * kMI + 4 * wave + u;
        if (ia >= d.dims[0]) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = p.b1 * kMJ + 4 * r + kq;
            if (j >= d.dims[1]) continue;
            double *row = out + (int64_t(ia) * d.dims[1] + j) * sb;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int k = p.b2 * kMK + 16 * c + kl;
                if (k < d.dims[2]) row[k] = acc[u][c][r];
            }
        }
    }
}

// ---------------------------------------------------------------- adjoint

// One group's factors: gxy[s][q] = gx (q < 16) or gy (16 <= q < 32) of
// staged atom s of the group, gdxy the displacement-weighted ones; bz[n][k]:
// matrix column n < 8 is gz of atom n, n >= 8 gdz of atom n - 8 (the row
// pitch keeps the lanes' 16-byte reads of consecutive columns in different
// banks).
constexpr int kBzPitch = kMK + 2;
struct AdjBuf64 {
    double gxy[kDGroup][kMI + kMJ], gdxy[kDGroup][kMI + kMJ];
    double bz[2 * kDGroup][kBzPitch];
};

// factors of staged atoms s0 .. s0 + kDGroup - 1 into buf (zeros past nb):
// wavefront w evaluates atoms w and w + 4 of the group, lane q entry q
template <bool WIDE>
__device__ __forceinline__ void adjoint_factors64(AdjBuf64 &buf, const SlotAtom64 *recs, const LaneAxis64 &la,
                                                  int s0, int nb, int wave, int lane)
{
    constexpr int R = kDGroup / 4;
    Entry64 v[R];
    bool more = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int s = s0 + wave + 4 * r;
        v[r] = entry64(la, recs[s < nb ? s : 0], s < nb);
        more = more || v[r].more;
    }
    if constexpr (WIDE) {
        if (__any(more)) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int s = s0 + wave + 4 * r;
                more_images64(la, recs[s < nb ? s : 0], s < nb, v[r].g, v[r].gd);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int st = wave + 4 * r;
        if (lane < kMI + kMJ) {
            buf.gxy[st][lane] = v[r].g;
            buf.gdxy[st][lane] = v[r].gd;
        } else {
            buf.bz[st][la.qq] = v[r].g;
            buf.bz[kDGroup + st][la.qq] = v[r].gd;
        }
    }
}

// One group's products: acc[u] is S of the tile i = 4 wave + u, columns
// n = lane % 16, rows j = 4 r + lane / 16
__device__ __forceinline__ void adjoint_products64(const AdjBuf64 &buf, const double (&g)[4][8], int lane,
                                                   doublex4 (&acc)[4])
{
    const int n = lane & 15, kq = lane >> 4;
    const double *bcol = &buf.bz[n][8 * kq];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = doublex4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < 8; ks += 2) {
        const double2 bv = *reinterpret_cast<const double2 *>(bcol + ks);
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(g[u][ks], bv.x, acc[u], 0, 0, 0);
#pragma unroll
        for (int u = 0; u < 4; ++u)
            acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(g[u][ks + 1], bv.y, acc[u], 0, 0, 0);
    }
}

// The fold with the transverse factors, then the sum over the four lane
// groups (fixed butterfly); lanes n < 16 write the wavefront's partials to
// red[n][0 .. 1]: [0] the x component (f = 0) or the z component (f = 1),
// [1] the y component (f = 0; f = 1 lanes compute a value nobody reads,
// which keeps the fold free of branches).
__device__ __forceinline__ void adjoint_fold64(const AdjBuf64 &buf, const doublex4 (&acc)[4], int wave, int lane,
                                               double (*red)[2])
{
    const int n = lane & 15, kq = lane >> 4;
    const int f = n >> 3, sl = n & 7;
    const double *cx = f == 0 ? buf.gdxy[sl] : buf.gxy[sl];
    double ax = 0.0, ay = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        double sy = 0.0, sdy = 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = kMI + 4 * r + kq;
            sy += buf.gxy[sl][j] * acc[u][r];
            sdy += buf.gdxy[sl][j] * acc[u][r];
        }
        const int i = 4 * wave + u;
        ax += cx[i] * sy;
        ay += buf.gxy[sl][i] * sdy;
    }
    ax += __shfl_xor(ax, 16, 64);
    ay += __shfl_xor(ay, 16, 64);
    ax += __shfl_xor(ax, 32, 64);
    ay += __shfl_xor(ay, 32, 64);
    if (kq == 0) {
        red[n][0] = ax;
        red[n][1] = ay;
    }
}

// fixed-order sum over the 4 wavefronts of the partials of staged atoms
// s0 .. s0 + kDGroup - 1 (below nb), stored under (atom, touched brick)
// from their records: threads t < 24
__device__ __forceinline__ void adjoint_reduce64(const SplatArgs &a, const double (*red)[2 * kDGroup][2],
                                                 const SlotAtom64 *recs, int s0, int nb, int t)
{
    if (t < 3 * kDGroup) {
        const int st = t / 3, x = t - 3 * st;
        const int nn = x == 2 ? kDGroup + st : st;
        const int comp = x == 1 ? 1 : 0;
        double v = 0.0;
        for (int w = 0; w < 4; ++w) v += red[w][nn][comp];
        if (s0 + st < nb) {
            const SlotAtom64 &r = recs[s0 + st];
            a.bpart[(int64_t(r.atom) * a.cap_pa + r.touch) * 3 + x] = v;
        }
    }
}

// adjoint: wave w holds grad_rho of its four row tiles in registers; per
// group of 8 staged atoms it forms S for them (16 columns n = 8 f + atom)
// and folds the transverse factors in.  The products of a group are issued
// first, the next group's factors are evaluated while they run, then the
// fold; the previous group's partials are reduced at the top.
template <bool WIDE>
__global__ __launch_bounds__(kDThreads) __attribute__((amdgpu_waves_per_eu(3))) void k_adjoint_mfma64(SplatArgs a)
{
    __shared__ SlotAtom64 recs[kDStage];
    __shared__ AdjBuf64 buf[2];
    __shared__ double red[2][4][2 * kDGroup][2];  // [group parity][wave][n][component]
    const int64_t b = brick_of_block(a);
    const int prob = brick_prob(a, b);
    const ProbDesc &d = a.desc[prob];
    const BrickPos p = brick_pos(d, b);
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    const int64_t off = a.offsets[b];
    const int cnt = int(a.offsets[b + 1] - off);
    if (cnt == 0) return;
    const LaneAxis64 la = lane_axis64(d, p, lane);

    // grad_rho of this lane's A rows: tile u (i = 4 wave + u), row j = lane
    // % 16, points k = 8 (lane / 16) + ks of its K slots, ks = 0 .. 7.  Loads
    // outside the grid read the workspace's zero block.
    double g[4][8];
    const double *src = reinterpret_cast<const double *>(a.grad_rho) + d.grid_off;
    const int jj = lane & 15, kq = lane >> 4;
    const int64_t sb = d.dims[2], sa = int64_t(d.dims[1]) * d.dims[2];
    if (a.grad_rows_vec16 && brick_inside(d, p) && (d.dims[2] & 1) == 0 && (d.grid_off & 1) == 0) {
        // a wavefront-uniform base plus a 32-bit lane offset, 16-byte loads
        const int w = __builtin_amdgcn_readfirstlane(wave);
        const double *base = src + (int64_t(p.b0 * kMI + 4 * w) * d.dims[1] + p.b1 * kMJ) * sb + p.b2 * kMK;
        const uint32_t loff = uint32_t(jj * d.dims[2] + 8 * kq);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int ks = 0; ks < 8; ks += 2) {
                const double2 v = *reinterpret_cast<const double2 *>(base + u * sa + loff + ks);
                g[u][ks] = v.x;
                g[u][ks + 1] = v.y;
            }
    } else {
        const double *zeros = reinterpret_cast<const double *>(a.zeros);
        const int j = p.b1 * kMJ + jj;
        const int k0 = p.b2 * kMK + 8 * kq;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int ia = p.b0 * kMI + 4 * wave + u;
            const bool in = ia < d.dims[0] && j < d.dims[1];
            const double *row = src + (in ? (int64_t(ia) * d.dims[1] + j) * sb + k0 : 0);
#pragma unroll
            for (int ks = 0; ks < 8; ++ks) g[u][ks] = *(in && k0 + ks < d.dims[2] ? row + ks : zeros);
        }
    }

    for (int blk = 0; blk < cnt; blk += kDStage) {
        const int nb = (cnt - blk) < kDStage ? (cnt - blk) : kDStage;
        stage64(recs, a, off, blk, nb, t);
        __syncthreads();
        const int ngroup = (nb + kDGroup - 1) / kDGroup;
        adjoint_factors64<WIDE>(buf[0], recs, la, 0, nb, wave, lane);
        __syncthreads();
        for (int gi = 0; gi < ngroup; ++gi) {
            if (gi > 0) adjoint_reduce64(a, red[(gi - 1) & 1], recs, (gi - 1) * kDGroup, nb, t);
            doublex4 acc[4];
            adjoint_products64(buf[gi & 1], g, lane, acc);
            if (gi + 1 < ngroup)
                adjoint_factors64<WIDE>(buf[(gi + 1) & 1], recs, la, (gi + 1) * kDGroup, nb, wave, lane);
            adjoint_fold64(buf[gi & 1], acc, wave, lane, red[gi & 1][wave]);
            __syncthreads();
        }
        adjoint_reduce64(a, red[(ngroup - 1) & 1], recs, (ngroup - 1) * kDGroup, nb, t);
        __syncthreads();  // recs, buf and red are reused by the next block
    }
}

hipError_t run_gather_mfma64(const SplatArgs &a, hipStream_t s)
{
    const dim3 grid(int(a.nbricks_total)), block(kDThreads);
    if (a.wide)
        hipLaunchKernelGGL(k_splat_mfma64<true>, grid, block, 0, s, a);
    else
        hipLaunchKernelGGL(k_splat_mfma64<false>, grid, block, 0, s, a);
    return hipGetLastError();
}

hipError_t run_adjoint_mfma64(const SplatArgs &a, hipStream_t s)
{
    const dim3 grid(int(a.nbricks_total)), block(kDThreads);
    if (a.wide)
        hipLaunchKernelGGL(k_adjoint_mfma64<true>, grid, block, 0, s, a);
    else
        hipLaunchKernelGGL(k_adjoint_mfma64<false>, grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace hartree
