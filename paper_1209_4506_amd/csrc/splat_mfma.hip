// FP32 splat and splat adjoint on the matrix cores, both with 16-bit split
// products (three per FP32-accurate product): the splat with
// v_mfma_f32_32x32x8f16, the adjoint with v_mfma_f32_32x32x16_f16.
//
// A brick is 16 x 16 columns (i, j) by 32 points along c.  Inside it both
// operations are dense contractions over the brick's atom list:
//
//   splat    rho[c][k]  = sum_a  W_a gx_a(i_c) gy_a(j_c)  *  gz_a(k)
//            (columns x atoms) . (atoms x k)
//   adjoint  S[c][a, f] = sum_k  grho[c][k]  *  gz_a(k) (f = 0) or gdz_a(k) (f = 1)
//            (columns x k) . (k x atom functions), then per atom
//            F_a = sum_c [gdx gy S0, gx gdy S0, gx gy S1]
//
// with the per-axis factors gx, gdx, ... (1-D periodic Gaussians and their
// displacement-weighted sums) evaluated in the kernel from per-slot records.  The 256
// columns (c = 16 i + j) form 8 row tiles of 32; wavefront w owns tiles 2w
// and 2w + 1, i.e. local i = 4w, 4w + 1 and 4w + 2, 4w + 3.
//
// A 16-bit split writes an FP32 value x (scaled into the 16-bit range by a
// power of two) as hi + lo, hi = fp16(x), lo = fp16(x - hi): 22 significant
// bits.  A product of two split values is hi hi' + hi lo' + lo hi' (the
// dropped lo lo' is 2^-22 of it), each exact in the FP32 accumulation.
//
// Operand layout of v_mfma_f32_32x32x8f16 (C = A B + C, A 32x8, B 8x32):
// element e of lane l is K slot 4 (l / 32) + e of both A (row l % 32) and B
// (column l % 32); after the call lane l holds C[i][l % 32] for
// i = 8 (r / 4) + 4 (l / 32) + r % 4 in its accumulator element r = 0 .. 15.
// v_mfma_f32_32x32x16_f16 has the same C layout, with 8 K slots per lane
// (slot 8 (l / 32) + e).  Which reduction index sits in which K slot is free
// as long as A and B agree: the splat puts atom 4 (l / 32) + e of a step in
// slot e; the adjoint puts point k = 16 kap + 8 (l / 32) + e in slot e of its
// product kap, so that each lane's grad_rho values are two runs of 8 points
// of one column, loaded once into registers.
#include "splat_common.hpp"

namespace hartree {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int mfma_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

constexpr int kMThreads = 256;   // four wavefronts per brick
constexpr int kAdjGroup = 16;    // atoms per MFMA column tile: 16 atoms x (g, gd)
constexpr int kStage = 128;      // atom records staged at once (whole lists, almost always)
static_assert(kStage % kAdjGroup == 0 && kStage <= kMThreads, "record staging");
constexpr int kRow = kMI + kMJ + kMK;  // table entries one atom needs in one brick

// The brick's 1-D factors are evaluated on the fly from the atoms' SlotAtom
// records (written by the binning sort): along axis x, brick point q has
// grid index g = b_x bsz_x + q and lies at offset r = (r0 + q) mod n_x from
// the window start; its unwrapped images are r, r + n_x, ... while inside the
// window width wl_x, each with displacement d = r h_x - xb_x and factor
// exp(-d^2 / (2 sigma^2)).
typedef SlotAtom StagedG;

// What lane q (0 .. 63) of a wavefront evaluates for every atom: entry q of
// the atom's factor row over this brick, q < 16 along a, q < 32 along b, the
// rest along c.  Fixed per lane for the whole kernel, kept in registers: the
// axis, the point's offset within the brick and its grid index, the axis
// length, and the spacing h as a float plus its rounding remainder hl.
struct LaneAxis {
    int x, qq, g, n;
    float h, hl;
};

static_assert(kRow == 64, "one factor entry per lane");
static_assert(kMI == kMJ, "a and b share one brick edge");

__device__ __forceinline__ LaneAxis lane_axis(const ProbDesc &d, const BrickPos &p, int q)
{
    LaneAxis la;
    la.x = q < kMI ? 0 : (q < kMI + kMJ ? 1 : 2);
    la.qq = q - (la.x == 0 ? 0 : (la.x == 1 ? kMI : kMI + kMJ));
    const int b = la.x == 0 ? p.b0 * kMI : (la.x == 1 ? p.b1 * kMJ : p.b2 * kMK);
    la.g = b + la.qq;
    la.n = d.dims[la.x];
    la.h = d.hf[la.x];
    la.hl = d.hfl[la.x];
    return la;
}

// threads t < nc copy the records of list entries c0 + t to LDS
__device__ __forceinline__ void stage_g(StagedG *dst, const SplatArgs &a, int64_t off, int c0, int nc, int t)
{
    if (t < nc) dst[t] = a.rec[off + c0 + t];
}

struct Entry {
    float g, gd, w;  // factor, displacement-weighted factor, the atom's weight
    bool more;       // the window holds further images of this point
};

// This lane's entry of one staged atom (a record in LDS): g = sum over the
// unwrapped images r, r + n, ... inside the window of 2^(-d^2 c2) with
// d = r h - xb, and gd = the same sum weighted by d.  brick_entry takes the
// first image without branches; more_images adds the others, which exist
// only for windows wider than the cell (callers run it when any lane of any
// atom reports `more`, so the common path stays straight-line code).
__device__ __forceinline__ float axis_disp(const LaneAxis &la, float xb, float xbl, int r)
{
    // r h - xb with h and xb each carried as two floats: one rounding
    return fmaf(float(r), la.h, -xb) + (float(r) * la.hl - xbl);
}

__device__ __forceinline__ Entry brick_entry(const LaneAxis &la, const StagedG *at, bool use)
{
    const float4 rx = *reinterpret_cast<const float4 *>(&at->ax[la.x]);
    const float2 cw = *reinterpret_cast<const float2 *>(&at->c2);
    const int r0 = __float_as_int(rx.z), wl = __float_as_int(rx.w);
    const bool ok = use && la.g < la.n;
    int r = r0 + la.qq;
    r = r >= la.n ? r - la.n : r;
    const float dd = axis_disp(la, rx.x, rx.y, r);
    float e = __builtin_amdgcn_exp2f(-(dd * dd) * cw.x);
    e = (ok && r < wl) ? e : 0.0f;
    return Entry{e, e * dd, cw.y, ok && r + la.n < wl};
}

__device__ __forceinline__ void more_images(const LaneAxis &la, const StagedG *at, bool use, float &gs, float &gds)
{
    const float4 rx = *reinterpret_cast<const float4 *>(&at->ax[la.x]);
    const float c2 = at->c2;
    const int r0 = __float_as_int(rx.z), wl = __float_as_int(rx.w);
    if (!(use && la.g < la.n)) return;
    int r = r0 + la.qq;
    r = r >= la.n ? r - la.n : r;
    for (r += la.n; r < wl; r += la.n) {
        const float dd = axis_disp(la, rx.x, rx.y, r);
        const float e = __builtin_amdgcn_exp2f(-(dd * dd) * c2);
        gs += e;
        gds += e * dd;
    }
}

// Splat pipeline step: kSub atoms, one K = 8 product set per tile.  While
// the products of step c run on the matrix cores, the wavefronts evaluate
// the factors of step c + 1 into the other LDS buffer, so the vector work
// fills the matrix cores' shadow.
constexpr int kSub = 8;
static_assert(kSub % 4 == 0 && kStage % kSub == 0, "pipeline step");

// One step's factors, entry-major so that a lane reads its four atoms of one
// entry as one 16-byte (8-byte) vector: fxy[q][s] = 2^ea W gx (q < 16) or gy
// (16 <= q < 32) of staged atom s of the step, zhi / zlo[k][s] the two halves
// of the 16-bit split of 2^eb gz(k).  Rows of 12 entries: the factor stage's
// stores of consecutive entries (one per lane) fall two to a bank at most
// (one for the 16-bit rows), and every read stays an aligned vector.
constexpr int kFacPitch = 12;
struct SplatBuf {
    float fxy[kMI + kMJ][kFacPitch];
    _Float16 zhi[kMK][kFacPitch], zlo[kMK][kFacPitch];
};
static_assert(kFacPitch >= kSub && kFacPitch % 4 == 0, "aligned 4-entry reads");

__device__ __forceinline__ void split16(float x, _Float16 &hi, _Float16 &lo)
{
    hi = _Float16(x);
    lo = _Float16(x - float(hi));
}

// factors of staged atoms s0 .. s0 + kSub - 1 into buf (zeros past nb).
// WIDE: some window may hold several images of a point (otherwise the first
// image is the only one, and the step stays one straight-line block)
template <bool WIDE>
__device__ __forceinline__ void splat_factors(SplatBuf &buf, const StagedG *recs, const LaneAxis &la, int s0, int nb,
                                              int wave, int lane, float ascale, float bscale)
{
    constexpr int R = kSub / 4;  // atoms per wavefront
    float v[R], wv[R];
    bool more = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int s = s0 + wave + 4 * r;
        const Entry e = brick_entry(la, recs + (s < nb ? s : 0), s < nb);
        v[r] = e.g;
        wv[r] = e.w;
        more = more || e.more;
    }
    if constexpr (WIDE) {
        if (__any(more)) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int s = s0 + wave + 4 * r;
                float gd = 0.0f;
                more_images(la, recs + (s < nb ? s : 0), s < nb, v[r], gd);
            }
        }
    }
    if (lane < kMI + kMJ) {
#pragma unroll
        for (int r = 0; r < R; ++r) buf.fxy[lane][wave + 4 * r] = la.x == 0 ? v[r] * wv[r] * ascale : v[r];
    } else {
        const int k = lane - kMI - kMJ;
#pragma unroll
        for (int r = 0; r < R; ++r) split16(v[r] * bscale, buf.zhi[k][wave + 4 * r], buf.zlo[k][wave + 4 * r]);
    }
}

// the 16-bit split of the products x[e] y[e]: hi = fp16(p) of the FP32
// product p, lo = fp16(x y - hi) with the residual exact (one fma).  p is
// pinned in a register first: otherwise the compiler may form hi once as
// fp16(p) and once as fp16(x y) (one rounding, by a mixed-precision fma),
// and the two differ near rounding midpoints, which would leave an error of
// one 16-bit ulp.
__device__ __forceinline__ void split_products(const float4 &x, const float4 &y, half4 &hi, half4 &lo)
{
    const float xs[4] = {x.x, x.y, x.z, x.w}, ys[4] = {y.x, y.y, y.z, y.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        float p = xs[e] * ys[e];
        asm("" : "+v"(p));
        const _Float16 h = _Float16(p);
        hi[e] = h;
        lo[e] = _Float16(fmaf(xs[e], ys[e], -float(h)));
    }
}

// products of one step: atom 4 kk + e of the step in K slot e of lane half
// kk.  (hi + lo)(hi' + lo') without lo lo', the small terms first; the two
// tiles' chains interleaved.
__device__ __forceinline__ void splat_products(const SplatBuf &buf, int kk, int col, int i0, int jj, floatx16 &acc0,
                                               floatx16 &acc1)
{
    const float4 y = *reinterpret_cast<const float4 *>(&buf.fxy[kMI + jj][4 * kk]);
    const float4 x0 = *reinterpret_cast<const float4 *>(&buf.fxy[i0][4 * kk]);
    const float4 x1 = *reinterpret_cast<const float4 *>(&buf.fxy[i0 + 2][4 * kk]);
    const half4 bh = *reinterpret_cast<const half4 *>(&buf.zhi[col][4 * kk]);
    const half4 bl = *reinterpret_cast<const half4 *>(&buf.zlo[col][4 * kk]);
    half4 ah0, al0, ah1, al1;
    split_products(x0, y, ah0, al0);
    split_products(x1, y, ah1, al1);
    acc0 = __builtin_amdgcn_mfma_f32_32x32x8f16(al0, bh, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_32x32x8f16(al1, bh, acc1, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_32x32x8f16(ah0, bl, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_32x32x8f16(ah1, bl, acc1, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_32x32x8f16(ah0, bh, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_32x32x8f16(ah1, bh, acc1, 0, 0, 0);
}

// Operand scales of the splat (uniform over a brick): the row operand
// 2^ea W gx gy and the column operand 2^eb gz stay below 2^13, inside the
// 16-bit range with room to spare, whatever the atoms' weights (W <= the
// problem's largest weight wmax from the binning).  A factor is one Gaussian
// (<= 1) unless the window is wider than the cell; then the periodic sum
// over images is at most 1 + sqrt(2 pi) sigma / L.  The exponents are
// clamped to +-60 (weights below 2^-47 lose relative precision).
__device__ __forceinline__ void splat_scales(const SplatArgs &a, const ProbDesc &d, int prob, int &ea, int &eb)
{
    double g[3] = {1.0, 1.0, 1.0};
    if (a.wide)
        for (int x = 0; x < 3; ++x) g[x] = 1.0 + 2.5066282746310002 * a.max_sigma / d.L[x];
    const double wb = a.qsum[a.nprob + prob] * g[0] * g[1];
    int e = 0;
    ea = 0;
    if (wb > 0.0 && wb < 1.0e300) {
        frexp(wb, &e);  // wb < 2^e
        ea = 13 - e;
    }
    ea = ea < -60 ? -60 : (ea > 60 ? 60 : ea);
    frexp(g[2], &e);
    eb = 13 - e;
    eb = eb < -60 ? -60 : eb;
}

// six workgroups per CU (80 registers): measured a little faster than the
// compiler's choice of five
template <bool WIDE>
__global__ __launch_bounds__(kMThreads) __attribute__((amdgpu_waves_per_eu(6))) void k_splat_mfma(SplatArgs a)
{
    __shared__ StagedG recs[kStage];
    __shared__ SplatBuf fac[2];  // double buffer of pipeline steps
    const int64_t b = brick_of_block(a);
    const int prob = brick_prob(a, b);
    const ProbDesc &d = a.desc[prob];
    const BrickPos p = brick_pos(d, b);
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    const int64_t off = a.offsets[b];
    const int cnt = int(a.offsets[b + 1] - off);
    const int kk = lane >> 5, col = lane & 31;
    // this lane's A rows: column 32 (2 wave + u) + col, i.e. local
    // i = 4 wave + 2 u + col / 16 and j = col % 16, for u = 0, 1
    const int i0 = 4 * wave + (col >> 4), jj = col & 15;
    const LaneAxis la = lane_axis(d, p, lane);
    int ea, eb;
    splat_scales(a, d, prob, ea, eb);
    const float ascale = __builtin_ldexpf(1.0f, ea), bscale = __builtin_ldexpf(1.0f, eb);
    const float unscale = __builtin_ldexpf(1.0f, -ea - eb);

    // the accumulators start at the background -Q / Omega (scaled like the products)
    const float bg = a.subtract_background ? float(a.qsum[prob] / (d.L[0] * d.L[1] * d.L[2])) : 0.0f;
    const float bgs = -bg * (ascale * bscale);
    floatx16 acc0, acc1;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        acc0[r] = bgs;
        acc1[r] = bgs;
    }

    for (int blk = 0; blk < cnt; blk += kStage) {
        const int nb = (cnt - blk) < kStage ? (cnt - blk) : kStage;
        stage_g(recs, a, off, blk, nb, t);
        __syncthreads();
        const int nsub = (nb + kSub - 1) / kSub;
        splat_factors<WIDE>(fac[0], recs, la, 0, nb, wave, lane, ascale, bscale);
        __syncthreads();
        for (int c = 0; c + 1 < nsub; ++c) {
            splat_factors<WIDE>(fac[(c + 1) & 1], recs, la, (c + 1) * kSub, nb, wave, lane, ascale, bscale);
            splat_products(fac[c & 1], kk, col, i0, jj, acc0, acc1);
            __syncthreads();
        }
        splat_products(fac[(nsub - 1) & 1], kk, col, i0, jj, acc0, acc1);
        __syncthreads();  // recs and fac are reused by the next block
    }
    float *out = reinterpret_cast<float *>(a.rho) + d.grid_off;
    const int64_t sb = d.dims[2], sa = int64_t(d.dims[1]) * d.dims[2];  // row strides along b and a
    if ((p.b0 + 1) * kMI <= d.dims[0] && (p.b1 + 1) * kMJ <= d.dims[1] && (p.b2 + 1) * kMK <= d.dims[2]) {
        // a brick inside the grid: the row of accumulator element r is
        // uniform across the wavefront apart from the lane's j offset 4 kk,
        // so each store is a wavefront-uniform base plus a 32-bit lane offset
        const int w = __builtin_amdgcn_readfirstlane(wave);
        float *base = out + (int64_t(p.b0 * kMI + 4 * w) * d.dims[1] + p.b1 * kMJ) * sb + p.b2 * kMK;
        const uint32_t loff = uint32_t(4 * kk * d.dims[2] + col);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int c8 = 8 * (r >> 2) + (r & 3);  // mfma_row without the lane's 4 kk (never crosses a 16-row line)
            float *row = base + ((c8 >> 4) * sa + (c8 & 15) * sb);
            row[loff] = acc0[r] * unscale;
            row[2 * sa + loff] = acc1[r] * unscale;
        }
        return;
    }
    const int k = p.b2 * kMK + col;
    if (k >= d.dims[2]) return;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int c = mfma_row(r, lane);  // row within the tile: local i offset c / 16, j = c % 16
        const int j = p.b1 * kMJ + (c & 15);
        const int ia = p.b0 * kMI + 4 * wave + (c >> 4);
        if (j < d.dims[1]) {
            if (ia < d.dims[0]) out[(int64_t(ia) * d.dims[1] + j) * d.dims[2] + k] = acc0[r] * unscale;
            if (ia + 2 < d.dims[0]) out[(int64_t(ia + 2) * d.dims[1] + j) * d.dims[2] + k] = acc1[r] * unscale;
        }
    }
}

// Adjoint pipeline step: one group of kAdjGroup atoms.  Its factors sit in
// one of two LDS buffers: gx | gy and gdx | gdy rows per atom, and the gz,
// gdz rows of the group's 32 matrix columns.
// Matrix columns n < 16 hold gz of atom n, n >= 16 gdz of atom n - 16, as
// the two halves of a 16-bit split (scaled by b_scale): x b_scale =
// hi + lo, hi = fp16(x b_scale), lo = fp16(x b_scale - hi).  Rows of kBPitch
// halves keep every 8-half run 16-byte aligned.
constexpr int kBPitch = kMK + 8;
struct AdjBuf {
    float gxy[kAdjGroup][kMI + kMJ + 1], gdxy[kAdjGroup][kMI + kMJ + 1];
    _Float16 bhi[2 * kAdjGroup][kBPitch], blo[2 * kAdjGroup][kBPitch];
};

// factors of staged atoms s0 .. s0 + kAdjGroup - 1 into buf (zeros past nb)
template <bool WIDE>
__device__ __forceinline__ void adjoint_factors(AdjBuf &buf, const StagedG *recs, const LaneAxis &la, int s0, int nb,
                                                int wave, int lane, float bscale)
{
    constexpr int R = kAdjGroup / 4;  // atoms per wavefront
    Entry v[R];
    bool more = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int s = s0 + wave + 4 * r;
        v[r] = brick_entry(la, recs + (s < nb ? s : 0), s < nb);
        more = more || v[r].more;
    }
    if constexpr (WIDE) {
        if (__any(more)) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int s = s0 + wave + 4 * r;
                more_images(la, recs + (s < nb ? s : 0), s < nb, v[r].g, v[r].gd);
            }
        }
    }
    const bool xy = lane < kMI + kMJ;
    const int zq = lane - kMI - kMJ;
    if (xy) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int st = wave + 4 * r;
            buf.gxy[st][lane] = v[r].g;
            buf.gdxy[st][lane] = v[r].gd;
        }
    } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int st = wave + 4 * r;
            split16(v[r].g * bscale, buf.bhi[st][zq], buf.blo[st][zq]);
            split16(v[r].gd * bscale, buf.bhi[kAdjGroup + st][zq], buf.blo[kAdjGroup + st][zq]);
        }
    }
}

// One group's products and fold, split in two so that the caller can
// evaluate the next group's factors while the products run on the matrix
// cores.  Lane l holds S[row][n] for column n = l % 32 (function f = n / 16
// of atom n % 16) and 16 rows of each of its two tiles: row r of tile u is
// local i = 4 wave + 2 u + r / 8 and j = 8 ((r / 4) % 2) + 4 half + r % 4, so
// the eight j values (and their gy, gdy) are the same for both tiles and
// both halves r / 8.
__device__ __forceinline__ void adjoint_products(const AdjBuf &buf, const half8 (&ah)[2][2], const half8 (&al)[2][2],
                                                 int lane, floatx16 (&acc)[2])
{
    const int half = lane >> 5, n = lane & 31;
    // B operand: column n at points 16 kap + 8 half + e, e = 0 .. 7, in the
    // same K slots as the A operand's grad_rho
    half8 bh[2], bl[2];
#pragma unroll
    for (int kap = 0; kap < 2; ++kap) {
        bh[kap] = *reinterpret_cast<const half8 *>(&buf.bhi[n][16 * kap + 8 * half]);
        bl[kap] = *reinterpret_cast<const half8 *>(&buf.blo[n][16 * kap + 8 * half]);
    }
    // the two tiles' product chains interleaved (each tile's own order is
    // fixed): (hi + lo)(hi' + lo') without lo lo', the small terms first
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[u][r] = 0.0f;
#pragma unroll
    for (int kap = 0; kap < 2; ++kap)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            acc[u] = __builtin_amdgcn_mfma_f32_32x32x16_f16(al[u][kap], bh[kap], acc[u], 0, 0, 0);
            acc[u] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah[u][kap], bl[kap], acc[u], 0, 0, 0);
        }
#pragma unroll
    for (int kap = 0; kap < 2; ++kap)
#pragma unroll
        for (int u = 0; u < 2; ++u) acc[u] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah[u][kap], bh[kap], acc[u], 0, 0, 0);
}

// The fold of the products with the transverse factors; writes the lane's
// two partial components to red[n][0 .. 1]: ax, the x component (f = 0) or
// the z component (f = 1), and ay, the y component (f = 0; f = 1 lanes
// compute a value nobody reads, which keeps the fold free of branches).
// The x coefficient of row i is gdx (f = 0) or gx (f = 1), that of ay gx.
__device__ __forceinline__ void adjoint_fold(const AdjBuf &buf, const floatx16 (&acc)[2], const float (&unscale)[2],
                                             int wave, int lane, float (*red)[2])
{
    const int n = lane & 31;
    const int f = n >> 4, sl = n & 15;
    float yv[8], dyv[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int j = mfma_row(r, lane) & 15;
        yv[r] = buf.gxy[sl][kMI + j];
        dyv[r] = buf.gdxy[sl][kMI + j];
    }
    float ax = 0.0f, ay = 0.0f;
    const float *cx = f == 0 ? buf.gdxy[sl] : buf.gxy[sl];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int i = 4 * wave + 2 * u + h;
            float sy = 0.0f, sdy = 0.0f;
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                sy += yv[r] * acc[u][8 * h + r];
                sdy += dyv[r] * acc[u][8 * h + r];
            }
            // the fold is linear in the products: undo the operand scales here
            ax += cx[i] * (sy * unscale[u]);
            ay += buf.gxy[sl][i] * (sdy * unscale[u]);
        }
    red[n][0] = ax;
    red[n][1] = ay;
}

// fixed-order sum over the 4 waves and 2 lane halves, in double, of the
// partials of staged atoms s0 .. s0 + kAdjGroup - 1 (below nb), stored
// under (atom, touched brick) from their records: threads t < 48
__device__ __forceinline__ void adjoint_reduce(const SplatArgs &a, const float (*red)[2][2 * kAdjGroup][2],
                                               const StagedG *recs, int s0, int nb, int t)
{
    if (t < 3 * kAdjGroup) {
        const int st = t / 3, x = t - 3 * st;
        const int nn = x == 2 ? kAdjGroup + st : st;
        const int comp = x == 1 ? 1 : 0;
        double v = 0.0;
        for (int w = 0; w < 4; ++w) v += double(red[w][0][nn][comp]) + double(red[w][1][nn][comp]);
        if (s0 + st < nb) {
            const StagedG &r = recs[s0 + st];
            a.bpart[(int64_t(r.atom) * a.cap_pa + r.touch) * 3 + x] = v;
        }
    }
}

// The wavefront's grad_rho rows of tile u (g0: u = 0, g1: u = 1) as the two
// halves of a 16-bit split of g 2^k_u, with k_u the power of two that puts
// the tile's largest magnitude in [2^13, 2^14) (clamped to the float range;
// an all-zero tile takes k_u = 14).  unscale[u] = 2^-(k_u + b_exp) undoes
// both operands' scales.
__device__ __forceinline__ void split_grad(const float (&g0)[16], const float (&g1)[16], half8 (&ah)[2][2],
                                           half8 (&al)[2][2], float (&unscale)[2], int b_exp)
{
    float m0 = 0.0f, m1 = 0.0f;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        m0 = fmaxf(m0, fabsf(g0[q]));
        m1 = fmaxf(m1, fabsf(g1[q]));
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        m0 = fmaxf(m0, __shfl_xor(m0, off, 64));
        m1 = fmaxf(m1, __shfl_xor(m1, off, 64));
    }
    int k[2] = {14 - __builtin_amdgcn_frexp_expf(m0), 14 - __builtin_amdgcn_frexp_expf(m1)};
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        k[u] = k[u] < -126 ? -126 : (k[u] > 127 ? 127 : k[u]);
        unscale[u] = __builtin_ldexpf(1.0f, -k[u] - b_exp);
        const float sc = __builtin_ldexpf(1.0f, k[u]);
#pragma unroll
        for (int kap = 0; kap < 2; ++kap)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                _Float16 hi, lo;
                split16((u == 0 ? g0[8 * kap + e] : g1[8 * kap + e]) * sc, hi, lo);
                ah[u][kap][e] = hi;
                al[u][kap][e] = lo;
            }
    }
}

// adjoint: wave w holds grad_rho of its two row tiles in registers; per
// group of 16 staged atoms it forms S for both tiles (32 columns n = 16 f +
// atom) and folds the transverse factors in.  While a group's products run
// on the matrix cores, the factors of the next group are evaluated, and the
// previous group's partials are reduced.
// Three workgroups per CU (a few registers spill to scratch): measured
// faster than two without spills.
template <int VM, bool WIDE>
__global__ __launch_bounds__(kMThreads) __attribute__((amdgpu_waves_per_eu(3))) void k_adjoint_mfma(SplatArgs a)
{
    __shared__ StagedG recs[kStage];
    __shared__ AdjBuf buf[2];
    __shared__ float red[2][4][2][2 * kAdjGroup][2];  // [step parity][wave][lane half][n][component]
    const int64_t b = brick_of_block(a);
    const int prob = brick_prob(a, b);
    const ProbDesc &d = a.desc[prob];
    const BrickPos p = brick_pos(d, b);
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    const int64_t off = a.offsets[b];
    const int cnt = int(a.offsets[b + 1] - off);
    if (cnt == 0) return;
    const int half = lane >> 5, col = lane & 31;
    const LaneAxis la = lane_axis(d, p, lane);

    // The first records are requested before grad_rho, so that storing them
    // to LDS (and evaluating the factors) waits for them alone while the
    // grad_rho loads are still in flight.  (Named vectors: a local array
    // here would live in scratch memory.)
    static_assert(sizeof(StagedG) == 64, "records move as four 16-byte vectors");
    const int ns0 = cnt < kStage ? cnt : kStage;
    const uint4 *rsrc = reinterpret_cast<const uint4 *>(a.rec + off + (t < ns0 ? t : 0));
    const uint4 rr0 = rsrc[0], rr1 = rsrc[1], rr2 = rsrc[2], rr3 = rsrc[3];

    // grad_rho of this lane's two A rows (local i = 4 wave + col / 16 and
    // + 2, j = col % 16) at the points of its K slots: entry q = 8 kap + e
    // (kap = 0, 1; e = 0 .. 7) is point k = 32 bk + 16 kap + 8 half + e, i.e.
    // float4 v at offset 16 (v / 2) + 4 (v % 2) from 32 bk + 8 half.
    // Every load is unconditional (an element outside the grid reads a zero
    // block of the workspace), so no branch or arithmetic on the loaded
    // values separates the loads from the record wait below: they stay in
    // flight until the matrix products.  vec: this problem's rows start
    // 16-byte aligned, each a multiple of 4 points; VM = 1: true of every
    // problem (known at compile time), 2: checked per problem, 0: never.
    float g0[16], g1[16];
    half8 ah[2][2], al[2][2];
    float unscale[2];
    const float bscale = __builtin_ldexpf(1.0f, a.b_exp);
    const float *src = reinterpret_cast<const float *>(a.grad_rho) + d.grid_off;
    const bool interior =
        (p.b0 + 1) * kMI <= d.dims[0] && (p.b1 + 1) * kMJ <= d.dims[1] && (p.b2 + 1) * kMK <= d.dims[2];
    const bool vec = VM == 1 || (VM == 2 && (d.dims[2] & 3) == 0 && (d.grid_off & 3) == 0);
    if (vec) {
        // the eight 16-byte vectors of the lane's two rows, addressed first
        // and loaded by one common sequence
        const float4 *pv0[4], *pv1[4];
        if (interior) {
            // a brick inside the grid: a wavefront-uniform base plus a
            // 32-bit lane offset, every load in range
            const int w = __builtin_amdgcn_readfirstlane(wave);
            const int64_t sb = d.dims[2], sa = int64_t(d.dims[1]) * d.dims[2];
            const float *base = src + (int64_t(p.b0 * kMI + 4 * w) * d.dims[1] + p.b1 * kMJ) * sb + p.b2 * kMK;
            const uint32_t loff = uint32_t(((col >> 4) * d.dims[1] + (col & 15)) * d.dims[2] + 8 * half);
            const float4 *r0 = reinterpret_cast<const float4 *>(base + loff);
            const float4 *r1 = reinterpret_cast<const float4 *>(base + 2 * sa + loff);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int vo = 4 * (q >> 1) + (q & 1);  // float4 offset of slot vector q
                pv0[q] = r0 + vo;
                pv1[q] = r1 + vo;
            }
        } else {
            const int j = p.b1 * kMJ + (col & 15);
            const int ia = p.b0 * kMI + 4 * wave + (col >> 4);
            const int k0 = p.b2 * kMK + 8 * half;
            const bool jin = j < d.dims[1];
            const bool in0 = jin && ia < d.dims[0], in1 = jin && ia + 2 < d.dims[0];
            const float *row0 = src + (in0 ? (int64_t(ia) * d.dims[1] + j) * d.dims[2] + k0 : 0);
            const float *row1 = src + (in1 ? (int64_t(ia + 2) * d.dims[1] + j) * d.dims[2] + k0 : 0);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int ko = 16 * (q >> 1) + 4 * (q & 1);
                const bool kin = k0 + ko < d.dims[2];  // whole vectors: Nc is a multiple of 4
                pv0[q] = reinterpret_cast<const float4 *>(in0 && kin ? row0 + ko : a.zeros);
                pv1[q] = reinterpret_cast<const float4 *>(in1 && kin ? row1 + ko : a.zeros);
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 v0 = *pv0[q], v1 = *pv1[q];
            g0[4 * q] = v0.x;
            g0[4 * q + 1] = v0.y;
            g0[4 * q + 2] = v0.z;
            g0[4 * q + 3] = v0.w;
            g1[4 * q] = v1.x;
            g1[4 * q + 1] = v1.y;
            g1[4 * q + 2] = v1.z;
            g1[4 * q + 3] = v1.w;
        }
    } else {
        const int j = p.b1 * kMJ + (col & 15);
        const int ia = p.b0 * kMI + 4 * wave + (col >> 4);
        const int k0 = p.b2 * kMK + 8 * half;
        const bool jin = j < d.dims[1];
        const bool in0 = jin && ia < d.dims[0], in1 = jin && ia + 2 < d.dims[0];
        const float *row0 = src + (in0 ? (int64_t(ia) * d.dims[1] + j) * d.dims[2] + k0 : 0);
        const float *row1 = src + (in1 ? (int64_t(ia + 2) * d.dims[1] + j) * d.dims[2] + k0 : 0);
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int ko = 16 * (m >> 3) + (m & 7);
            const bool kin = k0 + ko < d.dims[2];
            g0[m] = *(in0 && kin ? row0 + ko : a.zeros);
            g1[m] = *(in1 && kin ? row1 + ko : a.zeros);
        }
    }

    // keep the grad_rho loads issued above this point (the compiler would
    // otherwise sink them below the record store and its wait)
    asm volatile("" ::: "memory");
    if (t < ns0) {
        uint4 *dst = reinterpret_cast<uint4 *>(recs + t);
        dst[0] = rr0;
        dst[1] = rr1;
        dst[2] = rr2;
        dst[3] = rr3;
    }
    __syncthreads();

    for (int blk = 0; blk < cnt; blk += kStage) {
        const int nb = (cnt - blk) < kStage ? (cnt - blk) : kStage;
        if (blk > 0) {
            stage_g(recs, a, off, blk, nb, t);
            __syncthreads();
        }
        const int ngroup = (nb + kAdjGroup - 1) / kAdjGroup;
        adjoint_factors<WIDE>(buf[0], recs, la, 0, nb, wave, lane, bscale);
        __syncthreads();
        if (blk == 0) split_grad(g0, g1, ah, al, unscale, a.b_exp);
        for (int gi = 0; gi < ngroup; ++gi) {
            if (gi > 0) adjoint_reduce(a, red[(gi - 1) & 1], recs, (gi - 1) * kAdjGroup, nb, t);
            floatx16 acc[2];
            adjoint_products(buf[gi & 1], ah, al, lane, acc);
            if (gi + 1 < ngroup)
                adjoint_factors<WIDE>(buf[(gi + 1) & 1], recs, la, (gi + 1) * kAdjGroup, nb, wave, lane, bscale);
            adjoint_fold(buf[gi & 1], acc, unscale, wave, lane, red[gi & 1][wave][half]);
            __syncthreads();
        }
        adjoint_reduce(a, red[(ngroup - 1) & 1], recs, (ngroup - 1) * kAdjGroup, nb, t);
        __syncthreads();  // recs, buf and red are reused by the next block
    }
}

hipError_t run_gather_mfma(const SplatArgs &a, hipStream_t s)
{
    const dim3 grid(int(a.nbricks_total)), block(kMThreads);
    if (a.wide)
        hipLaunchKernelGGL(k_splat_mfma<true>, grid, block, 0, s, a);
    else
        hipLaunchKernelGGL(k_splat_mfma<false>, grid, block, 0, s, a);
    return hipGetLastError();
}

hipError_t run_adjoint_mfma(const SplatArgs &a, hipStream_t s)
{
    const dim3 grid(int(a.nbricks_total)), block(kMThreads);
    const int vm = a.grad_rows_vec16;  // 0, 1, 2 as the kernel's VM
    if (vm == 1 && a.wide)
        hipLaunchKernelGGL((k_adjoint_mfma<1, true>), grid, block, 0, s, a);
    else if (vm == 1)
        hipLaunchKernelGGL((k_adjoint_mfma<1, false>), grid, block, 0, s, a);
    else if (vm == 2 && a.wide)
        hipLaunchKernelGGL((k_adjoint_mfma<2, true>), grid, block, 0, s, a);
    else if (vm == 2)
        hipLaunchKernelGGL((k_adjoint_mfma<2, false>), grid, block, 0, s, a);
    else if (a.wide)
        hipLaunchKernelGGL((k_adjoint_mfma<0, true>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((k_adjoint_mfma<0, false>), grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace hartree
