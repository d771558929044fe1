// The five grid passes of the Hartree solve and the E_H finalize.
//
// Layouts: the real grid is [Na][Nb][Nc] (c fastest); the half spectrum kept
// in the workspace is [Na][Nb][Nh], Nh = Nc/2 + 1, and is transformed in
// place.  The passes follow the calculation flow of Sec. 3.2.4 (abc -> cab ->
// cba -> cab -> abc): on one GPU each change of "local axis" becomes a pass
// that streams the grid through one workgroup's LDS, transforming pencils
// along that axis.
//
//   P1  r2c along c      real grid -> half spectrum   (two real rows per complex pencil)
//   P2  FFT along b      in place
//   P3  FFT along a, x K(G)/N, E_H partials, inverse FFT along a   (fused; in place)
//   P4  inverse FFT along b
//   P5  c2r along c      half spectrum -> real grid
//
// K(G) = 4 pi / |G|^2 with K(0) = 0 (Eq. (6) in a neutral periodic cell);
// E_H = Omega / (2 N^2) sum_m w(m_c) K |X|^2, w = 1 on the m_c = 0 and
// Nyquist planes, 2 elsewhere (the half spectrum stands for both halves).
#pragma once

#include <map>
#include <mutex>
#include <type_traits>

#include "fft_core.hpp"
#include "kernels.hpp"

namespace hartree {

// A workgroup has 256 threads: P pencils (P = 1 << p_log2, chosen by the
// host per launch) with tpp = 256 / P threads each; the LDS tile holds
// n (P + pad) complex values (strided axes) or P row_pitch(n) (axis c), then
// the axis' n twiddle factors.
constexpr int kPassThreads = 256;

// 16-byte vectors of reals for the contiguous real-grid rows
template <typename T>
struct VecW;
template <>
struct VecW<float> {
    static constexpr int W = 4;
    typedef float V __attribute__((ext_vector_type(4)));
    __device__ static V zero() { return V{0.0f, 0.0f, 0.0f, 0.0f}; }
};
template <>
struct VecW<double> {
    static constexpr int W = 2;
    typedef double V __attribute__((ext_vector_type(2)));
    __device__ static V zero() { return V{0.0, 0.0}; }
};

// the problem and tile of work item `item`: the last i with start[i] <= item,
// by bisection over the launch's problems (uniform scalar loads)
__device__ __forceinline__ void find_item(const TileList &tl, int item, int &prob, int &tile)
{
    int lo = 0, hi = tl.count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (item >= tl.start[mid]) lo = mid;
        else hi = mid - 1;
    }
    prob = tl.prob[lo];
    tile = item - tl.start[lo];
}

template <typename T>
__device__ __forceinline__ void load_twiddles(Cx<T> *dst, const Cx<T> *src, int n, int tid, int nt)
{
    for (int i = tid; i < n; i += nt) dst[i] = src[i];
}

// ------------------------------------------------------ c-axis accessors
// The c axis is contiguous: threads run along a pencil (tip fastest), so the
// first stage of P1 reads, and the last stage of P5 writes, consecutive
// points of two real grid rows straight from and to global memory.  A
// complex pencil packs rows 2q (real part) and 2q + 1 (imaginary part).

// P1 input: element i of the pair.  MODE 0: x = rho;  1: x = grad_v + s rho;
// 2: x = s rho (no grad_v).  A row beyond the grid reads a valid row of the
// tile and is weighted by zero, so the loads carry no branches.
template <typename T, int MODE>
struct RealPairIn {
    static constexpr bool kLds = false;
    const T *r0, *r1;       // rows 2q and 2q + 1 of the source (grad_v, or rho in MODE 0)
    const T *h0, *h1;       // the same rows of rho (MODE 1, 2)
    T w0, w1;               // 1 for rows inside the grid, 0 beyond
    T s0, s1;               // scale of rho, times w
    // the real grids are read once per pass: streaming (non-temporal) loads
    // leave the caches to the half spectrum that the next passes reuse
    static __device__ __forceinline__ T ld(const T *p) { return __builtin_nontemporal_load(p); }
    __device__ __forceinline__ Cx<T> load(int i) const
    {
        if constexpr (MODE == 0) return Cx<T>{w0 * ld(r0 + i), w1 * ld(r1 + i)};
        else if constexpr (MODE == 1)
            return Cx<T>{w0 * ld(r0 + i) + s0 * ld(h0 + i), w1 * ld(r1 + i) + s1 * ld(h1 + i)};
        else return Cx<T>{s0 * ld(h0 + i), s1 * ld(h1 + i)};
    }
    // element u + t, u uniform: where the rows are the same for the whole
    // wavefront (a pencil per wavefront) the row pointers plus u stay in
    // scalar registers and t becomes a fixed 32-bit byte offset
    static __device__ __forceinline__ T ldu(const T *row, int u, int t)
    {
        return ld(reinterpret_cast<const T *>(reinterpret_cast<const char *>(row + u) + uint32_t(t) * uint32_t(sizeof(T))));
    }
    __device__ __forceinline__ Cx<T> load_at(int u, int t) const
    {
        if constexpr (MODE == 0) return Cx<T>{w0 * ldu(r0, u, t), w1 * ldu(r1, u, t)};
        else if constexpr (MODE == 1)
            return Cx<T>{w0 * ldu(r0, u, t) + s0 * ldu(h0, u, t), w1 * ldu(r1, u, t) + s1 * ldu(h1, u, t)};
        else return Cx<T>{s0 * ldu(h0, u, t), s1 * ldu(h1, u, t)};
    }
};

// P5 input: Z[i] = X[i] + i Y[i] from the half-spectrum rows of X and Y,
// with X[n - i] = conj X[i] beyond the stored half; the imaginary parts of
// the 0 and Nyquist bins are dropped (zero in exact arithmetic for the
// inverse of a Hermitian spectrum).  Conjugated: P5 runs the inverse.
template <typename T>
struct HermitianPairIn {
    static constexpr bool kLds = false;
    const Cx<T> *x0, *x1;   // rows beyond the grid point at a valid row
    int n, nh;
    T w0, w1;               // 1 inside the grid, 0 beyond
    __device__ __forceinline__ Cx<T> load(int i) const
    {
        const bool mirror = i >= nh;
        const int k = mirror ? n - i : i;
        Cx<T> xe = cscale(x0[k], w0);
        Cx<T> xo = cscale(x1[k], w1);
        if (mirror) {
            xe.y = -xe.y;
            xo.y = -xo.y;
        }
        if (i == 0 || 2 * i == n) {
            xe.y = T(0);
            xo.y = T(0);
        }
        return Cx<T>{xe.x - xo.y, -(xe.y + xo.x)};
    }
    __device__ __forceinline__ Cx<T> load_at(int u, int t) const { return load(u + t); }
};

// P5 output: the conjugate of the last stage's value is x + i y for the
// two real rows
template <typename T>
struct RealPairOut {
    static constexpr bool kLds = false;
    T *o0, *o1;
    bool v0, v1;
    __device__ __forceinline__ void store(int i, Cx<T> v) const
    {
        if (v0) __builtin_nontemporal_store(v.x, o0 + i);
        if (v1) __builtin_nontemporal_store(-v.y, o1 + i);
    }
    // element u + t, u uniform (see RealPairIn::load_at)
    __device__ __forceinline__ void store_at(int u, int t, Cx<T> v) const
    {
        const uint32_t off = uint32_t(t) * uint32_t(sizeof(T));
        if (v0) __builtin_nontemporal_store(v.x, reinterpret_cast<T *>(reinterpret_cast<char *>(o0 + u) + off));
        if (v1) __builtin_nontemporal_store(-v.y, reinterpret_cast<T *>(reinterpret_cast<char *>(o1 + u) + off));
    }
};

constexpr int kStageUnroll = 8;  // staging loads each thread keeps in flight

// Staged variants of the c-axis accessors (the multi-plan kernels of batched
// plans, whose short rows leave most lanes of a pencil idle in the first and
// last stages): a tile's rows are contiguous in the grid and in the half
// spectrum, so the workgroup moves them between global memory and an LDS
// block with every lane on consecutive elements, and the stages read and
// write that block.
// P1 input from the block: element i of rows 2q and 2q + 1
template <typename T>
struct LdsRealPairIn {
    static constexpr bool kLds = true;
    const T *r;  // row 2q of the block; row 2q + 1 follows at r + n
    int n;
    __device__ __forceinline__ Cx<T> load(int i) const { return Cx<T>{r[i], r[n + i]}; }
    __device__ __forceinline__ Cx<T> load_at(int u, int t) const { return load(u + t); }
};

// P5 output into the block: the conjugate of the last stage's value is
// x + i y for rows 2q and 2q + 1
template <typename T>
struct LdsRealPairOut {
    static constexpr bool kLds = false;
    T *o;  // row 2q of the block; row 2q + 1 follows at o + n
    int n;
    __device__ __forceinline__ void store(int i, Cx<T> v) const
    {
        o[i] = v.x;
        o[n + i] = -v.y;
    }
    __device__ __forceinline__ void store_at(int u, int t, Cx<T> v) const { store(u + t, v); }
};

// pencil-major tile pitch: n rounded so that consecutive pencils start in
// opposite halves of the LDS banks
__host__ __device__ constexpr int row_pitch(int n) { return n + ((16 - n % 32) + 32) % 32; }

// length of a compiled radix plan (0 for the run-time radix kernel)
constexpr int plan_length(int r0, int r1, int r2, int r3)
{
    return r0 == 0 ? 0 : r0 * (r1 > 0 ? r1 : 1) * (r2 > 0 ? r2 : 1) * (r3 > 0 ? r3 : 1);
}

// ---------------------------------------------------------------- P1
// MODE 0: x = rho.  MODE 1 (backward): x = grad_v + grad_e * dV * rho.
// MODE 2: x = grad_e * dV * rho.
// CP > 0 (passes along c; a compiled plan): tiles of exactly CP pencils
// (2 CP rows), launched only for that shape, with the pencil length (the
// plan's) compiled in as well, so tile offsets and loop bounds are constants.
// STAGE: the tile's rows are loaded into an LDS block after the twiddles
// first (2 P n reals; see LdsRealPairIn).
template <typename T, int MODE, int R0, int R1, int R2, int R3, int CP, bool STAGE = false>
__device__ __forceinline__ void r2c_tile(const PassArgs &a, int prob, int tile)
{
    constexpr int NT = kPassThreads;
    constexpr int NF = CP > 0 ? plan_length(R0, R1, R2, R3) : 0;
    const int P = CP > 0 ? CP : 1 << a.p_log2, TPP = NT / P;
    extern __shared__ __align__(16) unsigned char smem[];
    const ProbDesc &d = a.desc[prob];
    const int n = NF > 0 ? NF : d.dims[2], nh = NF > 0 ? NF / 2 + 1 : d.dims[3];
    const int ldp = row_pitch(n);
    const int64_t nrows = int64_t(d.dims[0]) * d.dims[1];
    const int64_t row0 = int64_t(tile) * 2 * P;
    const int rows = int((nrows - row0) < 2 * P ? (nrows - row0) : 2 * P);
    Cx<T> *buf = reinterpret_cast<Cx<T> *>(smem);
    Cx<T> *tw = buf + P * ldp;
    const int tid = threadIdx.x;
    load_twiddles(tw, reinterpret_cast<const Cx<T> *>(a.tw) + d.ax[2].tw_off, n, tid, NT);
    __syncthreads();

    // with 64 or more threads per pencil a wavefront holds one pencil: its
    // index is uniform and the row pointers stay in scalar registers
    const int q = (CP > 0 && NT / CP >= 64) ? __builtin_amdgcn_readfirstlane(tid / TPP) : tid / TPP;
    const int tip = tid & (TPP - 1);  // TPP is a power of two
    const bool v0 = 2 * q < rows, v1 = 2 * q + 1 < rows;
    const int64_t g_even = d.grid_off + (row0 + (v0 ? 2 * q : 0)) * n;
    const int64_t g_odd = d.grid_off + (row0 + (v1 ? 2 * q + 1 : 0)) * n;
    const T scale = MODE == 0 ? T(0) : T(a.grad_e[prob] * d.dv);
    const LdsRow<T> lr{buf, ldp, q, false};
    if constexpr (STAGE) {
        // the rows (zero beyond the grid) into the block, every lane on
        // consecutive reals
        T *blk = reinterpret_cast<T *>(tw + n);
        const int64_t g0 = d.grid_off + row0 * n;
        const T *x = reinterpret_cast<const T *>(a.in) + g0;
        const T *h = reinterpret_cast<const T *>(a.in2) + g0;
        // (kStageUnroll loads in flight per thread before their stores)
        const int cnt = rows * n, tot = 2 * P * n;
        for (int e0 = tid; e0 < tot; e0 += kStageUnroll * NT) {
            T v[kStageUnroll];
#pragma unroll
            for (int u = 0; u < kStageUnroll; ++u) {
                const int e = e0 + u * NT;
                v[u] = T(0);
                if (e < cnt) {
                    if constexpr (MODE == 0) v[u] = __builtin_nontemporal_load(x + e);
                    else if constexpr (MODE == 1)
                        v[u] = __builtin_nontemporal_load(x + e) + scale * __builtin_nontemporal_load(h + e);
                    else v[u] = scale * __builtin_nontemporal_load(h + e);
                }
            }
#pragma unroll
            for (int u = 0; u < kStageUnroll; ++u)
                if (e0 + u * NT < tot) blk[e0 + u * NT] = v[u];
        }
        __syncthreads();
        const LdsRealPairIn<T> in{blk + 2 * q * n, n};
        if (d.ax[2].nstages > 0) {
            LdsRow<T> out = lr;
            fft_any<T, R0, R1, R2, R3>(in, out, lr, tw, d.ax[2], tip, TPP);
        } else if (tip == 0) {
            lr.store(0, in.load(0));
        }
    } else {
        RealPairIn<T, MODE> in;
        in.r0 = reinterpret_cast<const T *>(a.in) + g_even;
        in.r1 = reinterpret_cast<const T *>(a.in) + g_odd;
        in.h0 = reinterpret_cast<const T *>(a.in2) + g_even;
        in.h1 = reinterpret_cast<const T *>(a.in2) + g_odd;
        in.w0 = v0 ? T(1) : T(0);
        in.w1 = v1 ? T(1) : T(0);
        in.s0 = scale * in.w0;
        in.s1 = scale * in.w1;
        if (d.ax[2].nstages > 0) {
            LdsRow<T> out = lr;
            fft_any<T, R0, R1, R2, R3>(in, out, lr, tw, d.ax[2], tip, TPP);
        } else if (tip == 0) {
            lr.store(0, in.load(0));
        }
    }
    __syncthreads();

    // X[k] = (Z[k] + conj Z[n-k]) / 2,  Y[k] = (Z[k] - conj Z[n-k]) / (2i)
    Cx<T> *dst = reinterpret_cast<Cx<T> *>(a.spec) + d.spec_off + row0 * nh;
    const int totalh = rows * nh;
    for (int e = tid; e < totalh; e += NT) {
        const int row = NF > 0 ? e / nh : int(fdiv(uint32_t(e), d.div_nh));
        const int k = e - row * nh;
        const Cx<T> *z = buf + (row >> 1) * ldp;
        const Cx<T> A = z[k];
        const Cx<T> B = z[k == 0 ? 0 : n - k];
        Cx<T> X;
        if ((row & 1) == 0)
            X = {T(0.5) * (A.x + B.x), T(0.5) * (A.y - B.y)};
        else
            X = {T(0.5) * (A.y + B.y), T(0.5) * (B.x - A.x)};
        dst[e] = X;
    }
}

template <typename T, int MODE, int R0, int R1, int R2, int R3, int CP = 0>
__global__ __launch_bounds__(256) void k_r2c_mode(PassArgs a)
{
    int prob, tile;
    find_item(a.tl, xcd_remap(blockIdx.x, gridDim.x), prob, tile);
    r2c_tile<T, MODE, R0, R1, R2, R3, CP>(a, prob, tile);
}

// ---------------------------------------------------------------- P5
// CP > 0: as for P1
// STAGE: the tile's half-spectrum rows are loaded into an LDS block after
// the twiddles first (2 P nh complex), and the real rows are written there
// and then copied out (2 P n reals, in the same block; see LdsRealPairOut).
template <typename T, int R0, int R1, int R2, int R3, int CP, bool STAGE = false>
__device__ __forceinline__ void c2r_tile(const PassArgs &a, int prob, int tile)
{
    constexpr int NT = kPassThreads;
    constexpr int NF = CP > 0 ? plan_length(R0, R1, R2, R3) : 0;
    const int P = CP > 0 ? CP : 1 << a.p_log2, TPP = NT / P;
    extern __shared__ __align__(16) unsigned char smem[];
    const ProbDesc &d = a.desc[prob];
    const int n = NF > 0 ? NF : d.dims[2], nh = NF > 0 ? NF / 2 + 1 : d.dims[3];
    const int ldp = row_pitch(n);
    const int64_t nrows = int64_t(d.dims[0]) * d.dims[1];
    const int64_t row0 = int64_t(tile) * 2 * P;
    const int rows = int((nrows - row0) < 2 * P ? (nrows - row0) : 2 * P);
    Cx<T> *buf = reinterpret_cast<Cx<T> *>(smem);
    Cx<T> *tw = buf + P * ldp;
    const int tid = threadIdx.x;
    load_twiddles(tw, reinterpret_cast<const Cx<T> *>(a.tw) + d.ax[2].tw_off, n, tid, NT);
    __syncthreads();

    const int q = (CP > 0 && NT / CP >= 64) ? __builtin_amdgcn_readfirstlane(tid / TPP) : tid / TPP;
    const int tip = tid & (TPP - 1);  // TPP is a power of two
    const bool v0 = 2 * q < rows, v1 = 2 * q + 1 < rows;
    const Cx<T> *spec = reinterpret_cast<const Cx<T> *>(a.spec) + d.spec_off + row0 * nh;
    const LdsRow<T> lr{buf, ldp, q, false};
    if constexpr (STAGE) {
        Cx<T> *blk = tw + n;
        const int cnt = rows * nh, tot = 2 * P * nh;
        for (int e0 = tid; e0 < tot; e0 += kStageUnroll * NT) {
            Cx<T> v[kStageUnroll];
#pragma unroll
            for (int u = 0; u < kStageUnroll; ++u) {
                const int e = e0 + u * NT;
                v[u] = e < cnt ? spec[e] : Cx<T>{T(0), T(0)};
            }
#pragma unroll
            for (int u = 0; u < kStageUnroll; ++u)
                if (e0 + u * NT < tot) blk[e0 + u * NT] = v[u];
        }
        __syncthreads();
        HermitianPairIn<T> in;
        in.x0 = blk + 2 * q * nh;
        in.x1 = blk + (2 * q + 1) * nh;
        in.n = n;
        in.nh = nh;
        in.w0 = T(1);
        in.w1 = T(1);
        // the last stage writes the real rows over the block, whose reads
        // all precede the first stage's barrier
        const LdsRealPairOut<T> out{reinterpret_cast<T *>(blk) + 2 * q * n, n};
        if (d.ax[2].nstages > 0) {
            fft_any<T, R0, R1, R2, R3>(in, out, lr, tw, d.ax[2], tip, TPP);
        } else if (tip == 0) {
            out.store(0, in.load(0));
        }
        __syncthreads();
        const T *rb = reinterpret_cast<const T *>(blk);
        T *dst = reinterpret_cast<T *>(a.out) + d.grid_off + row0 * n;
        for (int e = tid; e < rows * n; e += NT) __builtin_nontemporal_store(rb[e], dst + e);
    } else {
        HermitianPairIn<T> in;
        in.x0 = spec + (v0 ? 2 * q : 0) * nh;
        in.x1 = spec + (v1 ? 2 * q + 1 : 0) * nh;
        in.n = n;
        in.nh = nh;
        in.w0 = v0 ? T(1) : T(0);
        in.w1 = v1 ? T(1) : T(0);
        RealPairOut<T> out;
        out.o0 = reinterpret_cast<T *>(a.out) + d.grid_off + (row0 + 2 * q) * n;
        out.o1 = out.o0 + n;
        out.v0 = v0;
        out.v1 = v1;
        if (d.ax[2].nstages > 0) {
            fft_any<T, R0, R1, R2, R3>(in, out, lr, tw, d.ax[2], tip, TPP);
        } else if (tip == 0) {
            out.store(0, in.load(0));
        }
    }
}

template <typename T, int R0, int R1, int R2, int R3, int CP = 0>
__global__ __launch_bounds__(256) void k_c2r(PassArgs a)
{
    int prob, tile;
    find_item(a.tl, xcd_remap(blockIdx.x, gridDim.x), prob, tile);
    c2r_tile<T, R0, R1, R2, R3, CP>(a, prob, tile);
}

// ---------------------------------------------------------------- P2 / P4
// pencils along b: (a, h) for fixed a, P consecutive h per tile; the first
// stage reads the tile from the spectrum and the last writes it back.
// CP > 0: tiles of exactly CP pencils with no pitch pad, compiled in (as for
// the a pass).
template <typename T, int R0, int R1, int R2, int R3, int CP>
__device__ __forceinline__ void fft_b_tile(const PassArgs &a, int prob, int tile)
{
    constexpr int NT = kPassThreads;
    const int P = CP > 0 ? CP : 1 << a.p_log2;
    const int TPP = NT / P;
    const int PP = CP > 0 ? CP : P + a.pad;
    extern __shared__ __align__(16) unsigned char smem[];
    const ProbDesc &d = a.desc[prob];
    const int n = d.dims[1], nh = d.dims[3];
    if (d.ax[1].nstages == 0) return;  // a length-1 axis: identity
    const int tpo = (nh + P - 1) / P;
    const int outer = tile / tpo;
    const int h0 = (tile - outer * tpo) * P;
    const int valid = (nh - h0) < P ? (nh - h0) : P;
    Cx<T> *buf = reinterpret_cast<Cx<T> *>(smem);
    Cx<T> *tw = buf + n * PP;
    const int tid = threadIdx.x;
    load_twiddles(tw, reinterpret_cast<const Cx<T> *>(a.tw) + d.ax[1].tw_off, n, tid, NT);
    __syncthreads();
    const int p = tid & (P - 1), tip = CP > 0 ? tid / CP : tid >> a.p_log2;
    Cx<T> *g = reinterpret_cast<Cx<T> *>(a.spec) + d.spec_off + int64_t(outer) * n * nh + h0;
    GlobalPencil<T, (CP > 0)> gp{g, nh, tip * nh + (p < valid ? p : 0), p < valid, a.inv != 0};
    const LdsPencil<T> lp{buf, PP, p, false};
    fft_any<T, R0, R1, R2, R3>(gp, gp, lp, tw, d.ax[1], tip, TPP);
}

template <typename T, int R0, int R1, int R2, int R3, int CP = 0>
__global__ __launch_bounds__(256) void k_fft_b(PassArgs a)
{
    int prob, tile;
    find_item(a.tl, xcd_remap(blockIdx.x, gridDim.x), prob, tile);
    fft_b_tile<T, R0, R1, R2, R3, CP>(a, prob, tile);
}

// ---------------------------------------------------------------- P3
// K for one spectral index; the signed index of an axis is m (2m < N), m - N
// (2m > N), and at the Nyquist index of an even axis both +N/2 and -N/2 are
// averaged (no effect on an orthorhombic cell, where |G|^2 is even per axis).
template <typename T>
__device__ __forceinline__ T kernel_value(const ProbDesc &d, int ma, int mb, int mc)
{
    const int Na = d.dims[0], Nb = d.dims[1], Nc = d.dims[2];
    const T *B = nullptr;
    if constexpr (sizeof(T) == 4) B = reinterpret_cast<const T *>(d.Bf);
    else B = reinterpret_cast<const T *>(d.B);
    const int sa = (2 * ma < Na) ? ma : ma - Na;
    const int sb = (2 * mb < Nb) ? mb : mb - Nb;
    const int sc = mc;
    const bool nyq = !d.ortho && ((2 * ma == Na) || (2 * mb == Nb) || (2 * mc == Nc));
    const T fourpi = T(12.566370614359172953850573533118);
    if (!nyq) {
        const T ga = T(sa), gb = T(sb), gc = T(sc);
        const T gx = ga * B[0] + gb * B[3] + gc * B[6];
        const T gy = ga * B[1] + gb * B[4] + gc * B[7];
        const T gz = ga * B[2] + gb * B[5] + gc * B[8];
        const T g2 = gx * gx + gy * gy + gz * gz;
        return (g2 > T(0)) ? fourpi / g2 : T(0);
    }
    // average over the aliases of each Nyquist axis
    const int na = (2 * ma == Na) ? 2 : 1, nb = (2 * mb == Nb) ? 2 : 1, nc = (2 * mc == Nc) ? 2 : 1;
    T sum = T(0);
    for (int i = 0; i < na; ++i)
        for (int j = 0; j < nb; ++j)
            for (int k = 0; k < nc; ++k) {
                const T ga = T(i ? -sa : sa), gb = T(j ? -sb : sb), gc = T(k ? -sc : sc);
                const T gx = ga * B[0] + gb * B[3] + gc * B[6];
                const T gy = ga * B[1] + gb * B[4] + gc * B[7];
                const T gz = ga * B[2] + gb * B[5] + gc * B[8];
                const T g2 = gx * gx + gy * gy + gz * gz;
                sum += (g2 > T(0)) ? fourpi / g2 : T(0);
            }
    return sum / T(na * nb * nc);
}

// kernel_value out of line: the Nyquist cells of a non-orthorhombic cell are
// rare, and inlining their alias loop into every store of the last stage
// would multiply the kernel's code size
template <typename T>
__device__ __noinline__ T kernel_value_rare(const ProbDesc &d, int ma, int mb, int mc)
{
    return kernel_value<T>(d, ma, mb, mc);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// Destination of the last forward stage along a: element m_a of the thread's
// column is multiplied by K(G)/N on its way into the LDS tile, and (energy)
// w(m_c) K |X|^2 is accumulated in double.  With G = s_a b_a + g, where
// g = m_b b_b + m_c b_c is the column's share, |G|^2 is the quadratic
// s_a^2 |b_a|^2 + s_a (2 b_a . g) + |g|^2 whose three coefficients are formed
// once per thread (for an orthorhombic cell the middle one is exactly 0);
// cells where the Nyquist average applies take the general path of
// kernel_value.
template <typename T>
struct KernelMultiply {
    static constexpr bool kLds = true;
    static constexpr bool kTail = true;
    Cx<T> *buf;
    int pp, p;
    const ProbDesc *d;
    int mb, mc;
    bool energy;      // wavefront-uniform: accumulate the E_H partial
    T invn;
    double wgt;       // w(m_c), and 0 for a pencil beyond the tile edge
    double acc;
    int na;
    bool ortho;       // wavefront-uniform: a diagonal cell (no Nyquist average, q1 = 0)
    bool general;     // a Nyquist b or c index of a non-orthorhombic cell
    T q2, q1, q0;     // |G|^2 = (q2 s_a + q1) s_a + q0
    T fe;             // K |X|^2 summed over the current butterfly's outputs
    __device__ __forceinline__ void init()
    {
        fe = T(0);
        const T *B = nullptr;
        if constexpr (sizeof(T) == 4) B = reinterpret_cast<const T *>(d->Bf);
        else B = reinterpret_cast<const T *>(d->B);
        const int Nb = d->dims[1], Nc = d->dims[2];
        na = d->dims[0];
        ortho = d->ortho != 0;
        general = !ortho && (2 * mb == Nb || 2 * mc == Nc);
        const T sb = T((2 * mb < Nb) ? mb : mb - Nb), sc = T(mc);
        q2 = q1 = q0 = T(0);
        for (int x = 0; x < 3; ++x) {
            const T g = sb * B[3 + x] + sc * B[6 + x];
            q2 += B[x] * B[x];
            q1 += T(2) * B[x] * g;
            q0 += g * g;
        }
    }
    __device__ __forceinline__ void store(int i, Cx<T> v)
    {
        T K;
        if (ortho) {
            // a diagonal cell: b_a is orthogonal to b_b and b_c, so q1 = 0
            // and no index needs the Nyquist average
            const T sa = T((2 * i < na) ? i : i - na);
            const T g2 = q2 * sa * sa + q0;
            K = (g2 > T(0)) ? T(12.566370614359172953850573533118) * recip(g2) : T(0);
        } else if (general || 2 * i == na) {
            K = kernel_value_rare<T>(*d, i, mb, mc);
        } else {
            const T sa = T((2 * i < na) ? i : i - na);
            const T g2 = (q2 * sa + q1) * sa + q0;
            K = (g2 > T(0)) ? T(12.566370614359172953850573533118) * recip(g2) : T(0);
        }
        if (energy) acc += wgt * double(K * (v.x * v.x + v.y * v.y));
        buf[i * pp + p] = cscale(v, K * invn);
    }
    __device__ __forceinline__ void store_at(int u, int t, Cx<T> v) { store(u + t, v); }
    // The same for the outputs of the last compiled stage: element
    // i = base + lo with 0 <= base < ns, where lo, ns and the length n are
    // constants once the stage loop is unrolled.  s_a then needs no
    // per-element select where the whole run [lo, lo + ns) lies in one half
    // of the range, and in a diagonal cell only i = 0 can have G = 0.  The
    // energy terms of one butterfly are summed in the working precision and
    // added to the FP64 partial by end_butterfly.
    __device__ __forceinline__ void store_tail(int base, int lo, int ns, int n, Cx<T> v)
    {
        const int i = base + lo;
        T sa;
        if (2 * (lo + ns - 1) < n) sa = T(base) + T(lo);
        else if (2 * lo >= n) sa = T(base) + T(lo - n);
        else sa = T((2 * i < n) ? i : i - n);
        T K;
        if (ortho) {
            const T g2 = q2 * sa * sa + q0;
            K = T(12.566370614359172953850573533118) * recip(g2);
            if (lo == 0) K = (g2 > T(0)) ? K : T(0);
        } else if (general || 2 * i == na) {
            K = kernel_value_rare<T>(*d, i, mb, mc);
        } else {
            const T g2 = (q2 * sa + q1) * sa + q0;
            K = (g2 > T(0)) ? T(12.566370614359172953850573533118) * recip(g2) : T(0);
        }
        if (energy) fe += K * (v.x * v.x + v.y * v.y);
        buf[i * pp + p] = cscale(v, K * invn);
    }
    __device__ __forceinline__ void end_butterfly()
    {
        if (energy) {
            acc += wgt * double(fe);
            fe = T(0);
        }
    }
};

// mode 0: forward, energy, multiply, inverse.  mode 1: no energy.
// mode 2: forward and energy only (no potential).
// pencils along a: column (b, h) of the flattened [Nb][Nh] plane.
// CP > 0: a tile of exactly CP pencils with no pitch pad (the host launches
// it only for that shape), so the tile pitch and the threads per pencil are
// compile-time constants: LDS offsets become immediates and the per-stage
// bounds checks fold away.
template <typename T, int R0, int R1, int R2, int R3, int CP>
__device__ __forceinline__ void fft_a_tile(const PassArgs &a, int prob, int tile)
{
    constexpr int NT = kPassThreads;
    const int P = CP > 0 ? CP : 1 << a.p_log2;
    const int TPP = NT / P;
    const int PP = CP > 0 ? CP : P + a.pad;
    const int mode = a.mode;
    const bool energy = mode != 1;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[NT / 64];
    const ProbDesc &d = a.desc[prob];
    const int n = d.dims[0], nh = d.dims[3], Nc = d.dims[2];
    const int ncol = d.dims[1] * nh;
    const int col0 = tile * P;
    const int valid = (ncol - col0) < P ? (ncol - col0) : P;
    Cx<T> *buf = reinterpret_cast<Cx<T> *>(smem);
    Cx<T> *tw = buf + n * PP;
    const int tid = threadIdx.x;
    load_twiddles(tw, reinterpret_cast<const Cx<T> *>(a.tw) + d.ax[0].tw_off, n, tid, NT);
    __syncthreads();
    const int p = tid & (P - 1), tip = CP > 0 ? tid / CP : tid >> a.p_log2;
    const int col = col0 + (p < valid ? p : 0);
    const int mb = int(fdiv(uint32_t(col), d.div_nh));
    const int mc = col - mb * nh;
    Cx<T> *g = reinterpret_cast<Cx<T> *>(a.spec) + d.spec_off + col0;
    const int lane = tip * ncol + (p < valid ? p : 0);
    GlobalPencil<T, (CP > 0), true> gp{g, ncol, lane, p < valid, false};
    const LdsPencil<T> lp{buf, PP, p, false};
    KernelMultiply<T> km{buf, PP, p, &d, mb, mc, energy, T(d.inv_n),
                         p < valid ? ((mc == 0 || 2 * mc == Nc) ? 1.0 : 2.0) : 0.0, 0.0};
    km.init();
    if (d.ax[0].nstages == 0) {
        // length-1 axis: the multiply alone
        if (tip == 0) km.store(0, gp.load_at(0, 0));
    } else {
        fft_any<T, R0, R1, R2, R3>(gp, km, lp, tw, d.ax[0], tip, TPP);
    }
    __syncthreads();
    if (energy) {
        const double acc = wave_sum(km.acc);
        if ((tid & 63) == 0) red[tid >> 6] = acc;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int w = 0; w < NT / 64; ++w) s += red[w];
            a.partials[d.part_off + tile] = s;
        }
    }
    if (mode == 2) return;
    // inverse along a
    if (d.ax[0].nstages == 0) {
        if (tip == 0) gp.store_at(0, 0, lp.load(0));
    } else if constexpr (R0 > 0) {
        // a compiled plan: the inverse stages themselves
        fft_static<T, R0, R1, R2, R3, true>(lp, gp, lp, tw, d.ax[0], tip, TPP);
    } else {
        // run-time radices: the forward stages, conjugating on the way in
        // and on the way out
        const LdsPencil<T> lpc{buf, PP, p, true};
        GlobalPencil<T, (CP > 0), true> gpc{g, ncol, lane, p < valid, true};
        fft_any<T, R0, R1, R2, R3>(lpc, gpc, lp, tw, d.ax[0], tip, TPP);
    }
}

template <typename T, int R0, int R1, int R2, int R3, int CP = 0>
__global__ __launch_bounds__(256) void k_fft_a(PassArgs a)
{
    int prob, tile;
    find_item(a.tl, xcd_remap(blockIdx.x, gridDim.x), prob, tile);
    fft_a_tile<T, R0, R1, R2, R3, CP>(a, prob, tile);
}

// ----------------------------------------------------- multi-plan launches
// A batched plan runs each pass as one launch per (radix plan, tile shape)
// group.  When every problem's pencils along the pass axis have a compiled
// plan of the axis' multi-plan list (one per length from 32 to 240) and one
// common tile width CP, the host instead makes one launch of these kernels:
// each workgroup runs the plan recorded in its problem's axis descriptor.
// The resources of such a kernel are the largest over its plans (256 =
// 16 x 16 is left out: its two radix-16 stages need a third more registers
// than any of these, which would cost every plan occupancy).
constexpr bool multi_list_ok(const int *list)
{
    int prev = 0;
    for (int k = 0; k < kMultiPlans; ++k) {
        const int *r = kPlanRadix[list[k]];
        const int n = plan_length(r[0], r[1], r[2], r[3]);
        if (n <= prev || n > 240) return false;
        prev = n;
    }
    return true;
}
static_assert(multi_list_ok(kMultiPlansAB) && multi_list_ok(kMultiPlansC),
              "each multi-plan list has one plan per length, ascending, up to 240");

// whether every stage of a plan fits its registers with tpp threads per
// pencil (what the host checks for every configuration it accepts)
constexpr bool plan_fits(const int *r, int tpp)
{
    int n = 1;
    for (int s = 0; s < 4; ++s) n *= r[s] > 0 ? r[s] : 1;
    for (int s = 0; s < 4; ++s)
        if (r[s] > 0 && (n / r[s] + tpp - 1) / tpp > stage_maxb<float>(r[s])) return false;
    return true;
}
constexpr bool multi_auto_ok(const int *list, int x)
{
    for (int k = 0; k < kMultiPlans; ++k) {
        const int *r = kPlanRadix[list[k]];
        if (!plan_fits(r, kPassThreads / multi_auto_p(plan_length(r[0], r[1], r[2], r[3]), x))) return false;
    }
    return true;
}
static_assert(multi_auto_ok(kMultiPlansAB, 0) && multi_auto_ok(kMultiPlansC, 2),
              "the size-adapted tiles leave every listed plan enough threads per pencil");

// the tile width of plan entry E in a multi-plan kernel of width W (0: sized
// per length) along axis x
template <int W, int E, int X>
constexpr int multi_cp()
{
    return W > 0 ? W : multi_auto_p(plan_length(kPlanRadix[E][0], kPlanRadix[E][1], kPlanRadix[E][2],
                                                 kPlanRadix[E][3]), X);
}

// f(integral_constant<E>) for the entry E == plan of the list (none if the
// plan is not in it)
template <const int *LIST, int K = 0, typename F>
__device__ __forceinline__ void with_multi_plan(int plan, F &&f)
{
    if constexpr (K < kMultiPlans) {
        if (plan == LIST[K]) f(std::integral_constant<int, LIST[K]>());
        else with_multi_plan<LIST, K + 1>(plan, f);
    }
}

#define HARTREE_RADICES(I) kPlanRadix[I][0], kPlanRadix[I][1], kPlanRadix[I][2], kPlanRadix[I][3]

template <typename T, int MODE, int CP>
__global__ __launch_bounds__(256) void k_r2c_multi(PassArgs a)
{
    int prob, tile;
    find_item(a.tl, xcd_remap(blockIdx.x, gridDim.x), prob, tile);
    with_multi_plan<kMultiPlansC>(a.desc[prob].ax[2].cplan, [&](auto ic) {
        r2c_tile<T, MODE, HARTREE_RADICES(decltype(ic)::value), multi_cp<CP, decltype(ic)::value, 2>()>(a, prob, tile);
    });
}

template <typename T, int CP>
__global__ __launch_bounds__(256) void k_c2r_multi(PassArgs a)
{
    int prob, tile;
    find_item(a.tl, xcd_remap(blockIdx.x, gridDim.x), prob, tile);
    with_multi_plan<kMultiPlansC>(a.desc[prob].ax[2].cplan, [&](auto ic) {
        c2r_tile<T, HARTREE_RADICES(decltype(ic)::value), multi_cp<CP, decltype(ic)::value, 2>(), true>(a, prob, tile);
    });
}

template <typename T, int CP>
__global__ __launch_bounds__(256) void k_fft_b_multi(PassArgs a)
{
    int prob, tile;
    find_item(a.tl, xcd_remap(blockIdx.x, gridDim.x), prob, tile);
    with_multi_plan<kMultiPlansAB>(a.desc[prob].ax[1].cplan, [&](auto ic) {
        fft_b_tile<T, HARTREE_RADICES(decltype(ic)::value), multi_cp<CP, decltype(ic)::value, 1>()>(a, prob, tile);
    });
}

template <typename T, int CP>
__global__ __launch_bounds__(256) void k_fft_a_multi(PassArgs a)
{
    int prob, tile;
    find_item(a.tl, xcd_remap(blockIdx.x, gridDim.x), prob, tile);
    with_multi_plan<kMultiPlansAB>(a.desc[prob].ax[0].cplan, [&](auto ic) {
        fft_a_tile<T, HARTREE_RADICES(decltype(ic)::value), multi_cp<CP, decltype(ic)::value, 0>()>(a, prob, tile);
    });
}

#undef HARTREE_RADICES

// ------------------------------------------------------------- launchers

// A kernel that needs more than 64 KiB of dynamic LDS is opted in once per
// kernel (to the largest size asked so far), so that repeated launches, for
// instance under stream capture, make no attribute calls.
inline hipError_t lds_opt_in(const void *kern, size_t lds)
{
    static std::mutex mu;
    static std::map<const void *, size_t> granted;
    std::lock_guard<std::mutex> lock(mu);
    size_t &g = granted[kern];
    if (g >= lds) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e == hipSuccess) g = lds;
    return e;
}

template <typename F>
static hipError_t launch_pass(F kern, int grid, size_t lds, hipStream_t s, const PassArgs &a)
{
    if (grid <= 0) return hipSuccess;
    if (lds > 65536) {
        hipError_t e = lds_opt_in(reinterpret_cast<const void *>(kern), lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), lds, s, a);
    return hipGetLastError();
}

// Strided tiles of compiled width keep each thread's offset from the tile's
// first pencil, tip * stride + column, as a 32-bit byte offset: true when that
// fits for every problem of the launch (the largest stride, tpp - 1 tips).
template <typename T>
inline bool lane_offsets_fit(const PassArgs &a)
{
    const int64_t P = int64_t(1) << a.p_log2, tpp = kPassThreads / P;
    return ((tpp - 1) * a.col_stride + P) * int64_t(sizeof(Cx<T>)) < (int64_t(1) << 32);
}

// A launcher runs plan < 0 through the run-time radix kernel and otherwise
// entry `plan` of HARTREE_PLANS.  The LDS holds the tile and its twiddle
// table: n (P + pad) + n complex values.
typedef hipError_t (*PassLaunchFn)(int grid, size_t lds, hipStream_t s, const PassArgs &a);

template <typename T>
inline size_t pass_lds_bytes(const PassArgs &a, int maxn)
{
    // strided tiles n (P + pad); pencil-major tiles P row_pitch(n) <= P (n + 31)
    const size_t P = size_t(1) << a.p_log2;
    const size_t strided = (P + size_t(a.pad)) * maxn, rows = P * (maxn + 31);
    return sizeof(Cx<T>) * ((strided > rows ? strided : rows) + maxn);
}

// LDS of a size-adapted multi-plan launch along axis x whose longest pencil
// is maxn: the largest tile (and twiddle table) over the listed plans up to
// that length, n P (strided axes) or P row_pitch(n) (axis c)
// LDS block of the staged c-axis tiles: 2 P (n / 2 + 1) complex, which also
// holds the 2 P n reals of the c2r output
template <typename T>
inline size_t stage_lds(int P, int n)
{
    return sizeof(Cx<T>) * size_t(2 * P) * size_t(n / 2 + 1);
}

template <typename T>
inline size_t multi_auto_lds(int x, int maxn, bool staged = false)
{
    size_t most = 0;
    for (int k = 0; k < kMultiPlans; ++k) {
        const int *r = kPlanRadix[multi_plans(x)[k]];
        const int n = plan_length(r[0], r[1], r[2], r[3]);
        if (n > maxn) continue;
        const size_t P = size_t(multi_auto_p(n, x));
        const size_t e = sizeof(Cx<T>) * ((x == 2 ? P * size_t(row_pitch(n)) : P * size_t(n)) + size_t(n)) +
                         (staged ? stage_lds<T>(int(P), n) : 0);
        most = e > most ? e : most;
    }
    return most;
}

}  // namespace hartree
