// The five grid passes of the Hartree solve and the E_H finalize.
//
// Layouts: the real grid is [Na][Nb][Nc] (c fastest); the half spectrum kept
// in the workspace is [Na][Nb][Nh], Nh = Nc/2 + 1, and is transformed in
// place.  The passes follow the calculation flow of Sec. 3.2.4 (abc -> cab ->
// cba -> cab -> abc): on one GPU each change of "local axis" becomes a pass
// that streams the grid through LDS once, transforming pencils along that
// axis.
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
#include "fft_core.hpp"
#include "kernels.hpp"

namespace hartree {

// Pencils per workgroup (P) and threads per pencil (TPP) per length class.
// P * TPP = 256 threads; the tile holds NMAX * P complex values (64 KB).
template <typename T, int NMAX>
struct TileCfg {
    static constexpr int bytes = int(sizeof(Cx<T>));
    static constexpr int P = (65536 / bytes / NMAX) < 64 ? (65536 / bytes / NMAX) : 64;
    static constexpr int TPP = 256 / P;
    static constexpr int NT = P * TPP;
};

__device__ __forceinline__ void find_item(const TileList &tl, int item, int &prob, int &tile)
{
    int i = 0;
    while (i + 1 < tl.count && item >= tl.start[i + 1]) ++i;
    prob = tl.prob[i];
    tile = item - tl.start[i];
}

template <typename T>
__device__ __forceinline__ void load_twiddles(Cx<T> *dst, const Cx<T> *src, int n, int tid, int nt)
{
    for (int i = tid; i < n; i += nt) dst[i] = src[i];
}

// ---------------------------------------------------------------- P1
// MODE 0: x = rho.  MODE 1 (backward): x = grad_v + grad_e * dV * rho.
template <typename T, int NMAX, int MODE>
__global__ __launch_bounds__(256) void k_r2c(PassArgs a)
{
    using C = TileCfg<T, NMAX>;
    constexpr int P = C::P, TPP = C::TPP, NT = C::NT;
    extern __shared__ __align__(16) unsigned char smem[];
    int prob, tile;
    find_item(a.tl, xcd_remap(blockIdx.x, gridDim.x), prob, tile);
    const ProbDesc &d = a.desc[prob];
    const int n = d.dims[2], nh = d.dims[3];
    const int64_t nrows = int64_t(d.dims[0]) * d.dims[1];
    const int64_t row0 = int64_t(tile) * 2 * P;
    const int rows = int((nrows - row0) < 2 * P ? (nrows - row0) : 2 * P);
    Cx<T> *buf = reinterpret_cast<Cx<T> *>(smem);
    Cx<T> *tw = buf + n * P;
    const int tid = threadIdx.x;
    load_twiddles(tw, reinterpret_cast<const Cx<T> *>(a.tw) + d.ax[2].tw_off, n, tid, NT);

    const int64_t g0 = d.grid_off + row0 * n;
    const T *src = reinterpret_cast<const T *>(a.in) + g0;
    const T *rho = reinterpret_cast<const T *>(a.in2) + g0;
    T scale = T(0);
    if (MODE == 1 && a.grad_e != nullptr) scale = T(a.grad_e[prob] * d.dv);
    const int total = rows * n;
    T *bufr = reinterpret_cast<T *>(buf);
    for (int e = tid; e < 2 * P * n; e += NT) {
        const int row = int(fdiv(uint32_t(e), d.div_nc));
        const int k = e - row * n;
        T v = T(0);
        if (e < total) {
            if (MODE == 0) {
                v = src[e];
            } else {
                if (a.in != nullptr) v = src[e];
                if (a.grad_e != nullptr) v += scale * rho[e];
            }
        }
        bufr[2 * (k * P + (row >> 1)) + (row & 1)] = v;
    }
    __syncthreads();
    const int p = tid % P, tip = tid / P;
    fft_tile<T, NMAX, P, TPP, false>(buf, tw, d.ax[2], p, tip);

    // Z = x + i y for rows 2q, 2q+1:  X[k] = (Z[k] + conj Z[n-k]) / 2,
    // Y[k] = (Z[k] - conj Z[n-k]) / (2i)
    Cx<T> *dst = reinterpret_cast<Cx<T> *>(a.spec) + d.spec_off + row0 * nh;
    const int totalh = rows * nh;
    for (int e = tid; e < totalh; e += NT) {
        const int row = int(fdiv(uint32_t(e), d.div_nh));
        const int k = e - row * nh;
        const int q = row >> 1;
        const Cx<T> A = buf[k * P + q];
        const Cx<T> B = buf[(k == 0 ? 0 : n - k) * P + q];
        Cx<T> X;
        if ((row & 1) == 0)
            X = {T(0.5) * (A.x + B.x), T(0.5) * (A.y - B.y)};
        else
            X = {T(0.5) * (A.y + B.y), T(0.5) * (B.x - A.x)};
        dst[e] = X;
    }
}

// ---------------------------------------------------------------- P5
template <typename T, int NMAX>
__global__ __launch_bounds__(256) void k_c2r(PassArgs a)
{
    using C = TileCfg<T, NMAX>;
    constexpr int P = C::P, TPP = C::TPP, NT = C::NT;
    constexpr int ZPT = cdiv(NMAX * P, NT);
    extern __shared__ __align__(16) unsigned char smem[];
    int prob, tile;
    find_item(a.tl, xcd_remap(blockIdx.x, gridDim.x), prob, tile);
    const ProbDesc &d = a.desc[prob];
    const int n = d.dims[2], nh = d.dims[3];
    const int64_t nrows = int64_t(d.dims[0]) * d.dims[1];
    const int64_t row0 = int64_t(tile) * 2 * P;
    const int rows = int((nrows - row0) < 2 * P ? (nrows - row0) : 2 * P);
    Cx<T> *buf = reinterpret_cast<Cx<T> *>(smem);
    Cx<T> *tw = buf + P * (n + 2);
    const int tid = threadIdx.x;
    load_twiddles(tw, reinterpret_cast<const Cx<T> *>(a.tw) + d.ax[2].tw_off, n, tid, NT);

    // raw rows [2P][nh]
    const Cx<T> *src = reinterpret_cast<const Cx<T> *>(a.spec) + d.spec_off + row0 * nh;
    const int totalh = rows * nh;
    for (int e = tid; e < 2 * P * nh; e += NT) buf[e] = (e < totalh) ? src[e] : Cx<T>{T(0), T(0)};
    __syncthreads();

    // Z[k] = X[k] + i Y[k] over the full length, using X[n-k] = conj X[k];
    // the imaginary parts of the k = 0 and Nyquist bins are dropped (they
    // vanish in exact arithmetic: the inverse of a Hermitian spectrum is real)
    Cx<T> z[ZPT];
#pragma unroll
    for (int i = 0; i < ZPT; ++i) {
        const int e = tid + i * NT;
        if (e < n * P) {
            const int k = e / P, q = e % P;
            Cx<T> xe, xo;
            if (k < nh) {
                xe = buf[(2 * q) * nh + k];
                xo = buf[(2 * q + 1) * nh + k];
            } else {
                xe = buf[(2 * q) * nh + (n - k)];
                xo = buf[(2 * q + 1) * nh + (n - k)];
                xe.y = -xe.y;
                xo.y = -xo.y;
            }
            if (k == 0 || 2 * k == n) {
                xe.y = T(0);
                xo.y = T(0);
            }
            z[i] = {xe.x - xo.y, xe.y + xo.x};
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ZPT; ++i) {
        const int e = tid + i * NT;
        if (e < n * P) buf[e] = z[i];
    }
    __syncthreads();
    const int p = tid % P, tip = tid / P;
    fft_tile<T, NMAX, P, TPP, true>(buf, tw, d.ax[2], p, tip);

    T *dst = reinterpret_cast<T *>(a.out) + d.grid_off + row0 * n;
    const T *bufr = reinterpret_cast<const T *>(buf);
    const int total = rows * n;
    for (int e = tid; e < total; e += NT) {
        const int row = int(fdiv(uint32_t(e), d.div_nc));
        const int k = e - row * n;
        dst[e] = bufr[2 * (k * P + (row >> 1)) + (row & 1)];
    }
}

// ---------------------------------------------------------------- P2 / P4
// pencils along b: (a, h) for fixed a, P consecutive h per tile
template <typename T, int NMAX, bool INV>
__global__ __launch_bounds__(256) void k_fft_b(PassArgs a)
{
    using C = TileCfg<T, NMAX>;
    constexpr int P = C::P, TPP = C::TPP, NT = C::NT;
    extern __shared__ __align__(16) unsigned char smem[];
    int prob, tile;
    find_item(a.tl, xcd_remap(blockIdx.x, gridDim.x), prob, tile);
    const ProbDesc &d = a.desc[prob];
    const int n = d.dims[1], nh = d.dims[3];
    const int tpo = (nh + P - 1) / P;
    const int outer = tile / tpo;
    const int h0 = (tile - outer * tpo) * P;
    const int valid = (nh - h0) < P ? (nh - h0) : P;
    Cx<T> *buf = reinterpret_cast<Cx<T> *>(smem);
    Cx<T> *tw = buf + n * P;
    const int tid = threadIdx.x;
    load_twiddles(tw, reinterpret_cast<const Cx<T> *>(a.tw) + d.ax[1].tw_off, n, tid, NT);

    Cx<T> *g = reinterpret_cast<Cx<T> *>(a.spec) + d.spec_off + int64_t(outer) * n * nh + h0;
    for (int e = tid; e < n * P; e += NT) {
        const int row = e / P, p = e % P;
        buf[e] = (p < valid) ? g[int64_t(row) * nh + p] : Cx<T>{T(0), T(0)};
    }
    __syncthreads();
    const int p = tid % P, tip = tid / P;
    fft_tile<T, NMAX, P, TPP, INV>(buf, tw, d.ax[1], p, tip);
    for (int e = tid; e < n * P; e += NT) {
        const int row = e / P, pp = e % P;
        if (pp < valid) g[int64_t(row) * nh + pp] = buf[e];
    }
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

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// MODE 0: forward, energy, multiply, inverse.  MODE 1: no energy.
// MODE 2: forward and energy only (no potential).
// pencils along a: column (b, h) of the flattened [Nb][Nh] plane
template <typename T, int NMAX, int MODE>
__global__ __launch_bounds__(256) void k_fft_a(PassArgs a)
{
    using C = TileCfg<T, NMAX>;
    constexpr int P = C::P, TPP = C::TPP, NT = C::NT;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[NT / 64];
    int prob, tile;
    find_item(a.tl, xcd_remap(blockIdx.x, gridDim.x), prob, tile);
    const ProbDesc &d = a.desc[prob];
    const int n = d.dims[0], nh = d.dims[3], Nc = d.dims[2];
    const int ncol = d.dims[1] * nh;
    const int col0 = tile * P;
    const int valid = (ncol - col0) < P ? (ncol - col0) : P;
    Cx<T> *buf = reinterpret_cast<Cx<T> *>(smem);
    Cx<T> *tw = buf + n * P;
    const int tid = threadIdx.x;
    load_twiddles(tw, reinterpret_cast<const Cx<T> *>(a.tw) + d.ax[0].tw_off, n, tid, NT);

    Cx<T> *g = reinterpret_cast<Cx<T> *>(a.spec) + d.spec_off + col0;
    const int64_t stride = ncol;
    for (int e = tid; e < n * P; e += NT) {
        const int row = e / P, p = e % P;
        buf[e] = (p < valid) ? g[int64_t(row) * stride + p] : Cx<T>{T(0), T(0)};
    }
    __syncthreads();
    const int p = tid % P, tip = tid / P;
    fft_tile<T, NMAX, P, TPP, false>(buf, tw, d.ax[0], p, tip);

    double acc = 0.0;
    const T invn = T(d.inv_n);
    for (int e = tid; e < n * P; e += NT) {
        const int ma = e / P, pp = e % P;
        if (pp < valid) {
            const int col = col0 + pp;
            const int mb = int(fdiv(uint32_t(col), d.div_nh));
            const int mc = col - mb * nh;
            const T K = kernel_value<T>(d, ma, mb, mc);
            const Cx<T> X = buf[e];
            if (MODE != 1) {
                const double wgt = (mc == 0 || 2 * mc == Nc) ? 1.0 : 2.0;
                acc += wgt * double(K * (X.x * X.x + X.y * X.y));
            }
            if (MODE != 2) buf[e] = cscale(X, K * invn);
        }
    }
    if (MODE != 1) {
        acc = wave_sum(acc);
        if ((tid & 63) == 0) red[tid >> 6] = acc;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int w = 0; w < NT / 64; ++w) s += red[w];
            a.partials[d.part_off + tile] = s;
        }
    }
    if (MODE == 2) return;
    __syncthreads();
    fft_tile<T, NMAX, P, TPP, true>(buf, tw, d.ax[0], p, tip);
    for (int e = tid; e < n * P; e += NT) {
        const int row = e / P, pp = e % P;
        if (pp < valid) g[int64_t(row) * stride + pp] = buf[e];
    }
}

// ---------------------------------------------------------------- E_H
// one workgroup per problem: fixed-order sum of that problem's partials
__global__ __launch_bounds__(256) void k_finalize(const ProbDesc *desc, const double *partials, double *e_h)
{
    __shared__ double red[256];
    const ProbDesc &d = desc[blockIdx.x];
    double s = 0.0;
    for (int i = threadIdx.x; i < d.nparts; i += 256) s += partials[d.part_off + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) e_h[blockIdx.x] = d.eh_scale * red[0];
}

// ------------------------------------------------------------- host side

template <typename T>
static int tile_p(int nmax)
{
    switch (nmax) {
    case 64: return TileCfg<T, 64>::P;
    case 128: return TileCfg<T, 128>::P;
    case 256: return TileCfg<T, 256>::P;
    case 512: return TileCfg<T, 512>::P;
    case 1024: return TileCfg<T, 1024>::P;
    case 2048: return TileCfg<T, 2048>::P;
    default: return TileCfg<T, 4096>::P;
    }
}

int pass_pencils(int fp64, int nmax) { return fp64 ? tile_p<double>(nmax) : tile_p<float>(nmax); }

int length_class(int n)
{
    int c = 64;
    while (c < n) c <<= 1;
    return c;
}

#define HARTREE_NMAX_SWITCH(nmax, ...)           \
    switch (nmax) {                              \
    case 64: { constexpr int NM = 64; __VA_ARGS__; } break;     \
    case 128: { constexpr int NM = 128; __VA_ARGS__; } break;   \
    case 256: { constexpr int NM = 256; __VA_ARGS__; } break;   \
    case 512: { constexpr int NM = 512; __VA_ARGS__; } break;   \
    case 1024: { constexpr int NM = 1024; __VA_ARGS__; } break; \
    case 2048: { constexpr int NM = 2048; __VA_ARGS__; } break; \
    default: { constexpr int NM = 4096; __VA_ARGS__; } break;   \
    }

template <typename F>
static hipError_t launch(F kern, int grid, size_t lds, hipStream_t s, const PassArgs &a)
{
    if (grid <= 0) return hipSuccess;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), lds, s, a);
    return hipGetLastError();
}

template <typename T>
static hipError_t run_pass_t(PassKind kind, int nmax, int maxn, int grid, hipStream_t s, const PassArgs &a)
{
    const size_t cx = sizeof(Cx<T>);
    hipError_t err = hipSuccess;
    HARTREE_NMAX_SWITCH(nmax, {
        constexpr int P = TileCfg<T, NM>::P;
        switch (kind) {
        case PASS_R2C_FWD:
            err = launch(k_r2c<T, NM, 0>, grid, cx * (size_t(P) * maxn + maxn), s, a);
            break;
        case PASS_R2C_BWD:
            err = launch(k_r2c<T, NM, 1>, grid, cx * (size_t(P) * maxn + maxn), s, a);
            break;
        case PASS_C2R:
            err = launch(k_c2r<T, NM>, grid, cx * (size_t(P) * (maxn + 2) + maxn), s, a);
            break;
        case PASS_B_FWD:
            err = launch(k_fft_b<T, NM, false>, grid, cx * (size_t(P) * maxn + maxn), s, a);
            break;
        case PASS_B_INV:
            err = launch(k_fft_b<T, NM, true>, grid, cx * (size_t(P) * maxn + maxn), s, a);
            break;
        case PASS_A_FULL:
            err = launch(k_fft_a<T, NM, 0>, grid, cx * (size_t(P) * maxn + maxn), s, a);
            break;
        case PASS_A_NOENERGY:
            err = launch(k_fft_a<T, NM, 1>, grid, cx * (size_t(P) * maxn + maxn), s, a);
            break;
        case PASS_A_ENERGY:
            err = launch(k_fft_a<T, NM, 2>, grid, cx * (size_t(P) * maxn + maxn), s, a);
            break;
        }
    });
    return err;
}

hipError_t run_pass(int fp64, PassKind kind, int nmax, int maxn, int grid, hipStream_t s, const PassArgs &a)
{
    return fp64 ? run_pass_t<double>(kind, nmax, maxn, grid, s, a) : run_pass_t<float>(kind, nmax, maxn, grid, s, a);
}

hipError_t run_finalize(const ProbDesc *desc, const double *partials, double *e_h, int nprob, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize, dim3(nprob), dim3(256), 0, s, desc, partials, e_h);
    return hipGetLastError();
}

}  // namespace hartree
