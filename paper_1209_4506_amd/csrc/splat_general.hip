// Splat and splat adjoint in any periodic cell (the vector-unit path for
// cells that are not diagonal; diagonal cells use the separable kernels).
//
// In a general cell a Gaussian is not a product of per-axis factors, so each
// (grid point, atom) pair is evaluated directly: the point's displacement
// from the atom's nearest image inside the atom's index window is
//   d = u_a a' + u_b b' + u_c c' - rb,   a' = a / Na, ...,
// with u_x the point's unwrapped offset from the window start lo_x and
// rb = R - sum_x (lo_x / N_x) x-th cell row (formed in double, small), and
// the contribution is w exp(-|d|^2 / (2 sigma^2)) inside the cutoff sphere
// |d| <= cutoff sigma (the truncation of the CPU reference as well).
//
// One workgroup per brick (the plan's brick size); atoms come from the same
// sorted per-brick lists as the separable kernels, staged in LDS in chunks.
#include "splat_common.hpp"

namespace hartree {

constexpr int kGenThreads = 256;
constexpr int kGenChunk = 64;
// points per brick: FP32 plans use kMI x kMJ x kMK bricks, FP64 plans kBI x kBJ x kBK
template <typename T>
constexpr int gen_max_points()
{
    return sizeof(T) == 4 ? kMI * kMJ * kMK : kBI * kBJ * kBK;
}

template <typename T>
struct StagedC {
    T rb[3], rbl[3];  // rb and its rounding remainder (FP32 carries rb in two floats)
    int r0[3];   // (first index of the brick - lo_x) mod N_x
    int wl[3];   // window width per axis (0: touches nothing)
    T inv2s2, w, rc2;
};

template <typename T>
__device__ __forceinline__ void stage_general(StagedC<T> *dst, const SplatArgs &a, const ProbDesc &d,
                                              const int bidx[3], int64_t off, int c0, int nc, int t)
{
    if (t >= nc) return;
    const int atom = a.list_sorted[off + c0 + t];
    const AtomInfo in = a.info[atom];
    StagedC<T> s;
    double rb[3] = {in.X[0], in.X[1], in.X[2]};
    for (int x = 0; x < 3; ++x) {
        const double f = double(in.lo[x]) / d.dims[x];
        for (int c = 0; c < 3; ++c) rb[c] -= f * d.A[3 * x + c];
        s.r0[x] = wrapi(bidx[x] * d.bsz[x] - in.lo[x], d.dims[x]);
        s.wl[x] = in.hi[x] >= in.lo[x] ? in.hi[x] - in.lo[x] + 1 : 0;
    }
    for (int c = 0; c < 3; ++c) {
        s.rb[c] = T(rb[c]);
        s.rbl[c] = T(rb[c] - double(s.rb[c]));
    }
    s.inv2s2 = T(in.inv2s2);
    s.w = T(in.w);
    const double rc = a.cutoff * sqrt(0.5 / in.inv2s2);
    s.rc2 = T(rc * rc);
    dst[t] = s;
}

// Sum over the images of one atom inside its window of f(e, d) for the point
// at local offsets l = (li, lj, lk) of the brick (g = global index < N).
// e3 / e3l: the grid steps a / Na, b / Nb, c / Nc and their rounding
// remainders; each displacement component is formed with one rounding of
// the large terms (fma chain) plus the small remainder terms
template <typename T, typename F>
__device__ __forceinline__ void for_images(const StagedC<T> &at, const int l[3], const int n[3], const T e3[9],
                                           const T e3l[9], F f)
{
    int u0[3];
    for (int x = 0; x < 3; ++x) {
        int u = at.r0[x] + l[x];
        if (u >= n[x]) u -= n[x];
        u0[x] = u;
    }
    for (int ua = u0[0]; ua < at.wl[0]; ua += n[0])
        for (int ub = u0[1]; ub < at.wl[1]; ub += n[1])
            for (int uc = u0[2]; uc < at.wl[2]; uc += n[2]) {
                T dv[3];
                for (int c = 0; c < 3; ++c)
                    dv[c] = fma(T(ua), e3[c], fma(T(ub), e3[3 + c], fma(T(uc), e3[6 + c], -at.rb[c]))) +
                            (T(ua) * e3l[c] + T(ub) * e3l[3 + c] + T(uc) * e3l[6 + c] - at.rbl[c]);
                const T d2 = dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2];
                if (d2 <= at.rc2) f(expT<T>(-d2 * at.inv2s2), dv);
            }
}

struct BrickGeom {
    int bidx[3], bsz[3], n[3], npts;
};

__device__ __forceinline__ BrickGeom brick_geom(const ProbDesc &d, int64_t b)
{
    BrickGeom g;
    const int lb = int(b - d.brick_off);  // bricks of one problem fit 32 bits
    g.bidx[2] = lb % d.nbricks[2];
    g.bidx[1] = (lb / d.nbricks[2]) % d.nbricks[1];
    g.bidx[0] = lb / (d.nbricks[2] * d.nbricks[1]);
    for (int x = 0; x < 3; ++x) {
        g.bsz[x] = d.bsz[x];
        g.n[x] = d.dims[x];
    }
    g.npts = g.bsz[0] * g.bsz[1] * g.bsz[2];
    return g;
}

// local offsets of brick point p (c fastest)
__device__ __forceinline__ void brick_point(const BrickGeom &g, int p, int l[3])
{
    l[2] = p % g.bsz[2];
    l[1] = (p / g.bsz[2]) % g.bsz[1];
    l[0] = p / (g.bsz[2] * g.bsz[1]);
}

// point p of the brick lies inside the grid
__device__ __forceinline__ bool point_in_grid(const BrickGeom &g, const int l[3])
{
    return g.bidx[0] * g.bsz[0] + l[0] < g.n[0] && g.bidx[1] * g.bsz[1] + l[1] < g.n[1] &&
           g.bidx[2] * g.bsz[2] + l[2] < g.n[2];
}

template <typename T>
__global__ __launch_bounds__(kGenThreads) void k_splat_general(SplatArgs a)
{
    __shared__ StagedC<T> atoms[kGenChunk];
    __shared__ T acc[gen_max_points<T>()];  // the brick's running sums
    const int64_t b = blockIdx.x;
    const int prob = brick_prob(a, b);
    const ProbDesc &d = a.desc[prob];
    const BrickGeom g = brick_geom(d, b);
    T e3[9], e3l[9];
    for (int x = 0; x < 3; ++x)
        for (int c = 0; c < 3; ++c) {
            const double e = d.A[3 * x + c] / d.dims[x];
            e3[3 * x + c] = T(e);
            e3l[3 * x + c] = T(e - double(e3[3 * x + c]));
        }
    const int t = threadIdx.x;
    const int64_t off = a.offsets[b];
    const int cnt = int(a.offsets[b + 1] - off);
    for (int p = t; p < g.npts; p += kGenThreads) acc[p] = T(0);
    for (int c0 = 0; c0 < cnt; c0 += kGenChunk) {
        const int nc = (cnt - c0) < kGenChunk ? (cnt - c0) : kGenChunk;
        stage_general<T>(atoms, a, d, g.bidx, off, c0, nc, t);
        __syncthreads();
#pragma unroll 1
        for (int p = t; p < g.npts; p += kGenThreads) {
            int l[3];
            brick_point(g, p, l);
            if (!point_in_grid(g, l)) continue;
            T s = acc[p];
#pragma unroll 1
            for (int q = 0; q < nc; ++q) {
                const StagedC<T> &at = atoms[q];
                for_images<T>(at, l, g.n, e3, e3l, [&](T e, const T *) { s += at.w * e; });
            }
            acc[p] = s;
        }
        __syncthreads();
    }
    const T bg = a.subtract_background ? T(a.qsum[prob] / (d.dv * double(d.npts))) : T(0);
    T *out = reinterpret_cast<T *>(a.rho) + d.grid_off;
    for (int p = t; p < g.npts; p += kGenThreads) {
        int l[3];
        brick_point(g, p, l);
        if (!point_in_grid(g, l)) continue;
        const int i = g.bidx[0] * g.bsz[0] + l[0], j = g.bidx[1] * g.bsz[1] + l[1], k = g.bidx[2] * g.bsz[2] + l[2];
        out[(int64_t(i) * g.n[1] + j) * g.n[2] + k] = acc[p] - bg;
    }
}

template <typename T>
__device__ __forceinline__ T wave_sum_g(T v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// adjoint: per (brick, slot) the partial sum over the brick's points of
// grad_rho exp(-|d|^2 / (2 sigma^2)) d (the caller scales by w / sigma^2)
template <typename T>
__global__ __launch_bounds__(kGenThreads) void k_adjoint_general(SplatArgs a)
{
    __shared__ StagedC<T> atoms[kGenChunk];
    __shared__ T gr[gen_max_points<T>()];  // the brick's grad_rho (zero outside the grid)
    __shared__ T red[kGenThreads / 64][kGenChunk][3];
    const int64_t b = blockIdx.x;
    const int prob = brick_prob(a, b);
    const ProbDesc &d = a.desc[prob];
    const BrickGeom g = brick_geom(d, b);
    T e3[9], e3l[9];
    for (int x = 0; x < 3; ++x)
        for (int c = 0; c < 3; ++c) {
            const double e = d.A[3 * x + c] / d.dims[x];
            e3[3 * x + c] = T(e);
            e3l[3 * x + c] = T(e - double(e3[3 * x + c]));
        }
    const int t = threadIdx.x, wave = t >> 6;
    const int64_t off = a.offsets[b];
    const int cnt = int(a.offsets[b + 1] - off);
    if (cnt == 0) return;
    const T *src = reinterpret_cast<const T *>(a.grad_rho) + d.grid_off;
    for (int p = t; p < g.npts; p += kGenThreads) {
        int l[3];
        brick_point(g, p, l);
        T v = T(0);
        if (point_in_grid(g, l)) {
            const int i = g.bidx[0] * g.bsz[0] + l[0], j = g.bidx[1] * g.bsz[1] + l[1],
                      k = g.bidx[2] * g.bsz[2] + l[2];
            v = src[(int64_t(i) * g.n[1] + j) * g.n[2] + k];
        }
        gr[p] = v;
    }
    for (int c0 = 0; c0 < cnt; c0 += kGenChunk) {
        const int nc = (cnt - c0) < kGenChunk ? (cnt - c0) : kGenChunk;
        stage_general<T>(atoms, a, d, g.bidx, off, c0, nc, t);
        __syncthreads();
#pragma unroll 1
        for (int q = 0; q < nc; ++q) {
            const StagedC<T> &at = atoms[q];
            T f0 = T(0), f1 = T(0), f2 = T(0);
#pragma unroll 1
            for (int p = t; p < g.npts; p += kGenThreads) {
                int l[3];
                brick_point(g, p, l);
                if (!point_in_grid(g, l)) continue;
                const T gv = gr[p];
                for_images<T>(at, l, g.n, e3, e3l, [&](T e, const T *dv) {
                    const T s = gv * e;
                    f0 += s * dv[0];
                    f1 += s * dv[1];
                    f2 += s * dv[2];
                });
            }
            f0 = wave_sum_g(f0);
            f1 = wave_sum_g(f1);
            f2 = wave_sum_g(f2);
            if ((t & 63) == 0) {
                red[wave][q][0] = f0;
                red[wave][q][1] = f1;
                red[wave][q][2] = f2;
            }
        }
        __syncthreads();
        for (int e = t; e < nc * 3; e += kGenThreads) {
            const int q = e / 3, x = e - q * 3;
            double v = 0.0;
            for (int w = 0; w < kGenThreads / 64; ++w) v += double(red[w][q][x]);
            const int64_t slot = off + c0 + q;
            if (slot < a.capacity) a.bpart[slot * 3 + x] = v;
        }
        __syncthreads();
    }
}

hipError_t run_gather_general(const SplatArgs &a, hipStream_t s)
{
    if (a.fp64)
        hipLaunchKernelGGL(k_splat_general<double>, dim3(int(a.nbricks_total)), dim3(kGenThreads), 0, s, a);
    else
        hipLaunchKernelGGL(k_splat_general<float>, dim3(int(a.nbricks_total)), dim3(kGenThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t run_adjoint_general(const SplatArgs &a, hipStream_t s)
{
    if (a.fp64)
        hipLaunchKernelGGL(k_adjoint_general<double>, dim3(int(a.nbricks_total)), dim3(kGenThreads), 0, s, a);
    else
        hipLaunchKernelGGL(k_adjoint_general<float>, dim3(int(a.nbricks_total)), dim3(kGenThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace hartree
