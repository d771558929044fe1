// Mixed-radix (2/3/4/5/7/8) Stockham pencil FFT over an LDS tile, for gfx950.
//
// A workgroup holds P pencils of one axis in LDS as buf[n][P] (the pencil
// index runs fastest, so a wavefront's lanes touch consecutive words), plus
// the length-n twiddle table.  Each Stockham stage of radix R reads R
// elements per butterfly into registers, applies the twiddles and the
// radix-R DFT in registers, and writes them back in autosorted order; the
// output of the last stage is in natural order.  TPP threads share a pencil.
//
// Stage s (radix R, Ns = product of the earlier radices), butterfly j < n/R:
//   k = j mod Ns
//   v_q = x[j + q n/R] * W_{Ns R}^{q k},        q = 0..R-1
//   y[(j div Ns) Ns R + k + q Ns] = DFT_R(v)_q
// with W_m = exp(-2 pi i / m) (forward) or its conjugate (inverse).
#pragma once

#include "common.hpp"

namespace hartree {

template <typename T>
struct alignas(2 * sizeof(T)) Cx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ Cx<T> cadd(Cx<T> a, Cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ Cx<T> csub(Cx<T> a, Cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ Cx<T> cscale(Cx<T> a, T s) { return {a.x * s, a.y * s}; }
template <typename T>
__device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV>
__device__ __forceinline__ Cx<T> rot(Cx<T> a)
{
    return INV ? Cx<T>{-a.y, a.x} : Cx<T>{a.y, -a.x};
}

// cos(2 pi t / R) and sin(2 pi t / R) for the odd radices R = 3, 5, 7
// (literals to 40 digits; the compiler rounds them to T)
__host__ __device__ constexpr double odd_cos_base(int R, int t)
{
    return t == 0 ? 1.0
         : R == 3 ? -0.5
         : R == 5 ? (t == 1 ? 0.3090169943749474241022934171828190588611
                            : -0.8090169943749474241022934171828190588587)
         : (t == 1 ? 0.6234898018587335305250048840042398106325
          : t == 2 ? -0.2225209339563144042889025644967947594652
                   : -0.9009688679024191262361023195074450511656);
}
__host__ __device__ constexpr double odd_sin_base(int R, int t)
{
    return t == 0 ? 0.0
         : R == 3 ? 0.8660254037844386467637231707529361834714
         : R == 5 ? (t == 1 ? 0.9510565162951535721164393333793821434054
                            : 0.5877852522924731291687059546390727685988)
         : (t == 1 ? 0.7818314824680298087084445266740577502321
          : t == 2 ? 0.9749279121818236070181316829939312172330
                   : 0.4338837391175581204757683328483587546094);
}
template <int R>
__host__ __device__ constexpr double odd_cos(int t)
{
    return (t % R) <= R / 2 ? odd_cos_base(R, t % R) : odd_cos_base(R, R - t % R);
}
template <int R>
__host__ __device__ constexpr double odd_sin(int t)
{
    return (t % R) <= R / 2 ? odd_sin_base(R, t % R) : -odd_sin_base(R, R - t % R);
}

// Odd prime radix: pair inputs q and R-q.
//   y_0 = a_0 + sum_k b_k,  b_k = a_k + a_{R-k},  d_k = a_k - a_{R-k}
//   y_m = t_m + rot(u_m), y_{R-m} = t_m - rot(u_m),
//   t_m = a_0 + sum_k cos(2 pi k m / R) b_k,  u_m = sum_k sin(2 pi k m / R) d_k
template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_odd(Cx<T> *a)
{
    constexpr int H = (R - 1) / 2;
    Cx<T> b[H + 1], d[H + 1];
#pragma unroll
    for (int k = 1; k <= H; ++k) {
        b[k] = cadd(a[k], a[R - k]);
        d[k] = csub(a[k], a[R - k]);
    }
    Cx<T> y0 = a[0];
#pragma unroll
    for (int k = 1; k <= H; ++k) y0 = cadd(y0, b[k]);
    Cx<T> out[R];
    out[0] = y0;
#pragma unroll
    for (int m = 1; m <= H; ++m) {
        Cx<T> t = a[0], u = {T(0), T(0)};
#pragma unroll
        for (int k = 1; k <= H; ++k) {
            const T c = T(odd_cos<R>(k * m));
            const T s = T(odd_sin<R>(k * m));
            t.x += c * b[k].x;
            t.y += c * b[k].y;
            u.x += s * d[k].x;
            u.y += s * d[k].y;
        }
        Cx<T> ru = rot<T, INV>(u);
        out[m] = cadd(t, ru);
        out[R - m] = csub(t, ru);
    }
#pragma unroll
    for (int q = 0; q < R; ++q) a[q] = out[q];
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(Cx<T> &a0, Cx<T> &a1, Cx<T> &a2, Cx<T> &a3)
{
    Cx<T> s02 = cadd(a0, a2), d02 = csub(a0, a2);
    Cx<T> s13 = cadd(a1, a3), d13 = rot<T, INV>(csub(a1, a3));
    a0 = cadd(s02, s13);
    a2 = csub(s02, s13);
    a1 = cadd(d02, d13);
    a3 = csub(d02, d13);
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void butterfly(Cx<T> *a)
{
    if constexpr (R == 2) {
        Cx<T> t = a[0];
        a[0] = cadd(t, a[1]);
        a[1] = csub(t, a[1]);
    } else if constexpr (R == 4) {
        dft4<T, INV>(a[0], a[1], a[2], a[3]);
    } else if constexpr (R == 8) {
        // split into pairs 4 apart: e_q = a_q + a_{q+4}, f_q = (a_q - a_{q+4}) W_8^q;
        // even outputs are DFT4(e), odd outputs DFT4(f)
        constexpr T h = T(0.7071067811865475244008443621048490392848);
        Cx<T> e[4], f[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            e[q] = cadd(a[q], a[q + 4]);
            f[q] = csub(a[q], a[q + 4]);
        }
        // W_8 = (h, -h) forward, (h, h) inverse; W_8^2 = rot; W_8^3 = (-h, -h) / (-h, h)
        f[1] = cmul(f[1], Cx<T>{h, INV ? h : -h});
        f[2] = rot<T, INV>(f[2]);
        f[3] = cmul(f[3], Cx<T>{-h, INV ? h : -h});
        dft4<T, INV>(e[0], e[1], e[2], e[3]);
        dft4<T, INV>(f[0], f[1], f[2], f[3]);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            a[2 * m] = e[m];
            a[2 * m + 1] = f[m];
        }
    } else {
        dft_odd<T, R, INV>(a);
    }
}

constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }

// One Stockham stage of radix R over buf[n][P]; thread (p, tip).
template <typename T, int R, int P, int TPP, int MAXB, bool INV>
__device__ __forceinline__ void stockham_stage(Cx<T> *buf, const Cx<T> *tw, int n, int twstride,
                                               const FastDiv &nsd, int p, int tip)
{
    const int nb = n / R;
    Cx<T> v[MAXB][R];
#pragma unroll
    for (int m = 0; m < MAXB; ++m) {
        const int j = tip + m * TPP;
        if (j < nb) {
#pragma unroll
            for (int q = 0; q < R; ++q) v[m][q] = buf[(j + q * nb) * P + p];
        }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < MAXB; ++m) {
        const int j = tip + m * TPP;
        if (j < nb) {
            const int ns = int(nsd.d);
            const int jd = int(fdiv(uint32_t(j), nsd));
            const int k = j - jd * ns;
            const int tstep = k * twstride;
#pragma unroll
            for (int q = 1; q < R; ++q) {
                Cx<T> w = tw[q * tstep];
                if (INV) w.y = -w.y;
                v[m][q] = cmul(v[m][q], w);
            }
            butterfly<T, R, INV>(v[m]);
            const int base = jd * ns * R + k;
#pragma unroll
            for (int q = 0; q < R; ++q) buf[(base + q * ns) * P + p] = v[m][q];
        }
    }
    __syncthreads();
}

// Full transform of the P pencils in buf (length ap.n <= NMAX).  Callers
// synchronize before the call; the tile is complete on return.
template <typename T, int NMAX, int P, int TPP, bool INV>
__device__ __forceinline__ void fft_tile(Cx<T> *buf, const Cx<T> *tw, const AxisPlan &ap, int p, int tip)
{
    const int n = ap.n;
    const int ns_count = ap.nstages;
    for (int s = 0; s < ns_count; ++s) {
        const int r = ap.radix[s];
        const int ts = ap.twstride[s];
        const FastDiv nsd = ap.ns[s];
        switch (r) {
        case 2: stockham_stage<T, 2, P, TPP, cdiv(NMAX / 2, TPP), INV>(buf, tw, n, ts, nsd, p, tip); break;
        case 3: stockham_stage<T, 3, P, TPP, cdiv(NMAX / 3 + 1, TPP), INV>(buf, tw, n, ts, nsd, p, tip); break;
        case 4: stockham_stage<T, 4, P, TPP, cdiv(NMAX / 4, TPP), INV>(buf, tw, n, ts, nsd, p, tip); break;
        case 5: stockham_stage<T, 5, P, TPP, cdiv(NMAX / 5 + 1, TPP), INV>(buf, tw, n, ts, nsd, p, tip); break;
        case 7: stockham_stage<T, 7, P, TPP, cdiv(NMAX / 7 + 1, TPP), INV>(buf, tw, n, ts, nsd, p, tip); break;
        default: stockham_stage<T, 8, P, TPP, cdiv(NMAX / 8, TPP), INV>(buf, tw, n, ts, nsd, p, tip); break;
        }
    }
}

// Blocks are dispatched round-robin over the 8 XCDs (each with its own L2);
// renumber them so that consecutive work items land on the same XCD, where
// neighbouring tiles share cache lines at their edges.
__device__ __forceinline__ int xcd_remap(int b, int g)
{
    const int xcd = b & 7, local = b >> 3;
    const int per = g >> 3, rem = g & 7;
    return xcd * per + (xcd < rem ? xcd : rem) + local;
}

}  // namespace hartree
