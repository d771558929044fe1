// Mixed-radix Stockham pencil FFT for gfx950.
//
// A workgroup transforms P pencils of one axis.  Between stages the pencils
// of a strided axis live in LDS as buf[i * PP + p] (element i of pencil p,
// PP = P + pad with pad 0..3 chosen per axis, by a bank-conflict model or by
// the tuner); pencils along the contiguous axis live pencil-major,
// buf[p * ldp + i].  Threads are (p, tip) with p fastest, TPP threads per
// pencil.
//
// Stage s has radix R and Ns = product of the earlier radices; butterfly
// j < n/R of every pencil computes
//   k = j mod Ns
//   v_q = x[j + q n/R] * W_{Ns R}^{q k},                 q = 0 .. R-1
//   y[(j div Ns) Ns R + k + q Ns] = DFT_R(v)_q
// with W_m = exp(-2 pi i / m) (forward) or its conjugate (inverse); the output
// of the last stage is in natural order.  The first stage has no twiddles
// (Ns = 1) and in the last one (Ns = n/R) the output index is j + q Ns.
//
// Where the pencils are strided in memory (the b and a axes), the first stage
// reads its inputs straight from global memory and the last stage writes its
// outputs straight back: a wavefront then reads or writes whole runs of P
// consecutive complex values of each grid row, and the tile passes through
// LDS only between stages.
//
// Radices 2, 3, 4, 5, 7 and 8 are written out; 9 and 16 are built as
// two-level Cooley-Tukey products of those, and 6, 10 and 12 (coprime
// factors) as prime-factor products without inner twiddles, so most lengths
// of interest need at most three stages.
#pragma once

#include <type_traits>

#include "common.hpp"
#include "radix_consts.hpp"

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
// a times the conjugate of b
template <typename T>
__device__ __forceinline__ Cx<T> cmulc(Cx<T> a, Cx<T> b)
{
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV>
__device__ __forceinline__ Cx<T> rot(Cx<T> a)
{
    return INV ? Cx<T>{-a.y, a.x} : Cx<T>{a.y, -a.x};
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void butterfly(Cx<T> *a);

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
            const T c = T(unit_cos(R, k * m));
            const T s = T(unit_sin(R, k * m));
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

// Two-level product radix R = A B: with n = B n1 + n2 and k = k1 + A k2,
//   X[k] = sum_n2 W_B^(n2 k2) [ W_R^(n2 k1) sum_n1 x[B n1 + n2] W_A^(n1 k1) ].
template <typename T, int A, int B, bool INV>
__device__ __forceinline__ void dft_product(Cx<T> *x)
{
    constexpr int R = A * B;
    Cx<T> y[R];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) {
        Cx<T> t[A];
#pragma unroll
        for (int n1 = 0; n1 < A; ++n1) t[n1] = x[B * n1 + n2];
        butterfly<T, A, INV>(t);
#pragma unroll
        for (int k1 = 0; k1 < A; ++k1) {
            const int e = n2 * k1;
            if (e == 0) {
                y[k1 * B + n2] = t[k1];
            } else {
                const T c = T(unit_cos(R, e));
                const T s = T(unit_sin(R, e));
                y[k1 * B + n2] = cmul(t[k1], Cx<T>{c, INV ? s : -s});
            }
        }
    }
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
        Cx<T> t[B];
#pragma unroll
        for (int n2 = 0; n2 < B; ++n2) t[n2] = y[k1 * B + n2];
        butterfly<T, B, INV>(t);
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) x[k1 + A * k2] = t[k2];
    }
}

// inverse of a modulo m (a and m coprime), by search: compile-time only
constexpr int inv_mod(int a, int m)
{
    for (int i = 1; i < m; ++i)
        if ((a * i) % m == 1) return i;
    return 1;
}

// Coprime product radix R = A B (Good-Thomas prime-factor mapping): with the
// input map n = (B n1 + A n2) mod R and the output map
// k = (B B' k1 + A A' k2) mod R, where B' = B^-1 mod A and A' = A^-1 mod B,
// W_R^(n k) = W_A^(n1 k1) W_B^(n2 k2): an A x B two-dimensional DFT with no
// twiddle factors between the levels.  The maps are register renamings.
template <typename T, int A, int B, bool INV>
__device__ __forceinline__ void dft_coprime(Cx<T> *x)
{
    constexpr int R = A * B;
    constexpr int Bi = inv_mod(B % A, A), Ai = inv_mod(A % B, B);
    Cx<T> y[A][B];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) {
        Cx<T> t[A];
#pragma unroll
        for (int n1 = 0; n1 < A; ++n1) t[n1] = x[(B * n1 + A * n2) % R];
        butterfly<T, A, INV>(t);
#pragma unroll
        for (int k1 = 0; k1 < A; ++k1) y[k1][n2] = t[k1];
    }
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
        butterfly<T, B, INV>(y[k1]);
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) x[(B * Bi * k1 + A * Ai * k2) % R] = y[k1][k2];
    }
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void butterfly(Cx<T> *a)
{
    if constexpr (R == 1) {
    } else if constexpr (R == 2) {
        Cx<T> t = a[0];
        a[0] = cadd(t, a[1]);
        a[1] = csub(t, a[1]);
    } else if constexpr (R == 4) {
        dft4<T, INV>(a[0], a[1], a[2], a[3]);
    } else if constexpr (R == 8) {
        // pairs 4 apart: e_q = a_q + a_{q+4}, f_q = (a_q - a_{q+4}) W_8^q;
        // even outputs DFT4(e), odd outputs DFT4(f)
        constexpr T h = T(0.7071067811865475244008443621048490392848);
        Cx<T> e[4], f[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            e[q] = cadd(a[q], a[q + 4]);
            f[q] = csub(a[q], a[q + 4]);
        }
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
    } else if constexpr (R == 3 || R == 5 || R == 7) {
        dft_odd<T, R, INV>(a);
    } else if constexpr (R == 6) {
        dft_coprime<T, 2, 3, INV>(a);
    } else if constexpr (R == 9) {
        dft_product<T, 3, 3, INV>(a);
    } else if constexpr (R == 10) {
        dft_coprime<T, 2, 5, INV>(a);
    } else if constexpr (R == 12) {
        dft_coprime<T, 4, 3, INV>(a);
    } else {
        static_assert(R == 16, "unsupported radix");
        dft_product<T, 4, 4, INV>(a);
    }
}

constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }

// ------------------------------------------------------------------ access
// element i of the thread's pencil in the LDS tile
// An inverse transform runs the forward stages on conjugated data:
// F^-1 x = conj(F conj x) (unnormalized), so the accessor that feeds the
// first stage and the one that takes the last stage's output conjugate when
// cj is set.
template <typename T>
struct LdsPencil {
    static constexpr bool kLds = true;
    static constexpr bool kTail = false;
    Cx<T> *buf;
    int pp, p;
    bool cj;
    __device__ __forceinline__ Cx<T> load(int i) const
    {
        Cx<T> v = buf[i * pp + p];
        if (cj) v.y = -v.y;
        return v;
    }
    __device__ __forceinline__ void store(int i, Cx<T> v) const
    {
        if (cj) v.y = -v.y;
        buf[i * pp + p] = v;
    }
    // element u + t, u uniform across the wavefront (see GlobalPencil)
    __device__ __forceinline__ Cx<T> load_at(int u, int t) const { return load(u + t); }
    __device__ __forceinline__ void store_at(int u, int t, Cx<T> v) const { store(u + t, v); }
};

// element i of the thread's pencil in a pencil-major LDS tile
// (buf[p * ldp + i]), used where threads run along the pencil
template <typename T>
struct LdsRow {
    static constexpr bool kLds = true;
    static constexpr bool kTail = false;
    Cx<T> *buf;
    int ldp, p;
    bool cj;
    __device__ __forceinline__ Cx<T> load(int i) const
    {
        Cx<T> v = buf[p * ldp + i];
        if (cj) v.y = -v.y;
        return v;
    }
    __device__ __forceinline__ void store(int i, Cx<T> v) const
    {
        if (cj) v.y = -v.y;
        buf[p * ldp + i] = v;
    }
    __device__ __forceinline__ Cx<T> load_at(int u, int t) const { return load(u + t); }
    __device__ __forceinline__ void store_at(int u, int t, Cx<T> v) const { store(u + t, v); }
};

// Element u + tip of the thread's strided pencil in global memory, where the
// stage loops pass u (the part of the index that is the same for every lane
// of a wavefront) and tip separately: the uniform part moves a base pointer
// in scalar registers, and each lane adds its fixed offset lane = tip *
// stride + its pencil's column, so an access costs no vector arithmetic.
// L32: lane * sizeof(Cx<T>) fits 32 bits (the host launches such kernels
// only then), and the lane offset is a 32-bit byte offset.  A pencil beyond
// the tile edge (valid false) points at a valid pencil of the tile: it loads
// real data, is transformed like the others, and stores nothing.
// a wavefront-uniform 64-bit value pinned to scalar registers
__device__ __forceinline__ int64_t uniform64(int64_t x)
{
    asm("" : "+s"(x));
    return x;
}

template <typename T, bool L32, bool RUN = false>
struct GlobalPencil {
    static constexpr bool kLds = false;
    static constexpr bool kRun = L32 && RUN;
    Cx<T> *base;  // element 0 of the tile's first pencil (wavefront-uniform)
    int stride;   // elements between consecutive points of a pencil
    int lane;     // tip * stride + column of this thread's pencil (elements)
    bool valid;
    bool cj;
    __device__ __forceinline__ Cx<T> *at(int u) const
    {
        Cx<T> *row = base + int64_t(u) * stride;
        if constexpr (L32)
            return reinterpret_cast<Cx<T> *>(reinterpret_cast<char *>(row) +
                                              uint32_t(lane) * uint32_t(sizeof(Cx<T>)));
        else
            return row + lane;
    }
    __device__ __forceinline__ Cx<T> load_at(int u, int) const
    {
        Cx<T> v = *at(u);
        if (cj) v.y = -v.y;
        return v;
    }
    __device__ __forceinline__ void store_at(int u, int, Cx<T> v) const
    {
        if (cj) v.y = -v.y;
        if (valid) *at(u) = v;
    }
    // Elements u0 + q du (q = 0 .. K-1; u0 and du uniform) with L32 and RUN:
    // the row offset advances by a scalar step in scalar registers, and each
    // address is one 64-bit add of it to the lane's pointer (the compiler
    // otherwise forms the row chain with 64-bit multiply-adds on the vector
    // units).  Taken by the vector-bound a pass only: in the memory-bound b
    // pass the same form measured slower.
    __device__ __forceinline__ Cx<T> *lane_at(int64_t o) const
    {
        return reinterpret_cast<Cx<T> *>(reinterpret_cast<char *>(base + o) + uint32_t(lane) * uint32_t(sizeof(Cx<T>)));
    }
    template <int K>
    __device__ __forceinline__ void load_run(int u0, int du, Cx<T> (&out)[K]) const
    {
        int64_t o = uniform64(int64_t(u0) * stride);
        const int64_t step = int64_t(du) * stride;
#pragma unroll
        for (int q = 0; q < K; ++q) {
            Cx<T> v = *lane_at(o);
            if (cj) v.y = -v.y;
            out[q] = v;
            o = uniform64(o + step);
        }
    }
    template <int K>
    __device__ __forceinline__ void store_run(int u0, int du, const Cx<T> (&in)[K]) const
    {
        int64_t o = uniform64(int64_t(u0) * stride);
        const int64_t step = int64_t(du) * stride;
#pragma unroll
        for (int q = 0; q < K; ++q) {
            Cx<T> v = in[q];
            if (cj) v.y = -v.y;
            if (valid) *lane_at(o) = v;
            o = uniform64(o + step);
        }
    }
};

// whether an accessor takes runs of rows (load_run / store_run)
template <typename A, typename = void>
struct has_run : std::false_type {};
template <typename A>
struct has_run<A, std::void_t<decltype(A::kRun)>> : std::bool_constant<A::kRun> {};

// Butterflies per thread a stage holds in registers, by radix: a stage keeps
// at most 32 complex values per thread in float (21 in double, enough for
// every 7-smooth length up to 4096 at 256 threads per pencil).  The host
// picks the threads per pencil (tpp) so that every stage of a length fits:
// ceil((n / R) / tpp) <= MAXB(R).
template <typename T>
__host__ __device__ constexpr int stage_maxb(int R)
{
    return (sizeof(T) == 4 ? 32 : 21) / R > 0 ? (sizeof(T) == 4 ? 32 : 21) / R : 1;
}

// One Stockham stage.  Src and Dst are pencil accessors; when both are the
// same tile, SYNC separates all reads from all writes.
template <typename T, int R, int MAXB, bool FIRST, bool SYNC, typename Src, typename Dst>
__device__ __forceinline__ void stage(const Src &src, Dst &dst, const Cx<T> *tw, int n, int twstride,
                                      const FastDiv &nsd, int tip, int tpp)
{
    const int nb = n / R;
    Cx<T> v[MAXB][R];
#pragma unroll
    for (int m = 0; m < MAXB; ++m) {
        const int j = tip + m * tpp;
        if (j < nb) {
#pragma unroll
            for (int q = 0; q < R; ++q) v[m][q] = src.load_at(m * tpp + q * nb, tip);
        }
    }
    if (SYNC) __syncthreads();
#pragma unroll
    for (int m = 0; m < MAXB; ++m) {
        const int j = tip + m * tpp;
        if (j < nb) {
            int jd = j, k = 0, ns = 1;
            if (!FIRST) {
                ns = int(nsd.d);
                jd = int(fdiv(uint32_t(j), nsd));
                k = j - jd * ns;
                // twiddle indices stay below n <= 2^24: 24-bit products
                const int tstep = __mul24(k, twstride);
#pragma unroll
                for (int q = 1; q < R; ++q) v[m][q] = cmul(v[m][q], tw[__mul24(q, tstep)]);
            }
            butterfly<T, R, false>(v[m]);
            if constexpr (Dst::kLds) {
                const int base = jd * ns * R + k;
#pragma unroll
                for (int q = 0; q < R; ++q) dst.store(base + q * ns, v[m][q]);
            } else {
                // only the last stage writes global memory: ns = n / R,
                // so jd = 0 and k = j
#pragma unroll
                for (int q = 0; q < R; ++q) dst.store_at(m * tpp + q * ns, tip, v[m][q]);
            }
        }
    }
}

// The same stage with the length, the stride of its outputs (ns, the
// product of the earlier radices) and its twiddle stride known at compile
// time (the compiled radix plans): index arithmetic folds into constants.
// INV: the inverse transform's stage (conjugate twiddles and butterflies).
template <typename T, int R, int MAXB, bool FIRST, bool SYNC, int NB, int NS, int TWS, bool INV, typename Src,
          typename Dst>
__device__ __forceinline__ void stage_ct(const Src &src, Dst &dst, const Cx<T> *tw, int tip, int tpp)
{
    Cx<T> v[MAXB][R];
#pragma unroll
    for (int m = 0; m < MAXB; ++m) {
        const int j = tip + m * tpp;
        if (j < NB) {
            if constexpr (has_run<Src>::value) {
                src.template load_run<R>(m * tpp, NB, v[m]);
            } else {
#pragma unroll
                for (int q = 0; q < R; ++q) v[m][q] = src.load_at(m * tpp + q * NB, tip);
            }
        }
    }
    if (SYNC) __syncthreads();
#pragma unroll
    for (int m = 0; m < MAXB; ++m) {
        const int j = tip + m * tpp;
        if (j < NB) {
            // the first stage has NS = 1: k = 0 and no twiddles
            const int jd = j / NS;
            const int k = j - jd * NS;
            if (!FIRST) {
                const int tstep = __mul24(k, TWS);
#pragma unroll
                for (int q = 1; q < R; ++q) {
                    const Cx<T> w = tw[__mul24(q, tstep)];
                    v[m][q] = INV ? cmulc(v[m][q], w) : cmul(v[m][q], w);
                }
            }
            butterfly<T, R, INV>(v[m]);
            if constexpr (Dst::kLds) {
                const int base = jd * (NS * R) + k;
                if constexpr (Dst::kTail) {
                    // the last stage into a destination that needs each
                    // element's index split: base = j < NS, offsets q NS
#pragma unroll
                    for (int q = 0; q < R; ++q) dst.store_tail(base, q * NS, NS, NS * R, v[m][q]);
                    dst.end_butterfly();
                } else {
#pragma unroll
                    for (int q = 0; q < R; ++q) dst.store(base + q * NS, v[m][q]);
                }
            } else {
                // the last stage (NS = N / R): jd = 0, k = j
                if constexpr (has_run<Dst>::value) {
                    dst.template store_run<R>(m * tpp, NS, v[m]);
                } else {
#pragma unroll
                    for (int q = 0; q < R; ++q) dst.store_at(m * tpp + q * NS, tip, v[m][q]);
                }
            }
        }
    }
}

// Dispatch one stage on its runtime radix.
template <typename T, bool FIRST, bool SYNC, typename Src, typename Dst>
__device__ __forceinline__ void stage_any(int r, const Src &src, Dst &dst, const Cx<T> *tw, int n, int twstride,
                                          const FastDiv &nsd, int tip, int tpp)
{
#define HARTREE_STAGE(RR) \
    stage<T, RR, stage_maxb<T>(RR), FIRST, SYNC>(src, dst, tw, n, twstride, nsd, tip, tpp)
    switch (r) {
    case 2: HARTREE_STAGE(2); break;
    case 3: HARTREE_STAGE(3); break;
    case 4: HARTREE_STAGE(4); break;
    case 5: HARTREE_STAGE(5); break;
    case 7: HARTREE_STAGE(7); break;
    case 8: HARTREE_STAGE(8); break;
    case 9: HARTREE_STAGE(9); break;
    case 10: HARTREE_STAGE(10); break;
    case 16: HARTREE_STAGE(16); break;
    default: break;  // not produced by the plan search
    }
#undef HARTREE_STAGE
}

// Forward transform of a tile whose first stage reads from `src` and whose
// last stage writes to `dst` (either may be global memory or the LDS tile;
// conjugating accessors turn it into the inverse); the stages in between run
// in place on the LDS tile `lds`.  A single-stage length runs its stage into
// the tile and then copies it to dst.  On return every thread has finished
// writing; the caller synchronizes before reading the LDS tile.
template <typename T, typename Src, typename Dst, typename L>
__device__ __forceinline__ void fft_pencils(const Src &src, Dst &dst, const L &lds, const Cx<T> *tw,
                                            const AxisPlan &ap, int tip, int tpp)
{
    const int n = ap.n;
    const int S = ap.nstages;
    L l = lds;
    l.cj = false;
    // a stage that writes where the workgroup still reads (the LDS tile)
    // separates its reads from its writes with a barrier
    stage_any<T, true, Src::kLds>(ap.radix[0], src, l, tw, n, ap.twstride[0], ap.ns[0], tip, tpp);
    __syncthreads();
    if (S == 1) {
        for (int u = 0; u + tip < n; u += tpp) dst.store_at(u, tip, l.load(u + tip));
        return;
    }
    for (int s = 1; s + 1 < S; ++s) {
        stage_any<T, false, true>(ap.radix[s], l, l, tw, n, ap.twstride[s], ap.ns[s], tip, tpp);
        __syncthreads();
    }
    const int s = S - 1;
    stage_any<T, false, Dst::kLds>(ap.radix[s], l, dst, tw, n, ap.twstride[s], ap.ns[s], tip, tpp);
}

// The same transform with the stage radices fixed at compile time (R1..R3 = 0
// for absent stages).  Each stage then gets registers sized for its own
// radix; a kernel that switches between radices at run time (fft_pencils)
// must hold registers for the largest case in every stage, which costs
// occupancy.  INV: the inverse transform (unnormalized), with no
// conjugation of its input or output.
template <typename T, int R0, int R1, int R2, int R3, bool INV = false, typename Src, typename Dst, typename L>
__device__ __forceinline__ void fft_static(const Src &src, Dst &dst, const L &lds, const Cx<T> *tw,
                                           const AxisPlan &ap, int tip, int tpp)
{
    constexpr int S = (R0 > 0) + (R1 > 0) + (R2 > 0) + (R3 > 0);
    constexpr int N = R0 * (R1 > 0 ? R1 : 1) * (R2 > 0 ? R2 : 1) * (R3 > 0 ? R3 : 1);
    // stage s: ns = product of the earlier radices, twiddle stride n / (ns R)
    constexpr int NS1 = R0, NS2 = R0 * (R1 > 0 ? R1 : 1), NS3 = NS2 * (R2 > 0 ? R2 : 1);
    constexpr int Q1 = R1 > 0 ? R1 : 1, Q2 = R2 > 0 ? R2 : 1, Q3 = R3 > 0 ? R3 : 1;
    (void)ap;
    L l = lds;
    l.cj = false;
    stage_ct<T, R0, stage_maxb<T>(R0), true, Src::kLds, N / R0, 1, 1, INV>(src, l, tw, tip, tpp);
    __syncthreads();
    if constexpr (S == 1) {
        for (int u = 0; u + tip < N; u += tpp) dst.store_at(u, tip, l.load(u + tip));
    } else if constexpr (S == 2) {
        stage_ct<T, Q1, stage_maxb<T>(Q1), false, Dst::kLds, N / Q1, NS1, N / (NS1 * Q1), INV>(l, dst, tw, tip, tpp);
    } else {
        stage_ct<T, Q1, stage_maxb<T>(Q1), false, true, N / Q1, NS1, N / (NS1 * Q1), INV>(l, l, tw, tip, tpp);
        __syncthreads();
        if constexpr (S == 3) {
            stage_ct<T, Q2, stage_maxb<T>(Q2), false, Dst::kLds, N / Q2, NS2, N / (NS2 * Q2), INV>(l, dst, tw, tip,
                                                                                               tpp);
        } else {
            stage_ct<T, Q2, stage_maxb<T>(Q2), false, true, N / Q2, NS2, N / (NS2 * Q2), INV>(l, l, tw, tip, tpp);
            __syncthreads();
            stage_ct<T, Q3, stage_maxb<T>(Q3), false, Dst::kLds, N / Q3, NS3, N / (NS3 * Q3), INV>(l, dst, tw, tip,
                                                                                               tpp);
        }
    }
}

// Either form: R0 = 0 selects the run-time radix switch.
template <typename T, int R0, int R1, int R2, int R3, typename Src, typename Dst, typename L>
__device__ __forceinline__ void fft_any(const Src &src, Dst &dst, const L &lds, const Cx<T> *tw,
                                        const AxisPlan &ap, int tip, int tpp)
{
    if constexpr (R0 == 0)
        fft_pencils<T>(src, dst, lds, tw, ap, tip, tpp);
    else
        fft_static<T, R0, R1, R2, R3>(src, dst, lds, tw, ap, tip, tpp);
}

// Radix plans with their own compiled kernels: the stage radices that the
// plan search picks for common lengths (32, 48, 60, 64, 72, 90, 96, 120, 128,
// 150, 160, 180, 192, 200, 210, 240, 256, 288, 300, 320, 360, 384, 400, 420,
// 480, 512, 576, 600, 640, 720, 768, 800, 840, 960, 1024, 2048), then
// alternatives that the tuner may prefer: radix-6 stages for 360 and 180,
// whose butterfly counts (36 and 60 per pencil for 360) fill a 64-lane
// wavefront better than 40, 45 and 72; and plans of 48, 128 and 160 without
// a radix-16 stage, which the multi-plan kernels of the c passes take (a
// radix-16 butterfly there sets the whole kernel's registers); and radix-12
// first stages for 360, whose 30 butterflies per pencil take one round on 32
// threads (radix 10's 36 take two).  Entries are only ever appended, so that
// stored tuner choices keep their meaning.
// Other lengths run the run-time radix switch.
#define HARTREE_PLANS(X)                                                                                  \
    X(8, 4, 0, 0) X(16, 3, 0, 0) X(5, 4, 3, 0) X(8, 8, 0, 0) X(9, 8, 0, 0) X(10, 9, 0, 0) X(8, 4, 3, 0)   \
    X(8, 5, 3, 0) X(16, 8, 0, 0) X(10, 5, 3, 0) X(16, 10, 0, 0) X(9, 5, 4, 0) X(8, 8, 3, 0)              \
    X(8, 5, 5, 0) X(10, 7, 3, 0) X(10, 8, 3, 0) X(16, 16, 0, 0) X(9, 8, 4, 0) X(10, 10, 3, 0)            \
    X(8, 8, 5, 0) X(9, 8, 5, 0) X(16, 8, 3, 0) X(10, 10, 4, 0) X(7, 5, 4, 3) X(16, 10, 3, 0)             \
    X(8, 8, 8, 0) X(9, 8, 8, 0) X(8, 5, 5, 3) X(10, 8, 8, 0) X(10, 9, 8, 0) X(16, 16, 3, 0)              \
    X(10, 10, 8, 0) X(8, 7, 5, 3) X(8, 8, 5, 3) X(16, 16, 4, 0) X(16, 16, 8, 0)                          \
    X(10, 6, 6, 0) X(6, 6, 10, 0) X(6, 10, 6, 0) X(10, 6, 3, 0) X(6, 6, 5, 0)                           \
    X(8, 6, 0, 0) X(8, 4, 4, 0) X(8, 5, 4, 0) X(12, 5, 6, 0) X(12, 6, 5, 0)

// the plan table as compile-time constants (for kernels that pick a plan per
// workgroup)
#define HARTREE_ROW(R0, R1, R2, R3) {R0, R1, R2, R3},
constexpr int kPlanRadix[][4] = {HARTREE_PLANS(HARTREE_ROW)};
#undef HARTREE_ROW

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
