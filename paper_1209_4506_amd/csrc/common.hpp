// Shared host/device definitions of the MI355X Hartree library.
//
// A plan is described to the kernels by an array of ProbDesc (one per problem
// of a batched plan, one for a single plan) that lives in the caller-owned
// workspace.  Each ProbDesc carries the three 1-D transform plans (axes a, b,
// c), the grid and half-spectrum offsets, and the reciprocal metric that the
// Poisson kernel needs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hartree {

constexpr int kMaxStages = 12;  // 4096 = 8^4, so at most a handful; 12 leaves room for 2/3/5/7 mixes
constexpr int kMaxProb = 64;
constexpr int kMaxN = 4096;     // largest supported axis length

// Exact x / d for x * (m*d - 2^40) < 2^40, i.e. any x < 2^28 when d <= 4096.
struct FastDiv {
    uint32_t d;
    uint32_t pad;
    uint64_t m;  // ceil(2^40 / d)
};

__host__ __device__ inline FastDiv make_fastdiv(uint32_t d)
{
    FastDiv f;
    f.d = d;
    f.pad = 0;
    f.m = ((uint64_t(1) << 40) + d - 1) / d;
    return f;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t x, const FastDiv &f)
{
    return uint32_t((uint64_t(x) * f.m) >> 40);
}

// One 1-D complex transform of length n as a sequence of Stockham stages.
// Stage s has radix radix[s]; ns[s] is the product of the radices before it;
// the twiddle of butterfly position k, output q is W_n^(q*k*twstride[s]),
// read from the length-n table at tw_off (W_n^t = exp(-2 pi i t / n)).
struct AxisPlan {
    int32_t n;
    int32_t nstages;
    int32_t tw_off;  // complex-element offset of this length's table
    int32_t cplan;   // entry of the compiled plan table in use, or -1
    int32_t radix[kMaxStages];
    int32_t twstride[kMaxStages];
    FastDiv ns[kMaxStages];
};

struct ProbDesc {
    AxisPlan ax[3];     // transform plans along a, b, c
    int32_t dims[4];    // Na, Nb, Nc, Nh = Nc/2 + 1
    FastDiv div_nh;     // Nh
    FastDiv div_nc;     // Nc
    int64_t grid_off;   // element offset of this problem's real grid
    int64_t spec_off;   // complex-element offset of its half spectrum in the workspace
    int64_t npts;       // Na * Nb * Nc
    double B[9];        // reciprocal rows b_d (a_i . b_j = 2 pi delta_ij)
    float Bf[9];
    int32_t ortho;      // 1 when the cell is diagonal
    double inv_n;       // 1 / npts
    double eh_scale;    // Omega / (2 npts^2)
    double dv;          // Omega / npts
    double L[3];        // cell edges (orthorhombic cells)
    double h[3];        // grid spacing L / N per axis (orthorhombic cells)
    float hf[3];        // h as a float ...
    float hfl[3];       // ... and the float of its remainder h - hf
    double A[9];        // cell rows a, b, c (any cell)
    int32_t separable;  // 1: diagonal cell with positive edges (separable splat)
    int32_t pad4;
    int32_t part_off;   // first E_H partial slot of this problem
    int32_t nparts;     // number of E_H partial slots
    int64_t brick_off;  // first brick of this problem (splat bins)
    int32_t nbricks[3]; // bricks per axis
    int32_t pad2;
    int32_t bsz[3];     // brick edge in grid points per axis
    int32_t pad3;
};

// Splat bricks, one workgroup each: MI x MJ x MK grid points for the
// matrix-core kernels (diagonal cells), BI x BJ x BK for the FP64
// point-by-point kernels of any other cell.
constexpr int kBI = 8, kBJ = 8, kBK = 32;
constexpr int kMI = 16, kMJ = 16, kMK = 32;

// Per-atom data prepared on the device before binning.
struct AtomInfo {
    double X[3];     // position wrapped into [0, L)
    double w;        // Z (2 pi s^2)^(-3/2)
    double inv2s2;   // 1 / (2 s^2)
    int32_t lo[3];   // unwrapped first grid index of the truncation window per axis
    int32_t hi[3];   // unwrapped last grid index
    int32_t st[3];   // first brick the window touches per axis ...
    int32_t ct[3];   // ... and the number of bricks it touches (0 for an invalid atom)
    int32_t prob;    // problem index (batched plans)
    int32_t pad;
};

// One atom in one brick's sorted list, as the FP32 splat kernels use it
// (written by the binning sort): along axis x the brick's first point lies
// at offset r0[x] (mod n) from the window start lo; an unwrapped offset r
// inside the window width wl has displacement r h - xb, xb = X - lo h.
// One axis of an atom relative to a brick (16 bytes: one vector load).
struct SlotAxis {
    float xb;    // X - lo h, rounded to float ...
    float xbl;   // ... and the rounding remainder (xb + xbl = X - lo h to double accuracy)
    int32_t r0;  // offset of the brick's first point from the window start, mod n
    int32_t wl;  // window width in points; 0 for an atom that touches nothing
};

struct SlotAtom {
    SlotAxis ax[3];
    float c2;       // log2(e) / (2 sigma^2): the 1-D factor is 2^(-d^2 c2)
    float w;        // Z (2 pi sigma^2)^(-3/2)
    int32_t atom;   // the atom's index ...
    int32_t touch;  // ... and this brick's place in its enumeration of touched bricks
};

// The same for the FP64 splat kernels, in double precision: the unwrapped
// offset r has grid index lo + r and displacement (lo + r) h - X.
struct SlotAtom64 {
    double X[3];     // the wrapped position per axis
    double inv2s2;   // 1 / (2 sigma^2): the 1-D factor is exp(-d^2 inv2s2)
    double w;        // Z (2 pi sigma^2)^(-3/2)
    int32_t lo[3];   // window start per axis (unwrapped grid index)
    int32_t r0[3];   // offset of the brick's first point from the window start, mod n
    int32_t wl[3];   // window width in points; 0 for an atom that touches nothing
    int32_t atom;    // the atom's index ...
    int32_t touch;   // ... and this brick's place in its enumeration of touched bricks
    int32_t pad;
};

struct DeviceStatus {
    uint32_t bits;
    uint32_t pad[63];
};

}  // namespace hartree
