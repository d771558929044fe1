// FP32 splat and splat adjoint on the matrix cores (v_mfma_f32_32x32x2f32).
//
// Inside one brick (8 x 8 columns (i, j) by 32 points along c) both
// operations are dense contractions over the brick's atom list:
//
//   splat    rho[c][k]  = sum_a  W_a gx_a(i_c) gy_a(j_c)  *  gz_a(k)
//            (columns x atoms) . (atoms x k)
//   adjoint  S[c][a, f] = sum_k  grho[c][k]  *  gz_a(k) (f = 0) or gdz_a(k) (f = 1)
//            (columns x k) . (k x atom functions), then per atom
//            F_a = sum_c [gdx gy S0, gx gdy S0, gx gy S1]
//
// with the per-axis factors gx, gdx, ... of the VALU kernels (1-D periodic
// Gaussians and their displacement-weighted sums).  Each wavefront owns one
// 32-column half of the brick (and, for the adjoint, one column tile).
//
// Operand layout of v_mfma_f32_32x32x2f32 (C = A B + C, A 32x2, B 2x32):
// lane l supplies A[l % 32][l / 32] and B[l / 32][l % 32]; after the call
// lane l holds C[i][l % 32] for i = 8 (r / 4) + 4 (l / 32) + r % 4 in its
// accumulator element r = 0 .. 15.
#include "splat_common.hpp"

namespace hartree {

typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ int mfma_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

// brick index with consecutive bricks (which share cache lines at their
// edges along c) kept on one XCD
__device__ __forceinline__ int64_t brick_of_block() { return xcd_remap(blockIdx.x, gridDim.x); }

// Atoms are staged in groups of up to kGroup (global loads and table
// evaluation once per group, then the group's matrix work).  Four
// wavefronts per brick; table rows are padded to an odd number of words.
constexpr int kBrickWaves = 4;
constexpr int kSplatThreads = 64 * kBrickWaves;
constexpr int kGroup = 32;

// splat: wave w computes brick columns 32 (w & 1) .. +31 over the atom pairs
// with (pair index & 1) == (w >> 1); the two halves are summed at the end
__global__ __launch_bounds__(kSplatThreads) void k_splat_mfma(SplatArgs a)
{
    __shared__ StagedAtom atoms[kGroup];
    __shared__ float gxw[kGroup][kBI + 1], gy[kGroup][kBJ + 1];
    __shared__ float gz[kGroup][kBK];
    __shared__ float part[2][64][17];  // accumulators of the odd-pair waves
    const int64_t b = brick_of_block();
    const int prob = brick_prob(a, b);
    const ProbDesc &d = a.desc[prob];
    const int lb = int(b - d.brick_off);  // bricks of one problem fit 32 bits
    const int bk = lb % d.nbricks[2];
    const int bij = lb / d.nbricks[2];
    const int bj = bij % d.nbricks[1];
    const int bi = bij / d.nbricks[1];
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    const int mt = wave & 1, kh = wave >> 1;
    const int64_t off = a.offsets[b];
    const int cnt = int(a.offsets[b + 1] - off);
    // this lane's A row: brick column c = 32 mt + lane % 32
    const int ca = 32 * mt + (lane & 31);
    const int ci = ca >> 3, cj = ca & 7;
    const int kk = lane >> 5;

    floatx16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;

    for (int c0 = 0; c0 < cnt; c0 += kGroup) {
        const int ns = (cnt - c0) < kGroup ? (cnt - c0) : kGroup;
        stage_atoms(atoms, a, d, off, c0, ns, t);
        __syncthreads();
        for (int e = t; e < ns * (kBI + kBJ + kBK); e += kSplatThreads) {
            const int s = e / (kBI + kBJ + kBK), q = e % (kBI + kBJ + kBK);
            const StagedAtom &in = atoms[s];
            if (q < kBI) {
                gxw[s][q] = table_factor<float>(a, bi * kBI + q, d.dims[0], in, 0).x * float(in.w);
            } else if (q < kBI + kBJ) {
                const int qq = q - kBI;
                gy[s][qq] = table_factor<float>(a, bj * kBJ + qq, d.dims[1], in, 1).x;
            } else {
                const int qq = q - kBI - kBJ;
                gz[s][qq] = table_factor<float>(a, bk * kBK + qq, d.dims[2], in, 2).x;
            }
        }
        __syncthreads();
        for (int s0 = 2 * kh; s0 < ns; s0 += 4) {
            const int s = s0 + kk;
            const float av = (s < ns) ? gxw[s][ci] * gy[s][cj] : 0.0f;
            const float bv = (s < ns) ? gz[s][lane & 31] : 0.0f;
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    if (kh == 1) {
#pragma unroll
        for (int r = 0; r < 16; ++r) part[mt][lane][r] = acc[r];
    }
    __syncthreads();
    if (kh == 1) return;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] += part[mt][lane][r];
    const float bg = a.subtract_background ? float(a.qsum[prob] / (d.L[0] * d.L[1] * d.L[2])) : 0.0f;
    const int k = bk * kBK + (lane & 31);
    if (k >= d.dims[2]) return;
    float *out = reinterpret_cast<float *>(a.rho) + d.grid_off;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int c = 32 * mt + mfma_row(r, lane);
        const int i = bi * kBI + (c >> 3), j = bj * kBJ + (c & 7);
        if (i < d.dims[0] && j < d.dims[1]) out[(int64_t(i) * d.dims[1] + j) * d.dims[2] + k] = acc[r] - bg;
    }
}

constexpr int kAdjTile = 16;                   // atoms per MFMA column tile: 16 atoms x (gz, gdz)
constexpr int kAdjTiles = kGroup / kAdjTile;   // column tiles per group (2)

// adjoint: wave w computes the 32x32 tile (columns 32 (w & 1) .., column
// tile w >> 1) of S[c][n], n = (f, atom) = 16 f + atom
__global__ __launch_bounds__(kSplatThreads) void k_adjoint_mfma(SplatArgs a)
{
    __shared__ StagedAtom atoms[kGroup];
    __shared__ float gr[kBI * kBJ][kBK + 1];                 // brick of grad_rho, padded rows
    __shared__ float gzt[kAdjTiles][2 * kAdjTile][kBK + 1];  // per tile: gz (f = 0) and gdz (f = 1) rows
    __shared__ float gx[kGroup][kBI + 1], gdx[kGroup][kBI + 1], gy[kGroup][kBJ + 1], gdy[kGroup][kBJ + 1];
    __shared__ float red[kAdjTiles][2][2][kAdjTile][3];      // [tile][column half][lane half][atom][x]
    const int64_t b = brick_of_block();
    const int prob = brick_prob(a, b);
    const ProbDesc &d = a.desc[prob];
    const int lb = int(b - d.brick_off);  // bricks of one problem fit 32 bits
    const int bk = lb % d.nbricks[2];
    const int bij = lb / d.nbricks[2];
    const int bj = bij % d.nbricks[1];
    const int bi = bij / d.nbricks[1];
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    const int mt = wave & 1, tile = wave >> 1;
    const int64_t off = a.offsets[b];
    const int cnt = int(a.offsets[b + 1] - off);
    if (cnt == 0) return;

    // grad_rho brick: 64 rows of 32 consecutive points
    {
        const float *src = reinterpret_cast<const float *>(a.grad_rho) + d.grid_off;
        for (int e = t; e < kBI * kBJ * kBK; e += kSplatThreads) {
            const int c = e >> 5, k = e & 31;
            const int i = bi * kBI + (c >> 3), j = bj * kBJ + (c & 7), kg = bk * kBK + k;
            float v = 0.0f;
            if (i < d.dims[0] && j < d.dims[1] && kg < d.dims[2])
                v = src[(int64_t(i) * d.dims[1] + j) * d.dims[2] + kg];
            gr[c][k] = v;
        }
    }
    const int n = lane & 31;              // this lane's C column: f = n / 16, atom n % 16
    const int ca = 32 * mt + (lane & 31); // this lane's A row (brick column)
    const int kk = lane >> 5;
    const int f = n >> 4, sl = n & 15, half = lane >> 5;

    for (int c0 = 0; c0 < cnt; c0 += kGroup) {
        const int ns = (cnt - c0) < kGroup ? (cnt - c0) : kGroup;
        const int ntile = (ns + kAdjTile - 1) / kAdjTile;
        stage_atoms(atoms, a, d, off, c0, ns, t);
        __syncthreads();
        for (int e = t; e < ntile * kAdjTile * (kBI + kBJ + kBK); e += kSplatThreads) {
            const int s = e / (kBI + kBJ + kBK), q = e % (kBI + kBJ + kBK);
            const int tl = s / kAdjTile, st = s % kAdjTile;
            Cx<float> v{0.0f, 0.0f};
            if (q < kBI) {
                if (s < ns) v = table_factor<float>(a, bi * kBI + q, d.dims[0], atoms[s], 0);
                gx[s][q] = v.x;
                gdx[s][q] = v.y;
            } else if (q < kBI + kBJ) {
                const int qq = q - kBI;
                if (s < ns) v = table_factor<float>(a, bj * kBJ + qq, d.dims[1], atoms[s], 1);
                gy[s][qq] = v.x;
                gdy[s][qq] = v.y;
            } else {
                // padded atom slots give zero columns
                const int qq = q - kBI - kBJ;
                if (s < ns) v = table_factor<float>(a, bk * kBK + qq, d.dims[2], atoms[s], 2);
                gzt[tl][st][qq] = v.x;
                gzt[tl][kAdjTile + st][qq] = v.y;
            }
        }
        __syncthreads();
        if (tile < ntile) {
            floatx16 acc;
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
            for (int k0 = 0; k0 < kBK; k0 += 2) {
                const float av = gr[ca][k0 + kk];
                const float bv = gzt[tile][n][k0 + kk];
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
            }
            // lane holds S[c][n] for 16 columns c; fold in the transverse factors
            const int s = tile * kAdjTile + sl;
            float fx = 0.0f, fy = 0.0f, fz = 0.0f;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int c = 32 * mt + mfma_row(r, lane);
                const int ci = c >> 3, cj = c & 7;
                const float v = acc[r];
                if (f == 0) {
                    fx += gdx[s][ci] * gy[s][cj] * v;
                    fy += gx[s][ci] * gdy[s][cj] * v;
                } else {
                    fz += gx[s][ci] * gy[s][cj] * v;
                }
            }
            // lanes n and n + 16 (f = 0, 1) of each half carry the same atom
            if (f == 0) {
                red[tile][mt][half][sl][0] = fx;
                red[tile][mt][half][sl][1] = fy;
            } else {
                red[tile][mt][half][sl][2] = fz;
            }
        }
        __syncthreads();
        for (int e = t; e < ns * 3; e += kSplatThreads) {
            const int s2 = e / 3, x = e % 3;
            const int tl = s2 / kAdjTile, st = s2 % kAdjTile;
            const double v = (double(red[tl][0][0][st][x]) + double(red[tl][0][1][st][x])) +
                             (double(red[tl][1][0][st][x]) + double(red[tl][1][1][st][x]));
            const int64_t slot = off + c0 + s2;
            if (slot < a.capacity) a.bpart[slot * 3 + x] = v;
        }
        __syncthreads();
    }
}

hipError_t run_gather_mfma(const SplatArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_splat_mfma, dim3(int(a.nbricks_total)), dim3(kSplatThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t run_adjoint_mfma(const SplatArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_adjoint_mfma, dim3(int(a.nbricks_total)), dim3(kSplatThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace hartree
