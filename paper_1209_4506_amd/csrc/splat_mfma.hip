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
// 32-column half of the brick.
//
// Operand layout of v_mfma_f32_32x32x2f32 (C = A B + C, A 32x2, B 2x32):
// lane l supplies A[l % 32][l / 32] and B[l / 32][l % 32]; after the call
// lane l holds C[i][l % 32] for i = 8 (r / 4) + 4 (l / 32) + r % 4 in its
// accumulator element r = 0 .. 15.
#include "splat_common.hpp"

namespace hartree {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kMfmaThreads = 128;  // two wavefronts per brick

__device__ __forceinline__ int mfma_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

// splat: atoms in chunks of 32, two per MFMA step
__global__ __launch_bounds__(kMfmaThreads) void k_splat_mfma(SplatArgs a)
{
    __shared__ StagedAtom atoms[kChunk];
    __shared__ float gxw[kChunk][kBI], gy[kChunk][kBJ];
    __shared__ float gz[kChunk][kBK];
    const int64_t b = blockIdx.x;
    const int prob = brick_prob(a, b);
    const ProbDesc &d = a.desc[prob];
    const int64_t lb = b - d.brick_off;
    const int bk = int(lb % d.nbricks[2]);
    const int bj = int((lb / d.nbricks[2]) % d.nbricks[1]);
    const int bi = int(lb / (int64_t(d.nbricks[2]) * d.nbricks[1]));
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    const int64_t off = a.offsets[b];
    const int cnt = int(a.offsets[b + 1] - off);
    const double h[3] = {d.L[0] / d.dims[0], d.L[1] / d.dims[1], d.L[2] / d.dims[2]};
    // this lane's A row: brick column c = 32 wave + lane % 32
    const int ca = 32 * wave + (lane & 31);
    const int ci = ca >> 3, cj = ca & 7;
    const int kk = lane >> 5;

    floatx16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;

    for (int c0 = 0; c0 < cnt; c0 += kChunk) {
        const int nc = (cnt - c0) < kChunk ? (cnt - c0) : kChunk;
        stage_atoms(atoms, a, d, off, c0, nc, t);
        __syncthreads();
        for (int e = t; e < nc * (kBI + kBJ + kBK); e += kMfmaThreads) {
            const int s = e / (kBI + kBJ + kBK), q = e % (kBI + kBJ + kBK);
            const StagedAtom &in = atoms[s];
            float g, gd;
            if (q < kBI) {
                staged_factor<float, false>(bi * kBI + q, d.dims[0], h[0], in, 0, g, gd);
                gxw[s][q] = g * float(in.w);
            } else if (q < kBI + kBJ) {
                const int qq = q - kBI;
                staged_factor<float, false>(bj * kBJ + qq, d.dims[1], h[1], in, 1, g, gd);
                gy[s][qq] = g;
            } else {
                const int qq = q - kBI - kBJ;
                staged_factor<float, false>(bk * kBK + qq, d.dims[2], h[2], in, 2, g, gd);
                gz[s][qq] = g;
            }
        }
        __syncthreads();
        for (int s0 = 0; s0 < nc; s0 += 2) {
            const int s = s0 + kk;
            const float av = (s < nc) ? gxw[s][ci] * gy[s][cj] : 0.0f;
            const float bv = (s < nc) ? gz[s][lane & 31] : 0.0f;
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    const float bg = a.subtract_background ? float(a.qsum[prob] / (d.L[0] * d.L[1] * d.L[2])) : 0.0f;
    const int k = bk * kBK + (lane & 31);
    if (k >= d.dims[2]) return;
    float *out = reinterpret_cast<float *>(a.rho) + d.grid_off;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int c = 32 * wave + mfma_row(r, lane);
        const int i = bi * kBI + (c >> 3), j = bj * kBJ + (c & 7);
        if (i < d.dims[0] && j < d.dims[1]) out[(int64_t(i) * d.dims[1] + j) * d.dims[2] + k] = acc[r] - bg;
    }
}

constexpr int kAdjChunk = 16;  // atoms per MFMA column tile: 16 atoms x (gz, gdz)

// adjoint: per chunk of 16 atoms one 32x32 tile per wavefront,
// S[c][n] with n = (f, atom) = 16 f + atom
__global__ __launch_bounds__(kMfmaThreads) void k_adjoint_mfma(SplatArgs a)
{
    __shared__ StagedAtom atoms[kAdjChunk];
    __shared__ float gr[kBI * kBJ][kBK + 1];          // brick of grad_rho, padded rows
    __shared__ float gzt[2 * kAdjChunk][kBK + 1];     // gz (f = 0) and gdz (f = 1) rows
    __shared__ float gx[kAdjChunk][kBI], gdx[kAdjChunk][kBI], gy[kAdjChunk][kBJ], gdy[kAdjChunk][kBJ];
    __shared__ float red[2][2][kAdjChunk][3];         // [wave][half][atom][x]
    const int64_t b = blockIdx.x;
    const int prob = brick_prob(a, b);
    const ProbDesc &d = a.desc[prob];
    const int64_t lb = b - d.brick_off;
    const int bk = int(lb % d.nbricks[2]);
    const int bj = int((lb / d.nbricks[2]) % d.nbricks[1]);
    const int bi = int(lb / (int64_t(d.nbricks[2]) * d.nbricks[1]));
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    const int64_t off = a.offsets[b];
    const int cnt = int(a.offsets[b + 1] - off);
    if (cnt == 0) return;
    const double h[3] = {d.L[0] / d.dims[0], d.L[1] / d.dims[1], d.L[2] / d.dims[2]};

    // grad_rho brick: 64 rows of 32 consecutive points
    {
        const float *src = reinterpret_cast<const float *>(a.grad_rho) + d.grid_off;
        for (int e = t; e < kBI * kBJ * kBK; e += kMfmaThreads) {
            const int c = e >> 5, k = e & 31;
            const int i = bi * kBI + (c >> 3), j = bj * kBJ + (c & 7), kg = bk * kBK + k;
            float v = 0.0f;
            if (i < d.dims[0] && j < d.dims[1] && kg < d.dims[2])
                v = src[(int64_t(i) * d.dims[1] + j) * d.dims[2] + kg];
            gr[c][k] = v;
        }
    }
    const int n = lane & 31;            // this lane's C column: f = n / 16, atom n % 16
    const int ca = 32 * wave + (lane & 31);  // this lane's A row (brick column)
    const int kk = lane >> 5;

    for (int c0 = 0; c0 < cnt; c0 += kAdjChunk) {
        const int nc = (cnt - c0) < kAdjChunk ? (cnt - c0) : kAdjChunk;
        stage_atoms(atoms, a, d, off, c0, nc, t);
        __syncthreads();
        for (int e = t; e < nc * (kBI + kBJ + kBK); e += kMfmaThreads) {
            const int s = e / (kBI + kBJ + kBK), q = e % (kBI + kBJ + kBK);
            const StagedAtom &in = atoms[s];
            float g, gd;
            if (q < kBI) {
                staged_factor<float, true>(bi * kBI + q, d.dims[0], h[0], in, 0, g, gd);
                gx[s][q] = g;
                gdx[s][q] = gd;
            } else if (q < kBI + kBJ) {
                const int qq = q - kBI;
                staged_factor<float, true>(bj * kBJ + qq, d.dims[1], h[1], in, 1, g, gd);
                gy[s][qq] = g;
                gdy[s][qq] = gd;
            } else {
                const int qq = q - kBI - kBJ;
                staged_factor<float, true>(bk * kBK + qq, d.dims[2], h[2], in, 2, g, gd);
                gzt[s][qq] = g;
                gzt[kAdjChunk + s][qq] = gd;
            }
        }
        // unused atom slots of the last chunk contribute zero columns
        for (int e = t; e < (kAdjChunk - nc) * kBK; e += kMfmaThreads) {
            const int s = nc + e / kBK, q = e % kBK;
            gzt[s][q] = 0.0f;
            gzt[kAdjChunk + s][q] = 0.0f;
        }
        __syncthreads();
        floatx16 acc;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
        for (int k0 = 0; k0 < kBK; k0 += 2) {
            const float av = gr[ca][k0 + kk];
            const float bv = gzt[n][k0 + kk];
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
        }
        // lane holds S[c][n] for 16 columns c; fold in the transverse factors
        const int f = n >> 4, s = n & 15;
        float fx = 0.0f, fy = 0.0f, fz = 0.0f;
        if (s < nc) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int c = 32 * wave + mfma_row(r, lane);
                const int ci = c >> 3, cj = c & 7;
                const float v = acc[r];
                if (f == 0) {
                    fx += gdx[s][ci] * gy[s][cj] * v;
                    fy += gx[s][ci] * gdy[s][cj] * v;
                } else {
                    fz += gx[s][ci] * gy[s][cj] * v;
                }
            }
        }
        // lanes n and n + 16 (f = 0, 1) of each half carry the same atom
        const int half = lane >> 5;
        if (f == 0) {
            red[wave][half][s][0] = fx;
            red[wave][half][s][1] = fy;
        } else {
            red[wave][half][s][2] = fz;
        }
        __syncthreads();
        for (int e = t; e < nc * 3; e += kMfmaThreads) {
            const int s2 = e / 3, x = e % 3;
            const double v = (double(red[0][0][s2][x]) + double(red[0][1][s2][x])) +
                             (double(red[1][0][s2][x]) + double(red[1][1][s2][x]));
            const int64_t slot = off + c0 + s2;
            if (slot < a.capacity) a.bpart[slot * 3 + x] = v;
        }
        __syncthreads();
    }
}

hipError_t run_gather_mfma(const SplatArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_splat_mfma, dim3(int(a.nbricks_total)), dim3(kMfmaThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t run_adjoint_mfma(const SplatArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_adjoint_mfma, dim3(int(a.nbricks_total)), dim3(kMfmaThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace hartree
