// Host-side dispatch of the grid passes and the E_H finalize kernel.
#include "fft_passes.hpp"

namespace hartree {

hipError_t run_r2c_f32(int, int, int, hipStream_t, const PassArgs &);
hipError_t run_r2c_f64(int, int, int, hipStream_t, const PassArgs &);
hipError_t run_c2r_f32(int, int, int, hipStream_t, const PassArgs &);
hipError_t run_c2r_f64(int, int, int, hipStream_t, const PassArgs &);
hipError_t run_b_f32(int, int, int, hipStream_t, const PassArgs &);
hipError_t run_b_f64(int, int, int, hipStream_t, const PassArgs &);
hipError_t run_a_f32(int, int, int, hipStream_t, const PassArgs &);
hipError_t run_a_f64(int, int, int, hipStream_t, const PassArgs &);

// ---------------------------------------------------------------- E_H
// one workgroup per problem: fixed-order sum of that problem's partials
// one workgroup per problem: each thread sums its strided share of the
// partials in four independent chains (the loads issue together), then a
// fixed butterfly per wavefront and a fixed-order sum over the wavefronts
constexpr int kFinThreads = 1024;

__global__ __launch_bounds__(kFinThreads) void k_finalize(const ProbDesc *desc, const double *partials, double *e_h)
{
    __shared__ double red[kFinThreads / 64];
    const ProbDesc &d = desc[blockIdx.x];
    const double *pp = partials + d.part_off;
    const int t = threadIdx.x;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int i = t;
    for (; i + 3 * kFinThreads < d.nparts; i += 4 * kFinThreads) {
        s0 += pp[i];
        s1 += pp[i + kFinThreads];
        s2 += pp[i + 2 * kFinThreads];
        s3 += pp[i + 3 * kFinThreads];
    }
    for (; i < d.nparts; i += kFinThreads) s0 += pp[i];
    double s = (s0 + s1) + (s2 + s3);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((t & 63) == 0) red[t >> 6] = s;
    __syncthreads();
    if (t == 0) {
        double tot = 0.0;
        for (int w = 0; w < kFinThreads / 64; ++w) tot += red[w];
        e_h[blockIdx.x] = d.eh_scale * tot;
    }
}

// Pencils per workgroup for a length and its stage radices (log2; -1 if the
// length does not fit): enough threads per pencil that every stage's
// butterflies fit the registers, at most 64 pencils, and a tile that leaves
// room for two workgroups per CU.
int pass_min_tpp(int fp64, int n, const int *radix, int nstages)
{
    int tpp = 1;
    for (int s = 0; s < nstages; ++s) {
        const int nb = n / radix[s];
        const int mb = fp64 ? stage_maxb<double>(radix[s]) : stage_maxb<float>(radix[s]);
        const int need = (nb + mb - 1) / mb;
        while (tpp < need) tpp <<= 1;
    }
    return tpp;
}

size_t pass_tile_lds(int fp64, int n, int p_log2, int pad)
{
    const size_t P = size_t(1) << p_log2, cx = fp64 ? 16 : 8;
    const size_t strided = (P + size_t(pad)) * n, rows = P * (n + 31);
    return cx * ((strided > rows ? strided : rows) + n);
}

// Bank-conflict model of the strided tiles (element (i, p) at i (P + pad) + p):
// for every LDS access of every stage, the passes a wavefront needs on 64
// banks of 4 bytes, relative to the conflict-free count.
static double strided_lds_cost(int fp64, int n, const int *radix, int nstages, int p_log2, int pad)
{
    const int P = 1 << p_log2, tpp = kPassThreads >> p_log2, pitch = P + pad, wpe = fp64 ? 4 : 2;
    double total = 0.0, ideal = 0.0;
    int ns = 1;
    int count[64];
    for (int st = 0; st < nstages; ++st) {
        const int R = radix[st], nb = n / R, maxb = (nb + tpp - 1) / tpp;
        for (int wave = 0; wave < kPassThreads / 64; ++wave)
            for (int m = 0; m < maxb; ++m)
                for (int dir = 0; dir < 2; ++dir)
                    for (int q = 0; q < R; ++q) {
                        for (int b = 0; b < 64; ++b) count[b] = 0;
                        int lanes = 0;
                        for (int l = 0; l < 64; ++l) {
                            const int tid = wave * 64 + l, p = tid & (P - 1), tip = tid >> p_log2;
                            const int j = tip + m * tpp;
                            if (j >= nb) continue;
                            const int i = dir == 0 ? j + q * nb : (j / ns) * ns * R + j % ns + q * ns;
                            const long w0 = long(i * pitch + p) * wpe;
                            for (int k = 0; k < wpe; ++k) count[(w0 + k) & 63] += 1;
                            ++lanes;
                        }
                        if (!lanes) continue;
                        int mx = 0;
                        for (int b = 0; b < 64; ++b) mx = count[b] > mx ? count[b] : mx;
                        total += mx;
                        ideal += (lanes * wpe + 63) / 64;
                    }
        ns *= R;
    }
    return ideal > 0.0 ? total / ideal : 1.0;
}

int pass_default_pad(int fp64, int n, const int *radix, int nstages, int p_log2)
{
    int best = 1;
    double cbest = 0.0;
    for (int pad = 0; pad <= 3; ++pad) {
        const double c = strided_lds_cost(fp64, n, radix, nstages, p_log2, pad);
        if (pad == 0 || c < cbest - 1e-9) {
            cbest = c;
            best = pad;
        }
    }
    return best;
}

int pass_p_log2(int fp64, int n, const int *radix, int nstages, int max_p)
{
    const int tpp = pass_min_tpp(fp64, n, radix, nstages);
    if (tpp > kPassThreads) return -1;
    int P = kPassThreads / tpp;
    if (P > max_p) P = max_p;
    const size_t cx = fp64 ? 16 : 8;
    while (P > 1 && size_t(row_pitch(n) > n + 1 ? row_pitch(n) : n + 1) * (P + 1) * cx > 80 * 1024) P >>= 1;
    int l = 0;
    while ((1 << l) < P) ++l;
    return l;
}

#define HARTREE_ROW(R0, R1, R2, R3) {R0, R1, R2, R3},
static const int kPlanTable[][4] = {HARTREE_PLANS(HARTREE_ROW)};
#undef HARTREE_ROW

int plan_table_size() { return int(sizeof(kPlanTable) / sizeof(kPlanTable[0])); }

int plan_table_row(int id, int *radix)
{
    int ns = 0;
    for (int s = 0; s < 4; ++s) {
        radix[s] = kPlanTable[id][s];
        if (radix[s] > 0) ns = s + 1;
    }
    return ns;
}

// index of a radix sequence in HARTREE_PLANS, or -1
int find_plan(const int *radix, int nstages)
{
    const auto &plans = kPlanTable;
    const int np = plan_table_size();
    for (int i = 0; i < np; ++i) {
        bool same = true;
        for (int s = 0; s < 4; ++s) same = same && plans[i][s] == (s < nstages ? radix[s] : 0);
        if (same && nstages <= 4) return i;
    }
    return -1;
}

hipError_t run_pass(int fp64, PassKind kind, int plan, int p_log2, int pad, int maxn, int grid, hipStream_t s,
                    const PassArgs &a0)
{
    PassArgs a = a0;
    a.mode = 0;
    a.inv = 0;
    a.p_log2 = p_log2;
    a.pad = pad;
    switch (kind) {
    case PASS_R2C_FWD: return fp64 ? run_r2c_f64(plan, maxn, grid, s, a) : run_r2c_f32(plan, maxn, grid, s, a);
    case PASS_R2C_BWD:
        a.mode = 1;
        return fp64 ? run_r2c_f64(plan, maxn, grid, s, a) : run_r2c_f32(plan, maxn, grid, s, a);
    case PASS_C2R: return fp64 ? run_c2r_f64(plan, maxn, grid, s, a) : run_c2r_f32(plan, maxn, grid, s, a);
    case PASS_B_FWD: return fp64 ? run_b_f64(plan, maxn, grid, s, a) : run_b_f32(plan, maxn, grid, s, a);
    case PASS_B_INV:
        a.inv = 1;
        return fp64 ? run_b_f64(plan, maxn, grid, s, a) : run_b_f32(plan, maxn, grid, s, a);
    case PASS_A_FULL: return fp64 ? run_a_f64(plan, maxn, grid, s, a) : run_a_f32(plan, maxn, grid, s, a);
    case PASS_A_NOENERGY:
        a.mode = 1;
        return fp64 ? run_a_f64(plan, maxn, grid, s, a) : run_a_f32(plan, maxn, grid, s, a);
    default:
        a.mode = 2;
        return fp64 ? run_a_f64(plan, maxn, grid, s, a) : run_a_f32(plan, maxn, grid, s, a);
    }
}

__global__ void k_zero_bytes(uint32_t *p, size_t nwords)
{
    for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < nwords; i += size_t(gridDim.x) * blockDim.x)
        p[i] = 0u;
}

// zero a device array (byte count a multiple of 4) with a kernel
hipError_t run_zero(void *p, size_t bytes, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_bytes, dim3(2048), dim3(256), 0, s, static_cast<uint32_t *>(p), bytes / 4);
    return hipGetLastError();
}

hipError_t run_finalize(const ProbDesc *desc, const double *partials, double *e_h, int nprob, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize, dim3(nprob), dim3(kFinThreads), 0, s, desc, partials, e_h);
    return hipGetLastError();
}

}  // namespace hartree
