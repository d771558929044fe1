// Launch interface between the host library and the kernels.
#pragma once

#include "common.hpp"

namespace hartree {

// Work items of one launch: tiles of several problems, concatenated.
struct TileList {
    int32_t count;                 // problems in this launch
    int32_t total;                 // total tiles
    int32_t prob[kMaxProb];
    int32_t start[kMaxProb + 1];   // prefix tile counts
};

enum PassKind {
    PASS_R2C_FWD,
    PASS_R2C_BWD,
    PASS_C2R,
    PASS_B_FWD,
    PASS_B_INV,
    PASS_A_FULL,
    PASS_A_NOENERGY,
    PASS_A_ENERGY
};

struct PassArgs {
    const ProbDesc *desc;
    const void *tw;        // twiddle tables (complex, plan precision)
    void *spec;            // half spectrum (workspace)
    const void *in;        // real-grid input of P1 (rho, or grad_v in the backward; nullable there)
    const void *in2;       // rho for the backward P1
    void *out;             // real-grid output of P5
    double *partials;      // E_H partial slots
    const double *grad_e;  // backward: dL/dE_H per problem (nullable)
    int32_t mode;          // P1: 0 forward, 1 backward;  P3: 0 energy + potential, 1 potential, 2 energy
    int32_t inv;           // P2/P4: 1 for the inverse transform
    int32_t p_log2;        // pencils per workgroup, log2
    int32_t pad;           // strided tiles (P2-P4): LDS pitch P + pad complex values per pencil element
    int64_t col_stride;    // strided passes: the largest pencil stride (elements) of the launch's problems
    TileList tl;
};

// Multi-plan launches (FP32): one launch per pass for the problems of a
// batched plan when each one's axis takes a compiled plan of the axis' list
// below (one per length from 32 to 240: the table's first 16 entries along a
// and b; along c the entries for 48, 128 and 160 without a radix-16 stage),
// with one common tile width of 2^multi_log_p(x, 0 or 1) pencils and
// no pitch pad; such a launch carries plan kMultiPlan.
constexpr int kMultiPlans = 16;
constexpr int kMultiPlansAB[kMultiPlans] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15};
constexpr int kMultiPlansC[kMultiPlans] = {0, 41, 2, 3, 4, 5, 6, 7, 42, 9, 43, 11, 12, 13, 14, 15};
// the two fixed tile widths (log2) of multi-plan launches along axis x: 8
// and 16 pencils along a and b, 4 and 8 along c
constexpr int multi_log_p(int x, int k) { return x == 2 ? 2 + k : 3 + k; }
constexpr int kMultiPlan = -2;
// A third multi-plan shape sizes the tile per length instead: the most
// pencils (a power of two, at most 64 along a and b, 32 along c) whose
// points stay within 4096 (a) or 2048 (b, c), at least 8 (a, b) or 4 (c);
// its launches carry p_log2 = kMultiAutoLog.
constexpr int kMultiAutoLog = 15;
constexpr int multi_auto_p(int n, int x)
{
    int p = x == 2 ? 32 : 64;
    const int lo = x == 2 ? 4 : 8, target = x == 0 ? 4096 : 2048;
    while (p > lo && p * n > target) p >>= 1;
    return p;
}
// the multi-plan list of axis x (0 = a, 1 = b, 2 = c)
inline const int *multi_plans(int x) { return x == 2 ? kMultiPlansC : kMultiPlansAB; }

int pass_p_log2(int fp64, int n, const int *radix, int nstages, int max_p);
int pass_min_tpp(int fp64, int n, const int *radix, int nstages);
size_t pass_tile_lds(int fp64, int n, int p_log2, int pad);
int pass_default_pad(int fp64, int n, const int *radix, int nstages, int p_log2);
int find_plan(const int *radix, int nstages);
int plan_table_size();
int plan_table_row(int id, int *radix);  // fills radix[4], returns the stage count
hipError_t run_pass(int fp64, PassKind kind, int plan, int p_log2, int pad, int maxn, int grid, hipStream_t s,
                    const PassArgs &a);
hipError_t run_finalize(const ProbDesc *desc, const double *partials, double *e_h, int nprob, hipStream_t s);
hipError_t run_zero(void *p, size_t bytes, hipStream_t s);

// ---------------------------------------------------------------- splat

struct SplatArgs {
    const ProbDesc *desc;
    int32_t nprob;
    int32_t natoms;
    int32_t atom_off[kMaxProb + 1];  // prefix atom counts per problem
    const double *pos;
    const double *Z;
    const double *sigma;
    double cutoff;          // truncation radius in sigmas
    double max_sigma;
    AtomInfo *info;         // natoms
    int32_t *counts;        // nbricks_total + 1
    int32_t *offsets;       // nbricks_total + 1
    int32_t *cursor;        // nbricks_total
    int32_t *list;          // capacity
    int32_t *list_sorted;   // capacity
    int32_t *slot_of;       // max_atoms x cap_pa: sorted-list slot of each (atom, touched brick)
    SlotAtom *rec;          // capacity (FP32 plans): the sorted lists' atoms relative to their brick
    SlotAtom64 *rec64;      // capacity (FP64 plans): the same in double precision
    int32_t *order;         // nbricks_total (batched plans): bricks by descending atom count, or nullptr
    double *bpart;          // capacity x 3 (adjoint partials): per list slot, or per (atom, touched brick)
                            // (atom * cap_pa + touch) where the per-slot records exist (rec or rec64)
    int64_t capacity;
    int32_t cap_pa;         // most bricks one atom can touch
    int64_t nbricks_total;
    DeviceStatus *status;
    int32_t subtract_background;
    int32_t fp64;
    int32_t general;        // 1: some cell is not diagonal-positive: the general-cell kernels run
    int32_t wide;           // 1: a truncation window may be wider than its cell (several images per point)
    int32_t visit_stride;   // coprime to natoms: binning visits atom (w * visit_stride) mod natoms
    int32_t b_exp;          // FP32 adjoint: the c-axis factors enter the 16-bit products scaled by 2^b_exp
    void *rho;              // splat output grid
    const void *grad_rho;   // adjoint input grid
    int32_t grad_rows_vec16;  // 16-byte grad_rho row loads: 0 none, 1 every problem's rows, 2 per problem (aligned start)
    const float *zeros;     // 64 zero floats in the workspace (never written by kernels)
    double *grad_pos;       // adjoint output
    double *qsum;           // 2 nprob: total charge per problem, then the largest atom weight per problem
};

hipError_t run_bin(const SplatArgs &a, hipStream_t s);
hipError_t run_gather(const SplatArgs &a, hipStream_t s);
hipError_t run_adjoint(const SplatArgs &a, hipStream_t s);
hipError_t run_adjoint_final(const SplatArgs &a, hipStream_t s);
hipError_t run_gather_mfma(const SplatArgs &a, hipStream_t s);
hipError_t run_adjoint_mfma(const SplatArgs &a, hipStream_t s);
hipError_t run_gather_mfma64(const SplatArgs &a, hipStream_t s);
hipError_t run_adjoint_mfma64(const SplatArgs &a, hipStream_t s);
hipError_t run_gather_general(const SplatArgs &a, hipStream_t s);
hipError_t run_adjoint_general(const SplatArgs &a, hipStream_t s);

}  // namespace hartree
