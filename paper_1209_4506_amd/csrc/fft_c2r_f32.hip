// P5 (c2r along c) kernels, FP32: one per radix plan of HARTREE_PLANS plus the run-time
// radix kernel (one translation unit per pass and precision so the build
// compiles them in parallel), and per plan kernels for tiles of 2, 4 and 8
// pencils whose tile shape and pencil length are compiled in.
#include "fft_passes.hpp"

namespace hartree {
namespace {
template <int R0, int R1, int R2, int R3, int CP>
hipError_t launch_one(int grid, size_t lds, hipStream_t s, const PassArgs &a)
{
    return launch_pass(k_c2r<float, R0, R1, R2, R3, CP>, grid, lds, s, a);
}
#define HARTREE_ENTRY(R0, R1, R2, R3) &launch_one<R0, R1, R2, R3, 0>,
const PassLaunchFn kTable[] = {HARTREE_PLANS(HARTREE_ENTRY)};
#undef HARTREE_ENTRY
#define HARTREE_ENTRY(R0, R1, R2, R3) &launch_one<R0, R1, R2, R3, 2>,
const PassLaunchFn kFixed2[] = {HARTREE_PLANS(HARTREE_ENTRY)};
#undef HARTREE_ENTRY
#define HARTREE_ENTRY(R0, R1, R2, R3) &launch_one<R0, R1, R2, R3, 4>,
const PassLaunchFn kFixed4[] = {HARTREE_PLANS(HARTREE_ENTRY)};
#undef HARTREE_ENTRY
#define HARTREE_ENTRY(R0, R1, R2, R3) &launch_one<R0, R1, R2, R3, 8>,
const PassLaunchFn kFixed8[] = {HARTREE_PLANS(HARTREE_ENTRY)};
#undef HARTREE_ENTRY
}  // namespace

hipError_t run_c2r_f32(int plan, int maxn, int grid, hipStream_t s, const PassArgs &a)
{
    const size_t lds = pass_lds_bytes<float>(a, maxn);
    if (plan == kMultiPlan) {
        // the multi-plan c2r tiles stage their rows in LDS (stage_lds)
        const size_t lds_staged = lds + stage_lds<float>(1 << (a.p_log2 & 7), maxn);
        if (a.p_log2 == multi_log_p(2, 0))
            return launch_pass(k_c2r_multi<float, 1 << multi_log_p(2, 0)>, grid, lds_staged, s, a);
        if (a.p_log2 == multi_log_p(2, 1))
            return launch_pass(k_c2r_multi<float, 1 << multi_log_p(2, 1)>, grid, lds_staged, s, a);
        if (a.p_log2 == kMultiAutoLog)
            return launch_pass(k_c2r_multi<float, 0>, grid, multi_auto_lds<float>(2, maxn, true), s, a);
        return hipErrorInvalidValue;
    }
    if (plan < 0 || plan >= int(sizeof(kTable) / sizeof(kTable[0])))
        return launch_one<0, 0, 0, 0, 0>(grid, lds, s, a);
    if (a.pad == 0 && a.p_log2 == 1) return kFixed2[plan](grid, lds, s, a);
    if (a.pad == 0 && a.p_log2 == 2) return kFixed4[plan](grid, lds, s, a);
    if (a.pad == 0 && a.p_log2 == 3) return kFixed8[plan](grid, lds, s, a);
    return kTable[plan](grid, lds, s, a);
}
}  // namespace hartree
