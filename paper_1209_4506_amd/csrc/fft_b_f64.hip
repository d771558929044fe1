// P2/P4 (FFT along b) kernels, FP64: one per radix plan of HARTREE_PLANS plus the run-time
// radix kernel (one translation unit per pass and precision so the build
// compiles them in parallel).
#include "fft_passes.hpp"

namespace hartree {
namespace {
template <int R0, int R1, int R2, int R3>
hipError_t launch_one(int grid, size_t lds, hipStream_t s, const PassArgs &a)
{
    return launch_pass(k_fft_b<double, R0, R1, R2, R3>, grid, lds, s, a);
}
#define HARTREE_ENTRY(R0, R1, R2, R3) &launch_one<R0, R1, R2, R3>,
const PassLaunchFn kTable[] = {HARTREE_PLANS(HARTREE_ENTRY)};
#undef HARTREE_ENTRY
}  // namespace

hipError_t run_b_f64(int plan, int maxn, int grid, hipStream_t s, const PassArgs &a)
{
    const size_t lds = pass_lds_bytes<double>(a, maxn);
    if (plan == kMultiPlan) return hipErrorInvalidValue;  // multi-plan launches are FP32 only
    if (plan < 0 || plan >= int(sizeof(kTable) / sizeof(kTable[0]))) return launch_one<0, 0, 0, 0>(grid, lds, s, a);
    return kTable[plan](grid, lds, s, a);
}
}  // namespace hartree
