// The coupled sweeps whose arithmetic is FP32 (FP32 and 16-bit shifted
// storage), in a translation unit of their own so that they are compiled with
// contraction of a*b+c into fused multiply-adds (-ffp-contract=on, within an
// expression); the FP64 sweeps in lbm_api.hip keep the rounding of the
// formulas as written.
#include <hip/hip_runtime.h>

#define LBM_SWEEPS_ONLY
#include "lbm_kernels.hpp"

namespace lbm {
#define LBM_INSTANTIATE_SWEEP(S, P) template void launch_sweep<S, P>(const SweepArgs<S> &, const SweepLaunch &, hipStream_t);
LBM_FP32_SWEEPS(LBM_INSTANTIATE_SWEEP)
#undef LBM_INSTANTIATE_SWEEP
template void launch_fused<StoreF32>(const SweepArgs<StoreF32> &, const SweepArgs<StoreF32> &, const SweepLaunch &,
                                     hipStream_t);
template void launch_naive_step<StoreF32>(const SweepArgs<StoreF32> &, const SweepArgs<StoreF32> &, int, hipStream_t);
#define LBM_INSTANTIATE_LATTICE(S)                                                                            \
    template void launch_fused<S>(const SweepArgs<S> &, const SweepArgs<S> &, const SweepLaunch &, hipStream_t); \
    template void launch_naive_step<S>(const SweepArgs<S> &, const SweepArgs<S> &, int, hipStream_t);
LBM_FP32_LATTICES(LBM_INSTANTIATE_LATTICE)
#undef LBM_INSTANTIATE_LATTICE
}  // namespace lbm
