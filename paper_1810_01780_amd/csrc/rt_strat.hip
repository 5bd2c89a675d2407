// The stratified trace kernel: trace_body (rt_trace.hpp) for media
// stratified in depth, where the trial step needs stage values of z, the
// vertical direction component and the travel time only (trial_strat).
// Compiled apart from the other kernels: its code generation keeps constant
// materialisations inside the step loop instead of hoisting them, which
// frees the registers they would hold (136 instead of 168 VGPRs, no
// spills) and measured 4 % faster on the two-layer workload, while the
// general kernel measured slower with it.
#include <hip/hip_runtime.h>

#include "rt_trace.hpp"

namespace rt {

// Three waves per SIMD: the LDS of a block (47 KB: the per-wave rings and the
// per-lane search state) allows no more.
template <int MODEL, bool EV>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
trace_strat_kernel(KParams P) {
  trace_body<MODEL, 0, EV>(P);
}

namespace {
template <int MODEL, bool EV>
int blocks_of(int block) {
  static thread_local int cached[5] = {};
  int& c = cached[block / 64];
  if (c == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void*>(&trace_strat_kernel<MODEL, EV>), block, 0) !=
            hipSuccess ||
        nb < 1)
      nb = 1;
    c = nb;
  }
  return c;
}
}  // namespace

int strat_blocks_per_cu(int model, bool ev, int block) {
  if (model == RT_MODEL_EXACT)
    return ev ? blocks_of<RT_MODEL_EXACT, true>(block) : blocks_of<RT_MODEL_EXACT, false>(block);
  return ev ? blocks_of<RT_MODEL_PAPER, true>(block) : blocks_of<RT_MODEL_PAPER, false>(block);
}

hipError_t launch_strat(int model, bool ev, const KParams& P, int grid, int block,
                        hipStream_t s) {
  if (model == RT_MODEL_EXACT) {
    if (ev)
      hipLaunchKernelGGL((trace_strat_kernel<RT_MODEL_EXACT, true>), dim3(grid), dim3(block), 0,
                         s, P);
    else
      hipLaunchKernelGGL((trace_strat_kernel<RT_MODEL_EXACT, false>), dim3(grid), dim3(block),
                         0, s, P);
  } else {
    if (ev)
      hipLaunchKernelGGL((trace_strat_kernel<RT_MODEL_PAPER, true>), dim3(grid), dim3(block), 0,
                         s, P);
    else
      hipLaunchKernelGGL((trace_strat_kernel<RT_MODEL_PAPER, false>), dim3(grid), dim3(block),
                         0, s, P);
  }
  return hipGetLastError();
}

}  // namespace rt
