// FP32 instantiations of the fused sweep.
#include "launch.hpp"

namespace vdwlb {
hipError_t launch_sweep_f32(const vdwlb_plan& p, const void* fin, void* fout, hipStream_t s, void* mom) {
    return run_sweep_typed<float>(p, fin, fout, s, mom);
}
}  // namespace vdwlb
