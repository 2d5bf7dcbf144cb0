// FP64 instantiations of the fused sweep.
#include "launch.hpp"

namespace vdwlb {
hipError_t launch_sweep_f64(const vdwlb_plan& p, const void* fin, void* fout, hipStream_t s, void* mom) {
    return run_sweep_typed<double>(p, fin, fout, s, mom);
}
}  // namespace vdwlb
