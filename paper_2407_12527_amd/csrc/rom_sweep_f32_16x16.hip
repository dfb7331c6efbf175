// rom_sweep_f32_16x16.hip -- instantiations of the sweep kernel.
#include "rom_sweep.h"

namespace rom {

hipError_t launch_sweep_f32_16x16(const SweepArgs& a, int grid, bool dd, bool ang, int psi, int L, int mom, hipStream_t s)
{
    return launch_sweep_tile<float, 16, 16>(a, grid, dd, ang, psi, L, mom, s);
}

}  // namespace rom
