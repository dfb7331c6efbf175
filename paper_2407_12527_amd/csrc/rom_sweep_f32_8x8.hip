// rom_sweep_f32_8x8.hip -- instantiations of the sweep kernel.
#include "rom_sweep.h"

namespace rom {

hipError_t launch_sweep_f32_8x8(const SweepArgs& a, int grid, bool dd, bool ang, int psi, int L, int mom, hipStream_t s)
{
    return launch_sweep_tile<float, 8, 8>(a, grid, dd, ang, psi, L, mom, s);
}

}  // namespace rom
