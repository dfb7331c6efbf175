// rom_diag_f32.hip -- FP32 instantiations of the row-lane sweep kernel.  Bands of up to 8 row
// blocks keep the field loads two blocks ahead; 16-block bands (16 wavefronts, 128 VGPRs each)
// one block ahead.  The dense-kernel variants are in rom_diag_f32_ang.hip.
#include "rom_diag.h"

namespace rom {

hipError_t launch_diag_f32_ang(const DiagArgs& a, int grid, int nb, int R, int K, hipStream_t s);

hipError_t launch_diag_f32(const DiagArgs& a, int grid, int nb, int R, int K, bool ang, hipStream_t s)
{
    if (ang) return launch_diag_f32_ang(a, grid, nb, R, K, s);
    const bool deep = nb <= 8;
    if (R == 16) {
        if (K == 1) return deep ? launch_diag_t<float, 16, 1, 2>(a, grid, nb, s) : launch_diag_t<float, 16, 1, 1>(a, grid, nb, s);
        if (K == 2) return launch_diag_t<float, 16, 2, 2>(a, grid, nb, s);
        if (K == 4) return launch_diag_t<float, 16, 4, 2>(a, grid, nb, s);
    } else if (R == 64) {
        if (K == 1) return deep ? launch_diag_t<float, 64, 1, 2>(a, grid, nb, s) : launch_diag_t<float, 64, 1, 1>(a, grid, nb, s);
        if (K == 2) return launch_diag_t<float, 64, 2, 2>(a, grid, nb, s);
        if (K == 4) return launch_diag_t<float, 64, 4, 2>(a, grid, nb, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace rom
