// rom_diag_f32_ang.hip -- dense-kernel instantiations of the FP32 row-lane sweep kernel
// (per-ordinate sources in, BF16 weighted angular flux out), compiled apart from the isotropic
// ones so the two build in parallel.  Each keeps its per-step source loads PD blocks ahead.
#include "rom_diag.h"

// blocks of per-step sources a dense-kernel wavefront keeps in flight, per ordinates per lane
#ifndef ROM_DIAG_ANG_PD1
#define ROM_DIAG_ANG_PD1 2
#endif
#ifndef ROM_DIAG_ANG_PD2
#define ROM_DIAG_ANG_PD2 2
#endif
#ifndef ROM_DIAG_ANG_PD4
#define ROM_DIAG_ANG_PD4 3  // c4 sweep 301 -> 292 us against 2 (4: 302 us); 251 VGPRs, no spill
#endif

namespace rom {

hipError_t launch_diag_f32_ang(const DiagArgs& a, int grid, int nb, int R, int K, hipStream_t s)
{
    constexpr int P1 = ROM_DIAG_ANG_PD1, P2 = ROM_DIAG_ANG_PD2, P4 = ROM_DIAG_ANG_PD4;
    if (R == 16) {
        if (K == 1) return launch_diag_t<float, 16, 1, P1, true>(a, grid, nb, s);
        if (K == 2) return launch_diag_t<float, 16, 2, P2, true>(a, grid, nb, s);
        if (K == 4) return launch_diag_t<float, 16, 4, P4, true>(a, grid, nb, s);
    } else if (R == 64) {
        if (K == 1) return launch_diag_t<float, 64, 1, P1, true>(a, grid, nb, s);
        if (K == 2) return launch_diag_t<float, 64, 2, P2, true>(a, grid, nb, s);
        if (K == 4) return launch_diag_t<float, 64, 4, P4, true>(a, grid, nb, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace rom
