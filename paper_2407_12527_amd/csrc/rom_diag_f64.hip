// rom_diag_f64.hip -- FP64 instantiations of the row-lane sweep kernel (see rom_diag_f32.hip).
#include "rom_diag.h"

namespace rom {

hipError_t launch_diag_f64(const DiagArgs& a, int grid, int nb, int R, int K, hipStream_t s)
{
    const bool deep = nb <= 8;
    if (R == 16) {
        if (K == 1) return deep ? launch_diag_t<double, 16, 1, 2>(a, grid, nb, s) : launch_diag_t<double, 16, 1, 1>(a, grid, nb, s);
        if (K == 2) return launch_diag_t<double, 16, 2, 2>(a, grid, nb, s);
    } else if (R == 64) {
        if (K == 1) return deep ? launch_diag_t<double, 64, 1, 2>(a, grid, nb, s) : launch_diag_t<double, 64, 1, 1>(a, grid, nb, s);
        if (K == 2) return launch_diag_t<double, 64, 2, 2>(a, grid, nb, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace rom
