// rom_diag_f64.hip -- FP64 instantiations of the row-lane sweep kernel.
#include "rom_diag.h"

namespace rom {

hipError_t launch_diag_f64(const DiagArgs& a, int ntasks, int nb, int R, int K, hipStream_t s)
{
    if (R == 16) {
        if (K == 1) return launch_diag_t<double, 16, 1>(a, ntasks, nb, s);
        if (K == 2) return launch_diag_t<double, 16, 2>(a, ntasks, nb, s);
    } else if (R == 64) {
        if (K == 1) return launch_diag_t<double, 64, 1>(a, ntasks, nb, s);
        if (K == 2) return launch_diag_t<double, 64, 2>(a, ntasks, nb, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace rom
