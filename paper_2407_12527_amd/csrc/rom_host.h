// rom_host.h -- internal host-side declarations of librom.
#pragma once
#include <cstdint>

#include "../../include/rom.h"

namespace rom {

int zeta_bands(int m);
int ordinate_count(const rom_ord_spec& sp);
int generate_ordinates(const rom_ord_spec& sp, uint64_t seed, int64_t sample, double* dirs, double* w);
double phase_folded(int kind, double g, const double* u, const double* v);
int slab_ordinates(int kind, int n, uint64_t seed, int64_t sample, double* mu, double* w);

// The work of rom_sweep for a device-resident isotropic source [cells] and scalar flux [cells]
// (float, or double for ROM_PREC_FP64), every device buffer placed in the preallocated region
// scratch[0, cap); owner[3] (per device) records whose plan the region holds.  Queues the work on
// `stream` (a hipStream_t) and returns without waiting for it.
int sweep_in_scratch(rom_handle* h, void* scratch, size_t cap, uint64_t* owner, const void* src, void* phi,
                     int32_t precision, void* stream);

}  // namespace rom
