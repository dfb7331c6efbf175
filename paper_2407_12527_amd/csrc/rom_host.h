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

}  // namespace rom
