// mda_wave_ns64.hip -- the one-wave kernels built for 64 register slots per lane
// (instances of up to 64 facilities).
#define MDA_TILE 64
#include "mda_wave_tile.h"
