// mda_wave_ns32.hip -- the one-wave kernels built for 32 register slots per lane
// (instances of up to 32 facilities).
#define MDA_TILE 32
#include "mda_wave_tile.h"
