// mda_wave_ns8.hip -- the one-wave kernels built for 8 register slots per lane
// (instances of up to 8 facilities).
#define MDA_TILE 8
#include "mda_wave_tile.h"
