// mda_wave_ns56.hip -- the one-wave kernels built for 56 register slots per lane
// (instances of up to 56 facilities).
#define MDA_TILE 56
#include "mda_wave_tile.h"
