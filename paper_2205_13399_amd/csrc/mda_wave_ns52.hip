// mda_wave_ns52.hip -- the one-wave kernels built for 52 register slots per lane
// (instances of up to 52 facilities).
#define MDA_TILE 52
#include "mda_wave_tile.h"
