// mda_wave_ns28.hip -- the one-wave kernels built for 28 register slots per lane
// (instances of up to 28 facilities).
#define MDA_TILE 28
#include "mda_wave_tile.h"
