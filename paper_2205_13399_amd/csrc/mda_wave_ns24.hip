// mda_wave_ns24.hip -- the one-wave kernels built for 24 register slots per lane
// (instances of up to 24 facilities).
#define MDA_TILE 24
#include "mda_wave_tile.h"
