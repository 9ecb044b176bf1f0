// mda_wave_ns16.hip -- the one-wave kernels built for 16 register slots per lane
// (instances of up to 16 facilities).
#define MDA_TILE 16
#include "mda_wave_tile.h"
