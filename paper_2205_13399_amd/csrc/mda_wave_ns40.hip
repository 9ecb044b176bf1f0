// mda_wave_ns40.hip -- the one-wave kernels built for 40 register slots per lane
// (instances of up to 40 facilities).
#define MDA_TILE 40
#include "mda_wave_tile.h"
