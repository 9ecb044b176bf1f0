// mda_wave_ns48.hip -- the one-wave kernels built for 48 register slots per lane
// (instances of up to 48 facilities).
#define MDA_TILE 48
#include "mda_wave_tile.h"
