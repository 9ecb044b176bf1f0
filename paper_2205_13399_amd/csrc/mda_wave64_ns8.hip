// mda_wave64_ns8.hip -- the one-wave kernel with int64 energy differences,
// built for 8 register slots per lane (instances of up to 8 facilities).
#define MDA_TILE 8
#define MDA_F64 1
#include "mda_wave_tile.h"
