// mda_wave64_ns64.hip -- the one-wave kernel with int64 energy differences,
// built for 64 register slots per lane (instances of up to 64 facilities).
#define MDA_TILE 64
#define MDA_F64 1
#include "mda_wave_tile.h"
