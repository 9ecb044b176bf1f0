// mda_wave64_ns32.hip -- the one-wave kernel with int64 energy differences,
// built for 32 register slots per lane (instances of up to 32 facilities).
#define MDA_TILE 32
#define MDA_F64 1
#include "mda_wave_tile.h"
