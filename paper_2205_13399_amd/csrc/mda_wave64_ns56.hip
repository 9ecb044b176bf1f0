// mda_wave64_ns56.hip -- the one-wave kernel with int64 energy differences,
// built for 56 register slots per lane (instances of up to 56 facilities).
#define MDA_TILE 56
#define MDA_F64 1
#include "mda_wave_tile.h"
