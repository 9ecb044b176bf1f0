// mda_wave64_ns28.hip -- the one-wave kernel with int64 energy differences,
// built for 28 register slots per lane (instances of up to 28 facilities).
#define MDA_TILE 28
#define MDA_F64 1
#include "mda_wave_tile.h"
