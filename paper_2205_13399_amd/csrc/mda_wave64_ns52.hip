// mda_wave64_ns52.hip -- the one-wave kernel with int64 energy differences,
// built for 52 register slots per lane (instances of up to 52 facilities).
#define MDA_TILE 52
#define MDA_F64 1
#include "mda_wave_tile.h"
