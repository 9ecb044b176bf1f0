// mda_wave64_ns40.hip -- the one-wave kernel with int64 energy differences,
// built for 40 register slots per lane (instances of up to 40 facilities).
#define MDA_TILE 40
#define MDA_F64 1
#include "mda_wave_tile.h"
